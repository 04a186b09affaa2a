// launch.hpp -- host-side launchers of the gfx950 kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace lbmpcd {

// The LB step also advances the device clock and draws the grid shifts of the
// new LB step into shifts[n_inst][2][S][3] (slot = step parity) when S > 0.
hipError_t launch_lb_step(int dim, int lb_fp, const InstDesc* D, int n_inst, long long total, const void* fin,
                          void* fout, long long* clock, double* shifts, int S, hipStream_t s);
// With tb (tf) non-null the band kernel (interpolation) also writes the
// Chapman-Enskog tensor of the instances that use that exchange.  fbu holds
// the feedback's running means, [3][fb_stride] over the slab nodes of all
// instances.
hipError_t launch_band(int dim, int lb_fp, const InstDesc* D, int n_inst, long long total, void* f, double* acc,
                       double* fbu, long long fb_stride, double* ub, double* tb, DevStats* stats, int do_feedback,
                       hipStream_t s);
hipError_t launch_interp(int dim, const InstDesc* D, int n_inst, long long total, const double* ub, double* uf,
                         const double* tb, double* tf, hipStream_t s);
hipError_t launch_lb_init(int dim, int lb_fp, const InstDesc* D, int n_inst, long long total, void* f,
                          double* fbu, long long fb_stride, hipStream_t s);
hipError_t launch_moments(int dim, int lb_fp, const InstDesc* D, int inst, long long N, const void* f,
                          double* rho, double* u, double* pi, hipStream_t s);

// Buffers of one particle store, type-erased (positions, velocities, ids).
struct PartBuf {
    void* pos[3];
    void* vel[3];
    uint32_t* id;
};

template <typename PT>
inline PartPtrs<PT> typed(const PartBuf& b) {
    PartPtrs<PT> p;
    for (int q = 0; q < 3; ++q) { p.pos[q] = (PT*)b.pos[q]; p.vel[q] = (PT*)b.vel[q]; }
    p.id = b.id;
    return p;
}

struct ParticleLaunch {
    int dim, part_fp, mode;       // mode bit 0: collide, bit 1: stream, bit 2: MPCD-AT instead of SRD,
                                  // bit 3: Chapman-Enskog exchange (with streaming), bit 4:
                                  // deterministic (fixed-point integer sums)
    const InstDesc* D;
    int n_inst;
    long long tiles;              // workgroups (tiles of all instances)
    PartBuf in, out;
    uint32_t* fill_in;
    uint32_t* fill_out;
    const int* tile_inst;
    const double* ufine;
    const double* tfine;          // [6][buffer cells] Chapman-Enskog tensor (mode bit 3)
    double* acc;
    double* prof;
    DevStats* stats;
    const long long* clock;
    const double* shifts;         // [n_inst][2][S][3] grid shifts of the current and previous LB step
    int coll_dt, coll_s, str_s;   // collision step = clock + coll_dt, substeps
    int do_fb, do_prof;
    int diag_inst;                // instance whose cell centre-of-mass velocities are written
    double* cell_vcm;             // [dim][ncells] or null
    int cap_max;                  // largest tile capacity
    int wg_threads;               // 256 or 512 threads per workgroup (0: 256)
    int xcd_blocked;              // 1: each XCD's workgroups take a contiguous range of tiles
    long long cstride;            // bytes between component arrays (pos[k] = pos[0] + k cstride, vel[k] = pos[0] + (dim + k) cstride, id after vel)
    size_t lds_bytes;
    uint32_t* ovf;                // [2 + tiles] overflow list of a two-pass launch (zero-initialised), or
                                  // null: the context does not take the two-pass form
    int exp_max;                  // largest expected tile occupancy (particles per cell x cells per tile)
};

hipError_t launch_particles(const ParticleLaunch& L, hipStream_t s);
size_t particle_lds_bytes(int dim, int part_fp, int cap);

hipError_t launch_part_init(int dim, int part_fp, const InstDesc* D, int n_inst, long long total_particles,
                            PartBuf buf, hipStream_t s);
hipError_t launch_fill_sequential(const InstDesc* D, int n_inst, long long tiles, uint32_t* fill,
                                  uint32_t* fill_other, hipStream_t s);
// Per-instance kernels cover `slots` = ntiles * cap of that instance.
hipError_t launch_gather(int dim, int part_fp, const InstDesc* D, int inst, PartBuf buf, const uint32_t* fill,
                         double* pos_out, double* vel_out, int* cell_out, long long slots, long long t, int sub,
                         hipStream_t s);
hipError_t launch_cell_count(int dim, int part_fp, const InstDesc* D, int inst, PartBuf buf, const uint32_t* fill,
                             int* count_out, long long slots, long long t, int sub, hipStream_t s);
hipError_t launch_set_field(int dim, int part_fp, const InstDesc* D, int inst, PartBuf buf, const uint32_t* fill,
                            int which, const double* src, long long slots, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_exclusive_scan(int* a, long long n, hipStream_t s);
hipError_t launch_node_mean(const double* acc, long long nslab, int dim, int det, double* out, hipStream_t s);
hipError_t launch_profile_reduce(const InstDesc* D, int inst, int R, const double* prof, double* out,
                                 hipStream_t s);

}  // namespace lbmpcd
