// particles.hpp -- the fused MPCD step for gfx950 (the particle kernel template;
// kernels_mpcd.hip, kernels_mpcd_ce.hip and kernels_mpcd_det.hip instantiate it).
//
// Particle layout.  The cells of the shifted grid are grouped into tiles of
// Tx x Ty x Tz cells; every tile owns `cap` slots in each SoA component
// array (x, y, z, vx, vy, vz, id).  After the binning of an MPCD step every
// particle sits in the slots of the tile that contains its cell, in no
// particular order inside the tile.
//
// k_particles: one workgroup per tile, one launch per MPCD step.
//   phase 1 (collision of the previous binning, Eq. 4): cell occupancy and
//     momentum summed in LDS (FP64 atomics); the rotation of every cell
//     (2D sign / 3D axis) is drawn while the tile's particles are loading;
//     in wall-cut cells the virtual particles' momentum is added; every
//     particle is rotated about its cell's centre of mass in registers;
//   phase 2 (next MPCD step): Maxwell-Boltzmann redraw of buffer particles
//     (exchange step of Alg. 1; with mode bit 8 the first-order
//     Chapman-Enskog redraw instead) about the LB velocity of their fine cell,
//     which the workgroup copied into LDS for every buffer cell of the tile
//     while the particles were loading, streaming with the body force (Eq. 3) and
//     boundary conditions, samples of the last MPCD step of an LB step,
//     binning into the new shifted grid;
//   phase 3 (counting sort into tiles): each wave groups its particles by
//     destination tile with ballots; the first lane of a group claims a row
//     of a small LDS table of destination tiles; one global atomic per
//     destination reserves a run of slots, and every store writes the lanes
//     of a group to consecutive slots.
// Every particle is read once and written once per MPCD step.
#pragma once

#include <cmath>

#include "common.hpp"
#include "launch.hpp"

namespace lbmpcd {

// Particle buffers are passed as one base pointer each: component k of
// x, y, (z), vx, vy, (vz) at base + k * cs bytes, the ids after the last one.
template <typename PT>
struct PBuf {
    unsigned char* b;
    __device__ __forceinline__ PT* comp(int k, long long cs) const { return (PT*)(b + k * cs); }
    __device__ __forceinline__ uint32_t* id(int dim, long long cs) const { return (uint32_t*)(b + 2 * dim * cs); }
};

template <typename PT>
struct PArgs {
    const InstDesc* D;
    PBuf<PT> in, out;
    long long cs;
    uint32_t* fill_in;
    uint32_t* fill_out;
    const int* tile_inst;
    const double* ufine;
    const double* tfine;
    double* acc;
    double* prof;
    DevStats* stats;
    const long long* clock;
    const double* shifts;
    double* cell_vcm;
    int coll_dt, coll_s, str_s, do_fb, do_prof, diag_inst;
    long long ntiles;  // tiles of all instances
    long long xcd_per; // > 0: tiles per XCD of the XCD-blocked order, 0: workgroup b takes tile b
    // Overflow list: [0] tiles listed, [1] workgroups of the overflow pass
    // done, [2..] tiles.  ovf_mode 0: every tile fits the launch's slots;
    // 1: a tile with more particles than NT * PPT is listed and skipped;
    // 2: the overflow pass over the listed tiles.
    uint32_t* ovf;
    int ovf_mode;
};

// Binary32 particle arrays are read and written with buffer instructions:
// one resource per component array (its uniform 64-bit base in scalar
// registers) and a 32-bit byte offset per lane, so that no lane computes a
// 64-bit address (a channel's slots span less than 4 GiB per component).
// Binary64 particles keep global loads and stores, measured 1 % faster.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t comp_rsrc(const unsigned char* p) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, -1, 0x00020000);
}
template <typename PT>
__device__ __forceinline__ PT buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    if constexpr (sizeof(PT) == 4) return __builtin_bit_cast(PT, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
    else return __builtin_bit_cast(PT, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
template <typename PT>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t off, PT v) {
    if constexpr (sizeof(PT) == 4) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, 0, 0);
    else {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
    }
}

template <typename PT>
__device__ __forceinline__ PT wrap_periodic(PT x, PT lo, PT L) {
    if (x < lo) x = x + L;
    if (x >= lo + L) x = x - L;
    return x;
}

template <typename PT>
__device__ __forceinline__ PT fma_t(PT a, PT b, PT c);
template <>
__device__ __forceinline__ float fma_t<float>(float a, float b, float c) { return fmaf(a, b, c); }
template <>
__device__ __forceinline__ double fma_t<double>(double a, double b, double c) { return fma(a, b, c); }

template <typename PT>
__device__ __forceinline__ PT prev_below(PT v, PT toward);
template <>
__device__ __forceinline__ float prev_below<float>(float v, float toward) { return nextafterf(v, toward); }
template <>
__device__ __forceinline__ double prev_below<double>(double v, double toward) { return nextafter(v, toward); }

// Normal deviates of the exchange step, inlined: a call would make the
// caller save and restore most of its scalar registers around it.
template <int DIM>
__device__ __forceinline__ void reinject_normals(Key key, uint32_t id, uint32_t t, uint32_t sub, double* z) {
    rng_normals<DIM>(key, id, t, sub, P_REINJ, z);
}

// Chapman-Enskog exchange (a first-order Chapman-Enskog distribution about
// the LB velocity, sampled as Garcia and Alexander do, by acceptance-rejection
// against the Maxwellian): the weight of a thermal velocity z (units of
// sqrt(kT/m)) is 1 - T:zz.  Attempt k draws z from the Philox blocks 4k and
// 4k + 1 of the element's exchange stream -- attempt 0 is the Maxwell-
// Boltzmann draw -- and a uniform u from block 4k + 2, and is accepted when
// A u <= 1 - T:zz; A = 1 + CE_KAPPA b, b the largest absolute row sum of T.
// After CE_ATTEMPTS rejections the first draw stands.
template <int DIM>
__device__ __forceinline__ void ce_normals_at(Key key, uint32_t id, uint32_t t, uint32_t sub, uint32_t blk,
                                              double z[3]) {
    U4 w = rng_block(key, id, t, sub, P_REINJ, blk);
    if constexpr (DIM == 2) {
        box_muller(u01(w.x, w.y), u01(w.z, w.w), z[0], z[1]);
        z[2] = 0.0;
    } else {
        const double u0 = u01(w.x, w.y), u1 = u01(w.z, w.w);
        w = rng_block(key, id, t, sub, P_REINJ, blk + 1);
        double dummy;
        box_muller(u0, u1, z[0], z[1]);
        box_muller(u01(w.x, w.y), u01(w.z, w.w), z[2], dummy);
    }
}

// T:zz with T = (xx, yy, zz, xy, xz, yz), summed in that order
template <int DIM>
__device__ __forceinline__ double ce_contract(const double T[6], const double z[3]) {
    if constexpr (DIM == 2) return T[0] * z[0] * z[0] + T[1] * z[1] * z[1] + 2.0 * (T[3] * z[0] * z[1]);
    return T[0] * z[0] * z[0] + T[1] * z[1] * z[1] + T[2] * z[2] * z[2] +
           2.0 * (T[3] * z[0] * z[1] + T[4] * z[0] * z[2] + T[5] * z[1] * z[2]);
}

// The attempts after the first (rare: the first is accepted with
// probability about 1/A), out of line so that the particle kernel's unrolled
// exchange carries one call instead of a copy of the loop per particle.
struct CEDraw { double z0, z1, z2; };

template <int DIM>
__device__ __noinline__ CEDraw ce_retry(Key key, uint32_t id, uint32_t t, uint32_t sub, double T0, double T1,
                                        double T2, double T3, double T4, double T5, double A, CEDraw first) {
    const double T[6] = {T0, T1, T2, T3, T4, T5};
    for (int k = 1; k < CE_ATTEMPTS; ++k) {
        double zk[3];
        ce_normals_at<DIM>(key, id, t, sub, 4u * (uint32_t)k, zk);
        const U4 w = rng_block(key, id, t, sub, P_REINJ, 4u * (uint32_t)k + 2u);
        if (A * u01(w.x, w.y) <= 1.0 - ce_contract<DIM>(T, zk)) return CEDraw{zk[0], zk[1], zk[2]};
    }
    return first;
}

template <int DIM>
__device__ __forceinline__ void ce_redraw(Key key, uint32_t id, uint32_t t, uint32_t sub, const double* tf,
                                          long long NF, long long fc, double z[3]) {
    double T[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    T[0] = tf[fc];
    T[1] = tf[NF + fc];
    T[3] = tf[3 * NF + fc];
    if constexpr (DIM == 3) {
        T[2] = tf[2 * NF + fc];
        T[4] = tf[4 * NF + fc];
        T[5] = tf[5 * NF + fc];
    }
    const double r0 = fabs(T[0]) + fabs(T[3]) + fabs(T[4]);
    const double r1 = fabs(T[3]) + fabs(T[1]) + fabs(T[5]);
    const double r2 = fabs(T[4]) + fabs(T[5]) + fabs(T[2]);
    const double A = 1.0 + CE_KAPPA * fmax(r0, fmax(r1, r2));
    const U4 w = rng_block(key, id, t, sub, P_REINJ, 2u);
    if (A * u01(w.x, w.y) <= 1.0 - ce_contract<DIM>(T, z)) return;
    const CEDraw r = ce_retry<DIM>(key, id, t, sub, T[0], T[1], T[2], T[3], T[4], T[5], A, CEDraw{z[0], z[1], z[2]});
    z[0] = r.z0;
    z[1] = r.z1;
    z[2] = r.z2;
}

// Read-only tables (descriptors, tile owners, grid shifts, fill counts of
// tiles not yet processed) are read through the constant address space:
// scalar loads, which the compiler may not use for ordinary global pointers
// once the loop over tiles has stored anything.
template <typename T>
using cst = __attribute__((address_space(4))) const T;
template <typename T>
__device__ __forceinline__ cst<T>* cptr(const T* p) { return (cst<T>*)p; }

__device__ __forceinline__ void lds_add(double* p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void gl_add(double* p, double v) { unsafeAtomicAdd(p, v); }

// A sum in LDS or global memory: FP64 atomics, or with DET (deterministic
// mode) fixed-point integer atomics in the same 8-byte slot (to_fix).
template <bool DET>
__device__ __forceinline__ void sum_lds(double* p, double v) {
    if constexpr (DET) atomicAdd((unsigned long long*)p, to_fix(v));
    else lds_add(p, v);
}
template <bool DET>
__device__ __forceinline__ void sum_gl(double* p, double v) {
    if constexpr (DET) atomicAdd((unsigned long long*)p, to_fix(v));
    else gl_add(p, v);
}
template <bool DET>
__device__ __forceinline__ double sum_read(const double* p) {
    if constexpr (DET) return fix_bits(p);
    else return *p;
}

// LDS carve-up (bytes): header (counters and the table of destination tiles),
// sample windows, collision arrays and the tile's window of buffer-cell LB
// velocities.
constexpr int NHASH_BITS = 6;
constexpr int NHASH = 1 << NHASH_BITS;
constexpr size_t LDS_HDR = 1088;  // >= 4 * (4 + 3 * NHASH + 2), a multiple of 16
// Sample windows hold NREP interleaved replicas of every bin (lane l adds
// into replica l mod NREP), so that the lanes of a wave, which mostly sample
// the same one or two nodes, spread their FP64 atomics over more banks.
constexpr int NREP = 4;
constexpr size_t LDS_WIN = (size_t)(MAX_WIN + MAX_WJ) * NREP * 4 * sizeof(double);
// The exchange reads the LB velocity of a buffer particle's fine cell.  A
// particle binned into shifted cell i (shift in [0, a)) sits in unshifted
// fine cell i - 1 or i, so the particles of a tile of Tx x Ty x Tz cells read
// at most (Tx + 1)(Ty + 1)(Tz + 1) fine cells, which the workgroup copies into
// LDS at the start of the launch, where the loads overlap the particle loads
// and the collision instead of stalling the exchange.
constexpr size_t LDS_COLL = (size_t)MAX_NCT * 4 + (size_t)MAX_NCT * 9 * sizeof(double) +
                            (size_t)MAX_UFC * 3 * sizeof(double);
constexpr uint32_t DROP_SLOT = 0x7FFFFFFFu;  // never a slot: the slot total stays below it
constexpr long long OVF_GRID = 128;           // workgroups of the overflow pass
static_assert(4 * (4 + 3 * NHASH + 2) <= (int)LDS_HDR, "LDS header too small");

// Minimum resident waves per SIMD the register allocation must allow.  With
// binary32 particles (eight per thread) and in the Chapman-Enskog modes the
// kernel spills at four (128 VGPRs) and runs faster at three (on MI355X:
// 3.45 against 3.49 ms per MPCD step of the 3D channel with SRD, 4.93 against
// 5.78 with MPCD-AT, 4.70 against 7.3 with the Chapman-Enskog exchange); with
// binary64 particles (the batched 2D ensemble) four is as fast.  Six binary32
// particles per thread fit five waves with SRD and four with MPCD-AT without
// spilling; the Chapman-Enskog modes stay at three.
template <typename PT, int MODE, int PPT>
constexpr int particle_waves() {
    if (PPT == 6 && sizeof(PT) == 4) return (MODE & 8) ? 3 : (MODE & 4) ? 4 : 5;
    return (sizeof(PT) == 4 || (MODE & 8) != 0) ? 3 : 4;
}

// One workgroup per tile.
template <int DIM, typename PT, int NT, int PPT, int MODE>
__device__ __forceinline__ void particle_tile(const PArgs<PT>& A, long long T, unsigned char* smem) {
    constexpr bool COLL = (MODE & 1) != 0;
    constexpr bool STREAM = (MODE & 2) != 0;
    constexpr bool AT = (MODE & 4) != 0;  // MPCD-AT collision (Eq. 6) instead of SRD (Eq. 4)
    constexpr bool CE = (MODE & 8) != 0;  // Chapman-Enskog exchange instead of Maxwell-Boltzmann
    constexpr bool DET = (MODE & 16) != 0;  // deterministic: fixed-point integer sums
    uint32_t* wstat = (uint32_t*)smem;          // [4] far moves, misplaced, samples outside the LDS windows,
                                                // invalid particles
    uint32_t* hkey = wstat + 4;                 // [NHASH] destination tiles (local index)
    uint32_t* hcnt = hkey + NHASH;              // [NHASH + 1] particles per destination
    uint32_t* gbase = hcnt + NHASH + 1;         // [NHASH + 1] reserved run start
    double* wacc = (double*)(smem + LDS_HDR);   // [MAX_WIN][NREP][4] node sample window
    double* wprof = wacc + MAX_WIN * NREP * 4;  // [MAX_WJ][NREP][4] profile window
    unsigned char* uni = smem + LDS_HDR + LDS_WIN;
    uint32_t* ccnt = (uint32_t*)uni;                 // [MAX_NCT]
    double* csv = (double*)(uni + MAX_NCT * 4);      // [MAX_NCT][3]
    double* cvcm = csv + MAX_NCT * 3;                // [MAX_NCT][3]
    double* ucache = cvcm + MAX_NCT * 6;          // [3][MAX_UFC] LB velocities of the tile's buffer cells
    double* crot = cvcm + MAX_NCT * 3;               // [MAX_NCT][3] SRD sign/axis; MPCD-AT: sum, then mean, of the random velocities

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const long long cs = A.cs;
    const int ii = cptr(A.tile_inst)[T];
    cst<InstDesc>& d = cptr(A.D)[ii];
    const Key key = key_of(d);
    // The Philox key at a draw site, pinned to scalar registers there, so
    // that the compiler derives the round keys next to each draw (scalar
    // additions) instead of keeping twenty of them live across the kernel,
    // which spills other scalars into vector lanes.
    auto kfresh = [&]() {
        Key k = key;
        asm volatile("" : "+s"(k.k0), "+s"(k.k1));
        return k;
    };
    // tile coordinates in 32-bit arithmetic (a channel has fewer than 2^31 tiles)
    const uint32_t lt = (uint32_t)(T - d.tile_off);
    const uint32_t nxy = (uint32_t)d.ntx * (uint32_t)d.nty;
    const uint32_t tzu = lt / nxy, rem = lt - tzu * nxy;
    const uint32_t tyu = rem / (uint32_t)d.ntx;
    const int tx = (int)(rem - tyu * (uint32_t)d.ntx), ty = (int)tyu, tz = (int)tzu;
    const int cap = d.cap;
    const long long base = d.slot_off + (long long)lt * cap;
    // A channel's slots span less than 4 GiB per component, so every particle
    // access is a uniform 64-bit base plus a 32-bit lane offset.
    const unsigned char* tin = A.in.b + base * (long long)sizeof(PT);
    const unsigned char* tin_id = A.in.b + 2 * DIM * cs + base * 4;
    uint32_t n = cptr(A.fill_in)[T];
    if (A.ovf_mode == 1 && n > (uint32_t)(NT * PPT)) {
        // more particles than this launch's slots: left untouched for the
        // overflow pass, which takes the tiles of this list
        if (tid == 0) A.ovf[2 + atomicAdd(&A.ovf[0], 1u)] = (uint32_t)T;
        return;
    }
    if (n > (uint32_t)cap) n = (uint32_t)cap;
    const long long t_now = *cptr(A.clock);
    const PT rr = (PT)d.r;
    cst<double>* shtab = cptr(A.shifts) + (long long)ii * 2 * d.S * 3;
    const long long tcl = t_now + A.coll_dt;
    const uint32_t tc = (uint32_t)tcl;
    const uint32_t sc = (uint32_t)A.coll_s;

    // ---- load (the rotations below are drawn while the loads are in flight)
    uint32_t pid[PPT];
    PT px[PPT][3], pv[PPT][3];
    bool valid[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int s = tid + k * NT;
        valid[k] = s < (int)n;
#pragma unroll
        for (int c = 0; c < 3; ++c) { px[k][c] = (PT)0; pv[k][c] = (PT)0; }
        pid[k] = 0;
        if (valid[k]) {
            const uint32_t o = (uint32_t)s * (uint32_t)sizeof(PT);
            if constexpr (sizeof(PT) == 4) {
                pid[k] = buf_load<uint32_t>(comp_rsrc(tin_id), (uint32_t)s * 4u);
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    px[k][c] = buf_load<PT>(comp_rsrc(tin + c * cs), o);
                    pv[k][c] = buf_load<PT>(comp_rsrc(tin + (DIM + c) * cs), o);
                }
            } else {
                pid[k] = *(const uint32_t*)(tin_id + (uint32_t)s * 4u);
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    px[k][c] = *(const PT*)(tin + c * cs + o);
                    pv[k][c] = *(const PT*)(tin + (DIM + c) * cs + o);
                }
            }
        }
    }
    if (tid == 0 && n > (uint32_t)(3 * cap / 4)) atomicMax(&A.stats->max_fill, n);
    if (tid < 4) wstat[tid] = 0u;
    // window of fine cells (origin one cell below the tile on each axis);
    // only buffer rows are copied, and only for tiles that reach them
    if constexpr (STREAM) {
        const int uwx = d.Tx + 1, uwy = d.Ty + 1, uwz = (DIM == 3) ? d.Tz + 1 : 1;
        const int uJ0 = (ty << d.lTy) - 1;
        const int rbl = d.buf_lo * d.r, rbh = d.R - d.buf_hi * d.r;
        if (((uJ0 < rbl) || (uJ0 + uwy - 1 >= rbh)) && uwx * uwy * uwz <= MAX_UFC) {
            const int uI0 = (tx << d.lTx) - 1, uK0 = (DIM == 3) ? (tz << d.lTz) - 1 : 0;
            const long long NFc = (long long)d.Cx * d.NB * d.Cz;
            const double* ufc = A.ufine + d.ufine_off * DIM;
            for (int i = tid; i < uwx * uwy * uwz; i += NT) {
                const int ax = i % uwx, ay = (i / uwx) % uwy, az = i / (uwx * uwy);
                const int J = uJ0 + ay;
                if (J < 0 || J >= d.R || (J >= rbl && J < rbh)) continue;
                const int I = ((uI0 + ax) % d.Cx + d.Cx) % d.Cx;
                const int K = (DIM == 3) ? ((uK0 + az) % d.Cz + d.Cz) % d.Cz : 0;
                const int Jb = (J < rbl) ? J : J - (d.R - d.NB);
                const long long fc = ((long long)K * d.NB + Jb) * d.Cx + I;
#pragma unroll
                for (int q = 0; q < DIM; ++q) ucache[q * MAX_UFC + i] = ufc[q * NFc + fc];
            }
        }
    }

    // rotation of every cell of the tile (2D sign / 3D axis): independent of
    // the particles
    if constexpr (COLL) {
        for (int j = tid; j < d.nct; j += NT) {
            const int lx = j & (d.Tx - 1), ly = (j >> d.lTx) & (d.Ty - 1), lz = j >> (d.lTx + d.lTy);
            const int ix = (tx << d.lTx) + lx, iy = (ty << d.lTy) + ly, iz = (tz << d.lTz) + lz;
            const uint32_t cg = (uint32_t)(ix + d.Cx * (iy + d.CyB * iz));
            const U4 w = AT ? U4{0u, 0u, 0u, 0u} : rng_block(kfresh(), cg, tc, sc, P_ROT, 0);
            if constexpr (AT) {
                crot[3 * j] = 0.0; crot[3 * j + 1] = 0.0; crot[3 * j + 2] = 0.0;
            } else if constexpr (DIM == 2) {
                crot[3 * j] = (w.x & 1u) ? 1.0 : -1.0;
            } else {
                const double u0 = u01(w.x, w.y), u1 = u01(w.z, w.w);
                const double nz = 2.0 * u0 - 1.0;  // azimuth 2 pi u1
                const double sxy = sqrt(fmax(0.0, 1.0 - nz * nz));
                double sp, cp;
                sincos_2pi(u1, &sp, &cp);
                crot[3 * j] = sxy * cp;
                crot[3 * j + 1] = sxy * sp;
                crot[3 * j + 2] = nz;
            }
            ccnt[j] = 0u;
            csv[3 * j] = 0.0; csv[3 * j + 1] = 0.0; csv[3 * j + 2] = 0.0;
        }
        __syncthreads();
    }

    // ---- phase 1: collision (SRD, or MPCD-AT) of the binning these particles sit in
    if constexpr (COLL) {
        cst<double>* shc = shtab + ((tcl & 1) * d.S + sc) * 3;
        const PT sh[3] = {(PT)shc[0], (PT)shc[1], (PT)shc[2]};
        int lc[PPT];
        // MPCD-AT: each particle's random velocity (variance kT/m per
        // component, keyed by its id and the collision's MPCD step; binary32
        // normals for binary32 particles), kept in the particle precision
        // between the two passes over the cell
        [[maybe_unused]] PT vr[AT ? PPT : 1][3];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            lc[k] = -1;
            if (!valid[k]) continue;
            int ix = bin_coord<PT>(px[k][0], (PT)0, sh[0], rr);
            if (ix >= d.Cx) ix -= d.Cx;
            const int iy = bin_row<PT>(d, px[k][1], sh[1], rr);
            int iz = 0;
            if constexpr (DIM == 3) {
                iz = bin_coord<PT>(px[k][2], (PT)0, sh[2], rr);
                if (iz >= d.Cz) iz -= d.Cz;
            }
            const int lx = ix - (tx << d.lTx), ly = iy - (ty << d.lTy), lz = iz - (tz << d.lTz);
            if ((unsigned)lx >= (unsigned)d.Tx || (unsigned)ly >= (unsigned)d.Ty ||
                (unsigned)lz >= (unsigned)d.Tz) {
                atomicAdd(&wstat[1], 1u);
                continue;
            }
            const int c = lx + ((ly + (lz << d.lTy)) << d.lTx);
            lc[k] = c;
            atomicAdd(&ccnt[c], 1u);
#pragma unroll
            for (int q = 0; q < DIM; ++q) sum_lds<DET>(&csv[3 * c + q], (double)pv[k][q]);
            if constexpr (AT) {
                double z[3];
                if constexpr (sizeof(PT) == 4) {
                    float zf[3];
                    rng_normals32<DIM>(kfresh(), pid[k], tc, sc, P_AT, zf);
#pragma unroll
                    for (int q = 0; q < 3; ++q) z[q] = (double)zf[q];
                } else {
                    rng_normals<DIM>(kfresh(), pid[k], tc, sc, P_AT, z);
                }
#pragma unroll
                for (int q = 0; q < DIM; ++q) {
                    vr[k][q] = (PT)(d.sd * z[q]);
                    sum_lds<DET>(&crot[3 * c + q], (double)vr[k][q]);
                }
            }
        }
        __syncthreads();
        for (int j = tid; j < d.nct; j += NT) {
            const int lx = j & (d.Tx - 1), ly = (j >> d.lTx) & (d.Ty - 1), lz = j >> (d.lTx + d.lTy);
            const int ix = (tx << d.lTx) + lx, iy = (ty << d.lTy) + ly, iz = (tz << d.lTz) + lz;
            const uint32_t nc = ccnt[j];
            if (nc == 0u || ix >= d.Cx || iy >= d.CyB || iz >= d.Cz) continue;
            const uint32_t cg = (uint32_t)(ix + d.Cx * (iy + d.CyB * iz));
            // wall-cut cell below its nominal occupancy: nv virtual particles
            // with Maxwell-Boltzmann velocities (variance kT/m each), whose
            // velocity sum, of variance nv kT/m, enters the centre of mass
            double pvv[3] = {0.0, 0.0, 0.0}, mv = 0.0;
            const bool cut = ((double)sh[1] > 0.0) && ((d.bot_wall && iy == 0) || (d.top_wall && iy == d.R));
            if (cut && (int)nc < d.ppc) {
                double z[3];
                rng_normals<DIM>(kfresh(), cg, tc, sc, P_WALL, z);
                const int nv = d.ppc - (int)nc;
                const double sdv = sqrt((double)nv * d.kT / d.mass);
#pragma unroll
                for (int q = 0; q < DIM; ++q) pvv[q] = sdv * z[q];
                mv = (double)nv;
            }
#pragma unroll
            for (int q = 0; q < 3; ++q) cvcm[3 * j + q] = 0.0;
#pragma unroll
            for (int q = 0; q < DIM; ++q) cvcm[3 * j + q] = (sum_read<DET>(&csv[3 * j + q]) + pvv[q]) / ((double)nc + mv);
            if constexpr (AT) {
                // mean random velocity over the cell's real particles
#pragma unroll
                for (int q = 0; q < DIM; ++q) crot[3 * j + q] = sum_read<DET>(&crot[3 * j + q]) / (double)nc;
            }
            if (A.cell_vcm && ii == A.diag_inst) {
#pragma unroll
                for (int q = 0; q < DIM; ++q) A.cell_vcm[(long long)q * d.ncells + cg] = cvcm[3 * j + q];
            }
        }
        __syncthreads();
        const double ca = d.cos_a, sa = d.sin_a;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (lc[k] < 0) continue;
            const int c = lc[k];
            double vc[3] = {cvcm[3 * c], cvcm[3 * c + 1], cvcm[3 * c + 2]};
            if constexpr (AT) {
                // Eq. 6: centre of mass plus the random velocity less the cell mean
#pragma unroll
                for (int q = 0; q < DIM; ++q) pv[k][q] = (PT)(vc[q] + ((double)vr[k][q] - crot[3 * c + q]));
                continue;
            }
            double wv[3] = {0.0, 0.0, 0.0}, rv[3];
#pragma unroll
            for (int q = 0; q < DIM; ++q) wv[q] = (double)pv[k][q] - vc[q];
            if constexpr (DIM == 2) {
                const double s = crot[3 * c] * sa;
                rv[0] = ca * wv[0] - s * wv[1];
                rv[1] = s * wv[0] + ca * wv[1];
            } else {
                const double a0 = crot[3 * c], a1 = crot[3 * c + 1], a2 = crot[3 * c + 2];
                const double nw = a0 * wv[0] + a1 * wv[1] + a2 * wv[2];
                const double cx = a1 * wv[2] - a2 * wv[1];
                const double cy = a2 * wv[0] - a0 * wv[2];
                const double cz = a0 * wv[1] - a1 * wv[0];
                const double one_c = 1.0 - ca;
                rv[0] = wv[0] * ca + cx * sa + a0 * nw * one_c;
                rv[1] = wv[1] * ca + cy * sa + a1 * nw * one_c;
                rv[2] = wv[2] * ca + cz * sa + a2 * nw * one_c;
            }
#pragma unroll
            for (int q = 0; q < DIM; ++q) pv[k][q] = (PT)(vc[q] + rv[q]);
        }
        if constexpr (!STREAM) {
            // collision only: velocities go back to their slots
            unsigned char* tout = A.out.b + base * (long long)sizeof(PT);
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                if (!valid[k]) continue;
                const uint32_t o = (uint32_t)(tid + k * NT) * (uint32_t)sizeof(PT);
#pragma unroll
                for (int q = 0; q < DIM; ++q) *(PT*)(tout + (DIM + q) * cs + o) = pv[k][q];
            }
            if (tid == 0 && wstat[1]) atomicAdd(&A.stats->misplaced, (unsigned long long)wstat[1]);
            return;
        }
    }

    if constexpr (STREAM) {
        const uint32_t ts = (uint32_t)t_now;
        const uint32_t ss = (uint32_t)A.str_s;
        cst<double>* shs = shtab + ((t_now & 1) * d.S + ss) * 3;
        const PT sh[3] = {(PT)shs[0], (PT)shs[1], (PT)shs[2]};
        // sample windows (node sums for the feedback, fine rows for profiles)
        const int nslab_y = d.yhi - d.ylo;
        // non-negative quotients by r (a shift when r is a power of two)
        auto divr = [&](int v) { return d.lr >= 0 ? (v >> d.lr) : v / d.r; };
        const int wnx = divr(d.Tx + d.r - 1) + 2, wny = divr(d.Ty + d.r - 1) + 2;
        const int wnz = (DIM == 3) ? divr(d.Tz + d.r - 1) + 2 : 1;
        const int wx0 = divr(tx << d.lTx) - 1, wy0 = divr(ty << d.lTy) - 1;
        const int wz0 = (DIM == 3) ? divr(tz << d.lTz) - 1 : 0;
        const bool win_ok = wnx * wny * wnz <= MAX_WIN;
        const int wj0 = (ty << d.lTy) - 2, wnj = d.Ty + 4;
        const bool wj_ok = wnj <= MAX_WJ;
        const int copy = (int)(lt % (uint32_t)NCOPY);
        if (A.do_fb && win_ok)
            for (int i = tid; i < wnx * wny * wnz * NREP * 4; i += NT) wacc[i] = 0.0;
        if (A.do_prof && wj_ok)
            for (int i = tid; i < wnj * NREP * 4; i += NT) wprof[i] = 0.0;
        const int wrep = 4 * (lane & (NREP - 1));
        for (int i = tid; i < NHASH; i += NT) hkey[i] = BAD_SLOT;
        for (int i = tid; i <= NHASH; i += NT) hcnt[i] = 0u;
        __syncthreads();

        const double ylo_d = (double)d.ylo, yhi_d = (double)d.yhi;
        // the slab faces are integers, exact in either precision, so the
        // face tests compare in the particle precision
        const PT ylo_p = (PT)d.ylo, yhi_p = (PT)d.yhi;
        const int bw = d.bot_wall, tw = d.top_wall, ywrap = d.ywrap;
        const int rb_lo = d.buf_lo * d.r, rb_hi = d.R - d.buf_hi * d.r;
        const long long NF = (long long)d.Cx * d.NB * d.Cz;
        const double* uf = A.ufine + d.ufine_off * DIM;
        [[maybe_unused]] const double* tfl = CE ? A.tfine + d.ufine_off * CE_NT : nullptr;
        [[maybe_unused]] const bool ce_on = CE && d.ce;
        // per-tile constants in the particle precision (read once, not per particle)
        PT dtp, ghp[3], gdp[3];
        if constexpr (sizeof(PT) == 4) {
            dtp = (PT)d.dtf;
            for (int q = 0; q < 3; ++q) { ghp[q] = (PT)d.ghf[q]; gdp[q] = (PT)d.gdtf[q]; }
        } else {
            dtp = (PT)d.dt;
            for (int q = 0; q < 3; ++q) { ghp[q] = (PT)d.gh[q]; gdp[q] = (PT)d.gdt[q]; }
        }
        const PT nxp = (PT)d.nx, nzp = (PT)d.nz, nyp = (PT)d.ny;
        uint32_t dest[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) dest[k] = BAD_SLOT;
        // exchange step: redraw buffer particles about the LB velocity.  (A
        // version that first listed each wave's buffer particles densely in
        // LDS, so that mixed waves ran the normals once per 64 of them, was
        // measured: 1 % faster on the thin film, 2 % slower on the 3D channel.)
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (!valid[k]) continue;
            const int J0 = clampi((int)floor(((double)px[k][1] - ylo_d) * (double)d.r), 0, d.R - 1);
            if (J0 < rb_lo || J0 >= rb_hi) {
                const int I = clampi((int)floor((double)px[k][0] * (double)d.r), 0, d.Cx - 1);
                const int K = (DIM == 3) ? clampi((int)floor((double)px[k][2] * (double)d.r), 0, d.Cz - 1) : 0;
                const int Jb = (J0 < rb_lo) ? J0 : J0 - (d.R - d.NB);
                const long long fc = ((long long)K * d.NB + Jb) * d.Cx + I;
                double z[3], ulv[3];
                if (sizeof(PT) == 4 && !(CE && ce_on)) {
                    // binary32 particles draw binary32 normals (one Philox
                    // block); the Chapman-Enskog draws stay binary64
                    float zf[3];
                    rng_normals32<DIM>(kfresh(), pid[k], ts, ss, P_REINJ, zf);
#pragma unroll
                    for (int q = 0; q < 3; ++q) z[q] = (double)zf[q];
                } else {
                    reinject_normals<DIM>(kfresh(), pid[k], ts, ss, z);
                    if constexpr (CE) {
                        if (ce_on) ce_redraw<DIM>(kfresh(), pid[k], ts, ss, tfl, NF, fc, z);
                    }
                }
#pragma unroll
                for (int q = 0; q < DIM; ++q) ulv[q] = 0.0;
                {
                    // the LB velocity from the tile's LDS window, or from
                    // global memory for a particle outside it (misplaced, or
                    // a window too large for the LDS)
                    const int uwx = d.Tx + 1, uwy = d.Ty + 1, uwz = (DIM == 3) ? d.Tz + 1 : 1;
                    const int uJ0 = (ty << d.lTy) - 1;
                    const bool uc_ok = ((uJ0 < rb_lo) || (uJ0 + uwy - 1 >= rb_hi)) && uwx * uwy * uwz <= MAX_UFC;
                    int ax = I - ((tx << d.lTx) - 1);
                    if (ax < 0) ax += d.Cx;
                    const int ay = J0 - uJ0;
                    int az = 0;
                    if (DIM == 3) { az = K - ((tz << d.lTz) - 1); if (az < 0) az += d.Cz; }
                    if (uc_ok && ax < uwx && ay >= 0 && ay < uwy && az < uwz) {
                        const int ci = ax + uwx * (ay + uwy * az);
#pragma unroll
                        for (int q = 0; q < DIM; ++q) ulv[q] = ucache[q * MAX_UFC + ci];
                    } else {
#pragma unroll
                        for (int q = 0; q < DIM; ++q) ulv[q] = uf[q * NF + fc];
                    }
                }
#pragma unroll
                for (int q = 0; q < DIM; ++q) pv[k][q] = (PT)(ulv[q] + d.sd * z[q]);
            }
        }

        // streaming, Eq. 3, with the body force as constant acceleration
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (!valid[k]) continue;
            PT r0[3] = {px[k][0], px[k][1], px[k][2]}, v0[3] = {pv[k][0], pv[k][1], pv[k][2]};
            PT r1[3] = {r0[0], r0[1], r0[2]}, v1[3] = {v0[0], v0[1], v0[2]};
#pragma unroll
            for (int q = 0; q < DIM; ++q) {
                const PT vh = v0[q] + ghp[q];
                r1[q] = fma_t<PT>(vh, dtp, r0[q]);
                v1[q] = v0[q] + gdp[q];
            }
            const bool below = r1[1] < ylo_p, above = r1[1] >= yhi_p;
            if (!ywrap && (below || above)) {
                const int wall = below ? bw : tw;
                const double Yw = below ? ylo_d : yhi_d;
                double q1[3] = {(double)r1[0], (double)r1[1], (double)r1[2]};
                double w1[3] = {(double)v1[0], (double)v1[1], (double)v1[2]};
                if (wall) {
                    const double tcx = (Yw - (double)r0[1]) / (double)v0[1];
                    const double tr = d.dt - tcx;
#pragma unroll
                    for (int q = 0; q < DIM; ++q) {
                        double rc = (double)r0[q] + ((double)v0[q] + 0.5 * d.g[q] * tcx) * tcx;
                        const double vc = (double)v0[q] + d.g[q] * tcx;
                        if (q == 1) rc = Yw;
                        const double vr = -vc;
                        q1[q] = rc + (vr + 0.5 * d.g[q] * tr) * tr;
                        w1[q] = vr + d.g[q] * tr;
                    }
                } else if (bw || tw) {
                    q1[1] = 2.0 * Yw - q1[1];
                    w1[1] = -w1[1];
                } else {
                    q1[1] = (double)wrap_periodic<PT>(r1[1], (PT)d.ylo, (PT)(d.yhi - d.ylo));
                }
#pragma unroll
                for (int q = 0; q < DIM; ++q) { r1[q] = (PT)q1[q]; v1[q] = (PT)w1[q]; }
                if (r1[1] < ylo_p) r1[1] = ylo_p;
                if (r1[1] >= yhi_p) r1[1] = prev_below<PT>(yhi_p, ylo_p);
            } else if (ywrap) {
                r1[1] = wrap_periodic<PT>(r1[1], (PT)0, nyp);
            }
            r1[0] = wrap_periodic<PT>(r1[0], (PT)0, nxp);
            if constexpr (DIM == 3) r1[2] = wrap_periodic<PT>(r1[2], (PT)0, nzp);
            // A particle that left the domain by more than one period in this
            // step, or whose position or velocity is not finite, is an invalid
            // state (a diverged LB field hands out such velocities): it is
            // parked at the slab's lower corner at rest, so that every cell,
            // tile and slot index below stays in range, and counted (the next
            // synchronising call reports E_STATE).
            bool bad = !(r1[0] >= (PT)0 && r1[0] < nxp);
            if constexpr (DIM == 3) bad |= !(r1[2] >= (PT)0 && r1[2] < nzp);
            bad |= ywrap ? !(r1[1] >= (PT)0 && r1[1] < nyp) : !(r1[1] >= ylo_p && r1[1] < yhi_p);
#pragma unroll
            for (int q = 0; q < DIM; ++q) bad |= !isfinite(v1[q]);
            if (bad) {
#pragma unroll
                for (int q = 0; q < 3; ++q) v1[q] = (PT)0;
                r1[0] = (PT)0;
                r1[1] = ywrap ? (PT)0 : ylo_p;
                r1[2] = (PT)0;
                atomicAdd(&wstat[3], 1u);
            }
#pragma unroll
            for (int q = 0; q < 3; ++q) { px[k][q] = r1[q]; pv[k][q] = v1[q]; }
        }

        // samples right after streaming (last MPCD step of an LB step); the
        // loops over a thread's particles are split by task so that fewer
        // per-tile constants are live at once
        if (A.do_fb | A.do_prof) {
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                if (!valid[k]) continue;
                const int J = clampi((int)floor(((double)px[k][1] - ylo_d) * (double)d.r), 0, d.R - 1);
                double vals[4] = {1.0, (double)pv[k][0], (double)pv[k][1], DIM == 3 ? (double)pv[k][2] : 0.0};
                // the feedback projects the interior slab nodes only: buffer
                // rows are not sampled for it (the profile takes every row)
                if (A.do_fb && J >= rb_lo && J < rb_hi) {
                    const int ixn = clampi((int)floor((double)px[k][0]), 0, d.nx - 1);
                    const int iyn = d.lr >= 0 ? (J >> d.lr) : J / d.r;
                    const int izn = (DIM == 3) ? clampi((int)floor((double)px[k][2]), 0, d.nz - 1) : 0;
                    int ax = ixn - wx0; if (ax < 0) ax += d.nx; else if (ax >= d.nx) ax -= d.nx;
                    const int ay = iyn - wy0;
                    int az = izn - wz0;
                    if (DIM == 3) { if (az < 0) az += d.nz; else if (az >= d.nz) az -= d.nz; }
                    if (win_ok && ax < wnx && ay >= 0 && ay < wny && az < wnz) {
                        double* wb = wacc + 4 * NREP * (ax + wnx * (ay + wny * az)) + wrep;
#pragma unroll
                        for (int q = 0; q < DIM + 1; ++q) sum_lds<DET>(&wb[q], vals[q]);
                    } else {
                        const long long sidx = ((long long)izn * nslab_y + iyn) * d.nx + ixn;
                        double* gb = A.acc + (d.acc_off + sidx) * 4;
#pragma unroll
                        for (int q = 0; q < DIM + 1; ++q) sum_gl<DET>(&gb[q], vals[q]);
                        atomicAdd(&wstat[2], 1u);
                    }
                }
                if (A.do_prof) {
                    const int aj = J - wj0;
                    if (wj_ok && aj >= 0 && aj < wnj) {
#pragma unroll
                        for (int q = 0; q < DIM + 1; ++q) sum_lds<DET>(&wprof[4 * NREP * aj + wrep + q], vals[q]);
                    } else {
                        double* gb = A.prof + (d.prof_off + (long long)copy * d.R + J) * 4;
#pragma unroll
                        for (int q = 0; q < DIM + 1; ++q) sum_gl<DET>(&gb[q], vals[q]);
                        atomicAdd(&wstat[2], 1u);
                    }
                }
            }
        }

        // binning into the shifted grid of this MPCD step
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (!valid[k]) continue;
            int ix = bin_coord<PT>(px[k][0], (PT)0, sh[0], rr);
            if (ix >= d.Cx) ix -= d.Cx;
            const int iy = bin_row<PT>(d, px[k][1], sh[1], rr);
            int iz = 0;
            if constexpr (DIM == 3) {
                iz = bin_coord<PT>(px[k][2], (PT)0, sh[2], rr);
                if (iz >= d.Cz) iz -= d.Cz;
            }
            const int ntx = ix >> d.lTx, nty = iy >> d.lTy, ntz = iz >> d.lTz;
            dest[k] = (uint32_t)(ntx + d.ntx * (nty + d.nty * ntz));
            if (dest[k] >= (uint32_t)d.ntiles) {
                // unreachable for positions inside the domain (checked above);
                // kept so that no slot index can leave the channel's tiles
                dest[k] = lt;
                atomicAdd(&wstat[3], 1u);
            }
            // moves beyond the neighbour tiles (they are grouped like any other
            // destination; the count bounds the sample-window misses, so it is
            // kept in the MPCD steps that sample, and skipped in the others)
            if (A.do_fb | A.do_prof) {
                int dx = ntx - tx, dy = nty - ty, dz = ntz - tz;
                if (d.ntx > 2) { if (dx == d.ntx - 1) dx = -1; else if (dx == 1 - d.ntx) dx = 1; }
                if (DIM == 3 && d.ntz > 2) { if (dz == d.ntz - 1) dz = -1; else if (dz == 1 - d.ntz) dz = 1; }
                if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1) atomicAdd(&wstat[0], 1u);
            }
        }

        // ---- phase 3a: group each wave's particles by destination tile.
        // Lanes with equal destinations get consecutive ranks; the group's
        // first lane claims a row of the LDS destination table and the
        // group's offset in it, and hands both back with one permute.
        uint32_t pk[PPT];  // bit 31: direct slot; else (table row + 1) << 24 | rank
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const uint32_t key = dest[k];
            // Waterfall over the lanes still waiting: the lowest of them
            // names the next group, whose lanes (the active lanes with its
            // key) take their ranks from the active mask and leave the loop.
            int my_leader = 0;
            uint32_t my_rank = 0, lead_cnt = 0;
            if (key != BAD_SLOT) {
                for (;;) {
                    const uint32_t kv = (uint32_t)__builtin_amdgcn_readfirstlane((int)key);
                    if (key == kv) {
                        const unsigned long long m = __ballot(1);
                        my_leader = __ffsll(m) - 1;
                        my_rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                        lead_cnt = (uint32_t)__popcll(m);
                        break;
                    }
                }
            }
            const bool is_lead = key != BAD_SLOT && my_rank == 0u;
            uint32_t packed = 0u;
            if (is_lead) {
                int h = -1;
                uint32_t hh = (key * 2654435761u) >> (32 - NHASH_BITS);
#pragma unroll 1
                for (int probe = 0; probe < NHASH; ++probe) {
                    const uint32_t old = atomicCAS(&hkey[hh], BAD_SLOT, key);
                    if (old == BAD_SLOT || old == key) { h = (int)hh; break; }
                    hh = (hh + 1) & (NHASH - 1);
                }
                if (h >= 0) {
                    packed = ((uint32_t)(h + 1) << 24) | atomicAdd(&hcnt[h], lead_cnt);
                } else {
                    // more destinations than table rows: reserve directly
                    const uint32_t ob = atomicAdd(&A.fill_out[d.tile_off + key], lead_cnt);
                    packed = ob < 0xFFFFFFu ? ob : 0xFFFFFFu;
                }
            }
            packed = (uint32_t)__shfl((int)packed, my_leader);
            pk[k] = BAD_SLOT;
            if (key != BAD_SLOT) {
                const uint32_t row = packed >> 24;
                const uint32_t r_ = (packed & 0xFFFFFFu) + my_rank;
                if (row) {
                    pk[k] = (row << 24) | r_;
                } else {
                    pk[k] = r_ < (uint32_t)cap ? (0x80000000u | (uint32_t)(key * cap + r_)) : DROP_SLOT;
                }
            }
        }
        __syncthreads();
        // ---- phase 3b: one global atomic per destination reserves a run of
        // slots; each store writes the lanes of a group to consecutive slots
        if (tid < NHASH) {
            const uint32_t c = hcnt[tid];
            gbase[tid] = c > 0u ? atomicAdd(&A.fill_out[d.tile_off + hkey[tid]], c) : 0u;
        }
        __syncthreads();
        unsigned char* och = A.out.b + d.slot_off * (long long)sizeof(PT);
        unsigned char* och_id = A.out.b + 2 * DIM * cs + d.slot_off * 4;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const uint32_t e = pk[k];
            if (e == BAD_SLOT) continue;
            uint32_t g = 0u;  // slot within the channel
            bool ok = e != DROP_SLOT;
            if (ok && (e & 0x80000000u)) {
                g = e & 0x7FFFFFFFu;
            } else if (ok) {
                const int row = (int)(e >> 24) - 1;
                const uint32_t r_ = gbase[row] + (e & 0xFFFFFFu);
                ok = r_ < (uint32_t)cap;
                g = hkey[row] * (uint32_t)cap + r_;
            }
            if (!ok) {
                atomicAdd(&A.stats->dropped, 1ull);
                continue;
            }
            const uint32_t o = g * (uint32_t)sizeof(PT);
            if constexpr (sizeof(PT) == 4) {
                buf_store<uint32_t>(comp_rsrc(och_id), g * 4u, pid[k]);
#pragma unroll
                for (int q = 0; q < DIM; ++q) {
                    buf_store<PT>(comp_rsrc(och + q * cs), o, px[k][q]);
                    buf_store<PT>(comp_rsrc(och + (DIM + q) * cs), o, pv[k][q]);
                }
            } else {
                *(uint32_t*)(och_id + g * 4u) = pid[k];
#pragma unroll
                for (int q = 0; q < DIM; ++q) {
                    *(PT*)(och + q * cs + o) = px[k][q];
                    *(PT*)(och + (DIM + q) * cs + o) = pv[k][q];
                }
            }
        }
        // ---- sample windows to global memory
        if (A.do_fb && win_ok) {
            for (int i = tid; i < wnx * wny * wnz; i += NT) {
                double sum[4] = {0.0, 0.0, 0.0, 0.0};
                [[maybe_unused]] unsigned long long isum[4] = {0ull, 0ull, 0ull, 0ull};
#pragma unroll
                for (int r = 0; r < NREP; ++r)
#pragma unroll
                    for (int q = 0; q < DIM + 1; ++q) {
                        if constexpr (DET) isum[q] += ((const unsigned long long*)wacc)[4 * (NREP * i + r) + q];
                        else sum[q] += wacc[4 * (NREP * i + r) + q];
                    }
                if (DET ? isum[0] == 0ull : sum[0] == 0.0) continue;
                const int ax = i % wnx, ay = (i / wnx) % wny, az = i / (wnx * wny);
                int ixn = wx0 + ax; if (ixn < 0) ixn += d.nx; else if (ixn >= d.nx) ixn -= d.nx;
                const int iyn = wy0 + ay;
                int izn = wz0 + az;
                if (DIM == 3) { if (izn < 0) izn += d.nz; else if (izn >= d.nz) izn -= d.nz; }
                if (iyn < 0 || iyn >= nslab_y) continue;  // samples are clamped to the slab
                const long long sidx = ((long long)izn * nslab_y + iyn) * d.nx + ixn;
                double* gb = A.acc + (d.acc_off + sidx) * 4;
#pragma unroll
                for (int q = 0; q < DIM + 1; ++q) {
                    if constexpr (DET) atomicAdd((unsigned long long*)&gb[q], isum[q]);
                    else gl_add(&gb[q], sum[q]);
                }
            }
        }
        if (A.do_prof && wj_ok) {
            for (int i = tid; i < wnj; i += NT) {
                double sum[4] = {0.0, 0.0, 0.0, 0.0};
                [[maybe_unused]] unsigned long long isum[4] = {0ull, 0ull, 0ull, 0ull};
#pragma unroll
                for (int r = 0; r < NREP; ++r)
#pragma unroll
                    for (int q = 0; q < DIM + 1; ++q) {
                        if constexpr (DET) isum[q] += ((const unsigned long long*)wprof)[4 * (NREP * i + r) + q];
                        else sum[q] += wprof[4 * (NREP * i + r) + q];
                    }
                if (DET ? isum[0] == 0ull : sum[0] == 0.0) continue;
                const int J = wj0 + i;
                double* gb = A.prof + (d.prof_off + (long long)copy * d.R + J) * 4;
#pragma unroll
                for (int q = 0; q < DIM + 1; ++q) {
                    if constexpr (DET) atomicAdd((unsigned long long*)&gb[q], isum[q]);
                    else gl_add(&gb[q], sum[q]);
                }
            }
        }
        if (tid == 0) {
            A.fill_in[T] = 0u;
            if (wstat[0]) atomicAdd(&A.stats->far_moves, (unsigned long long)wstat[0]);
            if (wstat[1]) atomicAdd(&A.stats->misplaced, (unsigned long long)wstat[1]);
            if (wstat[2]) atomicAdd(&A.stats->window_misses, (unsigned long long)wstat[2]);
            if (wstat[3]) atomicAdd(&A.stats->bad_state, (unsigned long long)wstat[3]);
        }
    }
}

// One workgroup per tile.
template <int DIM, typename PT, int NT, int PPT, int MODE>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(particle_waves<PT, MODE, PPT>())))
k_particles(PArgs<PT> A) {
    extern __shared__ __align__(16) unsigned char smem[];
    // Workgroups are dealt to the eight XCDs in turn.  In the XCD-blocked
    // order the workgroups of one XCD take one contiguous range of tiles, so
    // the tiles that trade particles are mostly served by one L2, where the
    // partial lines of their destination runs merge.
    long long T = blockIdx.x;
    if (A.xcd_per > 0) {
        T = (long long)(blockIdx.x % 8) * A.xcd_per + blockIdx.x / 8;
        if (T >= A.ntiles) return;
    }
    particle_tile<DIM, PT, NT, PPT, MODE>(A, T, smem);
}

// The overflow pass (ovf_mode 2): the workgroups of a small grid take the
// listed tiles in turn; the last workgroup to finish clears the list.  A
// kernel of its own, so that the loop does not weigh on the register
// allocation of the one-tile kernel.
template <int DIM, typename PT, int NT, int PPT, int MODE>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(particle_waves<PT, MODE, PPT>())))
k_particles_ovf(PArgs<PT> A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t cnt = A.ovf[0];
    for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
        particle_tile<DIM, PT, NT, PPT, MODE>(A, (long long)A.ovf[2 + i], smem);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&A.ovf[1], 1u) == gridDim.x - 1) {
            A.ovf[0] = 0u;
            A.ovf[1] = 0u;
        }
    }
}

// ---------------------------------------------------------------------------
// launch templates; `Modes::run<DIM, PT, NT, PPT>` picks the instantiation
// of the mode (each translation unit instantiates its own set)
// ---------------------------------------------------------------------------
template <int DIM, typename PT, int NT, int PPT, int MODE, int OVF = 0>
static hipError_t launch_p4(const ParticleLaunch& L, hipStream_t s) {
    PArgs<PT> a;
    a.D = L.D;
    a.in.b = (unsigned char*)L.in.pos[0]; a.out.b = (unsigned char*)L.out.pos[0]; a.cs = L.cstride;
    a.fill_in = L.fill_in; a.fill_out = L.fill_out; a.tile_inst = L.tile_inst;
    a.ufine = L.ufine; a.tfine = L.tfine; a.acc = L.acc; a.prof = L.prof; a.stats = L.stats; a.clock = L.clock;
    a.shifts = L.shifts;
    a.coll_dt = L.coll_dt; a.coll_s = L.coll_s; a.str_s = L.str_s;
    a.do_fb = L.do_fb; a.do_prof = L.do_prof; a.diag_inst = L.diag_inst; a.cell_vcm = L.cell_vcm;
    a.ntiles = L.tiles;
    a.xcd_per = L.xcd_blocked ? (L.tiles + 7) / 8 : 0;
    a.ovf = L.ovf;
    a.ovf_mode = OVF;
    if constexpr (OVF == 2) {
        const long long grid = L.tiles < OVF_GRID ? L.tiles : OVF_GRID;
        hipLaunchKernelGGL((k_particles_ovf<DIM, PT, NT, PPT, MODE>), dim3((unsigned)grid), dim3(NT), L.lds_bytes, s,
                           a);
        return hipGetLastError();
    } else {
        const long long grid = L.xcd_blocked ? 8 * a.xcd_per : L.tiles;
        auto kern = k_particles<DIM, PT, NT, PPT, MODE>;
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NT), L.lds_bytes, s, a);
        return hipGetLastError();
    }
}

// Workgroup shape: threads x particles per thread must cover the largest
// tile capacity.  256 threads unless the caller asks for 512.
template <class Modes, int DIM, typename PT>
static hipError_t launch_p2(const ParticleLaunch& L, hipStream_t s) {
    if (L.wg_threads == 128) {
        if (L.cap_max <= 4 * 128) return Modes::template run<DIM, PT, 128, 4>(L, s);
        if (L.cap_max <= 8 * 128) return Modes::template run<DIM, PT, 128, 8>(L, s);
        return hipErrorInvalidValue;
    }
    if (L.wg_threads == 512) {
        if (L.cap_max <= 2 * 512) return Modes::template run<DIM, PT, 512, 2>(L, s);
        if (L.cap_max <= 4 * 512) return Modes::template run<DIM, PT, 512, 4>(L, s);
        return hipErrorInvalidValue;
    }
    if (L.cap_max <= 2 * 256) return Modes::template run<DIM, PT, 256, 2>(L, s);
    if (L.cap_max <= 4 * 256) return Modes::template run<DIM, PT, 256, 4>(L, s);
    if (L.cap_max <= 8 * 256) return Modes::template run<DIM, PT, 256, 8>(L, s);
    return hipErrorInvalidValue;
}

// Tiles of 1025-2048 slots at 256 threads: six slots per thread instead of
// eight leave the kernel fewer vector registers and, for binary32
// particles, one more wave per SIMD (SRD: 96 VGPRs and five waves instead
// of 113 and four; MPCD-AT: 123 and four instead of 152 and three); binary64
// particles stay at four waves and spill 24 bytes per lane instead of 108.
// A tile holding
// more than 1536 particles is skipped and listed by that launch and
// processed by a second launch over the list (512 threads, four slots per
// thread: a listed tile waits on one tile's latency, which more threads
// shorten).  It is rare: the
// tile's expected occupancy plus two standard deviations of its Poisson
// count must stay within 1536 for this form to be taken.
inline bool split_applies(const ParticleLaunch& L) {
    if (L.ovf == nullptr) return false;
    if ((L.wg_threads != 0 && L.wg_threads != 256) || L.cap_max <= 4 * 256 || L.cap_max > 8 * 256) return false;
    const double e = (double)L.exp_max;
    return e + 2.0 * std::sqrt(e) <= 6.0 * 256;
}

template <class Modes, int DIM, typename PT>
static hipError_t launch_split_dim(const ParticleLaunch& L, hipStream_t s) {
    hipError_t e = Modes::template run<DIM, PT, 256, 6, 1>(L, s);
    if (e == hipSuccess) e = Modes::template run<DIM, PT, 512, 4, 2>(L, s);
    return e;
}

template <class Modes>
static hipError_t launch_modes(const ParticleLaunch& L, hipStream_t s) {
    if (L.tiles <= 0) return hipSuccess;
    if (split_applies(L)) {
        if (L.part_fp == 64)
            return L.dim == 2 ? launch_split_dim<Modes, 2, double>(L, s) : launch_split_dim<Modes, 3, double>(L, s);
        return L.dim == 2 ? launch_split_dim<Modes, 2, float>(L, s) : launch_split_dim<Modes, 3, float>(L, s);
    }
    if (L.dim == 2 && L.part_fp == 64) return launch_p2<Modes, 2, double>(L, s);
    if (L.dim == 2) return launch_p2<Modes, 2, float>(L, s);
    if (L.part_fp == 64) return launch_p2<Modes, 3, double>(L, s);
    return launch_p2<Modes, 3, float>(L, s);
}

// The Chapman-Enskog modes (bit 8), instantiated in kernels_mpcd_ce.hip.
hipError_t launch_particles_ce(const ParticleLaunch& L, hipStream_t s);
// The deterministic modes (bit 16), instantiated in kernels_mpcd_det.hip.
hipError_t launch_particles_det(const ParticleLaunch& L, hipStream_t s);

}  // namespace lbmpcd
