// common.hpp -- device-side building blocks of the coupled LB-MPCD step for
// gfx950: instance descriptors, counter-based random numbers, lattice tables.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fmath.hpp"

namespace lbmpcd {

constexpr int WG = 256;           // threads per workgroup of every kernel
constexpr int NCOPY = 64;         // replicas of the profile accumulators
constexpr int MAX_NCT = 128;      // cells per particle tile
constexpr int MAX_WIN = 96;       // LDS bins of the feedback sample window: the nodes a tile's
                                  // particles can sample, (Tx/r + 2)(Ty/r + 2)(Tz/r + 2) rounded
                                  // up (48 for the thin film's 8x2x8 cells at r = 4); larger
                                  // windows fall back to global atomics per sample
constexpr int MAX_WJ = 16;        // LDS rows of the profile sample window
constexpr int NM_WIN = 64;        // nodes of the closure's LDS window of node sums (same formula)
constexpr int MAX_UFC = 256;      // fine cells of the exchange's LDS window of LB velocities,
                                  // (Tx + 1)(Ty + 1)(Tz + 1)
constexpr uint32_t BAD_SLOT = 0xFFFFFFFFu;

// Purposes of the random streams: the counter of every draw is
// (element, LB step, substep << 8 | purpose, block).
enum Purpose : uint32_t {
    P_INIT_POS = 1, P_INIT_VEL = 2, P_REINJ = 3, P_SHIFT = 4, P_ROT = 5, P_WALL = 6,
    P_MLP_INIT = 7,   // closure network initial weights
    P_MLP_BATCH = 8,  // closure training batch draws
    P_AT = 9,         // random velocities of the MPCD-AT collision
};

// Everything a kernel needs to know about one channel.  One array of these
// lives in the workspace; kernels find their instance from a global index by
// binary search over the *_off fields.
struct InstDesc {
    // lattice Boltzmann
    int nx, ny, nz, walls_y;
    long long N;          // nodes
    long long node_off;   // first node of this instance in the concatenated node arrays
    double omega, src;    // 1/tau and 1 - 1/(2 tau)
    double g[3];
    double rho0, tau;
    int init_flow, mpcd;
    // slab and its cells
    int ylo, yhi, buf_lo, buf_hi;
    int r, R, Cx, Cz, CyB, ywrap, bot_wall, top_wall, ppc, feedback, grid_shift, pad0;
    long long ncells, Np;
    long long part_off;   // first particle of this instance in the init enumeration
    long long init_per;   // largest initial tile occupancy (cells per tile x ppc)
    // particle tiles
    int Tx, Ty, Tz, ntx, nty, ntz, cap, nct;
    int lTx, lTy, lTz, lr; // log2 of the tile sides (powers of two) and of r (-1 if r is not one)
    long long ntiles, tile_off, slot_off;
    // band (rows of node velocities used by the interpolation)
    int by0, nyb;
    long long band_off;   // first band node
    int NB, pad1;         // buffer fine rows
    long long ufine_off;  // first buffer fine cell
    long long nslab, acc_off;  // slab nodes, first slab node in the feedback sums
    long long prof_off;   // first profile row (NCOPY copies of R rows each)
    // MPCD constants
    double a, dt, gh[3], gdt[3], sd, cos_a, sin_a, mass, kT;
    float ghf[3], gdtf[3], dtf, padf;  // binary32 roundings of gh, gdt, dt (binary32 particles)
    uint32_t key0, key1;
    int S, pad2;          // MPCD steps per LB step
    // Chapman-Enskog exchange: T = ce_scale dev(-Pi_neq) / rho at the band nodes
    int ce;               // 1: Chapman-Enskog draws in this instance's buffers
    int det;              // 1: the sample sums (acc, prof) hold fixed-point integers (to_fix below)
    double ce_scale;      // nu_x m / kT / (2 cs2 tau), nu_x the exchange's stress coefficient
    double fb_lam;        // feedback: weight of an LB step's node sample in the running mean (1/fb_window)
};

// Deterministic sums: a value v enters a sum as the 64-bit integer
// round(v 2^40) (ties to even), and the integer sums, which do not depend on
// the order of the atomic additions, are read back as q 2^-40.  Exact for the
// count (1 -> 2^40); 2^-41 at most per value otherwise; sums must stay below
// 2^23 in magnitude (velocities of a valid state are far below).
constexpr double FIX_ONE = 1099511627776.0;  // 2^40
__device__ __forceinline__ unsigned long long to_fix(double v) {
    return (unsigned long long)__double2ll_rn(v * FIX_ONE);
}
__device__ __forceinline__ double from_fix(unsigned long long q) { return (double)(long long)q * (1.0 / FIX_ONE); }
__device__ __forceinline__ double fix_bits(const double* p) {  // a fixed-point sum stored in a double slot
    return from_fix(*(const unsigned long long*)p);
}

// Components of the Chapman-Enskog tensor per band node / buffer cell
// (xx, yy, zz, xy, xz, yz; the z ones are zero in 2D).
constexpr int CE_NT = 6;
// acceptance-rejection: envelope 1 + CE_KAPPA b, at most CE_ATTEMPTS draws
constexpr double CE_KAPPA = 30.0;
constexpr int CE_ATTEMPTS = 32;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// multiplies whose high halves are mixed with the odd counter words and the
// key; the key advances by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        // one 32x32 -> 64 bit product per multiplier (v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        U4 n;
        n.x = hi1 ^ c.y ^ k0;
        n.y = lo1;
        n.z = hi0 ^ c.w ^ k1;
        n.w = lo0;
        c = n;
    }
    return c;
}

__host__ __device__ __forceinline__ double u01(uint32_t lo, uint32_t hi) {
    uint64_t v = ((uint64_t)hi << 32) | (uint64_t)lo;
    return (double)(v >> 11) * 0x1.0p-53;
}

// Philox key of one instance: (seed low word, seed high word ^ instance).
struct Key { uint32_t k0, k1; };
template <typename Desc>
__device__ __forceinline__ Key key_of(const Desc& d) { return Key{d.key0, d.key1}; }

__device__ __forceinline__ U4 rng_block(Key k, uint32_t elem, uint32_t t, uint32_t sub,
                                        uint32_t purpose, uint32_t blk) {
    return philox(U4{elem, t, (sub << 8) | purpose, blk}, k.k0, k.k1);
}

// Four uniforms of one stream element (two Philox blocks, 53 bits each).
__device__ __forceinline__ void rng_uniforms4(Key k, uint32_t elem, uint32_t t,
                                              uint32_t sub, uint32_t purpose, double u[4]) {
    U4 w = rng_block(k, elem, t, sub, purpose, 0);
    u[0] = u01(w.x, w.y);
    u[1] = u01(w.z, w.w);
    w = rng_block(k, elem, t, sub, purpose, 1);
    u[2] = u01(w.x, w.y);
    u[3] = u01(w.z, w.w);
}

// Box-Muller pair (the exchange step's generator of normal deviates):
// radius sqrt(-2 ln(1 - u0)), angle 2 pi u1.
__device__ __forceinline__ void box_muller(double u0, double u1, double& z0, double& z1) {
    const double r = sqrt(-2.0 * ln_unit(1.0 - u0));
    double s, c;
    sincos_2pi(u1, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// DIM standard normals of one element; the third comes from a second pair.
template <int DIM>
__device__ __forceinline__ void rng_normals(Key k, uint32_t elem, uint32_t t, uint32_t sub,
                                            uint32_t purpose, double z[3]) {
    if constexpr (DIM == 2) {
        U4 w = rng_block(k, elem, t, sub, purpose, 0);
        box_muller(u01(w.x, w.y), u01(w.z, w.w), z[0], z[1]);
        z[2] = 0.0;
    } else {
        double u[4], dummy;
        rng_uniforms4(k, elem, t, sub, purpose, u);
        box_muller(u[0], u[1], z[0], z[1]);
        box_muller(u[2], u[3], z[2], dummy);
    }
}

// DIM binary32 standard normals of one element, for particles stored in
// binary32: block 0 of the element's stream gives four 24-bit uniforms
// a_k = (w_k >> 8) 2^-24; Box-Muller pairs (a0, a1), (a2, a3) with radius
// sqrt(-2 ln(1 - a_even)) and angle 2 pi a_odd; the third 3D component is the
// cosine of the second pair.  Binary32 throughout (fmath.hpp).
template <int DIM>
__device__ __forceinline__ void rng_normals32(Key k, uint32_t elem, uint32_t t, uint32_t sub,
                                              uint32_t purpose, float z[3]) {
    const U4 w = rng_block(k, elem, t, sub, purpose, 0);
    float s, c;
    const float r0 = sqrtf(-2.0f * ln_unit32(1.0f - (float)(w.x >> 8) * 0x1p-24f));
    sincos_2pi32((float)(w.y >> 8) * 0x1p-24f, &s, &c);
    z[0] = r0 * c;
    z[1] = r0 * s;
    z[2] = 0.0f;
    if constexpr (DIM == 3) {
        const float r1 = sqrtf(-2.0f * ln_unit32(1.0f - (float)(w.z >> 8) * 0x1p-24f));
        sincos_2pi32((float)(w.w >> 8) * 0x1p-24f, &s, &c);
        z[2] = r1 * c;
    }
}

// ---------------------------------------------------------------------------
// Lattices: D2Q9 and D3Q19 with the textbook weights (c_s^2 = 1/3).
// ---------------------------------------------------------------------------
template <int DIM> struct Lat;

template <> struct Lat<2> {
    static constexpr int Q = 9;
    static constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    static constexpr double w[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                                    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
};

template <> struct Lat<3> {
    static constexpr int Q = 19;
    static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
    static constexpr double w[19] = {1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                                     1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                     1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                     1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
};

// Instance lookup: largest i with key(D[i]) <= gid (offsets are ascending).
template <typename F>
__device__ __forceinline__ int find_inst(const InstDesc* __restrict__ D, int n_inst, long long gid, F key) {
    int lo = 0, hi = n_inst - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (key(D[mid]) <= gid) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Device error and statistics block.
struct DevStats {
    unsigned long long dropped;     // particles lost to tile overflow
    unsigned long long misplaced;   // particles found outside their tile
    unsigned long long far_moves;   // particles moving beyond the neighbour tiles (sampling MPCD steps)
    unsigned int max_fill;          // largest tile occupancy seen
    unsigned int pad;
    unsigned long long window_misses;  // samples outside their tile's LDS window (global atomics)
    unsigned long long bad_state;   // particles that left the domain by more than a period or
                                    // turned non-finite, band nodes with rho <= 0 or non-finite moments
};

// Particle arrays of one buffer: positions, velocities, ids (slot-indexed).
template <typename PT>
struct PartPtrs {
    PT* pos[3];
    PT* vel[3];
    uint32_t* id;
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// One coordinate of the shifted-grid cell, floor((x - lo + shift) * r),
// evaluated in the particle store precision.
template <typename PT>
__device__ __forceinline__ int bin_coord(PT x, PT lo, PT sh, PT r) {
    PT t = x - lo;
    t = t + sh;
    t = t * r;
    return (int)floor(t);
}

// Row of the shifted grid of a slab position, periodic across the slab when
// the slab is the whole periodic box.  A binary32 sum y - ylo + shift can
// round up to the slab height plus a full cell at the top face; such a
// particle belongs to the grid's last row.
template <typename PT, typename Desc>
__device__ __forceinline__ int bin_row(const Desc& d, PT y, PT sh, PT r) {
    int iy = bin_coord<PT>(y, (PT)d.ylo, sh, r);
    if (d.ywrap && iy >= d.R) iy -= d.R;
    if (iy > d.CyB - 1) iy = d.CyB - 1;
    return iy;
}

// Random grid shift of MPCD step (t, sub): uniform in [0, a) per axis.
template <int DIM, typename PT>
__device__ __forceinline__ void grid_shift_of(const InstDesc& d, uint32_t t, uint32_t sub, PT sh[3]) {
    double u[4];
    rng_uniforms4(key_of(d), 0u, t, sub, P_SHIFT, u);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double v = (d.grid_shift && k < DIM) ? u[k] * d.a : 0.0;
        sh[k] = (PT)v;
    }
}

}  // namespace lbmpcd
