// kernels_mpcd.hip -- multiparticle-collision kernels for gfx950.
//
// Particle layout.  The cells of the shifted grid are grouped into tiles of
// Tx x Ty x Tz cells; every tile owns `cap` slots in each SoA component
// array (x, y, z, vx, vy, vz, id).  After the binning of an MPCD step every
// particle sits in the slots of the tile that contains its cell, in no
// particular order inside the tile.
//
// k_particles: one workgroup per tile, one launch per MPCD step.
//   phase 1 (collision of the previous binning, Eq. 4): cell occupancy and
//     momentum are summed in LDS (FP64 atomics), one thread per cell draws the
//     rotation (2D sign / 3D axis) and, in wall-cut cells, the virtual
//     particles' momentum, then every particle is rotated about its cell's
//     centre of mass in registers;
//   phase 2 (next MPCD step): Maxwell-Boltzmann redraw of buffer particles
//     (exchange step of Alg. 1), streaming with body force (Eq. 3) and
//     boundary conditions, sampling of the node velocity sums, binning into
//     the new shifted grid;
//   phase 3 (counting sort into tiles): destinations are counted per
//     neighbour tile in LDS, one global atomic per neighbour reserves a run
//     of slots, particles are staged in LDS ordered by destination and
//     written out in contiguous runs.
// Every particle is read once and written once per MPCD step.
#include "common.hpp"
#include "launch.hpp"

namespace lbmpcd {

template <typename PT>
struct PArgs {
    const InstDesc* D;
    int n_inst;
    PartPtrs<PT> in, out;
    uint32_t* fill_in;
    uint32_t* fill_out;
    const int* tile_inst;
    const double* ufine;
    double* acc;
    double* prof;
    DevStats* stats;
    const long long* clock;
    int coll_dt, coll_s, str_s, do_fb, do_prof, diag_inst;
    double* cell_vcm;
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

template <typename PT>
__device__ __forceinline__ int bin_coord(PT x, PT lo, PT sh, PT r) {
    PT t = x - lo;
    t = t + sh;
    t = t * r;
    return (int)floor(t);
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

__device__ __forceinline__ void lds_add(double* p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void gl_add(double* p, double v) { unsafeAtomicAdd(p, v); }

template <int DIM, typename PT>
__device__ __forceinline__ void grid_shift_of(const InstDesc& d, uint32_t t, uint32_t sub, PT sh[3]) {
    double u[4];
    rng_uniforms4(d, 0u, t, sub, P_SHIFT, u);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double v = (d.grid_shift && k < DIM) ? u[k] * d.a : 0.0;
        sh[k] = (PT)v;
    }
}

// LDS carve-up (bytes): header, sample windows, then a union of the
// collision arrays and the output staging area.
constexpr size_t LDS_HDR = 512;
constexpr size_t LDS_WIN = (size_t)(MAX_WIN + MAX_WJ) * 4 * sizeof(double);
constexpr size_t LDS_COLL = (size_t)MAX_NCT * 4 + (size_t)MAX_NCT * 9 * sizeof(double);

size_t particle_lds_bytes(int dim, int part_fp, int cap) {
    size_t stage = (size_t)cap * (8 + (size_t)2 * dim * (part_fp == 64 ? 8 : 4));
    return LDS_HDR + LDS_WIN + (stage > LDS_COLL ? stage : LDS_COLL);
}

template <int DIM, typename PT, int PPT, int MODE>
__global__ void __launch_bounds__(WG) k_particles(PArgs<PT> A) {
    constexpr bool COLL = (MODE & 1) != 0;
    constexpr bool STREAM = (MODE & 2) != 0;
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* dcnt = (uint32_t*)smem;          // [32] particles per destination code
    uint32_t* gbase = dcnt + 32;               // [32] reserved run start per code
    uint32_t* tile_of_code = gbase + 32;       // [32] destination tile (local index) per code
    uint32_t* s_off = tile_of_code + 32;       // [32] staging offset per code
    double* wacc = (double*)(smem + LDS_HDR);  // [MAX_WIN][4] node sample window
    double* wprof = wacc + MAX_WIN * 4;        // [MAX_WJ][4] profile window
    unsigned char* uni = smem + LDS_HDR + LDS_WIN;
    uint32_t* ccnt = (uint32_t*)uni;                 // [MAX_NCT]
    double* csv = (double*)(uni + MAX_NCT * 4);      // [MAX_NCT][3]
    double* cvcm = csv + MAX_NCT * 3;                // [MAX_NCT][3]
    double* crot = cvcm + MAX_NCT * 3;               // [MAX_NCT][3]

    const int tid = threadIdx.x;
    const long long T = blockIdx.x;
    const int ii = A.tile_inst[T];
    const InstDesc& d = A.D[ii];
    const long long lt = T - d.tile_off;
    const int tx = (int)(lt % d.ntx);
    const int ty = (int)((lt / d.ntx) % d.nty);
    const int tz = (int)(lt / ((long long)d.ntx * d.nty));
    const int cap = d.cap;
    const long long base = d.slot_off + lt * cap;
    uint32_t n = A.fill_in[T];
    if (n > (uint32_t)cap) n = (uint32_t)cap;
    if (tid == 0 && n > (uint32_t)(3 * cap / 4)) atomicMax(&A.stats->max_fill, n);

    const long long t_now = *A.clock;
    const PT rr = (PT)d.r;

    // ---- load
    uint32_t pid[PPT];
    PT px[PPT][3], pv[PPT][3];
    bool valid[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int s = tid + k * WG;
        valid[k] = s < (int)n;
        px[k][2] = (PT)0;
        pv[k][2] = (PT)0;
        pid[k] = 0;
        if (valid[k]) {
            pid[k] = A.in.id[base + s];
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                px[k][c] = A.in.pos[c][base + s];
                pv[k][c] = A.in.vel[c][base + s];
            }
        }
    }

    // ---- phase 1: SRD collision of the binning these particles sit in
    if constexpr (COLL) {
        const uint32_t tc = (uint32_t)(t_now + A.coll_dt);
        const uint32_t sc = (uint32_t)A.coll_s;
        PT sh[3];
        grid_shift_of<DIM, PT>(d, tc, sc, sh);
        for (int i = tid; i < MAX_NCT; i += WG) {
            ccnt[i] = 0u;
            csv[3 * i] = 0.0; csv[3 * i + 1] = 0.0; csv[3 * i + 2] = 0.0;
        }
        __syncthreads();
        int lc[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            lc[k] = -1;
            if (!valid[k]) continue;
            int ix = bin_coord<PT>(px[k][0], (PT)0, sh[0], rr);
            if (ix >= d.Cx) ix -= d.Cx;
            int iy = bin_coord<PT>(px[k][1], (PT)d.ylo, sh[1], rr);
            if (d.ywrap && iy >= d.R) iy -= d.R;
            int iz = 0;
            if constexpr (DIM == 3) {
                iz = bin_coord<PT>(px[k][2], (PT)0, sh[2], rr);
                if (iz >= d.Cz) iz -= d.Cz;
            }
            const int lx = ix - tx * d.Tx, ly = iy - ty * d.Ty, lz = iz - tz * d.Tz;
            if (lx < 0 || lx >= d.Tx || ly < 0 || ly >= d.Ty || lz < 0 || lz >= d.Tz) {
                atomicAdd(&A.stats->misplaced, 1ull);
                continue;
            }
            const int c = lx + d.Tx * (ly + d.Ty * lz);
            lc[k] = c;
            atomicAdd(&ccnt[c], 1u);
#pragma unroll
            for (int q = 0; q < DIM; ++q) lds_add(&csv[3 * c + q], (double)pv[k][q]);
        }
        __syncthreads();
        for (int j = tid; j < d.nct; j += WG) {
            const int lx = j % d.Tx, ly = (j / d.Tx) % d.Ty, lz = j / (d.Tx * d.Ty);
            const int ix = tx * d.Tx + lx, iy = ty * d.Ty + ly, iz = tz * d.Tz + lz;
            const uint32_t nc = ccnt[j];
            if (nc == 0u || ix >= d.Cx || iy >= d.CyB || iz >= d.Cz) continue;
            const uint32_t cg = (uint32_t)(ix + d.Cx * (iy + d.CyB * iz));
            double pvv[3] = {0.0, 0.0, 0.0}, mv = 0.0;
            const bool cut = ((double)sh[1] > 0.0) && ((d.bot_wall && iy == 0) || (d.top_wall && iy == d.R));
            if (cut && (int)nc < d.ppc) {
                double z[3];
                rng_normals<DIM>(d, cg, tc, sc, P_WALL, z);
                const int nv = d.ppc - (int)nc;
                const double sdv = sqrt((double)nv * d.kT / d.mass);
#pragma unroll
                for (int q = 0; q < DIM; ++q) pvv[q] = sdv * z[q] / d.mass;
                mv = (double)nv;
            }
#pragma unroll
            for (int q = 0; q < 3; ++q) cvcm[3 * j + q] = 0.0;
#pragma unroll
            for (int q = 0; q < DIM; ++q) cvcm[3 * j + q] = (csv[3 * j + q] + pvv[q]) / ((double)nc + mv);
            const U4 w = rng_block(d, cg, tc, sc, P_ROT, 0);
            if constexpr (DIM == 2) {
                crot[3 * j] = (w.x & 1u) ? 1.0 : -1.0;
            } else {
                const double u0 = u01(w.x, w.y), u1 = u01(w.z, w.w);
                const double nz = 2.0 * u0 - 1.0, phi = 6.283185307179586 * u1;
                const double sxy = sqrt(fmax(0.0, 1.0 - nz * nz));
                double sp, cp;
                sincos(phi, &sp, &cp);
                crot[3 * j] = sxy * cp;
                crot[3 * j + 1] = sxy * sp;
                crot[3 * j + 2] = nz;
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
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                if (!valid[k]) continue;
                const int s = tid + k * WG;
#pragma unroll
                for (int q = 0; q < DIM; ++q) A.out.vel[q][base + s] = pv[k][q];
            }
            return;
        }
        __syncthreads();  // the collision arrays are reused below
    }

    if constexpr (STREAM) {
        const uint32_t ts = (uint32_t)t_now;
        const uint32_t ss = (uint32_t)A.str_s;
        PT sh[3];
        grid_shift_of<DIM, PT>(d, ts, ss, sh);
        // sample windows (node sums for the feedback, fine rows for profiles)
        const int nslab_y = d.yhi - d.ylo;
        const int wnx = (d.Tx + d.r - 1) / d.r + 2, wny = (d.Ty + d.r - 1) / d.r + 2;
        const int wnz = (DIM == 3) ? (d.Tz + d.r - 1) / d.r + 2 : 1;
        const int wx0 = (tx * d.Tx) / d.r - 1, wy0 = (ty * d.Ty) / d.r - 1;
        const int wz0 = (DIM == 3) ? (tz * d.Tz) / d.r - 1 : 0;
        const bool win_ok = wnx * wny * wnz <= MAX_WIN;
        const int wj0 = ty * d.Ty - 2, wnj = d.Ty + 4;
        const bool wj_ok = wnj <= MAX_WJ;
        const int copy = (int)(lt % NCOPY);
        for (int i = tid; i < MAX_WIN * 4; i += WG) wacc[i] = 0.0;
        for (int i = tid; i < MAX_WJ * 4; i += WG) wprof[i] = 0.0;
        if (tid < 32) dcnt[tid] = 0u;
        __syncthreads();

        const double ylo_d = (double)d.ylo, yhi_d = (double)d.yhi;
        const int rb_lo = d.buf_lo * d.r, rb_hi = d.R - d.buf_hi * d.r;
        const long long NF = (long long)d.Cx * d.NB * d.Cz;
        const double* uf = A.ufine + d.ufine_off * DIM;
        const PT dtp = (PT)d.dt;
        int code[PPT];
        uint32_t lrank[PPT], dst[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            code[k] = -1;
            if (!valid[k]) continue;
            // exchange step: redraw buffer particles about the LB velocity
            const int J0 = clampi((int)floor(((double)px[k][1] - ylo_d) * (double)d.r), 0, d.R - 1);
            if (J0 < rb_lo || J0 >= rb_hi) {
                const int I = clampi((int)floor((double)px[k][0] * (double)d.r), 0, d.Cx - 1);
                const int K = (DIM == 3) ? clampi((int)floor((double)px[k][2] * (double)d.r), 0, d.Cz - 1) : 0;
                const int Jb = (J0 < rb_lo) ? J0 : J0 - (d.R - d.NB);
                const long long fc = ((long long)K * d.NB + Jb) * d.Cx + I;
                double z[3];
                rng_normals<DIM>(d, pid[k], ts, ss, P_REINJ, z);
#pragma unroll
                for (int q = 0; q < DIM; ++q) pv[k][q] = (PT)(uf[q * NF + fc] + d.sd * z[q]);
            }
            // streaming, Eq. 3, with the body force as constant acceleration
            PT r0[3] = {px[k][0], px[k][1], px[k][2]}, v0[3] = {pv[k][0], pv[k][1], pv[k][2]};
            PT r1[3] = {r0[0], r0[1], r0[2]}, v1[3] = {v0[0], v0[1], v0[2]};
#pragma unroll
            for (int q = 0; q < DIM; ++q) {
                const PT vh = v0[q] + (PT)d.gh[q];
                r1[q] = fma_t<PT>(vh, dtp, r0[q]);
                v1[q] = v0[q] + (PT)d.gdt[q];
            }
            const bool below = (double)r1[1] < ylo_d, above = (double)r1[1] >= yhi_d;
            if (!d.ywrap && (below || above)) {
                const int wall = below ? d.bot_wall : d.top_wall;
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
                } else if (d.bot_wall || d.top_wall) {
                    q1[1] = 2.0 * Yw - q1[1];
                    w1[1] = -w1[1];
                } else {
                    q1[1] = (double)wrap_periodic<PT>(r1[1], (PT)d.ylo, (PT)(d.yhi - d.ylo));
                }
#pragma unroll
                for (int q = 0; q < DIM; ++q) { r1[q] = (PT)q1[q]; v1[q] = (PT)w1[q]; }
                if ((double)r1[1] < ylo_d) r1[1] = (PT)d.ylo;
                if ((double)r1[1] >= yhi_d) r1[1] = prev_below<PT>((PT)d.yhi, (PT)d.ylo);
            } else if (d.ywrap) {
                r1[1] = wrap_periodic<PT>(r1[1], (PT)0, (PT)d.ny);
            }
            r1[0] = wrap_periodic<PT>(r1[0], (PT)0, (PT)d.nx);
            if constexpr (DIM == 3) r1[2] = wrap_periodic<PT>(r1[2], (PT)0, (PT)d.nz);
#pragma unroll
            for (int q = 0; q < 3; ++q) { px[k][q] = r1[q]; pv[k][q] = v1[q]; }

            // samples right after streaming
            const int J = clampi((int)floor(((double)px[k][1] - ylo_d) * (double)d.r), 0, d.R - 1);
            if (A.do_fb) {
                const int ixn = clampi((int)floor((double)px[k][0]), 0, d.nx - 1);
                const int iyn = J / d.r;
                const int izn = (DIM == 3) ? clampi((int)floor((double)px[k][2]), 0, d.nz - 1) : 0;
                int ax = ixn - wx0; if (ax < 0) ax += d.nx; else if (ax >= d.nx) ax -= d.nx;
                const int ay = iyn - wy0;
                int az = izn - wz0;
                if (DIM == 3) { if (az < 0) az += d.nz; else if (az >= d.nz) az -= d.nz; }
                double vals[4] = {1.0, (double)pv[k][0], (double)pv[k][1], DIM == 3 ? (double)pv[k][2] : 0.0};
                if (win_ok && ax < wnx && ay >= 0 && ay < wny && az < wnz) {
                    double* wb = wacc + 4 * (ax + wnx * (ay + wny * az));
#pragma unroll
                    for (int q = 0; q < DIM + 1; ++q) lds_add(&wb[q], vals[q]);
                } else {
                    const long long sidx = ((long long)izn * nslab_y + iyn) * d.nx + ixn;
                    double* gb = A.acc + (d.acc_off + sidx) * 4;
#pragma unroll
                    for (int q = 0; q < DIM + 1; ++q) gl_add(&gb[q], vals[q]);
                }
            }
            if (A.do_prof) {
                double vals[4] = {1.0, (double)pv[k][0], (double)pv[k][1], DIM == 3 ? (double)pv[k][2] : 0.0};
                const int aj = J - wj0;
                if (wj_ok && aj >= 0 && aj < wnj) {
#pragma unroll
                    for (int q = 0; q < DIM + 1; ++q) lds_add(&wprof[4 * aj + q], vals[q]);
                } else {
                    double* gb = A.prof + (d.prof_off + (long long)copy * d.R + J) * 4;
#pragma unroll
                    for (int q = 0; q < DIM + 1; ++q) gl_add(&gb[q], vals[q]);
                }
            }

            // binning into the shifted grid of this MPCD step
            int ix = bin_coord<PT>(px[k][0], (PT)0, sh[0], rr);
            if (ix >= d.Cx) ix -= d.Cx;
            int iy = bin_coord<PT>(px[k][1], (PT)d.ylo, sh[1], rr);
            if (d.ywrap && iy >= d.R) iy -= d.R;
            int iz = 0;
            if constexpr (DIM == 3) {
                iz = bin_coord<PT>(px[k][2], (PT)0, sh[2], rr);
                if (iz >= d.Cz) iz -= d.Cz;
            }
            const int ntx = ix / d.Tx, nty = iy / d.Ty, ntz = iz / d.Tz;
            int dx = ntx - tx, dy = nty - ty, dz = ntz - tz;
            if (d.ntx > 2) { if (dx == d.ntx - 1) dx = -1; else if (dx == 1 - d.ntx) dx = 1; }
            if (DIM == 3 && d.ntz > 2) { if (dz == d.ntz - 1) dz = -1; else if (dz == 1 - d.ntz) dz = 1; }
            if (d.ywrap && d.nty > 2) { if (dy == d.nty - 1) dy = -1; else if (dy == 1 - d.nty) dy = 1; }
            const bool near = dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1;
            if (near) {
                code[k] = (dx + 1) + 3 * ((dy + 1) + 3 * (dz + 1));
                lrank[k] = atomicAdd(&dcnt[code[k]], 1u);
            } else {
                code[k] = 27;
                lrank[k] = atomicAdd(&dcnt[27], 1u);
                const long long Tn = d.tile_off + ntx + (long long)d.ntx * (nty + (long long)d.nty * ntz);
                const uint32_t g = atomicAdd(&A.fill_out[Tn], 1u);
                atomicAdd(&A.stats->far_moves, 1ull);
                dst[k] = g < (uint32_t)cap ? (uint32_t)(d.slot_off + (Tn - d.tile_off) * cap + g) : BAD_SLOT;
            }
        }
        __syncthreads();
        // reserve a run of slots in every neighbour tile; staging offsets
        if (tid < 27) {
            const uint32_t c = dcnt[tid];
            uint32_t g = 0u;
            if (c > 0u) {
                const int dx = tid % 3 - 1, dy = (tid / 3) % 3 - 1, dz = tid / 9 - 1;
                int nx_ = tx + dx, ny_ = ty + dy, nz_ = tz + dz;
                if (nx_ < 0) nx_ += d.ntx; else if (nx_ >= d.ntx) nx_ -= d.ntx;
                if (nz_ < 0) nz_ += d.ntz; else if (nz_ >= d.ntz) nz_ -= d.ntz;
                if (ny_ < 0) ny_ += d.nty; else if (ny_ >= d.nty) ny_ -= d.nty;
                const long long Tn = d.tile_off + nx_ + (long long)d.ntx * (ny_ + (long long)d.nty * nz_);
                g = atomicAdd(&A.fill_out[Tn], c);
                gbase[tid] = g;
                tile_of_code[tid] = (uint32_t)(Tn - d.tile_off);
            }
        }
        __syncthreads();
        // exclusive prefix of the destination counts: staging offsets
        if (tid == 0) {
            uint32_t acc = 0u;
            for (int c = 0; c < 28; ++c) { s_off[c] = acc; acc += dcnt[c]; }
            s_off[28] = acc;
        }
        // flush the sample windows
        if (A.do_fb && win_ok) {
            for (int i = tid; i < wnx * wny * wnz; i += WG) {
                const double cnt = wacc[4 * i];
                if (cnt == 0.0) continue;
                const int ax = i % wnx, ay = (i / wnx) % wny, az = i / (wnx * wny);
                int ixn = wx0 + ax; if (ixn < 0) ixn += d.nx; else if (ixn >= d.nx) ixn -= d.nx;
                const int iyn = wy0 + ay;
                int izn = wz0 + az;
                if (DIM == 3) { if (izn < 0) izn += d.nz; else if (izn >= d.nz) izn -= d.nz; }
                if (iyn < 0 || iyn >= nslab_y) continue;  // cannot happen: samples are clamped to the slab
                const long long sidx = ((long long)izn * nslab_y + iyn) * d.nx + ixn;
                double* gb = A.acc + (d.acc_off + sidx) * 4;
#pragma unroll
                for (int q = 0; q < DIM + 1; ++q) gl_add(&gb[q], wacc[4 * i + q]);
            }
        }
        if (A.do_prof && wj_ok) {
            for (int i = tid; i < wnj; i += WG) {
                const double cnt = wprof[4 * i];
                if (cnt == 0.0) continue;
                const int J = wj0 + i;
                double* gb = A.prof + (d.prof_off + (long long)copy * d.R + J) * 4;
#pragma unroll
                for (int q = 0; q < DIM + 1; ++q) gl_add(&gb[q], wprof[4 * i + q]);
            }
        }
        __syncthreads();
        // stage particles in LDS ordered by destination
        uint32_t* sdst = (uint32_t*)uni;
        uint32_t* sid = sdst + cap;
        PT* spos = (PT*)(sid + cap);
        PT* svel = spos + (size_t)DIM * cap;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (code[k] < 0) continue;
            const int c = code[k];
            const uint32_t ss_ = s_off[c] + lrank[k];
            uint32_t g;
            if (c < 27) {
                const uint32_t r_ = gbase[c] + lrank[k];
                g = r_ < (uint32_t)cap ? (uint32_t)(d.slot_off + (long long)tile_of_code[c] * cap + r_) : BAD_SLOT;
            } else {
                g = dst[k];
            }
            if (g == BAD_SLOT) atomicAdd(&A.stats->dropped, 1ull);
            sdst[ss_] = g;
            sid[ss_] = pid[k];
#pragma unroll
            for (int q = 0; q < DIM; ++q) {
                spos[(size_t)q * cap + ss_] = px[k][q];
                svel[(size_t)q * cap + ss_] = pv[k][q];
            }
        }
        __syncthreads();
        for (int i = tid; i < (int)n; i += WG) {
            const uint32_t g = sdst[i];
            if (g == BAD_SLOT) continue;
            A.out.id[g] = sid[i];
#pragma unroll
            for (int q = 0; q < DIM; ++q) {
                A.out.pos[q][g] = spos[(size_t)q * cap + i];
                A.out.vel[q][g] = svel[(size_t)q * cap + i];
            }
        }
        if (tid == 0) A.fill_in[T] = 0u;
    }
}

// ---------------------------------------------------------------------------
// Initial particles: exactly ppc per fine cell, uniform inside the cell, ids
// in cell order; velocities Maxwell-Boltzmann about the initial flow.  They
// are placed in tiles in id order (no binning is pending after init).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double poiseuille_p(const InstDesc& d, double gk, double y) {
    double nu = (d.tau - 0.5) / 3.0, H = (double)d.ny, tau = d.tau;
    return gk * y * (H - y) / (2.0 * nu) + gk * (16.0 * tau * tau - 16.0 * tau + 1.0) / (24.0 * nu);
}

template <int DIM, typename PT>
__global__ void __launch_bounds__(WG) k_part_init(const InstDesc* __restrict__ D, int n_inst, long long total,
                                                  PartPtrs<PT> P) {
    long long gid = (long long)blockIdx.x * WG + threadIdx.x;
    if (gid >= total) return;
    int ii = find_inst(D, n_inst, gid, [](const InstDesc& d) { return d.part_off; });
    const InstDesc& d = D[ii];
    const long long id = gid - d.part_off;
    const long long cl = id / d.ppc;
    const int I = (int)(cl % d.Cx);
    const int J = (int)((cl / d.Cx) % d.R);
    const int K = (int)(cl / ((long long)d.Cx * d.R));
    double u[4], z[3];
    rng_uniforms4(d, (uint32_t)id, 0u, 0u, P_INIT_POS, u);
    const double r = (double)d.r;
    const double x = ((double)I + u[0]) / r;
    const double y = (double)d.ylo + ((double)J + u[1]) / r;
    const double zz = (DIM == 3) ? ((double)K + u[2]) / r : 0.0;
    rng_normals<DIM>(d, (uint32_t)id, 0u, 0u, P_INIT_VEL, z);
    const long long tile = id / d.init_per, slot = id % d.init_per;
    const long long g = d.slot_off + tile * d.cap + slot;
    P.id[g] = (uint32_t)id;
    P.pos[0][g] = (PT)x;
    P.pos[1][g] = (PT)y;
    if (DIM == 3) P.pos[2][g] = (PT)zz;
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
        const double u0 = d.init_flow ? poiseuille_p(d, d.g[q], y) : 0.0;
        P.vel[q][g] = (PT)(u0 + d.sd * z[q]);
    }
}

__global__ void __launch_bounds__(WG) k_fill_sequential(const InstDesc* __restrict__ D, int n_inst, long long tiles,
                                                        uint32_t* fill, uint32_t* other) {
    long long T = (long long)blockIdx.x * WG + threadIdx.x;
    if (T >= tiles) return;
    int ii = find_inst(D, n_inst, T, [](const InstDesc& d) { return d.tile_off; });
    const InstDesc& d = D[ii];
    const long long lt = T - d.tile_off;
    long long c = d.Np - lt * d.init_per;
    if (c < 0) c = 0;
    if (c > d.init_per) c = d.init_per;
    fill[T] = (uint32_t)c;
    other[T] = 0u;
}

// Particles of one instance in id order (and their cell in the binning of
// (t, sub)).
template <int DIM, typename PT>
__global__ void __launch_bounds__(WG) k_gather(const InstDesc* __restrict__ D, int inst, PartPtrs<PT> P,
                                               const uint32_t* __restrict__ fill, double* pos_out,
                                               double* vel_out, int* cell_out, long long t, int sub) {
    const InstDesc& d = D[inst];
    const long long s = (long long)blockIdx.x * WG + threadIdx.x;
    if (s >= d.ntiles * d.cap) return;
    const long long lt = s / d.cap;
    const int k = (int)(s % d.cap);
    uint32_t n = fill[d.tile_off + lt];
    if (n > (uint32_t)d.cap) n = (uint32_t)d.cap;
    if ((uint32_t)k >= n) return;
    const long long g = d.slot_off + s;
    const uint32_t id = P.id[g];
    if ((long long)id >= d.Np) return;
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
        if (pos_out) pos_out[(long long)q * d.Np + id] = (double)P.pos[q][g];
        if (vel_out) vel_out[(long long)q * d.Np + id] = (double)P.vel[q][g];
    }
    if (cell_out) {
        PT sh[3];
        grid_shift_of<DIM, PT>(d, (uint32_t)t, (uint32_t)sub, sh);
        const PT rr = (PT)d.r;
        int ix = bin_coord<PT>(P.pos[0][g], (PT)0, sh[0], rr);
        if (ix >= d.Cx) ix -= d.Cx;
        int iy = bin_coord<PT>(P.pos[1][g], (PT)d.ylo, sh[1], rr);
        if (d.ywrap && iy >= d.R) iy -= d.R;
        int iz = 0;
        if (DIM == 3) {
            iz = bin_coord<PT>(P.pos[2][g], (PT)0, sh[2], rr);
            if (iz >= d.Cz) iz -= d.Cz;
        }
        cell_out[id] = ix + d.Cx * (iy + d.CyB * iz);
    }
}

template <int DIM, typename PT>
__global__ void __launch_bounds__(WG) k_cell_count(const InstDesc* __restrict__ D, int inst, PartPtrs<PT> P,
                                                   const uint32_t* __restrict__ fill, int* count, long long t,
                                                   int sub) {
    const InstDesc& d = D[inst];
    const long long s = (long long)blockIdx.x * WG + threadIdx.x;
    if (s >= d.ntiles * d.cap) return;
    const long long lt = s / d.cap;
    const int k = (int)(s % d.cap);
    uint32_t n = fill[d.tile_off + lt];
    if (n > (uint32_t)d.cap) n = (uint32_t)d.cap;
    if ((uint32_t)k >= n) return;
    const long long g = d.slot_off + s;
    PT sh[3];
    grid_shift_of<DIM, PT>(d, (uint32_t)t, (uint32_t)sub, sh);
    const PT rr = (PT)d.r;
    int ix = bin_coord<PT>(P.pos[0][g], (PT)0, sh[0], rr);
    if (ix >= d.Cx) ix -= d.Cx;
    int iy = bin_coord<PT>(P.pos[1][g], (PT)d.ylo, sh[1], rr);
    if (d.ywrap && iy >= d.R) iy -= d.R;
    int iz = 0;
    if (DIM == 3) {
        iz = bin_coord<PT>(P.pos[2][g], (PT)0, sh[2], rr);
        if (iz >= d.Cz) iz -= d.Cz;
    }
    atomicAdd(&count[ix + d.Cx * (iy + d.CyB * iz)], 1);
}

// Overwrite positions (which = 0) or velocities (1) of one instance by id.
template <int DIM, typename PT>
__global__ void __launch_bounds__(WG) k_set_field(const InstDesc* __restrict__ D, int inst, PartPtrs<PT> P,
                                                  const uint32_t* __restrict__ fill, int which,
                                                  const double* __restrict__ src) {
    const InstDesc& d = D[inst];
    const long long s = (long long)blockIdx.x * WG + threadIdx.x;
    if (s >= d.ntiles * d.cap) return;
    const long long lt = s / d.cap;
    const int k = (int)(s % d.cap);
    uint32_t n = fill[d.tile_off + lt];
    if (n > (uint32_t)d.cap) n = (uint32_t)d.cap;
    if ((uint32_t)k >= n) return;
    const long long g = d.slot_off + s;
    const uint32_t id = P.id[g];
    if ((long long)id >= d.Np) return;
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
        const PT v = (PT)src[(long long)q * d.Np + id];
        if (which == 0) P.pos[q][g] = v; else P.vel[q][g] = v;
    }
}

__global__ void __launch_bounds__(WG) k_zero(uint32_t* p, long long nwords) {
    const long long i = (long long)blockIdx.x * WG + threadIdx.x;
    if (i < nwords) p[i] = 0u;
}

// Sum of the NCOPY profile replicas of one instance: out[R][4].
__global__ void __launch_bounds__(WG) k_profile_reduce(const InstDesc* __restrict__ D, int inst,
                                                       const double* __restrict__ prof, double* out) {
    const InstDesc& d = D[inst];
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i >= d.R * 4) return;
    const int J = i / 4, q = i % 4;
    double s = 0.0;
    for (int c = 0; c < NCOPY; ++c) s += prof[(d.prof_off + (long long)c * d.R + J) * 4 + q];
    out[i] = s;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(long long n) { return (unsigned)((n + WG - 1) / WG); }

template <typename PT>
static PartPtrs<PT> typed(const PartBuf& b) {
    PartPtrs<PT> p;
    for (int q = 0; q < 3; ++q) { p.pos[q] = (PT*)b.pos[q]; p.vel[q] = (PT*)b.vel[q]; }
    p.id = b.id;
    return p;
}

template <int DIM, typename PT, int PPT, int MODE>
static hipError_t launch_p4(const ParticleLaunch& L, hipStream_t s) {
    PArgs<PT> a;
    a.D = L.D; a.n_inst = L.n_inst;
    a.in = typed<PT>(L.in); a.out = typed<PT>(L.out);
    a.fill_in = L.fill_in; a.fill_out = L.fill_out; a.tile_inst = L.tile_inst;
    a.ufine = L.ufine; a.acc = L.acc; a.prof = L.prof; a.stats = L.stats; a.clock = L.clock;
    a.coll_dt = L.coll_dt; a.coll_s = L.coll_s; a.str_s = L.str_s;
    a.do_fb = L.do_fb; a.do_prof = L.do_prof; a.diag_inst = L.diag_inst; a.cell_vcm = L.cell_vcm;
    hipLaunchKernelGGL((k_particles<DIM, PT, PPT, MODE>), dim3((unsigned)L.tiles), dim3(WG), L.lds_bytes, s, a);
    return hipGetLastError();
}

template <int DIM, typename PT, int PPT>
static hipError_t launch_p3(const ParticleLaunch& L, hipStream_t s) {
    switch (L.mode) {
        case 1: return launch_p4<DIM, PT, PPT, 1>(L, s);
        case 2: return launch_p4<DIM, PT, PPT, 2>(L, s);
        case 3: return launch_p4<DIM, PT, PPT, 3>(L, s);
        default: return hipErrorInvalidValue;
    }
}

template <int DIM, typename PT>
static hipError_t launch_p2(const ParticleLaunch& L, hipStream_t s) {
    if (L.ppt <= 2) return launch_p3<DIM, PT, 2>(L, s);
    if (L.ppt <= 4) return launch_p3<DIM, PT, 4>(L, s);
    if (L.ppt <= 8) return launch_p3<DIM, PT, 8>(L, s);
    return hipErrorInvalidValue;
}

hipError_t launch_particles(const ParticleLaunch& L, hipStream_t s) {
    if (L.tiles <= 0) return hipSuccess;
    if (L.dim == 2 && L.part_fp == 64) return launch_p2<2, double>(L, s);
    if (L.dim == 2) return launch_p2<2, float>(L, s);
    if (L.part_fp == 64) return launch_p2<3, double>(L, s);
    return launch_p2<3, float>(L, s);
}

hipError_t launch_part_init(int dim, int part_fp, const InstDesc* D, int n_inst, long long total, PartBuf buf,
                            hipStream_t s) {
    if (total <= 0) return hipSuccess;
    dim3 g(nblk(total)), b(WG);
    if (dim == 2 && part_fp == 64) hipLaunchKernelGGL((k_part_init<2, double>), g, b, 0, s, D, n_inst, total, typed<double>(buf));
    else if (dim == 2) hipLaunchKernelGGL((k_part_init<2, float>), g, b, 0, s, D, n_inst, total, typed<float>(buf));
    else if (part_fp == 64) hipLaunchKernelGGL((k_part_init<3, double>), g, b, 0, s, D, n_inst, total, typed<double>(buf));
    else hipLaunchKernelGGL((k_part_init<3, float>), g, b, 0, s, D, n_inst, total, typed<float>(buf));
    return hipGetLastError();
}

hipError_t launch_fill_sequential(const InstDesc* D, int n_inst, long long tiles, uint32_t* fill,
                                  uint32_t* fill_other, hipStream_t s) {
    if (tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_sequential, dim3(nblk(tiles)), dim3(WG), 0, s, D, n_inst, tiles, fill, fill_other);
    return hipGetLastError();
}

hipError_t launch_gather(int dim, int part_fp, const InstDesc* D, int inst, PartBuf buf, const uint32_t* fill,
                         double* pos_out, double* vel_out, int* cell_out, long long slots, long long t, int sub,
                         hipStream_t s) {
    if (slots <= 0) return hipSuccess;
    dim3 g(nblk(slots)), b(WG);
    if (dim == 2 && part_fp == 64) hipLaunchKernelGGL((k_gather<2, double>), g, b, 0, s, D, inst, typed<double>(buf), fill, pos_out, vel_out, cell_out, t, sub);
    else if (dim == 2) hipLaunchKernelGGL((k_gather<2, float>), g, b, 0, s, D, inst, typed<float>(buf), fill, pos_out, vel_out, cell_out, t, sub);
    else if (part_fp == 64) hipLaunchKernelGGL((k_gather<3, double>), g, b, 0, s, D, inst, typed<double>(buf), fill, pos_out, vel_out, cell_out, t, sub);
    else hipLaunchKernelGGL((k_gather<3, float>), g, b, 0, s, D, inst, typed<float>(buf), fill, pos_out, vel_out, cell_out, t, sub);
    return hipGetLastError();
}

hipError_t launch_cell_count(int dim, int part_fp, const InstDesc* D, int inst, PartBuf buf, const uint32_t* fill,
                             int* count_out, long long slots, long long t, int sub, hipStream_t s) {
    if (slots <= 0) return hipSuccess;
    dim3 g(nblk(slots)), b(WG);
    if (dim == 2 && part_fp == 64) hipLaunchKernelGGL((k_cell_count<2, double>), g, b, 0, s, D, inst, typed<double>(buf), fill, count_out, t, sub);
    else if (dim == 2) hipLaunchKernelGGL((k_cell_count<2, float>), g, b, 0, s, D, inst, typed<float>(buf), fill, count_out, t, sub);
    else if (part_fp == 64) hipLaunchKernelGGL((k_cell_count<3, double>), g, b, 0, s, D, inst, typed<double>(buf), fill, count_out, t, sub);
    else hipLaunchKernelGGL((k_cell_count<3, float>), g, b, 0, s, D, inst, typed<float>(buf), fill, count_out, t, sub);
    return hipGetLastError();
}

hipError_t launch_set_field(int dim, int part_fp, const InstDesc* D, int inst, PartBuf buf, const uint32_t* fill,
                            int which, const double* src, long long slots, hipStream_t s) {
    if (slots <= 0) return hipSuccess;
    dim3 g(nblk(slots)), b(WG);
    if (dim == 2 && part_fp == 64) hipLaunchKernelGGL((k_set_field<2, double>), g, b, 0, s, D, inst, typed<double>(buf), fill, which, src);
    else if (dim == 2) hipLaunchKernelGGL((k_set_field<2, float>), g, b, 0, s, D, inst, typed<float>(buf), fill, which, src);
    else if (part_fp == 64) hipLaunchKernelGGL((k_set_field<3, double>), g, b, 0, s, D, inst, typed<double>(buf), fill, which, src);
    else hipLaunchKernelGGL((k_set_field<3, float>), g, b, 0, s, D, inst, typed<float>(buf), fill, which, src);
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    const long long nw = (long long)(bytes / 4);
    if (nw <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(nblk(nw)), dim3(WG), 0, s, (uint32_t*)p, nw);
    return hipGetLastError();
}

hipError_t launch_profile_reduce(const InstDesc* D, int inst, int R, const double* prof, double* out, hipStream_t s) {
    if (R <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_profile_reduce, dim3(nblk(4LL * R)), dim3(WG), 0, s, D, inst, prof, out);
    return hipGetLastError();
}

}  // namespace lbmpcd
