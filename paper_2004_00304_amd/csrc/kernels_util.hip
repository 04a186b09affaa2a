// kernels_util.hip -- initialisation, state transfer and diagnostic kernels
// of the particle store (not on the per-step hot path).
#include "common.hpp"
#include "launch.hpp"

namespace lbmpcd {

// ---------------------------------------------------------------------------
// Initial particles: exactly ppc per fine cell, uniform inside the cell, ids
// in cell order; velocities Maxwell-Boltzmann about the initial flow.  Each
// particle starts in the tile of its unshifted cell (no collision is pending
// after init).
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
    rng_uniforms4(key_of(d), (uint32_t)id, 0u, 0u, P_INIT_POS, u);
    const double r = (double)d.r;
    const double x = ((double)I + u[0]) / r;
    const double y = (double)d.ylo + ((double)J + u[1]) / r;
    const double zz = (DIM == 3) ? ((double)K + u[2]) / r : 0.0;
    rng_normals<DIM>(key_of(d), (uint32_t)id, 0u, 0u, P_INIT_VEL, z);
    // the tile of the unshifted cell; slots ranked over the tile's slab cells
    const int tx = I / d.Tx, ty = J / d.Ty, tz = K / d.Tz;
    const int cx = min(d.Tx, d.Cx - tx * d.Tx), cy = min(d.Ty, d.R - ty * d.Ty), cz = min(d.Tz, d.Cz - tz * d.Tz);
    (void)cz;
    const long long tile = tx + (long long)d.ntx * (ty + (long long)d.nty * tz);
    const long long lcell = (I - tx * d.Tx) + (long long)cx * ((J - ty * d.Ty) + (long long)cy * (K - tz * d.Tz));
    const long long slot = lcell * d.ppc + id % d.ppc;
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
    const int tx = (int)(lt % d.ntx), ty = (int)((lt / d.ntx) % d.nty), tz = (int)(lt / ((long long)d.ntx * d.nty));
    const int cx = max(0, min(d.Tx, d.Cx - tx * d.Tx));
    const int cy = max(0, min(d.Ty, d.R - ty * d.Ty));
    const int cz = max(0, min(d.Tz, d.Cz - tz * d.Tz));
    fill[T] = (uint32_t)((long long)cx * cy * cz * d.ppc);
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
        const int iy = bin_row<PT>(d, P.pos[1][g], sh[1], rr);
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
    const int iy = bin_row<PT>(d, P.pos[1][g], sh[1], rr);
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
    for (int c = 0; c < NCOPY; ++c) {
        const double* v = &prof[(d.prof_off + (long long)c * d.R + J) * 4 + q];
        s += d.det ? fix_bits(v) : *v;  // fixed-point sums in the deterministic mode
    }
    out[i] = s;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(long long n) { return (unsigned)((n + WG - 1) / WG); }


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

// Exclusive prefix sum of n ints in place, by one workgroup walking the
// array in chunks (a diagnostic field; n is the cell count of one channel).
__global__ void __launch_bounds__(WG) k_exclusive_scan(int* a, long long n) {
    __shared__ int part[WG];
    __shared__ int carry;
    const int tid = threadIdx.x;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (long long c0 = 0; c0 < n; c0 += WG) {
        const long long i = c0 + tid;
        const int v = i < n ? a[i] : 0;
        part[tid] = v;
        __syncthreads();
        // Hillis-Steele inclusive scan of the chunk
        for (int o = 1; o < WG; o <<= 1) {
            const int add = tid >= o ? part[tid - o] : 0;
            __syncthreads();
            part[tid] += add;
            __syncthreads();
        }
        if (i < n) a[i] = carry + part[tid] - v;
        __syncthreads();
        if (tid == WG - 1) carry += part[WG - 1];
        __syncthreads();
    }
}

hipError_t launch_exclusive_scan(int* a, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_exclusive_scan, dim3(1), dim3(WG), 0, s, a, n);
    return hipGetLastError();
}

// Mean particle velocity per slab node from the per-node sample sums
// [count, sum v_x, sum v_y, sum v_z]: out[q][node], zero where no particle.
__global__ void __launch_bounds__(WG) k_node_mean(const double* acc, long long nslab, int dim, int det,
                                                  double* out) {
    const long long i = (long long)blockIdx.x * WG + threadIdx.x;
    if (i >= nslab) return;
    const double* a = acc + 4 * i;
    double v[4];
    for (int q = 0; q < 4; ++q) v[q] = det ? fix_bits(a + q) : a[q];  // fixed point in the deterministic mode
    for (int q = 0; q < dim; ++q) out[(long long)q * nslab + i] = v[0] > 0.0 ? v[1 + q] / v[0] : 0.0;
}

hipError_t launch_node_mean(const double* acc, long long nslab, int dim, int det, double* out, hipStream_t s) {
    if (nslab <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_node_mean, dim3(nblk(nslab)), dim3(WG), 0, s, acc, nslab, dim, det, out);
    return hipGetLastError();
}

hipError_t launch_profile_reduce(const InstDesc* D, int inst, int R, const double* prof, double* out, hipStream_t s) {
    if (R <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_profile_reduce, dim3(nblk(4LL * R)), dim3(WG), 0, s, D, inst, prof, out);
    return hipGetLastError();
}

}  // namespace lbmpcd
