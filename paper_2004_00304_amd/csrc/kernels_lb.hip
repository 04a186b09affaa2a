// kernels_lb.hip -- lattice-Boltzmann kernels for gfx950.
//
// k_lb_step: one thread per node; reads the Q post-stream populations of its
// node (SoA, coalesced along x), applies the BGK collision with Guo forcing
// (Eq. 1-2 with a constant body force) in FP64, and pushes every
// post-collision population to the neighbour along c_i, or back into the
// opposite direction of the same node where the link crosses a wall
// (half-way bounce-back).  HBM-bound: one read and one write of Q values.
//
// k_band: per node of the rows the coupling needs; at interior slab nodes
// (feedback) moves the node's running mean of the MPCD velocity towards the
// last LB step's sample mean and projects the populations onto the
// equilibrium at that mean, clears the sample sums, and stores the node
// velocity for the interpolation; with the Chapman-Enskog exchange also the
// node's tensor T = (nu_x m/kT) dev S, S the BGK strain rate from the
// non-equilibrium second moment.  A band node with rho <= 0 or non-finite
// moments is counted as an invalid state.
//
// k_interp: per buffer fine cell, bi/trilinear interpolation of the node
// velocity (and T) to the cell centre (Alg. 2).
#include "common.hpp"
#include "launch.hpp"

namespace lbmpcd {

template <int DIM>
__device__ __forceinline__ void equilibrium_guo(const double* f, double omega, double src, const double g[3],
                                                double* fs) {
    using L = Lat<DIM>;
    constexpr int Q = L::Q;
    // Moments.  Lattice components are 0 or +-1: only the nonzero ones enter
    // a sum, as additions or subtractions (the dropped products are zeros,
    // which would leave every sum unchanged).
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        rho += f[i];
        const int c[3] = {L::cx[i], L::cy[i], L::cz[i]};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (c[k] > 0) j[k] += f[i];
            if (c[k] < 0) j[k] -= f[i];
        }
    }
    const double inv = 1.0 / rho;
    const double u[3] = {j[0] * inv + 0.5 * g[0], j[1] * inv + 0.5 * g[1], j[2] * inv + 0.5 * g[2]};
    const double F[3] = {rho * g[0], rho * g[1], rho * g[2]};
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double uu15 = 1.5 * uu;
    // Guo forcing (3 (c_k - u_k) + 9 (c.u) c_k) F_k per component: the
    // c_k = 0 terms are the same for every direction, and 3 (c_k - u_k) takes
    // two values for c_k = +-1
    double T0[3], Ap[3], Am[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T0[k] = (3.0 * (0.0 - u[k])) * F[k];
        Ap[k] = 3.0 * (1.0 - u[k]);
        Am[k] = 3.0 * (-1.0 - u[k]);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int c[3] = {L::cx[i], L::cy[i], L::cz[i]};
        // c.u over the nonzero components, in component order
        double cu = 0.0;
        bool first = true;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (c[k] == 0) continue;
            const double t = c[k] > 0 ? u[k] : -u[k];
            cu = first ? t : cu + t;
            first = false;
        }
        const double feq = (L::w[i] * rho) * (((1.0 + 3.0 * cu) + (4.5 * cu) * cu) - uu15);
        const double cu9 = 9.0 * cu;
        double Fi = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double t;
            if (c[k] == 0) t = T0[k];
            else if (c[k] > 0) t = (Ap[k] + cu9) * F[k];
            else t = (Am[k] - cu9) * F[k];
            Fi += t;
        }
        Fi *= L::w[i];
        fs[i] = f[i] - omega * (f[i] - feq) + src * Fi;
    }
}

template <int DIM>
__device__ __forceinline__ void feq_of(double rho, double u0, double u1, double u2, double* feq) {
    using L = Lat<DIM>;
    double uu = u0 * u0 + u1 * u1 + u2 * u2;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        double cu = (double)L::cx[i] * u0 + (double)L::cy[i] * u1 + (double)L::cz[i] * u2;
        feq[i] = L::w[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

template <int DIM, typename LT>
__global__ void __launch_bounds__(WG) k_lb_step(const InstDesc* __restrict__ D, int n_inst, long long total,
                                                const LT* __restrict__ fin, LT* __restrict__ fout,
                                                long long* __restrict__ clock, double* __restrict__ shifts, int S) {
    using L = Lat<DIM>;
    constexpr int Q = L::Q;
    if (blockIdx.x == 0) {
        // advance the LB step counter and draw the grid shifts of the new step
        // for every instance and MPCD step (slot = step parity)
        const long long t_new = clock[0] + 1;
        __syncthreads();
        if (threadIdx.x == 0) clock[0] = t_new;
        for (int i = threadIdx.x; i < n_inst * S; i += WG) {
            const int inst = i / S, s = i % S;
            double sh[3];
            grid_shift_of<DIM, double>(D[inst], (uint32_t)t_new, (uint32_t)s, sh);
            double* o = shifts + (((long long)inst * 2 + (t_new & 1)) * S + s) * 3;
            o[0] = sh[0]; o[1] = sh[1]; o[2] = sh[2];
        }
    }
    long long gid = (long long)blockIdx.x * WG + threadIdx.x;
    if (gid >= total) return;
    int ii = find_inst(D, n_inst, gid, [](const InstDesc& d) { return d.node_off; });
    const InstDesc& d = D[ii];
    long long n = gid - d.node_off;
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const long long N = d.N;
    int x, y, z;
    if (N < (1LL << 31)) {  // node coordinates in 32-bit arithmetic
        const uint32_t n32 = (uint32_t)n, row = n32 / (uint32_t)nx;
        x = (int)(n32 - row * (uint32_t)nx);
        y = (int)(row % (uint32_t)ny);
        z = (int)(row / (uint32_t)ny);
    } else {
        x = (int)(n % nx);
        y = (int)((n / nx) % ny);
        z = (int)(n / ((long long)nx * ny));
    }
    const LT* f_in = fin + d.node_off * Q;
    LT* f_out = fout + d.node_off * Q;
    const long long sxy = (long long)nx * ny;
    // Rows that touch neither a y nor a z face stream with offsets that are
    // the same for every node of the row (only x wraps): each population
    // array is addressed as a uniform base plus a 32-bit byte offset.  For a
    // channel whose x extent is a multiple of 64 a wave lies in one row, so
    // the test is uniform across the wave.
    const bool fast = N * (long long)sizeof(LT) < (1LL << 32) && y > 0 && y < ny - 1 &&
                      (DIM == 2 || (z > 0 && z < nz - 1));
    const uint32_t nb = (uint32_t)n * (uint32_t)sizeof(LT);
    const size_t qbytes = (size_t)N * sizeof(LT);
    double f[Q], fs[Q];
    if (fast) {
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] = (double)*(const LT*)((const unsigned char*)f_in + i * qbytes + nb);
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] = (double)f_in[i * N + n];
    }
    double g[3] = {d.g[0], d.g[1], d.g[2]};
    equilibrium_guo<DIM>(f, d.omega, d.src, g, fs);
    if (fast) {
        const int rowb = (int)(n - x);  // node index of x = 0 in this row
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            int xd = x + L::cx[i];
            if (L::cx[i] < 0 && xd < 0) xd += nx;
            if (L::cx[i] > 0 && xd >= nx) xd -= nx;
            const int nd = rowb + xd + L::cy[i] * nx + L::cz[i] * (int)sxy;
            *(LT*)((unsigned char*)f_out + i * qbytes + (uint32_t)nd * (uint32_t)sizeof(LT)) = (LT)fs[i];
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int yd = y + L::cy[i];
        if (d.walls_y && (yd < 0 || yd >= ny)) {
            f_out[L::opp[i] * N + n] = (LT)fs[i];
            continue;
        }
        if (yd < 0) yd += ny; else if (yd >= ny) yd -= ny;
        int xd = x + L::cx[i];
        if (xd < 0) xd += nx; else if (xd >= nx) xd -= nx;
        int zd = z;
        if constexpr (DIM == 3) {
            zd = z + L::cz[i];
            if (zd < 0) zd += nz; else if (zd >= nz) zd -= nz;
        }
        f_out[i * N + (long long)zd * sxy + (long long)yd * nx + xd] = (LT)fs[i];
    }
}

// Feedback projection, sample reset and node velocity of the band rows.
// fbu[k * fb_stride + slab node] holds the running mean of the MPCD velocity
// that the feedback projects.
template <int DIM, typename LT>
__global__ void __launch_bounds__(WG) k_band(const InstDesc* __restrict__ D, int n_inst, long long total,
                                             LT* __restrict__ f, double* __restrict__ acc,
                                             double* __restrict__ fbu, long long fb_stride,
                                             double* __restrict__ ub, double* __restrict__ tb,
                                             DevStats* __restrict__ stats, int do_feedback) {
    using L = Lat<DIM>;
    constexpr int Q = L::Q;
    long long gid = (long long)blockIdx.x * WG + threadIdx.x;
    if (gid >= total) return;
    int ii = find_inst(D, n_inst, gid, [](const InstDesc& d) { return d.band_off; });
    const InstDesc& d = D[ii];
    long long b = gid - d.band_off;
    const int nx = d.nx;
    int x = (int)(b % nx);
    int yb = (int)((b / nx) % d.nyb);
    int z = (int)(b / ((long long)nx * d.nyb));
    int y = d.by0 + yb;
    long long n = ((long long)z * d.ny + y) * nx + x;
    LT* fp = f + d.node_off * Q;
    const long long N = d.N;
    double fl[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) fl[i] = (double)fp[i * N + n];
    if (do_feedback && y >= d.ylo && y < d.yhi) {
        long long s = ((long long)z * (d.yhi - d.ylo) + (y - d.ylo)) * nx + x;
        double* a = acc + (d.acc_off + s) * 4;
        // fixed-point sums in the deterministic mode
        const double cnt = d.det ? fix_bits(a) : a[0], s0 = d.det ? fix_bits(a + 1) : a[1];
        const double s1 = d.det ? fix_bits(a + 2) : a[2], s2 = d.det ? fix_bits(a + 3) : a[3];
        a[0] = 0.0; a[1] = 0.0; a[2] = 0.0; a[3] = 0.0;
        if (d.feedback && y >= d.ylo + d.buf_lo && y < d.yhi - d.buf_hi && cnt > 0.0) {
            double rho = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) rho += fl[i];
            // running mean over LB steps of the node's sample means (weight
            // fb_lam per step; fb_lam = 1 projects the last sample alone)
            double* e = fbu + d.acc_off + s;
            const double lam = d.fb_lam;
            const double e0 = (1.0 - lam) * e[0] + lam * (s0 / cnt);
            const double e1 = (1.0 - lam) * e[fb_stride] + lam * (s1 / cnt);
            const double e2 = (1.0 - lam) * e[2 * fb_stride] + lam * (DIM == 3 ? s2 / cnt : 0.0);
            e[0] = e0;
            e[fb_stride] = e1;
            e[2 * fb_stride] = e2;
            double u0 = e0 - 0.5 * d.g[0];
            double u1 = e1 - 0.5 * d.g[1];
            double u2 = e2 - 0.5 * d.g[2];
            feq_of<DIM>(rho, u0, u1, u2, fl);
#pragma unroll
            for (int i = 0; i < Q; ++i) fp[i * N + n] = (LT)fl[i];
            // the velocity below is taken from the stored (rounded) values
#pragma unroll
            for (int i = 0; i < Q; ++i) fl[i] = (double)(LT)fl[i];
        }
    }
    double rho = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        rho += fl[i];
        j0 += fl[i] * (double)L::cx[i];
        j1 += fl[i] * (double)L::cy[i];
        j2 += fl[i] * (double)L::cz[i];
    }
    const long long NBd = (long long)nx * d.nyb * d.nz;
    double* u = ub + d.band_off * 3;
    const double ux = j0 / rho + 0.5 * d.g[0];
    const double uy = j1 / rho + 0.5 * d.g[1];
    const double uz = j2 / rho + 0.5 * d.g[2];
    if (!(rho > 0.0 && isfinite(rho) && isfinite(ux) && isfinite(uy) && isfinite(uz)))
        atomicAdd(&stats->bad_state, 1ull);
    u[b] = ux;
    u[NBd + b] = uy;
    u[2 * NBd + b] = uz;
    if (tb == nullptr || !d.ce) return;
    // Chapman-Enskog tensor: non-equilibrium second moment about the
    // physical velocity, its deviatoric part, scaled
    double pxx = 0.0, pyy = 0.0, pzz = 0.0, pxy = 0.0, pxz = 0.0, pyz = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double cx = (double)L::cx[i], cy = (double)L::cy[i], cz = (double)L::cz[i];
        pxx += fl[i] * (cx * cx);
        pyy += fl[i] * (cy * cy);
        pxy += fl[i] * (cx * cy);
        if constexpr (DIM == 3) {
            pzz += fl[i] * (cz * cz);
            pxz += fl[i] * (cx * cz);
            pyz += fl[i] * (cy * cz);
        }
    }
    const double cs2r = rho / 3.0;
    double sxx = -(pxx - cs2r - rho * ux * ux) / rho;
    double syy = -(pyy - cs2r - rho * uy * uy) / rho;
    double szz = DIM == 3 ? -(pzz - cs2r - rho * uz * uz) / rho : 0.0;
    const double sxy = -(pxy - rho * ux * uy) / rho;
    const double sxz = DIM == 3 ? -(pxz - rho * ux * uz) / rho : 0.0;
    const double syz = DIM == 3 ? -(pyz - rho * uy * uz) / rho : 0.0;
    const double tr = (sxx + syy + szz) / (double)DIM;
    sxx -= tr;
    syy -= tr;
    if constexpr (DIM == 3) szz -= tr;
    const double c = d.ce_scale;
    double* t = tb + d.band_off * CE_NT;
    t[b] = c * sxx;
    t[NBd + b] = c * syy;
    t[2 * NBd + b] = c * szz;
    t[3 * NBd + b] = c * sxy;
    t[4 * NBd + b] = c * sxz;
    t[5 * NBd + b] = c * syz;
}

// One interpolation axis: lower/upper node and weights.  Periodic axes wrap;
// on a walled axis the missing neighbour is the wall with zero velocity.
__device__ __forceinline__ void interp_axis(int Lx, int periodic, double X, int& i0, int& i1, double& w0,
                                            double& w1) {
    double xs = X - 0.5;
    double fl = floor(xs);
    int j0 = (int)fl;
    double wx = xs - fl;
    int j1 = j0 + 1;
    if (periodic) {
        // X lies in [0, Lx) (a cell centre), so j0 >= -1 and j1 <= Lx
        if (j0 < 0) j0 += Lx;
        if (j1 >= Lx) j1 -= Lx;
        i0 = j0; i1 = j1; w0 = 1.0 - wx; w1 = wx;
        return;
    }
    if (j0 < 0) {
        i0 = -1; i1 = 0; w0 = 0.0; w1 = 2.0 * X;
    } else if (j1 > Lx - 1) {
        i0 = Lx - 1; i1 = -1; w0 = 2.0 * (Lx - X); w1 = 0.0;
    } else {
        i0 = j0; i1 = j1; w0 = 1.0 - wx; w1 = wx;
    }
}

// bi/trilinear value of node field fld (band layout) at the weights below;
// a missing node (the wall) contributes zero
template <int DIM>
__device__ __forceinline__ double interp_value(const InstDesc& d, const double* fld, const int ix[2], const int iy[2],
                                               const int iz[2], const double wx[2], const double wy[2],
                                               const double wz[2]) {
    double val[2] = {0.0, 0.0};
#pragma unroll
    for (int c = 0; c < (DIM == 3 ? 2 : 1); ++c) {
        double row[2];
#pragma unroll
        for (int bb = 0; bb < 2; ++bb) {
            double a0 = 0.0, a1 = 0.0;
            if (iy[bb] >= 0) {
                long long base = ((long long)iz[c] * d.nyb + (iy[bb] - d.by0)) * d.nx;
                a0 = fld[base + ix[0]];
                a1 = fld[base + ix[1]];
            }
            row[bb] = wx[0] * a0 + wx[1] * a1;
        }
        val[c] = wy[0] * row[0] + wy[1] * row[1];
    }
    return (DIM == 3) ? wz[0] * val[0] + wz[1] * val[1] : val[0];
}

template <int DIM>
__global__ void __launch_bounds__(WG) k_interp(const InstDesc* __restrict__ D, int n_inst, long long total,
                                               const double* __restrict__ ub, double* __restrict__ uf,
                                               const double* __restrict__ tb, double* __restrict__ tf) {
    long long gid = (long long)blockIdx.x * WG + threadIdx.x;
    if (gid >= total) return;
    int ii = find_inst(D, n_inst, gid, [](const InstDesc& d) { return d.ufine_off; });
    const InstDesc& d = D[ii];
    long long q = gid - d.ufine_off;
    const int Cx = d.Cx, NB = d.NB;
    int I, Jb, K;
    if (q < 0x7FFFFFFFLL) {
        // 32-bit decode (an instance's buffer cells number fewer than 2^31
        // unless it is enormous)
        const uint32_t qu = (uint32_t)q, row = qu / (uint32_t)Cx;
        I = (int)(qu - row * (uint32_t)Cx);
        K = (int)(row / (uint32_t)NB);
        Jb = (int)(row - (uint32_t)K * (uint32_t)NB);
    } else {
        I = (int)(q % Cx);
        Jb = (int)((q / Cx) % NB);
        K = (int)(q / ((long long)Cx * NB));
    }
    int J = (Jb < d.buf_lo * d.r) ? Jb : Jb + (d.R - NB);
    const double r = (double)d.r;
    double X = ((double)I + 0.5) / r;
    double Y = (double)d.ylo + ((double)J + 0.5) / r;
    double Z = (DIM == 3) ? ((double)K + 0.5) / r : 0.5;
    int ix[2], iy[2], iz[2];
    double wx[2], wy[2], wz[2];
    interp_axis(d.nx, 1, X, ix[0], ix[1], wx[0], wx[1]);
    interp_axis(d.ny, !d.walls_y, Y, iy[0], iy[1], wy[0], wy[1]);
    if (DIM == 3) {
        interp_axis(d.nz, 1, Z, iz[0], iz[1], wz[0], wz[1]);
    } else {
        iz[0] = 0; iz[1] = 0; wz[0] = 1.0; wz[1] = 0.0;
    }
    const long long NBd = (long long)d.nx * d.nyb * d.nz;
    const double* u = ub + d.band_off * 3;
    const long long NF = (long long)Cx * NB * d.Cz;
    double* out = uf + d.ufine_off * DIM;
#pragma unroll
    for (int k = 0; k < DIM; ++k) out[k * NF + q] = interp_value<DIM>(d, u + k * NBd, ix, iy, iz, wx, wy, wz);
    if (tf == nullptr || !d.ce) return;
    const double* t = tb + d.band_off * CE_NT;
    double* tout = tf + d.ufine_off * CE_NT;
#pragma unroll
    for (int k = 0; k < CE_NT; ++k) tout[k * NF + q] = interp_value<DIM>(d, t + k * NBd, ix, iy, iz, wx, wy, wz);
}

// LB initial state: equilibrium at rho0 and the initial flow (physical
// velocity = first moment + g/2).
__device__ __forceinline__ double poiseuille(const InstDesc& d, double gk, double y) {
    double nu = (d.tau - 0.5) / 3.0, H = (double)d.ny, tau = d.tau;
    return gk * y * (H - y) / (2.0 * nu) + gk * (16.0 * tau * tau - 16.0 * tau + 1.0) / (24.0 * nu);
}

template <int DIM, typename LT>
__global__ void __launch_bounds__(WG) k_lb_init(const InstDesc* __restrict__ D, int n_inst, long long total,
                                                LT* __restrict__ f, double* __restrict__ fbu, long long fb_stride) {
    using L = Lat<DIM>;
    long long gid = (long long)blockIdx.x * WG + threadIdx.x;
    if (gid >= total) return;
    int ii = find_inst(D, n_inst, gid, [](const InstDesc& d) { return d.node_off; });
    const InstDesc& d = D[ii];
    long long n = gid - d.node_off;
    int y = (int)((n / d.nx) % d.ny);
    double u[3];
    for (int k = 0; k < 3; ++k) {
        double u0 = d.init_flow ? poiseuille(d, d.g[k], y + 0.5) : 0.0;
        u[k] = u0 - 0.5 * d.g[k];
    }
    double feq[L::Q];
    feq_of<DIM>(d.rho0, u[0], u[1], u[2], feq);
    LT* fp = f + d.node_off * L::Q;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) fp[i * d.N + n] = (LT)feq[i];
    // the feedback's running mean starts at the node's initial velocity
    if (fbu != nullptr && d.mpcd && y >= d.ylo && y < d.yhi) {
        const int x = (int)(n % d.nx), z = (int)(n / ((long long)d.nx * d.ny));
        const long long sn = d.acc_off + ((long long)z * (d.yhi - d.ylo) + (y - d.ylo)) * d.nx + x;
#pragma unroll
        for (int k = 0; k < 3; ++k) fbu[k * fb_stride + sn] = u[k] + 0.5 * d.g[k];
    }
}

// Moments of the post-stream populations of one instance: rho, physical u,
// Pi = sum f (c c - I/3).
template <int DIM, typename LT>
__global__ void __launch_bounds__(WG) k_moments(const InstDesc* __restrict__ D, int inst,
                                                const LT* __restrict__ f, double* __restrict__ rho_out,
                                                double* __restrict__ u_out, double* __restrict__ pi_out) {
    using L = Lat<DIM>;
    constexpr int Q = L::Q;
    const InstDesc& d = D[inst];
    long long n = (long long)blockIdx.x * WG + threadIdx.x;
    if (n >= d.N) return;
    const LT* fp = f + d.node_off * Q;
    double fl[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) fl[i] = (double)fp[i * d.N + n];
    double rho = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        rho += fl[i];
        j0 += fl[i] * (double)L::cx[i];
        j1 += fl[i] * (double)L::cy[i];
        j2 += fl[i] * (double)L::cz[i];
    }
    if (rho_out) rho_out[n] = rho;
    if (u_out) {
        u_out[n] = j0 / rho + 0.5 * d.g[0];
        u_out[d.N + n] = j1 / rho + 0.5 * d.g[1];
        u_out[2 * d.N + n] = j2 / rho + 0.5 * d.g[2];
    }
    if (pi_out) {
        const int A[6] = {0, 1, 2, 0, 0, 1}, B[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int ca = A[m] == 0 ? L::cx[i] : (A[m] == 1 ? L::cy[i] : L::cz[i]);
                const int cb = B[m] == 0 ? L::cx[i] : (B[m] == 1 ? L::cy[i] : L::cz[i]);
                double cc = (double)(ca * cb) - (A[m] == B[m] ? 1.0 / 3.0 : 0.0);
                acc += fl[i] * cc;
            }
            pi_out[m * d.N + n] = acc;
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(long long n) { return (unsigned)((n + WG - 1) / WG); }

hipError_t launch_lb_step(int dim, int lb_fp, const InstDesc* D, int n_inst, long long total, const void* fin,
                          void* fout, long long* clock, double* shifts, int S, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    dim3 g(blocks_for(total)), b(WG);
    if (dim == 2 && lb_fp == 64)
        hipLaunchKernelGGL((k_lb_step<2, double>), g, b, 0, s, D, n_inst, total, (const double*)fin, (double*)fout, clock, shifts, S);
    else if (dim == 2)
        hipLaunchKernelGGL((k_lb_step<2, float>), g, b, 0, s, D, n_inst, total, (const float*)fin, (float*)fout, clock, shifts, S);
    else if (lb_fp == 64)
        hipLaunchKernelGGL((k_lb_step<3, double>), g, b, 0, s, D, n_inst, total, (const double*)fin, (double*)fout, clock, shifts, S);
    else
        hipLaunchKernelGGL((k_lb_step<3, float>), g, b, 0, s, D, n_inst, total, (const float*)fin, (float*)fout, clock, shifts, S);
    return hipGetLastError();
}

hipError_t launch_band(int dim, int lb_fp, const InstDesc* D, int n_inst, long long total, void* f, double* acc,
                       double* fbu, long long fb_stride, double* ub, double* tb, DevStats* stats, int do_feedback,
                       hipStream_t s) {
    if (total <= 0) return hipSuccess;
    dim3 g(blocks_for(total)), b(WG);
    if (dim == 2 && lb_fp == 64)
        hipLaunchKernelGGL((k_band<2, double>), g, b, 0, s, D, n_inst, total, (double*)f, acc, fbu, fb_stride, ub, tb,
                           stats, do_feedback);
    else if (dim == 2)
        hipLaunchKernelGGL((k_band<2, float>), g, b, 0, s, D, n_inst, total, (float*)f, acc, fbu, fb_stride, ub, tb,
                           stats, do_feedback);
    else if (lb_fp == 64)
        hipLaunchKernelGGL((k_band<3, double>), g, b, 0, s, D, n_inst, total, (double*)f, acc, fbu, fb_stride, ub, tb,
                           stats, do_feedback);
    else
        hipLaunchKernelGGL((k_band<3, float>), g, b, 0, s, D, n_inst, total, (float*)f, acc, fbu, fb_stride, ub, tb,
                           stats, do_feedback);
    return hipGetLastError();
}

hipError_t launch_interp(int dim, const InstDesc* D, int n_inst, long long total, const double* ub, double* uf,
                         const double* tb, double* tf, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    dim3 g(blocks_for(total)), b(WG);
    if (dim == 2)
        hipLaunchKernelGGL((k_interp<2>), g, b, 0, s, D, n_inst, total, ub, uf, tb, tf);
    else
        hipLaunchKernelGGL((k_interp<3>), g, b, 0, s, D, n_inst, total, ub, uf, tb, tf);
    return hipGetLastError();
}

hipError_t launch_lb_init(int dim, int lb_fp, const InstDesc* D, int n_inst, long long total, void* f,
                          double* fbu, long long fb_stride, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    dim3 g(blocks_for(total)), b(WG);
    if (dim == 2 && lb_fp == 64)
        hipLaunchKernelGGL((k_lb_init<2, double>), g, b, 0, s, D, n_inst, total, (double*)f, fbu, fb_stride);
    else if (dim == 2)
        hipLaunchKernelGGL((k_lb_init<2, float>), g, b, 0, s, D, n_inst, total, (float*)f, fbu, fb_stride);
    else if (lb_fp == 64)
        hipLaunchKernelGGL((k_lb_init<3, double>), g, b, 0, s, D, n_inst, total, (double*)f, fbu, fb_stride);
    else
        hipLaunchKernelGGL((k_lb_init<3, float>), g, b, 0, s, D, n_inst, total, (float*)f, fbu, fb_stride);
    return hipGetLastError();
}

hipError_t launch_moments(int dim, int lb_fp, const InstDesc* D, int inst, long long N, const void* f,
                          double* rho, double* u, double* pi, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    dim3 g(blocks_for(N)), b(WG);
    if (dim == 2 && lb_fp == 64)
        hipLaunchKernelGGL((k_moments<2, double>), g, b, 0, s, D, inst, (const double*)f, rho, u, pi);
    else if (dim == 2)
        hipLaunchKernelGGL((k_moments<2, float>), g, b, 0, s, D, inst, (const float*)f, rho, u, pi);
    else if (lb_fp == 64)
        hipLaunchKernelGGL((k_moments<3, double>), g, b, 0, s, D, inst, (const double*)f, rho, u, pi);
    else
        hipLaunchKernelGGL((k_moments<3, float>), g, b, 0, s, D, inst, (const float*)f, rho, u, pi);
    return hipGetLastError();
}

}  // namespace lbmpcd
