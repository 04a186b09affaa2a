// kernels_mlp.hip -- the learned closure's network on gfx950 matrix cores.
//
// Dense layers of a small MLP (271 -> 128 -> 128 -> 128 -> 9, GELU) run as
// BF16 x BF16 -> FP32 products on the MFMA units (v_mfma_f32_32x32x8_bf16):
// one 64x64 output tile per workgroup, each of its four waves owning a
// 32x32 quarter.  Operands are read through LDS with arbitrary strides, so
// one kernel serves the forward product X W^T, the input gradient dZ W and
// the weight gradient dZ^T X of back-propagation.  The epilogue adds the
// bias, stores the pre-activation, applies GELU or multiplies by GELU' of
// the previous layer's pre-activation, and rounds to BF16 where the next
// product needs it.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "gelu.hpp"
#include "mlp.hpp"

namespace lbmpcd {

typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// BF16 with round-to-nearest-even: gfx950's conversion instruction
// (v_cvt_pk_bf16_f32); NaN stays NaN.
__device__ __forceinline__ uint16_t to_bf16(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }


constexpr int GT = 64;   // output tile side
constexpr int GK = 32;   // K step
constexpr int GKP = GK + 8;  // LDS row pitch (bf16), breaks bank conflicts

__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
    __shared__ uint16_t As[GT][GKP];  // [m][k]
    __shared__ uint16_t Bs[GT][GKP];  // [n][k]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const long long m0 = (long long)blockIdx.y * GT, n0 = (long long)blockIdx.x * GT;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;

    for (long long k0 = 0; k0 < g.K; k0 += GK) {
        // operand tiles to LDS, 8 elements per thread per operand; the
        // thread-to-element map follows whichever stride is unit
        for (int e = tid; e < GT * GK; e += 256) {
            int m, k;
            if (g.sak == 1) { m = e / GK; k = e % GK; } else { m = e % GT; k = e / GT; }
            const long long gm = m0 + m, gk = k0 + k;
            As[m][k] = (gm < g.M && gk < g.K) ? g.A[gm * g.sam + gk * g.sak] : (uint16_t)0;
            int n, kb;
            if (g.sbk == 1) { n = e / GK; kb = e % GK; } else { n = e % GT; kb = e / GT; }
            const long long gn = n0 + n, gkb = k0 + kb;
            Bs[n][kb] = (gn < g.N && gkb < g.K) ? g.B[gkb * g.sbk + gn * g.sbn] : (uint16_t)0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; kk += 16) {
            // v_mfma_f32_32x32x16_bf16: lane l holds row (column) l % 32 and
            // the 8 k values 8 (l / 32) .. 8 (l / 32) + 7 of the step
            s16x8 a, b;
            const int ar = wm * 32 + (lane & 31), br = wn * 32 + (lane & 31);
            const int kc = kk + 8 * (lane >> 5);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                a[j] = (short)As[ar][kc + j];
                b[j] = (short)Bs[br][kc + j];
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                          acc, 0, 0, 0);
        }
        __syncthreads();
    }

    // epilogue: lane holds column (lane & 31) of its quarter, rows
    // 8 (r / 4) + 4 (lane / 32) + r % 4 for r = 0..15
    const long long col = n0 + wn * 32 + (lane & 31);
    if (col >= g.N) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const long long row = m0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (row >= g.M) continue;
        float v = acc[r];
        if (g.beta != 0.0f) v += g.beta * g.C[row * g.ldc + col];
        if (g.bias) v += g.bias[col];
        if (g.Z) g.Z[row * g.ldz + col] = v;
        if (g.epi == EPI_GELU) v = gelu(v);
        else if (g.epi == EPI_GELU_GRAD) v *= gelu_grad(g.Zprev[row * g.ldzp + col]);
        if (g.C) g.C[row * g.ldc + col] = v;
        if (g.Cb) g.Cb[row * g.ldcb + col] = to_bf16(v);
    }
}

hipError_t launch_gemm(const GemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    dim3 grid((unsigned)((g.N + GT - 1) / GT), (unsigned)((g.M + GT - 1) / GT));
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// network passes
// ---------------------------------------------------------------------------
static inline unsigned nblk(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

size_t closure_bufs_bytes(long long rows, bool backward) {
    auto al = closure_al256;
    size_t b = closure_fwd_bytes(rows);
    if (backward) b += al((size_t)rows * NOUT * 4) + al((size_t)rows * NOUT * 2) +
                       3 * (al((size_t)rows * NH * 4) + al((size_t)rows * NH * 2));
    return b;
}

void closure_bufs_carve(unsigned char* base, long long rows, bool backward, ClosureBufs& b) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t o = 0;
    auto take = [&](size_t bytes) { unsigned char* p = base + o; o += al(bytes); return p; };
    b = ClosureBufs{};
    b.rows = rows;
    b.X = (uint16_t*)take((size_t)rows * NFP * 2);
    for (int l = 0; l < 3; ++l) {
        b.Z[l] = (float*)take((size_t)rows * NH * 4);
        b.H[l] = (uint16_t*)take((size_t)rows * NH * 2);
    }
    b.Y = (float*)take((size_t)rows * NOUT * 4);
    if (backward) {
        b.dY = (float*)take((size_t)rows * NOUT * 4);
        b.dYb = (uint16_t*)take((size_t)rows * NOUT * 2);
        for (int l = 0; l < 3; ++l) {
            b.dZ[l] = (float*)take((size_t)rows * NH * 4);
            b.dZb[l] = (uint16_t*)take((size_t)rows * NH * 2);
        }
    }
}

static GemmArgs gemm0() {
    GemmArgs g{};
    g.beta = 0.0f;
    g.epi = EPI_NONE;
    return g;
}

hipError_t mlp_forward(const float* P32, const uint16_t* Pb, const ClosureBufs& b, hipStream_t s) {
    const long long offW[4] = {OFF_W1, OFF_W2, OFF_W3, OFF_W4}, offB[4] = {OFF_B1, OFF_B2, OFF_B3, OFF_B4};
    for (int l = 0; l < 4; ++l) {
        GemmArgs g = gemm0();
        const long long K = l == 0 ? NFP : NH;
        const long long N = l == 3 ? NOUT : NH;
        g.M = b.rows; g.N = N; g.K = K;
        g.A = l == 0 ? b.X : b.H[l - 1]; g.sam = K; g.sak = 1;
        g.B = Pb + offW[l]; g.sbk = 1; g.sbn = K;  // B(k, n) = W[n][k]
        g.bias = P32 + offB[l];
        if (l < 3) {
            g.Z = b.Z[l]; g.ldz = NH;
            g.Cb = b.H[l]; g.ldcb = NH;
            g.epi = EPI_GELU;
        } else {
            g.C = b.Y; g.ldc = NOUT;
        }
        hipError_t e = launch_gemm(g, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// dY = 2 (Y - Yt) / (rows NOUT); loss += sum (Y - Yt)^2 / (rows NOUT)
__global__ void __launch_bounds__(256) k_mse(const float* Y, const float* Yt, long long n, float* dY,
                                             uint16_t* dYb, double* loss) {
    __shared__ double red[256];
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    double l = 0.0;
    if (i < n) {
        const float dd = Y[i] - Yt[i];
        const float g = 2.0f * dd / (float)n;
        dY[i] = g;
        dYb[i] = to_bf16(g);
        l = (double)dd * (double)dd / (double)n;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(loss, red[0]);
}

// db[c] = sum over rows of dZ[r][c]
__global__ void __launch_bounds__(256) k_colsum(const float* dZ, long long rows, int cols, float* db) {
    __shared__ float red[256];
    const int c = blockIdx.x;
    float acc = 0.0f;
    for (long long r = threadIdx.x; r < rows; r += 256) acc += dZ[r * cols + c];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[c] = red[0];
}

hipError_t mlp_backward(const uint16_t* Pb, const float* Yt, const ClosureBufs& b, float* G, double* loss,
                        hipStream_t s) {
    const long long R = b.rows;
    hipLaunchKernelGGL(k_mse, dim3(nblk(R * NOUT)), dim3(256), 0, s, b.Y, Yt, R * NOUT, b.dY, b.dYb, loss);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long offW[4] = {OFF_W1, OFF_W2, OFF_W3, OFF_W4}, offB[4] = {OFF_B1, OFF_B2, OFF_B3, OFF_B4};
    for (int l = 3; l >= 0; --l) {
        const long long K = l == 0 ? NFP : NH;      // inputs of layer l
        const long long N = l == 3 ? NOUT : NH;     // outputs of layer l
        const float* dZ = l == 3 ? b.dY : b.dZ[l];
        const uint16_t* dZb = l == 3 ? b.dYb : b.dZb[l];
        const uint16_t* In = l == 0 ? b.X : b.H[l - 1];
        // weight gradient dW[o][i] = sum_r dZ[r][o] In[r][i]
        GemmArgs g = gemm0();
        g.M = N; g.N = K; g.K = R;
        g.A = dZb; g.sam = 1; g.sak = N;
        g.B = In; g.sbk = K; g.sbn = 1;
        g.C = G + offW[l]; g.ldc = K;
        if ((e = launch_gemm(g, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_colsum, dim3((unsigned)N), dim3(256), 0, s, dZ, R, (int)N, G + offB[l]);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (l == 0) break;
        // input gradient, times GELU' of the previous pre-activation
        GemmArgs h = gemm0();
        h.M = R; h.N = K; h.K = N;
        h.A = dZb; h.sam = N; h.sak = 1;
        h.B = Pb + offW[l]; h.sbk = K; h.sbn = 1;  // B(k = o, n = i) = W[o][i]
        h.epi = EPI_GELU_GRAD; h.Zprev = b.Z[l - 1]; h.ldzp = NH;
        h.C = b.dZ[l - 1]; h.ldc = NH;
        h.Cb = b.dZb[l - 1]; h.ldcb = NH;
        if ((e = launch_gemm(h, s)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// Adam (Kingma & Ba) on the FP32 parameters, with the bias-corrected moment
// estimates; the BF16 copy follows.
__global__ void __launch_bounds__(256) k_adam(float* P, uint16_t* Pb, const float* G, float* m, float* v,
                                              long long n, float lr, float b1, float b2, float eps, float c1,
                                              float c2) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float g = G[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float p = P[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    P[i] = p;
    Pb[i] = to_bf16(p);
}

hipError_t mlp_adam(float* P32, uint16_t* Pb, const float* G, float* m, float* v, long long t, float lr,
                    float beta1, float beta2, float eps, hipStream_t s) {
    const float c1 = 1.0f - powf(beta1, (float)t), c2 = 1.0f - powf(beta2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(nblk(NPARAM)), dim3(256), 0, s, P32, Pb, G, m, v, NPARAM, lr, beta1, beta2,
                       eps, c1, c2);
    return hipGetLastError();
}

// Uniform(-a, a) weights with a = sqrt(6 / (fan_in + fan_out)) over the real
// inputs (Glorot), zero biases, zero padding columns, zero Adam moments.
__global__ void __launch_bounds__(256) k_mlp_init(float* P, uint16_t* Pb, float* m, float* v, uint32_t k0,
                                                  uint32_t k1) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= NPARAM) return;
    float w = 0.0f;
    long long off = 0;
    int fin = 0, fout = 0, K = 0;
    bool weight = false;
    if (i < OFF_B1) { off = OFF_W1; fin = NF; fout = NH; K = NFP; weight = true; }
    else if (i >= OFF_W2 && i < OFF_B2) { off = OFF_W2; fin = NH; fout = NH; K = NH; weight = true; }
    else if (i >= OFF_W3 && i < OFF_B3) { off = OFF_W3; fin = NH; fout = NH; K = NH; weight = true; }
    else if (i >= OFF_W4 && i < OFF_B4) { off = OFF_W4; fin = NH; fout = NOUT; K = NH; weight = true; }
    if (weight && (int)((i - off) % K) < fin) {
        const U4 r = rng_block(Key{k0, k1}, (uint32_t)i, 0u, 0u, P_MLP_INIT, 0u);
        const double a = sqrt(6.0 / (double)(fin + fout));
        w = (float)((2.0 * u01(r.x, r.y) - 1.0) * a);
    }
    P[i] = w;
    Pb[i] = to_bf16(w);
    m[i] = 0.0f;
    v[i] = 0.0f;
}

hipError_t mlp_init(float* P32, uint16_t* Pb, float* m, float* v, uint32_t k0, uint32_t k1, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_init, dim3(nblk(NPARAM)), dim3(256), 0, s, P32, Pb, m, v, k0, k1);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// data
// ---------------------------------------------------------------------------
// Column sums of x and x^2 (FP64), one thread per column, rows in blocks.
__global__ void __launch_bounds__(256) k_colstats(const float* X, long long n, int cols, long long rows_per,
                                                  double* sums) {
    const int c = blockIdx.y * 256 + threadIdx.x;
    if (c >= cols) return;
    const long long r0 = (long long)blockIdx.x * rows_per;
    const long long r1 = r0 + rows_per < n ? r0 + rows_per : n;
    double s1 = 0.0, s2 = 0.0;
    for (long long r = r0; r < r1; ++r) {
        const double x = X[r * cols + c];
        s1 += x;
        s2 += x * x;
    }
    atomicAdd(&sums[2 * c], s1);
    atomicAdd(&sums[2 * c + 1], s2);
}

__global__ void k_stats_final(const double* sx, const double* sy, long long n, float* stats) {
    const int c = threadIdx.x + blockIdx.x * blockDim.x;
    // The scale never drops below 1e-3 of the column's mean magnitude (nor
    // below 1e-12): columns that barely vary, such as the density of a
    // nearly incompressible flow, are not blown up to unit spread.
    auto fin = [&](const double* s, int col, float* mean, float* sd) {
        const double mu = s[2 * col] / (double)n;
        const double var = s[2 * col + 1] / (double)n - mu * mu;
        const double st = var > 0.0 ? sqrt(var) : 0.0;
        mean[col] = (float)mu;
        sd[col] = (float)fmax(fmax(st, 1e-3 * fabs(mu)), 1e-12);
    };
    if (c < NF) fin(sx, c, stats, stats + NF);
    if (c < NOUT) fin(sy, c, stats + 2 * NF, stats + 2 * NF + NOUT);
}

// Column sums of the network targets: velocity relative to the node's LB
// velocity, stress as is.
__global__ void __launch_bounds__(256) k_colstats_y(const float* Y, const float* X, long long n, long long rows_per,
                                                    double* sums) {
    const int c = threadIdx.x;
    if (c >= NOUT) return;
    const long long r0 = (long long)blockIdx.x * rows_per;
    const long long r1 = r0 + rows_per < n ? r0 + rows_per : n;
    double s1 = 0.0, s2 = 0.0;
    for (long long r = r0; r < r1; ++r) {
        const double y = (double)Y[r * NOUT + c] - (c < 3 ? (double)X[r * NF + UC + c] : 0.0);
        s1 += y;
        s2 += y * y;
    }
    atomicAdd(&sums[2 * c], s1);
    atomicAdd(&sums[2 * c + 1], s2);
}

hipError_t mlp_stats(const float* X, const float* Y, long long n, double* sums, float* stats, hipStream_t s) {
    hipError_t e = hipMemsetAsync(sums, 0, sizeof(double) * 2 * (NF + NOUT), s);
    if (e != hipSuccess) return e;
    const long long rows_per = 1024;
    const unsigned gx = (unsigned)((n + rows_per - 1) / rows_per);
    hipLaunchKernelGGL(k_colstats, dim3(gx, (NF + 255) / 256), dim3(256), 0, s, X, n, NF, rows_per, sums);
    hipLaunchKernelGGL(k_colstats_y, dim3(gx, 1), dim3(64), 0, s, Y, X, n, rows_per, sums + 2 * NF);
    hipLaunchKernelGGL(k_stats_final, dim3(2), dim3(256), 0, s, sums, sums + 2 * NF, n, stats);
    return hipGetLastError();
}

// Row r of the batch: source row idx (drawn uniformly from n with Philox when
// `draw`, else r), standardised; features to BF16 with zero padding.  Every
// kernel standardises a feature as (x - mean) times the binary32 reciprocal of
// its standard deviation, so that training and the fused inference see the
// same values (the fused kernel reads the reciprocals from LDS, a multiply per
// feature where a division took 6 % of its time).
__global__ void __launch_bounds__(256) k_gather(const float* X, const float* Y, long long n, const float* st,
                                                long long rows, int draw, uint32_t k0, uint32_t k1,
                                                uint32_t step, uint16_t* Xb, float* Yb) {
    const long long r = blockIdx.x;
    if (r >= rows) return;
    long long src = r;
    if (draw) {
        const U4 w = rng_block(Key{k0, k1}, (uint32_t)r, step, 0u, P_MLP_BATCH, 0u);
        const uint64_t v = ((uint64_t)w.y << 32) | w.x;
        src = (long long)(v % (uint64_t)n);
    }
    for (int c = threadIdx.x; c < NFP; c += 256) {
        float x = 0.0f;
        if (c < NF) x = (X[src * NF + c] - st[c]) * (1.0f / st[NF + c]);
        Xb[r * NFP + c] = to_bf16(x);
    }
    if (Y && threadIdx.x < NOUT) {
        const int c = threadIdx.x;
        const float y = Y[src * NOUT + c] - (c < 3 ? X[src * NF + UC + c] : 0.0f);
        Yb[r * NOUT + c] = (y - st[2 * NF + c]) / st[2 * NF + NOUT + c];
    }
}

hipError_t mlp_gather(const float* X, const float* Y, long long n, const float* stats, long long rows, bool draw,
                      uint32_t k0, uint32_t k1, uint32_t step, uint16_t* Xb, float* Yb, hipStream_t s) {
    hipLaunchKernelGGL(k_gather, dim3((unsigned)rows), dim3(256), 0, s, X, Y, n, stats, rows, draw ? 1 : 0, k0, k1,
                       step, Xb, Yb);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_refresh_bf16(const float* P, uint16_t* Pb, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) Pb[i] = to_bf16(P[i]);
}

hipError_t mlp_refresh_bf16(const float* P32, uint16_t* Pb, hipStream_t s) {
    hipLaunchKernelGGL(k_refresh_bf16, dim3(nblk(NPARAM)), dim3(256), 0, s, P32, Pb, NPARAM);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_destd(const float* Y, const float* st, const float* X, long long n,
                                               float* out) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int c = (int)(i % NOUT);
    const long long r = i / NOUT;
    out[i] = Y[i] * st[2 * NF + NOUT + c] + st[2 * NF + c] + (c < 3 ? X[r * NF + UC + c] : 0.0f);
}

hipError_t mlp_destandardize(const float* Y, const float* stats, const float* X, long long rows, float* out,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_destd, dim3(nblk(rows * NOUT)), dim3(256), 0, s, Y, stats, X, rows * NOUT, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// coupling
// ---------------------------------------------------------------------------
// Moments of node (x, y, z): rho, u = j / rho + g / 2, Pi_ab = sum f (c_a c_b
// - delta_ab / 3) in the order xx yy zz xy xz yz.
template <typename LT>
__device__ __forceinline__ void node_moments(const LT* fp, long long N, long long n, const double g[3],
                                             double m[10]) {
    using L = Lat<3>;
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0}, P[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const double fi = (double)fp[i * N + n];
        const double c0 = L::cx[i], c1 = L::cy[i], c2 = L::cz[i];
        rho += fi;
        j[0] += fi * c0; j[1] += fi * c1; j[2] += fi * c2;
        P[0] += fi * (c0 * c0 - 1.0 / 3.0);
        P[1] += fi * (c1 * c1 - 1.0 / 3.0);
        P[2] += fi * (c2 * c2 - 1.0 / 3.0);
        P[3] += fi * c0 * c1;
        P[4] += fi * c0 * c2;
        P[5] += fi * c1 * c2;
    }
    m[0] = rho;
    for (int a = 0; a < 3; ++a) m[1 + a] = j[a] / rho + 0.5 * g[a];
    for (int a = 0; a < 6; ++a) m[4 + a] = P[a];
}

// Features of one slab node: for the 27 neighbours (dz, dy, dx in -1..1, x
// and z periodic, y clamped to the channel) the 10 moments, then the shear
// rate sqrt(2 S:S) of the node with S = -(Pi - rho u u) / (2 rho c_s^2 tau).
template <typename LT>
__global__ void __launch_bounds__(256) k_features(const InstDesc* __restrict__ D, int inst, long long nslab,
                                                  const LT* __restrict__ f, double* facc, const float* st,
                                                  uint16_t* Xb, float* uc) {
    const long long sn = (long long)blockIdx.x * 256 + threadIdx.x;
    if (sn >= nslab) return;
    const InstDesc& d = D[inst];
    const int nsy = d.yhi - d.ylo;
    const int x = (int)(sn % d.nx), y = d.ylo + (int)((sn / d.nx) % nsy), z = (int)(sn / ((long long)d.nx * nsy));
    const LT* fp = f + d.node_off * Lat<3>::Q;
    // each feature goes straight to its output as it is formed
    auto emit = [&](int q, double v) {
        if (facc) facc[sn * NF + q] += v;
        if (Xb) Xb[sn * NFP + q] = to_bf16(((float)v - st[q]) * (1.0f / st[NF + q]));
    };
    int k = 0;
    double mc[10];
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int xx = x + dx; if (xx < 0) xx += d.nx; else if (xx >= d.nx) xx -= d.nx;
                int zz = z + dz; if (zz < 0) zz += d.nz; else if (zz >= d.nz) zz -= d.nz;
                int yy = y + dy; yy = yy < 0 ? 0 : (yy >= d.ny ? d.ny - 1 : yy);
                const long long n = ((long long)zz * d.ny + yy) * d.nx + xx;
                double m[10];
                node_moments<LT>(fp, d.N, n, d.g, m);
                for (int q = 0; q < 10; ++q) emit(k + q, m[q]);
                if (dx == 0 && dy == 0 && dz == 0)
                    for (int q = 0; q < 10; ++q) mc[q] = m[q];
                k += 10;
            }
    const double rho = mc[0], u[3] = {mc[1], mc[2], mc[3]};
    if (uc)
        for (int a = 0; a < 3; ++a) uc[sn * 3 + a] = (float)u[a];
    const int A[6] = {0, 1, 2, 0, 0, 1}, B[6] = {0, 1, 2, 1, 2, 2};
    double ss = 0.0;
    for (int q = 0; q < 6; ++q) {
        const double Sab = -(mc[4 + q] - rho * u[A[q]] * u[B[q]]) / (2.0 * rho * (1.0 / 3.0) * d.tau);
        ss += (q < 3 ? 1.0 : 2.0) * Sab * Sab;
    }
    emit(NF - 1, sqrt(2.0 * ss));
    if (Xb)
        for (int q = NF; q < NFP; ++q) Xb[sn * NFP + q] = 0;
}

hipError_t closure_features(int lb_fp, const InstDesc* D, int inst, long long nslab, const void* f, double* facc,
                            const float* stats, uint16_t* Xb, float* uc, hipStream_t s) {
    if (lb_fp == 64)
        hipLaunchKernelGGL(k_features<double>, dim3(nblk(nslab)), dim3(256), 0, s, D, inst, nslab,
                           (const double*)f, facc, stats, Xb, uc);
    else
        hipLaunchKernelGGL(k_features<float>, dim3(nblk(nslab)), dim3(256), 0, s, D, inst, nslab,
                           (const float*)f, facc, stats, Xb, uc);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_to_acc(const InstDesc* __restrict__ D, int inst, long long nslab,
                                                const float* Y, const float* st, const float* uc, double* acc,
                                                double* prof, int do_prof) {
    const long long sn = (long long)blockIdx.x * 256 + threadIdx.x;
    if (sn >= nslab) return;
    const InstDesc& d = D[inst];
    double u[3];
    for (int a = 0; a < 3; ++a)
        u[a] = (double)Y[sn * NOUT + a] * (double)st[2 * NF + NOUT + a] + (double)st[2 * NF + a] +
               (double)uc[sn * 3 + a];
    double* a = acc + (d.acc_off + sn) * 4;
    a[0] = 1.0; a[1] = u[0]; a[2] = u[1]; a[3] = u[2];
    if (do_prof) {
        const int nsy = d.yhi - d.ylo;
        const int yy = (int)((sn / d.nx) % nsy);
        const int copy = (int)(sn % NCOPY);
        for (int i = 0; i < d.r; ++i) {
            double* gb = prof + (d.prof_off + (long long)copy * d.R + (long long)yy * d.r + i) * 4;
            atomicAdd(&gb[0], 1.0);
            atomicAdd(&gb[1], u[0]);
            atomicAdd(&gb[2], u[1]);
            atomicAdd(&gb[3], u[2]);
        }
    }
}

hipError_t closure_to_acc(const InstDesc* D, int inst, long long nslab, const float* Y, const float* stats,
                          const float* uc, double* acc, double* prof, int do_prof, hipStream_t s) {
    hipLaunchKernelGGL(k_to_acc, dim3(nblk(nslab)), dim3(256), 0, s, D, inst, nslab, Y, stats, uc, acc, prof,
                       do_prof);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fused inference: features and the four layers in one kernel
// ---------------------------------------------------------------------------
constexpr int BMS = 12;  // floats per band node: 10 moments, shear rate, pad

// The 10 moments and the shear rate of every node of the rows [y0, y0 + nyb)
// that the slab's 3x3x3 stencils reach, computed exactly as the per-node
// feature kernel computes them.
template <typename LT>
__global__ void __launch_bounds__(256) k_band_moments(const InstDesc* __restrict__ D, int inst,
                                                      const LT* __restrict__ f, int y0, int nyb, float* M) {
    const InstDesc& d = D[inst];
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long long)d.nx * nyb * d.nz) return;
    const int x = (int)(i % d.nx), yb = (int)((i / d.nx) % nyb), z = (int)(i / ((long long)d.nx * nyb));
    const long long n = ((long long)z * d.ny + (y0 + yb)) * d.nx + x;
    double m[10];
    node_moments<LT>(f + d.node_off * Lat<3>::Q, d.N, n, d.g, m);
    const double rho = m[0], u[3] = {m[1], m[2], m[3]};
    const int A[6] = {0, 1, 2, 0, 0, 1}, B[6] = {0, 1, 2, 1, 2, 2};
    double ss = 0.0;
    for (int q = 0; q < 6; ++q) {
        const double Sab = -(m[4 + q] - rho * u[A[q]] * u[B[q]]) / (2.0 * rho * (1.0 / 3.0) * d.tau);
        ss += (q < 3 ? 1.0 : 2.0) * Sab * Sab;
    }
    // binary32 is what the features use of them: (float)m - mean, then / std
    float* o = M + i * BMS;
    for (int q = 0; q < 10; ++q) o[q] = (float)m[q];
    o[10] = (float)sqrt(2.0 * ss);
    o[11] = 0.0f;
}

// One workgroup of four waves per block of 128 slab nodes, 32 per wave.  The
// workgroup writes the block's standardised BF16 features into LDS; each
// wave then runs its 32 rows through the four layers on the matrix cores
// (v_mfma_f32_32x32x16_bf16, the k steps in the same order as the separate
// products, so the results are the same), the hidden activations going back
// into the wave's own rows of the LDS block between layers.  Weights are
// read from memory (they stay in the caches).  Outputs: the standardised
// network output Y and the centre node's LB velocity uc.
constexpr int FNT = 256;       // threads per workgroup: four waves
constexpr int FR = 32 * (FNT / 64);  // rows per workgroup, 32 per wave
constexpr int XPITCH = NFP + 8;  // LDS row pitch of the feature block (BF16 elements, 16-byte rows)
constexpr int HPITCH = NH + 8;   // LDS row pitch of a hidden block

// Weights of one layer in fragment order (see FRAG_L1): one thread per value.
__global__ void __launch_bounds__(256) k_frag_weights(const uint16_t* __restrict__ Pb, uint16_t* Pf) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= NFRAG) return;
    long long base, off;
    int K, ncb, nvalid;
    if (i < FRAG_L2) { base = FRAG_L1; off = OFF_W1; K = NFP; ncb = 4; nvalid = NH; }
    else if (i < FRAG_L3) { base = FRAG_L2; off = OFF_W2; K = NH; ncb = 4; nvalid = NH; }
    else if (i < FRAG_L4) { base = FRAG_L3; off = OFF_W3; K = NH; ncb = 4; nvalid = NH; }
    else { base = FRAG_L4; off = OFF_W4; K = NH; ncb = 1; nvalid = NOUT; }
    const long long e = i - base;
    const int j = (int)(e & 7), t = (int)((e >> 3) & 63);
    const long long sb = e >> 9;  // step * ncb + block
    const int b = (int)(sb % ncb), st = (int)(sb / ncb);
    const int n = 32 * b + (t & 31), k = 16 * st + 8 * (t >> 5) + j;
    Pf[i] = n < nvalid ? Pb[off + (long long)n * K + k] : (uint16_t)0;
}

// One layer for the wave's 32 rows: each k step of 16 loads the rows' inputs
// from LDS and every column block's weight fragment (one coalesced 1 KiB
// read per wave), then issues the products.
template <int K, int NCB>
__device__ __forceinline__ void mfma_layer(const uint16_t* act, int pitch, const uint16_t* Wf, f32x16 acc[4]) {
    constexpr int NS = K / 16;
    const int lane = threadIdx.x & 63, lr = lane & 31, h = lane >> 5;
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[nb][r] = 0.0f;
    const uint4* wf = (const uint4*)Wf + lane;
#pragma unroll
    for (int st = 0; st < NS; ++st) {
        // eight consecutive BF16 inputs as one 16-byte load (rows start at
        // multiples of 16 bytes)
        const bf16x8 a = __builtin_bit_cast(bf16x8, *(const uint4*)(act + lr * pitch + st * 16 + 8 * h));
#pragma unroll
        for (int nb = 0; nb < NCB; ++nb) {
            const uint4 b = wf[(st * NCB + nb) * 64];
            acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, __builtin_bit_cast(bf16x8, b), acc[nb], 0, 0, 0);
        }
    }
}

// bias, GELU, BF16 into the wave's rows (C layout: lane holds column lane & 31
// of each 32-column block, rows 8 (r / 4) + 4 (lane / 32) + r % 4)
__device__ __forceinline__ void hidden_out(const f32x16 acc[4], const float* bias, uint16_t* act) {
    const int lane = threadIdx.x & 63, lr = lane & 31, h = lane >> 5;
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        const int col = nb * 32 + lr;
        const float bc = bias[col];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 8 * (r >> 2) + 4 * h + (r & 3);
            act[row * HPITCH + col] = to_bf16(gelu(acc[nb][r] + bc));
        }
    }
}

__global__ void __launch_bounds__(FNT) k_mlp_fused(const InstDesc* __restrict__ D, int inst, long long nslab, int y0,
                                                   int nyb, const float* __restrict__ M, const float* __restrict__ st,
                                                   const uint16_t* __restrict__ Pf, const float* __restrict__ P32,
                                                   float* Y, float* uc) {
    __shared__ uint16_t xs[FR * XPITCH];
    __shared__ float sinv[NF];     // reciprocals of the features' standard deviations
    __shared__ int rxyz[3 * FR];   // node coordinates of the block's rows
    const InstDesc& d = D[inst];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long r0 = (long long)blockIdx.x * FR;
    const int nsy = d.yhi - d.ylo;
    for (int k = tid; k < NF; k += FNT) sinv[k] = 1.0f / st[NF + k];
    // the divisions by the channel's sizes once per row, not per stencil entry
    for (int r = tid; r < FR; r += FNT) {
        const long long sn = r0 + r < nslab ? r0 + r : 0;
        rxyz[3 * r] = (int)(sn % d.nx);
        rxyz[3 * r + 1] = d.ylo + (int)((sn / d.nx) % nsy);
        rxyz[3 * r + 2] = (int)(sn / ((long long)d.nx * nsy));
    }
    __syncthreads();
    auto band_index = [&](int r, int dx, int dy, int dz) {
        const int x = rxyz[3 * r], y = rxyz[3 * r + 1], z = rxyz[3 * r + 2];
        int xx = x + dx; if (xx < 0) xx += d.nx; else if (xx >= d.nx) xx -= d.nx;
        int zz = z + dz; if (zz < 0) zz += d.nz; else if (zz >= d.nz) zz -= d.nz;
        int yy = y + dy; yy = yy < 0 ? 0 : (yy >= d.ny ? d.ny - 1 : yy);
        return ((long long)zz * nyb + (yy - y0)) * d.nx + xx;
    };
    // standardised features of the block: stencil entry s of row r (lanes of
    // a wave take consecutive rows of one stencil entry)
#pragma unroll 4
    for (int it = tid; it < FR * 27; it += FNT) {
        const int r = it % FR, s = it / FR;
        const long long sn = r0 + r;
        uint16_t* xr = xs + r * XPITCH + s * 10;
        if (sn >= nslab) {
            for (int q = 0; q < 10; ++q) xr[q] = 0;
            continue;
        }
        const float* m = M + band_index(r, s % 3 - 1, (s / 3) % 3 - 1, s / 9 - 1) * BMS;
        for (int q = 0; q < 10; ++q) {
            const int k = s * 10 + q;
            xr[q] = to_bf16((m[q] - st[k]) * sinv[k]);
        }
    }
    for (int r = tid; r < FR; r += FNT) {
        const long long sn = r0 + r;
        uint16_t* xr = xs + r * XPITCH;
        for (int q = NF - 1; q < NFP; ++q) xr[q] = 0;
        if (sn >= nslab) continue;
        const float* m = M + band_index(r, 0, 0, 0) * BMS;
        xr[NF - 1] = to_bf16((m[10] - st[NF - 1]) * sinv[NF - 1]);
        for (int a = 0; a < 3; ++a) uc[sn * 3 + a] = m[1 + a];
    }
    __syncthreads();

    uint16_t* own = xs + wave * 32 * XPITCH;  // this wave's rows; hidden blocks reuse them
    f32x16 acc[4];
    mfma_layer<NFP, 4>(own, XPITCH, Pf + FRAG_L1, acc);
    __syncthreads();
    hidden_out(acc, P32 + OFF_B1, own);
    __syncthreads();
    mfma_layer<NH, 4>(own, HPITCH, Pf + FRAG_L2, acc);
    __syncthreads();
    hidden_out(acc, P32 + OFF_B2, own);
    __syncthreads();
    mfma_layer<NH, 4>(own, HPITCH, Pf + FRAG_L3, acc);
    __syncthreads();
    hidden_out(acc, P32 + OFF_B3, own);
    __syncthreads();
    mfma_layer<NH, 1>(own, HPITCH, Pf + FRAG_L4, acc);
    const int lr = lane & 31, h = lane >> 5;
    if (lr < NOUT) {
        const float bc = P32[OFF_B4 + lr];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const long long sn = r0 + wave * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
            if (sn < nslab) Y[sn * NOUT + lr] = acc[0][r] + bc;
        }
    }
}

hipError_t closure_predict(int lb_fp, const InstDesc* D, int inst, long long nslab, long long nband, int y0,
                           int nyb, const void* f, float* M, const float* stats, const uint16_t* Pb,
                           uint16_t* Pf, const float* P32, float* Y, float* uc, hipStream_t s) {
    hipLaunchKernelGGL(k_frag_weights, dim3(nblk(NFRAG)), dim3(256), 0, s, Pb, Pf);
    if (lb_fp == 64)
        hipLaunchKernelGGL(k_band_moments<double>, dim3(nblk(nband)), dim3(256), 0, s, D, inst, (const double*)f,
                           y0, nyb, M);
    else
        hipLaunchKernelGGL(k_band_moments<float>, dim3(nblk(nband)), dim3(256), 0, s, D, inst, (const float*)f,
                           y0, nyb, M);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_fused, dim3(nblk(nslab, FR)), dim3(FNT), 0, s, D, inst, nslab, y0, nyb, M, stats, Pf,
                       P32, Y, uc);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_destd_uc(const float* Y, const float* st, const float* uc, long long n,
                                                  float* out) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int c = (int)(i % NOUT);
    const long long r = i / NOUT;
    out[i] = Y[i] * st[2 * NF + NOUT + c] + st[2 * NF + c] + (c < 3 ? uc[r * 3 + c] : 0.0f);
}

hipError_t mlp_destandardize_uc(const float* Y, const float* stats, const float* uc, long long rows, float* out,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_destd_uc, dim3(nblk(rows * NOUT)), dim3(256), 0, s, Y, stats, uc, rows * NOUT, out);
    return hipGetLastError();
}

// One workgroup per particle tile: count, sum v and sum v v of every
// particle's LB node (all particles of the slab lie in slab nodes).  A tile
// of the shifted grid covers few nodes, so the sums go through an LDS window
// of those nodes (NMREP interleaved replicas of each, lane l adding into
// replica l mod NMREP) and reach memory with one global atomic per node and
// moment; a particle outside the window adds to memory directly.
constexpr int NMREP = 8;    // 40 KB of LDS with 10 FP64 sums per node and replica

template <typename PT>
__global__ void __launch_bounds__(256) k_node_moments(const InstDesc* __restrict__ D, int inst,
                                                      const unsigned char* pos0, long long cs,
                                                      const uint32_t* fill, double* nm) {
    __shared__ double win[NM_WIN * NMREP * 10];
    const InstDesc& d = D[inst];
    const uint32_t T = blockIdx.x;  // tile within the channel
    const uint32_t nxy = (uint32_t)d.ntx * (uint32_t)d.nty;
    const int tz = (int)(T / nxy), rem = (int)(T - (uint32_t)tz * nxy);
    const int ty = rem / d.ntx, tx = rem - ty * d.ntx;
    const int r = d.r, nsy = d.yhi - d.ylo;
    // nodes that particles binned in this tile can occupy (one cell of margin per side)
    const int wx0 = (tx * d.Tx) / r - 1, wy0 = (ty * d.Ty) / r - 1, wz0 = (tz * d.Tz) / r - 1;
    const int wnx = (d.Tx + r - 1) / r + 2, wny = (d.Ty + r - 1) / r + 2, wnz = (d.Tz + r - 1) / r + 2;
    const bool win_ok = wnx * wny * wnz <= NM_WIN;
    const int nwin = win_ok ? wnx * wny * wnz : 0;
    for (int i = threadIdx.x; i < nwin * NMREP * 10; i += 256) win[i] = 0.0;
    __syncthreads();
    const uint32_t n = min(fill[d.tile_off + T], (uint32_t)d.cap);
    const PT* c[6];
    for (int q = 0; q < 6; ++q) c[q] = (const PT*)(pos0 + q * cs) + d.slot_off + (long long)T * d.cap;
    const int A[6] = {0, 1, 2, 0, 0, 1}, B[6] = {0, 1, 2, 1, 2, 2};
    const int rep = (threadIdx.x & 63) & (NMREP - 1);
    for (uint32_t k = threadIdx.x; k < n; k += 256) {
        const int x = min(max((int)floor((double)c[0][k]), 0), d.nx - 1);
        const int y = min(max((int)floor((double)c[1][k]), d.ylo), d.yhi - 1);
        const int z = min(max((int)floor((double)c[2][k]), 0), d.nz - 1);
        const double v[3] = {(double)c[3][k], (double)c[4][k], (double)c[5][k]};
        double m[10];
        m[0] = 1.0;
        for (int a = 0; a < 3; ++a) m[1 + a] = v[a];
        for (int q = 0; q < 6; ++q) m[4 + q] = v[A[q]] * v[B[q]];
        int ax = x - wx0; if (ax < 0) ax += d.nx; else if (ax >= d.nx) ax -= d.nx;
        int az = z - wz0; if (az < 0) az += d.nz; else if (az >= d.nz) az -= d.nz;
        const int ay = (y - d.ylo) - wy0;
        double* o;
        if (win_ok && ax < wnx && ay >= 0 && ay < wny && az < wnz)
            o = win + 10 * (NMREP * (ax + wnx * (ay + wny * az)) + rep);
        else
            o = nm + (((long long)z * nsy + (y - d.ylo)) * d.nx + x) * 10;
        for (int q = 0; q < 10; ++q) atomicAdd(&o[q], m[q]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nwin * 10; i += 256) {
        const int w = i / 10, q = i - 10 * w;
        double sum = 0.0, cnt = 0.0;
        for (int rr = 0; rr < NMREP; ++rr) {
            sum += win[10 * (NMREP * w + rr) + q];
            cnt += win[10 * (NMREP * w + rr)];
        }
        if (cnt == 0.0) continue;  // no particle in this node
        const int ax = w % wnx, ay = (w / wnx) % wny, az = w / (wnx * wny);
        int x = wx0 + ax; if (x < 0) x += d.nx; else if (x >= d.nx) x -= d.nx;
        int z = wz0 + az; if (z < 0) z += d.nz; else if (z >= d.nz) z -= d.nz;
        const int yl = wy0 + ay;
        if (yl < 0 || yl >= nsy) continue;
        atomicAdd(&nm[(((long long)z * nsy + yl) * d.nx + x) * 10 + q], sum);
    }
}

hipError_t closure_node_moments(int part_fp, const InstDesc* D, int inst, long long ntiles, const void* pos0,
                                long long cstride, const uint32_t* fill, double* nm, hipStream_t s) {
    if (part_fp == 64)
        hipLaunchKernelGGL(k_node_moments<double>, dim3((unsigned)ntiles), dim3(256), 0, s, D, inst,
                           (const unsigned char*)pos0, cstride, fill, nm);
    else
        hipLaunchKernelGGL(k_node_moments<float>, dim3((unsigned)ntiles), dim3(256), 0, s, D, inst,
                           (const unsigned char*)pos0, cstride, fill, nm);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_collect_finish(long long nslab, int K, double mass, const double* facc,
                                                        const double* nm, float* X, float* Y) {
    const long long sn = (long long)blockIdx.x * 256 + threadIdx.x;
    if (sn >= nslab) return;
    for (int q = 0; q < NF; ++q) X[sn * NF + q] = (float)(facc[sn * NF + q] / K);
    if (!Y) return;
    const double* o = nm + sn * 10;
    const double cnt = o[0];
    double u[3] = {0.0, 0.0, 0.0};
    if (cnt > 0.0)
        for (int a = 0; a < 3; ++a) u[a] = o[1 + a] / cnt;
    for (int a = 0; a < 3; ++a) Y[sn * NOUT + a] = (float)u[a];
    const int A[6] = {0, 1, 2, 0, 0, 1}, B[6] = {0, 1, 2, 1, 2, 2};
    for (int q = 0; q < 6; ++q)
        Y[sn * NOUT + 3 + q] = (float)(mass * (o[4 + q] - cnt * u[A[q]] * u[B[q]]) / K);
}

hipError_t closure_collect_finish(long long nslab, int K, double mass, const double* facc, const double* nm,
                                  float* X, float* Y, hipStream_t s) {
    hipLaunchKernelGGL(k_collect_finish, dim3(nblk(nslab)), dim3(256), 0, s, nslab, K, mass, facc, nm, X, Y);
    return hipGetLastError();
}

}  // namespace lbmpcd
