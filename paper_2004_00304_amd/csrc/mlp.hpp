// mlp.hpp -- launchers of the learned closure's kernels (host side).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace lbmpcd {

// The closure network: 271 features (the 3x3x3 stencil of rho, u(3) and
// Pi(6) around a slab node, plus the node's shear rate) -> 128 -> 128 -> 128
// -> 9 outputs (the node's MPCD mean velocity (3) and kinetic stress (6)),
// GELU between layers.  The first layer's inputs are padded to 288.
constexpr int NF = 271, NFP = 288, NH = 128, NOUT = 9;
// Flat FP32 parameter block: W1[NH][NFP] b1[NH] W2[NH][NH] b2 W3[NH][NH] b3
// W4[NOUT][NH] b4[NOUT] (each weight matrix is [out][in]).
constexpr long long OFF_W1 = 0;
constexpr long long OFF_B1 = OFF_W1 + (long long)NH * NFP;
constexpr long long OFF_W2 = OFF_B1 + NH;
constexpr long long OFF_B2 = OFF_W2 + (long long)NH * NH;
constexpr long long OFF_W3 = OFF_B2 + NH;
constexpr long long OFF_B3 = OFF_W3 + (long long)NH * NH;
constexpr long long OFF_W4 = OFF_B3 + NH;
constexpr long long OFF_B4 = OFF_W4 + (long long)NOUT * NH;
constexpr long long NPARAM = OFF_B4 + NOUT;
// The BF16 weights in the order the fused inference kernel reads them: for
// layer l, k step s (16 inputs), 32-column block b and lane t of a wave, the
// 8 values W[32 b + t % 32][16 s + 8 (t / 32) + j], j = 0..7 (zero past the
// last output), so that every lane's 16 bytes of a (step, block) are
// contiguous.
constexpr long long FRAG_L1 = 0;
constexpr long long FRAG_L2 = FRAG_L1 + (long long)(NFP / 16) * 4 * 512;
constexpr long long FRAG_L3 = FRAG_L2 + (long long)(NH / 16) * 4 * 512;
constexpr long long FRAG_L4 = FRAG_L3 + (long long)(NH / 16) * 4 * 512;
constexpr long long NFRAG = FRAG_L4 + (long long)(NH / 16) * 1 * 512;
// Standardisation: feature mean[NF], std[NF], target mean[NOUT], std[NOUT].
constexpr long long NSTATS = 2 * NF + 2 * NOUT;
// The network's velocity outputs are relative to the LB velocity of the node
// itself: the centre entry (dz = dy = dx = 0, the 14th of 27) of the
// stencil, features UC..UC+2.  Targets and forward outputs in physical units
// are absolute.
constexpr int UC = 13 * 10 + 1;

enum GemmEpilogue { EPI_NONE = 0, EPI_GELU = 1, EPI_GELU_GRAD = 2 };

// C(m, n) = beta * C(m, n) + sum_k A(m, k) B(k, n) (+ bias[n]), BF16 operands
// A(m, k) = A[m * sam + k * sak], B(k, n) = B[k * sbk + n * sbn], FP32
// accumulation.  Outputs (any may be null): Z = value before the activation,
// C = value after it (FP32), Cb = the same rounded to BF16.
struct GemmArgs {
    long long M, N, K;
    const uint16_t* A; long long sam, sak;
    const uint16_t* B; long long sbk, sbn;
    const float* bias;
    float* C; long long ldc; float beta;
    uint16_t* Cb; long long ldcb;
    float* Z; long long ldz;
    const float* Zprev; long long ldzp;  // EPI_GELU_GRAD: multiply by GELU'(Zprev)
    int epi;
};

hipError_t launch_gemm(const GemmArgs& g, hipStream_t s);

// Activations of a batch of rows: inputs, pre-activations and BF16 outputs of
// the hidden layers, the network output, and the gradients of back-propagation.
struct ClosureBufs {
    long long rows;
    uint16_t* X;              // [rows][NFP] standardised features (BF16)
    float* Z[3];              // [rows][NH] hidden pre-activations
    uint16_t* H[3];           // [rows][NH] hidden activations (BF16)
    float* Y;                 // [rows][NOUT] output (standardised units)
    float* dY; uint16_t* dYb; // [rows][NOUT] loss gradient
    float* dZ[3]; uint16_t* dZb[3];  // [rows][NH] hidden pre-activation gradients
};
// Bytes of ClosureBufs for `rows` rows, and the carve-up of such an area
// (every buffer starts on a 256-byte boundary).
constexpr size_t closure_al256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t closure_fwd_bytes(long long rows) {
    return closure_al256((size_t)rows * NFP * 2) +
           3 * (closure_al256((size_t)rows * NH * 4) + closure_al256((size_t)rows * NH * 2)) +
           closure_al256((size_t)rows * NOUT * 4);
}
size_t closure_bufs_bytes(long long rows, bool backward);
void closure_bufs_carve(unsigned char* base, long long rows, bool backward, ClosureBufs& b);

// Network passes.  P32: FP32 parameters, Pb: their BF16 copy.
hipError_t mlp_forward(const float* P32, const uint16_t* Pb, const ClosureBufs& b, hipStream_t s);
// Loss (mean squared error over rows x NOUT, accumulated into *loss) and the
// parameter gradient G (FP32, layout of the parameter block) of one batch.
hipError_t mlp_backward(const uint16_t* Pb, const float* Yt, const ClosureBufs& b, float* G, double* loss,
                        hipStream_t s);
hipError_t mlp_adam(float* P32, uint16_t* Pb, const float* G, float* m, float* v, long long t, float lr,
                    float beta1, float beta2, float eps, hipStream_t s);
hipError_t mlp_init(float* P32, uint16_t* Pb, float* m, float* v, uint32_t k0, uint32_t k1, hipStream_t s);
hipError_t mlp_refresh_bf16(const float* P32, uint16_t* Pb, hipStream_t s);
// Output rows in standardised units -> physical units.
hipError_t mlp_destandardize(const float* Y, const float* stats, const float* X, long long rows, float* out,
                             hipStream_t s);

// Data: column statistics of raw features / targets, standardised batches.
hipError_t mlp_stats(const float* X, const float* Y, long long n, double* sums, float* stats, hipStream_t s);
hipError_t mlp_gather(const float* X, const float* Y, long long n, const float* stats, long long rows,
                      bool draw, uint32_t k0, uint32_t k1, uint32_t step, uint16_t* Xb, float* Yb, hipStream_t s);

// Coupling: features of the slab nodes of one channel from its populations,
// either raw into an FP64 accumulator (facc, [nslab][NF]) or standardised
// into BF16 network inputs (Xb, [nslab][NFP]).
hipError_t closure_features(int lb_fp, const InstDesc* D, int inst, long long nslab, const void* f,
                            double* facc, const float* stats, uint16_t* Xb, float* uc, hipStream_t s);
// Network output -> feedback sums (count 1, predicted velocity) of every slab
// node; with do_prof also into the profile accumulators.
hipError_t closure_to_acc(const InstDesc* D, int inst, long long nslab, const float* Y, const float* stats,
                          const float* uc, double* acc, double* prof, int do_prof, hipStream_t s);
// Fused inference of every slab node of the current populations: the moments
// and shear rate of the band rows [y0, y0 + nyb) into M (nband x 12 floats),
// then features and the four layers in one kernel (Pf: scratch for the
// weights in fragment order, NFRAG BF16 values).  Y: standardised output
// [nslab][NOUT]; uc: the node's LB velocity [nslab][3].
hipError_t closure_predict(int lb_fp, const InstDesc* D, int inst, long long nslab, long long nband, int y0,
                           int nyb, const void* f, float* M, const float* stats, const uint16_t* Pb,
                           uint16_t* Pf, const float* P32, float* Y, float* uc, hipStream_t s);
// Physical units from a standardised output and the nodes' LB velocities.
hipError_t mlp_destandardize_uc(const float* Y, const float* stats, const float* uc, long long rows, float* out,
                                hipStream_t s);
// Particle moments per slab node (count, sum v, sum v v) of one channel;
// one workgroup per particle tile.
hipError_t closure_node_moments(int part_fp, const InstDesc* D, int inst, long long ntiles, const void* pos0,
                                long long cstride, const uint32_t* fill, double* nm, hipStream_t s);
// Averages of a collection window of K LB steps: features X [nslab][NF] and
// targets Y [nslab][NOUT] (mean velocity, kinetic stress per unit volume).
hipError_t closure_collect_finish(long long nslab, int K, double mass, const double* facc, const double* nm,
                                  float* X, float* Y, hipStream_t s);

}  // namespace lbmpcd
