// api.hip -- host side of the C ABI declared in include/lbmpcd.h: parameter
// validation, workspace layout, launch sequencing on the caller's stream,
// transfers and error reporting.  The library allocates no device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbmpcd.h"
#include "common.hpp"
#include "mlp.hpp"
#include "launch.hpp"

using namespace lbmpcd;

// Activations of lbmpcd_closure_forward_noalloc: a file-scope device array, one
// copy on every device the library runs on, held until the process ends.  In
// host code this name is only a stand-in for the symbol; the device address of
// each copy comes from hipGetSymbolAddress (noalloc_scratch below).
static __device__ __align__(256) unsigned char scratch[closure_fwd_bytes(LBMPCD_NOALLOC_MAX_ROWS)];

struct lbmpcd_ctx {
    int n_inst = 0, dim = 2, lb_fp = 64, part_fp = 64, S = 1, Q = 9, mpcd = 0;
    std::vector<lbmpcd_params> params;
    std::vector<InstDesc> desc;
    hipStream_t stream = nullptr;
    int device = 0;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    InstDesc* d_desc = nullptr;
    int* d_tile_inst = nullptr;
    void* f[2] = {nullptr, nullptr};
    int fcur = 0;
    PartBuf part[2];
    int pcur = 0;
    uint32_t* fill[2] = {nullptr, nullptr};
    double* ub = nullptr;
    double* uf = nullptr;
    double* tb = nullptr;         // [6][band nodes] Chapman-Enskog tensor (reinject 1)
    double* tf = nullptr;         // [6][buffer cells] the same, interpolated
    double* acc = nullptr;
    double* fbu = nullptr;      // [3][total_slab] running means the feedback projects
    double* prof = nullptr;
    double* shifts = nullptr;   // [n_inst][2][S][3] grid shifts drawn by the LB kernel
    DevStats* stats = nullptr;
    uint32_t* ovf = nullptr;      // [2 + total_tiles] overflow list of the two-pass particle launch
    long long* clock = nullptr;
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    size_t prof_bytes = 0, acc_bytes = 0;
    long long total_nodes = 0, total_band = 0, total_ufine = 0, total_tiles = 0, total_slots = 0,
              total_particles = 0, total_slab = 0;
    size_t lds = 0;
    int cap_max = 0;              // largest tile capacity
    int exp_max = 0;              // largest expected tile occupancy
    bool split_ok = false;        // the particle launch may take the six-slot form
    int wg_threads = 0;           // particle kernel workgroup size
    int coll_bit = 0;             // 4 for the MPCD-AT collision (particle kernel mode bit)
    int ce_bit = 0;               // 8 for the Chapman-Enskog exchange (particle kernel mode bit)
    int det_bit = 0;              // 16 for the deterministic mode (particle kernel mode bit)
    int xcd_blocked = 1;          // XCD-blocked tile order of the particle kernel
    long long cstride = 0;        // bytes between the component arrays of a particle buffer
    long long t = 0;
    bool pending = false, sampling = false, any_feedback = false;
    long long sampled_steps = 0;
    std::string err;
    int sticky = 0;
    // kernel timing (host-side event objects only)
    bool timing = false;
    struct Mark { int cls; hipEvent_t a, b; };
    std::vector<Mark> marks;
    std::vector<hipEvent_t> pool;
    double timing_ms[5] = {0, 0, 0, 0, 0};
    long long timing_n[5] = {0, 0, 0, 0, 0};
    // steady-state steps replayed from a captured graph
    bool use_graphs = true;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_key = -1;
    // learned closure (channel 0)
    bool closure = false;          // region reserved
    float* cl_P = nullptr;         // [NPARAM] FP32 parameters
    uint16_t* cl_Pb = nullptr;     // [NPARAM] BF16 copy
    uint16_t* cl_Pf = nullptr;     // [NFRAG] BF16 weights in the fused kernel's fragment order
    float* cl_G = nullptr;         // [NPARAM] gradient
    float* cl_m = nullptr;         // [NPARAM] Adam first moment
    float* cl_v = nullptr;         // [NPARAM] Adam second moment
    float* cl_stats = nullptr;     // [NSTATS] standardisation
    double* cl_sums = nullptr;     // [2 (NF + NOUT)] column sums
    double* cl_loss = nullptr;     // [1]
    double* cl_facc = nullptr;     // [nslab][NF] feature sums of a collection window
    double* cl_nm = nullptr;       // [nslab][10] particle moment sums
    float* cl_uc = nullptr;        // [nslab][3] LB velocity of each slab node (surrogate step)
    ClosureBufs cl_inf;            // inference activations, one row per slab node
    long long cl_nslab = 0;
    bool cl_ready = false;         // parameters and statistics set
    bool cl_collect = false;       // collection window: features after every LB collide-stream
    bool cl_on = false;            // surrogate replaces the MPCD steps
    bool cl_fell_back = false;     // a check found the surrogate off by more than cl_tol
    double cl_tol = 0.02, cl_last_err = -1.0;
    int cl_every = 0, cl_burst = 40;
    long long cl_since = 0, cl_adam_t = 0;
};

namespace {

thread_local std::string g_err;

int fail(lbmpcd_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg; else g_err = msg;
    return code;
}

// Device address of the `scratch` array on each device, resolved once per
// device (with that device current) at lbmpcd_init.
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

int resolve_noalloc_scratch(int device, std::string& msg) {
    if (device < 0 || device >= MAX_DEVICES) { msg = "device index beyond the library's table"; return LBMPCD_E_DEVICE; }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return 0;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        msg = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return LBMPCD_E_DEVICE;
    }
    g_scratch_ptr[device] = p;
    return 0;
}

void* noalloc_scratch(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

#define HIPCHK(ctx, expr)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(ctx, LBMPCD_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Geometry {
    // per-instance derived sizes
    int R = 0, Cx = 0, Cz = 1, CyB = 0, ywrap = 0, bot_wall = 0, top_wall = 0;
    int Tx = 1, Ty = 1, Tz = 1, ntx = 0, nty = 0, ntz = 0, cap = 0, nct = 0;
    long long ncells = 0, Np = 0, ntiles = 0, init_per = 0;
    int by0 = 0, nyb = 0, NB = 0;
    long long nband = 0, nufine = 0, nslab = 0;
};

int ilog2(int v) {
    int l = 0;
    while ((1 << (l + 1)) <= v) ++l;
    return l;
}

int choose_tile(const lbmpcd_params& p, Geometry& g, std::string& msg) {
    int T[3] = {p.tile[0], p.tile[1], p.tile[2]};
    if (T[0] <= 0 || T[1] <= 0 || (p.dim == 3 && T[2] <= 0)) {
        // aim at ~1280 expected particles per tile
        const int per_tile = p.tile_target > 0 ? p.tile_target : 1280;
        int target = std::max(8, std::min(MAX_NCT, per_tile / std::max(1, p.ppc)));
        // shapes below 8 cells serve only dense cells (hundreds of particles
        // per cell, as in the paper's runs), whose tiles would overflow
        static const int opts3[][3] = {{1, 1, 1}, {2, 1, 1}, {2, 2, 1}, {2, 2, 2},
                                       {4, 2, 2}, {4, 4, 2}, {4, 4, 4}, {4, 4, 8}};
        static const int opts2[][3] = {{1, 1, 1}, {2, 1, 1}, {2, 2, 1}, {4, 2, 1},
                                       {4, 4, 1}, {8, 4, 1}, {8, 8, 1}, {16, 8, 1}};
        const int(*opts)[3] = p.dim == 3 ? opts3 : opts2;
        int pick = 7;
        for (int i = 0; i < 8; ++i) {
            if (opts[i][0] * opts[i][1] * opts[i][2] >= target) { pick = i; break; }
        }
        // the next smaller shape when the capacity would exceed the kernel's limit
        const double cf0 = p.capacity_factor > 0 ? p.capacity_factor : 1.3;
        while (pick > 0 && std::ceil(cf0 * p.ppc * opts[pick][0] * opts[pick][1] * opts[pick][2]) + 64 > 8 * WG)
            --pick;
        T[0] = opts[pick][0]; T[1] = opts[pick][1]; T[2] = opts[pick][2];
        // The list fixes the number of cells; among the shapes of that many
        // cells (sides powers of two, at least two rows unless the list's
        // shape has one) whose LDS windows fit, the one with the fewest tiles
        // over the shifted grid, then the smallest surface (fewer particles
        // change tiles); taken when it saves at least 1 % of the tiles.  The
        // grid's R + 1 rows are rarely a multiple of Ty, and the last layer of
        // tiles holds only the remainder: on the thin film's 17 rows 4-row
        // tiles leave a layer of one-row tiles (a fifth of the workgroups
        // nearly empty), 2-row tiles one in nine.  Measured per particle
        // launch: film 4x4x8 7.24 ms, 8x2x8 6.76; 3D channel 4x4x4 3.22 ms,
        // 4x2x8 3.10, 8x1x8 3.13 (fewer tiles, but one-row tiles lose more
        // particles every step).
        const int S = T[0] * T[1] * T[2], r = p.refine;
        const int ty_min = T[1] >= 2 ? 2 : 1;
        auto fits = [&](int tx, int ty, int tz) {
            const int wx = (tx + r - 1) / r + 2, wy = (ty + r - 1) / r + 2;
            const int wz = p.dim == 3 ? (tz + r - 1) / r + 2 : 1;
            const int uw = (tx + 1) * (ty + 1) * (p.dim == 3 ? tz + 1 : 1);
            return uw <= MAX_UFC && wx * wy * wz <= (p.dim == 3 ? std::min(MAX_WIN, NM_WIN) : MAX_WIN) &&
                   ty + 4 <= MAX_WJ;
        };
        auto tiles = [&](int tx, int ty, int tz) {
            return (long long)((g.Cx + tx - 1) / tx) * ((g.CyB + ty - 1) / ty) * ((g.Cz + tz - 1) / tz);
        };
        const bool fits0 = fits(T[0], T[1], T[2]);
        const long long n0 = tiles(T[0], T[1], T[2]);
        long long best_n = -1;
        int best_s = 0, B[3] = {T[0], T[1], T[2]};
        for (int tx = 1; tx <= S; tx *= 2)
            for (int ty = ty_min; tx * ty <= S; ty *= 2) {
                const int tz = S / (tx * ty);
                if (p.dim == 2 && tz != 1) continue;
                if (!fits(tx, ty, tz)) continue;
                const long long n = tiles(tx, ty, tz);
                const int sf = tx * ty + ty * tz + tx * tz;
                if (best_n < 0 || n < best_n || (n == best_n && sf < best_s)) {
                    best_n = n; best_s = sf;
                    B[0] = tx; B[1] = ty; B[2] = tz;
                }
            }
        if (best_n >= 0 && (!fits0 || best_n * 100 <= n0 * 99)) {
            T[0] = B[0]; T[1] = B[1]; T[2] = B[2];
        }
    }
    if (p.dim == 2) T[2] = 1;
    for (int k = 0; k < 3; ++k)
        if (T[k] & (T[k] - 1)) { msg = "tile sides must be powers of two"; return 1; }
    g.Tx = T[0]; g.Ty = T[1]; g.Tz = T[2];
    g.nct = g.Tx * g.Ty * g.Tz;
    if (g.nct > MAX_NCT) { msg = "tile has more than 128 cells"; return 1; }
    double cf = p.capacity_factor > 0 ? p.capacity_factor : 1.3;
    long long cap = (long long)std::ceil(cf * p.ppc * g.nct) + 64;
    cap = (long long)align_up((size_t)cap, 64);
    if (cap > 8 * WG) { msg = "tile capacity exceeds 2048 particles; use a smaller tile"; return 1; }
    g.cap = (int)cap;
    return 0;
}

int geometry(const lbmpcd_params& p, Geometry& g, std::string& msg) {
    if (!p.mpcd) return 0;
    const int r = p.refine;
    g.R = (p.yhi - p.ylo) * r;
    g.Cx = p.n[0] * r;
    g.Cz = p.dim == 3 ? p.n[2] * r : 1;
    g.ywrap = (!p.walls_y && p.ylo == 0 && p.yhi == p.n[1] && p.buf_lo == 0 && p.buf_hi == 0) ? 1 : 0;
    g.CyB = g.ywrap ? g.R : g.R + 1;
    g.bot_wall = (p.walls_y && p.ylo == 0) ? 1 : 0;
    g.top_wall = (p.walls_y && p.yhi == p.n[1]) ? 1 : 0;
    g.ncells = (long long)g.Cx * g.CyB * g.Cz;
    g.Np = (long long)g.Cx * g.R * g.Cz * p.ppc;
    if (choose_tile(p, g, msg)) return 1;
    g.ntx = (g.Cx + g.Tx - 1) / g.Tx;
    g.nty = (g.CyB + g.Ty - 1) / g.Ty;
    g.ntz = (g.Cz + g.Tz - 1) / g.Tz;
    g.ntiles = (long long)g.ntx * g.nty * g.ntz;
    // the particle kernels address a channel's slots with 32-bit offsets
    if (g.ntiles >= (1LL << 31) || g.ntiles * g.cap * (p.part_fp / 8) >= (1LL << 32)) {
        msg = "the particle slots of one channel exceed 4 GiB per component";
        return 1;
    }
    // initial placement: the particles of every slab cell in the tile of that cell
    g.init_per = (long long)g.nct * p.ppc;
    if (g.init_per > g.cap) { msg = "initial placement exceeds the tile capacity"; return 1; }
    g.by0 = std::max(p.ylo - 1, 0);
    int by1 = std::min(p.yhi + 1, p.n[1]);
    g.nyb = by1 - g.by0;
    g.nband = (long long)p.n[0] * g.nyb * p.n[2];
    g.NB = (p.buf_lo + p.buf_hi) * r;
    g.nufine = (long long)g.Cx * g.NB * g.Cz;
    g.nslab = (long long)p.n[0] * (p.yhi - p.ylo) * p.n[2];
    return 0;
}

double ce_nu(const lbmpcd_params& p);

int validate_one(const lbmpcd_params& p, std::string& msg) {
    if (p.abi_version != LBMPCD_ABI_VERSION) { msg = "abi_version mismatch"; return LBMPCD_E_INVALID; }
    if (p.struct_size != sizeof(lbmpcd_params)) { msg = "struct_size mismatch"; return LBMPCD_E_INVALID; }
    if (p.dim != 2 && p.dim != 3) { msg = "dim must be 2 or 3"; return LBMPCD_E_INVALID; }
    if (p.n[0] < 1 || p.n[1] < 1 || p.n[2] < 1) { msg = "n must be positive"; return LBMPCD_E_INVALID; }
    if (p.dim == 2 && (p.n[2] != 1 || p.g[2] != 0.0)) { msg = "2D needs nz = 1 and g_z = 0"; return LBMPCD_E_INVALID; }
    if (p.lb_fp != 32 && p.lb_fp != 64) { msg = "lb_fp must be 32 or 64"; return LBMPCD_E_INVALID; }
    if (!(p.tau > 0.5)) { msg = "tau must exceed 1/2"; return LBMPCD_E_INVALID; }
    if (!(p.rho0 > 0.0)) { msg = "rho0 must be positive"; return LBMPCD_E_INVALID; }
    if (p.init_flow && !p.walls_y) { msg = "init_flow needs walls"; return LBMPCD_E_INVALID; }
    if ((long long)p.n[0] * p.n[1] * p.n[2] > (1LL << 40)) { msg = "domain too large"; return LBMPCD_E_INVALID; }
    if (p.closure && !p.mpcd) { msg = "the closure needs the MPCD slab"; return LBMPCD_E_INVALID; }
    if (!p.mpcd) return 0;
    if (p.collision != 0 && p.collision != 1) { msg = "collision must be 0 (SRD) or 1 (MPCD-AT)"; return LBMPCD_E_UNSUPPORTED; }
    if (p.wg_threads != 0 && p.wg_threads != 128 && p.wg_threads != 256 && p.wg_threads != 512) { msg = "wg_threads must be 0, 128, 256 or 512"; return LBMPCD_E_INVALID; }
    if (p.tile_target < 0 || p.tile_target > 8 * WG) { msg = "tile_target out of range"; return LBMPCD_E_INVALID; }
    if (p.closure && p.dim != 3) { msg = "the closure needs dim 3"; return LBMPCD_E_INVALID; }
    if (p.part_fp != 32 && p.part_fp != 64) { msg = "part_fp must be 32 or 64"; return LBMPCD_E_INVALID; }
    if (p.ylo < 0 || p.yhi > p.n[1] || p.ylo >= p.yhi) { msg = "slab outside the domain"; return LBMPCD_E_INVALID; }
    if (p.refine < 1 || p.substeps < 1 || p.ppc < 1) { msg = "refine, substeps, ppc must be >= 1"; return LBMPCD_E_INVALID; }
    if (p.substeps > 255) { msg = "at most 255 substeps"; return LBMPCD_E_INVALID; }
    if (p.buf_lo < 0 || p.buf_hi < 0 || p.buf_lo + p.buf_hi > p.yhi - p.ylo) { msg = "buffers exceed the slab"; return LBMPCD_E_INVALID; }
    const bool bw = p.walls_y && p.ylo == 0, tw = p.walls_y && p.yhi == p.n[1];
    if ((bw && p.buf_lo) || (tw && p.buf_hi)) { msg = "a wall face has no buffer"; return LBMPCD_E_INVALID; }
    if ((bw || tw) && p.g[1] != 0.0) { msg = "walls in the slab need g_y = 0"; return LBMPCD_E_INVALID; }
    if (!(p.mass > 0.0) || p.kT < 0.0) { msg = "mass must be positive, kT non-negative"; return LBMPCD_E_INVALID; }
    if (p.reinject != 0 && p.reinject != 1) { msg = "reinject must be 0 or 1"; return LBMPCD_E_INVALID; }
    if (!std::isfinite(p.ce_nu)) { msg = "ce_nu must be finite"; return LBMPCD_E_INVALID; }
    if (p.fb_window < 0) { msg = "fb_window must be >= 0"; return LBMPCD_E_INVALID; }
    if (p.deterministic != 0 && p.deterministic != 1) { msg = "deterministic must be 0 or 1"; return LBMPCD_E_INVALID; }
    if (p.schedule != 0 && p.schedule != 1) { msg = "schedule must be 0 or 1"; return LBMPCD_E_INVALID; }
    if (p.deterministic && p.mpcd && (p.closure || p.reinject)) {
        msg = "the deterministic mode covers neither the closure nor the Chapman-Enskog exchange";
        return LBMPCD_E_UNSUPPORTED;
    }
    if (p.reinject && !(p.kT > 0.0)) { msg = "the Chapman-Enskog exchange needs kT > 0"; return LBMPCD_E_INVALID; }
    const bool ywrap = !p.walls_y && p.ylo == 0 && p.yhi == p.n[1] && p.buf_lo == 0 && p.buf_hi == 0;
    if (!p.walls_y && !ywrap && (p.ylo < 1 || p.yhi > p.n[1] - 1)) {
        msg = "without walls the slab must be the whole periodic box or stay one row clear of y = 0, ny";
        return LBMPCD_E_UNSUPPORTED;
    }
    Geometry g;
    if (geometry(p, g, msg)) return LBMPCD_E_INVALID;
    if (g.Np >= (1LL << 32) - 1) { msg = "too many particles for 32-bit ids"; return LBMPCD_E_INVALID; }
    if (p.reinject && !std::isfinite(ce_nu(p))) {
        msg = "the default Chapman-Enskog coefficient is not finite for this collision rule (SRD at alpha = 0); set ce_nu";
        return LBMPCD_E_INVALID;
    }
    return 0;
}

// Kinetic part of the MPCD viscosity: MPCD-AT Eq. 7's first term; SRD the
// kinetic terms of the SRD literature (2D and 3D).
double nu_kinetic(const lbmpcd_params& p) {
    const double N = (double)p.ppc, q = N - 1.0 + std::exp(-N), kin = p.kT / p.substeps / p.mass;
    if (p.collision == 1) return kin * (N / q - 0.5);
    const double al = p.alpha_deg * 3.14159265358979323846 / 180.0;
    if (p.dim == 2) return kin * (N / (q * (1.0 - std::cos(2.0 * al))) - 0.5);
    return kin * (5.0 * N / (q * (4.0 - 2.0 * std::cos(al) - 2.0 * std::cos(2.0 * al))) - 0.5);
}

// Stress coefficient of the Chapman-Enskog exchange: the kinetic stress the
// MPCD fluid carries right after a collision, when the exchange redraws the
// buffer.  Streaming through the shear adds kT dt/m per unit shear rate over
// a step and nu_kin is the step average, so right after the collision it is
// nu_kin - kT dt/(2m).  ce_nu != 0 overrides it.
double ce_nu(const lbmpcd_params& p) {
    if (p.ce_nu != 0.0) return p.ce_nu;
    return nu_kinetic(p) - 0.5 * p.kT / p.substeps / p.mass;
}

// LB steps of the feedback's running mean when fb_window is 0
constexpr int FB_WINDOW_DEFAULT = 50;

// The six-slot form of the particle launch (six particles per thread at 256
// threads, then an overflow pass over the tiles holding more than 1536) is
// offered for tiles of 1025-2048 slots whose expected occupancy plus two
// Poisson standard deviations is within 1536.  With the default shape it is
// taken only for grids of at least SPLIT_MIN_TILES tiles: below that the
// launch is one round of workgroups, which the extra launch only delays.
constexpr long long SPLIT_MIN_TILES = 4096;
static bool six_slot_fits(int cap_max, int exp_max) {
    const double e = (double)exp_max;
    return cap_max > 4 * 256 && cap_max <= 8 * 256 && e + 2.0 * std::sqrt(e) <= 6.0 * 256;
}

// Default particle workgroup: 256 threads.  Binary64 particles in tiles of
// more than 1024 slots take 512 threads (four particles per thread) unless
// the six-slot form applies at 256, which is faster: eight binary64
// particles per thread spill.
static int default_wg_threads(int part_fp, int cap_max, int exp_max, long long tiles) {
    if (part_fp != 64 || cap_max <= 4 * 256) return 256;
    return (six_slot_fits(cap_max, exp_max) && tiles >= SPLIT_MIN_TILES) ? 256 : 512;
}

struct Layout {
    size_t desc, tile_inst, f0, f1, ub, uf, tb, tf, acc, fbu, prof, fill0, fill1, stats, ovf, clock, shifts, scratch, end;
    size_t cl_P, cl_Pb, cl_Pf, cl_G, cl_m, cl_v, cl_stats, cl_sums, cl_loss, cl_facc, cl_nm, cl_uc, cl_inf;
    size_t part[2];       // particle buffer: 2 dim component arrays of cstride bytes, then ids
    size_t cstride;
    size_t acc_bytes, prof_bytes, scratch_bytes;
};

int build(const lbmpcd_params* p, int n, std::vector<InstDesc>& D, Layout& L, long long tot[7], std::string& msg) {
    D.assign(n, InstDesc{});
    long long node = 0, band = 0, ufine = 0, tiles = 0, slots = 0, parts = 0, slab = 0, prow = 0;
    size_t max_field = 0;
    const int Q = p[0].dim == 2 ? 9 : 19;
    for (int i = 0; i < n; ++i) {
        const lbmpcd_params& q = p[i];
        Geometry g;
        if (geometry(q, g, msg)) return LBMPCD_E_INVALID;
        InstDesc& d = D[i];
        d.nx = q.n[0]; d.ny = q.n[1]; d.nz = q.n[2]; d.walls_y = q.walls_y;
        d.N = (long long)q.n[0] * q.n[1] * q.n[2];
        d.node_off = node;
        d.omega = 1.0 / q.tau;
        d.src = 1.0 - 0.5 / q.tau;
        for (int k = 0; k < 3; ++k) d.g[k] = q.g[k];
        d.rho0 = q.rho0; d.tau = q.tau; d.init_flow = q.init_flow; d.mpcd = q.mpcd;
        d.ylo = q.ylo; d.yhi = q.yhi; d.buf_lo = q.buf_lo; d.buf_hi = q.buf_hi;
        d.r = q.refine; d.R = g.R; d.Cx = g.Cx; d.Cz = g.Cz; d.CyB = g.CyB; d.ywrap = g.ywrap;
        d.bot_wall = g.bot_wall; d.top_wall = g.top_wall; d.ppc = q.ppc; d.feedback = q.feedback;
        d.grid_shift = q.grid_shift;
        d.ncells = g.ncells; d.Np = g.Np; d.part_off = parts; d.init_per = g.init_per;
        d.Tx = g.Tx; d.Ty = g.Ty; d.Tz = g.Tz; d.ntx = g.ntx; d.nty = g.nty; d.ntz = g.ntz;
        d.lTx = ilog2(g.Tx); d.lTy = ilog2(g.Ty); d.lTz = ilog2(g.Tz);
        d.lr = (p[i].refine & (p[i].refine - 1)) == 0 ? ilog2(p[i].refine) : -1;
        d.cap = g.cap; d.nct = g.nct; d.ntiles = g.ntiles; d.tile_off = tiles; d.slot_off = slots;
        d.by0 = g.by0; d.nyb = g.nyb; d.band_off = band; d.NB = g.NB; d.ufine_off = ufine;
        d.nslab = g.nslab; d.acc_off = slab; d.prof_off = prow;
        d.a = q.mpcd ? 1.0 / q.refine : 0.0;
        d.dt = q.mpcd ? 1.0 / q.substeps : 0.0;
        for (int k = 0; k < 3; ++k) { d.gh[k] = 0.5 * q.g[k] * d.dt; d.gdt[k] = q.g[k] * d.dt; }
        for (int k = 0; k < 3; ++k) { d.ghf[k] = (float)d.gh[k]; d.gdtf[k] = (float)d.gdt[k]; }
        d.dtf = (float)d.dt;
        d.sd = q.mass > 0 ? std::sqrt(q.kT / q.mass) : 0.0;
        const double alpha = q.alpha_deg * 3.141592653589793 / 180.0;
        d.cos_a = std::cos(alpha);
        d.sin_a = std::sin(alpha);
        d.mass = q.mass; d.kT = q.kT;
        d.key0 = (uint32_t)(q.seed & 0xFFFFFFFFu);
        d.key1 = (uint32_t)(q.seed >> 32) ^ q.instance;
        d.S = q.mpcd ? q.substeps : 0;
        d.ce = (q.mpcd && q.reinject) ? 1 : 0;
        d.det = q.deterministic ? 1 : 0;
        d.ce_scale = d.ce ? ce_nu(q) * q.mass / q.kT / (2.0 * q.tau / 3.0) : 0.0;
        d.fb_lam = 1.0 / (double)(q.fb_window > 0 ? q.fb_window : FB_WINDOW_DEFAULT);
        node += d.N;
        band += g.nband;
        ufine += g.nufine;
        tiles += g.ntiles;
        slots += g.ntiles * (long long)g.cap;
        parts += g.Np;
        slab += g.nslab;
        prow += (long long)NCOPY * g.R;
        size_t fsz = std::max<size_t>((size_t)d.N * 8 * 6, (size_t)d.N * Q * 8);
        fsz = std::max<size_t>(fsz, (size_t)g.Np * 8 * q.dim);
        fsz = std::max<size_t>(fsz, (size_t)g.ncells * 8 * q.dim);
        max_field = std::max(max_field, fsz);
    }
    if (slots >= 0x7FFFFFFFLL) { msg = "too many particle slots for 31-bit slot indices"; return LBMPCD_E_INVALID; }
    tot[0] = node; tot[1] = band; tot[2] = ufine; tot[3] = tiles; tot[4] = slots; tot[5] = parts; tot[6] = slab;
    const int dim = p[0].dim;
    const size_t lbw = p[0].lb_fp == 64 ? 8 : 4, pw = p[0].part_fp == 64 ? 8 : 4;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + std::max<size_t>(bytes, 1), 256); return at; };
    L.desc = take(sizeof(InstDesc) * n);
    L.tile_inst = take(4 * (size_t)tiles);
    L.f0 = take((size_t)Q * node * lbw);
    L.f1 = take((size_t)Q * node * lbw);
    L.ub = take(3 * (size_t)band * 8);
    L.uf = take((size_t)dim * ufine * 8);
    const bool ce = p[0].mpcd && p[0].reinject;
    L.tb = take(ce ? (size_t)CE_NT * band * 8 : 0);
    L.tf = take(ce ? (size_t)CE_NT * ufine * 8 : 0);
    L.acc_bytes = 4 * (size_t)slab * 8;
    L.acc = take(L.acc_bytes);
    L.fbu = take(3 * (size_t)slab * 8);
    L.prof_bytes = 4 * (size_t)prow * 8;
    L.prof = take(L.prof_bytes);
    L.fill0 = take(4 * (size_t)tiles);
    L.fill1 = take(4 * (size_t)tiles);
    L.cstride = align_up((size_t)slots * pw, 256);
    for (int b = 0; b < 2; ++b) L.part[b] = take(2 * (size_t)dim * L.cstride + (size_t)slots * 4);
    L.stats = take(sizeof(DevStats));
    L.ovf = take(4 * ((size_t)tiles + 2));
    L.clock = take(sizeof(long long));
    L.shifts = take(sizeof(double) * 6 * (size_t)n * (p[0].mpcd ? p[0].substeps : 1));
    L.scratch_bytes = std::min<size_t>(align_up(max_field, 256), (size_t)64 << 20);
    L.scratch = take(L.scratch_bytes);
    if (p[0].closure) {
        L.cl_P = take(4 * (size_t)NPARAM);
        L.cl_Pb = take(2 * (size_t)NPARAM);
        L.cl_Pf = take(2 * (size_t)NFRAG);
        L.cl_G = take(4 * (size_t)NPARAM);
        L.cl_m = take(4 * (size_t)NPARAM);
        L.cl_v = take(4 * (size_t)NPARAM);
        L.cl_stats = take(4 * (size_t)NSTATS);
        L.cl_sums = take(8 * 2 * (size_t)(NF + NOUT));
        L.cl_loss = take(8);
        L.cl_facc = take(8 * (size_t)slab * NF);
        L.cl_nm = take(8 * (size_t)slab * 10);
        L.cl_uc = take(4 * (size_t)slab * 3);
        L.cl_inf = take(closure_bufs_bytes(slab, false));
    }
    L.end = o;
    return 0;
}

int validate_all(const lbmpcd_params* p, int n, std::string& msg) {
    if (!p || n < 1) { msg = "need at least one instance"; return LBMPCD_E_INVALID; }
    for (int i = 0; i < n; ++i) {
        int e = validate_one(p[i], msg);
        if (e) { msg = "instance " + std::to_string(i) + ": " + msg; return e; }
        if (p[i].dim != p[0].dim || p[i].lb_fp != p[0].lb_fp || p[i].mpcd != p[0].mpcd ||
            (p[0].mpcd && (p[i].part_fp != p[0].part_fp || p[i].substeps != p[0].substeps))) {
            msg = "all instances must share dim, lb_fp, mpcd, part_fp and substeps";
            return LBMPCD_E_INVALID;
        }
        if (p[i].wg_threads != p[0].wg_threads || p[i].collision != p[0].collision ||
            (p[0].mpcd && p[i].reinject != p[0].reinject) || p[i].deterministic != p[0].deterministic ||
            p[i].schedule != p[0].schedule) {
            msg = "all instances must share wg_threads, the collision rule, the exchange rule, the "
                  "deterministic mode and the schedule";
            return LBMPCD_E_INVALID;
        }
        if (p[i].closure && n != 1) {
            msg = "the learned closure serves a context of one channel";
            return LBMPCD_E_UNSUPPORTED;
        }
    }
    return 0;
}

hipEvent_t take_event(lbmpcd_ctx* c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Fold recorded event pairs into the per-class sums (synchronises).
int drain_marks(lbmpcd_ctx* c) {
    if (c->marks.empty()) return 0;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto& m : c->marks) {
        float ms = 0.f;
        if (m.a && m.b && hipEventElapsedTime(&ms, m.a, m.b) == hipSuccess) {
            c->timing_ms[m.cls] += ms;
            c->timing_n[m.cls] += 1;
        }
        if (m.a) c->pool.push_back(m.a);
        if (m.b) c->pool.push_back(m.b);
    }
    c->marks.clear();
    return 0;
}

// Launch `f` bracketed by timing events of class `cls` when timing is on.
template <typename F>
hipError_t timed(lbmpcd_ctx* c, int cls, F f) {
    if (!c->timing) return f();
    if (c->marks.size() > 4096) drain_marks(c);
    hipEvent_t a = take_event(c), b = take_event(c);
    if (a) (void)hipEventRecord(a, c->stream);
    hipError_t e = f();
    if (b) (void)hipEventRecord(b, c->stream);
    c->marks.push_back({cls, a, b});
    return e;
}

int finalize(lbmpcd_ctx* c) {
    if (!c->pending || !c->mpcd) return 0;
    ParticleLaunch L{};
    L.dim = c->dim; L.part_fp = c->part_fp; L.mode = 1 | c->coll_bit | c->det_bit;
    L.D = c->d_desc; L.n_inst = c->n_inst; L.tiles = c->total_tiles;
    L.in = c->part[c->pcur]; L.out = c->part[c->pcur];
    L.fill_in = c->fill[c->pcur]; L.fill_out = c->fill[c->pcur ^ 1];
    L.tile_inst = c->d_tile_inst; L.ufine = c->uf; L.tfine = c->tf; L.acc = c->acc; L.prof = c->prof;
    L.stats = c->stats; L.clock = c->clock; L.shifts = c->shifts;
    L.coll_dt = 0; L.coll_s = c->S - 1; L.str_s = 0;
    L.diag_inst = -1; L.cell_vcm = nullptr; L.lds_bytes = c->lds; L.cap_max = c->cap_max; L.ovf = c->split_ok ? c->ovf : nullptr; L.exp_max = c->exp_max; L.wg_threads = c->wg_threads; L.cstride = c->cstride; L.xcd_blocked = c->xcd_blocked;
    HIPCHK(c, launch_particles(L, c->stream));
    c->pending = false;
    return 0;
}

int check_device_errors(lbmpcd_ctx* c) {
    DevStats s;
    HIPCHK(c, hipMemcpyAsync(&s, c->stats, sizeof(s), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // an invalid state first: the parked invalid particles can overflow the
    // tile they are parked in, which is then a consequence, not the cause
    if (s.bad_state) {
        c->sticky = LBMPCD_E_STATE;
        c->err = std::to_string(s.bad_state) +
                 " invalid particles or band nodes (a particle moved more than a period in one MPCD step or "
                 "turned non-finite, or a node next to the slab had rho <= 0 or non-finite moments)" +
                 (s.dropped ? "; " + std::to_string(s.dropped) + " particles dropped by tile overflow" : "");
    } else if (s.dropped) {
        c->sticky = LBMPCD_E_OVERFLOW;
        c->err = std::to_string(s.dropped) + " particles dropped by tile overflow (raise capacity_factor)";
    } else if (s.misplaced) {
        c->sticky = LBMPCD_E_STATE;
        c->err = std::to_string(s.misplaced) + " particles found outside their tile";
    }
    return c->sticky;
}

}  // namespace

extern "C" {

const char* lbmpcd_strerror(int code) {
    switch (code) {
        case LBMPCD_OK: return "ok";
        case LBMPCD_E_INVALID: return "invalid argument";
        case LBMPCD_E_NOMEM: return "workspace too small or host allocation failed";
        case LBMPCD_E_DEVICE: return "HIP error";
        case LBMPCD_E_OVERFLOW: return "particle tile overflow";
        case LBMPCD_E_STATE: return "inconsistent device state";
        case LBMPCD_E_UNSUPPORTED: return "unsupported parameter combination";
        default: return "unknown error";
    }
}

const char* lbmpcd_last_error(const lbmpcd_ctx* c) { return c ? c->err.c_str() : g_err.c_str(); }

int lbmpcd_viscosity(const lbmpcd_params* p, double* nu_lb, double* nu_mpcd) {
    std::string msg;
    if (!p) return fail(nullptr, LBMPCD_E_INVALID, "null parameters");
    if (int e = validate_one(*p, msg)) return fail(nullptr, e, msg);
    if (nu_lb) *nu_lb = (p->tau - 0.5) / 3.0;
    if (!nu_mpcd) return 0;
    if (!p->mpcd) return fail(nullptr, LBMPCD_E_INVALID, "no MPCD region");
    const double dt = 1.0 / p->substeps, a = 1.0 / p->refine, N = (double)p->ppc;
    const double q = N - 1.0 + std::exp(-N), kin = p->kT * dt / p->mass;
    if (p->collision == 1) {
        *nu_mpcd = kin * (N / q - 0.5) + a * a / (12.0 * dt) * q / N;  // Eq. 7
        return 0;
    }
    const double al = p->alpha_deg * 3.14159265358979323846 / 180.0;
    if (p->dim == 2) {
        *nu_mpcd = kin * (N / (q * (1.0 - std::cos(2.0 * al))) - 0.5) + a * a * (1.0 - std::cos(al)) * q / (12.0 * dt * N);
        return 0;
    }
    *nu_mpcd = kin * (5.0 * N / (q * (4.0 - 2.0 * std::cos(al) - 2.0 * std::cos(2.0 * al))) - 0.5) +
               a * a * (1.0 - std::cos(al)) * q / (18.0 * dt * N);
    return 0;
}

int lbmpcd_workspace_size(const lbmpcd_params* p, int32_t n_inst, size_t* bytes) {
    if (!bytes) return fail(nullptr, LBMPCD_E_INVALID, "bytes is null");
    std::string msg;
    int e = validate_all(p, n_inst, msg);
    if (e) return fail(nullptr, e, msg);
    std::vector<InstDesc> D;
    Layout L;
    long long tot[7];
    e = build(p, n_inst, D, L, tot, msg);
    if (e) return fail(nullptr, e, msg);
    *bytes = L.end;
    return 0;
}

int lbmpcd_init(const lbmpcd_params* p, int32_t n_inst, void* dev_workspace, size_t bytes, void* hip_stream,
                lbmpcd_ctx** out) {
    if (!out) return fail(nullptr, LBMPCD_E_INVALID, "out is null");
    *out = nullptr;
    std::string msg;
    int e = validate_all(p, n_inst, msg);
    if (e) return fail(nullptr, e, msg);
    lbmpcd_ctx* c = new (std::nothrow) lbmpcd_ctx();
    if (!c) return fail(nullptr, LBMPCD_E_NOMEM, "host allocation failed");
    Layout L;
    long long tot[7];
    e = build(p, n_inst, c->desc, L, tot, msg);
    if (e) { delete c; return fail(nullptr, e, msg); }
    if (!dev_workspace || bytes < L.end) {
        delete c;
        return fail(nullptr, LBMPCD_E_NOMEM, "workspace is null or smaller than lbmpcd_workspace_size");
    }
    c->n_inst = n_inst;
    c->params.assign(p, p + n_inst);
    c->dim = p[0].dim; c->lb_fp = p[0].lb_fp; c->part_fp = p[0].part_fp; c->S = p[0].substeps;
    c->Q = c->dim == 2 ? 9 : 19; c->mpcd = p[0].mpcd;
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return fail(nullptr, LBMPCD_E_DEVICE, "no HIP device"); }
    if (int se = resolve_noalloc_scratch(c->device, msg)) { delete c; return fail(nullptr, se, msg); }
    c->ws = (char*)dev_workspace;
    c->ws_bytes = bytes;
    c->total_nodes = tot[0]; c->total_band = tot[1]; c->total_ufine = tot[2]; c->total_tiles = tot[3];
    c->total_slots = tot[4]; c->total_particles = tot[5]; c->total_slab = tot[6];
    c->d_desc = (InstDesc*)(c->ws + L.desc);
    c->d_tile_inst = (int*)(c->ws + L.tile_inst);
    c->f[0] = c->ws + L.f0;
    c->f[1] = c->ws + L.f1;
    c->ub = (double*)(c->ws + L.ub);
    c->uf = (double*)(c->ws + L.uf);
    if (p[0].mpcd && p[0].reinject) {
        c->tb = (double*)(c->ws + L.tb);
        c->tf = (double*)(c->ws + L.tf);
        c->ce_bit = 8;
    }
    c->acc = (double*)(c->ws + L.acc);
    c->fbu = (double*)(c->ws + L.fbu);
    c->prof = (double*)(c->ws + L.prof);
    c->acc_bytes = L.acc_bytes;
    c->prof_bytes = L.prof_bytes;
    c->fill[0] = (uint32_t*)(c->ws + L.fill0);
    c->fill[1] = (uint32_t*)(c->ws + L.fill1);
    c->cstride = (long long)L.cstride;
    for (int b = 0; b < 2; ++b) {
        unsigned char* pb = (unsigned char*)(c->ws + L.part[b]);
        for (int k = 0; k < 3; ++k) {
            c->part[b].pos[k] = k < c->dim ? pb + (size_t)k * L.cstride : nullptr;
            c->part[b].vel[k] = k < c->dim ? pb + (size_t)(c->dim + k) * L.cstride : nullptr;
        }
        c->part[b].id = (uint32_t*)(pb + (size_t)2 * c->dim * L.cstride);
    }
    c->stats = (DevStats*)(c->ws + L.stats);
    c->ovf = (uint32_t*)(c->ws + L.ovf);
    c->clock = (long long*)(c->ws + L.clock);
    c->shifts = (double*)(c->ws + L.shifts);
    if (p[0].closure) {
        c->closure = true;
        c->cl_P = (float*)(c->ws + L.cl_P);
        c->cl_Pb = (uint16_t*)(c->ws + L.cl_Pb);
        c->cl_Pf = (uint16_t*)(c->ws + L.cl_Pf);
        c->cl_G = (float*)(c->ws + L.cl_G);
        c->cl_m = (float*)(c->ws + L.cl_m);
        c->cl_v = (float*)(c->ws + L.cl_v);
        c->cl_stats = (float*)(c->ws + L.cl_stats);
        c->cl_sums = (double*)(c->ws + L.cl_sums);
        c->cl_loss = (double*)(c->ws + L.cl_loss);
        c->cl_facc = (double*)(c->ws + L.cl_facc);
        c->cl_nm = (double*)(c->ws + L.cl_nm);
        c->cl_uc = (float*)(c->ws + L.cl_uc);
        c->cl_nslab = c->desc[0].nslab;
        closure_bufs_carve((unsigned char*)(c->ws + L.cl_inf), c->cl_nslab, false, c->cl_inf);
    }
    c->scratch = c->ws + L.scratch;
    c->scratch_bytes = L.scratch_bytes;
    int cap_max = 64;
    for (const InstDesc& d : c->desc) {
        cap_max = std::max(cap_max, d.cap);
        c->exp_max = std::max(c->exp_max, d.ppc * d.nct);
        if (d.feedback) c->any_feedback = true;
    }
    c->cap_max = cap_max;
    c->wg_threads = p[0].wg_threads ? p[0].wg_threads
                                    : default_wg_threads(c->part_fp, cap_max, c->exp_max, c->total_tiles);
    // an explicit 256 takes the six-slot form wherever it fits; the default
    // only on grids large enough to gain from it
    c->split_ok = c->wg_threads == 256 && six_slot_fits(cap_max, c->exp_max) &&
                  (p[0].wg_threads == 256 || c->total_tiles >= SPLIT_MIN_TILES);
    c->lds = particle_lds_bytes(c->dim, c->part_fp, cap_max);
    c->coll_bit = p[0].collision == 1 ? 4 : 0;
    c->det_bit = (p[0].mpcd && p[0].deterministic) ? 16 : 0;
    c->xcd_blocked = p[0].schedule == 0 ? 1 : 0;

    // tile -> instance table
    std::vector<int> tinst((size_t)std::max<long long>(c->total_tiles, 1));
    for (int i = 0; i < n_inst; ++i)
        for (long long T = 0; T < c->desc[i].ntiles; ++T) tinst[(size_t)(c->desc[i].tile_off + T)] = i;
    hipStream_t s = c->stream;
    auto chk = [&](hipError_t he, const char* what) -> int {
        if (he != hipSuccess) {
            g_err = std::string(what) + ": " + hipGetErrorString(he);
            return LBMPCD_E_DEVICE;
        }
        return 0;
    };
    const long long clock0 = -1;
    int rc = 0;
    rc = rc ? rc : chk(hipMemcpyAsync(c->d_desc, c->desc.data(), sizeof(InstDesc) * n_inst, hipMemcpyHostToDevice, s), "desc");
    rc = rc ? rc : chk(hipMemcpyAsync(c->d_tile_inst, tinst.data(), 4 * (size_t)c->total_tiles, hipMemcpyHostToDevice, s), "tile table");
    rc = rc ? rc : chk(hipMemcpyAsync(c->clock, &clock0, sizeof(clock0), hipMemcpyHostToDevice, s), "clock");
    rc = rc ? rc : chk(launch_zero(c->stats, sizeof(DevStats), s), "stats");
    rc = rc ? rc : chk(launch_zero(c->ovf, 4 * ((size_t)c->total_tiles + 2), s), "overflow list");
    rc = rc ? rc : chk(launch_zero(c->acc, c->acc_bytes, s), "acc");
    rc = rc ? rc : chk(launch_zero(c->prof, c->prof_bytes, s), "prof");
    rc = rc ? rc : chk(launch_zero(c->ub, 3 * 8 * (size_t)c->total_band, s), "ub");
    rc = rc ? rc : chk(launch_zero(c->uf, (size_t)c->dim * 8 * c->total_ufine, s), "uf");
    if (c->tf) {
        rc = rc ? rc : chk(launch_zero(c->tb, (size_t)CE_NT * 8 * c->total_band, s), "tb");
        rc = rc ? rc : chk(launch_zero(c->tf, (size_t)CE_NT * 8 * c->total_ufine, s), "tf");
    }
    rc = rc ? rc : chk(launch_zero(c->fbu, 3 * 8 * (size_t)c->total_slab, s), "fbu");
    rc = rc ? rc : chk(launch_lb_init(c->dim, c->lb_fp, c->d_desc, n_inst, c->total_nodes, c->f[0],
                                      c->mpcd ? c->fbu : nullptr, c->total_slab, s), "lb init");
    if (c->mpcd) {
        rc = rc ? rc : chk(launch_fill_sequential(c->d_desc, n_inst, c->total_tiles, c->fill[0], c->fill[1], s), "fill");
        rc = rc ? rc : chk(launch_part_init(c->dim, c->part_fp, c->d_desc, n_inst, c->total_particles, c->part[0], s), "particles");
    }
    rc = rc ? rc : chk(hipStreamSynchronize(s), "init sync");
    if (rc) { delete c; return rc; }
    *out = c;
    return 0;
}

namespace {

// Enqueue one coupled LB step on stream s (the context's stream, or the
// capture stream while a graph is recorded).
// The network's standardised output (cl_inf.Y) and the nodes' LB velocities
// (cl_uc) for the current populations, by the fused inference kernel.  The
// band moments it needs overlay the feature buffer of the separate products.
static hipError_t closure_predict_now(lbmpcd_ctx* c, hipStream_t s) {
    const InstDesc& d = c->desc[0];
    const long long nband = (long long)d.nx * d.nyb * d.nz;
    return closure_predict(c->lb_fp, c->d_desc, 0, c->cl_nslab, nband, d.by0, d.nyb, c->f[c->fcur],
                           (float*)c->cl_inf.X, c->cl_stats, c->cl_Pb, c->cl_Pf, c->cl_P, c->cl_inf.Y,
                           c->cl_uc, s);
}

int enqueue_one_step(lbmpcd_ctx* c, hipStream_t s) {
    {
        HIPCHK(c, timed(c, 0, [&] {
                   return launch_lb_step(c->dim, c->lb_fp, c->d_desc, c->n_inst, c->total_nodes, c->f[c->fcur],
                                         c->f[c->fcur ^ 1], c->clock, c->shifts, c->mpcd ? c->S : 0, s);
               }));
        c->fcur ^= 1;
        if (c->cl_on) {
            // surrogate: the network's velocity of every slab node stands in
            // for the MPCD samples -- in the profile, and with feedback in
            // the projection onto the LB equilibria
            HIPCHK(c, timed(c, 4, [&] {
                       hipError_t e = closure_predict_now(c, s);
                       if (e == hipSuccess)
                           e = closure_to_acc(c->d_desc, 0, c->cl_nslab, c->cl_inf.Y, c->cl_stats, c->cl_uc, c->acc,
                                              c->prof, c->sampling ? 1 : 0, s);
                       return e;
                   }));
            if (c->any_feedback)
                HIPCHK(c, timed(c, 1, [&] {
                           return launch_band(c->dim, c->lb_fp, c->d_desc, c->n_inst, c->total_band,
                                              c->f[c->fcur], c->acc, c->fbu, c->total_slab, c->ub, nullptr,
                                              c->stats, 1, s);
                       }));
            return 0;
        }
        if (c->cl_collect)
            HIPCHK(c, closure_features(c->lb_fp, c->d_desc, 0, c->cl_nslab, c->f[c->fcur], c->cl_facc, nullptr,
                                       nullptr, nullptr, s));
        if (c->mpcd) {
            HIPCHK(c, timed(c, 1, [&] {
                       return launch_band(c->dim, c->lb_fp, c->d_desc, c->n_inst, c->total_band, c->f[c->fcur],
                                          c->acc, c->fbu, c->total_slab, c->ub, c->tb, c->stats,
                                          c->any_feedback ? 1 : 0, s);
                   }));
            HIPCHK(c, timed(c, 2, [&] {
                       return launch_interp(c->dim, c->d_desc, c->n_inst, c->total_ufine, c->ub, c->uf, c->tb,
                                            c->tf, s);
                   }));
            for (int sub = 0; sub < c->S; ++sub) {
                ParticleLaunch L{};
                L.dim = c->dim; L.part_fp = c->part_fp;
                L.mode = ((sub == 0 && !c->pending) ? 2 : (3 | c->coll_bit)) | c->ce_bit | c->det_bit;
                L.D = c->d_desc; L.n_inst = c->n_inst; L.tiles = c->total_tiles;
                L.in = c->part[c->pcur]; L.out = c->part[c->pcur ^ 1];
                L.fill_in = c->fill[c->pcur]; L.fill_out = c->fill[c->pcur ^ 1];
                L.tile_inst = c->d_tile_inst; L.ufine = c->uf; L.tfine = c->tf; L.acc = c->acc; L.prof = c->prof;
                L.stats = c->stats; L.clock = c->clock; L.shifts = c->shifts;
                L.coll_dt = sub > 0 ? 0 : -1;
                L.coll_s = sub > 0 ? sub - 1 : c->S - 1;
                L.str_s = sub;
                // samples are taken in the last MPCD step of the LB step
                L.do_fb = (c->any_feedback && sub == c->S - 1) ? 1 : 0;
                L.do_prof = (c->sampling && sub == c->S - 1) ? 1 : 0;
                L.diag_inst = -1; L.cell_vcm = nullptr; L.lds_bytes = c->lds; L.cap_max = c->cap_max; L.ovf = c->split_ok ? c->ovf : nullptr; L.exp_max = c->exp_max; L.wg_threads = c->wg_threads; L.cstride = c->cstride; L.xcd_blocked = c->xcd_blocked;
                HIPCHK(c, timed(c, 3, [&] { return launch_particles(L, s); }));
                c->pcur ^= 1;
                c->pending = true;
            }
        }
    }
    return 0;
}

// Record two coupled steps (after which both ping-pong parities are back
// where they started) into an executable graph.  Kernels read the LB step
// index from the device clock, so the graph can be replayed indefinitely.
int build_graph(lbmpcd_ctx* c) {
    if (c->graph_exec) {
        (void)hipGraphExecDestroy(c->graph_exec);
        c->graph_exec = nullptr;
    }
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    const int f0 = c->fcur, p0 = c->pcur;
    const bool pend0 = c->pending, timing0 = c->timing;
    c->timing = false;
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    int e = enqueue_one_step(c, c->cap_stream);
    if (!e) e = enqueue_one_step(c, c->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t he = hipStreamEndCapture(c->cap_stream, &g);
    c->fcur = f0; c->pcur = p0; c->pending = pend0; c->timing = timing0;
    if (e) { if (g) (void)hipGraphDestroy(g); return e; }
    if (he != hipSuccess) return fail(c, LBMPCD_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(he));
    he = hipGraphInstantiateWithFlags(&c->graph_exec, g, 0);
    (void)hipGraphDestroy(g);
    if (he != hipSuccess) return fail(c, LBMPCD_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(he));
    c->graph_key = (c->cl_on ? 8 : 0) | (c->fcur << 2) | (c->pcur << 1) | (c->sampling ? 1 : 0);
    return 0;
}

}  // namespace

int lbmpcd_step(lbmpcd_ctx* c, int32_t n_lb_steps) {
    if (!c) return fail(nullptr, LBMPCD_E_INVALID, "null context");
    if (c->sticky) return c->sticky;
    if (n_lb_steps < 0) return fail(c, LBMPCD_E_INVALID, "negative step count");
    int it = 0;
    while (it < n_lb_steps) {
        if (c->cl_on && c->cl_every > 0 && c->cl_since >= c->cl_every) {
            // periodic check of the surrogate against a burst of plain MPCD steps
            double err = 0.0;
            if (int e = lbmpcd_closure_check(c, c->cl_burst, &err)) return e;
        }
        const bool steady = !c->mpcd || c->pending || c->cl_on;
        if (c->use_graphs && !c->timing && steady && n_lb_steps - it >= 2) {
            const int key = (c->cl_on ? 8 : 0) | (c->fcur << 2) | (c->pcur << 1) | (c->sampling ? 1 : 0);
            if (!c->graph_exec || c->graph_key != key)
                if (int e = build_graph(c)) return e;
            HIPCHK(c, hipGraphLaunch(c->graph_exec, c->stream));
            if (c->cl_on) c->cl_since += 2;
            c->t += 2;
            if (c->sampling) c->sampled_steps += 2;
            it += 2;
            continue;
        }
        if (int e = enqueue_one_step(c, c->stream)) return e;
        if (c->cl_on) c->cl_since += 1;
        c->t++;
        if (c->sampling) c->sampled_steps++;
        ++it;
    }
    return 0;
}

int lbmpcd_graphs(lbmpcd_ctx* c, int32_t enable) {
    if (!c) return fail(nullptr, LBMPCD_E_INVALID, "null context");
    c->use_graphs = enable != 0;
    return 0;
}

int lbmpcd_field_bytes(const lbmpcd_ctx* c, int32_t field, int32_t inst, size_t* bytes) {
    if (!c || !bytes || inst < 0 || inst >= c->n_inst) return LBMPCD_E_INVALID;
    const InstDesc& d = c->desc[inst];
    const size_t N = (size_t)d.N;
    switch (field) {
        case LBMPCD_RHO: *bytes = N * 8; break;
        case LBMPCD_U: *bytes = 3 * N * 8; break;
        case LBMPCD_PI: *bytes = 6 * N * 8; break;
        case LBMPCD_POP: *bytes = (size_t)c->Q * N * (c->lb_fp == 64 ? 8 : 4); break;
        case LBMPCD_PART_POS:
        case LBMPCD_PART_VEL:
        case LBMPCD_PART_VEL_PENDING: *bytes = (size_t)c->dim * d.Np * 8; break;
        case LBMPCD_CELL_ID: *bytes = (size_t)d.Np * 4; break;
        case LBMPCD_CELL_COUNT: *bytes = (size_t)d.ncells * 4; break;
        case LBMPCD_CELL_VCM: *bytes = (size_t)c->dim * d.ncells * 8; break;
        case LBMPCD_PROFILE: *bytes = (size_t)d.R * 4 * 8; break;
        case LBMPCD_UFINE: *bytes = (size_t)c->dim * d.Cx * d.R * d.Cz * 8; break;
        case LBMPCD_TFINE: *bytes = (size_t)CE_NT * d.Cx * d.R * d.Cz * 8; break;
        case LBMPCD_STATS: *bytes = 10 * 8; break;
        case LBMPCD_CELL_START: *bytes = (size_t)d.ncells * 4; break;
        case LBMPCD_NODE_MPCD_U:
        case LBMPCD_NODE_FB_U: *bytes = (size_t)c->dim * d.nslab * 8; break;
        default: return LBMPCD_E_INVALID;
    }
    return 0;
}

namespace {

// Produce a derived field into device memory `dst`.
int produce(lbmpcd_ctx* c, int32_t field, int32_t inst, void* dst, size_t nbytes) {
    const InstDesc& d = c->desc[inst];
    hipStream_t s = c->stream;
    const long long slots = d.ntiles * (long long)d.cap;
    const long long tl = c->t - 1;
    const int sl = c->S - 1;
    switch (field) {
        case LBMPCD_RHO:
            HIPCHK(c, launch_moments(c->dim, c->lb_fp, c->d_desc, inst, d.N, c->f[c->fcur], (double*)dst, nullptr, nullptr, s));
            return 0;
        case LBMPCD_U:
            HIPCHK(c, launch_moments(c->dim, c->lb_fp, c->d_desc, inst, d.N, c->f[c->fcur], nullptr, (double*)dst, nullptr, s));
            return 0;
        case LBMPCD_PI:
            HIPCHK(c, launch_moments(c->dim, c->lb_fp, c->d_desc, inst, d.N, c->f[c->fcur], nullptr, nullptr, (double*)dst, s));
            return 0;
        case LBMPCD_POP: {
            const size_t w = c->lb_fp == 64 ? 8 : 4;
            HIPCHK(c, hipMemcpyAsync(dst, (char*)c->f[c->fcur] + (size_t)d.node_off * c->Q * w, nbytes,
                                     hipMemcpyDeviceToDevice, s));
            return 0;
        }
        case LBMPCD_PART_POS:
        case LBMPCD_PART_VEL:
        case LBMPCD_PART_VEL_PENDING:
            // collisions move no particle; velocities complete the pending collision
            // unless the pre-collision values are asked for
            if (field == LBMPCD_PART_VEL)
                if (int e = finalize(c)) return e;
            HIPCHK(c, launch_gather(c->dim, c->part_fp, c->d_desc, inst, c->part[c->pcur], c->fill[c->pcur],
                                    field == LBMPCD_PART_POS ? (double*)dst : nullptr,
                                    field != LBMPCD_PART_POS ? (double*)dst : nullptr, nullptr, slots, tl, sl, s));
            return 0;
        case LBMPCD_CELL_ID:
            if (c->t == 0) return fail(c, LBMPCD_E_STATE, "no binning before the first step");
            HIPCHK(c, launch_gather(c->dim, c->part_fp, c->d_desc, inst, c->part[c->pcur], c->fill[c->pcur],
                                    nullptr, nullptr, (int*)dst, slots, tl, sl, s));
            return 0;
        case LBMPCD_CELL_COUNT:
            if (c->t == 0) return fail(c, LBMPCD_E_STATE, "no binning before the first step");
            HIPCHK(c, launch_zero(dst, nbytes, s));
            HIPCHK(c, launch_cell_count(c->dim, c->part_fp, c->d_desc, inst, c->part[c->pcur], c->fill[c->pcur],
                                        (int*)dst, slots, tl, sl, s));
            return 0;
        case LBMPCD_CELL_START:
            if (int e = produce(c, LBMPCD_CELL_COUNT, inst, dst, nbytes)) return e;
            HIPCHK(c, launch_exclusive_scan((int*)dst, d.ncells, s));
            return 0;
        case LBMPCD_NODE_MPCD_U:
            if (!d.feedback) return fail(c, LBMPCD_E_STATE, "node sample averages are kept only with feedback 1");
            HIPCHK(c, launch_node_mean(c->acc + d.acc_off * 4, d.nslab, c->dim, d.det, (double*)dst, s));
            return 0;
        case LBMPCD_NODE_FB_U:
            if (!d.feedback) return fail(c, LBMPCD_E_STATE, "the feedback's running mean exists only with feedback 1");
            for (int k = 0; k < c->dim; ++k)
                HIPCHK(c, hipMemcpyAsync((double*)dst + (size_t)k * d.nslab, c->fbu + (size_t)k * c->total_slab + d.acc_off,
                                         (size_t)d.nslab * 8, hipMemcpyDeviceToDevice, s));
            return 0;
        case LBMPCD_CELL_VCM: {
            if (!c->pending) return fail(c, LBMPCD_E_STATE, "cell velocities exist only right after lbmpcd_step");
            HIPCHK(c, launch_zero(dst, nbytes, s));
            ParticleLaunch L{};
            L.dim = c->dim; L.part_fp = c->part_fp; L.mode = 1 | c->coll_bit | c->det_bit;
            L.D = c->d_desc; L.n_inst = c->n_inst; L.tiles = c->total_tiles;
            // the pending collision is evaluated into the idle particle buffer, so
            // the state (and the other instances' pending collisions) is untouched
            L.in = c->part[c->pcur]; L.out = c->part[c->pcur ^ 1];
            L.fill_in = c->fill[c->pcur]; L.fill_out = c->fill[c->pcur ^ 1];
            L.tile_inst = c->d_tile_inst; L.ufine = c->uf; L.tfine = c->tf; L.acc = c->acc; L.prof = c->prof;
            L.stats = c->stats; L.clock = c->clock; L.shifts = c->shifts; L.shifts = c->shifts;
            L.coll_dt = 0; L.coll_s = c->S - 1; L.str_s = 0;
            L.diag_inst = inst; L.cell_vcm = (double*)dst; L.lds_bytes = c->lds; L.cap_max = c->cap_max; L.ovf = c->split_ok ? c->ovf : nullptr; L.exp_max = c->exp_max; L.wg_threads = c->wg_threads; L.cstride = c->cstride; L.xcd_blocked = c->xcd_blocked;
            HIPCHK(c, launch_particles(L, s));
            return 0;
        }
        case LBMPCD_PROFILE:
            HIPCHK(c, launch_profile_reduce(c->d_desc, inst, d.R, c->prof, (double*)dst, s));
            return 0;
        case LBMPCD_UFINE:
        case LBMPCD_TFINE: {
            // expand the buffer rows to the full slab layout [ncomp][Cz][R][Cx]
            const bool tens = field == LBMPCD_TFINE;
            if (tens && !c->tf) return fail(c, LBMPCD_E_STATE, "TFINE needs the Chapman-Enskog exchange");
            const int ncomp = tens ? CE_NT : c->dim;
            const double* base = tens ? c->tf + d.ufine_off * CE_NT : c->uf + d.ufine_off * c->dim;
            HIPCHK(c, launch_zero(dst, nbytes, s));
            const size_t row = (size_t)d.Cx * 8;
            for (int q = 0; q < ncomp; ++q)
                for (int K = 0; K < d.Cz; ++K)
                    for (int Jb = 0; Jb < d.NB; ++Jb) {
                        const int J = Jb < d.buf_lo * d.r ? Jb : Jb + (d.R - d.NB);
                        const double* src = base + (size_t)q * d.Cx * d.NB * d.Cz + ((size_t)K * d.NB + Jb) * d.Cx;
                        double* to = (double*)dst + (size_t)q * d.Cx * d.R * d.Cz + ((size_t)K * d.R + J) * d.Cx;
                        HIPCHK(c, hipMemcpyAsync(to, src, row, hipMemcpyDeviceToDevice, s));
                    }
            return 0;
        }
        default:
            return fail(c, LBMPCD_E_INVALID, "unknown field");
    }
}

}  // namespace

int lbmpcd_moments(lbmpcd_ctx* c, int32_t field, int32_t inst, void* dst, size_t dst_bytes, int32_t on_dev) {
    if (!c) return fail(nullptr, LBMPCD_E_INVALID, "null context");
    if (inst < 0 || inst >= c->n_inst) return fail(c, LBMPCD_E_INVALID, "bad instance");
    size_t need = 0;
    if (lbmpcd_field_bytes(c, field, inst, &need)) return fail(c, LBMPCD_E_INVALID, "bad field");
    if (!dst || dst_bytes < need) return fail(c, LBMPCD_E_INVALID, "destination too small");
    if (field == LBMPCD_STATS) {
        DevStats s;
        HIPCHK(c, hipMemcpyAsync(&s, c->stats, sizeof(s), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        int64_t v[10] = {c->t, c->sampled_steps, (int64_t)s.dropped, (int64_t)s.misplaced, (int64_t)s.far_moves,
                         (int64_t)s.max_fill, c->desc[inst].Np, c->desc[inst].ncells, (int64_t)s.window_misses,
                         (int64_t)s.bad_state};
        if (on_dev) HIPCHK(c, hipMemcpy(dst, v, sizeof(v), hipMemcpyHostToDevice));
        else std::memcpy(dst, v, sizeof(v));
        return 0;
    }
    if (!c->mpcd && field >= LBMPCD_PART_POS && field != LBMPCD_STATS)
        return fail(c, LBMPCD_E_INVALID, "no particles in this context");
    if (on_dev) return produce(c, field, inst, dst, need);
    if (need > c->scratch_bytes) return fail(c, LBMPCD_E_INVALID, "field too large for a host transfer; pass device memory");
    if (int e = produce(c, field, inst, c->scratch, need)) return e;
    HIPCHK(c, hipMemcpyAsync(dst, c->scratch, need, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return check_device_errors(c);
}

int lbmpcd_get_state(lbmpcd_ctx* c, int32_t field, int32_t inst, void* dst, size_t bytes, int32_t on_dev) {
    if (field != LBMPCD_POP && field != LBMPCD_PART_POS && field != LBMPCD_PART_VEL &&
        field != LBMPCD_PART_VEL_PENDING)
        return fail(c, LBMPCD_E_INVALID, "get_state handles POP, PART_POS, PART_VEL, PART_VEL_PENDING");
    return lbmpcd_moments(c, field, inst, dst, bytes, on_dev);
}

int lbmpcd_set_state(lbmpcd_ctx* c, int32_t field, int32_t inst, const void* src, size_t bytes, int32_t on_dev) {
    if (!c) return fail(nullptr, LBMPCD_E_INVALID, "null context");
    if (inst < 0 || inst >= c->n_inst) return fail(c, LBMPCD_E_INVALID, "bad instance");
    if (field != LBMPCD_POP && field != LBMPCD_PART_POS && field != LBMPCD_PART_VEL)
        return fail(c, LBMPCD_E_INVALID, "set_state handles POP, PART_POS, PART_VEL");
    size_t need = 0;
    lbmpcd_field_bytes(c, field, inst, &need);
    if (!src || bytes < need) return fail(c, LBMPCD_E_INVALID, "source too small");
    const InstDesc& d = c->desc[inst];
    hipStream_t s = c->stream;
    if (field == LBMPCD_POP) {
        const size_t w = c->lb_fp == 64 ? 8 : 4;
        HIPCHK(c, hipMemcpyAsync((char*)c->f[c->fcur] + (size_t)d.node_off * c->Q * w, src, need,
                                 on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        HIPCHK(c, hipStreamSynchronize(s));
        return 0;
    }
    if (!c->mpcd) return fail(c, LBMPCD_E_INVALID, "no particles in this context");
    if (int e = finalize(c)) return e;
    const void* dsrc = src;
    if (!on_dev) {
        if (need > c->scratch_bytes) return fail(c, LBMPCD_E_INVALID, "field too large for a host transfer");
        HIPCHK(c, hipMemcpyAsync(c->scratch, src, need, hipMemcpyHostToDevice, s));
        dsrc = c->scratch;
    }
    HIPCHK(c, launch_set_field(c->dim, c->part_fp, c->d_desc, inst, c->part[c->pcur], c->fill[c->pcur],
                               field == LBMPCD_PART_POS ? 0 : 1, (const double*)dsrc,
                               d.ntiles * (long long)d.cap, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return 0;
}

int lbmpcd_sample(lbmpcd_ctx* c, int32_t mode) {
    if (!c) return fail(nullptr, LBMPCD_E_INVALID, "null context");
    if (mode == 1) {
        HIPCHK(c, launch_zero(c->prof, c->prof_bytes, c->stream));
        c->sampling = true;
        c->sampled_steps = 0;
    } else if (mode == 0) {
        c->sampling = false;
    } else {
        return fail(c, LBMPCD_E_INVALID, "mode must be 0 or 1");
    }
    return 0;
}

int lbmpcd_sync(lbmpcd_ctx* c) {
    if (!c) return fail(nullptr, LBMPCD_E_INVALID, "null context");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->mpcd) return check_device_errors(c);
    return c->sticky;
}

int lbmpcd_timing(lbmpcd_ctx* c, int32_t mode) {
    if (!c) return fail(nullptr, LBMPCD_E_INVALID, "null context");
    if (mode == 1) {
        if (int e = drain_marks(c)) return e;
        for (int k = 0; k < 5; ++k) { c->timing_ms[k] = 0; c->timing_n[k] = 0; }
        c->timing = true;
    } else if (mode == 0) {
        c->timing = false;
    } else {
        return fail(c, LBMPCD_E_INVALID, "mode must be 0 or 1");
    }
    return 0;
}

int lbmpcd_timing_read(lbmpcd_ctx* c, double* out, int32_t n_classes) {
    if (!c || !out || n_classes < 0) return fail(c, LBMPCD_E_INVALID, "bad arguments");
    if (int e = drain_marks(c)) return e;
    for (int k = 0; k < n_classes; ++k) {
        out[2 * k] = k < 5 ? c->timing_ms[k] : 0.0;
        out[2 * k + 1] = k < 5 ? (double)c->timing_n[k] : 0.0;
    }
    return 0;
}

int lbmpcd_autotune(const lbmpcd_params* p, int32_t n_inst, void* dev_workspace, size_t bytes,
                    void* hip_stream, int32_t lb_steps, lbmpcd_tuning* out) {
    if (!out || out->struct_size != sizeof(lbmpcd_tuning))
        return fail(nullptr, LBMPCD_E_INVALID, "out is null or its struct_size is wrong");
    if (lb_steps < 1) return fail(nullptr, LBMPCD_E_INVALID, "lb_steps must be >= 1");
    std::string msg;
    if (int e = validate_all(p, n_inst, msg)) return fail(nullptr, e, msg);
    for (int i = 0; i < n_inst; ++i)
        if (p[i].tile[0] || p[i].tile[1] || p[i].tile[2])
            return fail(nullptr, LBMPCD_E_INVALID, "autotune needs tile = 0 (the tile follows tile_target)");
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess) {
        if (ev[0]) (void)hipEventDestroy(ev[0]);
        return fail(nullptr, LBMPCD_E_DEVICE, "event creation failed");
    }
    static const int targets[] = {160, 320, 640, 1280};
    static const int wgs[] = {256, 512};
    std::vector<lbmpcd_params> q(p, p + n_inst);
    double best = -1.0;
    int rc = 0;
    out->tried = 0;
    out->ms_default = -1.0;
    for (int tt : targets) {
        for (int cand = 0; cand < 4; ++cand) {
            const int wg = wgs[cand & 1], sched = cand >> 1;
            for (auto& x : q) { x.tile_target = tt; x.wg_threads = wg; x.schedule = sched; }
            size_t need = 0;
            if (lbmpcd_workspace_size(q.data(), n_inst, &need) != LBMPCD_OK || need > bytes) continue;
            lbmpcd_ctx* c = nullptr;
            if (lbmpcd_init(q.data(), n_inst, dev_workspace, bytes, hip_stream, &c) != LBMPCD_OK) {
                if (c) lbmpcd_destroy(c);
                continue;  // e.g. a tile whose capacity exceeds the kernel's limit
            }
            float ms = 0.f;
            int e = lbmpcd_step(c, lb_steps);
            if (!e && hipEventRecord(ev[0], s) != hipSuccess) e = LBMPCD_E_DEVICE;
            if (!e) e = lbmpcd_step(c, lb_steps);
            if (!e && hipEventRecord(ev[1], s) != hipSuccess) e = LBMPCD_E_DEVICE;
            if (!e) e = lbmpcd_sync(c);
            if (!e && hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess) e = LBMPCD_E_DEVICE;
            if (e) {
                g_err = "autotune candidate (" + std::to_string(tt) + ", " + std::to_string(wg) + ", " +
                        std::to_string(sched) + "): " + c->err;
                lbmpcd_destroy(c);
                rc = e;
                break;
            }
            // the shape the library takes with tile_target = wg_threads = 0
            const int default_wg = default_wg_threads(c->part_fp, c->cap_max, c->exp_max, c->total_tiles);
            lbmpcd_destroy(c);
            const double per = (double)ms / lb_steps;
            ++out->tried;
            if (tt == 1280 && wg == default_wg && sched == 0) out->ms_default = per;
            if (best < 0 || per < best) {
                best = per;
                out->tile_target = tt;
                out->wg_threads = wg;
                out->schedule = sched;
                out->ms_per_step = per;
            }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (rc) return rc;
    if (best < 0) return fail(nullptr, LBMPCD_E_NOMEM, "no candidate fits the workspace");
    return 0;
}

// ---------------------------------------------------------------------------
// learned closure
// ---------------------------------------------------------------------------
namespace {

int need_closure(lbmpcd_ctx* c) {
    if (!c) return fail(nullptr, LBMPCD_E_INVALID, "null context");
    if (c->sticky) return c->sticky;
    if (!c->closure) return fail(c, LBMPCD_E_STATE, "the context was created without closure = 1");
    return 0;
}

size_t train_scratch_bytes(long long rows) {
    return closure_bufs_bytes(rows, true) + align_up((size_t)rows * NOUT * 4, 256);
}

// One standardised batch of `rows` rows (drawn, or the first rows of X, Y).
int closure_batch(lbmpcd_ctx* c, const float* X, const float* Y, long long n, long long rows, bool draw,
                  uint32_t step, void* scratch, ClosureBufs& b, float*& Yb) {
    closure_bufs_carve((unsigned char*)scratch, rows, true, b);
    Yb = (float*)((unsigned char*)scratch + closure_bufs_bytes(rows, true));
    const InstDesc& d = c->desc[0];
    HIPCHK(c, mlp_gather(X, Y, n, c->cl_stats, rows, draw, d.key0, d.key1, step, b.X, Yb, c->stream));
    return 0;
}

}  // namespace

int lbmpcd_closure_scratch_size(int64_t n, int32_t batch, size_t* bytes) {
    if (!bytes || n < 1) return fail(nullptr, LBMPCD_E_INVALID, "bad arguments");
    const long long rows = batch > 0 && batch < n ? batch : n;
    *bytes = train_scratch_bytes(rows);
    return 0;
}

int lbmpcd_closure_collect(lbmpcd_ctx* c, int32_t lb_steps, float* X, float* Y) {
    if (int e = need_closure(c)) return e;
    if (lb_steps < 1 || !X || !Y) return fail(c, LBMPCD_E_INVALID, "need lb_steps >= 1 and device X, Y");
    if (c->cl_on) return fail(c, LBMPCD_E_STATE, "collection runs the plain coupled step; disable the closure");
    const InstDesc& d = c->desc[0];
    HIPCHK(c, hipMemsetAsync(c->cl_facc, 0, sizeof(double) * c->cl_nslab * NF, c->stream));
    HIPCHK(c, hipMemsetAsync(c->cl_nm, 0, sizeof(double) * c->cl_nslab * 10, c->stream));
    for (int k = 0; k < lb_steps; ++k) {
        c->cl_collect = true;
        int e = enqueue_one_step(c, c->stream);
        c->cl_collect = false;
        if (e) return e;
        c->t++;
        if (c->sampling) c->sampled_steps++;
        // the samples are taken from the collided state
        if (int e2 = finalize(c)) return e2;
        HIPCHK(c, closure_node_moments(c->part_fp, c->d_desc, 0, d.ntiles, c->part[c->pcur].pos[0],
                                       c->cstride, c->fill[c->pcur], c->cl_nm, c->stream));
    }
    HIPCHK(c, closure_collect_finish(c->cl_nslab, lb_steps, d.mass, c->cl_facc, c->cl_nm, X, Y, c->stream));
    return 0;
}

int lbmpcd_closure_features(lbmpcd_ctx* c, float* X) {
    if (int e = need_closure(c)) return e;
    if (!X) return fail(c, LBMPCD_E_INVALID, "X is null");
    HIPCHK(c, hipMemsetAsync(c->cl_facc, 0, sizeof(double) * c->cl_nslab * NF, c->stream));
    HIPCHK(c, closure_features(c->lb_fp, c->d_desc, 0, c->cl_nslab, c->f[c->fcur], c->cl_facc, nullptr, nullptr,
                               nullptr, c->stream));
    // one window of one step: the feature sums are the features
    HIPCHK(c, closure_collect_finish(c->cl_nslab, 1, 1.0, c->cl_facc, nullptr, X, nullptr, c->stream));
    return 0;
}

int lbmpcd_closure_train(lbmpcd_ctx* c, const float* X, const float* Y, int64_t n, const lbmpcd_train_opts* o,
                         void* scratch, size_t scratch_bytes, float* loss_per_epoch) {
    if (int e = need_closure(c)) return e;
    if (!o || o->struct_size != sizeof(lbmpcd_train_opts)) return fail(c, LBMPCD_E_INVALID, "bad train options");
    if (!X || !Y || n < 1 || o->epochs < 1 || !(o->lr > 0.0f)) return fail(c, LBMPCD_E_INVALID, "bad arguments");
    const long long rows = o->batch > 0 && o->batch < n ? o->batch : n;
    if (!scratch || scratch_bytes < train_scratch_bytes(rows))
        return fail(c, LBMPCD_E_NOMEM, "scratch smaller than lbmpcd_closure_scratch_size");
    hipStream_t s = c->stream;
    if (!c->cl_ready) {
        HIPCHK(c, mlp_stats(X, Y, n, c->cl_sums, c->cl_stats, s));
        const uint32_t k0 = (uint32_t)(o->seed & 0xFFFFFFFFu), k1 = (uint32_t)(o->seed >> 32);
        HIPCHK(c, mlp_init(c->cl_P, c->cl_Pb, c->cl_m, c->cl_v, k0, k1, s));
        c->cl_adam_t = 0;
        c->cl_ready = true;
    }
    const long long steps = (n + rows - 1) / rows;
    for (int ep = 0; ep < o->epochs; ++ep) {
        HIPCHK(c, hipMemsetAsync(c->cl_loss, 0, sizeof(double), s));
        for (long long st = 0; st < steps; ++st) {
            ClosureBufs b;
            float* Yb = nullptr;
            if (int e = closure_batch(c, X, Y, n, rows, rows < n, (uint32_t)(c->cl_adam_t + 1), scratch, b, Yb))
                return e;
            HIPCHK(c, mlp_forward(c->cl_P, c->cl_Pb, b, s));
            HIPCHK(c, mlp_backward(c->cl_Pb, Yb, b, c->cl_G, c->cl_loss, s));
            ++c->cl_adam_t;
            HIPCHK(c, mlp_adam(c->cl_P, c->cl_Pb, c->cl_G, c->cl_m, c->cl_v, c->cl_adam_t, o->lr, o->beta1,
                               o->beta2, o->eps, s));
        }
        if (loss_per_epoch) {
            double l = 0.0;
            HIPCHK(c, hipMemcpyAsync(&l, c->cl_loss, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(c, hipStreamSynchronize(s));
            loss_per_epoch[ep] = (float)(l / (double)steps);
        }
    }
    return 0;
}

int lbmpcd_closure_loss_grad(lbmpcd_ctx* c, const float* X, const float* Y, int64_t n, void* scratch,
                             size_t scratch_bytes, double* loss, float* grad) {
    if (int e = need_closure(c)) return e;
    if (!c->cl_ready) return fail(c, LBMPCD_E_STATE, "closure parameters are not set");
    if (!X || !Y || n < 1) return fail(c, LBMPCD_E_INVALID, "bad arguments");
    if (!scratch || scratch_bytes < train_scratch_bytes(n))
        return fail(c, LBMPCD_E_NOMEM, "scratch smaller than lbmpcd_closure_scratch_size(n, n)");
    hipStream_t s = c->stream;
    ClosureBufs b;
    float* Yb = nullptr;
    if (int e = closure_batch(c, X, Y, n, n, false, 0u, scratch, b, Yb)) return e;
    HIPCHK(c, hipMemsetAsync(c->cl_loss, 0, sizeof(double), s));
    HIPCHK(c, mlp_forward(c->cl_P, c->cl_Pb, b, s));
    HIPCHK(c, mlp_backward(c->cl_Pb, Yb, b, c->cl_G, c->cl_loss, s));
    if (loss) HIPCHK(c, hipMemcpyAsync(loss, c->cl_loss, sizeof(double), hipMemcpyDeviceToHost, s));
    if (grad) HIPCHK(c, hipMemcpyAsync(grad, c->cl_G, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return 0;
}

int lbmpcd_closure_forward(lbmpcd_ctx* c, const float* X, int64_t n, float* Y, void* scratch, size_t scratch_bytes) {
    if (int e = need_closure(c)) return e;
    if (!c->cl_ready) return fail(c, LBMPCD_E_STATE, "closure parameters are not set");
    if (!X || !Y || n < 1) return fail(c, LBMPCD_E_INVALID, "bad arguments");
    if (!scratch || scratch_bytes < train_scratch_bytes(n))
        return fail(c, LBMPCD_E_NOMEM, "scratch smaller than lbmpcd_closure_scratch_size(n, n)");
    ClosureBufs b;
    float* Yb = nullptr;
    if (int e = closure_batch(c, X, nullptr, n, n, false, 0u, scratch, b, Yb)) return e;
    HIPCHK(c, mlp_forward(c->cl_P, c->cl_Pb, b, c->stream));
    HIPCHK(c, mlp_destandardize(b.Y, c->cl_stats, X, n, Y, c->stream));
    return 0;
}

int lbmpcd_closure_forward_noalloc(lbmpcd_ctx* c, const float* X, int64_t n, float* Y) {
    if (int e = need_closure(c)) return e;
    if (!c->cl_ready) return fail(c, LBMPCD_E_STATE, "closure parameters are not set");
    if (!X || !Y || n < 1) return fail(c, LBMPCD_E_INVALID, "bad arguments");
    if (n > LBMPCD_NOALLOC_MAX_ROWS)
        return fail(c, LBMPCD_E_INVALID, "n exceeds LBMPCD_NOALLOC_MAX_ROWS (" +
                                             std::to_string(LBMPCD_NOALLOC_MAX_ROWS) + ") rows; split the call");
    void* ptr = noalloc_scratch(c->device);
    if (!ptr) return fail(c, LBMPCD_E_STATE, "the device's scratch array was not resolved at lbmpcd_init");
    ClosureBufs b;
    closure_bufs_carve((unsigned char*)ptr, n, false, b);
    const InstDesc& d = c->desc[0];
    HIPCHK(c, mlp_gather(X, nullptr, n, c->cl_stats, n, false, d.key0, d.key1, 0u, b.X, nullptr, c->stream));
    HIPCHK(c, mlp_forward(c->cl_P, c->cl_Pb, b, c->stream));
    HIPCHK(c, mlp_destandardize(b.Y, c->cl_stats, X, n, Y, c->stream));
    return 0;
}

int lbmpcd_closure_predict(lbmpcd_ctx* c, float* Y) {
    if (int e = need_closure(c)) return e;
    if (!c->cl_ready) return fail(c, LBMPCD_E_STATE, "closure parameters are not set");
    if (!Y) return fail(c, LBMPCD_E_INVALID, "Y is null");
    HIPCHK(c, closure_predict_now(c, c->stream));
    HIPCHK(c, mlp_destandardize_uc(c->cl_inf.Y, c->cl_stats, c->cl_uc, c->cl_nslab, Y, c->stream));
    return 0;
}

int lbmpcd_closure_weights(lbmpcd_ctx* c, int32_t get_or_set, float* buf, size_t bytes) {
    if (int e = need_closure(c)) return e;
    const size_t need = sizeof(float) * (size_t)(NPARAM + NSTATS);
    if (!buf || bytes < need) return fail(c, LBMPCD_E_INVALID, "buffer smaller than the parameter block");
    hipStream_t s = c->stream;
    if (get_or_set == 0) {
        if (!c->cl_ready) return fail(c, LBMPCD_E_STATE, "closure parameters are not set");
        HIPCHK(c, hipMemcpyAsync(buf, c->cl_P, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(buf + NPARAM, c->cl_stats, sizeof(float) * NSTATS, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
    } else if (get_or_set == 1) {
        HIPCHK(c, hipMemcpyAsync(c->cl_P, buf, sizeof(float) * NPARAM, hipMemcpyHostToDevice, s));
        HIPCHK(c, hipMemcpyAsync(c->cl_stats, buf + NPARAM, sizeof(float) * NSTATS, hipMemcpyHostToDevice, s));
        HIPCHK(c, mlp_refresh_bf16(c->cl_P, c->cl_Pb, s));
        HIPCHK(c, hipMemsetAsync(c->cl_m, 0, sizeof(float) * NPARAM, s));
        HIPCHK(c, hipMemsetAsync(c->cl_v, 0, sizeof(float) * NPARAM, s));
        HIPCHK(c, hipStreamSynchronize(s));
        c->cl_adam_t = 0;
        c->cl_ready = true;
    } else {
        return fail(c, LBMPCD_E_INVALID, "get_or_set must be 0 or 1");
    }
    return 0;
}

int lbmpcd_closure_enable(lbmpcd_ctx* c, int32_t on, double fallback_tol, int32_t check_every, int32_t check_steps) {
    if (int e = need_closure(c)) return e;
    if (on && !c->cl_ready) return fail(c, LBMPCD_E_STATE, "closure parameters are not set");
    if (fallback_tol < 0.0 || check_every < 0 || check_steps < 0)
        return fail(c, LBMPCD_E_INVALID, "negative tolerance or check interval");
    // the particles rest while the surrogate runs: complete their pending
    // collision now, in the grid shift it was binned with
    if (on && !c->cl_on)
        if (int e = finalize(c)) return e;
    c->cl_on = on != 0;
    c->cl_tol = fallback_tol > 0.0 ? fallback_tol : 0.02;
    c->cl_every = check_every;
    c->cl_burst = check_steps > 0 ? check_steps : 40;
    c->cl_since = 0;
    c->cl_fell_back = false;
    return 0;
}

int lbmpcd_closure_check(lbmpcd_ctx* c, int32_t burst_steps, double* rel_err) {
    if (int e = need_closure(c)) return e;
    if (!c->cl_ready) return fail(c, LBMPCD_E_STATE, "closure parameters are not set");
    if (burst_steps < 2 || !rel_err) return fail(c, LBMPCD_E_INVALID, "need burst_steps >= 2 and rel_err");
    const InstDesc& d = c->desc[0];
    const bool was_on = c->cl_on, was_sampling = c->sampling;
    c->cl_on = false;
    // plain MPCD burst; its second half is averaged
    if (int e = lbmpcd_step(c, burst_steps - burst_steps / 2)) return e;
    if (int e = lbmpcd_sample(c, 1)) return e;
    if (int e = lbmpcd_step(c, burst_steps / 2)) return e;
    std::vector<double> pm((size_t)d.R * 4), pp((size_t)d.R * 4);
    if (int e = lbmpcd_moments(c, LBMPCD_PROFILE, 0, pm.data(), pm.size() * 8, 0)) return e;
    // the surrogate's profile of the current state
    HIPCHK(c, launch_zero(c->prof, c->prof_bytes, c->stream));
    HIPCHK(c, closure_predict_now(c, c->stream));
    // written into the sample sums and profile; the sums are cleared again below
    HIPCHK(c, closure_to_acc(c->d_desc, 0, c->cl_nslab, c->cl_inf.Y, c->cl_stats, c->cl_uc, c->acc, c->prof, 1,
                             c->stream));
    if (int e = lbmpcd_moments(c, LBMPCD_PROFILE, 0, pp.data(), pp.size() * 8, 0)) return e;
    HIPCHK(c, launch_zero(c->acc, c->acc_bytes, c->stream));
    HIPCHK(c, launch_zero(c->prof, c->prof_bytes, c->stream));
    c->sampling = was_sampling;
    c->sampled_steps = 0;
    // relative L2 error of the streamwise profile over the LB node rows
    // between the buffers (the network predicts node averages)
    double num = 0.0, den = 0.0;
    for (int y = d.buf_lo; y < (d.yhi - d.ylo) - d.buf_hi; ++y) {
        double cm = 0, sm = 0, cp = 0, sp = 0;
        for (int J = y * d.r; J < (y + 1) * d.r; ++J) {
            cm += pm[4 * J]; sm += pm[4 * J + 1];
            cp += pp[4 * J]; sp += pp[4 * J + 1];
        }
        if (cm <= 0.0 || cp <= 0.0) continue;
        const double um = sm / cm, up = sp / cp;
        num += (up - um) * (up - um);
        den += um * um;
    }
    const double err = den > 0.0 ? std::sqrt(num / den) : 0.0;
    *rel_err = err;
    c->cl_last_err = err;
    c->cl_since = 0;
    if (err > c->cl_tol) {
        c->cl_fell_back = true;
        c->cl_on = false;
    } else {
        c->cl_on = was_on;
    }
    return 0;
}

int lbmpcd_closure_status(const lbmpcd_ctx* c, int32_t* on, int32_t* fell_back, double* last_err) {
    if (!c) return fail(nullptr, LBMPCD_E_INVALID, "null context");
    if (on) *on = c->cl_on ? 1 : 0;
    if (fell_back) *fell_back = c->cl_fell_back ? 1 : 0;
    if (last_err) *last_err = c->cl_last_err;
    return 0;
}

int lbmpcd_closure_gemm_bf16(int64_t M, int64_t N, int64_t K, const uint16_t* A, const uint16_t* B, float* C,
                             void* hip_stream) {
    if (M < 0 || N < 0 || K < 1 || !A || !B || !C) return fail(nullptr, LBMPCD_E_INVALID, "bad arguments");
    GemmArgs g{};
    g.M = M; g.N = N; g.K = K;
    g.A = A; g.sam = K; g.sak = 1;
    g.B = B; g.sbk = 1; g.sbn = K;
    g.C = C; g.ldc = N;
    g.epi = EPI_NONE;
    const hipError_t e = launch_gemm(g, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(nullptr, LBMPCD_E_DEVICE, hipGetErrorString(e));
    return 0;
}

void lbmpcd_destroy(lbmpcd_ctx* c) {
    if (!c) return;
    for (auto& m : c->marks) {
        if (m.a) (void)hipEventDestroy(m.a);
        if (m.b) (void)hipEventDestroy(m.b);
    }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
}

}  // extern "C"
