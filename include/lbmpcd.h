/*
 * lbmpcd.h -- C ABI of the MI355X coupled lattice-Boltzmann / multiparticle
 * collision (LB-MPCD) time step (Montessori, Tiribocchi, Lauricella, Succi,
 * arXiv 2004.00304).
 *
 * The library advances one or more independent channels: a coarse LB solver
 * over the whole channel (Sec. 2.1, Eq. 1-2; BGK with a body force, periodic
 * along x and z, half-way bounce-back walls at y = 0 and y = ny) coupled to a
 * fine MPCD solver in a slab y in [ylo, yhi) (Sec. 2.2, Eq. 3-4: ballistic
 * streaming, random grid shift, cell binning, stochastic rotation; or the
 * collision with Andersen thermostat of Eq. 6).  The two
 * are joined by the coupling procedure of Alg. 1 and Alg. 2: after each LB
 * step the LB velocity is interpolated to the fine cells of the buffer and
 * the buffer particles are redrawn from the Maxwell-Boltzmann distribution
 * about it (Box-Muller), or (reinject = 1) from the first-order
 * Chapman-Enskog distribution that the end of Sec. 2.3 names for strong
 * gradients; optionally (feedback 1, not in the paper, which couples one
 * way) a running time average of the MPCD velocity is projected back onto LB
 * equilibria in the slab interior.
 *
 * Conventions (lattice units, dx = dt_LB = 1):
 *   - node (i,j,k) sits at (i+1/2, j+1/2, k+1/2); walls at y = 0 and y = ny;
 *   - populations are stored SoA, f[q][z][y][x] with x fastest; D2Q9 order
 *     (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1); D3Q19
 *     order rest, +-x, +-y, +-z, (+-1,+-1,0), (+-1,0,+-1), (0,+-1,+-1) in the
 *     pairs (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) and likewise;
 *   - the stored LB state is the post-stream population (after the optional
 *     feedback projection); reported velocity = first moment / rho + g/2;
 *   - the MPCD collision cell side is a = 1/refine, the MPCD step is
 *     dt = 1/substeps; particle ids are 0..Np-1 in initial cell order.
 *
 * Ownership: the caller owns all device memory (one workspace buffer of
 * lbmpcd_workspace_size bytes, on the device that is current at init) and
 * the HIP stream.  The library never allocates device memory; it owns only
 * the host-side context.  All calls enqueue work on the stream given at init
 * and return without synchronising, except where a host buffer is read or
 * written (then the call synchronises the stream).
 *
 * Errors: every int-returning call returns 0 (LBMPCD_OK) or a positive code
 * below; no exception or abort crosses the ABI.  lbmpcd_last_error gives a
 * message.  Device-side overflow or state corruption is latched and reported
 * by the next synchronising call (lbmpcd_sync, moments, get_state):
 * E_OVERFLOW when a tile overflowed (E_STATE takes precedence: invalid
 * particles are parked in one tile, which may overflow); E_STATE when a particle moved more than
 * one period in one MPCD step or its position or velocity became non-finite
 * (it is parked at the slab's lower corner at rest, so every index the
 * kernels derive stays in range), when a node of the rows next to the slab
 * had rho <= 0 or non-finite moments, or when particles were found outside
 * their tile.  After a latched error lbmpcd_step returns it and does nothing.
 * A context is not thread-safe; use one context per stream.
 */
#ifndef LBMPCD_H
#define LBMPCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBMPCD_ABI_VERSION 6u

enum lbmpcd_status {
    LBMPCD_OK = 0,
    LBMPCD_E_INVALID = 1,     /* bad argument or parameter set */
    LBMPCD_E_NOMEM = 2,       /* workspace too small, host allocation failed */
    LBMPCD_E_DEVICE = 3,      /* a HIP call failed */
    LBMPCD_E_OVERFLOW = 4,    /* a particle tile overflowed its capacity */
    LBMPCD_E_STATE = 5,       /* device state is inconsistent */
    LBMPCD_E_UNSUPPORTED = 6  /* valid but not implemented combination */
};

/* Fields of lbmpcd_moments / lbmpcd_get_state / lbmpcd_set_state. */
enum lbmpcd_field {
    LBMPCD_RHO = 0,        /* double[nz][ny][nx]                                   */
    LBMPCD_U = 1,          /* double[3][nz][ny][nx], physical velocity (incl. g/2) */
    LBMPCD_PI = 2,         /* double[6][nz][ny][nx]: xx yy zz xy xz yz, sum f (cc - I/3) */
    LBMPCD_POP = 3,        /* lb_fp[Q][nz][ny][nx] post-stream populations (get/set) */
    LBMPCD_PART_POS = 4,   /* double[dim][Np] by particle id (get/set)             */
    LBMPCD_PART_VEL = 5,   /* double[dim][Np] by particle id (get/set)             */
    LBMPCD_CELL_ID = 6,    /* int32[Np]: cell of each particle in the last binning */
    LBMPCD_CELL_COUNT = 7, /* int32[ncells]: occupancy of the last binning         */
    LBMPCD_CELL_VCM = 8,   /* double[dim][ncells]: centre-of-mass velocity of the
                              pending collision (only right after lbmpcd_step; the
                              state is not changed)                               */
    LBMPCD_PROFILE = 9,    /* double[R][4]: per fine row sum n, sum v_x, v_y, v_z  */
    LBMPCD_UFINE = 10,     /* double[dim][nz*r][R][nx*r]: buffer-cell LB velocity  */
    LBMPCD_STATS = 11,     /* int64[10]: lb steps, sampled steps, dropped particles,
                              misplaced particles, far moves (particles that moved
                              beyond the neighbour tiles, counted in the MPCD steps
                              that take samples), max tile fill,
                              particles, cells, samples that missed their tile's LDS
                              window and went to global atomics (a slow path: 0
                              for the default tiles at refinement >= 2), invalid
                              particles and band nodes (see Errors above)          */
    LBMPCD_PART_VEL_PENDING = 12, /* double[dim][Np] by id: velocities before the
                              collision of the last MPCD step (get only)          */
    LBMPCD_CELL_START = 13, /* int32[ncells]: where each cell of the last binning
                              starts in the cell order of a stable counting sort
                              (exclusive prefix sum of CELL_COUNT; the library
                              keeps particles grouped by tile, not in that order) */
    LBMPCD_NODE_MPCD_U = 14, /* double[dim][nx*(yhi-ylo)*nz]: mean velocity of the
                              particles sampled in each slab node (x fastest, then
                              y - ylo, then z) in the last LB step, the sample the
                              feedback's running mean takes in next; needs
                              feedback 1 (E_STATE otherwise); 0 where no particle
                              was sampled                                          */
    LBMPCD_TFINE = 15,     /* double[6][nz*r][R][nx*r]: the Chapman-Enskog tensor T of
                              each buffer cell (xx yy zz xy xz yz; zero outside the
                              buffers) of the last exchange step; needs reinject 1
                              (E_STATE otherwise)                                  */
    LBMPCD_NODE_FB_U = 16  /* double[dim][nx*(yhi-ylo)*nz]: the running mean of the
                              MPCD velocity per slab node (layout of NODE_MPCD_U)
                              that the feedback projects; interior nodes only (the
                              buffer nodes keep their initial velocity); needs
                              feedback 1 (E_STATE otherwise)                       */
};

typedef struct lbmpcd_params {
    uint32_t abi_version;  /* LBMPCD_ABI_VERSION */
    uint32_t struct_size;  /* sizeof(lbmpcd_params) */
    int32_t dim;           /* 2: D2Q9, 3: D3Q19 */
    int32_t n[3];          /* LB nodes nx, ny, nz (nz = 1 in 2D) */
    int32_t lb_fp;         /* population storage: 32 or 64 */
    double tau, rho0;      /* BGK relaxation time (> 1/2), initial density */
    double g[3];           /* body acceleration; LB force density rho*g (Guo forcing) */
    int32_t walls_y;       /* 1: bounce-back walls at y = 0, ny; 0: periodic y */
    int32_t mpcd;          /* 0: LB only */
    int32_t ylo, yhi;      /* MPCD slab rows [ylo, yhi), full x and z extent */
    int32_t buf_lo, buf_hi;/* buffer depth (LB rows) at the LB-facing faces; a face
                              on a wall has no buffer */
    int32_t refine;        /* r: cell side a = 1/r */
    int32_t substeps;      /* S: MPCD steps per LB step */
    int32_t ppc;           /* initial particles per cell */
    int32_t part_fp;       /* particle storage: 32 or 64 (cell sums always 64) */
    double mass, kT, alpha_deg;
    int32_t collision;     /* 0: SRD (stochastic rotation, Eq. 4); 1: MPCD with Andersen
                              thermostat (Eq. 6): every particle gets the cell's centre of
                              mass plus its own Gaussian velocity (variance kT/m per
                              component) less the cell mean of those; all instances of a
                              context share it */
    int32_t grid_shift;    /* 1: random grid shift every MPCD step */
    int32_t feedback;      /* 1: project a running time average of the MPCD velocity
                              onto the LB equilibria of the slab's interior nodes
                              (not the buffers); 0: the paper's one-way coupling */
    int32_t init_flow;     /* 0: rest, 1: discrete Poiseuille profile (needs walls) */
    uint64_t seed;         /* Philox key (low, high ^ instance) */
    uint32_t instance;     /* instance number inside the key */
    int32_t tile[3];       /* particle tile in cells per axis (powers of two); 0 = from tile_target */
    double capacity_factor;/* tile capacity / expected occupancy; 0 = default 1.3 */
    int32_t tile_target;   /* expected particles per tile when tile[] is 0; 0 = default 1280 */
    int32_t wg_threads;    /* particle kernel workgroup: 128, 256 or 512 threads; 0 = 256,
                              or 512 for binary64 particles in tiles of over 1024 slots
                              unless the six-slot form applies.  Six-slot form: at 256
                              threads, tiles of 1025-2048 slots whose expected
                              occupancy plus two Poisson standard deviations is within
                              1536 run six particles per thread, then an overflow pass
                              over the tiles holding more; taken with an explicit 256,
                              and by default on grids of at least 4096 tiles.
                              All instances of a context must agree. */
    int32_t closure;       /* 1: reserve the learned closure (lbmpcd_closure_*); needs
                              dim 3, mpcd and a single channel */
    int32_t reinject;      /* exchange step (Sec. 2.3) in the buffer cells: 0 the paper's
                              Maxwell-Boltzmann draw about the interpolated LB velocity; 1 a
                              first-order Chapman-Enskog draw about it, the remedy Sec. 2.3
                              names for strong gradients: the Maxwellian times 1 - T:z z,
                              z the thermal velocity in units of sqrt(kT/m), T = (ce_nu m/kT)
                              dev S with S = -(sum f c c - rho I/3 - rho u u)/(2 rho tau/3)
                              the lattice's strain rate, interpolated like u; sampled by
                              acceptance-rejection against the Maxwellian (envelope
                              1 + 30 x the largest absolute row sum of T, at most 32
                              attempts, else the first attempt's draw).  Needs kT > 0;
                              all instances of a context share it */
    double ce_nu;          /* stress coefficient of the Chapman-Enskog exchange (any finite
                              value), or 0: the kinetic stress the MPCD fluid carries right
                              after its collision, the instant of the exchange,
                              nu_kin - kT dt/(2m), with nu_kin the kinetic viscosity of the
                              collision rule (MPCD-AT: Eq. 7's first term, so the default is
                              kT dt/m (N/(N-1+e^-N) - 1); SRD: kT dt/m [N/((N-1+e^-N)
                              (1-cos 2a)) - 1/2] in 2D, kT dt/m [5N/((N-1+e^-N)(4-2cos a
                              -2cos 2a)) - 1/2] in 3D, negative at large angles) */
    int32_t fb_window;     /* feedback: W in LB steps.  Every LB step the running mean of
                              an interior slab node moves towards the mean velocity of
                              the particles sampled in the node in the previous LB step
                              by the weight 1/W (e <- (1 - 1/W) e + (1/W) u_sample); it
                              starts at the node's initial velocity, and the node's
                              post-stream populations become the equilibrium at the LB
                              density and that velocity.  0: W = 50.  1: the last sample
                              alone, which drives the LB unstable: a node of r^d cells
                              holds a few hundred particles, whose mean carries thermal
                              noise of the size of the flow (the paper averages its
                              MPCD profiles over many samples, Sec. 3.1). */
    int32_t deterministic; /* 1: two runs of the same parameters give identical bits.  The
                              particle kernel's sums (cell velocity sums, the MPCD-AT sums,
                              the sample windows and node and profile sums) become 64-bit
                              integer sums of the values in units of 2^-40, which do not
                              depend on the order the atomics land in; the ordinary FP64
                              sums do, at the level of their last bits.  Results differ
                              from the FP64 sums by at most 2^-41 per summed value.  All
                              instances of a context share it; not with the closure or
                              the Chapman-Enskog exchange.  0: FP64 sums. */
    int32_t schedule;      /* order in which the particle kernel's workgroups take tiles:
                              0 XCD-blocked (the workgroups the hardware deals to one of
                              the eight XCDs take one contiguous range of tiles, so that
                              neighbouring tiles, which trade particles, share an L2);
                              1 linear (workgroup b takes tile b).  All instances of a
                              context share it; the results do not depend on it. */
} lbmpcd_params;

/*
 * Workspace bytes for n_inst channels described by p[0..n_inst-1].  All
 * channels of one context share dim, lb_fp, part_fp, substeps and refine.
 * Returns E_INVALID (with no context, see lbmpcd_strerror) for bad params,
 * among them a channel whose particle slots (tiles x capacity) exceed 4 GiB
 * per component (about 830M binary32 or 415M binary64 particles at the
 * default capacity).
 */
int lbmpcd_workspace_size(const lbmpcd_params* p, int32_t n_inst, size_t* bytes);

/*
 * Kinematic viscosities of one parameter set, in LB units (host only, no
 * device work): nu_lb = (tau - 1/2) / 3 of the BGK lattice (Sec. 2.1), and
 * nu_mpcd of the MPCD fluid at its step dt = 1/substeps, cell side
 * a = 1/refine and N = ppc particles per cell: for MPCD-AT (collision 1)
 * Eq. 7, kT dt / m [N / (N - 1 + e^-N) - 1/2] + a^2 / (12 dt) (N - 1 + e^-N) / N;
 * for 2D SRD the kinetic part kT dt / m [N / ((N - 1 + e^-N)(1 - cos 2 alpha))
 * - 1/2] plus the collisional part a^2 (1 - cos alpha)(N - 1 + e^-N) / (12 dt N)
 * of the SRD literature (Ihle, Tuzel, Kroll; not in the paper); for 3D SRD
 * kT dt / m [5N / ((N - 1 + e^-N)(4 - 2 cos alpha - 2 cos 2 alpha)) - 1/2]
 * + a^2 (1 - cos alpha)(N - 1 + e^-N) / (18 dt N) (the same literature).
 * Either output may be NULL.  E_INVALID for bad parameters.
 */
int lbmpcd_viscosity(const lbmpcd_params* p, double* nu_lb, double* nu_mpcd);

/*
 * Initialise n_inst channels in the caller's device workspace (bytes at
 * least lbmpcd_workspace_size) and bind them to hip_stream (a hipStream_t,
 * may be NULL for the default stream).  Particles: exactly ppc per fine cell,
 * uniform inside the cell, Maxwell-Boltzmann velocities of variance kT/m
 * about the initial flow; LB: equilibrium at rho0 and the initial flow.
 * *out receives the context, or NULL on failure.
 */
int lbmpcd_init(const lbmpcd_params* p, int32_t n_inst, void* dev_workspace, size_t bytes,
                void* hip_stream, struct lbmpcd_ctx** out);

/*
 * Advance every channel by n_lb_steps coupled steps (Alg. 1/2): LB collide
 * and stream, optional feedback projection, interpolation of the LB
 * velocity to the buffer cells, then per MPCD step: Maxwell-Boltzmann redraw
 * in the buffer, streaming with wall / periodic / slab re-wrap conditions,
 * random grid shift, binning and the collision (SRD or MPCD-AT).  Asynchronous.
 */
int lbmpcd_step(struct lbmpcd_ctx* c, int32_t n_lb_steps);

/*
 * Derived fields of instance inst (RHO, U, PI, CELL_ID, CELL_COUNT,
 * CELL_VCM, PROFILE, UFINE, STATS) into dst (dst_bytes at least the field's
 * size, see lbmpcd_field_bytes).  dst_on_device = 1: dst is device memory on
 * the context's device and the call is asynchronous; 0: host memory, the
 * call synchronises.  Host transfers of fields larger than the workspace's
 * staging area return E_INVALID.
 */
int lbmpcd_moments(struct lbmpcd_ctx* c, int32_t field, int32_t inst, void* dst,
                   size_t dst_bytes, int32_t dst_on_device);

/* Bytes of a field of instance inst. */
int lbmpcd_field_bytes(const struct lbmpcd_ctx* c, int32_t field, int32_t inst, size_t* bytes);

/*
 * Time averaging of the MPCD velocity profile (Sec. 3.1: averaging over
 * samples suppresses the particle noise).  mode 1: zero the accumulators and
 * start sampling, once per LB step after the streaming of its last MPCD
 * step; 0: stop.
 */
int lbmpcd_sample(struct lbmpcd_ctx* c, int32_t mode);

/*
 * Checkpoint / restore of POP, PART_POS, PART_VEL of instance inst.  get has
 * the same transfer rules as moments; set replaces the field (particle
 * positions must lie inside the slab) and leaves the state fully collided.
 */
int lbmpcd_get_state(struct lbmpcd_ctx* c, int32_t field, int32_t inst, void* dst, size_t bytes,
                     int32_t dst_on_device);
int lbmpcd_set_state(struct lbmpcd_ctx* c, int32_t field, int32_t inst, const void* src,
                     size_t bytes, int32_t src_on_device);

/* Wait for the stream and report latched device errors. */
int lbmpcd_sync(struct lbmpcd_ctx* c);

/*
 * Kernel timing with HIP events recorded on the context's stream around every
 * launch of lbmpcd_step.  mode 1: reset and start; 0: stop.  Kernel classes:
 * 0 LB collide-stream, 1 feedback/band, 2 interpolation, 3 particle (MPCD)
 * step.  lbmpcd_timing_read synchronises and writes, for k < n_classes,
 * out[2k] = summed milliseconds and out[2k+1] = number of launches.
 */
int lbmpcd_timing(struct lbmpcd_ctx* c, int32_t mode);
int lbmpcd_timing_read(struct lbmpcd_ctx* c, double* out, int32_t n_classes);

/*
 * Replay of steady-state steps from a captured HIP graph (default on).  Two
 * coupled steps are recorded once per buffer parity and sampling state and
 * replayed on the context's stream; steps with a pending state change, with
 * timing on, or an odd remainder are launched directly.  enable 0 launches
 * every kernel directly.
 */
int lbmpcd_graphs(struct lbmpcd_ctx* c, int32_t enable);

/* Free the host context; never frees caller memory. */
void lbmpcd_destroy(struct lbmpcd_ctx* c);

/*
 * Launch-shape autotuner (not part of the method: it picks how the particle
 * step is cut into work, never what it computes).  Candidates are the tile
 * sizes tile_target in {160, 320, 640, 1280} expected particles per tile
 * (each instance's tile then follows from its own particles per cell) times
 * the particle kernel's workgroup size wg_threads in {256, 512} times the
 * tile order schedule in {0, 1} (lbmpcd_params.schedule).  Each
 * candidate is initialised in dev_workspace (candidates that need more than
 * `bytes`, or are invalid for the parameters, are skipped), run for
 * 2 * lb_steps coupled steps and timed over the last lb_steps with HIP events
 * on hip_stream; the workspace contents are overwritten.  p[i].tile must be
 * zero.  *out receives the fastest candidate; the results of the method do
 * not depend on the choice.  Synchronises the stream.
 */
typedef struct lbmpcd_tuning {
    uint32_t struct_size;  /* sizeof(lbmpcd_tuning), set by the caller */
    int32_t tile_target;   /* chosen expected particles per tile */
    int32_t wg_threads;    /* chosen workgroup size */
    int32_t tried;         /* candidates measured */
    double ms_per_step;    /* ms per coupled LB step of the chosen candidate */
    double ms_default;     /* ms per coupled LB step of the library's default shape (tile
                              target 1280, its default workgroup, schedule 0), -1 if not
                              measured */
    int32_t schedule;      /* chosen tile order */
} lbmpcd_tuning;

int lbmpcd_autotune(const lbmpcd_params* p, int32_t n_inst, void* dev_workspace, size_t bytes,
                    void* hip_stream, int32_t lb_steps, lbmpcd_tuning* out);

/*
 * Learned closure.  Not part of the method of the paper: a surrogate that,
 * where thermal fluctuations are not needed, stands in for the MPCD slab.
 * With one-way coupling (feedback 0, as in the paper's Alg. 1/2) it supplies
 * the MPCD averages (the time-averaged profile) from the LB state without
 * advancing particles; with feedback 1 its velocity also replaces the
 * particle averages in the projection onto the LB equilibria, where any
 * bias of the prediction acts like an extra body force (the periodic check
 * below guards against that).  A network (MLP 271 -> 128 -> 128 -> 128 -> 9,
 * GELU, BF16 weights and activations, FP32 accumulation on the matrix
 * cores) maps the LB moments around a slab node -- rho, u and Pi (Sec. 2.1,
 * the moments of the populations) of the 3x3x3 neighbourhood, x and z
 * periodic, y clamped -- and the node's shear rate sqrt(2 S:S), S = -(Pi -
 * rho u u) / (2 rho c_s^2 tau), to the node's MPCD mean velocity (3) and
 * kinetic stress sum m (v - u)(v - u) per unit volume (xx yy zz xy xz yz).
 * The network's velocity outputs are relative to the node's own LB velocity
 * (features 131..133, the centre of the stencil); targets Y and the outputs
 * of lbmpcd_closure_forward are absolute.
 * Features are standardised and targets too (mean and standard deviation of
 * the training set), the loss is the mean squared error in standardised
 * units, training is Adam on FP32 parameters with a BF16 copy for the
 * products.  Contexts must be created with closure = 1 (dim 3, one channel).  The parameter block (lbmpcd_closure_weights) is FP32:
 * W1[128][288] b1[128] W2[128][128] b2[128] W3[128][128] b3[128] W4[9][128]
 * b4[9] (weights [out][in]; W1's inputs 271..287 are zero), then the
 * statistics mean_x[271] std_x[271] mean_y[9] std_y[9]: 71737 floats.
 * Device pointers X, Y hold rows of 271 raw features and 9 raw targets.
 */
typedef struct lbmpcd_train_opts {
    uint32_t struct_size;  /* sizeof(lbmpcd_train_opts) */
    int32_t epochs;        /* passes of ceil(n / batch) Adam steps */
    int32_t batch;         /* rows per step, drawn uniformly with Philox; >= n: all rows in order */
    float lr, beta1, beta2, eps;  /* Adam */
    uint64_t seed;         /* initial weights (Glorot uniform) when none are set */
} lbmpcd_train_opts;

/* Scratch bytes of lbmpcd_closure_train / loss_grad / forward for n rows. */
int lbmpcd_closure_scratch_size(int64_t n, int32_t batch, size_t* bytes);

/*
 * Training data from the plain coupled step: advances lb_steps LB steps and
 * writes, per slab node (x fastest, then y - ylo, then z), the features
 * averaged over the window (after every LB collide-stream) into X and the
 * targets (post-collision particle moments after every LB step) into Y.
 * Asynchronous; the closure must be disabled.
 */
int lbmpcd_closure_collect(struct lbmpcd_ctx* c, int32_t lb_steps, float* X, float* Y);

/*
 * Train on n rows: statistics and initial weights are set on the first call
 * (or by lbmpcd_closure_weights), later calls continue.  loss_per_epoch
 * (host, epochs entries, may be NULL) receives the mean batch loss of each
 * epoch; the call then synchronises once per epoch.
 */
int lbmpcd_closure_train(struct lbmpcd_ctx* c, const float* X, const float* Y, int64_t n,
                         const lbmpcd_train_opts* opts, void* scratch, size_t scratch_bytes,
                         float* loss_per_epoch);

/* Loss and parameter gradient (host, NPARAM = 71177 floats, may be NULL) on n rows; synchronises. */
int lbmpcd_closure_loss_grad(struct lbmpcd_ctx* c, const float* X, const float* Y, int64_t n, void* scratch,
                             size_t scratch_bytes, double* loss, float* grad);

/* Raw features of every slab node of the current populations (device X, nslab x 271). */
int lbmpcd_closure_features(struct lbmpcd_ctx* c, float* X);

/* Network output in physical units for n rows of raw features (device Y, n x 9). */
int lbmpcd_closure_forward(struct lbmpcd_ctx* c, const float* X, int64_t n, float* Y, void* scratch,
                           size_t scratch_bytes);

/*
 * lbmpcd_closure_forward without allocation, for callers that cannot
 * allocate device memory at the call (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc).  Same result as
 * lbmpcd_closure_forward on the same X (same kernels and operands): device X
 * [n][271] raw features in, device Y [n][9] physical outputs out, both owned
 * by the caller.  The activations live in a file-scope device array of the
 * library (about 24 MB, one copy on every device the library runs on, held
 * until the process ends; its address is resolved once per device at
 * lbmpcd_init); no scratch argument, and the call allocates and frees
 * nothing.  n must be at most LBMPCD_NOALLOC_MAX_ROWS (E_INVALID otherwise,
 * before any work is enqueued).  All calls on one device share the array:
 * calls that overlap on one device (several streams or threads) race and
 * must be serialised by the caller.  Asynchronous on the context's stream;
 * E_STATE before the parameters are set.
 */
#define LBMPCD_NOALLOC_MAX_ROWS 8192
int lbmpcd_closure_forward_noalloc(struct lbmpcd_ctx* c, const float* X, int64_t n, float* Y);

/* Network output in physical units for every slab node of the current
 * populations (device Y, nslab x 9, slab nodes x fastest, then y - ylo, then
 * z), computed by the fused inference kernel that the surrogate step uses:
 * band moments, features and the four layers in two launches.  Equal to
 * lbmpcd_closure_forward on lbmpcd_closure_features' output.  Asynchronous;
 * E_STATE before the parameters are set. */
int lbmpcd_closure_predict(struct lbmpcd_ctx* c, float* Y);

/* get_or_set 0: copy the parameter block out (host); 1: load it (resets Adam). Synchronises. */
int lbmpcd_closure_weights(struct lbmpcd_ctx* c, int32_t get_or_set, float* buf, size_t bytes);

/*
 * on 1: lbmpcd_step runs LB collide-stream and the network on every slab
 * node (profile samples; with feedback, the projection with the predicted
 * velocity); no particle step.
 * Every check_every LB steps (0: never) a check with check_steps plain
 * steps (lbmpcd_closure_check) runs, synchronously, and falls back to the
 * plain MPCD step for good when the error exceeds fallback_tol (0: 0.02).
 */
int lbmpcd_closure_enable(struct lbmpcd_ctx* c, int32_t on, double fallback_tol, int32_t check_every,
                          int32_t check_steps);

/*
 * Plain coupled burst of burst_steps LB steps (the particles resume from
 * their last state; the profile of the second half is kept) against the
 * network's profile of the final LB state: relative L2 error of the
 * streamwise velocity averaged over each LB node row between the buffers
 * (the network predicts node averages).  Disables
 * the closure when above the tolerance.  Resets the profile accumulators.
 */
int lbmpcd_closure_check(struct lbmpcd_ctx* c, int32_t burst_steps, double* rel_err);

int lbmpcd_closure_status(const struct lbmpcd_ctx* c, int32_t* on, int32_t* fell_back, double* last_err);

/*
 * The matrix-core product of the closure on its own: C[M][N] = A[M][K] B[N][K]^T,
 * BF16 row-major operands, FP32 result, on hip_stream.  Asynchronous.
 */
int lbmpcd_closure_gemm_bf16(int64_t M, int64_t N, int64_t K, const uint16_t* A, const uint16_t* B, float* C,
                             void* hip_stream);

const char* lbmpcd_strerror(int code);
const char* lbmpcd_last_error(const struct lbmpcd_ctx* c);

typedef struct lbmpcd_ctx lbmpcd_ctx;

#ifdef __cplusplus
}
#endif
#endif
