/*
 * lbmpcd_oracle.h -- plain, slow, single-threaded FP64 CPU reference of the
 * coupled lattice-Boltzmann / multiparticle-collision (LB-MPCD) time step of
 * Montessori, Tiribocchi, Lauricella and Succi, "A coupled lattice
 * Boltzmann-Multiparticle collision method for multi-resolution
 * hydrodynamics" (arXiv 2004.00304).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path.  Only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * load it.  It shares no source with the HIP library (its own parameter
 * struct, its own Philox, its own lattice tables) and never includes the
 * product headers.
 *
 * Everything is double precision.  When part_fp32 is set, particle positions
 * and velocities are rounded to binary32 at every point where they are stored,
 * and the streaming update is evaluated in binary32, so that the oracle takes
 * the same float-valued binning decisions as a binary32 particle store.
 *
 * Errors: functions returning int return 0 on success and a positive code on
 * failure (1 = invalid parameters, 2 = out of memory, 5 = invalid state: orc_step
 * stops after an LB step in which a particle left the domain by more than one
 * period, or had a non-finite position or velocity, or a node of the rows the
 * coupling reads had a non-positive or non-finite density or a non-finite
 * velocity; such particles are parked at the slab's lower corner at rest, so
 * every index stays in range).
 */
#ifndef LBMPCD_ORACLE_H
#define LBMPCD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Problem statement of the paper's results section (Poiseuille channel, body
 * force along the flow, periodic along the flow, no-slip walls) extended to
 * D3Q19 and to a refined MPCD slab with buffers (Sec. 2.3, Alg. 1 and 2). */
typedef struct orc_params {
    int32_t dim;            /* 2 (D2Q9) or 3 (D3Q19) */
    int32_t nx, ny, nz;     /* LB nodes; nz = 1 in 2D */
    double tau, rho0;       /* BGK relaxation time (Eq. 1), initial density */
    double g[3];            /* body acceleration; LB force density is rho*g */
    int32_t walls_y;        /* 1: half-way bounce-back walls at y=0 and y=ny; 0: periodic y */
    int32_t mpcd;           /* 0: LB only */
    int32_t ylo, yhi;       /* MPCD slab [ylo, yhi) in LB rows, full x and z extent */
    int32_t buf_lo, buf_hi; /* buffer (coupling region) depth in LB rows at the LB-facing faces */
    int32_t refine;         /* r: collision cell side a = 1/r LB units */
    int32_t substeps;       /* S: MPCD steps per LB step, delta_t = 1/S */
    int32_t ppc;            /* initial particles per collision cell */
    int32_t part_fp32;      /* 1: binary32 particle store */
    double mass, kT, alpha_deg;
    int32_t grid_shift;     /* 1: random grid shift every MPCD step */
    int32_t feedback;       /* 1: project MPCD averages back onto LB equilibria */
    int32_t init_flow;      /* 0: rest, 1: discrete Poiseuille steady profile */
    uint64_t seed;
    uint32_t instance;
    int32_t collision;      /* 0: SRD rotation (Eq. 4); 1: MPCD with Andersen thermostat (Eq. 6) */
    int32_t reinject;       /* exchange step: 0 Maxwell-Boltzmann (Sec. 2.3); 1 first-order
                               Chapman-Enskog about the LB strain rate (the remedy the paper
                               names for strong gradients, Sec. 2.3) */
    double ce_nu;           /* viscosity coefficient of the Chapman-Enskog stress (finite);
                               0: the kinetic stress the MPCD fluid carries right after its
                               collision, the instant of the exchange: nu_kin - kT dt / (2m) */
    int32_t fb_window;      /* feedback: LB steps W of the running mean of the node samples
                               that is projected (weight 1/W per LB step); 0 = 50; 1 = the
                               last LB step's sample alone */
} orc_params;

typedef struct orc_state orc_state;

/* ---- stateful simulation --------------------------------------------- */
int  orc_create(const orc_params* p, orc_state** out);
void orc_destroy(orc_state* s);
int  orc_step(orc_state* s, int32_t n_lb_steps);
/* mode 1: reset and start accumulating the time-averaged profile; 0: stop */
void orc_sample(orc_state* s, int32_t mode);

int64_t orc_num_particles(const orc_state* s);
int32_t orc_num_cells(const orc_state* s);       /* cells of the shifted binning grid */
int32_t orc_num_fine_rows(const orc_state* s);   /* fine rows of the slab */
int64_t orc_lb_step_count(const orc_state* s);

/* post-stream populations f[q][z][y][x] */
void orc_get_f(const orc_state* s, double* f);
void orc_set_f(orc_state* s, const double* f);
/* post-collision populations (BGK+Guo collision of the stored state) */
void orc_get_fstar(const orc_state* s, double* f);
/* rho[N], u[3][N] (u includes the half-force shift), pi[6][N] (xx,yy,zz,xy,xz,yz) */
void orc_get_moments(const orc_state* s, double* rho, double* u, double* pi);
/* particles by id: pos[d][Np], vel[d][Np] */
void orc_get_particles(const orc_state* s, double* pos, double* vel);
void orc_set_particles(orc_state* s, const double* pos, const double* vel);
/* binning of the last MPCD step: cell of each particle, cell counts, cell
 * starts of the stable counting sort, sorted order (particle ids), and the
 * centre-of-mass velocity of every cell (virtual wall particles included) */
void orc_get_binning(const orc_state* s, int32_t* cell_of, int32_t* count,
                     int32_t* start, int32_t* order, double* vcm);
/* interpolated LB velocity at every fine cell of the slab, [d][K][J][I] */
void orc_get_ufine(const orc_state* s, double* ufine);
/* time-averaged profile accumulators per fine row: [J][0]=sum n, [J][1+k]=sum v_k */
void orc_get_profile(const orc_state* s, double* acc, int64_t* n_lb_steps_sampled);
/* per-LB-step sample accumulators of the slab [(iz*R + J)*nx + ix][4] */
void orc_get_step_acc(const orc_state* s, double* acc);
/* running mean of the node samples that the feedback projects: [nz][yhi-ylo][nx][3] */
void orc_get_fb_u(const orc_state* s, double* out);
/* grid shift of the last MPCD step */
void orc_get_shift(const orc_state* s, double sh[3]);
/* recompute the buffer fine-cell velocities from the current populations */
void orc_refresh_ufine(orc_state* s);

/* geometry-only state for the per-element functions below (no arrays) */
int orc_create_geometry(const orc_params* p, orc_state** out);
/* grid shift of MPCD step (t, sub) */
void orc_grid_shift(const orc_state* s, uint32_t t, uint32_t sub, double sh[3]);
/* shifted-grid cell of n positions pos[dim][n] */
void orc_bin_positions(const orc_state* s, const double sh[3], int64_t n, const double* pos, int32_t* cell);
/* exchange step + streaming of one MPCD step for n particles in place; u[dim][n]
 * is the interpolated LB velocity of each particle's fine cell and tens[6][n]
 * its Chapman-Enskog tensor (NULL: Maxwell-Boltzmann exchange) */
void orc_exchange_stream(const orc_state* s, uint32_t t, uint32_t sub, int64_t n, const uint32_t* ids,
                         double* pos, double* vel, const double* u, const double* tens);
int32_t orc_in_buffer(const orc_state* s, const double r[3]);
/* buffer fine-cell velocities ufine[3][Cz][R][Cx] from node velocities unode[3][N] */
void orc_interpolate(const orc_state* s, const double* unode, double* ufine);
/* collision (SRD or MPCD-AT, per the parameters) of the n particles
 * (vel[dim][n], in place) of cell c; ids[n] are the particles' ids (the
 * MPCD-AT draws are keyed by them; may be NULL for SRD) */
void orc_collide_cell(const orc_state* s, int32_t c, uint32_t t, uint32_t sub, const double sh[3], int32_t n,
                      const int32_t* ids, double* vel, double vcm[3]);

/* ---- building blocks, exported for the pins ---------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u01(uint32_t lo, uint32_t hi);
/* Philox4x32-10 of the counters first .. first + n - 1 (as 128-bit integers)
 * under one key: out[4n] */
void orc_philox_stream(const uint32_t key[2], uint64_t first, uint64_t n, uint32_t* out);
/* lattice tables: returns Q; c is Q*3 ints, w is Q doubles, opp is Q ints */
int  orc_lattice(int32_t dim, int32_t* c, double* w, int32_t* opp);
void orc_feq(int32_t dim, double rho, const double u[3], double* feq);
/* one BGK+Guo collision of a single node's populations (in place) */
void orc_collide_node(int32_t dim, double tau, const double g[3], double* f);
/* Box-Muller pair from two uniforms */
void orc_box_muller(double u0, double u1, double* z0, double* z1);
/* binary32 normals of binary32 particles: ln on (0, 1], sin/cos of 2 pi u,
 * the normals of one Philox block (z[2] = 0 in 2D), and n blocks at once */
float orc_ln32(float x);
void orc_sincos32(float u, float* sn, float* cs);
void orc_normals32(const uint32_t w[4], int32_t dim, float z[3]);
void orc_normals32_n(const uint32_t* w, int64_t n, int32_t dim, float* z);
/* SRD rotation of n velocities (vel[d][n]) about their centre of mass */
void orc_srd_rotate(int32_t dim, int32_t n, double* vel, double cos_a, double sin_a,
                    double sign2d, const double axis[3], const double p_virt[3], double m_virt,
                    double vcm_out[3]);
/* MPCD-AT collision (Eq. 6) of n velocities (vel[d][n], in place) given
 * their random velocities vran[d][n]: v <- v_cm + vran - mean(vran), the
 * centre of mass including virtual wall momentum p_virt and mass m_virt */
void orc_at_collide(int32_t dim, int32_t n, double* vel, const double* vran, const double p_virt[3],
                    double m_virt, double vcm_out[3]);
/* kinematic viscosity of MPCD-AT (Eq. 7): kT dt / m [N / (N - 1 + e^-N) - 1/2]
 * + a^2 / (12 dt) (N - 1 + e^-N) / N */
double orc_nu_at(double kT, double mass, double dt, double a, double N);
/* kinetic part of the MPCD viscosity of the parameter set: MPCD-AT the first
 * term of Eq. 7; SRD the kinetic term of the SRD literature in 2D and 3D */
double orc_nu_kinetic(const orc_params* p);
/* coefficient of the Chapman-Enskog exchange's stress: ce_nu, or by default
 * orc_nu_kinetic(p) - kT dt / (2m) */
double orc_ce_nu(const orc_params* p);
/* Chapman-Enskog tensor T[6] (xx,yy,zz,xy,xz,yz) of every node from the
 * current populations: out[6][N] */
void orc_ce_tensor(const orc_state* s, double* out);
/* buffer fine-cell tensors tfine[6][Cz][R][Cx] of the last exchange step */
void orc_get_tfine(const orc_state* s, double* tfine);
/* d standard normals of element `id` accepted against the Maxwellian with the
 * weight 1 - T:zz (T[6] as above); returns the attempt that was accepted
 * (CE_ATTEMPTS when none was, and z is then the first attempt's draw) */
int32_t orc_ce_normals(const orc_params* p, uint32_t id, uint32_t t, uint32_t sub, const double T[6],
                       double z[3]);
/* stable counting sort of cell ids: count[nc], start[nc], order[n] */
void orc_counting_sort(int32_t n, const int32_t* cell, int32_t nc,
                       int32_t* count, int32_t* start, int32_t* order);

#ifdef __cplusplus
}
#endif
#endif
