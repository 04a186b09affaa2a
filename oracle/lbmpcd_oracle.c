/*
 * lbmpcd_oracle.c -- plain FP64 CPU reference of the coupled LB-MPCD time
 * step (arXiv 2004.00304).  TEST INFRASTRUCTURE ONLY: loaded by the tests, the
 * smoke check and the CPU-baseline leg of the benchmark, never by the product
 * path.  Shares no code with the HIP library.
 *
 * Every loop below is the definition written out, one node / one particle /
 * one cell at a time, in the order of the paper's coupling procedure
 * (Alg. 1 and Alg. 2): LB collision, LB streaming, interpolation of the LB
 * velocity to the fine grid, exchange (Maxwell-Boltzmann redraw in the
 * buffer), MPCD streaming with boundary conditions, MPCD collision.
 *
 * Readings of points the paper leaves open are marked READING and listed in
 * the design notes: lattice weights, Guo forcing, wall positions, random grid
 * shift, substeps, virtual wall particles, sampling instant, feedback, and the
 * Chapman-Enskog form of the exchange step.
 */
#include "lbmpcd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------
 * Counter-based random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11).  Four 32-bit counter
 * words, two key words, ten rounds; each round multiplies the two even words
 * by fixed odd constants and mixes the high halves with the odd words and the
 * key; the key is bumped by the Weyl constants between rounds.
 * ---------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Philox4x32-10 of the consecutive 128-bit counters first, first + 1, ...
 * (n of them, below 2^64) under one key: out[4n], the stream a counter-mode
 * generator seeded with the key produces. */
void orc_philox_stream(const uint32_t key[2], uint64_t first, uint64_t n, uint32_t* out) {
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t c = first + i;
        uint32_t ctr[4] = {(uint32_t)c, (uint32_t)(c >> 32), 0u, 0u};
        orc_philox4x32_10(ctr, key, out + 4 * i);
    }
}

/* uniform in [0,1) from the top 53 bits of a 64-bit word (hi:lo) */
double orc_u01(uint32_t lo, uint32_t hi) {
    uint64_t x = ((uint64_t)hi << 32) | (uint64_t)lo;
    return (double)(x >> 11) * 0x1.0p-53;
}

/* READING: purposes of the random streams; the counter is
 * (element, LB step, substep<<8 | purpose, block). */
enum { P_INIT_POS = 1, P_INIT_VEL = 2, P_REINJ = 3, P_SHIFT = 4, P_ROT = 5, P_WALL = 6, P_AT = 9 };

static void rng_block(const orc_params* p, uint32_t elem, uint32_t t, uint32_t sub,
                      uint32_t purpose, uint32_t blk, uint32_t out[4]) {
    uint32_t key[2] = {(uint32_t)(p->seed & 0xFFFFFFFFu),
                       (uint32_t)(p->seed >> 32) ^ p->instance};
    uint32_t ctr[4] = {elem, t, (sub << 8) | purpose, blk};
    orc_philox4x32_10(ctr, key, out);
}

/* four uniforms u[0..3] of one stream element (two Philox blocks) */
static void rng_uniforms4(const orc_params* p, uint32_t elem, uint32_t t, uint32_t sub,
                          uint32_t purpose, double u[4]) {
    uint32_t w[4];
    rng_block(p, elem, t, sub, purpose, 0, w);
    u[0] = orc_u01(w[0], w[1]);
    u[1] = orc_u01(w[2], w[3]);
    rng_block(p, elem, t, sub, purpose, 1, w);
    u[2] = orc_u01(w[0], w[1]);
    u[3] = orc_u01(w[2], w[3]);
}

/* Box-Muller (the paper's exchange step names it): two uniforms give two
 * independent standard normals.  READING: the trigonometric form with
 * 1-u0 inside the logarithm so that u0 = 0 is finite. */
void orc_box_muller(double u0, double u1, double* z0, double* z1) {
    double r = sqrt(-2.0 * log(1.0 - u0));
    double th = 6.283185307179586 * u1;
    *z0 = r * cos(th);
    *z1 = r * sin(th);
}

/* READING (binary32 normals): particles stored in binary32 draw the normal
 * deviates of the Maxwell-Boltzmann exchange step and of MPCD-AT in binary32
 * arithmetic.  One Philox block w[0..3] of the element's stream gives four
 * uniforms a_k = (w_k >> 8) 2^-24 (exact in binary32); the pairs (a0, a1) and
 * (a2, a3) give Box-Muller pairs with radius sqrt(-2 ln(1 - a_even)) and angle
 * 2 pi a_odd (z0 = rho cos, z1 = rho sin; in 3D z2 is the cosine of the second
 * pair).  ln and sin/cos are the series below, every step one IEEE binary32
 * operation (fmaf, correctly rounded division and square root), so that any
 * implementation of the definition yields the same bits. */

/* ln x for x in (0, 1], binary32: x = m 2^e with m in [sqrt(1/2), sqrt(2));
 * ln m = 2 atanh s with s = (m - 1)/(m + 1) = f/(2 + f), f = m - 1 exact;
 * 2 atanh s = 2s (1 + z/3 + z^2/5 + z^3/7 + z^4/9 + ...), z = s^2 < 0.0295,
 * summed to z^4/9: the first omitted term, z^5/11, is below 2e-9 of the sum,
 * a thirtieth of a binary32 unit.  Constants: sqrt(1/2) and ln 2 rounded to
 * binary32, 1/(2k+1) as binary32 quotients. */
float orc_ln32(float x) {
    int e;
    float m = frexpf(x, &e); /* m in [1/2, 1) */
    if (m < 0x1.6a09e6p-1f) {
        m = m + m;
        e = e - 1;
    }
    const float f = m - 1.0f;
    const float s = f / (2.0f + f);
    const float z = s * s;
    float c = 1.0f / 9.0f;
    c = fmaf(c, z, 1.0f / 7.0f);
    c = fmaf(c, z, 1.0f / 5.0f);
    c = fmaf(c, z, 1.0f / 3.0f);
    const float s2 = s + s;
    const float lnm = fmaf(s2 * z, c, s2);
    return fmaf((float)e, 0x1.62e430p-1f, lnm);
}

/* sin and cos of 2 pi u for u in [0, 1), binary32: 4u = q + y' exactly with
 * q = rint(4u) (ties to even) and |y'| <= 1/2; y = y' (pi/2), |y| <= pi/4;
 * sin y = y - y^3/3! + ... to y^9/9!, cos y = 1 - y^2/2! + ... to y^8/8!
 * (first omitted terms below 2e-9 and 2.5e-8 on that interval, under half a
 * binary32 unit of the result); the
 * quadrant q mod 4 then swaps and negates them.  pi/2 rounded to binary32. */
void orc_sincos32(float u, float* sn, float* cs) {
    const float t = 4.0f * u;
    const float q = rintf(t);
    const float y = (t - q) * 0x1.921fb6p+0f;
    const float z = y * y;
    float ps = 1.0f / 362880.0f;
    ps = fmaf(ps, z, -1.0f / 5040.0f);
    ps = fmaf(ps, z, 1.0f / 120.0f);
    ps = fmaf(ps, z, -1.0f / 6.0f);
    const float sy = fmaf(ps * z, y, y);
    float pc = 1.0f / 40320.0f;
    pc = fmaf(pc, z, -1.0f / 720.0f);
    pc = fmaf(pc, z, 1.0f / 24.0f);
    pc = fmaf(pc, z, -0.5f);
    const float cy = fmaf(pc, z, 1.0f);
    const int quad = (int)q & 3;
    /* angle = quad pi/2 + y */
    switch (quad) {
        case 0: *sn = sy; *cs = cy; break;
        case 1: *sn = cy; *cs = -sy; break;
        case 2: *sn = -sy; *cs = -cy; break;
        default: *sn = -cy; *cs = sy; break;
    }
}

/* The binary32 normals of one Philox block (READING above); z[2] = 0 in 2D. */
void orc_normals32(const uint32_t w[4], int32_t dim, float z[3]) {
    float a[4];
    for (int k = 0; k < 4; ++k) a[k] = (float)(w[k] >> 8) * 0x1p-24f;
    float sn, cs;
    const float r0 = sqrtf(-2.0f * orc_ln32(1.0f - a[0]));
    orc_sincos32(a[1], &sn, &cs);
    z[0] = r0 * cs;
    z[1] = r0 * sn;
    z[2] = 0.0f;
    if (dim == 3) {
        const float r1 = sqrtf(-2.0f * orc_ln32(1.0f - a[2]));
        orc_sincos32(a[3], &sn, &cs);
        z[2] = r1 * cs;
    }
}

/* n blocks at once (tests): w[4n] -> z[3n] */
void orc_normals32_n(const uint32_t* w, int64_t n, int32_t dim, float* z) {
    for (int64_t i = 0; i < n; ++i) orc_normals32(w + 4 * i, dim, z + 3 * i);
}

/* d binary32 normals of one stream element (block 0), widened */
static void rng_normals32(const orc_params* p, uint32_t elem, uint32_t t, uint32_t sub, uint32_t purpose,
                          double z[3]) {
    uint32_t w[4];
    float zf[3];
    rng_block(p, elem, t, sub, purpose, 0, w);
    orc_normals32(w, p->dim, zf);
    for (int k = 0; k < 3; ++k) z[k] = (double)zf[k];
}

/* d standard normals of one stream element from the Philox blocks blk and
 * blk + 1 */
static void rng_normals_at(const orc_params* p, uint32_t elem, uint32_t t, uint32_t sub,
                           uint32_t purpose, uint32_t blk, double z[3]) {
    uint32_t w[4];
    double u[4], dummy;
    rng_block(p, elem, t, sub, purpose, blk, w);
    u[0] = orc_u01(w[0], w[1]);
    u[1] = orc_u01(w[2], w[3]);
    rng_block(p, elem, t, sub, purpose, blk + 1, w);
    u[2] = orc_u01(w[0], w[1]);
    u[3] = orc_u01(w[2], w[3]);
    orc_box_muller(u[0], u[1], &z[0], &z[1]);
    orc_box_muller(u[2], u[3], &z[2], &dummy);
    if (p->dim == 2) z[2] = 0.0;
}

/* d standard normals of one stream element */
static void rng_normals(const orc_params* p, uint32_t elem, uint32_t t, uint32_t sub,
                        uint32_t purpose, double z[3]) {
    rng_normals_at(p, elem, t, sub, purpose, 0, z);
}

/* ------------------------------------------------------------------------
 * Lattice (Sec. 2.1).  The paper fixes D2Q9 and c_s^2 = 1/3 but does not
 * print the weights; READING: the textbook D2Q9 and D3Q19 weights.
 * ---------------------------------------------------------------------- */
static const int C9[9][3] = {{0, 0, 0}, {1, 0, 0},  {0, 1, 0},   {-1, 0, 0}, {0, -1, 0},
                             {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const int C19[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                               {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                               {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                               {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

int orc_lattice(int32_t dim, int32_t* c, double* w, int32_t* opp) {
    int Q = (dim == 2) ? 9 : 19;
    for (int i = 0; i < Q; ++i) {
        const int* ci = (dim == 2) ? C9[i] : C19[i];
        int c2 = ci[0] * ci[0] + ci[1] * ci[1] + ci[2] * ci[2];
        for (int k = 0; k < 3; ++k) c[3 * i + k] = ci[k];
        if (dim == 2)
            w[i] = (c2 == 0) ? 4.0 / 9.0 : (c2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
        else
            w[i] = (c2 == 0) ? 1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    for (int i = 0; i < Q; ++i)
        for (int j = 0; j < Q; ++j)
            if (c[3 * j] == -c[3 * i] && c[3 * j + 1] == -c[3 * i + 1] &&
                c[3 * j + 2] == -c[3 * i + 2])
                opp[i] = j;
    return Q;
}

/* Second-order equilibrium, Eq. 2, with c_s^2 = 1/3. */
void orc_feq(int32_t dim, double rho, const double u[3], double* feq) {
    int32_t c[57], opp[19];
    double w[19];
    int Q = orc_lattice(dim, c, w, opp);
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        double cu = c[3 * i] * u[0] + c[3 * i + 1] * u[1] + c[3 * i + 2] * u[2];
        feq[i] = w[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* BGK collision of Eq. 1 with a constant body force.  READING: Guo forcing --
 * the equilibrium velocity carries half the force impulse and the source
 * term is (1 - 1/2tau) w_i [3(c_i - u) + 9 (c_i.u) c_i] . rho g. */
void orc_collide_node(int32_t dim, double tau, const double g[3], double* f) {
    int32_t c[57], opp[19];
    double w[19], feq[19];
    int Q = orc_lattice(dim, c, w, opp);
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        rho += f[i];
        for (int k = 0; k < 3; ++k) j[k] += f[i] * c[3 * i + k];
    }
    double u[3], F[3];
    for (int k = 0; k < 3; ++k) {
        u[k] = j[k] / rho + 0.5 * g[k];
        F[k] = rho * g[k];
    }
    orc_feq(dim, rho, u, feq);
    double omega = 1.0 / tau, src = 1.0 - 0.5 / tau;
    for (int i = 0; i < Q; ++i) {
        double cu = c[3 * i] * u[0] + c[3 * i + 1] * u[1] + c[3 * i + 2] * u[2];
        double Fi = 0.0;
        for (int k = 0; k < 3; ++k) Fi += (3.0 * (c[3 * i + k] - u[k]) + 9.0 * cu * c[3 * i + k]) * F[k];
        Fi *= w[i];
        f[i] = f[i] - omega * (f[i] - feq[i]) + src * Fi;
    }
}

/* ------------------------------------------------------------------------
 * SRD collision, Eq. 4: v_k <- v_cm + R (v_k - v_cm).  In 2D R rotates by
 * sign2d*alpha; in 3D R rotates by alpha about the unit vector axis
 * (Rodrigues' formula).  p_virt/m_virt add the momentum and mass of virtual
 * wall particles to the centre of mass (READING of the wall rule of Lamura et
 * al. that the paper cites).  Unit particle mass inside this routine; the
 * caller scales.  vel is [dim][n].
 * ---------------------------------------------------------------------- */
void orc_srd_rotate(int32_t dim, int32_t n, double* vel, double cos_a, double sin_a,
                    double sign2d, const double axis[3], const double p_virt[3], double m_virt,
                    double vcm_out[3]) {
    if (n <= 0) return;
    double P[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < dim; ++k)
        for (int i = 0; i < n; ++i) P[k] += vel[k * n + i];
    double vcm[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < dim; ++k) vcm[k] = (P[k] + p_virt[k]) / ((double)n + m_virt);
    if (vcm_out)
        for (int k = 0; k < 3; ++k) vcm_out[k] = vcm[k];
    for (int i = 0; i < n; ++i) {
        double wv[3] = {0.0, 0.0, 0.0}, r[3];
        for (int k = 0; k < dim; ++k) wv[k] = vel[k * n + i] - vcm[k];
        if (dim == 2) {
            double s = sign2d * sin_a;
            r[0] = cos_a * wv[0] - s * wv[1];
            r[1] = s * wv[0] + cos_a * wv[1];
        } else {
            double nw = axis[0] * wv[0] + axis[1] * wv[1] + axis[2] * wv[2];
            double cx = axis[1] * wv[2] - axis[2] * wv[1];
            double cy = axis[2] * wv[0] - axis[0] * wv[2];
            double cz = axis[0] * wv[1] - axis[1] * wv[0];
            double one_c = 1.0 - cos_a;
            r[0] = wv[0] * cos_a + cx * sin_a + axis[0] * nw * one_c;
            r[1] = wv[1] * cos_a + cy * sin_a + axis[1] * nw * one_c;
            r[2] = wv[2] * cos_a + cz * sin_a + axis[2] * nw * one_c;
        }
        for (int k = 0; k < dim; ++k) vel[k * n + i] = vcm[k] + r[k];
    }
}

/* ------------------------------------------------------------------------
 * MPCD with Andersen thermostat, Eq. 6: every particle of the cell gets the
 * centre-of-mass velocity plus its own random velocity minus the cell mean
 * of the random velocities (the sum over the cell's N_c particles).  The
 * centre of mass includes virtual wall particles as for SRD (READING); the
 * mean of the random part runs over the real particles only (Eq. 6 divides
 * by the actual number N_c).  vel and vran are [dim][n].
 * ---------------------------------------------------------------------- */
void orc_at_collide(int32_t dim, int32_t n, double* vel, const double* vran, const double p_virt[3],
                    double m_virt, double vcm_out[3]) {
    if (n <= 0) return;
    double P[3] = {0.0, 0.0, 0.0}, Sr[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < dim; ++k)
        for (int i = 0; i < n; ++i) {
            P[k] += vel[k * n + i];
            Sr[k] += vran[k * n + i];
        }
    double vcm[3] = {0.0, 0.0, 0.0}, mean[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < dim; ++k) {
        vcm[k] = (P[k] + p_virt[k]) / ((double)n + m_virt);
        mean[k] = Sr[k] / (double)n;
    }
    if (vcm_out)
        for (int k = 0; k < 3; ++k) vcm_out[k] = vcm[k];
    for (int k = 0; k < dim; ++k)
        for (int i = 0; i < n; ++i) vel[k * n + i] = vcm[k] + (vran[k * n + i] - mean[k]);
}

/* Eq. 7 (the paper's viscosity of MPCD-AT) */
double orc_nu_at(double kT, double mass, double dt, double a, double N) {
    const double q = N - 1.0 + exp(-N);
    return kT * dt / mass * (N / q - 0.5) + a * a / (12.0 * dt) * q / N;
}

/* Kinetic part of the MPCD viscosity (the part carried by the particles'
 * velocity distribution, which is what the Chapman-Enskog exchange has to
 * reproduce).  MPCD-AT: the first term of Eq. 7.  SRD (not in the paper; the
 * SRD literature's kinetic terms): 2D kT dt/m [N/((N-1+e^-N)(1-cos 2 alpha))
 * - 1/2], 3D kT dt/m [5N/((N-1+e^-N)(4-2cos alpha-2cos 2 alpha)) - 1/2]. */
double orc_nu_kinetic(const orc_params* p) {
    const double N = (double)p->ppc, q = N - 1.0 + exp(-N);
    const double kin = p->kT * (1.0 / p->substeps) / p->mass;
    if (p->collision == 1) return kin * (N / q - 0.5);
    const double al = p->alpha_deg * 3.141592653589793 / 180.0;
    if (p->dim == 2) return kin * (N / (q * (1.0 - cos(2.0 * al))) - 0.5);
    return kin * (5.0 * N / (q * (4.0 - 2.0 * cos(al) - 2.0 * cos(2.0 * al))) - 0.5);
}

/* READING: the stress the exchange has to reproduce is the one the MPCD fluid
 * carries at the instant of the exchange, right after a collision.  Over the
 * streaming step that follows, ballistic motion through the shear adds
 * kT dt/m per unit shear rate to the kinetic stress coefficient, and the
 * kinetic viscosity is its average over the step; so right after the collision
 * the coefficient is nu_kin - kT dt / (2m).  For MPCD-AT that is
 * kT dt/m (N/(N-1+e^-N) - 1), of order 1/N; for SRD it is negative at
 * large angles. */
double orc_ce_nu(const orc_params* p) {
    if (p->ce_nu != 0.0) return p->ce_nu;
    return orc_nu_kinetic(p) - 0.5 * p->kT * (1.0 / p->substeps) / p->mass;
}

/* ------------------------------------------------------------------------
 * Chapman-Enskog exchange (READING; the paper names sampling from an Enskog
 * distribution, after Garcia and Alexander, as the remedy when velocity
 * gradients are strong, Sec. 2.3).  To first order in the gradients the
 * velocity distribution about u is the Maxwellian times 1 - T:zz, with z the
 * thermal velocity in units of sqrt(kT/m) and T = (nu_x m / kT) dev S, S the
 * strain rate and nu_x the stress coefficient of orc_ce_nu; its covariance is
 * (kT/m)(I - 2T), i.e. the kinetic stress 2 rho nu_x dev S.  Heat flux is absent (isothermal fluid).  Samples come
 * by acceptance-rejection against the Maxwellian: attempt k draws z from the
 * Philox blocks 4k and 4k+1 of the exchange stream (attempt 0 is the
 * Maxwell-Boltzmann draw itself) and a uniform u from block 4k+2, and accepts
 * when A u <= 1 - T:zz, with the envelope A = 1 + 30 b, b the largest absolute
 * row sum of T (a bound on |T:zz| / |z|^2).  After CE_ATTEMPTS rejections the
 * first attempt's draw is kept.
 * ---------------------------------------------------------------------- */
#define CE_ATTEMPTS 32
#define CE_KAPPA 30.0

/* T:zz with T[6] = (xx, yy, zz, xy, xz, yz) */
static double ce_contract(const double T[6], const double z[3]) {
    return T[0] * z[0] * z[0] + T[1] * z[1] * z[1] + T[2] * z[2] * z[2] +
           2.0 * (T[3] * z[0] * z[1] + T[4] * z[0] * z[2] + T[5] * z[1] * z[2]);
}

static double ce_envelope(const double T[6]) {
    double r0 = fabs(T[0]) + fabs(T[3]) + fabs(T[4]);
    double r1 = fabs(T[3]) + fabs(T[1]) + fabs(T[5]);
    double r2 = fabs(T[4]) + fabs(T[5]) + fabs(T[2]);
    double b = fmax(r0, fmax(r1, r2));
    return 1.0 + CE_KAPPA * b;
}

int32_t orc_ce_normals(const orc_params* p, uint32_t id, uint32_t t, uint32_t sub, const double T[6],
                       double z[3]) {
    const double A = ce_envelope(T);
    double z0[3];
    for (int32_t k = 0; k < CE_ATTEMPTS; ++k) {
        double zk[3];
        uint32_t w[4];
        rng_normals_at(p, id, t, sub, P_REINJ, 4u * (uint32_t)k, zk);
        if (k == 0)
            for (int d = 0; d < 3; ++d) z0[d] = zk[d];
        rng_block(p, id, t, sub, P_REINJ, 4u * (uint32_t)k + 2u, w);
        double u = orc_u01(w[0], w[1]);
        if (A * u <= 1.0 - ce_contract(T, zk)) {
            for (int d = 0; d < 3; ++d) z[d] = zk[d];
            return k;
        }
    }
    for (int d = 0; d < 3; ++d) z[d] = z0[d];
    return CE_ATTEMPTS;
}

/* Stable counting sort: histogram, exclusive prefix sum, scatter in input order. */
void orc_counting_sort(int32_t n, const int32_t* cell, int32_t nc, int32_t* count,
                       int32_t* start, int32_t* order) {
    memset(count, 0, sizeof(int32_t) * (size_t)nc);
    for (int32_t i = 0; i < n; ++i) count[cell[i]]++;
    int32_t acc = 0;
    for (int32_t c = 0; c < nc; ++c) {
        start[c] = acc;
        acc += count[c];
    }
    int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
    memcpy(fill, start, sizeof(int32_t) * (size_t)nc);
    for (int32_t i = 0; i < n; ++i) order[fill[cell[i]]++] = i;
    free(fill);
}

/* ------------------------------------------------------------------------
 * State
 * ---------------------------------------------------------------------- */
struct orc_state {
    orc_params p;
    int Q;
    int32_t c[57], opp[19];
    double w[19];
    int64_t N;          /* LB nodes */
    double *f, *ftmp;   /* post-stream populations [q][N] */
    /* slab */
    int R, Cx, Cz, CyB; /* fine rows, fine columns, binning rows */
    int ywrap;          /* slab periodic in y (no faces) */
    int bot_wall, top_wall;
    int64_t Np;
    int32_t ncells;
    double *pos[3], *vel[3];
    int32_t *cell_of, *count, *start, *order;
    double* vcm;        /* [3][ncells] */
    double* ufine;      /* [3][Cz][R][Cx] */
    double* unode;      /* [3][N] */
    double* tnode;      /* [6][N] Chapman-Enskog tensor of every node */
    double* tfine;      /* [6][Cz][R][Cx] interpolated to the buffer fine cells */
    double* acc;        /* [(iz*R+J)*nx+ix][4] */
    double* fbu;        /* [((iz*(yhi-ylo))+y-ylo)*nx+ix][3] running mean the feedback projects */
    double* prof;       /* [R][4] */
    int64_t prof_steps;
    int sampling;
    int64_t t;          /* completed LB steps */
    double shift[3];    /* grid shift of the last MPCD step */
    double dt, cos_a, sin_a, a;
    double* scratch;    /* per-cell velocity gather */
    int64_t bad;        /* invalid particles / band nodes found in the last LB step */
};

static int64_t node_index(const orc_state* s, int x, int y, int z) {
    return ((int64_t)z * s->p.ny + y) * s->p.nx + x;
}

/* Particle store rounding (binary32 store when part_fp32). */
static double st(const orc_state* s, double v) { return s->p.part_fp32 ? (double)(float)v : v; }

/* READING: the exact discrete steady state of BGK + Guo forcing + half-way
 * bounce-back for a body-force driven channel with nodes at y = j + 1/2 and
 * walls at y = 0 and y = H: a parabola plus a constant slip term. */
static double poiseuille(const orc_params* p, double gk, double y) {
    double nu = (p->tau - 0.5) / 3.0, H = (double)p->ny, tau = p->tau;
    return gk * y * (H - y) / (2.0 * nu) + gk * (16.0 * tau * tau - 16.0 * tau + 1.0) / (24.0 * nu);
}

static int validate(const orc_params* p) {
    if (p->dim != 2 && p->dim != 3) return 1;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return 1;
    if (p->dim == 2 && (p->nz != 1 || p->g[2] != 0.0)) return 1;
    if (!(p->tau > 0.5) || !(p->rho0 > 0.0)) return 1;
    if (p->init_flow && !p->walls_y) return 1;
    if (!p->mpcd) return 0;
    if (p->ylo < 0 || p->yhi > p->ny || p->ylo >= p->yhi) return 1;
    if (p->refine < 1 || p->substeps < 1 || p->ppc < 1) return 1;
    if (p->buf_lo < 0 || p->buf_hi < 0 || p->buf_lo + p->buf_hi > p->yhi - p->ylo) return 1;
    int bw = p->walls_y && p->ylo == 0, tw = p->walls_y && p->yhi == p->ny;
    if ((bw && p->buf_lo) || (tw && p->buf_hi)) return 1;
    if ((bw || tw) && p->g[1] != 0.0) return 1;
    if (!(p->mass > 0.0) || p->kT < 0.0) return 1;
    if (p->collision != 0 && p->collision != 1) return 1;
    if (p->reinject != 0 && p->reinject != 1) return 1;
    if (p->reinject && (!(p->kT > 0.0) || !isfinite(p->ce_nu))) return 1;
    if (p->reinject && !isfinite(orc_ce_nu(p))) return 1;  /* SRD at alpha = 0 without ce_nu */
    if (p->fb_window < 0) return 1;
    return 0;
}

void orc_destroy(orc_state* s) {
    if (!s) return;
    free(s->f); free(s->ftmp);
    for (int k = 0; k < 3; ++k) { free(s->pos[k]); free(s->vel[k]); }
    free(s->cell_of); free(s->count); free(s->start); free(s->order);
    free(s->vcm); free(s->ufine); free(s->unode); free(s->acc); free(s->prof); free(s->fbu);
    free(s->tnode); free(s->tfine);
    free(s->scratch);
    free(s);
}

/* Slab and cell geometry of the parameter set (no arrays). */
static void setup_geometry(orc_state* s) {
    const orc_params* p = &s->p;
    int r = p->refine, d = p->dim;
    s->R = (p->yhi - p->ylo) * r;
    s->Cx = p->nx * r;
    s->Cz = (d == 3) ? p->nz * r : 1;
    s->ywrap = (!p->walls_y && p->ylo == 0 && p->yhi == p->ny && p->buf_lo == 0 && p->buf_hi == 0);
    s->CyB = s->ywrap ? s->R : s->R + 1;
    s->bot_wall = p->walls_y && p->ylo == 0;
    s->top_wall = p->walls_y && p->yhi == p->ny;
    s->ncells = s->Cx * s->CyB * s->Cz;
    s->Np = (int64_t)s->Cx * s->R * s->Cz * p->ppc;
    s->a = 1.0 / r;
    s->dt = 1.0 / p->substeps;
    double alpha = p->alpha_deg * 3.141592653589793 / 180.0;
    s->cos_a = cos(alpha);
    s->sin_a = sin(alpha);
}

int orc_create_geometry(const orc_params* p, orc_state** out) {
    *out = NULL;
    int e = validate(p);
    if (e) return e;
    if (!p->mpcd) return 1;
    orc_state* s = (orc_state*)calloc(1, sizeof(orc_state));
    if (!s) return 2;
    s->p = *p;
    s->Q = orc_lattice(p->dim, s->c, s->w, s->opp);
    s->N = (int64_t)p->nx * p->ny * p->nz;
    setup_geometry(s);
    *out = s;
    return 0;
}

int orc_create(const orc_params* p, orc_state** out) {
    *out = NULL;
    int e = validate(p);
    if (e) return e;
    orc_state* s = (orc_state*)calloc(1, sizeof(orc_state));
    if (!s) return 2;
    s->p = *p;
    s->Q = orc_lattice(p->dim, s->c, s->w, s->opp);
    s->N = (int64_t)p->nx * p->ny * p->nz;
    s->f = (double*)calloc((size_t)(s->Q * s->N), sizeof(double));
    s->ftmp = (double*)calloc((size_t)(s->Q * s->N), sizeof(double));
    s->unode = (double*)calloc((size_t)(3 * s->N), sizeof(double));
    if (!s->f || !s->ftmp || !s->unode) { orc_destroy(s); return 2; }
    /* LB initial state: equilibrium at rho0 and the initial velocity field
     * (physical velocity = first moment + g/2). */
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                double u[3] = {0.0, 0.0, 0.0}, feq[19];
                for (int k = 0; k < 3; ++k) {
                    double u0 = p->init_flow ? poiseuille(p, p->g[k], y + 0.5) : 0.0;
                    u[k] = u0 - 0.5 * p->g[k];
                }
                orc_feq(p->dim, p->rho0, u, feq);
                int64_t n = node_index(s, x, y, z);
                for (int i = 0; i < s->Q; ++i) s->f[i * s->N + n] = feq[i];
            }

    if (p->mpcd) {
        int r = p->refine, d = p->dim;
        setup_geometry(s);
        for (int k = 0; k < 3; ++k) {
            s->pos[k] = (double*)calloc((size_t)s->Np, sizeof(double));
            s->vel[k] = (double*)calloc((size_t)s->Np, sizeof(double));
        }
        s->cell_of = (int32_t*)calloc((size_t)s->Np, sizeof(int32_t));
        s->order = (int32_t*)calloc((size_t)s->Np, sizeof(int32_t));
        s->count = (int32_t*)calloc((size_t)s->ncells, sizeof(int32_t));
        s->start = (int32_t*)calloc((size_t)s->ncells, sizeof(int32_t));
        s->vcm = (double*)calloc((size_t)(3 * s->ncells), sizeof(double));
        s->ufine = (double*)calloc((size_t)(3 * s->Cx * s->R * s->Cz), sizeof(double));
        s->tnode = (double*)calloc((size_t)(6 * s->N), sizeof(double));
        s->tfine = (double*)calloc((size_t)(6 * s->Cx * s->R * s->Cz), sizeof(double));
        s->acc = (double*)calloc((size_t)(4 * p->nx * s->R * p->nz), sizeof(double));
        s->prof = (double*)calloc((size_t)(4 * s->R), sizeof(double));
        s->fbu = (double*)calloc((size_t)(3 * p->nx * (p->yhi - p->ylo) * p->nz), sizeof(double));
        s->scratch = (double*)malloc(sizeof(double) * 3 * 4096);
        for (int k = 0; k < 3; ++k)
            if (!s->pos[k] || !s->vel[k]) { orc_destroy(s); return 2; }
        if (!s->cell_of || !s->order || !s->count || !s->start || !s->vcm || !s->ufine ||
            !s->acc || !s->prof || !s->scratch || !s->tnode || !s->tfine || !s->fbu) {
            orc_destroy(s);
            return 2;
        }
        /* the running mean of the feedback starts at the initial velocity of
         * every slab node */
        for (int z = 0; z < p->nz; ++z)
            for (int y = p->ylo; y < p->yhi; ++y)
                for (int x = 0; x < p->nx; ++x)
                    for (int k = 0; k < 3; ++k)
                        s->fbu[3 * (((int64_t)z * (p->yhi - p->ylo) + (y - p->ylo)) * p->nx + x) + k] =
                            p->init_flow ? poiseuille(p, p->g[k], y + 0.5) : 0.0;
        /* READING: exactly ppc particles in every fine cell, uniform inside the
         * cell, ids in cell order; Maxwell-Boltzmann velocities of variance
         * kT/m about the initial flow. */
        double sd = sqrt(p->kT / p->mass);
        for (int K = 0; K < s->Cz; ++K)
            for (int J = 0; J < s->R; ++J)
                for (int I = 0; I < s->Cx; ++I) {
                    int64_t cl = ((int64_t)K * s->R + J) * s->Cx + I;
                    for (int q = 0; q < p->ppc; ++q) {
                        int64_t id = cl * p->ppc + q;
                        double u[4], z[3];
                        rng_uniforms4(p, (uint32_t)id, 0, 0, P_INIT_POS, u);
                        double x = (I + u[0]) / r;
                        double y = p->ylo + (J + u[1]) / r;
                        double zz = (d == 3) ? (K + u[2]) / r : 0.0;
                        s->pos[0][id] = st(s, x);
                        s->pos[1][id] = st(s, y);
                        s->pos[2][id] = st(s, zz);
                        rng_normals(p, (uint32_t)id, 0, 0, P_INIT_VEL, z);
                        for (int k = 0; k < d; ++k) {
                            double u0 = p->init_flow ? poiseuille(p, p->g[k], y) : 0.0;
                            s->vel[k][id] = st(s, u0 + sd * z[k]);
                        }
                    }
                }
    }
    *out = s;
    return 0;
}

int64_t orc_num_particles(const orc_state* s) { return s->Np; }
int32_t orc_num_cells(const orc_state* s) { return s->ncells; }
int32_t orc_num_fine_rows(const orc_state* s) { return s->R; }
int64_t orc_lb_step_count(const orc_state* s) { return s->t; }

/* ------------------------------------------------------------------------
 * LB step (Eq. 1, Alg. 1: collision then streaming).  Streaming pushes the
 * post-collision population along c_i; periodic in x and z (and y without
 * walls); half-way bounce-back on links crossing y = 0 or y = ny (the
 * second-order no-slip scheme of the results section).
 * ---------------------------------------------------------------------- */
static void lb_collide_stream(orc_state* s) {
    const orc_params* p = &s->p;
    double fn[19];
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t n = node_index(s, x, y, z);
                for (int i = 0; i < s->Q; ++i) fn[i] = s->f[i * s->N + n];
                orc_collide_node(p->dim, p->tau, p->g, fn);
                for (int i = 0; i < s->Q; ++i) {
                    int yd = y + s->c[3 * i + 1];
                    if (p->walls_y && (yd < 0 || yd >= p->ny)) {
                        s->ftmp[s->opp[i] * s->N + n] = fn[i];
                        continue;
                    }
                    int xd = (x + s->c[3 * i] + p->nx) % p->nx;
                    yd = (yd + p->ny) % p->ny;
                    int zd = (z + s->c[3 * i + 2] + p->nz) % p->nz;
                    s->ftmp[i * s->N + node_index(s, xd, yd, zd)] = fn[i];
                }
            }
    double* tmp = s->f;
    s->f = s->ftmp;
    s->ftmp = tmp;
}

/* density and physical velocity (first moment / rho + g/2) of one node */
static void node_moments(const orc_state* s, int64_t n, double* rho, double u[3]) {
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < s->Q; ++i) {
        double fi = s->f[i * s->N + n];
        r += fi;
        for (int k = 0; k < 3; ++k) j[k] += fi * s->c[3 * i + k];
    }
    *rho = r;
    for (int k = 0; k < 3; ++k) u[k] = j[k] / r + 0.5 * s->p.g[k];
}

/* READING (feedback, not in the paper, which couples one way only): at LB
 * nodes of the slab that are not buffer nodes, replace the post-stream
 * populations by the equilibrium at the LB density and at a time average of
 * the MPCD velocity sampled over the node, so that the node's physical
 * velocity equals that average.  The average is a running mean over the LB
 * steps: every LB step that sampled the node moves it towards the step's
 * sample mean by the weight 1/W (W = fb_window LB steps, 50 by default); it
 * starts at the node's initial velocity.  The paper averages MPCD profiles
 * over many samples because a single sample is dominated by thermal noise
 * (Sec. 3.1); a node of r^d cells holds a few hundred particles, whose mean
 * carries a noise of the size of the flow itself, and projecting it
 * instantaneously (W = 1) drives the LB unstable. */
#define FB_WINDOW_DEFAULT 50
static void feedback_override(orc_state* s) {
    const orc_params* p = &s->p;
    int r = p->refine;
    const double lam = 1.0 / (double)(p->fb_window > 0 ? p->fb_window : FB_WINDOW_DEFAULT);
    for (int z = 0; z < p->nz; ++z)
        for (int y = p->ylo + p->buf_lo; y < p->yhi - p->buf_hi; ++y)
            for (int x = 0; x < p->nx; ++x) {
                double cnt = 0.0, sv[3] = {0.0, 0.0, 0.0};
                for (int J = (y - p->ylo) * r; J < (y - p->ylo + 1) * r; ++J) {
                    const double* a = s->acc + 4 * (((int64_t)z * s->R + J) * p->nx + x);
                    cnt += a[0];
                    for (int k = 0; k < 3; ++k) sv[k] += a[1 + k];
                }
                if (cnt <= 0.0) continue;
                int64_t n = node_index(s, x, y, z);
                double* e = s->fbu + 3 * (((int64_t)z * (p->yhi - p->ylo) + (y - p->ylo)) * p->nx + x);
                double rho = 0.0;
                for (int i = 0; i < s->Q; ++i) rho += s->f[i * s->N + n];
                double u[3], feq[19];
                for (int k = 0; k < 3; ++k) {
                    e[k] = (1.0 - lam) * e[k] + lam * (sv[k] / cnt);
                    u[k] = e[k] - 0.5 * p->g[k];
                }
                orc_feq(p->dim, rho, u, feq);
                for (int i = 0; i < s->Q; ++i) s->f[i * s->N + n] = feq[i];
            }
}

/* Bilinear (2D) / trilinear (3D) interpolation of the node-centred LB
 * velocity to the centres of the buffer fine cells (Alg. 2).  READING: next
 * to a wall the missing node is the wall itself with zero velocity. */
static void interp_axis(int L, int periodic, double X, int* i0, int* i1, double* w0, double* w1) {
    double xs = X - 0.5;
    double fl = floor(xs);
    int j0 = (int)fl;
    double wx = xs - fl;
    int j1 = j0 + 1;
    if (periodic) {
        j0 = (j0 % L + L) % L;
        j1 = (j1 % L + L) % L;
        *i0 = j0; *i1 = j1; *w0 = 1.0 - wx; *w1 = wx;
        return;
    }
    if (j0 < 0) {            /* between the wall at 0 and node 0 */
        *i0 = -1; *i1 = 0; *w0 = 0.0; *w1 = 2.0 * X;
    } else if (j1 > L - 1) { /* between node L-1 and the wall at L */
        *i0 = L - 1; *i1 = -1; *w0 = 2.0 * (L - X); *w1 = 0.0;
    } else {
        *i0 = j0; *i1 = j1; *w0 = 1.0 - wx; *w1 = wx;
    }
}

static void interpolate_from(const orc_state* s, int ncomp, const double* unode, double* ufine);

/* Chapman-Enskog tensor of node n (READING): the strain rate of the BGK
 * lattice from the non-equilibrium second moment of the post-stream
 * populations, S = -(sum f c c - rho cs2 I - rho u u) / (2 rho cs2 tau) with
 * the physical velocity u, its deviatoric part over the d axes, scaled by
 * nu_x m / kT (nu_x of orc_ce_nu).  T[6] = (xx, yy, zz, xy, xz, yz); zero components in 2D. */
static void node_ce_tensor(const orc_state* s, int64_t n, double T[6]) {
    static const int ab[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
    const orc_params* p = &s->p;
    const double cs2 = 1.0 / 3.0;
    double rho, u[3];
    node_moments(s, n, &rho, u);
    double S[6];
    for (int m = 0; m < 6; ++m) {
        int a = ab[m][0], b = ab[m][1];
        double pi = 0.0;
        for (int i = 0; i < s->Q; ++i) pi += s->f[i * s->N + n] * (double)(s->c[3 * i + a] * s->c[3 * i + b]);
        double pneq = pi - (a == b ? rho * cs2 : 0.0) - rho * u[a] * u[b];
        S[m] = -pneq / (2.0 * rho * cs2 * p->tau);
    }
    if (p->dim == 2) S[2] = S[4] = S[5] = 0.0;
    double tr = (S[0] + S[1] + S[2]) / (double)p->dim;
    S[0] -= tr;
    S[1] -= tr;
    if (p->dim == 3) S[2] -= tr;
    double c = orc_ce_nu(p) * p->mass / p->kT;
    for (int m = 0; m < 6; ++m) T[m] = c * S[m];
}

static void interpolate_buffers(orc_state* s) {
    const orc_params* p = &s->p;
    const int by0 = p->ylo > 0 ? p->ylo - 1 : 0, by1 = p->yhi < p->ny ? p->yhi + 1 : p->ny;
    for (int64_t n = 0; n < s->N; ++n) {
        double rho, u[3];
        node_moments(s, n, &rho, u);
        for (int k = 0; k < 3; ++k) s->unode[k * s->N + n] = u[k];
        /* READING: a node of the rows the coupling reads (the slab and one
         * row either side) with non-positive or non-finite density or a
         * non-finite velocity is an invalid state */
        const int y = (int)((n / p->nx) % p->ny);
        if (y >= by0 && y < by1 && !(rho > 0.0 && isfinite(rho) && isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2])))
            s->bad++;
    }
    interpolate_from(s, s->p.dim, s->unode, s->ufine);
    if (s->p.reinject) {
        for (int64_t n = 0; n < s->N; ++n) {
            double T[6];
            node_ce_tensor(s, n, T);
            for (int m = 0; m < 6; ++m) s->tnode[m * s->N + n] = T[m];
        }
        interpolate_from(s, 6, s->tnode, s->tfine);
    }
}

/* buffer fine-cell values ufine[ncomp][Cz][R][Cx] of the node fields unode[ncomp][N]
 * (the velocity, ncomp = d, or the Chapman-Enskog tensor, ncomp = 6) */
static void interpolate_from(const orc_state* s, int ncomp, const double* unode, double* ufine) {
    const orc_params* p = &s->p;
    int r = p->refine;
    int64_t nf = (int64_t)s->Cx * s->R * s->Cz;
    for (int K = 0; K < s->Cz; ++K)
        for (int J = 0; J < s->R; ++J) {
            int inbuf = (J < p->buf_lo * r) || (J >= s->R - p->buf_hi * r);
            if (!inbuf) continue;
            for (int I = 0; I < s->Cx; ++I) {
                double X = (I + 0.5) / r, Y = p->ylo + (J + 0.5) / r;
                double Z = (p->dim == 3) ? (K + 0.5) / r : 0.5;
                int ix[2], iy[2], iz[2];
                double wx[2], wy[2], wz[2];
                interp_axis(p->nx, 1, X, &ix[0], &ix[1], &wx[0], &wx[1]);
                interp_axis(p->ny, !p->walls_y, Y, &iy[0], &iy[1], &wy[0], &wy[1]);
                if (p->dim == 3)
                    interp_axis(p->nz, 1, Z, &iz[0], &iz[1], &wz[0], &wz[1]);
                else {
                    iz[0] = 0; iz[1] = 0; wz[0] = 1.0; wz[1] = 0.0;
                }
                for (int k = 0; k < ncomp; ++k) {
                    double val[2] = {0.0, 0.0};
                    for (int c = 0; c < (p->dim == 3 ? 2 : 1); ++c) {
                        double row[2];
                        for (int b = 0; b < 2; ++b) {
                            double u0 = (iy[b] < 0) ? 0.0 : unode[k * s->N + node_index(s, ix[0], iy[b], iz[c])];
                            double u1 = (iy[b] < 0) ? 0.0 : unode[k * s->N + node_index(s, ix[1], iy[b], iz[c])];
                            row[b] = wx[0] * u0 + wx[1] * u1;
                        }
                        val[c] = wy[0] * row[0] + wy[1] * row[1];
                    }
                    double v = (p->dim == 3) ? wz[0] * val[0] + wz[1] * val[1] : val[0];
                    ufine[k * nf + ((int64_t)K * s->R + J) * s->Cx + I] = v;
                }
            }
        }
}

/* ------------------------------------------------------------------------
 * MPCD step pieces
 * ---------------------------------------------------------------------- */
static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* fine row of a particle (y relative to the slab bottom times r) */
static int fine_row(const orc_state* s, double y) {
    return clampi((int)floor((y - s->p.ylo) * s->p.refine), 0, s->R - 1);
}

/* Exchange step (Alg. 1): particles whose unshifted position lies in a
 * buffer get a fresh velocity from the Maxwell-Boltzmann distribution about
 * the interpolated LB velocity; variance kT/m per component. */
/* fine cell (unshifted) of a position; -1 when it is not a buffer cell */
static int64_t buffer_cell(const orc_state* s, const double r[3]) {
    const orc_params* p = &s->p;
    int rf = p->refine;
    int J = fine_row(s, r[1]);
    int inbuf = (J < p->buf_lo * rf) || (J >= s->R - p->buf_hi * rf);
    if (!inbuf) return -1;
    int I = clampi((int)floor(r[0] * rf), 0, s->Cx - 1);
    int K = (p->dim == 3) ? clampi((int)floor(r[2] * rf), 0, s->Cz - 1) : 0;
    return ((int64_t)K * s->R + J) * s->Cx + I;
}

/* redraw one buffer particle about the LB velocity u of its fine cell; with
 * the Chapman-Enskog exchange T is the cell's tensor (NULL otherwise) */
static void reinject_one(const orc_state* s, uint32_t id, uint32_t t, uint32_t sub, const double u[3],
                         const double* T, double v[3]) {
    const orc_params* p = &s->p;
    double sd = sqrt(p->kT / p->mass);
    double z[3];
    if (p->reinject && T)
        orc_ce_normals(p, id, t, sub, T, z);
    else if (p->part_fp32)
        rng_normals32(p, id, t, sub, P_REINJ, z);
    else
        rng_normals(p, id, t, sub, P_REINJ, z);
    for (int d = 0; d < p->dim; ++d) v[d] = st(s, u[d] + sd * z[d]);
}

static void reinject(orc_state* s, uint32_t t, uint32_t sub) {
    int64_t nf = (int64_t)s->Cx * s->R * s->Cz;
    for (int64_t k = 0; k < s->Np; ++k) {
        double r[3] = {s->pos[0][k], s->pos[1][k], s->pos[2][k]};
        int64_t fc = buffer_cell(s, r);
        if (fc < 0) continue;
        double u[3] = {0.0, 0.0, 0.0}, v[3], T[6];
        for (int d = 0; d < s->p.dim; ++d) u[d] = s->ufine[d * nf + fc];
        for (int m = 0; m < 6; ++m) T[m] = s->tfine[m * nf + fc];
        reinject_one(s, (uint32_t)k, t, sub, u, T, v);
        for (int d = 0; d < s->p.dim; ++d) s->vel[d][k] = v[d];
    }
}

static double wrap_periodic(const orc_state* s, double x, double lo, double L) {
    if (s->p.part_fp32) {
        float xf = (float)x, lf = (float)lo, Lf = (float)L;
        if (xf < lf) xf = xf + Lf;
        if (xf >= lf + Lf) xf = xf - Lf;
        return (double)xf;
    }
    if (x < lo) x = x + L;
    if (x >= lo + L) x = x - L;
    return x;
}

/* Ballistic streaming, Eq. 3, with the body force as a constant acceleration
 * over the step (READING): r += (v + g dt/2) dt, v += g dt.  Boundaries:
 * periodic along x and z; at a wall the particle is bounced back (velocity
 * reversed at the crossing instant, remaining flight continued); at an
 * LB-facing slab face the particle is re-wrapped periodically across the
 * slab (paper: no particles are injected, mass is conserved), or, when the
 * opposite face is a wall, reflected specularly. */
static int stream_one(const orc_state* s, double r[3], double v[3]) {
    const orc_params* p = &s->p;
    double dt = s->dt;
    double r0[3], v0[3];
    for (int d = 0; d < 3; ++d) { r0[d] = r[d]; v0[d] = v[d]; }
    double r1[3] = {r0[0], r0[1], r0[2]}, v1[3] = {v0[0], v0[1], v0[2]};
    for (int d = 0; d < p->dim; ++d) {
        double gh = 0.5 * p->g[d] * dt, gdt = p->g[d] * dt;
        if (p->part_fp32) {
            float vh = (float)v0[d] + (float)gh;
            r1[d] = (double)fmaf(vh, (float)dt, (float)r0[d]);
            v1[d] = (double)((float)v0[d] + (float)gdt);
        } else {
            double vh = v0[d] + gh;
            r1[d] = fma(vh, dt, r0[d]);
            v1[d] = v0[d] + gdt;
        }
    }
    double ylo = p->ylo, yhi = p->yhi;
    int below = r1[1] < ylo, above = r1[1] >= yhi;
    if (!s->ywrap && (below || above)) {
        int wall = below ? s->bot_wall : s->top_wall;
        double Yw = below ? ylo : yhi;
        if (wall) {
            /* crossing instant from the straight y flight (g_y = 0) */
            double vhy = v0[1];
            double tc = (Yw - r0[1]) / vhy;
            double tr = dt - tc;
            for (int d = 0; d < p->dim; ++d) {
                double rc = r0[d] + (v0[d] + 0.5 * p->g[d] * tc) * tc;
                double vc = v0[d] + p->g[d] * tc;
                if (d == 1) rc = Yw;
                double vr = -vc;
                r1[d] = rc + (vr + 0.5 * p->g[d] * tr) * tr;
                v1[d] = vr + p->g[d] * tr;
            }
        } else if (s->bot_wall || s->top_wall) {
            r1[1] = 2.0 * Yw - r1[1];
            v1[1] = -v1[1];
        } else {
            r1[1] = wrap_periodic(s, r1[1], ylo, yhi - ylo);
        }
        for (int d = 0; d < p->dim; ++d) { r1[d] = st(s, r1[d]); v1[d] = st(s, v1[d]); }
        /* keep the particle inside [ylo, yhi) after a reflection */
        if (r1[1] < ylo) r1[1] = ylo;
        if (r1[1] >= yhi)
            r1[1] = p->part_fp32 ? (double)nextafterf((float)yhi, (float)ylo) : nextafter(yhi, ylo);
    } else if (s->ywrap) {
        r1[1] = wrap_periodic(s, r1[1], 0.0, (double)p->ny);
    }
    r1[0] = wrap_periodic(s, r1[0], 0.0, (double)p->nx);
    if (p->dim == 3) r1[2] = wrap_periodic(s, r1[2], 0.0, (double)p->nz);
    /* READING (the paper has no such case): a particle that left the domain
     * by more than one period in one MPCD step, or whose position or velocity
     * is not finite, is an invalid state of the run (a diverged LB field
     * handing out such velocities, say).  It is parked at the lower corner of
     * the slab with zero velocity, so that every index derived from it stays
     * in range, and the step reports the state as invalid. */
    int bad = !(r1[0] >= 0.0 && r1[0] < (double)p->nx);
    if (p->dim == 3) bad |= !(r1[2] >= 0.0 && r1[2] < (double)p->nz);
    bad |= !(r1[1] >= (s->ywrap ? 0.0 : ylo) && r1[1] < (s->ywrap ? (double)p->ny : yhi));
    for (int d = 0; d < p->dim; ++d) bad |= !isfinite(v1[d]);
    if (bad) {
        for (int d = 0; d < 3; ++d) v1[d] = 0.0;
        r1[0] = 0.0;
        r1[1] = s->ywrap ? 0.0 : ylo;
        r1[2] = 0.0;
    }
    for (int d = 0; d < p->dim; ++d) { r[d] = r1[d]; v[d] = v1[d]; }
    return bad;
}

static void stream_particle(orc_state* s, int64_t k) {
    double r[3], v[3];
    for (int d = 0; d < 3; ++d) { r[d] = s->pos[d][k]; v[d] = s->vel[d][k]; }
    s->bad += stream_one(s, r, v);
    for (int d = 0; d < s->p.dim; ++d) { s->pos[d][k] = r[d]; s->vel[d][k] = v[d]; }
}

/* READING: the sample instant is right after streaming.  The per-LB-step
 * accumulators feed the feedback, which projects the interior slab nodes
 * only, so particles in buffer rows are not sampled for it; while sampling is
 * on every sample also adds to the time-averaged profile of its fine row,
 * buffers included (the paper averages the profiles over samples to
 * suppress the particle noise, Sec. 3.1). */
static void sample_particle(orc_state* s, int64_t k) {
    const orc_params* p = &s->p;
    int ix = clampi((int)floor(s->pos[0][k]), 0, p->nx - 1);
    int J = fine_row(s, s->pos[1][k]);
    int iz = (p->dim == 3) ? clampi((int)floor(s->pos[2][k]), 0, p->nz - 1) : 0;
    const int r = p->refine;
    if (J >= p->buf_lo * r && J < s->R - p->buf_hi * r) {
        double* a = s->acc + 4 * (((int64_t)iz * s->R + J) * p->nx + ix);
        a[0] += 1.0;
        for (int d = 0; d < p->dim; ++d) a[1 + d] += s->vel[d][k];
    }
    if (s->sampling) {
        double* q = s->prof + 4 * J;
        q[0] += 1.0;
        for (int d = 0; d < p->dim; ++d) q[1 + d] += s->vel[d][k];
    }
}

/* READING: random grid shift (Ihle-Kroll) drawn once per MPCD step,
 * uniform in [0,a) per axis. */
static void draw_shift(const orc_state* s, uint32_t t, uint32_t sub, double sh[3]) {
    double u[4];
    rng_uniforms4(&s->p, 0, t, sub, P_SHIFT, u);
    for (int d = 0; d < 3; ++d) {
        double v = (s->p.grid_shift && d < s->p.dim) ? u[d] * s->a : 0.0;
        sh[d] = st(s, v);
    }
}

/* one binning coordinate: floor((x - lo + shift) * r) in the store precision */
static int bin_coord(const orc_state* s, double x, double lo, double sh) {
    if (s->p.part_fp32) {
        float t = (float)x - (float)lo;
        t = t + (float)sh;
        t = t * (float)s->p.refine;
        return (int)floorf(t);
    }
    double t = x - lo;
    t = t + sh;
    t = t * (double)s->p.refine;
    return (int)floor(t);
}

static int32_t cell_of_pos(const orc_state* s, const double r[3], const double sh[3]) {
    const orc_params* p = &s->p;
    int ix = bin_coord(s, r[0], 0.0, sh[0]);
    if (ix >= s->Cx) ix -= s->Cx;
    int iy = bin_coord(s, r[1], (double)p->ylo, sh[1]);
    if (s->ywrap && iy >= s->R) iy -= s->R;
    /* a binary32 sum y - ylo + shift can round up to the slab height plus
     * a full cell; the particle belongs to the last row of the grid */
    if (iy > s->CyB - 1) iy = s->CyB - 1;
    int iz = 0;
    if (p->dim == 3) {
        iz = bin_coord(s, r[2], 0.0, sh[2]);
        if (iz >= s->Cz) iz -= s->Cz;
    }
    return (int32_t)(ix + s->Cx * (iy + s->CyB * iz));
}

static int32_t particle_cell(const orc_state* s, int64_t k, const double sh[3]) {
    double r[3] = {s->pos[0][k], s->pos[1][k], s->pos[2][k]};
    return cell_of_pos(s, r, sh);
}

/* Collision of every cell: SRD (Eq. 4; READING: 2D sign and 3D axis per
 * cell and step from the ROT stream) or MPCD-AT (Eq. 6); cells cut by a wall
 * get virtual particles up to the nominal occupancy. */
/* Collision of the n particles (ids[n]) of cell c: v is [dim][n] (unit-mass
 * velocities, updated in place and rounded to the store precision); vcm
 * receives the centre-of-mass velocity including virtual wall particles. */
static void collide_one(const orc_state* s, int32_t c, uint32_t t, uint32_t sub, const double sh[3], int32_t n,
                        const int32_t* ids, double* v, double vcm_out[3]) {
    const orc_params* p = &s->p;
    int d = p->dim;
    int iy = (c / s->Cx) % s->CyB;
    /* READING (the wall rule of Lamura et al., which the paper cites): a
     * wall-cut cell holding n < N0 particles is filled up with N0 - n virtual
     * particles at rest in the wall frame, each with a Maxwell-Boltzmann
     * velocity of variance kT/m per component.  Only their velocity sum
     * enters the centre of mass: a normal deviate of variance
     * (N0 - n) kT/m per component, i.e. momentum sqrt((N0 - n) m kT) xi.
     * The collision routines work with unit-mass velocity sums, so this sum
     * is passed as is, with the mass N0 - n in particle units. */
    double pvu[3] = {0.0, 0.0, 0.0}, mv = 0.0;
    int cut = (sh[1] > 0.0) && ((s->bot_wall && iy == 0) || (s->top_wall && iy == s->R));
    if (cut && n < p->ppc) {
        double z[3];
        rng_normals(p, (uint32_t)c, t, sub, P_WALL, z);
        int nv = p->ppc - n;
        double sdv = sqrt((double)nv * p->kT / p->mass);
        for (int k = 0; k < d; ++k) pvu[k] = sdv * z[k];
        mv = (double)nv;
    }
    if (p->collision == 1) {
        /* MPCD-AT: one Gaussian velocity per particle (READING: variance
         * kT/m per component, as for the exchange step), keyed by the
         * particle's id and the collision's MPCD step, drawn in binary32 for
         * binary32 particles (READING above); stored in the particle
         * precision before use */
        double* vr = (double*)malloc(sizeof(double) * 3 * (size_t)n);
        const double sd = sqrt(p->kT / p->mass);
        for (int i = 0; i < n; ++i) {
            double z[3];
            if (p->part_fp32)
                rng_normals32(p, (uint32_t)ids[i], t, sub, P_AT, z);
            else
                rng_normals(p, (uint32_t)ids[i], t, sub, P_AT, z);
            for (int k = 0; k < d; ++k) vr[k * n + i] = st(s, sd * z[k]);
        }
        double vc[3] = {0.0, 0.0, 0.0};
        orc_at_collide(d, n, v, vr, pvu, mv, vc);
        free(vr);
        for (int k = 0; k < 3; ++k) vcm_out[k] = vc[k];
        for (int i = 0; i < d * n; ++i) v[i] = st(s, v[i]);
        return;
    }
    uint32_t w[4];
    rng_block(p, (uint32_t)c, t, sub, P_ROT, 0, w);
    double sign2d = (w[0] & 1u) ? 1.0 : -1.0;
    double axis[3] = {0.0, 0.0, 1.0};
    if (d == 3) {
        double u0 = orc_u01(w[0], w[1]), u1 = orc_u01(w[2], w[3]);
        double nz = 2.0 * u0 - 1.0, phi = 6.283185307179586 * u1;
        double sxy = sqrt(fmax(0.0, 1.0 - nz * nz));
        axis[0] = sxy * cos(phi);
        axis[1] = sxy * sin(phi);
        axis[2] = nz;
    }
    double vc[3] = {0.0, 0.0, 0.0};
    orc_srd_rotate(d, n, v, s->cos_a, s->sin_a, sign2d, axis, pvu, mv, vc);
    for (int k = 0; k < 3; ++k) vcm_out[k] = vc[k];
    for (int i = 0; i < d * n; ++i) v[i] = st(s, v[i]);
}

static void collide_cells(orc_state* s, uint32_t t, uint32_t sub, const double sh[3]) {
    const orc_params* p = &s->p;
    int d = p->dim;
    for (int32_t c = 0; c < s->ncells; ++c) {
        int32_t n = s->count[c];
        for (int k = 0; k < 3; ++k) s->vcm[k * s->ncells + c] = 0.0;
        if (n == 0) continue;
        double* v = s->scratch;
        if (n > 4096) v = (double*)malloc(sizeof(double) * 3 * (size_t)n);
        for (int i = 0; i < n; ++i) {
            int32_t id = s->order[s->start[c] + i];
            for (int k = 0; k < d; ++k) v[k * n + i] = s->vel[k][id];
        }
        double vc[3];
        collide_one(s, c, t, sub, sh, n, s->order + s->start[c], v, vc);
        for (int k = 0; k < d; ++k) s->vcm[k * s->ncells + c] = vc[k];
        for (int i = 0; i < n; ++i) {
            int32_t id = s->order[s->start[c] + i];
            for (int k = 0; k < d; ++k) s->vel[k][id] = v[k * n + i];
        }
        if (v != s->scratch) free(v);
    }
}

static void mpcd_substep(orc_state* s, uint32_t t, uint32_t sub) {
    /* READING: one sample per LB step, right after the streaming of its last
     * MPCD step */
    const int sample = (int)sub == s->p.substeps - 1;
    reinject(s, t, sub);
    for (int64_t k = 0; k < s->Np; ++k) {
        stream_particle(s, k);
        if (sample) sample_particle(s, k);
    }
    double sh[3];
    draw_shift(s, t, sub, sh);
    for (int d = 0; d < 3; ++d) s->shift[d] = sh[d];
    for (int64_t k = 0; k < s->Np; ++k) s->cell_of[k] = particle_cell(s, k, sh);
    orc_counting_sort((int32_t)s->Np, s->cell_of, s->ncells, s->count, s->start, s->order);
    collide_cells(s, t, sub, sh);
}

int orc_step(orc_state* s, int32_t n_lb_steps) {
    const orc_params* p = &s->p;
    for (int32_t it = 0; it < n_lb_steps; ++it) {
        s->bad = 0;
        lb_collide_stream(s);
        if (p->mpcd) {
            if (p->feedback) feedback_override(s);
            memset(s->acc, 0, sizeof(double) * 4 * (size_t)p->nx * s->R * p->nz);
            interpolate_buffers(s);
            for (int sub = 0; sub < p->substeps; ++sub) mpcd_substep(s, (uint32_t)s->t, (uint32_t)sub);
            if (s->sampling) s->prof_steps++;
        }
        s->t++;
        if (s->bad) return 5; /* invalid state (non-finite or runaway particles or band nodes) */
    }
    return 0;
}

void orc_sample(orc_state* s, int32_t mode) {
    if (mode == 1) {
        if (s->prof) memset(s->prof, 0, sizeof(double) * 4 * (size_t)s->R);
        s->prof_steps = 0;
        s->sampling = 1;
    } else {
        s->sampling = 0;
    }
}

void orc_get_f(const orc_state* s, double* f) { memcpy(f, s->f, sizeof(double) * (size_t)(s->Q * s->N)); }
void orc_set_f(orc_state* s, const double* f) { memcpy(s->f, f, sizeof(double) * (size_t)(s->Q * s->N)); }

void orc_get_fstar(const orc_state* s, double* out) {
    double fn[19];
    for (int64_t n = 0; n < s->N; ++n) {
        for (int i = 0; i < s->Q; ++i) fn[i] = s->f[i * s->N + n];
        orc_collide_node(s->p.dim, s->p.tau, s->p.g, fn);
        for (int i = 0; i < s->Q; ++i) out[i * s->N + n] = fn[i];
    }
}

/* Hydrodynamic moments of the post-stream populations (Sec. 2.1):
 * rho = sum f, rho u = sum f c (+ rho g/2, Guo), Pi = sum f (c c - cs2 I). */
void orc_get_moments(const orc_state* s, double* rho, double* u, double* pi) {
    for (int64_t n = 0; n < s->N; ++n) {
        double r, uu[3];
        node_moments(s, n, &r, uu);
        if (rho) rho[n] = r;
        if (u)
            for (int k = 0; k < 3; ++k) u[k * s->N + n] = uu[k];
        if (pi) {
            static const int ab[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
            for (int m = 0; m < 6; ++m) {
                int a = ab[m][0], b = ab[m][1];
                double acc = 0.0;
                for (int i = 0; i < s->Q; ++i) {
                    double cc = (double)(s->c[3 * i + a] * s->c[3 * i + b]) - (a == b ? 1.0 / 3.0 : 0.0);
                    acc += s->f[i * s->N + n] * cc;
                }
                pi[m * s->N + n] = acc;
            }
        }
    }
}

void orc_get_particles(const orc_state* s, double* pos, double* vel) {
    for (int d = 0; d < s->p.dim; ++d) {
        if (pos) memcpy(pos + d * s->Np, s->pos[d], sizeof(double) * (size_t)s->Np);
        if (vel) memcpy(vel + d * s->Np, s->vel[d], sizeof(double) * (size_t)s->Np);
    }
}

void orc_set_particles(orc_state* s, const double* pos, const double* vel) {
    for (int d = 0; d < s->p.dim; ++d) {
        for (int64_t k = 0; k < s->Np; ++k) {
            if (pos) s->pos[d][k] = st(s, pos[d * s->Np + k]);
            if (vel) s->vel[d][k] = st(s, vel[d * s->Np + k]);
        }
    }
}

void orc_get_binning(const orc_state* s, int32_t* cell_of, int32_t* count, int32_t* start,
                     int32_t* order, double* vcm) {
    if (cell_of) memcpy(cell_of, s->cell_of, sizeof(int32_t) * (size_t)s->Np);
    if (count) memcpy(count, s->count, sizeof(int32_t) * (size_t)s->ncells);
    if (start) memcpy(start, s->start, sizeof(int32_t) * (size_t)s->ncells);
    if (order) memcpy(order, s->order, sizeof(int32_t) * (size_t)s->Np);
    if (vcm) memcpy(vcm, s->vcm, sizeof(double) * 3 * (size_t)s->ncells);
}

void orc_get_ufine(const orc_state* s, double* ufine) {
    memcpy(ufine, s->ufine, sizeof(double) * 3 * (size_t)s->Cx * s->R * s->Cz);
}

void orc_get_profile(const orc_state* s, double* acc, int64_t* n) {
    if (acc) memcpy(acc, s->prof, sizeof(double) * 4 * (size_t)s->R);
    if (n) *n = s->prof_steps;
}

void orc_get_shift(const orc_state* s, double sh[3]) {
    for (int d = 0; d < 3; ++d) sh[d] = s->shift[d];
}

void orc_refresh_ufine(orc_state* s) {
    if (s->p.mpcd) interpolate_buffers(s);
}

void orc_get_fb_u(const orc_state* s, double* out) {
    memcpy(out, s->fbu, sizeof(double) * 3 * (size_t)s->p.nx * (s->p.yhi - s->p.ylo) * s->p.nz);
}

void orc_get_step_acc(const orc_state* s, double* acc) {
    memcpy(acc, s->acc, sizeof(double) * 4 * (size_t)s->p.nx * s->R * s->p.nz);
}

/* ------------------------------------------------------------------------
 * Per-element building blocks on caller arrays, for checking sampled outputs
 * of runs too large for the full oracle.  `s` may come from
 * orc_create_geometry (no arrays).  Arrays are [dim][n].
 * ---------------------------------------------------------------------- */
void orc_grid_shift(const orc_state* s, uint32_t t, uint32_t sub, double sh[3]) { draw_shift(s, t, sub, sh); }

void orc_bin_positions(const orc_state* s, const double sh[3], int64_t n, const double* pos, int32_t* cell) {
    for (int64_t k = 0; k < n; ++k) {
        double r[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < s->p.dim; ++d) r[d] = pos[d * n + k];
        cell[k] = cell_of_pos(s, r, sh);
    }
}

/* Exchange step (buffer particles redrawn about u, given per particle) and
 * streaming of one MPCD step, in place. */
void orc_exchange_stream(const orc_state* s, uint32_t t, uint32_t sub, int64_t n, const uint32_t* ids,
                         double* pos, double* vel, const double* u, const double* tens) {
    for (int64_t k = 0; k < n; ++k) {
        double r[3] = {0.0, 0.0, 0.0}, v[3] = {0.0, 0.0, 0.0}, uu[3] = {0.0, 0.0, 0.0}, T[6];
        for (int d = 0; d < s->p.dim; ++d) {
            r[d] = pos[d * n + k];
            v[d] = vel[d * n + k];
            uu[d] = u[d * n + k];
        }
        for (int m = 0; m < 6; ++m) T[m] = tens ? tens[m * n + k] : 0.0;
        if (buffer_cell(s, r) >= 0) reinject_one(s, ids[k], t, sub, uu, tens ? T : NULL, v);
        (void)stream_one(s, r, v);
        for (int d = 0; d < s->p.dim; ++d) {
            pos[d * n + k] = r[d];
            vel[d * n + k] = v[d];
        }
    }
}

/* 1 when the fine cell of the position is a buffer cell */
int32_t orc_in_buffer(const orc_state* s, const double r[3]) { return buffer_cell(s, r) >= 0; }

/* Collision of one cell (index c of the shifted grid of (t, sub)). */
void orc_collide_cell(const orc_state* s, int32_t c, uint32_t t, uint32_t sub, const double sh[3], int32_t n,
                      const int32_t* ids, double* vel, double vcm[3]) {
    int32_t* seq = NULL;
    if (!ids) {
        seq = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        for (int32_t i = 0; i < n; ++i) seq[i] = i;
        ids = seq;
    }
    collide_one(s, c, t, sub, sh, n, ids, vel, vcm);
    free(seq);
}

/* Buffer fine-cell velocities [3][Cz][R][Cx] (zero outside the buffers) from
 * given node velocities [3][N] (bi/trilinear interpolation, Alg. 2). */
void orc_interpolate(const orc_state* s, const double* unode, double* ufine) {
    memset(ufine, 0, sizeof(double) * 3 * (size_t)s->Cx * s->R * s->Cz);
    interpolate_from(s, s->p.dim, unode, ufine);
}

void orc_ce_tensor(const orc_state* s, double* out) {
    for (int64_t n = 0; n < s->N; ++n) {
        double T[6];
        node_ce_tensor(s, n, T);
        for (int m = 0; m < 6; ++m) out[m * s->N + n] = T[m];
    }
}

void orc_get_tfine(const orc_state* s, double* tfine) {
    memcpy(tfine, s->tfine, sizeof(double) * 6 * (size_t)s->Cx * s->R * s->Cz);
}
