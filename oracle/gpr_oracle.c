/*
 * gpr_oracle.c -- FP64 CPU oracle of the Gen.ParRep hot path (arXiv 1807.02431).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU-baseline leg
 * of the benchmark; never by the product path.  Shares no code with the GPU library.
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared gpr_oracle.c -lm
 *
 * Plain loops in FP64.  Each function names the passage of the paper it follows.  Where
 * the paper leaves a choice open (integrator splitting, random numbers, event order at a
 * check, how the integral of Eq. 2 is discretised) the reading used is stated beside it.
 */
#include "gpr_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define COULOMB_F 138.935458
#define STREAM_NOISE 0
#define STREAM_INIT 1
#define STREAM_BRANCH 2

enum { PH_IDLE = 0, PH_DECORR = 1, PH_DEPHASE = 2, PH_CONVERGED = 3, PH_PARALLEL = 4, PH_DEPHASE_FIXED = 5 };

struct gro_sys {
    int kind, n, R;
    double *mass;
    double *sigma, *eps, *charge;
    double cutoff, eps_rf;
    int nb; int *bond; double *b_r0, *b_k;
    int na; int *ang; double *a_t0, *a_k;
    int nt; int *tor; int *t_n; double *t_k, *t_p0;
    int nr; int *res; double *r_ref, *r_k;
    int np; int *p14; double scale14;
    unsigned char *skip;          /* n*n: 1 = pair not in the nonbonded sum */
    double kT, gamma, dt;
    uint64_t seed;
    int t_gr, tcd, tcp;
    double tol;
    int64_t t_min;
    gro_state_spec st;
    int *st_group;
    int nobs;
    gro_obs_spec obs[GRO_NMAXOBS];
    int *obs_ga[GRO_NMAXOBS], *obs_gb[GRO_NMAXOBS];

    /* dynamic state */
    double *q, *v, *F, *U;        /* [R][3][n], [R][3][n], [R][3][n], [R] */
    int64_t s;                    /* global step counter (noise counter) */
    int64_t tsim;                 /* simulation clock in steps */
    int omega;
    int phase;
    /* transient propagation, resumable */
    int dc_from, dc_omega; int64_t dc_resid, dc_steps;
    /* convergence step, resumable */
    int64_t dp_t, nsamp, n_branch;
    double *S1, *S2;              /* [R][nobs] */
    /* original ParRep dephasing, resumable */
    double *snap;                 /* [3][3][n]: q, v, F of the reference walker when it began */
    double snapU;
    int64_t *resid;               /* [R] steps in Omega since the replica's last (re)start */
    int *done;                    /* [R] the replica has its sample */
    double *samp, *sampU;         /* [R][3][3][n] samples (q, v, F) and their energies [R] */
    double shift[GRO_NMAXOBS];
    /* parallel step, resumable */
    int64_t par_M;
    /* steps taken by gro_advance since creation: its sampling and check schedule */
    int64_t adv_t;
};

static char g_err[512];
static void set_err(const char *m) { snprintf(g_err, sizeof g_err, "%s", m); }
const char *gro_error(void) { return g_err; }

/* ------------------------------------------------------------------ Philox4x32-10
 * Counter-based generator of Salmon, Moraes, Dror and Shaw (SC'11): ten rounds of
 * two 32x32->64 multiplications; the high halves are xored with the other two counter
 * words and the round key, and the key is bumped by the Weyl constants between rounds. */
void gro_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t m0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t m1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(m1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)m1;
        uint32_t n2 = (uint32_t)(m0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)m0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox_words(uint64_t seed, uint32_t atom, int64_t step, uint32_t replica,
                         uint32_t stream, uint32_t w[4])
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint64_t us = (uint64_t)step;
    uint32_t ctr[4] = { atom, (uint32_t)us, replica,
                        (stream << 24) | ((uint32_t)(us >> 32) & 0xFFFFFFu) };
    gro_philox4x32_10(ctr, key, w);
}

/* uniform in (0,1): an odd multiple of 2^-24, exact in binary32 and binary64 */
static double unit_open(uint32_t w) { return ldexp(2.0 * (double)(w >> 9) + 1.0, -24); }

/* three standard normal deviates by the Box-Muller transform */
static void gauss3(const uint32_t w[4], double g[3])
{
    const double two_pi = 6.283185307179586476925286766559;
    double u0 = unit_open(w[0]), u1 = unit_open(w[1]);
    double u2 = unit_open(w[2]), u3 = unit_open(w[3]);
    double ra = sqrt(-2.0 * log(u0)), rb = sqrt(-2.0 * log(u2));
    g[0] = ra * cos(two_pi * u1);
    g[1] = ra * sin(two_pi * u1);
    g[2] = rb * cos(two_pi * u3);
}

void gro_noise(uint64_t seed, int32_t replica, int64_t step, int32_t stream, int32_t n_atoms,
               uint32_t *words, double *gauss)
{
    for (int i = 0; i < n_atoms; i++) {
        uint32_t w[4];
        double g[3];
        philox_words(seed, (uint32_t)i, step, (uint32_t)replica, (uint32_t)stream, w);
        gauss3(w, g);
        if (words) for (int k = 0; k < 4; k++) words[4 * i + k] = w[k];
        if (gauss) for (int k = 0; k < 3; k++) gauss[3 * i + k] = g[k];
    }
}

/* ------------------------------------------------------------------ geometry helpers */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static void getp(const double *q, int n, int i, double *p) { p[0] = q[i]; p[1] = q[n + i]; p[2] = q[2 * n + i]; }
static void addf(double *F, int n, int i, const double *f)
{
    F[i] += f[0]; F[n + i] += f[1]; F[2 * n + i] += f[2];
}

/* signed angle between the planes (i,j,k) and (j,k,l): the IUPAC dihedral, trans = pi.
 * Its magnitude is the angle between the plane normals m = r_ij x r_kj and
 * w = r_kj x r_kl; its sign is that of r_ij . w. */
static double dihedral(const double *q, int n, const int *a)
{
    double pi_[3], pj[3], pk[3], pl[3], rij[3], rkj[3], rkl[3], m[3], w[3];
    getp(q, n, a[0], pi_); getp(q, n, a[1], pj); getp(q, n, a[2], pk); getp(q, n, a[3], pl);
    for (int d = 0; d < 3; d++) { rij[d] = pi_[d] - pj[d]; rkj[d] = pk[d] - pj[d]; rkl[d] = pk[d] - pl[d]; }
    cross3(rij, rkj, m);
    cross3(rkj, rkl, w);
    double c = dot3(m, w) / sqrt(dot3(m, m) * dot3(w, w));
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    double phi = acos(c);
    return dot3(rij, w) < 0.0 ? -phi : phi;
}

/* ------------------------------------------------------------------ force field (Sec. 3.2)
 * U(q) and F = -grad U.  Plain loops over every term and every atom pair. */
static double eval_molecular(const gro_sys *S, const double *q, double *F)
{
    const int n = S->n;
    double U = 0.0;
    memset(F, 0, sizeof(double) * 3 * (size_t)n);

    /* harmonic bonds 1/2 k (r - r0)^2 */
    for (int b = 0; b < S->nb; b++) {
        int i = S->bond[2 * b], j = S->bond[2 * b + 1];
        double pi_[3], pj[3], d[3], f[3];
        getp(q, n, i, pi_); getp(q, n, j, pj);
        for (int k = 0; k < 3; k++) d[k] = pj[k] - pi_[k];
        double r = sqrt(dot3(d, d));
        double dr = r - S->b_r0[b];
        U += 0.5 * S->b_k[b] * dr * dr;
        double g = S->b_k[b] * dr / r;           /* force on i is +g d */
        for (int k = 0; k < 3; k++) f[k] = g * d[k];
        addf(F, n, i, f);
        for (int k = 0; k < 3; k++) f[k] = -f[k];
        addf(F, n, j, f);
    }

    /* harmonic angles 1/2 k (theta - theta0)^2, vertex at the middle atom */
    for (int a = 0; a < S->na; a++) {
        int i = S->ang[3 * a], j = S->ang[3 * a + 1], k = S->ang[3 * a + 2];
        double pi_[3], pj[3], pk[3], u[3], w[3], fi[3], fk[3], fj[3];
        getp(q, n, i, pi_); getp(q, n, j, pj); getp(q, n, k, pk);
        for (int d = 0; d < 3; d++) { u[d] = pi_[d] - pj[d]; w[d] = pk[d] - pj[d]; }
        double lu = sqrt(dot3(u, u)), lw = sqrt(dot3(w, w));
        double c = dot3(u, w) / (lu * lw);
        if (c > 1.0) c = 1.0;
        if (c < -1.0) c = -1.0;
        double th = acos(c);
        double s = sqrt(1.0 - c * c);
        double dth = th - S->a_t0[a];
        U += 0.5 * S->a_k[a] * dth * dth;
        /* d theta / d cos = -1/sin; d cos / d p_i = w/(lu lw) - c u/lu^2 */
        double g = S->a_k[a] * dth / s;          /* -dU/dtheta * dtheta/dcos = k dth / s */
        for (int d = 0; d < 3; d++) {
            fi[d] = g * (w[d] / (lu * lw) - c * u[d] / (lu * lu));
            fk[d] = g * (u[d] / (lu * lw) - c * w[d] / (lw * lw));
            fj[d] = -fi[d] - fk[d];
        }
        addf(F, n, i, fi); addf(F, n, j, fj); addf(F, n, k, fk);
    }

    /* periodic torsions k (1 + cos(n phi - phi0)).  Gradient of phi: the classical
     * result for the dihedral (e.g. Bekker's thesis; Blondel and Karplus 1996):
     * dphi/dp_i = -|r_kj|/|m|^2 m, dphi/dp_l = |r_kj|/|w|^2 w, and the two middle atoms
     * take the remainder so that the net force and torque vanish. */
    for (int t = 0; t < S->nt; t++) {
        const int *A = S->tor + 4 * t;
        double pi_[3], pj[3], pk[3], pl[3], rij[3], rkj[3], rkl[3], m[3], w[3];
        getp(q, n, A[0], pi_); getp(q, n, A[1], pj); getp(q, n, A[2], pk); getp(q, n, A[3], pl);
        for (int d = 0; d < 3; d++) { rij[d] = pi_[d] - pj[d]; rkj[d] = pk[d] - pj[d]; rkl[d] = pk[d] - pl[d]; }
        cross3(rij, rkj, m);
        cross3(rkj, rkl, w);
        double phi = dihedral(q, n, A);
        double mult = (double)S->t_n[t];
        U += S->t_k[t] * (1.0 + cos(mult * phi - S->t_p0[t]));
        double dUdphi = -S->t_k[t] * mult * sin(mult * phi - S->t_p0[t]);
        double lkj2 = dot3(rkj, rkj), lkj = sqrt(lkj2);
        double m2 = dot3(m, m), w2 = dot3(w, w);
        /* dphi/dp_i = |r_kj|/|m|^2 m and dphi/dp_l = -|r_kj|/|w|^2 w for phi signed by
         * r_ij . w; F = -dU/dphi dphi/dp */
        double fi[3], fl[3], fj[3], fk[3];
        for (int d = 0; d < 3; d++) {
            fi[d] = -dUdphi * (lkj / m2) * m[d];
            fl[d] = dUdphi * (lkj / w2) * w[d];
        }
        double p = dot3(rij, rkj) / lkj2, qq = dot3(rkl, rkj) / lkj2;
        for (int d = 0; d < 3; d++) {
            double sv = p * fi[d] - qq * fl[d];
            fj[d] = -fi[d] + sv;
            fk[d] = -fl[d] - sv;
        }
        addf(F, n, A[0], fi); addf(F, n, A[1], fj); addf(F, n, A[2], fk); addf(F, n, A[3], fl);
    }

    /* harmonic position restraints 1/2 k |r - r_ref|^2 */
    for (int r = 0; r < S->nr; r++) {
        int i = S->res[r];
        double p[3], f[3];
        getp(q, n, i, p);
        double e = 0.0;
        for (int d = 0; d < 3; d++) {
            double x = p[d] - S->r_ref[3 * r + d];
            e += x * x;
            f[d] = -S->r_k[r] * x;
        }
        U += 0.5 * S->r_k[r] * e;
        addf(F, n, i, f);
    }

    /* 1-4 pairs: scale14 (Lennard-Jones + vacuum Coulomb), no cutoff */
    for (int pp = 0; pp < S->np; pp++) {
        int i = S->p14[2 * pp], j = S->p14[2 * pp + 1];
        double pi_[3], pj[3], d[3], f[3];
        getp(q, n, i, pi_); getp(q, n, j, pj);
        for (int k = 0; k < 3; k++) d[k] = pi_[k] - pj[k];
        double r2 = dot3(d, d), r = sqrt(r2);
        double sij = 0.5 * (S->sigma[i] + S->sigma[j]);
        double eij = sqrt(S->eps[i] * S->eps[j]);
        double sr6 = pow(sij / r, 6.0);
        double qq = COULOMB_F * S->charge[i] * S->charge[j];
        double u = 4.0 * eij * (sr6 * sr6 - sr6) + qq / r;
        double fs = 24.0 * eij * (2.0 * sr6 * sr6 - sr6) / r2 + qq / (r2 * r);   /* -dU/dr / r */
        U += S->scale14 * u;
        for (int k = 0; k < 3; k++) f[k] = S->scale14 * fs * d[k];
        addf(F, n, i, f);
        for (int k = 0; k < 3; k++) f[k] = -f[k];
        addf(F, n, j, f);
    }

    /* nonbonded: every pair i<j not skipped; cutoff == 0 -> vacuum Coulomb on all pairs,
     * cutoff > 0 -> pairs with r < cutoff, reaction-field Coulomb */
    const double rc = S->cutoff;
    double krf = 0.0, crf = 0.0;
    if (rc > 0.0) {
        krf = (S->eps_rf - 1.0) / ((2.0 * S->eps_rf + 1.0) * rc * rc * rc);
        crf = 1.0 / rc + krf * rc * rc;
    }
    for (int i = 0; i < n; i++) {
        for (int j = i + 1; j < n; j++) {
            if (S->skip[(size_t)i * n + j]) continue;
            double pi_[3], pj[3], d[3], f[3];
            getp(q, n, i, pi_); getp(q, n, j, pj);
            for (int k = 0; k < 3; k++) d[k] = pi_[k] - pj[k];
            double r2 = dot3(d, d);
            if (rc > 0.0 && !(r2 < rc * rc)) continue;
            double r = sqrt(r2);
            double sij = 0.5 * (S->sigma[i] + S->sigma[j]);
            double eij = sqrt(S->eps[i] * S->eps[j]);
            double sr6 = pow(sij / r, 6.0);
            double qq = COULOMB_F * S->charge[i] * S->charge[j];
            double u = 4.0 * eij * (sr6 * sr6 - sr6);
            double fs = 24.0 * eij * (2.0 * sr6 * sr6 - sr6) / r2;
            if (rc > 0.0) {
                u += qq * (1.0 / r + krf * r2 - crf);
                fs += qq * (1.0 / (r2 * r) - 2.0 * krf);
            } else {
                u += qq / r;
                fs += qq / (r2 * r);
            }
            U += u;
            for (int k = 0; k < 3; k++) f[k] = fs * d[k];
            addf(F, n, i, f);
            for (int k = 0; k < 3; k++) f[k] = -f[k];
            addf(F, n, j, f);
        }
    }
    return U;
}

/* the metastable toy: U(x,y) = (x^2-1)^2 + 2 y^2 */
static double eval_toy(const double *q, double *F)
{
    double x = q[0], y = q[1];
    F[0] = -4.0 * x * (x * x - 1.0);
    F[1] = -4.0 * y;
    F[2] = 0.0;
    return (x * x - 1.0) * (x * x - 1.0) + 2.0 * y * y;
}

static double eval(const gro_sys *S, const double *q, double *F)
{
    return S->kind == GRO_TOY2D ? eval_toy(q, F) : eval_molecular(S, q, F);
}

int gro_eval(const gro_sys *S, const double *q, double *F, double *U)
{
    double *Fl = (double *)malloc(sizeof(double) * 3 * (size_t)S->n);
    if (!Fl) return GRO_ENOMEM;
    double u = eval(S, q, Fl);
    if (F) memcpy(F, Fl, sizeof(double) * 3 * (size_t)S->n);
    if (U) *U = u;
    free(Fl);
    return GRO_OK;
}

/* ------------------------------------------------------------------ parameter gradient
 * dU/dtheta at positions q for the per-atom Lennard-Jones eps_i and sigma_i, the charges q_i
 * and the torsion force constants k_t: the energy terms of eval_molecular differentiated by
 * hand, term by term over the same pairs.
 *   eps_ij = sqrt(eps_i eps_j):  d eps_ij / d eps_i = eps_ij / (2 eps_i)     (eps_i > 0)
 *   sigma_ij = (sigma_i + sigma_j) / 2:  d / d sigma_i = 1/2 d / d sigma_ij, and with
 *     s = sigma_ij / r,  d/d sigma_ij [4 eps (s^12 - s^6)] = 4 eps (12 s^12 - 6 s^6) / sigma_ij
 *   Coulomb f q_i q_j g(r), g = 1/r (vacuum, 1-4) or 1/r + k_rf r^2 - c_rf (reaction field):
 *     d / d q_i = f q_j g(r)
 *   torsion k (1 + cos(n phi - phi0)):  d / dk = 1 + cos(n phi - phi0)
 * 1-4 pairs carry their scale factor.  Outputs are overwritten: dU_eps, dU_sig, dU_q [n],
 * dU_k [number of torsions] (each may be NULL). */
int gro_param_grad(const gro_sys *S, const double *q, double *dU_eps, double *dU_sig, double *dU_q, double *dU_k)
{
    const int n = S->n;
    if (S->kind != GRO_MOLECULAR) return GRO_EINVAL;
    double *ge = (double *)calloc((size_t)n, sizeof(double));
    double *gs = (double *)calloc((size_t)n, sizeof(double));
    double *gq = (double *)calloc((size_t)n, sizeof(double));
    if (!ge || !gs || !gq) { free(ge); free(gs); free(gq); return GRO_ENOMEM; }

    /* one pair: scale * [LJ + Coulomb with kernel g] */
    #define PAIR_GRAD(I, J, R, G, SCALE)                                                   \
        do {                                                                               \
            const double sij = 0.5 * (S->sigma[I] + S->sigma[J]);                          \
            const double eij = sqrt(S->eps[I] * S->eps[J]);                                \
            const double s6 = pow(sij / (R), 6.0), s12 = s6 * s6;                          \
            const double ulj = 4.0 * eij * (s12 - s6);                                     \
            const double dsig = 0.5 * 4.0 * eij * (12.0 * s12 - 6.0 * s6) / sij;           \
            ge[I] += (SCALE) * ulj / (2.0 * S->eps[I]);                                    \
            ge[J] += (SCALE) * ulj / (2.0 * S->eps[J]);                                    \
            gs[I] += (SCALE) * dsig;                                                       \
            gs[J] += (SCALE) * dsig;                                                       \
            gq[I] += (SCALE) * COULOMB_F * S->charge[J] * (G);                             \
            gq[J] += (SCALE) * COULOMB_F * S->charge[I] * (G);                             \
        } while (0)

    for (int pp = 0; pp < S->np; pp++) {
        int i = S->p14[2 * pp], j = S->p14[2 * pp + 1];
        double pi_[3], pj[3], d[3];
        getp(q, n, i, pi_); getp(q, n, j, pj);
        for (int k = 0; k < 3; k++) d[k] = pi_[k] - pj[k];
        const double r = sqrt(dot3(d, d));
        PAIR_GRAD(i, j, r, 1.0 / r, S->scale14);
    }
    const double rc = S->cutoff;
    double krf = 0.0, crf = 0.0;
    if (rc > 0.0) {
        krf = (S->eps_rf - 1.0) / ((2.0 * S->eps_rf + 1.0) * rc * rc * rc);
        crf = 1.0 / rc + krf * rc * rc;
    }
    for (int i = 0; i < n; i++) {
        for (int j = i + 1; j < n; j++) {
            if (S->skip[(size_t)i * n + j]) continue;
            double pi_[3], pj[3], d[3];
            getp(q, n, i, pi_); getp(q, n, j, pj);
            for (int k = 0; k < 3; k++) d[k] = pi_[k] - pj[k];
            const double r2 = dot3(d, d);
            if (rc > 0.0 && !(r2 < rc * rc)) continue;
            const double r = sqrt(r2);
            const double g = rc > 0.0 ? 1.0 / r + krf * r2 - crf : 1.0 / r;
            PAIR_GRAD(i, j, r, g, 1.0);
        }
    }
    #undef PAIR_GRAD
    if (dU_k)
        for (int t = 0; t < S->nt; t++)
            dU_k[t] = 1.0 + cos((double)S->t_n[t] * dihedral(q, n, S->tor + 4 * t) - S->t_p0[t]);
    if (dU_eps) memcpy(dU_eps, ge, sizeof(double) * (size_t)n);
    if (dU_sig) memcpy(dU_sig, gs, sizeof(double) * (size_t)n);
    if (dU_q) memcpy(dU_q, gq, sizeof(double) * (size_t)n);
    free(ge); free(gs); free(gq);
    return GRO_OK;
}

/* ------------------------------------------------------------------ replica access */
static double *Q(const gro_sys *S, int r) { return S->q + (size_t)r * 3 * S->n; }
static double *Vv(const gro_sys *S, int r) { return S->v + (size_t)r * 3 * S->n; }
static double *Ff(const gro_sys *S, int r) { return S->F + (size_t)r * 3 * S->n; }

static void copy_replica(gro_sys *S, int dst, int src)
{
    size_t b = sizeof(double) * 3 * (size_t)S->n;
    memcpy(Q(S, dst), Q(S, src), b);
    memcpy(Vv(S, dst), Vv(S, src), b);
    memcpy(Ff(S, dst), Ff(S, src), b);
    S->U[dst] = S->U[src];
}

static double kinetic(const gro_sys *S, const double *v)
{
    double K = 0.0;
    for (int i = 0; i < S->n; i++) {
        double s = v[i] * v[i] + v[S->n + i] * v[S->n + i] + v[2 * S->n + i] * v[2 * S->n + i];
        K += 0.5 * S->mass[i] * s;
    }
    return K;
}

static void com(const gro_sys *S, const double *q, const int *g, int ng, double *c)
{
    double mt = 0.0;
    c[0] = c[1] = c[2] = 0.0;
    for (int a = 0; a < ng; a++) {
        int i = g[a];
        double m = S->mass[i];
        c[0] += m * q[i]; c[1] += m * q[S->n + i]; c[2] += m * q[2 * S->n + i];
        mt += m;
    }
    c[0] /= mt; c[1] /= mt; c[2] /= mt;
}

/* ------------------------------------------------------------------ states (Sec. 2.2) */
int32_t gro_state_of(const gro_sys *S, const double *q)
{
    const gro_state_spec *st = &S->st;
    switch (st->kind) {
    case GRO_STATE_SIGN_X:
        return q[st->atoms[0]] >= 0.0 ? 1 : 0;
    case GRO_STATE_DIHEDRAL_BOXES: {
        double phi = dihedral(q, S->n, st->atoms);
        double psi = dihedral(q, S->n, st->atoms + 4);
        for (int b = 0; b < st->n_boxes; b++) {
            const double *B = st->box[b];
            if (B[0] < phi && phi <= B[1] && B[2] < psi && psi <= B[3]) return b;
        }
        return -1;
    }
    case GRO_STATE_COM_SPHERE: {
        double c[3];
        com(S, q, S->st_group, st->n_group, c);
        double d2 = 0.0;
        for (int k = 0; k < 3; k++) d2 += (c[k] - st->center[k]) * (c[k] - st->center[k]);
        return sqrt(d2) < st->radius ? 1 : 0;
    }
    }
    return -1;
}

/* ------------------------------------------------------------------ observables (Eq. 2) */
int gro_observables_of(const gro_sys *S, const double *q, const double *v, double U, double *out)
{
    for (int j = 0; j < S->nobs; j++) {
        const gro_obs_spec *o = &S->obs[j];
        double val = 0.0;
        switch (o->kind) {
        case GRO_OBS_COORD: val = q[o->atoms[1] * S->n + o->atoms[0]]; break;
        case GRO_OBS_POTENTIAL: val = U; break;
        case GRO_OBS_KINETIC: val = kinetic(S, v); break;
        case GRO_OBS_DIHEDRAL: val = dihedral(q, S->n, o->atoms); break;
        case GRO_OBS_COM_DISTANCE: {
            double a[3], b[3];
            com(S, q, S->obs_ga[j], o->n_a, a);
            com(S, q, S->obs_gb[j], o->n_b, b);
            val = sqrt((a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]) + (a[2] - b[2]) * (a[2] - b[2]));
            break;
        }
        case GRO_OBS_RMS_VELOCITY: {
            double s = 0.0;
            for (int a = 0; a < o->n_a; a++) {
                int i = S->obs_ga[j][a];
                s += v[i] * v[i] + v[S->n + i] * v[S->n + i] + v[2 * S->n + i] * v[2 * S->n + i];
            }
            val = sqrt(s / o->n_a);
            break;
        }
        default: return GRO_EINVAL;
        }
        out[j] = val;
    }
    return GRO_OK;
}

static void obs_of_replica(const gro_sys *S, int r, double *out)
{
    gro_observables_of(S, Q(S, r), Vv(S, r), S->U[r], out);
}

/* ------------------------------------------------------------------ BAOAB step (Eq. 1)
 * One step of replica r with the noise of global step s:
 *   B: v += dt/2 F/m   A: q += dt/2 v   O: v = c1 v + sqrt((1-c1^2) kT/m) xi
 *   A: q += dt/2 v     F = F(q)         B: v += dt/2 F/m
 * c1 = exp(-gamma dt): gamma is read as a friction rate (1/time), so that the friction
 * term of Eq. 1 is gamma p for every mass (identical to Eq. 1 for the unit-mass toy). */
static void step_replica(gro_sys *S, int r, int64_t s)
{
    const int n = S->n;
    const int dims = S->kind == GRO_TOY2D ? 2 : 3;
    double *q = Q(S, r), *v = Vv(S, r), *F = Ff(S, r);
    const double h = 0.5 * S->dt;
    const double c1 = exp(-S->gamma * S->dt);
    const double c2 = sqrt(1.0 - c1 * c1);
    for (int d = 0; d < dims; d++)
        for (int i = 0; i < n; i++) {
            v[d * n + i] += h * F[d * n + i] / S->mass[i];
            q[d * n + i] += h * v[d * n + i];
        }
    for (int i = 0; i < n; i++) {
        uint32_t w[4];
        double g[3];
        philox_words(S->seed, (uint32_t)i, s, (uint32_t)r, STREAM_NOISE, w);
        gauss3(w, g);
        double sd = c2 * sqrt(S->kT / S->mass[i]);
        for (int d = 0; d < dims; d++) {
            v[d * n + i] = c1 * v[d * n + i] + sd * g[d];
            q[d * n + i] += h * v[d * n + i];
        }
    }
    S->U[r] = eval(S, q, F);
    for (int d = 0; d < dims; d++)
        for (int i = 0; i < n; i++) v[d * n + i] += h * F[d * n + i] / S->mass[i];
}

/* one tick of the global clock for replicas [0, nrep) */
static int step_all(gro_sys *S, int nrep)
{
    for (int r = 0; r < nrep; r++) step_replica(S, r, S->s);
    S->s += 1;
    for (int r = 0; r < nrep; r++)
        if (!isfinite(S->U[r])) { set_err("non-finite energy"); return GRO_EUNSTABLE; }
    return GRO_OK;
}

/* ------------------------------------------------------------------ lifecycle */
static void *dupmem(const void *p, size_t b)
{
    if (!p || b == 0) return NULL;
    void *d = malloc(b);
    if (d) memcpy(d, p, b);
    return d;
}

void gro_destroy(gro_sys *S)
{
    if (!S) return;
    free(S->mass); free(S->sigma); free(S->eps); free(S->charge);
    free(S->bond); free(S->b_r0); free(S->b_k);
    free(S->ang); free(S->a_t0); free(S->a_k);
    free(S->tor); free(S->t_n); free(S->t_k); free(S->t_p0);
    free(S->res); free(S->r_ref); free(S->r_k);
    free(S->p14); free(S->skip); free(S->st_group);
    for (int j = 0; j < GRO_NMAXOBS; j++) { free(S->obs_ga[j]); free(S->obs_gb[j]); }
    free(S->q); free(S->v); free(S->F); free(S->U); free(S->S1); free(S->S2);
    free(S->snap); free(S->resid); free(S->done); free(S->samp); free(S->sampU);
    free(S);
}

static int idx_ok(const int32_t *a, int cnt, int n)
{
    for (int k = 0; k < cnt; k++) if (a[k] < 0 || a[k] >= n) return 0;
    return 1;
}

int gro_create(const gro_spec *d, gro_sys **out)
{
    *out = NULL;
    if (!d || (d->kind != GRO_TOY2D && d->kind != GRO_MOLECULAR)) { set_err("bad kind"); return GRO_EINVAL; }
    if (d->n_atoms < 1 || d->n_replicas < 2 || !d->mass || !d->pos) { set_err("bad sizes"); return GRO_EINVAL; }
    if (d->kind == GRO_TOY2D && d->n_atoms != 1) { set_err("toy has one particle"); return GRO_EINVAL; }
    if (!(d->dt > 0) || !(d->kT > 0) || d->gamma < 0) { set_err("bad dynamics parameters"); return GRO_EINVAL; }
    if (d->t_gr < 1 || d->t_check_dephase < 1 || d->t_check_parallel < 1) { set_err("bad periods"); return GRO_EINVAL; }
    if (d->n_obs < 0 || d->n_obs > GRO_NMAXOBS) { set_err("bad n_obs"); return GRO_EINVAL; }
    const int n = d->n_atoms, R = d->n_replicas;
    for (int i = 0; i < n; i++) if (!(d->mass[i] > 0)) { set_err("mass <= 0"); return GRO_EINVAL; }
    if (d->kind == GRO_MOLECULAR) {
        if (!d->sigma || !d->epsilon || !d->charge) { set_err("missing nonbonded parameters"); return GRO_EINVAL; }
        if (!idx_ok(d->bond_atoms, 2 * d->n_bonds, n) || !idx_ok(d->angle_atoms, 3 * d->n_angles, n) ||
            !idx_ok(d->torsion_atoms, 4 * d->n_torsions, n) || !idx_ok(d->restraint_atom, d->n_restraints, n) ||
            !idx_ok(d->pair14_atoms, 2 * d->n_pairs14, n) || !idx_ok(d->exclusion_atoms, 2 * d->n_exclusions, n)) {
            set_err("term atom index out of range"); return GRO_EINVAL;
        }
    }
    gro_sys *S = (gro_sys *)calloc(1, sizeof(gro_sys));
    if (!S) return GRO_ENOMEM;
    S->kind = d->kind; S->n = n; S->R = R;
    S->mass = (double *)dupmem(d->mass, sizeof(double) * n);
    if (d->kind == GRO_MOLECULAR) {
        S->sigma = (double *)dupmem(d->sigma, sizeof(double) * n);
        S->eps = (double *)dupmem(d->epsilon, sizeof(double) * n);
        S->charge = (double *)dupmem(d->charge, sizeof(double) * n);
        S->cutoff = d->cutoff; S->eps_rf = d->eps_rf;
        S->nb = d->n_bonds; S->bond = (int *)dupmem(d->bond_atoms, sizeof(int) * 2 * S->nb);
        S->b_r0 = (double *)dupmem(d->bond_r0, sizeof(double) * S->nb);
        S->b_k = (double *)dupmem(d->bond_k, sizeof(double) * S->nb);
        S->na = d->n_angles; S->ang = (int *)dupmem(d->angle_atoms, sizeof(int) * 3 * S->na);
        S->a_t0 = (double *)dupmem(d->angle_theta0, sizeof(double) * S->na);
        S->a_k = (double *)dupmem(d->angle_k, sizeof(double) * S->na);
        S->nt = d->n_torsions; S->tor = (int *)dupmem(d->torsion_atoms, sizeof(int) * 4 * S->nt);
        S->t_n = (int *)dupmem(d->torsion_n, sizeof(int) * S->nt);
        S->t_k = (double *)dupmem(d->torsion_k, sizeof(double) * S->nt);
        S->t_p0 = (double *)dupmem(d->torsion_phi0, sizeof(double) * S->nt);
        S->nr = d->n_restraints; S->res = (int *)dupmem(d->restraint_atom, sizeof(int) * S->nr);
        S->r_ref = (double *)dupmem(d->restraint_ref, sizeof(double) * 3 * S->nr);
        S->r_k = (double *)dupmem(d->restraint_k, sizeof(double) * S->nr);
        S->np = d->n_pairs14; S->p14 = (int *)dupmem(d->pair14_atoms, sizeof(int) * 2 * S->np);
        S->scale14 = d->scale14;
        S->skip = (unsigned char *)calloc((size_t)n * n, 1);
        if (!S->skip) { gro_destroy(S); return GRO_ENOMEM; }
        for (int e = 0; e < d->n_exclusions; e++) {
            int i = d->exclusion_atoms[2 * e], j = d->exclusion_atoms[2 * e + 1];
            S->skip[(size_t)i * n + j] = S->skip[(size_t)j * n + i] = 1;
        }
        for (int p = 0; p < S->np; p++) {
            int i = S->p14[2 * p], j = S->p14[2 * p + 1];
            S->skip[(size_t)i * n + j] = S->skip[(size_t)j * n + i] = 1;
        }
        for (int i = 0; i < n; i++) S->skip[(size_t)i * n + i] = 1;
    }
    S->kT = d->kT; S->gamma = d->gamma; S->dt = d->dt; S->seed = d->seed;
    S->t_gr = d->t_gr; S->tcd = d->t_check_dephase; S->tcp = d->t_check_parallel;
    S->tol = d->tol; S->t_min = d->t_min;
    S->st = d->state;
    if (S->st.kind == GRO_STATE_COM_SPHERE) {
        if (S->st.n_group < 1 || !idx_ok(S->st.group, S->st.n_group, n)) { gro_destroy(S); set_err("bad state group"); return GRO_EINVAL; }
        S->st_group = (int *)dupmem(S->st.group, sizeof(int) * S->st.n_group);
    } else if (S->st.kind == GRO_STATE_SIGN_X) {
        if (!idx_ok(S->st.atoms, 1, n)) { gro_destroy(S); set_err("bad state atom"); return GRO_EINVAL; }
    } else if (S->st.kind == GRO_STATE_DIHEDRAL_BOXES) {
        if (!idx_ok(S->st.atoms, 8, n) || S->st.n_boxes < 1 || S->st.n_boxes > GRO_NMAXBOX) { gro_destroy(S); set_err("bad state boxes"); return GRO_EINVAL; }
    } else { gro_destroy(S); set_err("bad state kind"); return GRO_EINVAL; }
    S->st.group = NULL;
    S->nobs = d->n_obs;
    for (int j = 0; j < S->nobs; j++) {
        S->obs[j] = d->obs[j];
        if (S->obs[j].n_a > 0) {
            if (!idx_ok(d->obs[j].group_a, d->obs[j].n_a, n)) { gro_destroy(S); set_err("bad observable group"); return GRO_EINVAL; }
            S->obs_ga[j] = (int *)dupmem(d->obs[j].group_a, sizeof(int) * S->obs[j].n_a);
        }
        if (S->obs[j].n_b > 0) {
            if (!idx_ok(d->obs[j].group_b, d->obs[j].n_b, n)) { gro_destroy(S); set_err("bad observable group"); return GRO_EINVAL; }
            S->obs_gb[j] = (int *)dupmem(d->obs[j].group_b, sizeof(int) * S->obs[j].n_b);
        }
        S->obs[j].group_a = S->obs[j].group_b = NULL;
        int k = S->obs[j].kind;
        if (k < GRO_OBS_COORD || k > GRO_OBS_RMS_VELOCITY) { gro_destroy(S); set_err("bad observable kind"); return GRO_EINVAL; }
        if ((k == GRO_OBS_COM_DISTANCE && (S->obs[j].n_a < 1 || S->obs[j].n_b < 1)) ||
            (k == GRO_OBS_RMS_VELOCITY && S->obs[j].n_a < 1) ||
            (k == GRO_OBS_DIHEDRAL && !idx_ok(S->obs[j].atoms, 4, n)) ||
            (k == GRO_OBS_COORD && (!idx_ok(S->obs[j].atoms, 1, n) || S->obs[j].atoms[1] < 0 || S->obs[j].atoms[1] > 2))) {
            gro_destroy(S); set_err("bad observable"); return GRO_EINVAL;
        }
    }
    size_t rs = (size_t)R * 3 * n;
    S->q = (double *)calloc(rs, sizeof(double));
    S->v = (double *)calloc(rs, sizeof(double));
    S->F = (double *)calloc(rs, sizeof(double));
    S->U = (double *)calloc(R, sizeof(double));
    S->S1 = (double *)calloc((size_t)R * GRO_NMAXOBS, sizeof(double));
    S->S2 = (double *)calloc((size_t)R * GRO_NMAXOBS, sizeof(double));
    S->snap = (double *)calloc((size_t)9 * n, sizeof(double));
    S->resid = (int64_t *)calloc((size_t)R, sizeof(int64_t));
    S->done = (int *)calloc((size_t)R, sizeof(int));
    S->samp = (double *)calloc((size_t)R * 9 * n, sizeof(double));
    S->sampU = (double *)calloc((size_t)R, sizeof(double));
    if (!S->q || !S->v || !S->F || !S->U || !S->S1 || !S->S2 || !S->snap || !S->resid || !S->done || !S->samp ||
        !S->sampU) { gro_destroy(S); return GRO_ENOMEM; }

    /* replica 0 from the descriptor; velocities drawn from Maxwell-Boltzmann if absent */
    memcpy(S->q, d->pos, sizeof(double) * 3 * n);
    if (S->kind == GRO_TOY2D) S->q[2] = 0.0;
    if (d->vel) {
        memcpy(S->v, d->vel, sizeof(double) * 3 * n);
    } else {
        for (int i = 0; i < n; i++) {
            uint32_t w[4];
            double g[3];
            philox_words(S->seed, (uint32_t)i, 0, 0u, STREAM_INIT, w);
            gauss3(w, g);
            double sd = sqrt(S->kT / S->mass[i]);
            for (int dd = 0; dd < 3; dd++) S->v[dd * n + i] = sd * g[dd];
        }
    }
    if (S->kind == GRO_TOY2D) S->v[2] = 0.0;
    S->U[0] = eval(S, S->q, S->F);
    for (int r = 1; r < R; r++) copy_replica(S, r, 0);
    S->s = 0; S->tsim = 0; S->phase = PH_IDLE;
    S->omega = gro_state_of(S, S->q);
    double o0[GRO_NMAXOBS];
    obs_of_replica(S, 0, o0);
    for (int j = 0; j < S->nobs; j++) S->shift[j] = o0[j];
    *out = S;
    return GRO_OK;
}

/* ------------------------------------------------------------------ queries */
double gro_simulated_time(const gro_sys *S) { return (double)S->tsim * S->dt; }
int64_t gro_simulated_steps(const gro_sys *S) { return S->tsim; }
int64_t gro_global_step(const gro_sys *S) { return S->s; }
int32_t gro_current_state(const gro_sys *S) { return S->omega; }

int gro_energy_forces(const gro_sys *S, int32_t r0, int32_t nr, double *E, double *F)
{
    if (r0 < 0 || nr < 0 || r0 + nr > S->R) { set_err("replica range"); return GRO_EINVAL; }
    for (int k = 0; k < nr; k++) {
        if (E) E[k] = S->U[r0 + k];
        if (F) memcpy(F + (size_t)k * 3 * S->n, Ff(S, r0 + k), sizeof(double) * 3 * S->n);
    }
    return GRO_OK;
}

int gro_get_state(const gro_sys *S, int32_t r, double *q, double *v)
{
    if (r < 0 || r >= S->R) { set_err("replica index"); return GRO_EINVAL; }
    if (q) memcpy(q, Q(S, r), sizeof(double) * 3 * S->n);
    if (v) memcpy(v, Vv(S, r), sizeof(double) * 3 * S->n);
    return GRO_OK;
}

int gro_set_state(gro_sys *S, int32_t r, const double *q, const double *v)
{
    if (r < 0 || r >= S->R || !q) { set_err("replica index"); return GRO_EINVAL; }
    memcpy(Q(S, r), q, sizeof(double) * 3 * S->n);
    if (v) memcpy(Vv(S, r), v, sizeof(double) * 3 * S->n);
    if (S->kind == GRO_TOY2D) { Q(S, r)[2] = 0.0; Vv(S, r)[2] = 0.0; }
    S->U[r] = eval(S, Q(S, r), Ff(S, r));
    S->phase = PH_IDLE;
    return GRO_OK;
}

int gro_get_accumulators(const gro_sys *S, int64_t *n, double *S1, double *S2, double *shift)
{
    if (n) *n = S->nsamp;
    for (int r = 0; r < S->R; r++)
        for (int j = 0; j < S->nobs; j++) {
            if (S1) S1[r * S->nobs + j] = S->S1[r * GRO_NMAXOBS + j];
            if (S2) S2[r * S->nobs + j] = S->S2[r * GRO_NMAXOBS + j];
        }
    if (shift) for (int j = 0; j < S->nobs; j++) shift[j] = S->shift[j];
    return GRO_OK;
}

int gro_observe(const gro_sys *S, double *obs, int32_t *state)
{
    for (int r = 0; r < S->R; r++) {
        if (obs) obs_of_replica(S, r, obs + (size_t)r * S->nobs);
        if (state) state[r] = gro_state_of(S, Q(S, r));
    }
    return GRO_OK;
}

/* ------------------------------------------------------------------ Gelman-Rubin (Eq. 3)
 * With samples taken at the right end of each t_GR interval, t^-1 int_0^t O ds is the
 * sample mean and the time integrals of Eq. 3 are sample means.  Writing Ob_k = S1_k/n
 * (shifted by the common c), the numerator of Eq. 3 is mean_k(S2_k/n) - (mean_k Ob_k)^2
 * and the denominator mean_k(S2_k/n - Ob_k^2).  The paper fixes no summation order; sums
 * over workers use one canonical pairwise tree, so that the result is reproducible bit for
 * bit: the m terms are padded with zeros to the next power of two p and each node of the
 * tree adds its lower half to its upper half, (x[lo .. lo+p/2) sum) + (x[lo+p/2 .. lo+p) sum). */
static double pairwise_pow2(const double *x, int m, int lo, int p)
{
    if (p == 1) return lo < m ? x[lo] : 0.0;
    int h = p / 2;
    return pairwise_pow2(x, m, lo, h) + pairwise_pow2(x, m, lo + h, h);
}

static double pairwise(const double *x, int m)
{
    if (m <= 0) return 0.0;
    int p = 1;
    while (p < m) p *= 2;
    return pairwise_pow2(x, m, 0, p);
}

int gro_rhat(int32_t nw, int32_t n_obs, int64_t n, const double *S1, const double *S2, double *rhat)
{
    if (nw < 1 || n_obs < 0 || n < 1) { set_err("rhat sizes"); return GRO_EINVAL; }
    double *ob = (double *)malloc(sizeof(double) * nw);
    double *a = (double *)malloc(sizeof(double) * nw);
    double *w = (double *)malloc(sizeof(double) * nw);
    if (!ob || !a || !w) { free(ob); free(a); free(w); return GRO_ENOMEM; }
    const double dn = (double)n;
    for (int j = 0; j < n_obs; j++) {
        for (int k = 0; k < nw; k++) {
            ob[k] = S1[(size_t)k * n_obs + j] / dn;
            a[k] = S2[(size_t)k * n_obs + j] / dn;
            double o2 = ob[k] * ob[k];
            w[k] = a[k] - o2;
        }
        double m1 = pairwise(ob, nw) / (double)nw;
        double m2 = pairwise(a, nw) / (double)nw;
        double m1sq = m1 * m1;
        double num = m2 - m1sq;
        double den = pairwise(w, nw) / (double)nw;
        rhat[j] = den > 0.0 ? num / den : INFINITY;
    }
    free(ob); free(a); free(w);
    return GRO_OK;
}

/* ------------------------------------------------------------------ F-V branching (Sec. 2.4.1)
 * Survivors S = workers not exited at this check, ascending.  Each exited worker, in
 * increasing index, copies the survivor S[floor(u |S| / 2^32)], u a fresh Philox word;
 * clones made at this check are never donors at the same check. */
int gro_fv_plan(uint64_t seed, int64_t step, int32_t R, const uint8_t *exited, int32_t *donor)
{
    if (R < 1) { set_err("R"); return GRO_EINVAL; }
    int *surv = (int *)malloc(sizeof(int) * R);
    if (!surv) return GRO_ENOMEM;
    int ns = 0;
    for (int r = 1; r < R; r++) if (!exited[r]) surv[ns++] = r;
    donor[0] = -1;
    for (int r = 1; r < R; r++) {
        if (ns == 0) { donor[r] = -2; continue; }
        if (!exited[r]) { donor[r] = -1; continue; }
        uint32_t w[4];
        philox_words(seed, 0u, step, (uint32_t)r, STREAM_BRANCH, w);
        uint64_t pick = ((uint64_t)w[0] * (uint64_t)ns) >> 32;
        donor[r] = surv[pick];
    }
    if (ns == 0) donor[0] = -2;
    free(surv);
    return GRO_OK;
}

/* ------------------------------------------------------------------ Eq. 5 */
int gro_exit_vote(int32_t R, const int64_t *fec, int64_t t_check, int64_t *M, int32_t *k, int64_t *tau)
{
    int64_t best = 0;
    int kk = 0;
    for (int r = 0; r < R; r++) {
        if (fec[r] <= 0) continue;
        if (best == 0 || fec[r] < best) { best = fec[r]; kk = r + 1; }
    }
    if (best == 0) return GRO_BUDGET;
    *M = best;
    *k = kk;
    *tau = ((int64_t)R * (best - 1) + kk) * t_check;
    return GRO_OK;
}

/* ------------------------------------------------------------------ transient propagation
 * Sec. 2.4 step 1, plus a residence time t_corr before the state is accepted as Omega.
 * Exits are looked for every t_check_dephase steps, as in the other steps. */
int gro_decorrelate(gro_sys *S, int64_t t_corr, int64_t max_steps, gro_event *ev)
{
    if (S->phase != PH_DECORR) {
        S->phase = PH_DECORR;
        S->dc_omega = gro_state_of(S, Q(S, 0));
        S->dc_from = S->dc_omega;
        S->dc_resid = 0;
        S->dc_steps = 0;
    }
    int64_t taken = 0;
    for (;;) {
        if (S->dc_omega != -1 && S->dc_resid >= t_corr) {
            S->omega = S->dc_omega;
            S->phase = PH_IDLE;
            ev->kind = 0; ev->from_state = S->dc_from; ev->to_state = S->dc_omega; ev->pad = 0;
            ev->resident_steps = S->dc_resid; ev->steps_taken = S->dc_steps;
            return GRO_OK;
        }
        if (taken >= max_steps) return GRO_BUDGET;
        for (int k = 0; k < S->tcd; k++) {
            int rc = step_all(S, 1);
            if (rc) return rc;
            S->tsim += 1;
        }
        taken += S->tcd;
        S->dc_steps += S->tcd;
        int st = gro_state_of(S, Q(S, 0));
        if (st == S->dc_omega) {
            S->dc_resid += S->tcd;
        } else if (S->dc_omega == -1) {
            S->dc_omega = st;              /* entered a state: t_reach ends here */
            S->dc_resid = 0;
        } else {
            ev->kind = 1; ev->from_state = S->dc_omega; ev->to_state = st; ev->pad = 0;
            ev->resident_steps = S->dc_resid + S->tcd; ev->steps_taken = S->dc_steps;
            S->omega = st;
            S->phase = PH_IDLE;
            return GRO_OK;
        }
    }
}

/* ------------------------------------------------------------------ convergence step
 * Sec. 2.4.1 with the clock updates that follow Eq. 4.  Readings: the workers start as
 * copies of the reference walker (its configuration is broadcast); the reference walker
 * is neither averaged nor a donor; observables are sampled every t_GR steps (right end of
 * each interval); at a check the reference-exit test comes first, then branching, then
 * the R-hat test; if every worker exits at once they are all re-copied from the reference
 * walker and the accumulators restart. */
static void dephase_reset_workers(gro_sys *S)
{
    for (int r = 1; r < S->R; r++) copy_replica(S, r, 0);
    memset(S->S1, 0, sizeof(double) * (size_t)S->R * GRO_NMAXOBS);
    memset(S->S2, 0, sizeof(double) * (size_t)S->R * GRO_NMAXOBS);
    S->nsamp = 0;
}

static void accumulate_workers(gro_sys *S)
{
    double o[GRO_NMAXOBS];
    for (int r = 1; r < S->R; r++) {
        obs_of_replica(S, r, o);
        for (int j = 0; j < S->nobs; j++) {
            double x = o[j] - S->shift[j];
            S->S1[r * GRO_NMAXOBS + j] += x;
            S->S2[r * GRO_NMAXOBS + j] += x * x;
        }
    }
    S->nsamp += 1;
}

static int rhat_workers(gro_sys *S, double *rh)
{
    int nw = S->R - 1, no = S->nobs;
    double *a = (double *)malloc(sizeof(double) * (size_t)(nw * (no ? no : 1)));
    double *b = (double *)malloc(sizeof(double) * (size_t)(nw * (no ? no : 1)));
    if (!a || !b) { free(a); free(b); return GRO_ENOMEM; }
    for (int k = 0; k < nw; k++)
        for (int j = 0; j < no; j++) {
            a[k * no + j] = S->S1[(k + 1) * GRO_NMAXOBS + j];
            b[k * no + j] = S->S2[(k + 1) * GRO_NMAXOBS + j];
        }
    int rc = GRO_OK;
    if (S->nsamp >= 1) rc = gro_rhat(nw, no, S->nsamp, a, b, rh);
    else for (int j = 0; j < no; j++) rh[j] = INFINITY;
    free(a); free(b);
    return rc;
}

int gro_dephase(gro_sys *S, int64_t max_steps, gro_dephase_result *o)
{
    if (S->phase != PH_DEPHASE) {
        if (S->omega == -1) { set_err("reference walker is in no state"); return GRO_EPHASE; }
        dephase_reset_workers(S);
        double o0[GRO_NMAXOBS];
        obs_of_replica(S, 0, o0);
        for (int j = 0; j < S->nobs; j++) S->shift[j] = o0[j];
        S->dp_t = 0;
        S->n_branch = 0;
        S->phase = PH_DEPHASE;
    }
    uint8_t *ex = (uint8_t *)malloc(S->R);
    int32_t *donor = (int32_t *)malloc(sizeof(int32_t) * S->R);
    if (!ex || !donor) { free(ex); free(donor); return GRO_ENOMEM; }
    int64_t taken = 0;
    int rc = GRO_BUDGET;
    while (taken < max_steps) {
        int e = step_all(S, S->R);
        if (e) { rc = e; break; }
        S->dp_t += 1;
        taken += 1;
        if (S->dp_t % S->t_gr == 0) accumulate_workers(S);
        if (S->dp_t % S->tcd != 0) continue;
        int st0 = gro_state_of(S, Q(S, 0));
        if (st0 != S->omega) {
            S->tsim += S->dp_t;
            o->outcome = 1; o->to_state = st0; o->t_steps = S->dp_t;
            o->n_branch = S->n_branch; o->n_samples = S->nsamp;
            rhat_workers(S, o->rhat);
            S->omega = st0;
            S->phase = PH_IDLE;
            rc = GRO_OK;
            break;
        }
        for (int r = 0; r < S->R; r++) ex[r] = (uint8_t)(r > 0 && gro_state_of(S, Q(S, r)) != S->omega);
        gro_fv_plan(S->seed, S->s, S->R, ex, donor);
        if (S->R > 1 && donor[1] == -2) {
            S->n_branch += S->R - 1;
            dephase_reset_workers(S);
        } else {
            for (int r = 1; r < S->R; r++) {
                if (donor[r] < 0) continue;
                int j = donor[r];
                copy_replica(S, r, j);
                for (int k = 0; k < S->nobs; k++) {
                    S->S1[r * GRO_NMAXOBS + k] = S->S1[j * GRO_NMAXOBS + k];
                    S->S2[r * GRO_NMAXOBS + k] = S->S2[j * GRO_NMAXOBS + k];
                }
                S->n_branch += 1;
            }
        }
        double rh[GRO_NMAXOBS];
        rhat_workers(S, rh);
        int conv = S->dp_t >= S->t_min && S->nsamp >= 2;
        for (int j = 0; j < S->nobs && conv; j++) conv = rh[j] < 1.0 + S->tol;
        if (conv) {
            S->tsim += S->dp_t;
            o->outcome = 0; o->to_state = S->omega; o->t_steps = S->dp_t;
            o->n_branch = S->n_branch; o->n_samples = S->nsamp;
            for (int j = 0; j < S->nobs; j++) o->rhat[j] = rh[j];
            S->phase = PH_CONVERGED;
            rc = GRO_OK;
            break;
        }
    }
    free(ex); free(donor);
    return rc;
}

/* ------------------------------------------------------------------ original ParRep dephasing
 * The dephasing of the original ParRep algorithm (Sec. 2.4.3), which Gen.ParRep replaces by
 * the Fleming-Viot process: every replica starts from the reference walker's configuration
 * and is propagated within Omega; its end point is kept as a sample of the QSD once it has
 * stayed in Omega for t_phase.  Readings: the reference walker is one of the R samples; exits
 * are tested every t_check_dephase steps; a replica found outside Omega at a check restarts
 * from the configuration the reference walker had when the dephasing began (its noise goes
 * on with the global step counter); a replica that has stayed t_phase keeps the state it had
 * at that check as its sample (it goes on moving with the others, and what it does then is
 * discarded); when every replica has its sample, all are set to their samples.  The
 * dephasing time is not added to the simulation clock (the samples are prepared in parallel
 * and their time is discarded). */
static void save_replica(const gro_sys *S, int r, double *dst, double *dstU)
{
    const size_t b = sizeof(double) * 3 * (size_t)S->n;
    memcpy(dst, Q(S, r), b);
    memcpy(dst + 3 * S->n, Vv(S, r), b);
    memcpy(dst + 6 * S->n, Ff(S, r), b);
    *dstU = S->U[r];
}

static void load_replica(gro_sys *S, int r, const double *src, double U)
{
    const size_t b = sizeof(double) * 3 * (size_t)S->n;
    memcpy(Q(S, r), src, b);
    memcpy(Vv(S, r), src + 3 * S->n, b);
    memcpy(Ff(S, r), src + 6 * S->n, b);
    S->U[r] = U;
}

int gro_dephase_fixed(gro_sys *S, int64_t t_phase, int64_t max_steps, gro_dephase_result *o)
{
    const size_t per = (size_t)9 * S->n;      /* q, v, F of one replica */
    if (S->phase != PH_DEPHASE_FIXED) {
        if (S->omega == -1) { set_err("reference walker is in no state"); return GRO_EPHASE; }
        if (t_phase < 0) { set_err("t_phase < 0"); return GRO_EINVAL; }
        save_replica(S, 0, S->snap, &S->snapU);
        for (int r = 1; r < S->R; r++) copy_replica(S, r, 0);
        for (int r = 0; r < S->R; r++) { S->resid[r] = 0; S->done[r] = 0; }
        S->dp_t = 0;
        S->n_branch = 0;
        S->phase = PH_DEPHASE_FIXED;
    }
    int64_t taken = 0;
    while (taken < max_steps) {
        int e = step_all(S, S->R);
        if (e) return e;
        S->dp_t += 1;
        taken += 1;
        if (S->dp_t % S->tcd != 0) continue;
        int all = 1;
        for (int r = 0; r < S->R; r++) {
            if (S->done[r]) continue;
            if (gro_state_of(S, Q(S, r)) != S->omega) {
                load_replica(S, r, S->snap, S->snapU);
                S->resid[r] = 0;
                S->n_branch += 1;
                all = 0;
            } else {
                S->resid[r] += S->tcd;
                if (S->resid[r] >= t_phase) {
                    save_replica(S, r, S->samp + (size_t)r * per, &S->sampU[r]);
                    S->done[r] = 1;
                } else {
                    all = 0;
                }
            }
        }
        if (all) {
            for (int r = 0; r < S->R; r++) load_replica(S, r, S->samp + (size_t)r * per, S->sampU[r]);
            o->outcome = 0; o->to_state = S->omega; o->t_steps = S->dp_t;
            o->n_branch = S->n_branch; o->n_samples = 0;
            for (int j = 0; j < GRO_NMAXOBS; j++) o->rhat[j] = 0.0;
            S->phase = PH_CONVERGED;
            return GRO_OK;
        }
    }
    return GRO_BUDGET;
}

/* ------------------------------------------------------------------ parallel step
 * Sec. 2.4.2: the R dephased samples (reference walker included) step independently;
 * the exit test is done every t_check_parallel steps; at the first check M with an exit,
 * k is the smallest 1-based index among the exited replicas, tau = (R(M-1)+k) t_check
 * (Eq. 5), t_sim += tau (Eq. 6) and the exit configuration of replica k becomes the new
 * starting point of the reference walker. */
int gro_parallel_step(gro_sys *S, int64_t max_checks, gro_exit_result *o)
{
    if (S->phase == PH_CONVERGED) { S->phase = PH_PARALLEL; S->par_M = 0; }
    else if (S->phase != PH_PARALLEL) { set_err("parallel step needs a converged dephasing"); return GRO_EPHASE; }
    int64_t *fec = (int64_t *)malloc(sizeof(int64_t) * S->R);
    if (!fec) return GRO_ENOMEM;
    int64_t checks = 0;
    int rc = GRO_BUDGET;
    while (checks < max_checks) {
        int e = GRO_OK;
        for (int k = 0; k < S->tcp && e == GRO_OK; k++) e = step_all(S, S->R);
        if (e) { rc = e; break; }
        S->par_M += 1;
        checks += 1;
        /* first exit check of each replica: earlier checks found none, so every replica
         * outside Omega now first left it at check M; Eq. 5 then picks (M, k, tau) */
        for (int r = 0; r < S->R; r++) fec[r] = gro_state_of(S, Q(S, r)) != S->omega ? S->par_M : 0;
        int64_t M, tau;
        int32_t k;
        if (gro_exit_vote(S->R, fec, S->tcp, &M, &k, &tau) != GRO_OK) continue;
        S->tsim += tau;
        if (k != 1) copy_replica(S, 0, k - 1);
        int st = gro_state_of(S, Q(S, 0));
        o->M = M; o->k = k; o->to_state = st; o->tau_steps = tau; o->tau = (double)tau * S->dt;
        S->omega = st;
        S->phase = PH_IDLE;
        rc = GRO_OK;
        break;
    }
    free(fec);
    return rc;
}

/* ------------------------------------------------------------------ fixed-work stepping
 * All replicas step nsteps; observables of the workers are accumulated every t_GR and
 * every replica is tested every t_check_dephase; nothing is acted on.  The schedule runs on
 * the steps taken by every call since creation (adv_t), so that several short calls sample
 * and test as one long call would; fec[r] receives the index (counted over all calls) of
 * the first check of this call that found replica r outside Omega, 0 if none. */
int gro_advance(gro_sys *S, int64_t nsteps, int64_t *fec)
{
    int64_t *first = (int64_t *)calloc(S->R, sizeof(int64_t));
    if (!first) return GRO_ENOMEM;
    for (int64_t k = 0; k < nsteps; k++) {
        int e = step_all(S, S->R);
        if (e) { free(first); return e; }
        const int64_t t = ++S->adv_t;
        if (t % S->t_gr == 0) accumulate_workers(S);
        if (t % S->tcd == 0) {
            for (int r = 0; r < S->R; r++)
                if (first[r] == 0 && gro_state_of(S, Q(S, r)) != S->omega) first[r] = t / S->tcd;
            double rh[GRO_NMAXOBS];
            rhat_workers(S, rh);
        }
    }
    if (fec) memcpy(fec, first, sizeof(int64_t) * S->R);
    free(first);
    return GRO_OK;
}

/* ------------------------------------------------------------------ sampled stepping
 * Steps only replicas [r_lo, r_hi) for nsteps ticks of the global clock.  Replicas do not
 * interact between checks, so these replicas follow exactly the trajectory they would
 * have in a full run; used to compare sampled replicas of large systems. */
int gro_step_replicas(gro_sys *S, int64_t nsteps, int32_t r_lo, int32_t r_hi)
{
    if (r_lo < 0 || r_hi > S->R || r_lo > r_hi || nsteps < 0) { set_err("replica range"); return GRO_EINVAL; }
    for (int64_t t = 0; t < nsteps; t++) {
        for (int r = r_lo; r < r_hi; r++) step_replica(S, r, S->s);
        S->s += 1;
        for (int r = r_lo; r < r_hi; r++)
            if (!isfinite(S->U[r])) { set_err("non-finite energy"); return GRO_EUNSTABLE; }
    }
    return GRO_OK;
}
