/*
 * lb2p_oracle.c -- plain FP64 CPU oracle of the consistent two-phase lattice
 * Boltzmann method of Zelko & Duenweg (arXiv:1402.2920).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark.  The GPU library never includes, links or calls
 * it, and it shares no code or table with the GPU path.
 *
 * The step follows the paper's Supplemental Material, items 1-12, in order:
 * every item that says "at each lattice site" is a complete sweep over the
 * lattice before the next item starts.  Loops are plain; the only
 * parallelism is an OpenMP split of independent site loops.
 *
 * Readings where the paper is silent or misprinted (each is also listed in
 * the design notes of the repository):
 *   R1  Table I's rest weight w0 is misprinted; w0 is taken from the
 *       normalisation sum_i w_i = 1 (Sec. III, eq. tensor0_revised).
 *   R2  n_eq uses the local weights w_i(c_s^2(rho)); Delta^int and
 *       Delta^corr use W_i = w_i(c0^2), c0^2 = c_s^2(rho0) at the fixed
 *       reference density rho0 (Secs. VI, VIII; Supplemental item 11).
 *   R3  The c_s^2 multiplying j~ in Xi' is c0^2 (Sec. VIII), the value that
 *       makes the third moment of Delta^corr equal to Xi.
 *   R4  Every derivative of items 4, 5, 10, 11 uses the first-derivative
 *       stencil of Sec. IV B; the force uses the stencil of Sec. IV E.
 *   R5  Products are formed per site before they are differentiated.
 *   R6  The j~ iteration starts from zero and stops when
 *       max_r |j~new - j~| <= tol * max_r |j0'| (component max norm).
 *   R8  Streaming is the push form of Supplemental item 11.
 *   R9  Initial populations are n_eq(rho, u) with local weights.
 *   R10 psi and psi' vanish for rho <= rho1 and rho >= rho3 (App. B).
 */
#include "lb2p_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Shells and stencils                                                       */
/* ------------------------------------------------------------------------ */

/* A vector belongs to the shell of representative `rep` when its absolute
 * components are a permutation of rep (Tables I-III list one representative
 * per shell).  Vectors are enumerated in lexicographic order of (x, y, z)
 * from -4 to 4, shell by shell. */
static int in_shell(int dim, const int *v, const int *rep)
{
    int a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) { a[k] = abs(v[k]); b[k] = rep[k]; }
    /* sort both descending */
    for (int i = 0; i < dim; ++i)
        for (int j = i + 1; j < dim; ++j) {
            if (a[j] > a[i]) { int t = a[i]; a[i] = a[j]; a[j] = t; }
            if (b[j] > b[i]) { int t = b[i]; b[i] = b[j]; b[j] = t; }
        }
    for (int k = 0; k < dim; ++k) if (a[k] != b[k]) return 0;
    return 1;
}

/* Expand shells into vectors; returns the count. */
static int expand_shells(int dim, int nshell, const int reps[][3],
                         int (*out)[3], int *shell_of)
{
    int n = 0;
    for (int k = 0; k < nshell; ++k) {
        int zr = (dim == 3) ? 4 : 0;
        for (int x = -4; x <= 4; ++x)
            for (int y = -4; y <= 4; ++y)
                for (int z = -zr; z <= zr; ++z) {
                    int v[3] = {x, y, z};
                    if (in_shell(dim, v, reps[k])) {
                        out[n][0] = x; out[n][1] = y; out[n][2] = z;
                        if (shell_of) shell_of[n] = k;
                        ++n;
                    }
                }
    }
    return n;
}

/* Table I (D3Q59) and Table II (D2Q21) shell representatives. */
static const int REP3[8][3] = {{0,0,0},{1,0,0},{1,1,0},{1,1,1},
                               {2,0,0},{2,2,0},{2,2,2},{4,0,0}};
static const int REP2[6][3] = {{0,0,0},{1,0,0},{1,1,0},{2,0,0},
                               {2,2,0},{4,0,0}};

int orc_velocities(int Q, int *c, int *shell)
{
    int v[64][3], sh[64], n;
    if (Q == 59) n = expand_shells(3, 8, REP3, v, sh);
    else if (Q == 21) n = expand_shells(2, 6, REP2, v, sh);
    else return -1;
    if (n != Q) return -1;
    for (int i = 0; i < n; ++i) {
        if (c) { c[3*i] = v[i][0]; c[3*i+1] = v[i][1]; c[3*i+2] = v[i][2]; }
        if (shell) shell[i] = sh[i];
    }
    return n;
}

/* Shell weights as functions of sigma2 = c_s^2 (Tables I and II). */
static void shell_weights(int Q, double s, double *wk)
{
    if (Q == 59) {
        wk[1] = 2.0 * s * (8.0/45.0 - s/3.0 + s*s/6.0);
        wk[2] = s * (8.0/45.0 - s/3.0 + s*s/6.0);
        wk[3] = s / 12.0 * (-16.0/15.0 + 4.0*s - 2.5*s*s);
        wk[4] = s / 96.0 * (-24.0/5.0 + 17.0*s - 9.0*s*s);
        wk[5] = s / 192.0 * (-8.0/15.0 + s + s*s);
        wk[6] = s / 192.0 * (4.0/15.0 - s + s*s);
        wk[7] = s / 384.0 * (4.0/15.0 - s + s*s);
        /* R1: w0 from the normalisation sum_i w_i = 1; shell sizes
         * 6, 12, 8, 6, 12, 8, 6 (Table I, column b). */
        wk[0] = 1.0 - (6*wk[1] + 12*wk[2] + 8*wk[3] + 6*wk[4]
                       + 12*wk[5] + 8*wk[6] + 6*wk[7]);
    } else {
        wk[0] = 1.0 - 22.5 * s * (7.0/60.0 - 7.0/48.0*s + s*s/16.0);
        wk[1] = s / 3.0 * (32.0/15.0 - 4.0*s + 2.0*s*s);
        wk[2] = s * (s/3.0 - s*s/4.0);
        wk[3] = s * (-1.0/18.0 + 3.0/16.0*s - s*s/12.0);
        wk[4] = s / 96.0 * (-0.5*s + 1.5*s*s);
        wk[5] = s / 384.0 * (4.0/15.0 - s + s*s);
    }
}

int orc_weights(int Q, double sigma2, double *w)
{
    int sh[64];
    double wk[8];
    if (orc_velocities(Q, NULL, sh) != Q) return -1;
    shell_weights(Q, sigma2, wk);
    for (int i = 0; i < Q; ++i) w[i] = wk[sh[i]];
    return Q;
}

/* Finite-difference stencils of Table III: vectors d_i and coefficients tau_i. */
typedef struct { int n; int d[32][3]; double tau[32]; } stencil;

static void make_stencil(int dim, int nshell, const int reps[][3],
                         const double *tau, stencil *S)
{
    int v[32][3], sh[32];
    S->n = expand_shells(dim, nshell, reps, v, sh);
    for (int i = 0; i < S->n; ++i) {
        S->d[i][0] = v[i][0]; S->d[i][1] = v[i][1]; S->d[i][2] = v[i][2];
        S->tau[i] = tau[sh[i]];
    }
}

/* Columns "d_alpha d_alpha" (Sec. IV C) and traceless "d_alpha d_beta"
 * (Sec. IV D) of Table III. */
static void second_stencils(int dim, stencil *LAP, stencil *TRL)
{
    if (dim == 3) {
        static const int rl[2][3] = {{0,0,0},{1,0,0}};
        static const double tl[2] = {-6.0, 1.0};
        static const int rt[2][3] = {{1,0,0},{1,1,0}};
        static const double tt[2] = {0.5, 0.25};
        make_stencil(3, 2, rl, tl, LAP);
        make_stencil(3, 2, rt, tt, TRL);
    } else {
        static const int rl[2][3] = {{0,0,0},{1,0,0}};
        static const double tl[2] = {-4.0, 1.0};
        static const int rt[2][3] = {{1,0,0},{1,1,0}};
        static const double tt[2] = {1.0, 0.25};
        make_stencil(2, 2, rl, tl, LAP);
        make_stencil(2, 2, rt, tt, TRL);
    }
}

/* Column "d_alpha" (Sec. IV B) and column "d_alpha d_beta d_beta" (Sec. IV E). */
static void stencils(int dim, stencil *D1, stencil *D3)
{
    if (dim == 3) {
        static const int r1[2][3] = {{1,0,0},{2,0,0}};
        static const double t1[2] = {2.0/3.0, -1.0/24.0};
        static const int r3[3][3] = {{1,0,0},{1,1,0},{2,0,0}};
        static const double t3[3] = {-3.0, 0.5, 0.25};
        make_stencil(3, 2, r1, t1, D1);
        make_stencil(3, 3, r3, t3, D3);
    } else {
        static const int r1[2][3] = {{1,0,0},{2,0,0}};
        static const double t1[2] = {2.0/3.0, -1.0/24.0};
        static const int r3[3][3] = {{1,0,0},{1,1,0},{2,0,0}};
        static const double t3[3] = {-2.0, 0.5, 0.25};
        make_stencil(2, 2, r1, t1, D1);
        make_stencil(2, 3, r3, t3, D3);
    }
}

/* Everything about the lattice that does not change during a run. */
typedef struct {
    int Q, dim;
    int c[64][3];
    int shell[64];
    double W[64];      /* W_i = w_i(c0^2), reference weights (R2) */
    double c0sq;       /* c0^2 = c_s^2(rho0)                       */
    stencil D1, D3;
    stencil LAP, TRL;  /* Laplacian and traceless second derivative */
} lattice;

/* ------------------------------------------------------------------------ */
/* Lattice helpers                                                           */
/* ------------------------------------------------------------------------ */

static int dim_of(const orc_params *P) { return P->Q == 59 ? 3 : 2; }
static long nsites(const orc_params *P) { return (long)P->nx * P->ny * P->nz; }

static long neighbour(const orc_params *P, long s, int dx, int dy, int dz)
{
    long nx = P->nx, ny = P->ny, nz = P->nz;
    long x = s % nx, y = (s / nx) % ny, z = s / (nx * ny);
    x = ((x + dx) % nx + nx) % nx;
    y = ((y + dy) % ny + ny) % ny;
    z = ((z + dz) % nz + nz) % nz;
    return x + nx * (y + ny * z);
}

/* sum_i tau_i d_{i,alpha} g(r + d_i) for component `comp` of a field stored
 * with `stride` doubles per site (Sec. IV, a = 1). */
static double apply_stencil(const orc_params *P, const stencil *S,
                            const double *g, int stride, int comp,
                            long s, int alpha)
{
    double acc = 0.0;
    for (int i = 0; i < S->n; ++i) {
        if (S->d[i][alpha] == 0) continue;
        long t = neighbour(P, s, S->d[i][0], S->d[i][1], S->d[i][2]);
        acc += S->tau[i] * S->d[i][alpha] * g[t * stride + comp];
    }
    return acc;
}

static double delta(int a, int b) { return a == b ? 1.0 : 0.0; }

/* d_a d_b g at site s from the Table III second-derivative stencils: the
 * traceless part sum_i tau_i (d_ia d_ib - d_ab |d_i|^2 / dim) g(r + d_i)
 * (Sec. IV D) plus d_ab / dim times the Laplacian sum_i tau_i g(r + d_i)
 * (Sec. IV C).  H[3a + b] for a, b < dim. */
static void hessian(const orc_params *P, const stencil *LAP, const stencil *TRL, int dim,
                    const double *g, int stride, int comp, long s, double *H)
{
    double lap = 0.0;
    for (int i = 0; i < LAP->n; ++i) {
        long t = neighbour(P, s, LAP->d[i][0], LAP->d[i][1], LAP->d[i][2]);
        lap += LAP->tau[i] * g[t * stride + comp];
    }
    for (int k = 0; k < 9; ++k) H[k] = 0.0;
    for (int i = 0; i < TRL->n; ++i) {
        long t = neighbour(P, s, TRL->d[i][0], TRL->d[i][1], TRL->d[i][2]);
        double v = g[t * stride + comp], dd = 0.0;
        for (int a = 0; a < dim; ++a) dd += TRL->d[i][a] * TRL->d[i][a];
        for (int a = 0; a < dim; ++a)
            for (int b = 0; b < dim; ++b)
                H[3*a + b] += TRL->tau[i] * (TRL->d[i][a] * TRL->d[i][b] - delta(a, b) * dd / dim) * v;
    }
    for (int a = 0; a < dim; ++a) H[4*a] += lap / dim;
}

/* ------------------------------------------------------------------------ */
/* Equation of state (App. B)                                                */
/* ------------------------------------------------------------------------ */

void orc_eos(const orc_params *P, double rho, double *out)
{
    double D = P->rho2 - P->rho1;
    double rho3 = 2.0 * P->rho2 - P->rho1;
    double psi = 0.0, dpsi = 0.0, cs2 = P->cs2_1;
    if (rho > P->rho1 && rho < rho3) {
        double th = M_PI * (rho - P->rho1) / D;
        psi = P->A * sin(th);
        dpsi = P->A * M_PI / D * cos(th);
        /* c_s^2(rho) = c_s^2(rho1) exp(int_{rho1}^{rho} psi) */
        cs2 = P->cs2_1 * exp(P->A * D / M_PI * (1.0 - cos(th)));
    }
    double p = rho * cs2;                       /* p = rho c_s^2                 */
    double dp = cs2 * (1.0 + rho * psi);        /* (rho/p) dp/drho = 1 + rho psi */
    double P1 = p - rho * dp;                   /* p - rho dp/drho               */
    double P2 = rho * cs2 * (psi * (2.0 + rho * psi) + rho * dpsi); /* rho d2p/drho2 */
    out[0] = cs2; out[1] = p; out[2] = dp; out[3] = P1; out[4] = P2; out[5] = psi;
}

static double cs2_of(const orc_params *P, double rho)
{
    double e[6];
    orc_eos(P, rho, e);
    return e[0];
}

static void lattice_setup(const orc_params *P, lattice *L)
{
    int c[64 * 3];
    L->Q = P->Q;
    L->dim = dim_of(P);
    orc_velocities(P->Q, c, L->shell);
    for (int i = 0; i < P->Q; ++i)
        for (int a = 0; a < 3; ++a) L->c[i][a] = c[3*i + a];
    L->c0sq = cs2_of(P, P->rho0);
    orc_weights(P->Q, L->c0sq, L->W);
    stencils(L->dim, &L->D1, &L->D3);
    second_stencils(L->dim, &L->LAP, &L->TRL);
}

/* ------------------------------------------------------------------------ */
/* Equilibrium (Sec. III, eq. equilibrium) and initial state                 */
/* ------------------------------------------------------------------------ */

static void equilibrium(const orc_params *P, const lattice *L, double rho,
                        const double *u, double *neq)
{
    double wk[8];
    double cs2 = cs2_of(P, rho);
    shell_weights(L->Q, cs2, wk);          /* local weights w_i(rho) (R2) */
    double uu = u[0]*u[0] + u[1]*u[1] + u[2]*u[2];
    for (int i = 0; i < L->Q; ++i) {
        double uc = u[0]*L->c[i][0] + u[1]*L->c[i][1] + u[2]*L->c[i][2];
        neq[i] = wk[L->shell[i]] * rho * (1.0 + uc / cs2 + uc * uc / (2.0 * cs2 * cs2)
                                          - uu / (2.0 * cs2));
    }
}

void orc_equilibrium(const orc_params *P, double rho, const double *u, double *neq)
{
    lattice L;
    lattice_setup(P, &L);
    equilibrium(P, &L, rho, u, neq);
}

void orc_init(const orc_params *P, const double *rho, const double *u, double *n)
{
    long N = nsites(P);
    lattice L;
    lattice_setup(P, &L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < N; ++s) {
        double neq[64];
        equilibrium(P, &L, rho[s], &u[3*s], neq);
        for (int i = 0; i < L.Q; ++i) n[(long)i * N + s] = neq[i];
    }
}

/* ------------------------------------------------------------------------ */
/* Items 3-5: one pass of the correction-current map                         */
/* ------------------------------------------------------------------------ */

/* Given j~ (jt), compute j~new:
 *   u = (j0' + j~)/rho                                              (item 3)
 *   q_ab = (p - rho dp/drho) d_ab d_g u_g + p (d_b u_a + d_a u_b)   (item 4)
 *   j~new_a = -(h^2/12) d_b q_ab                                    (item 5) */
static void jtilde_map(const orc_params *P, const lattice *L, const double *rho,
                       const double *j0p, const double *jt, double *jt_new,
                       double *u, double *q)
{
    long N = nsites(P);
    int dim = L->dim;

#pragma omp parallel for schedule(static)
    for (long s = 0; s < N; ++s)
        for (int a = 0; a < 3; ++a)
            u[3*s + a] = (j0p[3*s + a] + jt[3*s + a]) / rho[s];

#pragma omp parallel for schedule(static)
    for (long s = 0; s < N; ++s) {
        double e[6], G[3][3] = {{0}}, trG = 0.0;
        orc_eos(P, rho[s], e);
        double p = e[1], P1 = e[3];
        for (int a = 0; a < dim; ++a)          /* G[a][b] = d_a u_b */
            for (int b = 0; b < dim; ++b)
                G[a][b] = apply_stencil(P, &L->D1, u, 3, b, s, a);
        for (int g = 0; g < dim; ++g) trG += G[g][g];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                q[9*s + 3*a + b] = (a < dim && b < dim)
                    ? P1 * delta(a, b) * trG + p * (G[b][a] + G[a][b]) : 0.0;
    }

#pragma omp parallel for schedule(static)
    for (long s = 0; s < N; ++s)
        for (int a = 0; a < 3; ++a) {
            double acc = 0.0;
            if (a < dim)
                for (int b = 0; b < dim; ++b)
                    acc += apply_stencil(P, &L->D1, q, 9, 3*a + b, s, b);
            jt_new[3*s + a] = -acc / 12.0;
        }
}

void orc_jtilde_map(const orc_params *P, const double *rho, const double *j0p,
                    const double *jt, double *jt_new)
{
    long N = nsites(P);
    lattice L;
    lattice_setup(P, &L);
    double *u = (double *)calloc((size_t)N * 3, sizeof(double));
    double *q = (double *)calloc((size_t)N * 9, sizeof(double));
    jtilde_map(P, &L, rho, j0p, jt, jt_new, u, q);
    free(u);
    free(q);
}

/* ------------------------------------------------------------------------ */
/* Items 1-8                                                                 */
/* ------------------------------------------------------------------------ */

int orc_fields(const orc_params *P, const double *n, double *rho_o, double *j0_o,
               double *f_o, double *jt_o, double *u_o, orc_info *info)
{
    long N = nsites(P);
    lattice L;
    lattice_setup(P, &L);
    int Q = L.Q, dim = L.dim;

    double *rho = (double *)calloc((size_t)N, sizeof(double));
    double *j0 = (double *)calloc((size_t)N * 3, sizeof(double));
    double *f = (double *)calloc((size_t)N * 3, sizeof(double));
    double *j0p = (double *)calloc((size_t)N * 3, sizeof(double));
    double *jt = (double *)calloc((size_t)N * 3, sizeof(double));
    double *jtn = (double *)calloc((size_t)N * 3, sizeof(double));
    double *uw = (double *)calloc((size_t)N * 3, sizeof(double));
    double *qw = (double *)calloc((size_t)N * 9, sizeof(double));

    /* Item 1: rho = sum_i n_i, j0 = sum_i n_i c_i (j~ = 0 is set below). */
#pragma omp parallel for schedule(static)
    for (long s = 0; s < N; ++s) {
        double r = 0.0, m[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; ++i) {
            double ni = n[(long)i * N + s];
            r += ni;
            for (int a = 0; a < 3; ++a) m[a] += ni * L.c[i][a];
        }
        rho[s] = r;
        for (int a = 0; a < 3; ++a) j0[3*s + a] = m[a];
    }

    /* Item 2: f_a = kappa rho d_a d_b d_b rho (Sec. IV E), j0' = j0 + (h/2) f. */
#pragma omp parallel for schedule(static)
    for (long s = 0; s < N; ++s)
        for (int a = 0; a < 3; ++a) {
            double fa = 0.0;
            if (a < dim) fa = P->kappa * rho[s] * apply_stencil(P, &L.D3, rho, 1, 0, s, a);
            f[3*s + a] = fa;
            j0p[3*s + a] = j0[3*s + a] + 0.5 * fa;
        }

    /* Items 3-8: fixed-point iteration for j~, started from zero (R6). */
    double jscale = 0.0;
    for (long k = 0; k < 3 * N; ++k) {
        double ak = fabs(j0p[k]);
        if (!(ak <= jscale) && jscale == jscale) jscale = ak;   /* a NaN, once seen, stays */
    }
    int iters = 0, converged = 0;
    double resid = 0.0;
    if (!(P->flags & ORC_NO_CORR)) {
        while (iters < P->max_iter) {
            jtilde_map(P, &L, rho, j0p, jt, jtn, uw, qw);          /* items 3-5 */
            ++iters;
            resid = 0.0;                                            /* item 6    */
            for (long k = 0; k < 3 * N; ++k) {
                double dk = fabs(jtn[k] - jt[k]);
                if (!(dk <= resid) && resid == resid) resid = dk;   /* a NaN, once seen, stays */
            }
            memcpy(jt, jtn, sizeof(double) * 3 * (size_t)N);        /* items 7, 8 */
            if (resid <= P->tol * jscale) { converged = 1; break; }
            if (resid != resid) break;               /* non-finite: give up  */
        }
    } else {
        converged = 1;   /* j~ = 0 identically when the correction is off */
    }

    /* Item 8: j = j0' + j~, u = j / rho. */
    if (rho_o) memcpy(rho_o, rho, sizeof(double) * (size_t)N);
    if (j0_o) memcpy(j0_o, j0, sizeof(double) * 3 * (size_t)N);
    if (f_o) memcpy(f_o, f, sizeof(double) * 3 * (size_t)N);
    if (jt_o) memcpy(jt_o, jt, sizeof(double) * 3 * (size_t)N);
    if (u_o)
        for (long s = 0; s < N; ++s)
            for (int a = 0; a < 3; ++a)
                u_o[3*s + a] = (j0p[3*s + a] + jt[3*s + a]) / rho[s];
    if (info) {
        info->iters = iters; info->resid = resid;
        info->jscale = jscale; info->converged = converged;
    }
    free(rho); free(j0); free(f); free(j0p); free(jt); free(jtn); free(uw); free(qw);
    return converged ? 0 : 1;
}

/* ------------------------------------------------------------------------ */
/* Items 9-11: closure tensors Sigma and Xi'                                 */
/* ------------------------------------------------------------------------ */

void orc_closure(const orc_params *P, const double *rho, const double *j,
                 const double *jt, double *Sigma, double *Xip)
{
    long N = nsites(P);
    lattice L;
    lattice_setup(P, &L);
    int dim = L.dim;
    const stencil *D1 = &L.D1;
    double g = P->gamma;
    double c0sq = L.c0sq;

    double *u = (double *)calloc((size_t)N * 3, sizeof(double));
    double *pf = (double *)calloc((size_t)N, sizeof(double));      /* p            */
    double *P1f = (double *)calloc((size_t)N, sizeof(double));     /* p - rho p'   */
    double *por = (double *)calloc((size_t)N, sizeof(double));     /* p/rho        */
    double *puu = (double *)calloc((size_t)N * 9, sizeof(double)); /* p u_b u_g    */
    double *G = (double *)calloc((size_t)N * 9, sizeof(double));   /* d_a u_b      */
    double *J = (double *)calloc((size_t)N * 9, sizeof(double));   /* d_a j_b      */
    double *Pg = (double *)calloc((size_t)N * 3, sizeof(double));  /* d_a p        */
    double *M = (double *)calloc((size_t)N * 27, sizeof(double));  /* d_a(p u_b u_g) */
    double *C = (double *)calloc((size_t)N * 3, sizeof(double));   /* d_a(p/rho)   */
    double *X = (double *)calloc((size_t)N, sizeof(double));
    double *T = (double *)calloc((size_t)N * 9, sizeof(double));
    double *Y = (double *)calloc((size_t)N * 3, sizeof(double));

    /* Item 9: per-site values and products (R5): u = j/rho, p, p/rho, p u u. */
#pragma omp parallel for schedule(static)
    for (long s = 0; s < N; ++s) {
        double e[6];
        orc_eos(P, rho[s], e);
        for (int a = 0; a < 3; ++a) u[3*s + a] = j[3*s + a] / rho[s];
        pf[s] = e[1];
        P1f[s] = e[3];
        por[s] = e[1] / rho[s];
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c)
                puu[9*s + 3*b + c] = e[1] * u[3*s + b] * u[3*s + c];
    }

    /* Item 10: first-order lattice derivatives. */
#pragma omp parallel for schedule(static)
    for (long s = 0; s < N; ++s) {
        for (int a = 0; a < dim; ++a) {
            for (int b = 0; b < dim; ++b) {
                G[9*s + 3*a + b] = apply_stencil(P, D1, u, 3, b, s, a);
                J[9*s + 3*a + b] = apply_stencil(P, D1, j, 3, b, s, a);
                for (int c = 0; c < dim; ++c)
                    M[27*s + 9*a + 3*b + c] = apply_stencil(P, D1, puu, 9, 3*b + c, s, a);
            }
            Pg[3*s + a] = apply_stencil(P, D1, pf, 1, 0, s, a);
            C[3*s + a] = apply_stencil(P, D1, por, 1, 0, s, a);
        }
    }

    /* Item 11, first part: the per-site fields that are differentiated again:
     *   X    = (p - rho dp/drho) d_g u_g,
     *   T_ag = p (d_a u_g + d_g u_a),
     *   Y_b  = rho^-1 d_b p + u_g d_g u_b. */
#pragma omp parallel for schedule(static)
    for (long s = 0; s < N; ++s) {
        double e[6], trG = 0.0;
        orc_eos(P, rho[s], e);
        for (int a = 0; a < dim; ++a) trG += G[9*s + 4*a];
        X[s] = e[3] * trG;
        for (int a = 0; a < dim; ++a)
            for (int c = 0; c < dim; ++c)
                T[9*s + 3*a + c] = e[1] * (G[9*s + 3*a + c] + G[9*s + 3*c + a]);
        for (int b = 0; b < dim; ++b) {
            double acc = Pg[3*s + b] / rho[s];
            for (int c = 0; c < dim; ++c) acc += u[3*s + c] * G[9*s + 3*c + b];
            Y[3*s + b] = acc;
        }
    }

    double KS1 = -0.25 * (g + 1.0) * (g + 1.0) / (g - 1.0);     /* -h^2/4 (g+1)^2/(g-1)   */
    double KS2 = (g * g + 4.0 * g + 1.0) / (6.0 * (g - 1.0));   /*  h^2/6 (g^2+4g+1)/(g-1) */
    double KX = (g * g + 4.0 * g + 1.0) / (3.0 * (g + 1.0));    /*  h/3 (g^2+4g+1)/(g+1)   */

    /* Item 11, second part: derivatives of X, T, Y and the two tensors. */
#pragma omp parallel for schedule(static)
    for (long s = 0; s < N; ++s) {
        double e[6], DX[3] = {0}, DT[3] = {0}, DY[3][3] = {{0}};
        orc_eos(P, rho[s], e);
        double p = e[1], dp = e[2], P1 = e[3], P2 = e[4];
        const double *us = &u[3*s], *Gs = &G[9*s], *Ms = &M[27*s], *Cs = &C[3*s];
        double trG = 0.0, trJ = 0.0, trDY = 0.0;
        for (int a = 0; a < dim; ++a) { trG += Gs[4*a]; trJ += J[9*s + 4*a]; }
        if (P->flags & ORC_STENCIL_CLOSURE) {
            /* The same three derivatives with the outer operator carried
             * through the products (product rule), so that every second
             * derivative acts on p or on u alone and takes the Table III
             * stencils of Secs. IV C-D (hessian); first derivatives stay
             * Sec. IV B:
             *   d_a X      = (d_a P1) tr G + P1 d_a d_g u_g
             *   d_g T_ag   = (d_g p)(G_ag + G_ga) + p (d_a d_g u_g + d_g d_g u_a)
             *   d_a Y_b    = -rho^-2 (d_a rho)(d_b p) + rho^-1 d_a d_b p
             *                + G_ag G_gb + u_g d_a d_g u_b                     */
            double Hu[3][9] = {{0}}, Hp[9], DP1[3] = {0}, Drho[3] = {0};
            for (int c = 0; c < dim; ++c) hessian(P, &L.LAP, &L.TRL, dim, u, 3, c, s, Hu[c]);
            hessian(P, &L.LAP, &L.TRL, dim, pf, 1, 0, s, Hp);
            for (int a = 0; a < dim; ++a) {
                DP1[a] = apply_stencil(P, D1, P1f, 1, 0, s, a);
                Drho[a] = apply_stencil(P, D1, rho, 1, 0, s, a);
            }
            double ddiv[3] = {0}, lapu[3] = {0};   /* d_a d_g u_g, d_g d_g u_a */
            for (int a = 0; a < dim; ++a)
                for (int c = 0; c < dim; ++c) {
                    ddiv[a] += Hu[c][3*a + c];
                    lapu[a] += Hu[a][3*c + c];
                }
            for (int a = 0; a < dim; ++a) {
                DX[a] = DP1[a] * trG + P1 * ddiv[a];
                DT[a] = p * (ddiv[a] + lapu[a]);
                for (int c = 0; c < dim; ++c)
                    DT[a] += Pg[3*s + c] * (Gs[3*a + c] + Gs[3*c + a]);
                for (int b = 0; b < dim; ++b) {
                    double v = -Drho[a] * Pg[3*s + b] / (rho[s] * rho[s]) + Hp[3*a + b] / rho[s];
                    for (int c = 0; c < dim; ++c)
                        v += Gs[3*a + c] * Gs[3*c + b] + us[c] * Hu[b][3*a + c];
                    DY[a][b] = v;
                }
            }
        } else {
            for (int a = 0; a < dim; ++a) {
                DX[a] = apply_stencil(P, D1, X, 1, 0, s, a);
                for (int c = 0; c < dim; ++c)
                    DT[a] += apply_stencil(P, D1, T, 9, 3*a + c, s, c);
                for (int b = 0; b < dim; ++b)
                    DY[a][b] = apply_stencil(P, D1, Y, 3, b, s, a);
            }
        }
        for (int a = 0; a < dim; ++a) trDY += DY[a][a];

        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double S = 0.0;
                if (a < dim && b < dim) {
                    double br1 = us[a] * DX[b] + us[b] * DX[a]
                               + us[b] * DT[a] + us[a] * DT[b];
                    double br2 = -dp * trJ * (Gs[3*a + b] + Gs[3*b + a])
                               - p * DY[a][b] - p * DY[b][a]
                               - P1 * delta(a, b) * trDY
                               + P2 * delta(a, b) * trG * trJ;
                    S = KS1 * br1 + KS2 * br2;
                }
                Sigma[9*s + 3*a + b] = S;
            }

        /* Xi'_{abg}: the bracket is summed over the three ways of singling out
         * one index, (ab|g), (ag|b), (bg|a). */
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int c = 0; c < 3; ++c) {
                    double X3 = 0.0;
                    if (a < dim && b < dim && c < dim) {
                        double br = Ms[9*c + 3*a + b] + delta(a, b) * (p * Cs[c] + P1 * us[c] * trG)
                                  + Ms[9*b + 3*a + c] + delta(a, c) * (p * Cs[b] + P1 * us[b] * trG)
                                  + Ms[9*a + 3*b + c] + delta(b, c) * (p * Cs[a] + P1 * us[a] * trG);
                        X3 = KX * br + (1.0 - g) * c0sq
                             * (delta(a, b) * jt[3*s + c] + delta(a, c) * jt[3*s + b]
                                + delta(b, c) * jt[3*s + a]);
                    }
                    Xip[27*s + 9*a + 3*b + c] = X3;
                }
    }

    free(u); free(pf); free(P1f); free(por); free(puu); free(G); free(J); free(Pg);
    free(M); free(C); free(X); free(T); free(Y);
}

/* ------------------------------------------------------------------------ */
/* Item 11, per velocity                                                     */
/* ------------------------------------------------------------------------ */

static void site_collision(const orc_params *P, const lattice *L,
                          const double *n_site, double rho, const double *u,
                          const double *f, const double *jt,
                          const double *Sigma, const double *Xip,
                          double *d_bulk, double *d_int, double *d_corr)
{
    int Q = L->Q, dim = L->dim;
    double neq[64];
    double g = P->gamma, c0sq = L->c0sq;
    const double *W = L->W;                          /* W_i = w_i(rho0) (R2) */
    equilibrium(P, L, rho, u, neq);                  /* local weights        */
    int no_corr = P->flags & ORC_NO_CORR;

    for (int i = 0; i < Q; ++i) {
        const int *ci = L->c[i];
        double cf = 0.0, cj = 0.0;
        for (int a = 0; a < dim; ++a) { cf += ci[a] * f[a]; cj += ci[a] * jt[a]; }
        d_bulk[i] = (g - 1.0) * (n_site[i] - neq[i]);
        d_int[i] = 0.5 * (1.0 + g) * W[i] / c0sq * cf;
        double h2 = 0.0, h3 = 0.0;
        for (int a = 0; a < dim; ++a)
            for (int b = 0; b < dim; ++b) {
                h2 += Sigma[3*a + b] * (ci[a] * ci[b] - c0sq * delta(a, b));
                for (int e = 0; e < dim; ++e)
                    h3 += Xip[9*a + 3*b + e]
                          * (ci[a] * ci[b] * ci[e]
                             - c0sq * (delta(a, b) * ci[e] + delta(a, e) * ci[b]
                                       + delta(b, e) * ci[a]));
            }
        d_corr[i] = no_corr ? 0.0
                  : (g - 1.0) * W[i] / c0sq * cj
                    + W[i] / (2.0 * c0sq * c0sq) * h2
                    + W[i] / (6.0 * c0sq * c0sq * c0sq) * h3;
    }
}

void orc_hessian(const orc_params *P, const double *g, double *H)
{
    long N = nsites(P);
    lattice L;
    lattice_setup(P, &L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < N; ++s) hessian(P, &L.LAP, &L.TRL, L.dim, g, 1, 0, s, &H[9*s]);
}

void orc_site_collision(const orc_params *P, const double *n_site, double rho,
                        const double *u, const double *f, const double *jt,
                        const double *Sigma, const double *Xip,
                        double *d_bulk, double *d_int, double *d_corr)
{
    lattice L;
    lattice_setup(P, &L);
    site_collision(P, &L, n_site, rho, u, f, jt, Sigma, Xip, d_bulk, d_int, d_corr);
}

/* ------------------------------------------------------------------------ */
/* Items 1-12                                                                */
/* ------------------------------------------------------------------------ */

int orc_step(const orc_params *P, double *n, int nsteps, orc_info *info)
{
    long N = nsites(P);
    lattice L;
    lattice_setup(P, &L);
    int Q = L.Q;
    double *rho = (double *)malloc(sizeof(double) * (size_t)N);
    double *f = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    double *jt = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    double *u = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    double *j = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    double *Sig = (double *)malloc(sizeof(double) * 9 * (size_t)N);
    double *Xi = (double *)malloc(sizeof(double) * 27 * (size_t)N);
    double *nn = (double *)malloc(sizeof(double) * (size_t)Q * (size_t)N);
    int status = 0;
    orc_info inf = {0, 0.0, 0.0, 1};

    for (int step = 0; step < nsteps; ++step) {
        status |= orc_fields(P, n, rho, NULL, f, jt, u, &inf);     /* items 1-8 */
        for (long s = 0; s < N; ++s)
            for (int a = 0; a < 3; ++a) j[3*s + a] = rho[s] * u[3*s + a];
        if (!(P->flags & ORC_NO_CORR)) {
            orc_closure(P, rho, j, jt, Sig, Xi);                    /* items 9-11 */
        } else {
            memset(Sig, 0, sizeof(double) * 9 * (size_t)N);
            memset(Xi, 0, sizeof(double) * 27 * (size_t)N);
        }
        /* Item 11: collide and push to r + c_i on a new lattice. */
#pragma omp parallel for schedule(static)
        for (long s = 0; s < N; ++s) {
            double ns[64], db[64], di[64], dc[64];
            for (int i = 0; i < Q; ++i) ns[i] = n[(long)i * N + s];
            site_collision(P, &L, ns, rho[s], &u[3*s], &f[3*s], &jt[3*s],
                           &Sig[9*s], &Xi[27*s], db, di, dc);
            for (int i = 0; i < Q; ++i) {
                long t = neighbour(P, s, L.c[i][0], L.c[i][1], L.c[i][2]);
                nn[(long)i * N + t] = ns[i] + db[i] + di[i] + dc[i];
            }
        }
        /* Item 12: the new lattice becomes the current one. */
        memcpy(n, nn, sizeof(double) * (size_t)Q * (size_t)N);
    }
    if (info) *info = inf;
    free(rho); free(f); free(jt); free(u); free(j); free(Sig); free(Xi); free(nn);
    return status ? 1 : 0;
}

void orc_totals(const orc_params *P, const double *n, double *mass, double *mom)
{
    long N = nsites(P);
    lattice L;
    lattice_setup(P, &L);
    double m = 0.0, p[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < L.Q; ++i)
        for (long s = 0; s < N; ++s) {
            double v = n[(long)i * N + s];
            m += v;
            for (int a = 0; a < 3; ++a) p[a] += v * L.c[i][a];
        }
    *mass = m;
    for (int a = 0; a < 3; ++a) mom[a] = p[a];
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
