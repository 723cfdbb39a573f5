/*
 * lb2p_oracle.h -- plain FP64 CPU oracle of the consistent two-phase lattice
 * Boltzmann step (Zelko & Duenweg, "Consistent two-phase Lattice Boltzmann
 * model for gas-liquid systems", arXiv:1402.2920).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library includes, links or
 * calls this code; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no header, table or helper with the HIP path.
 *
 * Conventions (oracle side):
 *   - lattice units h = a = 1 (Tables I and II);
 *   - site index s = x + nx*(y + ny*z), periodic in every direction;
 *   - populations n[i*N + s] are the PRE-collision populations n_i(r,t) of the
 *     lattice Boltzmann equation (Sec. II, eq. "boltzmann");
 *   - vector fields are stored per site as 3 doubles (z component 0 in 2D),
 *     rank-2 tensors as 3x3 and rank-3 tensors as 3x3x3 row-major blocks.
 */
#ifndef LB2P_ORACLE_H
#define LB2P_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int Q;              /* 21 (D2Q21, needs nz == 1) or 59 (D3Q59)              */
    int nx, ny, nz;
    double gamma;       /* BGK relaxation parameter, -1 < gamma < 1 (Sec. II)  */
    double kappa;       /* interfacial stiffness (Sec. II, Cahn-Hilliard term) */
    double rho1, rho2, A, cs2_1;   /* EOS construction of App. B             */
    double rho0;        /* fixed reference density of Delta^int, Delta^corr   */
    double tol;         /* j~ iteration: stop when max|j~new - j~|
                           <= tol * max|j0'|  (all sites, all components)      */
    int max_iter;       /* iteration cap                                       */
    int flags;          /* ORC_NO_CORR: drop Delta^corr and j~ (textbook BGK)  */
} orc_params;

#define ORC_NO_CORR 1
#define ORC_STENCIL_CLOSURE 2   /* items 10-11: the derivatives of X, T, Y taken
                                   with the product rule, second derivatives of p
                                   and u by the Table III Laplacian and traceless
                                   stencils (Secs. IV C-D); the Supplemental
                                   preamble allows moving the operators so */

/* Per-step diagnostics of the implicit velocity solve. */
typedef struct {
    int iters;          /* iterations used in the last step                   */
    double resid;       /* last max|j~new - j~|                               */
    double jscale;      /* max|j0'| used to scale the stop rule               */
    int converged;      /* 1 if the stop rule was met before max_iter         */
} orc_info;

/* d_a d_b g of a scalar field g[N] at every site from the Table III
 * second-derivative stencils (Secs. IV C-D): H[9*s + 3*a + b]. */
void orc_hessian(const orc_params *P, const double *g, double *H);

/* Velocity set: fills c[Q*3] and shell[Q]; returns Q or -1. */
int orc_velocities(int Q, int *c, int *shell);

/* Shell weights w_k(sigma2) of Table I / II expanded to all Q velocities. */
int orc_weights(int Q, double sigma2, double *w);

/* EOS of App. B at one density: out = {cs2, p, dp/drho, P1, P2, psi}. */
void orc_eos(const orc_params *P, double rho, double *out);

/* n_eq of eq. (equilibrium) at one site, local weights. */
void orc_equilibrium(const orc_params *P, double rho, const double *u, double *neq);

/* Initial populations n_i = n_eq(rho(r), u(r)); u holds 3 doubles per site. */
void orc_init(const orc_params *P, const double *rho, const double *u, double *n);

/* Items 1-8 of the supplemental algorithm on the current state n.
 * Outputs (any may be NULL): rho[N], j0[3N], f[3N], jt[3N] (converged j~),
 * u[3N] (hydrodynamic velocity j/rho).  Returns 0 on convergence, 1 if the
 * iteration hit max_iter. */
int orc_fields(const orc_params *P, const double *n, double *rho, double *j0,
               double *f, double *jt, double *u, orc_info *info);

/* Items 9-11: closure tensors from the converged fields rho, j = rho u and
 * j~: Sigma[9N] (3x3 per site) and Xi'[27N] (3x3x3 per site). */
void orc_closure(const orc_params *P, const double *rho, const double *j,
                 const double *jt, double *Sigma, double *Xip);

/* Per-site collision terms (item 11, per velocity). */
void orc_site_collision(const orc_params *P, const double *n_site, double rho,
                        const double *u, const double *f, const double *jt,
                        const double *Sigma, const double *Xip,
                        double *d_bulk, double *d_int, double *d_corr);

/* nsteps full steps (items 1-12): n is replaced by the new pre-collision
 * populations.  Returns 0, or 1 if any step's iteration did not converge. */
int orc_step(const orc_params *P, double *n, int nsteps, orc_info *info);

/* Single-site summed moments: mass and momentum of n (FP64). */
void orc_totals(const orc_params *P, const double *n, double *mass, double *mom);

/* One pass of the j~ map for a given field j~ (items 3-5); out = j~new. */
void orc_jtilde_map(const orc_params *P, const double *rho, const double *j0p,
                    const double *jt, double *jt_new);

int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
