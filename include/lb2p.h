/*
 * lb2p.h -- C ABI of the MI355X (gfx950) implementation of the consistent
 * two-phase lattice Boltzmann step of Zelko & Duenweg, "Consistent two-phase
 * Lattice Boltzmann model for gas-liquid systems" (arXiv:1402.2920).
 *
 * One call of lb2p_step advances the lattice by one time step h = 1: the
 * Supplemental Material's items 1-12 (moments, equation of state, interface
 * force, the implicit solve for the correction current j~ and the flow
 * velocity u, the closure tensors Sigma and Xi', the bulk, interface and
 * correction collision operators, streaming).  Lattice units h = a = 1
 * (Tables I and II); every boundary is periodic (Sec. VI).
 *
 * Conventions common to every entry point
 *   - Every function returns an lb2p_status; no C++ exception crosses the ABI.
 *   - Site index s = x + nx*(y + ny*z).  Scalar fields are arrays [N], vector
 *     fields are structure-of-arrays [d][N] (d = 2 for D2Q21, 3 for D3Q59).
 *     N = nx*ny*nz (nz = 1 for D2Q21).
 *   - Pointers marked "host or device" are host memory when on_device == 0 and
 *     device memory of the context's GPU when on_device != 0.  The caller owns
 *     them; the library reads/writes them only during the call, which is
 *     synchronous with respect to the caller's buffers (device pointers are
 *     used on the context's stream, which the call synchronises before
 *     returning).
 *   - The context owns all device state (two population buffers and the
 *     per-site fields) until lb2p_destroy.
 *   - Errors LB2P_ENOCONV and LB2P_ENONFINITE are sticky: every later call
 *     reports them until the next lb2p_init / lb2p_set_populations.
 *   - Threads: distinct contexts may be used from different threads at once
 *     (the only state they share, the process-wide cache of tuned tile
 *     shapes, is locked).  Calls on one context must not overlap.
 */
#ifndef LB2P_H
#define LB2P_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LB2P_OK = 0,
    LB2P_EINVAL = 1,      /* bad argument: lattice, grid side < 8, gamma not in
                             (-1,1), kappa < 0, tol < 0, null pointer, ...     */
    LB2P_EEOS = 2,        /* equation of state outside App. B's admissible set,
                             or a reference weight w_i(rho0) not positive      */
    LB2P_ENOCONV = 3,     /* j~ iteration reached max_iter before tol; the step
                             is still taken with the last iterate              */
    LB2P_ENONFINITE = 4,  /* NaN or Inf found in the density                   */
    LB2P_ENOMEM = 5,      /* device allocation failed                          */
    LB2P_EHIP = 6,        /* HIP runtime error                                 */
    LB2P_ESTATE = 7,      /* call out of order (e.g. step before init)        */
    LB2P_ESIZE = 8        /* output larger than the static staging area of
                             lb2p_moments_noalloc                              */
} lb2p_status;

/* Velocity sets of Tables I (D3Q59) and II (D2Q21). */
typedef enum { LB2P_D2Q21 = 21, LB2P_D3Q59 = 59 } lb2p_lattice;

/* Population storage.  F64 computes in FP64; every other form computes in
 * FP32.  BF16/F16 store the moving populations as deviations from
 * o_i = W_i rho_ref scaled by 1/W_i, where W_i are the rest weights at the
 * reference density rho_ref (lb2p_params.store_rho_ref).  In every form the
 * rest population is held apart at higher precision (FP64 beside F64/F32,
 * FP32 beside BF16/F16) and set by the collision from the site's mass
 * balance (sum_i Delta_i = 0, Sec. VI), so the lattice mass is conserved to
 * the rounding of that plane. */
typedef enum {
    LB2P_STORE_F64 = 0,
    LB2P_STORE_F32 = 1,
    LB2P_STORE_BF16 = 2,
    LB2P_STORE_F16 = 3
} lb2p_storage;

/* Element type of caller buffers. */
typedef enum { LB2P_DTYPE_F64 = 0, LB2P_DTYPE_F32 = 1 } lb2p_dtype;

/* Field selectors for lb2p_get_field (state of the last step's items 1-11,
 * or of the last lb2p_moments call).  Tensor components are listed with the
 * field. */
typedef enum {
    LB2P_FIELD_RHO = 0,     /* [N]      density, item 1                       */
    LB2P_FIELD_J0 = 1,      /* [d][N]   sum_i n_i c_i, item 1                 */
    LB2P_FIELD_FORCE = 2,   /* [d][N]   interface force f, item 2             */
    LB2P_FIELD_JTILDE = 3,  /* [d][N]   correction current j~, items 3-8      */
    LB2P_FIELD_U = 4,       /* [d][N]   flow velocity u = j/rho, item 8       */
    LB2P_FIELD_SIGMA = 5,   /* [3][N] 2D: xx yy xy; [6][N] 3D: xx yy zz xy xz yz */
    LB2P_FIELD_XI = 6       /* [4][N] 2D: xxx yyy xxy xyy;
                               [10][N] 3D: xxx yyy zzz xxy xxz xyy xzz yyz yzz xyz */
} lb2p_field;

/* App. B: psi(rho) = A sin(pi (rho-rho1)/(rho2-rho1)) on (rho1, 2 rho2 - rho1),
 * zero elsewhere; c_s^2(rho) = cs2_rho1 exp(int_{rho1}^{rho} psi); p = rho c_s^2. */
typedef struct {
    double rho1, rho2, A, cs2_rho1;
} lb2p_eos;

typedef struct {
    int lattice;            /* lb2p_lattice                                    */
    int nx, ny, nz;         /* every side >= 8; nz == 1 for D2Q21; fewer
                               than 2^29 sites per domain (its FP64 mass
                               plane stays below 4 GiB)                        */
    int storage;            /* lb2p_storage                                    */
    double gamma;           /* BGK parameter, -1 < gamma < 1 (Sec. II); the
                               shear viscosity is (1/2)(1+gamma)/(1-gamma) p
                               (Sec. VII).  Measured: gamma > 0 lets the
                               update grow grid-scale noise (a gamma = 0.4
                               sound wave reaches NaN within a few hundred
                               steps); gamma <= 0 stays bounded            */
    double kappa;           /* interfacial stiffness >= 0 (Sec. II)            */
    lb2p_eos eos;           /* equation of state (App. B)                      */
    double rho0;            /* fixed reference density of Delta^int and
                               Delta^corr (Secs. VI, VIII)                     */
    double tol;             /* j~ iteration stops when max_r |j~new - j~| <=
                               tol * max_r |j0'|  (Sec. IX)                    */
    int max_iter;           /* iteration cap (> 0)                             */
    int fixed_iter;         /* > 0: exactly this many iterations, no test and
                               no host synchronisation inside lb2p_step        */
    int warm_start;         /* start of the j~ iteration: 0 zero, 1 the previous
                               step's j~ (Sec. IX allows both), 2 the linear
                               extrapolation 2 j~(t-1) - j~(t-2), 3 the
                               quadratic one j~(t-3) + 3 (j~(t-1) - j~(t-2))
                               (lower orders until enough steps exist); the
                               fixed point and the stop rule do not depend
                               on it                                           */
    int check_every;        /* tolerance mode: the host reads the number of
                               converged domains first one pass after the
                               previous solve's pass count (passes launched
                               after a domain converged exit at once), then
                               every check_every passes (0 = every pass)      */
    double store_rho_ref;   /* reference density of BF16/F16 deviation storage
                               (<= 0: mean of the density given to lb2p_init) */
    int flags;              /* LB2P_FLAG_* (0 = defaults)                      */
    int graph_steps;        /* > 0 with fixed_iter > 0: lb2p_step replays a
                               HIP graph of this many captured steps           */
    int solver;             /* lb2p_solver: how the j~ fixed point is reached  */
    double spectral_bound;  /* Chebyshev only: upper bound b < 1 of the
                               spectrum of the map's linear part (0 = bound
                               from the EOS, see lb2p_solver)                  */
    int iter_prec;          /* lb2p_iter_prec: precision of the per-site
                               fields and of the j~ iteration (Sec. IX) on
                               FP32/BF16/F16 storage                           */
} lb2p_params;

/* lb2p_params.iter_prec.  The populations keep their storage format in
 * every case; this selects the precision of everything else (the per-site
 * fields of items 1-11, so also of the j~ iteration).
 *   LB2P_ITER_AUTO: FP64 with F64 storage; otherwise FP32, unless the stop
 *     rule's tolerance (tolerance mode) is below LB2P_F32_TOL_FLOOR, where
 *     the FP32 iteration can no longer meet it: then FP64.
 *   LB2P_ITER_F32:  FP32 (EINVAL with F64 storage).
 *   LB2P_ITER_F64:  FP64.
 * In the FP32 iteration the iterate u is an FP32 number, so the stop rule's
 * |G(j~) - j~| = |G + j0' - rho u| cannot fall much below the rounding of
 * rho u next to max|j0'|; the floor is measured on the slab workload (the
 * rule stalls at tol 1e-7; 2e-7 and above converge). */
typedef enum { LB2P_ITER_AUTO = 0, LB2P_ITER_F32 = 1, LB2P_ITER_F64 = 2 } lb2p_iter_prec;
#define LB2P_F32_TOL_FLOOR 2e-7

/* lb2p_params.solver.  Both reach the fixed point of items 3-8 and stop on
 * the same rule (max_r |G(j~) - j~| <= tol * max_r |j0'|, Sec. IX).
 *   LB2P_SOLVER_FIXED_POINT: the paper's iteration j~ <- G(j~).
 *   LB2P_SOLVER_CHEBYSHEV:   Chebyshev semi-iteration on the same map (the
 *     faster solvers Sec. IX leaves open).  The linear part of G is similar
 *     to a symmetric positive semi-definite operator when the bulk viscosity
 *     is positive, so its spectrum is real in [0, b].  The default b is
 *     1.05 * (|s|^2_max / 12) * max over (rho1, rho3) of c_s^2 (2 - rho psi),
 *     with |s|^2_max = d * max_k ((4/3) sin k - (1/6) sin 2k)^2 the largest
 *     plane-wave symbol of the first-derivative stencil (Sec. IV B).
 *     lb2p_create returns LB2P_EINVAL when b >= 1 (the map is then not a
 *     contraction and the semi-iteration does not apply). */
typedef enum { LB2P_SOLVER_FIXED_POINT = 0, LB2P_SOLVER_CHEBYSHEV = 1 } lb2p_solver;

/* lb2p_params.flags: LB2P_FLAG_UNFUSED_SOLVE runs each pass of the j~
 * iteration as two separate sweeps (item 4, then item 5 and the update of
 * j~) instead of the fused kernel, which carries the iterate as u =
 * (j0' + j~)/rho and forms j~ after the last pass (D2Q21 and D3Q59); both
 * compute the same map and stop on the same rule. */
#define LB2P_FLAG_UNFUSED_SOLVE 1
/* LB2P_FLAG_STENCIL_CLOSURE: a second formulation of items 10-11 (the
 * Supplemental preamble notes that the differential operators may be moved
 * left or right, giving algorithms that agree to the Chapman-Enskog order
 * but differ numerically).  The derivatives of X = P1 div u,
 * T_ag = p (d_a u_g + d_g u_a) and Y_b = rho^-1 d_b p + u_g d_g u_b are taken
 * with the product rule, so that every second derivative acts on p or on u
 * alone and uses the Table III stencils for the Laplacian (Sec. IV C) and
 * the traceless d_a d_b (Sec. IV D) in place of two nested first
 * derivatives; Xi' and the rest of the step are unchanged. */
#define LB2P_FLAG_STENCIL_CLOSURE 2

/* Diagnostics of the state (FP64 sums over all sites). */
typedef struct {
    double mass;            /* sum_r rho                                       */
    double mom[3];          /* sum_r j0                                        */
    int iters;              /* iterations used by the last j~ solve            */
    double resid;           /* last max_r |j~new - j~|                         */
    double jscale;          /* max_r |j0'| of the last solve                   */
    int nonfinite;          /* 1 if a NaN/Inf density was seen                 */
} lb2p_stats;

typedef struct lb2p_ctx lb2p_ctx;

/* Fill *out with defaults for a lattice and grid: gamma 0, kappa 0, the EOS
 * rho1 0.3, rho2 1.0, A 0, cs2_rho1 0.45, rho0 = rho1, the given storage,
 * tol 1e-13 (F64), 4e-7 (F32: twice the floor of the FP32 iteration; on the
 * slab workload the FP32 velocity stays within 1e-5 of FP64 over 100 steps)
 * or half the format's unit roundoff (BF16 2^-9, F16 2^-12: j0' comes from
 * populations rounded to that relative size, so a tighter rule only spends
 * passes on storage noise), max_iter 200, warm_start 1, iter_prec AUTO, no
 * graph. */
lb2p_status lb2p_default_params(int lattice, int nx, int ny, int nz, int storage,
                                lb2p_params *out);

/* Validate params (Sec. II gamma range, App. B admissibility: weights positive
 * for every c_s^2 the EOS takes, a two-phase region psi < -1/rho, positive
 * bulk viscosity psi < (2/d)/rho (Sec. VII); W_i(rho0) > 0) and allocate the
 * device state on the current HIP device.  hip_stream is a hipStream_t (NULL
 * = default stream); every later call enqueues its work there.
 * Errors: EINVAL, EEOS, ENOMEM, EHIP. */
lb2p_status lb2p_create(const lb2p_params *params, void *hip_stream, lb2p_ctx **out);

/* A context advancing ndom independent periodic lattices together (each
 * with its own grid, gamma, kappa, EOS and rho0; all with the same lattice,
 * storage and iteration settings, taken from per_dom[0]).  Every buffer the
 * other calls take or return then holds the domains packed in order:
 * a scalar field is [S] with S = sum of the domain sizes, domain d starting
 * at off_d = sum of the sizes before it; a vector field is [d][S].  The stop
 * rule of the j~ iteration applies to each domain separately.
 * Errors: as lb2p_create, and EINVAL when the shared settings differ. */
lb2p_status lb2p_create_batch(int ndom, const lb2p_params *per_dom, void *hip_stream,
                              lb2p_ctx **out);

/* FP64 totals per domain of the current state: out[4*d + k] = mass (k=0)
 * and momentum x, y, z (k=1..3) of domain d; host memory [4*ndom].
 * Errors: EINVAL, ESTATE, EHIP. */
lb2p_status lb2p_domain_totals(lb2p_ctx *ctx, double *out);

/* The last j~ solve of each domain (of the last lb2p_step, or of
 * lb2p_moments when that ran since): the passes it ran, the residual
 * max_r |j~new - j~| of its last pass and max_r |j0'|, the two sides of the
 * stop rule of Sec. IX, and whether the rule held (1) or max_iter ended it
 * (0; always 1 with a fixed pass count).  Host arrays of ndom entries; any
 * may be NULL.  Synchronises the context's stream.
 * Errors: EINVAL, ESTATE (no solve yet), EHIP. */
lb2p_status lb2p_domain_solve(lb2p_ctx *ctx, int *iters, double *resid, double *jscale, int *converged);

/* Pick the kernel block shapes of this context by timing `steps` steps of
 * each candidate on the current state (which is saved and restored), and
 * remember the choice per (lattice, storage, domain sizes) for the process.
 * If LB2P_TUNE_CACHE names a file, choices are read from and appended to it.
 * Errors: ESTATE, ENOMEM, EHIP. */
lb2p_status lb2p_autotune(lb2p_ctx *ctx, int steps);

/* Set the choices the autotuner makes: the site kernels' block shape
 * (bx x by threads with bx * by = 256, one site each, a bx x by patch of a
 * plane; or bx = 256, by = 0: blocks of 256 consecutive sites in index
 * order, which leave no lane idle on narrow domains) and the plane count tz
 * of the 3D solve pass's chunks.  Results do not depend on the choice.
 * Errors: EINVAL (NULL context, another shape, tz < 1), ENOMEM, EHIP. */
lb2p_status lb2p_set_tiling(lb2p_ctx *ctx, int bx, int by, int tz);

/* Set the initial populations n_i(r, 0) = n_eq(rho(r), u(r)) of Sec. III with
 * the local weights.  rho [N], u [d][N]; dtype lb2p_dtype; host or device.
 * Resets the sticky status and the warm-start j~ to zero.
 * Errors: EINVAL, EHIP. */
lb2p_status lb2p_init(lb2p_ctx *ctx, const void *rho, const void *u, int dtype, int on_device);

/* Advance nsteps >= 0 time steps (Supplemental items 1-12 each).
 * Asynchronous on the context's stream when fixed_iter > 0; otherwise the
 * host reads the convergence count back during each solve (check_every),
 * and the max_iter count and the non-finite flag once per call.  In that
 * mode the rest of a step is enqueued before the host waits for the solve's
 * first read (it runs only if every domain's stop rule held, else it is
 * enqueued again after the remaining passes), so the call returns with the
 * last step's closure and collision still in flight on the stream.
 * Returns ENOCONV if any step's solve hit max_iter, ENONFINITE once a NaN or
 * Inf density was seen (sticky until lb2p_init).
 * Errors: ESTATE (no init), ENOCONV, EHIP. */
lb2p_status lb2p_step(lb2p_ctx *ctx, int nsteps);

/* Density and converged flow velocity u = j/rho of the CURRENT state
 * (items 1-8 evaluated without colliding).  rho_out [N], u_out [d][N]
 * (either may be NULL); dtype lb2p_dtype; host or device.  st may be NULL.
 * A query: the state and what the next lb2p_step starts its solve from (the
 * last step's j~) are unchanged, so later steps give the same results
 * whether or not it was called.  It reads the non-finite flag of the steps
 * since the last synchronising call (lb2p_step does so itself only in the
 * tolerance mode, fixed_iter == 0).
 * Errors: ESTATE, ENOCONV, ENONFINITE, EHIP. */
lb2p_status lb2p_moments(lb2p_ctx *ctx, void *rho_out, void *u_out, int dtype,
                         int on_device, lb2p_stats *st);

/* lb2p_moments for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc).  The
 * same results as lb2p_moments, bit for bit.  Where lb2p_moments allocates
 * a stream-ordered device buffer per call (to convert a host output to the
 * other precision), this call stages the conversion in a static device
 * array of LB2P_NOALLOC_STAGE_BYTES that every GPU running the library
 * holds until the process ends; device outputs are converted in place.  It
 * calls no hipMalloc/hipFree.  Errors: as lb2p_moments, and LB2P_ESIZE
 * (nothing done) when a host output needs conversion and d * N elements of
 * dtype exceed the array.  The array is shared by every context on one GPU
 * and keeps the last call's contents: calls that overlap on one GPU (from
 * different threads or processes sharing the library) race on it. */
#define LB2P_NOALLOC_STAGE_BYTES (64ull << 20)
lb2p_status lb2p_moments_noalloc(lb2p_ctx *ctx, void *rho_out, void *u_out, int dtype,
                                 int on_device, lb2p_stats *st);

/* One per-site field of the last evaluated items 1-11 (see lb2p_field), as
 * dtype into out (host or device), component-major.  Sigma and Xi' are only
 * defined after a lb2p_step (they are not part of lb2p_moments).
 * Errors: EINVAL, ESTATE, EHIP. */
lb2p_status lb2p_get_field(lb2p_ctx *ctx, int field, void *out, int dtype, int on_device);

/* Pre-collision populations n_i(r, t) as [Q][N] FP64 in the library's
 * velocity order (lb2p_velocities); host or device.  set_ replaces the state
 * (and resets the sticky status); get_ decodes the stored form.
 * Errors: EINVAL, ESTATE, EHIP. */
lb2p_status lb2p_get_populations(lb2p_ctx *ctx, double *n_out, int on_device);
lb2p_status lb2p_set_populations(lb2p_ctx *ctx, const double *n_in, int on_device);

/* The library's velocity order: c_out[3*Q] (z = 0 for D2Q21).  Returns Q in
 * *q_out.  Host memory.  Errors: EINVAL. */
lb2p_status lb2p_velocities(int lattice, int *c_out, int *q_out);

/* Diagnostics (FP64 totals of mass and momentum of the current state, last
 * solve's iteration count and residual, non-finite flag).  Errors: EHIP. */
lb2p_status lb2p_stats_get(lb2p_ctx *ctx, lb2p_stats *st);

/* Kernel classes timed by the optional profiler. */
typedef enum {
    LB2P_K_MOMENTS = 0,    /* item 1 (pull + moments)                        */
    LB2P_K_FORCE = 1,      /* item 2 (interface force, start of the solve)   */
    LB2P_K_ITER_Q = 2,     /* item 4 of one pass                             */
    LB2P_K_ITER_JT = 3,    /* items 5-6 of one pass                          */
    LB2P_K_CLOSURE1 = 4,   /* items 9-10 and Xi'                             */
    LB2P_K_CLOSURE2 = 5,   /* Sigma                                          */
    LB2P_K_COLLIDE = 6,    /* item 11 per velocity and item 12               */
    LB2P_K_ITER_FUSED = 7, /* items 3-6 of one pass in one kernel (velocity
                              form, both lattices)                        */
    LB2P_NKERNEL = 8
} lb2p_kernel;

/* Diagnostic timing: when enabled, every launch of the selected classes
 * (lb2p_profile_classes; by default all of the above) is bracketed by HIP
 * events on the context's stream, and every launch of the others is
 * counted.  enable resets the totals; read synchronises the stream and
 * returns, per class, the summed event time in ms (ms_out[LB2P_NKERNEL];
 * 0 for a class not selected) and the launch count
 * (count_out[LB2P_NKERNEL]).  Errors: EINVAL. */
lb2p_status lb2p_profile_enable(lb2p_ctx *ctx, int on);
lb2p_status lb2p_profile_read(lb2p_ctx *ctx, double *ms_out, long long *count_out);

/* Select the classes the profiler brackets with events: bit (1u << k) for
 * class k of lb2p_kernel; (1u << LB2P_NKERNEL) - 1 selects all (the
 * default).  Each bracketed launch adds two event records to the stream, which
 * the GPU processes between kernels, so a caller that times one class
 * selects only that one.  Applies to launches after the call; totals are
 * kept.  Errors: EINVAL (NULL context, or a bit at LB2P_NKERNEL or above). */
lb2p_status lb2p_profile_classes(lb2p_ctx *ctx, unsigned mask);

/* Solve passes that did work since lb2p_profile_enable (while profiling is
 * on): per solve, the pass count at which the last domain met the stop rule
 * (in fixed mode, or when max_iter ends it: the passes launched).  The
 * solve-pass launch counts of lb2p_profile_read also hold the launches after
 * the stop rule held, which return at once; their event time is a few
 * microseconds each.  Errors: EINVAL (NULL argument). */
lb2p_status lb2p_profile_passes(lb2p_ctx *ctx, long long *passes_out);

/* Release everything the context owns.  NULL is accepted. */
void lb2p_destroy(lb2p_ctx *ctx);

/* Static description of a status code. */
const char *lb2p_strerror(lb2p_status st);

#ifdef __cplusplus
}
#endif
#endif /* LB2P_H */
