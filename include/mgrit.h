/*
 * mgrit.h -- C-ABI of libmgrit: MGRIT / Parareal for the periodic
 * constant-coefficient linear advection equation u_t + alpha u_x = 0 on
 * x in [-1, 1), on one AMD Instinct MI355X (gfx950).
 *
 * Method: De Sterck, Falgout, Friedhoff, Krzysik, MacLachlan, "Optimizing
 * MGRIT and Parareal coarse-grid operators for linear advection"
 * (Numer. Linear Algebra Appl. 2021, arXiv:1910.03726).
 *
 * Space-time problem (Sec. 2.1-2.2, eq. (3)): n_x periodic unknowns,
 * dx = 2/n_x, x_i = -1 + i dx; Courant number c = alpha dt/dx (eq. (5));
 * n_t steps u^{n+1} = Phi u^n from u^0 = u0, with Phi one step of a
 * Runge-Kutta method (ERKp or SDIRKp, Appendix A) applied to the p-th order
 * upwind discretization Up of -alpha d/dx (Sec. 2.1).
 *
 * Conventions for every entry point:
 *   - Return 0 on success, a negative MGRIT_E* code otherwise; no C++
 *     exception crosses this boundary.  mgrit_strerror() names the code.
 *   - Pointers named *_dev are device pointers (HIP, the current device of
 *     the plan); *_host are host pointers.  The caller owns every buffer it
 *     passes; a plan owns its own device workspace and copies of all taps.
 *   - Space-time arrays are row-major [time level][n_x], FP64.
 *   - A periodic stencil (mgrit_taps) means
 *         (Psi u)_i = sum_t weight[t] * u[(i - offset[t]) mod n_x],
 *     i.e. the circulant matrix whose first column holds weight[t] at row
 *     offset[t] (Sec. 4.1).  Offsets may be any integers.
 *   - Entry points that launch GPU work run on the plan's HIP stream.
 *     mgrit_solve and mgrit_plan_create return only after their GPU work
 *     has finished; phi_apply_batch is asynchronous on the stream.
 *   - A plan is not thread-safe: calls on one plan must not overlap.
 */
#ifndef MGRIT_H
#define MGRIT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define MGRIT_OK 0
#define MGRIT_EINVAL (-1)     /* invalid argument or unsupported shape       */
#define MGRIT_EUNSTABLE (-2)  /* ERK Courant number above the CFL limit       */
#define MGRIT_ENOMEM (-3)     /* device or host allocation failed            */
#define MGRIT_EHIP (-4)       /* a HIP runtime call failed                    */
#define MGRIT_ENOTCONV (-5)   /* maxit reached above tol (history is filled)  */
#define MGRIT_EDIVERGED (-6)  /* non-finite residual norm                     */
#define MGRIT_EIMAG (-7)      /* least-squares imaginary part above 1e-8      */
#define MGRIT_ENODEV (-8)     /* no usable gfx950 device                      */
#define MGRIT_ECAPACITY (-9)  /* caller's output arrays are too small         */
#define MGRIT_EBUSY (-10)     /* serving: admission refused (HBM budget)      */
#define MGRIT_ESCRATCH (-11)  /* mgrit_solve_static: plan exceeds the static
                                 workspace (MGRIT_STATIC_BYTES)              */

/* ---- discretizations (Sec. 2.1; tableaux of Appendix A) ----------------- */
#define MGRIT_ERK1 1
#define MGRIT_ERK2 2
#define MGRIT_ERK3 3
#define MGRIT_ERK4 4
#define MGRIT_ERK5 5
#define MGRIT_SDIRK1 11
#define MGRIT_SDIRK2 12
#define MGRIT_SDIRK3 13
#define MGRIT_SDIRK4 14

/* ---- solver options ----------------------------------------------------- */
#define MGRIT_CYCLE_V 0      /* V-cycles (Sec. 4.4)                           */
#define MGRIT_CYCLE_F 1      /* F-cycles: coarse problem by F- then V-cycle   */
#define MGRIT_RELAX_FCF 0    /* FCF-relaxation (Sec. 2.2, the paper's choice) */
#define MGRIT_RELAX_F 1      /* F-relaxation (Parareal)                       */
#define MGRIT_FP64 0         /* all arithmetic in FP64                        */
#define MGRIT_FP32_RELAX 1   /* FP32 relaxation of FP64 iterates: with FCF,
                                the second fine pass acts on the C-point
                                update in FP32; with F-relaxation, FP32 inner
                                cycles inside FP64 iterative refinement     */
#define MGRIT_FP32_IR 2      /* FP32 inner cycles (both fine passes FP32,
                                FCF or F) inside FP64 iterative refinement:
                                FP64 residual of the iterate, inner solve of
                                the error system, FP64 update              */

/* coarse-operator pattern rules for mgrit_psi_optimize */
#define MGRIT_PSI_AUTO 0     /* ETA for SDIRK, WINDOW for ERK                 */
#define MGRIT_PSI_WINDOW 1   /* contiguous window of Phi^m (Sec. 4.3)         */
#define MGRIT_PSI_ETA 2      /* thresholding |phi^m| >= eta max (Sec. 4.6)    */
#define MGRIT_PSI_REDISC 3   /* rediscretization: ERK Phi with step m^(l-1) dt */

/* how the coarsest level's system is solved (mgrit_plan_set_coarse_solver) */
#define MGRIT_COARSE_AUTO 0     /* the faster of the two by the plan's model   */
#define MGRIT_COARSE_SWEEP 1    /* time step after time step, as written       */
#define MGRIT_COARSE_SPECTRAL 2 /* per Fourier mode of the circulant Psi       */

/* what mgrit_solve writes to u_out_dev */
#define MGRIT_OUT_NONE 0     /* nothing                                       */
#define MGRIT_OUT_FINAL 1    /* u^{n_t}: n_x values                           */
#define MGRIT_OUT_CPOINTS 2  /* u^{jm}, j = 0..n_t/m: (n_t/m + 1) x n_x       */
#define MGRIT_OUT_ALL 3      /* u^n, n = 0..n_t: (n_t + 1) x n_x              */

typedef struct {
    int nnz;        /* number of taps (in: capacity for outputs)             */
    int* offset;    /* nnz offsets (caller-owned)                            */
    double* weight; /* nnz weights (caller-owned)                            */
} mgrit_taps;

typedef struct mgrit_plan_s* mgrit_plan_t;

/* Statistics of the last mgrit_solve on a plan. */
typedef struct {
    int iterations;        /* fine-level coarse-grid corrections applied      */
    int outer_iterations;  /* MGRIT_FP32_RELAX: FP64 fine passes (FCF) or
                              FP64 refinement steps (F-relaxation);
                              MGRIT_FP32_IR: FP64 refinement steps; else 0 */
    int fine_passes_fp64;  /* fine-level relaxation passes run in FP64        */
    int fine_passes_fp32;  /* fine-level relaxation passes run in FP32        */
    double final_residual; /* sqrt(dx dt sum r^2) of the returned iterate     */
    double solve_ms;       /* wall time of the solve (host clock)             */
    long long batched_launches; /* mgrit_solve_batch: relaxation launches of
                              this plan that ran merged with other plans'   */
} mgrit_stats;

/* Per-kernel-class GPU time, collected with HIP events when profiling is on. */
#define MGRIT_PROF_RELAX_FINE 0   /* fine-level relaxation passes (A and B) */
#define MGRIT_PROF_RELAX_COARSE 1 /* relaxation on levels >= 2              */
#define MGRIT_PROF_COARSEST 2     /* sequential coarsest-level sweeps       */
#define MGRIT_PROF_NORM 3         /* residual-norm reductions               */
#define MGRIT_PROF_OTHER 4        /* interpolation, axpy, copies            */
#define MGRIT_PROF_CLASSES 5
typedef struct {
    double ms[MGRIT_PROF_CLASSES];    /* summed kernel time per class      */
    long long launches[MGRIT_PROF_CLASSES];
    double fine_dof_steps;            /* fine DOF-steps executed by class 0 */
} mgrit_profile;

/* ---- host-only setup (no GPU needed) ------------------------------------ */

/* Library version, e.g. 100 for 1.0.0. */
int mgrit_version(void);

/* Static description of a return code; never NULL. */
const char* mgrit_strerror(int code);

/* max over theta in [0, pi] of |R(c * s(theta))|, the amplification of one
 * step of `scheme` on Fourier mode theta (Lemma 1; used for the CFL limit of
 * eq. (5) / Table 1).  Writes *amp.  Host only. */
int mgrit_max_amplification(int scheme, double cfl, double* amp);

/* Phi of an ERK scheme as one periodic stencil (Corollary 1: Phi = R(dt L)
 * is a sparse circulant), offsets folded into [0, n_x).  Up to `capacity`
 * taps are written to offsets/weights; *nnz receives the count.  SDIRK
 * schemes return MGRIT_EINVAL (their Phi is dense).  Host only. */
int mgrit_phi_taps(int scheme, double cfl, int nx, int capacity, int* offsets,
                   double* weights, int* nnz);

/* Coarse operators Psi_2..Psi_levels of an MGRIT hierarchy (Sec. 4, 4.4,
 * 4.6): Phi_{l+1} minimizes the weighted spectral error of eq. (9) against
 * Phi_l^m over the sparsity pattern given by `rule`:
 *   MGRIT_PSI_WINDOW: contiguous window of phi~^m = first column of Phi_l^m;
 *       width widths[l-1] if `widths` is non-NULL, else
 *       max(nnz(Phi_l), span of {o : |phi~^m_o| >= 0.02 max}); placed to
 *       maximize the sum of |phi~^m| inside (smallest start on ties);
 *   MGRIT_PSI_ETA: {o : |phi~^m_o| >= eta max} with `eta`, or the table of
 *       Sec. 4.6 for (p, m) if eta <= 0;
 *   MGRIT_PSI_REDISC: ERK only; Psi_l = the ERK stencil at Courant number
 *       m^(l-1) c (no least squares).
 * Weights w_k = 1/(1 - |lambda_k| + 1e-6)^2 on the eigenvalues of Phi_l.
 * Eq. (9) is solved for real weights: for a real stepper the rows k and
 * n_x - k are complex conjugates, so the minimiser over complex weights is
 * real.  For n_x a power of two through its normal equations (the Gram
 * matrix of the weighted Fourier columns depends only on offset
 * differences: one FFT of the weights), refined against the residual over
 * the whole spectrum until the correction is below 1e-13 of the weights;
 * otherwise, or if the refinement stalls, by Householder QR of the real
 * form (k <= n_x/2, real and imaginary parts as separate equations).
 * out[l-2] for l = 2..levels must carry arrays with room for out[.].nnz
 * taps (capacity on input, count on output).  *max_imag (may be NULL)
 * receives the largest imaginary part of the weights, 0 in the real form
 * (MGRIT_EIMAG above 1e-8).  Host only. */
int mgrit_psi_optimize(int scheme, double cfl, int nx, int m, int levels,
                       int rule, const int* widths, double eta,
                       mgrit_taps* out, double* max_imag);

/* ERK coarse operators with windows chosen by the two-level convergence
 * bound of Sec. 3 (eq. (7)): level by level (Psi_{l+1} against
 * Phi_l^m, Sec. 4.4), the contiguous window of phi~^m placed as for
 * MGRIT_PSI_WINDOW, its width the narrowest from the window rule's width up
 * to MGRIT_PSI_BOUND_MAX_WIDTH (the widest register-resident stencil of the
 * relaxation kernels) whose bound
 *     max_k sqrt(m) |lambda_k|^m |lambda_k^m - mu_k| sum_{j < n_l/m - 1} |mu_k|^j
 * (n_l the steps of level l, n_1 = nt) is at most max(target, 1e-10)
 * (bounds below 1e-10 are at the rounding level of the fit), else the
 * narrowest width whose bound is within 0.1 % of the smallest.  Wider
 * coarse stencils cost the relaxation kernels little (their passes are
 * bound by memory traffic and latency) and save iterations.  Each candidate width is one weighted least-squares
 * solve (eq. (9)), so this setup takes tens of milliseconds per level at
 * n_x = 8192.  out as for mgrit_psi_optimize (room for up to
 * MGRIT_PSI_BOUND_MAX_WIDTH taps per level); bounds (may be NULL) receives
 * the bound of each level's choice.  SDIRK schemes: MGRIT_EINVAL (their
 * patterns are thresholded, Sec. 4.6).  Host only. */
#define MGRIT_PSI_BOUND_MAX_WIDTH 64
int mgrit_psi_optimize_bound(int scheme, double cfl, int nx, int nt, int m,
                             int levels, double target, mgrit_taps* out,
                             double* bounds, double* max_imag);

/* ---- plans and solves (GPU) --------------------------------------------- */

/* Create a plan for the space-time system of eq. (3) (Sec. 2.2) and its
 * MGRIT hierarchy (Sec. 4.4): n_x, n_t, alpha, Courant number c, scheme,
 * coarsening factor m and `levels` >= 2 levels (n_t divisible by
 * m^(levels-1); each
 * level has >= 2 coarse intervals).  psi: levels-1 coarse stencils
 * (Psi_2..Psi_levels), copied into the plan.  cycle/relax/precision: the
 * MGRIT_* options above.  hip_stream: a hipStream_t (NULL = default
 * stream).  ERK plans with c above the CFL limit (amplification > 1+1e-6)
 * return MGRIT_EUNSTABLE.  SDIRK plans need n_x a multiple of 64.
 * Allocates the device workspace; *plan receives the handle. */
int mgrit_plan_create(mgrit_plan_t* plan, int nx, int nt, double alpha,
                      double cfl, int scheme, int m, int levels,
                      const mgrit_taps* psi, int cycle, int relax,
                      int precision, void* hip_stream);

/* A plan for inflow/outflow boundaries (Sec. 4.5): u_t + alpha u_x = 0 on
 * (-1, 1] with u(-1, t) = g(t), ERK schemes only, FP64 only.
 *   Grid: unknowns at x_i = -1 + i dx, i = 1..n_x, dx = 2/n_x (u0 and all
 *         outputs hold these n_x values); dt = c dx / alpha.
 *   Fine step: ERKp+Up with outflow ghosts from the degree p-1 polynomial
 *         through the last p unknowns, and inflow ghosts from a Taylor series
 *         about x = -1 whose space derivatives the PDE turns into time
 *         derivatives (inverse Lax-Wendroff), with stage-consistent boundary
 *         data for every ERK stage; the step is u^{n+1} = Phi u^n + f^{n+1}.
 *   inflow: host, n_t rows of n_derivs >= p+1 values, row n holding
 *         g(t_n), g'(t_n), ..., g^(p)(t_n) at t_n = n dt (further columns
 *         ignored); copied into the plan as the per-step forcing.
 *   psi:  the periodic coarse stencils (as for mgrit_plan_create), applied
 *         truncated to the interval (terms with i - offset outside 0..n_x-1
 *         dropped; offsets taken in (-n_x/2, n_x/2]).
 * The coarsest level is swept (no spectral solve: Psi is not circulant).
 * When every offset of the truncated coarsest Psi is >= 1, Psi is strictly
 * lower triangular and Psi^q = 0 for q = ceil(n_x / smallest offset); a
 * step then depends on the last q states only, and with
 * MGRIT_COARSE_AUTO (the default) the sweep runs in parallel chunks of q
 * steps, each started from zero q steps before its first stored row
 * (mgrit_plan_describe: "(chunked sweep)"), giving the step-by-step
 * sweep's values bit for bit; MGRIT_COARSE_SWEEP keeps the step-by-step
 * sweep.
 * phi_apply_batch on such a plan steps every row from t = 0 with the
 * plan's inflow data (k <= n_t).  The plan also holds the forcing table
 * (n_t rows of at most s r_l FP64 values, s stages, r_l the upwind reach of
 * Up), which mgrit_plan_estimate_bytes does not count.  Other arguments and errors as
 * mgrit_plan_create; n_x up to 10232 (two FP64 rows in a CU's 160 KB of
 * LDS). */
int mgrit_plan_create_inflow(mgrit_plan_t* plan, int nx, int nt, double alpha,
                             double cfl, int scheme, int m, int levels,
                             const mgrit_taps* psi, int cycle, int relax,
                             const double* inflow, int n_derivs,
                             void* hip_stream);

/* The fine step of mgrit_plan_create_inflow's problem as its kernels apply
 * it: phi (may be NULL) receives Phi as a dense n_x x n_x row-major matrix,
 * B (may be NULL) the n_x x (p+1) matrix with f^{n+1} = B (g^(d)(t_n))_d,
 * *n_derivs the p+1 columns of B.  Host only (for checks). */
int mgrit_inflow_operator(int scheme, double cfl, double alpha, int nx,
                          double* phi, double* B, int* n_derivs);

/* Solve the space-time system to sqrt(dx dt sum r^2) <= tol (Sec. 2.2).
 *   u0_dev:    n_x initial values u^0 (device).
 *   uinit_dev: initial iterate at the C-points, (n_t/m + 1) x n_x (row 0 is
 *              ignored and replaced by u0), or NULL for the plan's seeded
 *              U[0,1) iterate (splitmix64 stream of mgrit_plan_set_seed).
 *   maxit:     maximum coarse-grid corrections (>= 0).
 *   u_out_dev: output per out_kind (MGRIT_OUT_*), may be NULL for NONE.
 *   res_hist_host: may be NULL, else room for maxit+1 doubles: the
 *              residual norm before each correction (for MGRIT_FP32_IR, and
 *              MGRIT_FP32_RELAX with F-relaxation: the FP64 refinement
 *              residuals).
 *   iters_out: may be NULL; receives the number of corrections.
 * Returns MGRIT_ENOTCONV if maxit is reached (outputs still written),
 * MGRIT_EDIVERGED on a non-finite norm.  Synchronous. */
int mgrit_solve(mgrit_plan_t plan, const double* u0_dev,
                const double* uinit_dev, double tol, int maxit,
                double* u_out_dev, int out_kind, double* res_hist_host,
                int* iters_out);

/* n solves at once (the same iteration as mgrit_solve for each, Sec. 2.2
 * and 4.4), stepped together on the plans' common stream: at every pass
 * the relaxation launches of plans with the same kernel and launch shape
 * (same n_x, scheme, level sizes and precision; any Courant number, Psi,
 * u0, tolerance) run as one launch over their concatenated grids, so that
 * small solves fill the device together.  Each result equals that of
 * mgrit_solve on the same plan and inputs, bit for bit.
 *   plans:   n distinct plans created on the same hip_stream (else
 *            MGRIT_EINVAL, nothing run).
 *   u0, tol, maxit, out_kind, status: n entries each; uinit, u_out, hist
 *            may be NULL (all entries NULL), else n entries, each as in
 *            mgrit_solve; iters may be NULL, else n entries.
 *   status:  per plan, what mgrit_solve would have returned.
 * Returns MGRIT_OK once every solve has ended (see status), MGRIT_EINVAL
 * for invalid arguments, or the first HIP error.  Synchronous. */
int mgrit_solve_batch(int n, const mgrit_plan_t* plans,
                      const double* const* u0_dev,
                      const double* const* uinit_dev, const double* tol,
                      const int* maxit, double* const* u_out_dev,
                      const int* out_kind, double* const* res_hist_host,
                      int* iters_out, int* status);

/* How solves on this plan compute the coarsest level's solution
 * x^0 = 0, x^s = Psi x^(s-1) + g^s, s = 1..n (the exact coarse solve of
 * Sec. 2.2 and 4.4):
 *   MGRIT_COARSE_SWEEP:    the n steps one after another (launches of a
 *                          few steps each, spatially tiled);
 *   MGRIT_COARSE_SPECTRAL: Psi is circulant, so the discrete Fourier
 *                          transform diagonalises it (Sec. 4.1): every row
 *                          g^s is transformed, each Fourier mode k runs its
 *                          own recurrence X^s_k = mu_k X^(s-1)_k + G^s_k
 *                          (mu_k the eigenvalues of Psi), and the rows are
 *                          transformed back -- the same solution up to
 *                          rounding, in three launches instead of n steps;
 *                          needs n_x a power of two up to 8192 (else
 *                          MGRIT_EINVAL);
 *   MGRIT_COARSE_AUTO:     (the default) the one the plan's cost model
 *                          expects to be faster.
 * mgrit_plan_describe reports "(spectral solve)" when it is used. */
int mgrit_plan_set_coarse_solver(mgrit_plan_t plan, int mode);

/* out[b] = Phi^k in[b] for b = 0..batch-1, rows of n_x values (device,
 * row-major, in and out may not overlap; k = 0 copies), Phi the fine time
 * step u^{n+1} = Phi u^n of eq. (3) (Sec. 2.1; one collapsed stencil for ERK
 * schemes, Corollary 1).  The fine stepper of the plan in the plan's
 * precision of relaxation; asynchronous on the plan stream.  batch = 0 does
 * nothing (in and out may then be NULL); MGRIT_EINVAL for a negative batch
 * or k, or NULL rows. */
int phi_apply_batch(mgrit_plan_t plan, const double* in_dev, double* out_dev,
                    int batch, int ksteps);

/* Device bytes the plan holds (its HBM footprint, for admission). */
int mgrit_plan_bytes(mgrit_plan_t plan, size_t* hbm_bytes);

/* Upper bound of the device bytes mgrit_plan_create would allocate for
 * these sizes (no allocation; host only). */
int mgrit_plan_estimate_bytes(int nx, int nt, int m, int levels, int precision,
                              size_t* bytes);

/* Seed of the U[0,1) initial iterate used when uinit_dev is NULL. */
int mgrit_plan_set_seed(mgrit_plan_t plan, unsigned long long seed);

/* Statistics of the last solve. */
int mgrit_get_stats(mgrit_plan_t plan, mgrit_stats* stats);

/* Turn per-kernel HIP-event timing on (1) or off (0); turning it on clears
 * the counters.  mgrit_get_profile reads them. */
int mgrit_set_profiling(mgrit_plan_t plan, int enable);
int mgrit_get_profile(mgrit_plan_t plan, mgrit_profile* prof);

/* The same timing split by level, pass and precision, with the algorithmic
 * work of every launch: the bytes the pass must move between HBM and the
 * chip (C-point rows read and written, right-hand side rows, rows stored
 * by interpolation; n_x * 8 bytes per row) and its flops (2 nnz per point
 * and step for a stencil of nnz taps, the recurrence count of the SDIRK
 * stage solves, Sec. 2.1 and Corollary 1), so that a roofline fraction can
 * be formed per pass.  Passes: */
#define MGRIT_PASS_FC 0        /* F- then C-relaxation (pass A)              */
#define MGRIT_PASS_RES 1       /* F-relaxation + C-point residual (pass B)   */
#define MGRIT_PASS_F 2         /* F-relaxation storing every point           */
#define MGRIT_PASS_SWEEP 3     /* coarsest level: sequential sweep           */
#define MGRIT_PASS_SPECTRAL 4  /* coarsest level: spectral solve             */
#define MGRIT_PASS_NORM 5      /* residual-norm reduction                    */
#define MGRIT_PASS_COPY 6      /* C-point copies, refinement updates         */
typedef struct {
    int level;          /* 0 = fine                                          */
    int pass;           /* MGRIT_PASS_*                                      */
    int precision;      /* 0 FP64 arithmetic, 1 FP32                         */
    long long launches;
    double ms;          /* summed HIP-event time of the launches             */
    double bytes;       /* summed algorithmic HBM bytes                      */
    double flops;       /* summed algorithmic flops                          */
} mgrit_prof_entry;
/* Writes min(capacity, number of entries) entries, sorted by level, pass,
 * precision; *count receives the number of entries.  Profiling must have
 * been turned on (mgrit_set_profiling) for the launches to be counted. */
int mgrit_get_profile_detail(mgrit_plan_t plan, mgrit_prof_entry* out,
                             int capacity, int* count);

/* Operator complexity of the plan's hierarchy, eq. (10). */
int mgrit_operator_complexity(mgrit_plan_t plan, double* oc);

/* Short text naming the kernels the plan selected (static per plan). */
const char* mgrit_plan_describe(mgrit_plan_t plan);

/* Release the plan and its device memory (NULL is a no-op). */
void mgrit_destroy(mgrit_plan_t plan);

/* ---- allocation-free solve ------------------------------------------------ */

/* Bytes of the static per-device workspace of mgrit_solve_static. */
#define MGRIT_STATIC_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * solve of mgrit_plan_create + mgrit_solve + mgrit_destroy with the same
 * arguments and results, bit for bit, but with every device array of the
 * plan (C-point iterates, residuals, coarse-level arrays, per-workgroup
 * partial sums, the norm word, taps, stage data and spectral rows) carved
 * from one static array of MGRIT_STATIC_BYTES that the library reserves
 * on each GPU it runs on until the process ends.  No hipMalloc, hipFree or
 * pinned host allocation happens in the call (host bookkeeping uses the
 * C++ heap).
 *   Arguments: as mgrit_plan_create (the plan's inputs; inflow boundaries
 *   are not offered here) followed by those of mgrit_solve; the work runs
 *   on hip_stream and the call returns after it has finished.
 *   Errors: those of mgrit_plan_create and mgrit_solve, and
 *   MGRIT_ESCRATCH when the plan's arrays do not fit the workspace (the
 *   space-time arrays take about 3 (n_t/m + 1) n_x doubles plus the coarse
 *   levels; nothing is launched then).
 *   Sharing: every call on a GPU uses that GPU's one workspace, which keeps
 *   the last call's contents (nothing in it is assumed to start at zero).
 *   Calls on the same device are serialized by the library (a call holds
 *   the device's workspace until its GPU work has finished), so callers on
 *   several threads or streams of one GPU wait for each other rather than
 *   race; work outside these calls that writes the workspace's memory is
 *   not possible, since its address never leaves the library. */
int mgrit_solve_static(int nx, int nt, double alpha, double cfl, int scheme,
                       int m, int levels, const mgrit_taps* psi, int cycle,
                       int relax, int precision, void* hip_stream,
                       const double* u0_dev, const double* uinit_dev,
                       double tol, int maxit, double* u_out_dev,
                       int out_kind, double* res_hist_host, int* iters_out);

#ifdef __cplusplus
}
#endif

#endif /* MGRIT_H */
