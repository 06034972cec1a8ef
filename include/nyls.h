/*
 * nyls.h -- C ABI of the Nystrom-accelerated primal LS-SVM ODE solver (gfx950 / MI355X).
 *
 * Method: arXiv 2510.04094.  A p-th order ODE
 *     y^(p)(t) - sum_{k=1..p} f_k(t) y^(p-k)(t) = r(t),   y^(d_j)(t_{i_j}) = v_j  (j = 1..p)
 * (Sec. 3.1) is solved with the model y_hat(t) = omega^T phi(t) + b, where phi is the
 * explicit Nystrom feature map of the RBF kernel K(u, v) = exp(-(u - v)^2 / sigma^2)
 * (App. A.2, eq32): K_mm = U Lambda U^T over m landmarks, phi(t) = Lambda^{-1/2} U^T k_m(t)
 * restricted to eigenvalues lambda_k > tau * lambda_1, and phi^(d) its time derivatives
 * (Sec. 3).  Linear ODEs solve the Lemma 1 KKT system (Sec. 3.1); first-order nonlinear
 * ODEs y' = F(t, y) iterate Newton on the Lemma 2 system (Sec. 3.2, App. A.5).
 *
 * Conventions for every function below
 *   - All array arguments are DEVICE pointers unless marked "host", FP64 unless marked
 *     otherwise, row-major, owned by the caller.  The library never frees them.
 *   - Work functions only enqueue kernels on `stream` (no host synchronisation, no
 *     allocation) and return 0, or a negative NYLS_E* code when an argument is invalid;
 *     nothing is enqueued then.  nyls_solve (NYLS_FP64, NYLS_MIXED) forks part of its work onto
 *     streams the plan owns and joins it back on `stream` (events), so later work on
 *     `stream` is ordered after all of it; graph capture of `stream` captures all of it.
 *     Numerical outcomes are reported per instance in the `status` bitmask (NYLS_S*),
 *     readable after the stream is synchronised.
 *   - `ws` is a caller-allocated device workspace of nyls_workspace_size(plan) bytes.  It
 *     carries state between calls: nyls_solve leaves the basis, factors and solution there
 *     for nyls_predict / nyls_backward; nyls_newton_step keeps its basis there.  One plan
 *     with one workspace must not be used from two streams at once; distinct plans can.
 *   - Per-instance padded layouts use MAXM = max m over the batch and KN = MAXM + 1 + 4.
 *   - Only the plan functions allocate (the device descriptor table; an NYLS_FP64 or
 *     NYLS_MIXED plan also creates two non-blocking streams at default priority and six
 *     events).
 */
#ifndef NYLS_H
#define NYLS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NYLS_MAX_P 4   /* highest ODE order */
#define NYLS_MAX_M 256 /* most landmarks per instance (above 128: NYLS_FP64 solves, predictions
                          and adjoints only, see nyls_problem) */
#define NYLS_MAX_N (1 << 25) /* most grid points per instance */

/* Arithmetic of the solve (nyls_plan_create `mode`). */
enum {
  NYLS_FP64 = 0,          /* every step in FP64 */
  NYLS_MIXED = 1,         /* FP32 kernel values, rotated into the eigenbasis and contracted
                             on the matrix cores (FP32 MFMA, FP64 cross-tile sums), FP64
                             eigen, solve and matrix-free FP64 iterative refinement;
                             m <= 126; bases with m + 2 > 64 take the FP64 Gram of
                             NYLS_FP64 instead of the FP32 one */
  NYLS_FP64_EXPLICIT = 2  /* reference-style FP64: explicit feature matrices, one instance
                             per launch sequence (a baseline, not the fast path) */
};

/* Return codes (negative: nothing was enqueued). */
enum {
  NYLS_OK = 0,
  NYLS_E_NULL = -1,       /* a required pointer is NULL */
  NYLS_E_BATCH = -2,      /* batch < 1 */
  NYLS_E_MODE = -3,       /* unknown mode, or the call does not support the plan's mode */
  NYLS_E_ORDER = -4,      /* p outside 1..NYLS_MAX_P */
  NYLS_E_SIZE = -5,       /* n < 2, n > NYLS_MAX_N, m < 2, m > n or m > NYLS_MAX_M (126 in mixed
                             mode, 128 in explicit mode and for the Newton and leverage calls) */
  NYLS_E_PARAM = -6,      /* sigma <= 0, gamma <= 0, tau outside [0, 1), or non-finite */
  NYLS_E_GRID = -7,       /* uniform grid with dt <= 0, or explicit grid missing */
  NYLS_E_LANDMARK = -8,   /* landmark indices not strictly ascending inside [0, n) */
  NYLS_E_COND = -9,       /* condition order outside 0..p-1, index outside [0, n), or a
                             duplicated (order, index) pair */
  NYLS_E_NONLINEAR = -10, /* Newton call on a plan whose instances are not all of order 1, or
                             all of order 2 */
  NYLS_E_HIP = -11,       /* a HIP runtime call failed */
  NYLS_E_ARG = -12        /* another argument is out of range (e.g. dmax, refine steps) */
};

/* Per-instance status bits (device int32 array written by the work functions). */
enum {
  NYLS_S_TRUNCATED = 1,       /* info: the basis kept r < m eigenpairs */
  NYLS_S_SINGULAR = 2,        /* a zero pivot in the KKT / Schur factorisation */
  NYLS_S_NONFINITE = 4,       /* a NaN or Inf appeared in the solution */
  NYLS_S_EIG_NOCONV = 8,      /* the eigensolver hit its iteration limit */
  NYLS_S_SMALL_PIVOT = 16,    /* Newton: a diagonal y-block entry |d_i| < 1e-10 gamma was met
                                 (up to 32 such points per step stay in the dense system:
                                 the step is exact; see NYLS_S_PIVOT_OVERFLOW) */
  NYLS_S_REFINE_NOCONV = 32,  /* refinement ended with its last change of y_hat above
                                 1e-8 max|y_hat| */
  NYLS_S_FP64_RESOLVED = 64,  /* NYLS_MIXED: refinement on the FP32 Gram did not converge, the
                                 instance was solved again with the FP64 Gram */
  NYLS_S_PARAM_KEPT = 128,    /* nyls_plan_set_params: the new sigma or gamma was not taken */
  NYLS_S_PIVOT_OVERFLOW = 256 /* Newton: more than 32 small pivots (or a non-finite one); the
                                 others were divided out as usual */
};

/*
 * One ODE instance, as stated in Sec. 3.1 (linear) or App. A.5 (nonlinear, p = 1).
 *   p          order, 1..4
 *   n          grid size; grid t_i = t0 + i*dt when uniform != 0, else t[i] (device,
 *              strictly ascending)
 *   m          number of landmarks (sub-sample size), 2 <= m <= min(n, NYLS_MAX_M).  Bases
 *              of more than 128 landmarks (the long-time runs of Sec. 4 use up to 200) are
 *              taken by NYLS_FP64 plans only, and by nyls_solve, nyls_predict,
 *              nyls_features and nyls_backward: such an instance is always split over chunks
 *              of grid points (nyls_tuning.split; 1024 points unless a size is set), its
 *              eigensolver and KKT factors work in the workspace instead of on-chip memory,
 *              and its passes run two wavefronts per chunk, one per half of the landmarks.
 *   lidx       HOST array of m strictly ascending grid indices, or NULL for the
 *              equidistant rule i_s = floor(s (n-1)/(m-1) + 1/2), s = 0..m-1 (Sec. 4.1)
 *   f          device [p][n]: f[(k-1)*n + i] = f_k(t_i); unused by the nonlinear path
 *   r          device [n]: forcing r(t_i); unused by the nonlinear path
 *   v          device [p]: condition values v_j
 *   cond_d/i   condition j prescribes y^(cond_d[j]) at grid index cond_i[j] (j < p).
 *              Grid points that carry a condition carry no ODE residual (IVP: the
 *              residual set is 2..n as in Lemma 1; two-point BVP: 2..n-1, App. A.4).
 *   sigma      RBF bandwidth (the kernel divides by sigma^2), > 0
 *   gamma      regularisation constant of the residual term, > 0
 *   tau        relative eigenvalue cut-off in [0, 1): eigenpairs with
 *              lambda_k <= tau * lambda_1 are dropped (the paper assumes K_mm positive
 *              definite; in FP64 it is numerically singular for smooth kernels)
 */
typedef struct nyls_problem {
  int32_t p, n, m, uniform;
  double t0, dt;
  const double* t;
  const int32_t* lidx;
  const double* f;
  const double* r;
  const double* v;
  int32_t cond_d[NYLS_MAX_P];
  int32_t cond_i[NYLS_MAX_P];
  double sigma, gamma, tau;
} nyls_problem;

typedef struct nyls_plan nyls_plan;

/* Validate `batch` instances (host array) and upload their descriptors; *out receives the
 * plan.  mode is NYLS_FP64, NYLS_MIXED or NYLS_FP64_EXPLICIT.  Device data pointers are
 * stored, not copied: they must stay valid while the plan is used, and new values written
 * into them are picked up by the next call.  Returns 0 or a NYLS_E* code (then *out = NULL). */
int nyls_plan_create(const nyls_problem* probs, int32_t batch, int32_t mode, nyls_plan** out);
void nyls_plan_destroy(nyls_plan* plan);
/* sigma and gamma of every instance from DEVICE arrays [batch] (Sec. 3.1: the kernel width
 * and the weight of the residual term), written into the plan's device descriptors by a
 * kernel on `stream`: no host synchronisation, so a training loop or a captured graph can
 * change them between solves without rebuilding the plan.  Either array may be NULL (kept).
 * A value that is not finite and positive, or a sigma below 4 dt for an instance whose plan
 * uses the strided Gaussian recurrence (uniform grid created with dt <= sigma / 4), is not
 * taken: that instance keeps both previous values and status[i] = NYLS_S_PARAM_KEPT, else
 * status[i] = 0 (status may be NULL).  The values persist for later calls, including across
 * nyls_plan_set_tuning.  Returns NYLS_E_NULL for a NULL plan. */
int nyls_plan_set_params(nyls_plan* plan, const double* sigma, const double* gamma, int32_t* status,
                         hipStream_t stream);
/* Launch choices of a plan (set by nyls_plan_set_tuning, e.g. from an autotuner's cache).
 * Every combination computes the same method; they differ in speed, and in rounding only
 * where the arithmetic order differs (the Gram path and its last column block, the point
 * ranges of split passes).
 *   eig_ql       0 = tridiagonal QL one lane per instance (ql_lanes instances per wavefront)
 *                with the plane rotations replayed onto Q by one wavefront per instance (for
 *                m > 64 only when the plan has at least 32 such instances, else as 1);
 *                1 = the whole QL inside one wavefront per instance
 *   ql_lanes     1..64 (default 64)
 *   gram_valu    FP64 Gram for m + 2 <= 64: 0 = one wavefront per instance on the matrix
 *                cores; 1 = 256-thread LDS tiles on the VALU
 *   tail_layout  1 = a last block of at most four landmarks (m = 16 k + 1..4) is walked in
 *                the tail layout by the refinement/output passes and accumulated on the VALU by
 *                the matrix-core Gram; 0 = treated as a full 16-slot block
 *   overlap      1 = FP64 solves run the kernel-space Gram on the plan's side stream beside
 *                the eigensolver (and, in batches with bases on both sides of 64 landmarks,
 *                the eigensolver of the m <= 64 ones on a second side stream beside that of
 *                the larger ones); FP64 and mixed solves run the refinement/output passes of
 *                different landmark-slot classes (m <= 32, <= 64, larger) on the three
 *                streams; 0 = everything in order on the caller's stream
 *   split        FP64 solves of long instances: grid points per workgroup when the Gram and
 *                the refinement/output passes of one instance are split over many
 *                workgroups (a multiple of 64, at least 512; every instance runs the chunked
 *                kernels, with one chunk when n <= split), 0 = never split, -1 = automatic
 *                (1024 when the plan has at most 64 instances, for those with n >= 4096;
 *                else never).  Instances with m > 128 are split whatever the setting (in
 *                chunks of 1024 points unless a size is set)
 * Defaults: {0, 64, 0, 1, 1, -1}. */
typedef struct nyls_tuning {
  int32_t eig_ql, ql_lanes, gram_valu, tail_layout, overlap, split;
} nyls_tuning;
/* Apply `tuning` to the plan (host call: updates the device descriptors synchronously; no
 * work of this plan may be in flight).  Returns NYLS_E_ARG for out-of-range fields.  The
 * workspace size (nyls_workspace_size) depends on `split`: query it again afterwards. */
int nyls_plan_set_tuning(nyls_plan* plan, const nyls_tuning* tuning);
int nyls_plan_get_tuning(const nyls_plan* plan, nyls_tuning* tuning);

/* Bytes of device workspace every work function of this plan needs. */
size_t nyls_workspace_size(const nyls_plan* plan);
/* Sum of n over the batch: length of per-grid-point outputs (yhat, dL/dr, ...).
 * Instance i's points start at the prefix sum of the n before it. */
int64_t nyls_total_points(const nyls_plan* plan);
/* MAXM of the batch (the padded stride of omega, eigval and phi). */
int32_t nyls_max_m(const nyls_plan* plan);
/* Copy each instance's diagnostics block from `ws` into info [batch][8] (device, FP64):
 *   [0] retained rank r, [1] status bits, [2] eigensolver sweeps, [3] last change of
 *   y_hat measured by the refinement, [4] 1 if the FP64 Gram was accumulated in the
 *   eigenbasis, [5] refinement passes of the last nyls_solve, [6] refinement passes of the
 *   last nyls_backward, [7] unused (0).  Values are those of the work functions enqueued
 *   before it on `stream`. */
int nyls_instance_info(const nyls_plan* plan, const void* ws, double* info, hipStream_t stream);

/* Copy each instance's eigendecomposition K_mm = U Lambda U^T (App. A.2, eq32) from `ws`:
 *   lam  [batch][MAXM] eigenvalues, descending (entries k >= m zero)
 *   U    [batch][MAXM][MAXM] eigenvectors as columns, U[i][s][k] (row s, column k; entries
 *        outside m x m zero), each signed so its largest-magnitude entry is positive
 * Either pointer may be NULL (not copied); both device memory.  Valid after a call that
 * forms the basis (nyls_solve, nyls_solve_static, nyls_features, nyls_assemble,
 * nyls_newton_init) and before the next plan change; values are those of the work
 * enqueued before it on `stream`.  Nothing here changes ws. */
int nyls_basis(const nyls_plan* plan, const void* ws, double* lam, double* U, hipStream_t stream);

/* Feature map (App. A.2 eq32, Sec. 3): eigendecompose K_mm and evaluate
 * phi^(d)(t) for d = 0..dmax (dmax <= 4) at caller times.
 *   t_eval    [E] evaluation times, instance i owns t_eval[eval_off[i] .. eval_off[i+1])
 *   eval_off  [batch+1] int64 offsets (device)
 *   phi       [E][dmax+1][MAXM]: phi[e][d][k], columns k >= rank are zero
 *   eigval    [batch][MAXM] eigenvalues of K_mm, descending (may be NULL)
 *   rank      [batch] int32 retained rank r (may be NULL)
 * Eigenvectors are signed so that their largest-magnitude entry is positive. */
int nyls_features(const nyls_plan* plan, const double* t_eval, const int64_t* eval_off,
                  int32_t dmax, double* phi, double* eigval, int32_t* rank, void* ws,
                  hipStream_t stream);

/* Leverage-score landmark sampling (Sec. 4.1 compares equidistant, random and
 * leverage-score landmarks; the paper gives no score formula).  Ridge leverage scores of
 * every grid point in the feature space of the plan's own (pilot) basis,
 *     l_i = phi(t_i)^T (Phi^T Phi + ridge I)^{-1} phi(t_i),   Phi = [phi(t_i)]_{i < n},
 *   ridge   > 0, or 0 for 1/gamma of each instance (the ridge of the LS-SVM objective)
 *   scores  [total points] output
 * Builds the basis in `ws` first (as nyls_features does) and leaves intermediate products in
 * it, so nyls_predict and nyls_backward need a new nyls_solve afterwards. */
int nyls_leverage_scores(const nyls_plan* plan, double ridge, double* scores, void* ws,
                         hipStream_t stream);

/* m distinct landmarks per instance (m of its plan) drawn with probabilities proportional to
 * scores, without replacement, by exponential keys ln(u_i) / scores_i (the m largest; ties
 * to the lower index; Efraimidis and Spirakis, 2006):
 *   u     [total points] caller-drawn uniforms in (0, 1]
 *   ends  nonzero: grid points 0 and n-1 are always landmarks and m - 2 keys are taken
 *         from the interior
 *   lidx  [batch][MAXM] int32 output, ascending; entries past m are -1.
 * A new plan with these indices as nyls_problem.lidx solves on the sampled basis. */
int nyls_leverage_sample(const nyls_plan* plan, const double* scores, const double* u,
                         int32_t ends, int32_t* lidx, hipStream_t stream);

/* Assemble the Lemma 1 system (Sec. 3.1) in feature coordinates (omega, b, lambda):
 *   kkt [batch][KN*KN]: instance i's N = m+1+p system in the leading N x N block
 *       (row stride N), rows/columns of dropped eigen-directions replaced by identity;
 *   rhs [batch][KN]. */
int nyls_assemble(const nyls_plan* plan, double* kkt, double* rhs, void* ws, hipStream_t stream);

/* Solve the Lemma 1 system and evaluate y_hat on the grid.
 *   refine_steps  most FP64 iterative-refinement steps after the solve, 0..8.  Each step
 *                 forms the exact residual matrix-free from one pass over the points (and
 *                 writes y_hat of the current solution).  The iteration stops once the
 *                 change of y_hat (measured, or bounded by |d omega|_2 + |d b|) falls below
 *                 1e-11 max|y_hat|, or once a change is more than half the previous one
 *                 (rounding floor reached); when the correction just solved is predicted
 *                 to be that small (the last measured change times the ratio of the two
 *                 latest corrections' bounds) no further residual is formed, and a pass
 *                 that only evaluates y_hat applies and measures it.  The fused modes
 *                 factor an approximation of the system (a kernel-space FP64 Gram, or an
 *                 FP32 Gram), so >= 2 steps are recommended when K_mm is ill-conditioned;
 *                 NYLS_FP64_EXPLICIT assembles the exact system (0 steps suffice).
 *   omega [batch][MAXM], bias [batch], lambda [batch][4], yhat [total points] (each may
 *   be NULL except yhat), status [batch] int32.  The basis, LU factors and solution stay
 *   in `ws` for nyls_predict and nyls_backward. */
int nyls_solve(const nyls_plan* plan, int32_t refine_steps, double* omega, double* bias,
               double* lambda, double* yhat, int32_t* status, void* ws, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): nyls_solve with its workspace in a
 * library-owned device array of NYLS_STATIC_WS_BYTES per GPU (held from library load until
 * the process ends) instead of a caller-allocated `ws`.  Same kernels, arguments and
 * results as nyls_solve; the call allocates nothing.
 *   - Returns NYLS_E_SIZE when nyls_workspace_size(plan) exceeds NYLS_STATIC_WS_BYTES
 *     (about 350 instances at m = 50), NYLS_E_MODE for NYLS_FP64_EXPLICIT plans (their GEMM
 *     library may allocate), NYLS_E_HIP when the array's device address cannot be found.
 *   - The used part of the array is cleared (by a kernel on `stream`) before the solve.
 *   - All calls on one GPU share that GPU's array: calls that overlap in time on one GPU
 *     (different streams or threads) race and give wrong results; serialise them.  The
 *     array keeps the last call's basis, factors and solution, but nyls_predict and
 *     nyls_backward take a caller workspace, so they cannot continue from this call. */
#define NYLS_STATIC_WS_BYTES ((size_t)64 << 20)
int nyls_solve_static(const nyls_plan* plan, int32_t refine_steps, double* omega, double* bias,
                      double* lambda, double* yhat, int32_t* status, hipStream_t stream);

/* y_hat^(d)(t) = alpha^T k_m^(d)(t) + [d == 0] b at caller times, from the solution a
 * previous nyls_solve or nyls_newton_step left in `ws` (d = 0..4). */
int nyls_predict(const nyls_plan* plan, const double* t_eval, const int64_t* eval_off,
                 int32_t d, double* out, const void* ws, hipStream_t stream);

/* Newton iteration on the Lemma 2 system (Sec. 3.2) of a nonlinear ODE
 *     p = 1:  y'  = F(t, y)          (App. A.5)
 *     p = 2:  y'' = F(t, y, y')      (the appendix section on Problem 15)
 * with unknowns (omega, b, lambda_1..lambda_p, y_i over the residual set): y itself enters F
 * through the auxiliary unknown y_i, y' through the model, omega^T phi'(t_i).  Every
 * instance of the plan must have the same order, 1 or 2 (else NYLS_E_NONLINEAR), and its p
 * conditions as in nyls_problem (IVP or two-point BVP).  State x is [batch][XS] with
 * XS = nyls_newton_state_stride(plan) = MAXM + 1 + p + NMAX (NMAX = max n):
 * x = (omega[MAXM], b, lambda[p], y[n]) with y indexed by grid point (entries at condition
 * points are unused).
 *
 * nyls_newton_init: build the basis (and, for p = 1, the constant Jacobian blocks) in `ws`
 * and write the starting point omega = 0, lambda = 0, b = y_i = the value of the first
 * condition on y itself (0 if there is none) into x. */
int nyls_newton_init(const nyls_plan* plan, double* x, void* ws, hipStream_t stream);
int64_t nyls_newton_state_stride(const nyls_plan* plan);

/* The state values F is evaluated at, for the current x: u [p][total points] with
 * u[0][i] = y_i (y_hat(t_i) at condition points) and, for p = 2, u[1][i] = y_hat'(t_i). */
int nyls_newton_state(const nyls_plan* plan, const double* x, double* u, const void* ws,
                      hipStream_t stream);

/* One step x <- x - J^{-1} Y of Lemma 2's Newton method (Sec. 3.2).
 *   F    [total points] F at the state values u of nyls_newton_state
 *   dF   [p][total points] dF/du_a (a = 0: y, a = 1: y')
 *   d2F  [p][p][total points] d2F/du_a du_b (symmetric; zero gives the Gauss-Newton step)
 *        (for p = 1 these are F, Fy and Fyy)
 *   x    [batch][XS] in/out
 *   step_inf  [batch] |dx|_inf of this step (may be NULL)
 * The diagonal y-block d_i = gamma (1 + F_y^2 - rho_i F_yy) is eliminated first (Schur
 * complement on (omega, b, lambda)), so a step costs O(n m^2 + m^3); for p = 2 the whole
 * weighted Gram is formed again each step (the y' dependence makes every block depend on
 * the iterate).  |d_i| < 1e-10 gamma sets NYLS_S_SMALL_PIVOT; for p = 1 up to 32 such
 * points per instance are not divided out but stay unknowns of the dense system, which is
 * then solved by LU in the workspace (the step is the exact Newton step; more than 32 set
 * NYLS_S_PIVOT_OVERFLOW).  Afterwards nyls_predict evaluates the current y_hat. */
int nyls_newton_step(const nyls_plan* plan, const double* F, const double* dF,
                     const double* d2F, double* x, double* step_inf, int32_t* status,
                     void* ws, hipStream_t stream);

/* The Riccati right-hand side F(t, y) = q(t) - y^2 of the first-order nonlinear workload,
 * evaluated at the current Newton state x: F = q_i - y_i^2, Fy = -2 y_i, Fyy = -2 (0 when
 * gauss_newton != 0, i.e. the Gauss-Newton y-block).  q, F, Fy, Fyy are [total points].
 * First-order plans only (else NYLS_E_NONLINEAR). */
int nyls_riccati_eval(const nyls_plan* plan, const double* q, const double* x,
                      int32_t gauss_newton, double* F, double* Fy, double* Fyy,
                      hipStream_t stream);

/* Adjoint of nyls_solve (FP64): gradients of a loss l(y_hat(s_1..s_J)) given
 * g_j = dl/dy_hat(s_j), reusing the factorisation left in `ws` by nyls_solve.
 *   t_obs [J_total], obs_off [batch+1] int64, dl_dyobs [J_total]
 *   dl_df [4][total points]: dl/df_k(t_i) of instance i at dl_df[(k-1)*total + off_i + i]
 *         (rows k > p left untouched); dl_dr [total points];
 *   dl_dv [batch][4]; dl_dsigma [batch]; dl_dgamma [batch]  (outputs may be NULL)
 * Gradients w.r.t. the data f, r, v are exact derivatives of the Lemma 1 solution;
 * sigma enters through the kernel values and through K_mm (spectral derivative).  The
 * adjoint solve is refined in FP64 (matrix-free, up to three steps) because the stored
 * factors are of an approximate system; it stops once the correction, or the next one
 * predicted from the contraction seen so far, is below 1e-8 of the solution, or at the
 * rounding floor.  Not available for
 * NYLS_FP64_EXPLICIT plans. */
int nyls_backward(const nyls_plan* plan, const double* t_obs, const int64_t* obs_off,
                  const double* dl_dyobs, double* dl_df, double* dl_dr, double* dl_dv,
                  double* dl_dsigma, double* dl_dgamma, void* ws, hipStream_t stream);

/* Optional kernel timing for measurement tools: when enabled, every kernel launch of the
 * work functions is bracketed by HIP events on its stream (a few microseconds per launch).
 * nyls_profile_read synchronises the recorded events and returns the accumulated time
 * and launch count of one kernel: 0 basis/eigen, 1 FP64 Gram, 2 FP32 (MFMA) Gram, 3 KKT
 * assembly + LU, 4 refinement/output pass, 5 features, 6 predict, 7 explicit baseline,
 * 8 Newton step, 9 adjoint.  Host-side state, not thread-safe. */
void nyls_profile_enable(int32_t on);
int nyls_profile_read(int32_t kernel, double* total_ms, int64_t* count);
void nyls_profile_reset(void);

/* Static text for a NYLS_E* code or a single NYLS_S* bit. */
const char* nyls_error_string(int32_t code);

#ifdef __cplusplus
}
#endif
#endif /* NYLS_H */
