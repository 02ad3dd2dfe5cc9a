/*
 * inla_bta.h -- C ABI of the MI355X (gfx950) library that evaluates the INLA
 * hyperparameter objective f(theta) = -log pi~(theta | y) and its gradient for
 * Gaussian latent models whose precision matrices are block tridiagonal with an
 * arrowhead (BTA): nt dense time blocks of size b = ns (the spatial nodes) on
 * the diagonal, dense coupling blocks between consecutive time steps, and a
 * dense border of width a = nb (the fixed effects, ordered last).
 *
 * Paper: "Parallelized integrated nested Laplace approximations for fast
 * Bayesian inference".  Objective: Sec. "Parallel Optimization" (f as the
 * negative log of eq. post_theta_approx).  Factorization, log-determinant and
 * forward/backward substitution: Sec. "Sparse Linear Algebra".  Selected
 * inversion: Sec. "Partial Inversion" (eq. sel_inv_cov, eq. takahashi_identity,
 * eq. takahashi_recursion), applied here block-wise.  Batches of independent
 * theta points: Sec. "Parallel Optimization" (all central-difference points of
 * eq. central_diff are independent) and Sec. "Parallel Line Search".
 *
 * Conventions shared by every entry point:
 *   - FP64 only.  All matrices are column-major.
 *   - Pointers named *_dev, and every block pointer inside inla_bta, are device
 *     pointers owned by the caller; the library never frees them.
 *   - Every call except inla_model_create is enqueued on the caller's HIP
 *     stream (a hipStream_t passed as void*; NULL = the default stream) and
 *     returns before the device work finishes.  Results become valid once the
 *     caller synchronises that stream.
 *   - Argument errors, allocation failures and launch failures are returned
 *     synchronously as an inla_status; inla_last_error() gives details for the
 *     calling thread.  Numerical failure (a non-positive pivot) is reported
 *     asynchronously through the per-item status/info outputs.
 *   - Calls that use the library's internal workspace (factor, selinv, eval)
 *     serialise on an internal lock; issuing them from several threads is safe
 *     but they do not overlap.
 */
#ifndef INLA_BTA_H
#define INLA_BTA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  INLA_OK = 0,
  INLA_ERR_ARG = -1,     /* invalid argument (dims, pointers, theta out of range) */
  INLA_ERR_NOT_SPD = -2, /* reserved for synchronous SPD failures (async ones use info) */
  INLA_ERR_BUDGET = -3,  /* one item alone exceeds the HBM budget */
  INLA_ERR_HIP = -4,     /* a HIP runtime call or kernel launch failed */
  INLA_ERR_NOMEM = -5,   /* device or host allocation failed */
  INLA_ERR_STATE = -6    /* library not usable (no device, wrong architecture) */
} inla_status;

/*
 * One BTA matrix.  Block (t,t) is D[t], block (t+1,t) is S[t], block (A,t) is
 * R[t], block (A,A) is T.  Storage is contiguous per kind:
 *   D: nt blocks b x b, block t at D + t*b*b, leading dimension b;
 *   S: nt-1 blocks b x b, block t at S + t*b*b, leading dimension b (NULL if nt == 1);
 *   R: nt blocks a x b, block t at R + t*a*b, leading dimension a (NULL if a == 0);
 *   T: a x a, leading dimension a (NULL if a == 0).
 * As an input precision matrix only the lower triangles of D[t] and T are read.
 *
 * Factor format written by inla_factor_logdet (the inverse-diagonal block
 * Cholesky form, Q = L L^T):
 *   D[t] <- inv(L_tt)          lower triangular, zeros stored above the diagonal
 *   S[t] <- L_{t+1,t}          full block
 *   R[t] <- L_{A,t}            full block
 *   T    <- inv(L_AA)          lower triangular, zeros stored above the diagonal
 * Keeping the inverses of the diagonal factor blocks turns every later use
 * (the off-diagonal solves, the substitution sweeps, the selected inversion)
 * into plain matrix products.  log|Q| = -2 sum log diag(D[t]) - 2 sum log diag(T).
 */
typedef struct {
  int32_t b, nt, a;
  double *D, *S, *R, *T;
} inla_bta;

/* Opaque model: grid stencils, A^T A split into BTA blocks, A in CSR, y. */
typedef struct inla_model inla_model;

/*
 * Host description of one model (copied by inla_model_create).
 * Latent order x = (u_0, ..., u_{nt-1}, beta), u_t in R^{N*N} with node
 * (ix, iy) at index iy*N + ix; n = N*N*nt + nb.
 *   N, nt, nb  : grid side (>= 1), time steps (>= 1), fixed effects (0..64)
 *   h          : grid spacing; C = h^2 I in Q_s = tau^2 (kappa^2 C + G) C^{-1} (kappa^2 C + G)
 *   beta_prior_prec : prior precision of every fixed effect
 *   m, A_rowptr (m+1, int64), A_col (int32), A_val : observation matrix, m x n CSR.
 *                Every row's space-time entries must lie in one time block.
 *   y          : m responses
 *   theta_prior_mean, theta_prior_prec : 4 each, independent Gaussian hyperprior
 * theta = (log tau, log kappa, atanh rho, log tau_y): spatial scale, spatial
 * range parameter, AR1 correlation in time, Gaussian noise precision.
 */
typedef struct {
  int32_t N, nt, nb;
  double h;
  double beta_prior_prec;
  int64_t m;
  const int64_t *A_rowptr;
  const int32_t *A_col;
  const double *A_val;
  const double *y;
  const double *theta_prior_mean;
  const double *theta_prior_prec;
} inla_model_desc;

/*
 * Options of inla_eval_f / inla_eval_f_grad (NULL = all zero).
 *   hbm_budget_bytes : device bytes the batch may occupy; items are admitted
 *                      in waves that fit (0: free memory minus a 4 GiB reserve)
 *   recompute        : 1 = Q_prior and Q_c of an item share one BTA storage
 *                      and workspace and are processed one after the other
 *                      (about half the memory per item, two dependent chains
 *                      instead of one batched chain); 2 = never; 0 = when it
 *                      needs fewer admission waves.  Selected-inverse blocks
 *                      are never stored in either mode: each is recomputed
 *                      from the stored factor and consumed as it is produced.
 *                      When the selected inversion's per-step launches would
 *                      have few tiles, its factor-only parts of every step
 *                      (V_t, U_t, inv(L_tt)^T inv(L_tt); about one more BTA
 *                      matrix of memory) are formed up front if that needs
 *                      no more admission waves (the results agree bitwise
 *                      with 64-wide tiles, to rounding with 128-wide ones).
 *   keep_sigma       : 1 = also keep the selected inverse of Q_c: item i's
 *                      Sigma blocks on the BTA pattern (D[t] full symmetric
 *                      blocks, S[t] = block (t+1,t), R[t], T) are written to
 *                      the caller's storage sigma_out[i] (a host array of
 *                      n_items descriptors of device storage, each of the
 *                      item's model shape; Sec. "Partial Inversion"); no
 *                      graph is captured for such a call, and its matrices
 *                      are eliminated from the first time block on (see
 *                      below).  0 = not kept.
 *   sigma_out        : see keep_sigma (ignored when keep_sigma = 0)
 *   tile             : 64 or 128 forces the tile of the b x b products;
 *                      0 = the autotuner's entry for this call signature if
 *                      autotune_cache is set, else a built-in rule
 *   autotune_cache   : path of a JSON file (or NULL).  On the first call with
 *                      a new signature (the multiset of item shapes and the
 *                      outputs asked for) every candidate (the tile edge and
 *                      the product kernel's layout, then the fused and the
 *                      batched Cholesky step with the best of those) is timed
 *                      once on the caller's stream, synchronously, and the
 *                      fastest is stored; later calls and processes read it
 *                      back.
 * Results with different tile layouts agree to rounding (about 1e-15
 * relative), not bitwise.
 *
 * Elimination order: a matrix with four or more time blocks is eliminated
 * from both ends at once -- time blocks 0, 1, .. up to the middle block
 * m = ceil(nt/2) and nt-1, nt-2, .. down to m+1 in the same launches, the
 * middle block last before the arrow -- which halves the sequential chain of
 * the factorization, the substitution and the selected inversion (every
 * elimination order of the blocks gives the same determinant, mode and
 * inverse; rounding differs, about 1e-15 relative).  It reads each coupling
 * block of the backward half as the transpose of the stored one, which the
 * assembled precision matrices satisfy (each is a multiple of the symmetric
 * spatial precision).  INLA_TWIST=0 in the environment keeps the one-sided
 * order.
 */
typedef struct {
  double hbm_budget_bytes;
  int32_t recompute;
  int32_t keep_sigma;
  int32_t tile;
  int32_t reserved;
  const char *autotune_cache;
  const inla_bta *sigma_out;
} inla_opts;

/*
 * Build a model on the current device (Sec. "Latent Gaussian Models").
 * Copies the description, builds the spatial stencil and the per-time-step
 * A^T A, Z^T A and Z^T Z blocks on the host, uploads them, and synchronises
 * `hip_stream`.  *out is owned by the caller and freed by inla_model_destroy.
 */
inla_status inla_model_create(const inla_model_desc *desc, void *hip_stream, inla_model **out);
void inla_model_destroy(inla_model *model);
/* Shape of a model: b = N*N, nt, a = nb, n, m (any output pointer may be NULL). */
inla_status inla_model_shape(const inla_model *model, int32_t *b, int32_t *nt, int32_t *a,
                             int64_t *n, int64_t *m);

/*
 * Assemble Q_prior(theta) (which = 0) or Q_c(theta) = Q_prior + tau_y A^T A
 * (which = 1) into the caller's BTA storage `out` (shape must equal the
 * model's; every block is written in full, both triangles).  With which = 1
 * and rhs_dev != NULL also writes b = tau_y A^T y (n doubles).  theta_dev: 4
 * doubles on the device.  Sec. "Latent Gaussian Models", and Sec.
 * "Approximating pi(theta_j | y)" for conditioning keeping the pattern.
 */
inla_status inla_assemble(const inla_model *model, const double *theta_dev, int32_t which,
                          inla_bta *out, double *rhs_dev, void *hip_stream);

/*
 * In-place block Cholesky of one BTA matrix (Sec. "Sparse Linear Algebra"),
 * into the inverse-diagonal factor format described at inla_bta.
 * logdet_dev (1 double, may be NULL) <- log|Q|;  info_dev (1 int32, may be
 * NULL) <- 0, or the 1-based row of the first non-positive pivot, in which
 * case the factor and log-determinant are not meaningful (log|Q| is NaN).
 */
inla_status inla_factor_logdet(inla_bta *QL, double *logdet_dev, int32_t *info_dev, void *hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * factorization as inla_factor_logdet, with the same results bit for bit, but
 * its workspace (two b x b panels, the arrow panel, the diagonal-tile scratch,
 * the log-determinant partial sums and the item descriptor) lives in one
 * fixed device array of INLA_NOALLOC_SCRATCH_BYTES per GPU instead of the
 * library's growable workspace.  The array is set up on the first call on a
 * device (with that device current) and held until the process ends; no
 * call allocates or frees device memory, and none stages data in host memory.
 * A matrix whose workspace does not fit (about 2 b^2 + a b + nt ceil(b/64)
 * doubles; b up to about 2048) is rejected with INLA_ERR_BUDGET before
 * anything is enqueued.  Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU (on different streams without ordering between
 * them) race.  Not profiled by inla_profile_begin/end.
 */
#define INLA_NOALLOC_SCRATCH_BYTES (64u << 20)
inla_status inla_factor_logdet_noalloc(inla_bta *QL, double *logdet_dev, int32_t *info_dev,
                                       void *hip_stream);

/*
 * Solve Q X = RHS with the factor from inla_factor_logdet by forward then
 * backward substitution (Sec. "Sparse Linear Algebra").  rhs_dev, x_dev:
 * n x nrhs column-major (n = b*nt + a); they may alias.
 */
inla_status inla_solve(const inla_bta *L, const double *rhs_dev, double *x_dev, int32_t nrhs,
                       void *hip_stream);

/*
 * Selected inversion of Q from its factor (Sec. "Partial Inversion"): the
 * blocks of Sigma = Q^{-1} on the BTA pattern, computed by the block form of
 * the Takahashi recursion from the last time block to the first.
 * sigma_or_null: if non-NULL, receives Sigma's D (full symmetric blocks), S
 * (block (t+1,t)), R and T blocks, same shapes as L.  diag_or_null: if
 * non-NULL, receives the n marginal variances diag(Q^{-1}).
 */
inla_status inla_selinv(const inla_bta *L, inla_bta *sigma_or_null, double *diag_or_null,
                        void *hip_stream);

/*
 * f(theta) for n_items independent (model, theta) items in one batched pass
 * (Sec. "Parallel Optimization": independent evaluations run together).
 * models[i] may repeat.  theta_dev: n_items x 4 (row i = item i).
 *   f_dev      : n_items
 *   mu_or_null : concatenation over items of the posterior mode mu (n_i each)
 *   var_or_null: concatenation over items of the marginal variances diag(Q_c^{-1})
 *   status_dev : n_items int32: 0 ok, 1 = Q_prior not positive definite,
 *                2 = Q_c not positive definite, 3 = theta outside the parameter
 *                space (a non-finite entry, or tanh(theta_3) = +-1 in FP64);
 *                f (and the gradient) are NaN for such an item, the other
 *                items of the batch are unaffected
 * Items are admitted in waves so that the BTA storage stays within the HBM
 * budget of opts (NULL opts = defaults).
 */
inla_status inla_eval_f(const inla_model *const *models, int32_t n_items, const double *theta_dev,
                        double *f_dev, double *mu_or_null, double *var_or_null, int32_t *status_dev,
                        const inla_opts *opts, void *hip_stream);

/*
 * As inla_eval_f, plus grad_dev (n_items x 4) <- the exact gradient of f,
 * from the selected-inversion blocks of Q_prior and Q_c:
 *   df/dtheta_k = p_k (theta_k - m_k) - 1/2 tr(Q_p^{-1} dQ_p/dtheta_k)
 *                 + 1/2 tr(Q_c^{-1} dQ_c/dtheta_k) + 1/2 mu^T (dQ_p/dtheta_k) mu
 *                 + [k = 4] (tau_y/2 |y - A mu|^2 - m/2).
 * The selected-inverse blocks are consumed as they are produced and not kept.
 */
inla_status inla_eval_f_grad(const inla_model *const *models, int32_t n_items,
                             const double *theta_dev, double *f_dev, double *grad_dev,
                             double *mu_or_null, double *var_or_null, int32_t *status_dev,
                             const inla_opts *opts, void *hip_stream);

/*
 * f now, its gradient later (the backward pass of an automatic-differentiation
 * framework, or the one accepted point of a line search).  inla_eval_f_keep
 * computes f (and mu) for the batch like inla_eval_f and, when the batch's two
 * factors per item fit the HBM budget in one wave, keeps them in a device
 * allocation owned by the returned state; inla_eval_grad_kept then runs only
 * the selected inversions of the kept factors with their trace reductions
 * (the selected-inverse blocks are recomputed from the stored factors,
 * Sec. "Partial Inversion") and returns f, grad f, the status and optionally
 * the marginal variances -- the same values, bit for bit, as inla_eval_f_grad
 * under the same options.  When the factors do not fit (or recompute = 1 asks
 * for shared storage) the state keeps only theta, and inla_eval_grad_kept runs
 * the whole evaluation again (inla_eval_state_kept tells which).  The models
 * must outlive the state; inla_eval_grad_kept may be called more than once;
 * inla_eval_state_destroy waits for the state's last call and frees it.
 * keep_sigma is not accepted here.
 */
typedef struct inla_eval_state inla_eval_state;
inla_status inla_eval_f_keep(const inla_model *const *models, int32_t n_items,
                             const double *theta_dev, double *f_dev, double *mu_or_null,
                             int32_t *status_dev, const inla_opts *opts, void *hip_stream,
                             inla_eval_state **state_out);
inla_status inla_eval_grad_kept(inla_eval_state *state, double *f_dev, double *grad_dev,
                                double *var_or_null, int32_t *status_dev, void *hip_stream);
int32_t inla_eval_state_kept(const inla_eval_state *state);
void inla_eval_state_destroy(inla_eval_state *state);

/*
 * Robust quadratic fit (Sec. "Parallel Line Search": the second-order
 * polynomial through the line-search points by robust regression with
 * bisquare weights).  Host-only: x, y are n >= 3 host doubles (finite, x not
 * all equal); coef[3] receives q(x) = coef[0] + coef[1] x + coef[2] x^2.
 * Iteratively reweighted least squares from the ordinary fit: residual scale
 * s = median |r_i| / 0.6745, weights w_i = (1 - (r_i / (4.685 s))^2)^2 for
 * |r_i| < 4.685 s, else 0, until the weights change by less than 1e-12 (at
 * most 200 rounds); with s = 0 the points off the fit get weight 0.
 * weights_or_null receives the final weights (n doubles).  INLA_ERR_ARG for
 * bad input or fewer than three usable points.
 */
inla_status inla_robust_quadratic_fit(const double *x, const double *y, int32_t n, double *coef,
                                      double *weights_or_null);

/*
 * Options of inla_bfgs_minimize (NULL = defaults; a field <= 0 = its default).
 *   max_iter  : BFGS iterations (300)
 *   n_points  : candidate points on the search interval per iteration (6);
 *               two stabilising points are added on the other side of theta
 *   gamma     : upper bound of the step length along -p (1: the quasi-Newton step)
 *   gtol      : stop when max_k |df/dtheta_k| <= gtol (1e-6)
 *   ftol      : stop when an iteration lowers f by <= ftol max(1, |f|) (1e-13)
 *   eval_opts : options of the evaluations (NULL = defaults)
 *   max_step  : an iteration's interval is shortened so that no theta_k moves
 *               by more than max_step (2.0)
 */
typedef struct {
  int32_t max_iter;
  int32_t n_points;
  double gamma;
  double gtol;
  double ftol;
  const inla_opts *eval_opts;
  double max_step;
} inla_bfgs_opts;

/* reason: 0 gradient below gtol, 1 decrease of f below ftol, 2 max_iter,
 * 3 no point of the search interval (shrunk 8 times by 4) lowered f. */
typedef struct {
  double theta[4], f, grad[4];
  int32_t iterations, f_evals, grad_evals, reason;
} inla_bfgs_result;

/*
 * Minimise f(theta) for one model from theta0 (4 host doubles): BFGS
 * (eq. bfgs_update) with the exact adjoint gradient at every accepted iterate,
 * and the parallel line search of Sec. "Parallel Line Search" (Fig.
 * parallel_linsearch): with p = H grad f (H the inverse-Hessian approximation,
 * the first direction of unit length) and gamma shortened to max_step / max |p_k|
 * where it would move some theta_k farther, the n_points candidates
 * theta - alpha p, alpha = gamma i / n_points, and the two stabilising points
 * alpha = -gamma/8, -gamma/4 are evaluated in ONE batched inla_eval_f call; a
 * robust quadratic (inla_robust_quadratic_fit) through them and f(theta) is
 * minimised on (0, gamma] and that point becomes the next iterate (if an
 * evaluated candidate is lower than f there, that candidate; if nothing
 * lowers f, the interval shrinks by 4; the next iteration's interval is
 * max(gamma, 2 alpha) for the step alpha just taken).  The inverse Hessian is scaled by
 * s^T y / y^T y at the first update and updated only when s^T y > 0.
 * Synchronises hip_stream once per evaluation (the decisions are on the host).
 * history_or_null: host buffer of (max_iter + 1) x 8 doubles, row l =
 * (f, max |grad f|, alpha, theta[4], f evaluations so far) after iteration l.
 * Returns INLA_ERR_NOT_SPD if f cannot be evaluated at theta0.
 */
inla_status inla_bfgs_minimize(const inla_model *model, const double *theta0,
                               const inla_bfgs_opts *opts, inla_bfgs_result *res,
                               double *history_or_null, void *hip_stream);

/*
 * Options of inla_integrate (NULL = defaults; a field <= 0 = its default).
 *   h         : step of the central differences of the gradient (1e-3)
 *   dz        : grid step in standardised coordinates (1)
 *   dpi       : keep a point when f(theta) - f(theta*) < dpi (2.5)
 *   max_steps : steps per direction of the axis exploration (6)
 *   max_box   : the box of grid points may hold at most this many (20000)
 *   eval_opts : options of the evaluations (NULL = defaults)
 */
typedef struct {
  double h;
  double dz;
  double dpi;
  int32_t max_steps;
  int32_t max_box;
  const inla_opts *eval_opts;
} inla_integrate_opts;

/* Result of inla_integrate.  Matrices are row-major; eigvec[4 i + j] is entry
 * i of eigenvector j.  lo[j] / hi[j]: the axis ranges, in grid steps, on the
 * negative / positive side of direction j.  n_points: the points kept (K);
 * n_box: the candidates evaluated. */
typedef struct {
  double f_mode, grad_mode[4];
  double hessian[16];
  double eigval[4], eigvec[16];
  double theta_mean[4], theta_cov[16];
  double log_evidence;
  int32_t lo[4], hi[4];
  int32_t n_box, n_points, f_evals, grad_evals;
} inla_integrate_result;

/*
 * The integration step after the mode search for one model (Sec. "Latent
 * Gaussian Models": points around theta* at which pi~(theta | y) is evaluated
 * for the numerical integration of the hyperparameter marginals; Sec.
 * "Approximating pi(x_i | y)", eq. LatParam: the latent marginals integrated
 * over those points, one partial inversion per point; Sec. "Parallelization
 * of Function Evaluations": the points and their partial inversions are
 * independent and evaluated in batched calls).  The paper fixes no design of
 * the points; this one is the standardised grid of Rue, Martino and Chopin
 * (2009):
 *   1. H = Hessian of f at theta_mode by central differences of the adjoint
 *      gradient (theta_mode and theta_mode +- h e_k in ONE batched
 *      inla_eval_f_grad call), symmetrised;
 *   2. H = V diag(lambda) V^T, lambda ascending, each eigenvector's
 *      largest-magnitude entry positive (INLA_ERR_NOT_SPD if some
 *      lambda <= 0); theta(z) = theta_mode + V diag(lambda^{-1/2}) z;
 *   3. along each direction +-e_j in z, steps s = 1..max_steps of length dz
 *      while f(theta(s dz e_j)) - f* < dpi (all 2 x 4 x max_steps points in one
 *      batched inla_eval_f call): the ranges lo[j], hi[j];
 *   4. every z = dz s, s integer in the box [-lo, hi], evaluated in batched
 *      calls (INLA_ERR_ARG if the box holds more than max_box points) and kept
 *      when f - f* < dpi (f* = f(theta_mode) of step 1; an item whose Q is not
 *      positive definite counts as f = +inf);
 *   5. w_k = exp(-(f_k - f*)) / sum; E[theta|y], Cov[theta|y] the weighted
 *      sums; log pi(y) = -f* + log sum exp(-(f_k - f*)) + 4 log dz
 *      - sum_j log(lambda_j) / 2;
 *   6. if x_mean_dev or x_var_dev is non-NULL (device, n doubles each): the
 *      mean and variance of the mixture sum_k w_k N(mu(theta^k),
 *      diag Q_c(theta^k)^{-1}) (eq. LatParam with the Gaussian conditionals),
 *      mu and the marginal variances at the K points from batched inla_eval_f
 *      calls (K selected inversions).
 * points_or_null: host, up to points_cap rows of 10 doubles, one per kept
 * point in lexicographic order of s: s[4], theta[4], f, w.
 * Synchronises hip_stream (the decisions are on the host); allocates device
 * buffers for the batches (at most about 1 GiB for the latent step).
 */
inla_status inla_integrate(const inla_model *model, const double *theta_mode,
                           const inla_integrate_opts *opts, inla_integrate_result *res,
                           double *points_or_null, int32_t points_cap, double *x_mean_dev,
                           double *x_var_dev, void *hip_stream);

/* Options of inla_eval_f_grad_poisson (NULL = defaults; a field <= 0 = its default). */
typedef struct {
  int32_t max_iter;   /* Newton iterations (100) */
  int32_t warm;       /* 1: start from x_mode_dev as given; 0: from x = 0 */
  double tol;         /* stop when max |x_new - x| <= tol (1 + max |x|) (1e-12) */
} inla_newton_opts;

/* status: 0 ok; 1 Q_prior, 2 Q_c(x) not positive definite; 4 Newton's method
 * did not converge in max_iter iterations, or 60 halvings of a step did not
 * keep the objective (f and grad are NaN unless 0).
 * log_lik = log pi(y | x*) with its log y! terms; quad = x*^T Q_prior x*. */
typedef struct {
  double f, grad[4];
  double logdet_p, logdet_c, log_lik, quad;
  int32_t iterations, halvings, status, pad_;
} inla_newton_result;

/*
 * f(theta) and its exact gradient for one model with a Poisson likelihood,
 * y_i ~ Poisson(exp(eta_i)), eta = A x, the model's responses taken as counts
 * (INLA_ERR_ARG if some y_i is not a non-negative integer); theta_4 enters only
 * through its prior.  Sec. "Latent Gaussian Models": a non-Gaussian likelihood
 * makes the Gaussian approximation an inner optimisation whose mode and
 * normalising constant are recomputed in every iteration.  Newton's method on
 * the mode x* from x = 0 (or from x_mode_dev with opts->warm): per iteration
 * Q_c(x) = Q_prior + A^T diag(exp(A x)) A is assembled and factored
 * (inla_assemble, the observation terms, inla_factor_logdet) and
 * Q_c(x) x_new = A^T (y + e (eta - 1)) solved; the step is halved until
 * log pi(x | theta) + log pi(y | x) does not decrease (status 4 if 60 halvings
 * do not get there).  Then
 *   f = -log pi(theta) - 1/2 log|Q_prior| + 1/2 x*^T Q_prior x* - log pi(y | x*)
 *       + 1/2 log|Q_c(x*)|
 *   df/dtheta_k = p_k (theta_k - m_k) - 1/2 tr(Q_prior^{-1} dQ_k) + 1/2 x*^T dQ_k x*
 *       + 1/2 tr(Q_c^{-1} dQ_k) - z^T dQ_k x*,  z = Q_c^{-1} A^T c,
 *       c_i = 1/2 exp(eta*_i) (A Q_c^{-1} A^T)_ii
 * (dQ_k = dQ_prior/dtheta_k, zero for k = 4; the last term is the implicit
 * one of the moving mode) from the selected inverses of both factors.
 * theta: 4 host doubles.  x_mode_dev (n, device, may be NULL): receives x*
 * (and gives the start with warm).  var_dev (n, device, may be NULL):
 * receives diag Q_c(x*)^{-1}.  Allocates three BTA matrices and O(n + m)
 * vectors per call; synchronises hip_stream once per Newton step.
 */
inla_status inla_eval_f_grad_poisson(const inla_model *model, const double *theta,
                                     const inla_newton_opts *opts, inla_newton_result *res,
                                     double *x_mode_dev, double *var_dev, void *hip_stream);

/*
 * Instrumentation for benchmarks.  Between inla_profile_begin() and
 * inla_profile_end() every kernel launch of the library is bracketed by HIP
 * events on the stream it runs on.  inla_profile_end waits for those events
 * and writes, per profiling slot k < nslots, out[3k+0] = launches,
 * out[3k+1] = summed kernel time in milliseconds, out[3k+2] = algorithmic
 * FP64 flops of those launches (the dense-block operation counts of the
 * method, not the flops of padded tiles).  Slots 0..17 are the phases of the
 * tile kernels (Cholesky of the first diagonal tile, the steps that factor and
 * invert the diagonal block tile by tile and, beside them, the next diagonal
 * tile's Cholesky, or both fused in one launch, the b x b off-diagonal solve and its
 * arrow/copy remainder, the b x b Schur update and its remainder, arrow
 * Cholesky, the selected-inversion steps with their remainders, and the
 * selected inversion's V_t, U_t and inv(L_tt)^T inv(L_tt) of every step formed
 * in one launch each (used instead of the step-by-step forms when those would
 * have few tiles), in that order); then substitution sweeps, trace
 * reductions, assembly, the rest, and a last slot whose out[0] is the number
 * of evaluations the records cover (a replayed graph re-records its events,
 * so it counts once) and out[1] the number of unreadable records, then four
 * slots per kernel: the 64-tile kernel (Cholesky steps, side phases), the
 * in-tile Cholesky kernel, the product kernel (64- or 128-wide tiles), and
 * all other kernels.
 * inla_profile_slots() returns the slot count.  Profiling drops any captured
 * graph of inla_eval_f / inla_eval_f_grad when it starts and ends.
 */
inla_status inla_profile_begin(void);
inla_status inla_profile_end(double *out, int32_t nslots);
int32_t inla_profile_slots(void);

/* Release the library's cached device workspace (it is re-grown on demand). */
void inla_release_workspace(void);

const char *inla_status_string(inla_status s);
/* Thread-local text of the last synchronous error ("" if none). */
const char *inla_last_error(void);

/*
 * Build id: the first 16 hex digits of the SHA-256 of the library's source
 * files (kernels, engine, internal headers and this header) it was compiled
 * from, or "unknown".  Bindings compare it with the sources beside them so
 * that a library left over from older sources is refused, not run.
 */
const char *inla_build_id(void);

#ifdef __cplusplus
}
#endif
#endif /* INLA_BTA_H */
