/*
 * lowrank.h -- C ABI of the MI355X (gfx950) low-rank approximation library.
 *
 * The library computes an orthonormal U_k (d x k) whose projector
 * Pi = U_k U_k^T approximately minimises ||X - Pi X||_F for a d x n matrix X
 * (problem statement, Section 1 of Gonen & Shalev-Shwartz, "Faster Low-rank
 * Approximation using Adaptive Gap-based Preconditioning").  The method is the
 * q = k branch of the paper's Algorithm "main" (Section 3.2): block power
 * iteration with oversampling (d x p block, k < p) on the shift-and-invert
 * operator (lambda I - XX^T)^{-1} (Section 1, item 2; Algorithm "subspace
 * iteration", Section 2.2.1), every product with that operator computed by a
 * minibatch SVRG solver (Section 2.3, Theorem "svrgSolve"), the shift set by
 * Algorithm "shiftTune" (Appendix B), and a final Rayleigh-Ritz step
 * (Algorithm "second stage", Section 2.2.2).
 *
 * Conventions
 *   - X is d x n with data points as columns (Section 1).  Dense X is stored
 *     column-major: element (r, i) at values[i * ld + r], ld >= d.
 *   - All matrix pointers passed to the library are DEVICE pointers unless a
 *     parameter says "host".  d x p blocks are FP64, column-major, leading
 *     dimension d.
 *   - Every call returns lr_status; LR_OK is 0.  lowrank_last_error() gives a
 *     human-readable message for the last failing call on this thread.
 *   - No C++ type or exception crosses this boundary.
 *
 * Ownership
 *   - The caller owns X, U_out and every other buffer it passes.  X must stay
 *     valid and unchanged between lowrank_plan and the end of lowrank_solve.
 *   - A plan owns its device workspace, allocated in lowrank_plan and released
 *     in lowrank_destroy; lowrank_solve allocates nothing.
 *   - A plan is not thread-safe.  Separate plans on separate streams may run
 *     concurrently.  All work of a plan is enqueued on the stream given to
 *     lowrank_plan; calls return after the results they report are complete.
 */
#ifndef LOWRANK_H
#define LOWRANK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LR_MAX_P 64          /* largest block width p supported */
#define LR_MAX_SHIFT_ROUNDS 64
#define LR_MAX_SLOTS 16       /* largest number of worker slots of a server */

typedef enum {
  LR_OK = 0,
  LR_EINVAL = 1,    /* bad argument: sizes (need 1 <= k < p < d, p <= n, p <= LR_MAX_P),
                       null pointer, unsupported dtype/layout, or NaN/Inf in X */
  LR_ENOMEM = 2,    /* device allocation failed */
  LR_ENOGAP = 3,    /* estimated gap budget theta_k - theta_p is numerically zero
                       (the paper assumes sigma_k > sigma_{p+1}, Theorem "mainResult") */
  LR_ENOCONV = 4,   /* an inner solve hit max_epochs, or the outer loop hit max_outer
                       (U_out is still written in the latter case) */
  LR_ESHIFT = 5,    /* the inner solver diverged or the shift estimate was not
                       positive: lambda not above lambda_1; or shift tuning did not
                       reach the interval of eq. (shiftClose) within max_shift_rounds */
  LR_ENOTSPD = 6,   /* Cholesky-QR met a Gram matrix that is not positive definite
                       (block lost rank: a Cholesky pivot at or below 1e-14 of
                       its diagonal entry, e.g. when rank(X) < p) */
  LR_EDEVICE = 7,   /* a HIP runtime call or kernel launch failed */
  LR_EBUSY = 8
} lr_status;

typedef enum { LR_F64 = 0, LR_F32 = 1, LR_BF16 = 2 } lr_dtype;
typedef enum { LR_DENSE_COLMAJOR = 0, LR_CSC = 1 } lr_layout;

/* The input matrix, all pointers on the device; values of `dtype` (BF16 as raw
 * uint16 bit patterns).
 *   LR_DENSE_COLMAJOR: values holds d x n elements, (r, i) at values[i*ld + r];
 *     nnz, col_ptr and row_idx are ignored.
 *   LR_CSC (compressed columns, i.e. CSR of X^T; the paper allows sparse X with
 *     per-pass cost nnz(X), Section 1 footnote and Theorem "svrgSolve"): column
 *     i's entries are [col_ptr[i], col_ptr[i+1]) of row_idx / values; col_ptr
 *     has n + 1 entries rising from 0 to nnz (< 2^31); row ids lie in [0, d) and
 *     increase within each column.  lowrank_plan checks this structure on the
 *     device (LR_EINVAL otherwise) and builds a row-ordered copy of X that the
 *     plan owns; ld is ignored.  The request server takes dense X only. */
typedef struct lr_matrix {
  int64_t d, n, ld, nnz;
  int32_t dtype;          /* lr_dtype */
  int32_t layout;         /* lr_layout */
  const void* values;
  const int32_t* col_ptr;
  const int32_t* row_idx;
} lr_matrix;

/* The decisions a solve took (or, for replay, is told to take).
 *   lambda       shift used by every shift-and-invert solve
 *   mu_hat       estimate of lambda - lambda_1 used to size the inner solver
 *   delta_hat    gap budget estimate (theta_k - theta_p) / 1.5 (Section 3)
 *   eta, m, b    inner solver step size, steps per epoch, minibatch size
 *   tau          relative residual at which an inner solve stops
 *   eps_stop     outer stopping threshold eps / (k mu_F)
 *   first_solve  solve index of the first shift-and-invert solve (= number of
 *                shift-tuning rounds); solve indices key the sampling streams
 *   outer        number of outer iterations L
 *   epochs       host array, epochs of each of the `outer` solves.  For
 *                lowrank_get_schedule the caller provides it with capacity
 *                n_epochs (entries beyond capacity are dropped); for replay it
 *                must hold `outer` entries. */
typedef struct lr_schedule {
  double lambda, mu_hat, delta_hat, eta, tau, eps_stop;
  int64_t m, b;
  int32_t first_solve, outer;
  int32_t n_epochs;
  int32_t* epochs;
} lr_schedule;

/* Options.  Fill with lowrank_options_default, then override.
 *   seed            64-bit key of every Philox stream (initial blocks, samples)
 *   shift_mode      0: lambda0 = theta_1 + ||r_1|| + Delta/10 ; 1: 1.5 theta_1
 *                   (the literal start of Algorithm "shiftTune")
 *   est_iters       plain subspace-iteration steps of the estimate phase (4)
 *   max_outer, max_epochs, max_shift_rounds: iteration caps (2000, 60, 30)
 *   polish          plain FP64 power steps before the final Rayleigh-Ritz (0)
 *   batch           minibatch size b; 0 = automatic
 *   eta_scale       multiplies the automatic step size (1.0)
 *   tau_shift       inner-solve tolerance during shift tuning (1e-2)
 *   replay          NULL, or a schedule to follow instead of estimating the
 *                   shift and deciding when to stop (lambda, mu_hat, eta, m, b,
 *                   first_solve, outer and epochs are used)
 *   timing          1: record HIP events around passes and inner-step loops
 *                   and report their durations in lr_report
 *   precision       LR_PREC_F64 (default): all arithmetic FP64.
 *                   LR_PREC_BF16_STEPS (dense BF16 X only, else LR_EINVAL): the
 *                   inner minibatch steps run on BF16 matrix cores, their FP64
 *                   operands carried as hi + lo BF16 parts with FP32
 *                   accumulation; the full-gradient passes that start every
 *                   epoch, Cholesky-QR, Rayleigh-Ritz and the shift/gap
 *                   estimates stay FP64, so each inner solve is refined against
 *                   exactly computed residuals.  Results agree with the FP64
 *                   form to the accuracy of the solve, not bit for bit.
 *                   LR_PREC_F32_STEPS (dense FP32 or BF16 X only, else
 *                   LR_EINVAL): the inner minibatch steps run on FP32 matrix
 *                   cores (FP32 products, FP32 accumulation within a wave, FP64
 *                   between waves) on FP32 copies of the step difference and of
 *                   the sampled products; the difference itself is kept and
 *                   updated in FP64, and everything outside the steps stays FP64
 *                   as above.  Same agreement as the BF16 form.
 *                   LR_PREC_MC_PASS (dense FP32 or BF16 X with ld % 8 == 0 and
 *                   a 16-byte aligned base, else LR_EINVAL): the full-gradient
 *                   passes of the shift-and-invert solves run on BF16 matrix
 *                   cores.  W and T = X^T W are carried as three BF16 parts
 *                   (24 significant bits), FP32 X as three parts (exact), BF16 X
 *                   as itself; products of parts with index sum below three are
 *                   accumulated in FP32 and added into FP64 every 256 terms.
 *                   The estimate phase, shift tuning, Cholesky-QR and the final
 *                   Rayleigh-Ritz stay FP64; inner steps FP64.
 *                   LR_PREC_MC: matrix-core passes as LR_PREC_MC_PASS and
 *                   matrix-core inner steps (the BF16 form for BF16 X, the FP32
 *                   form for FP32 X).  Results of both agree with the FP64 form
 *                   to the accuracy the passes carry, not bit for bit.
 *   adaptive        0 (default): the q = k branch of Algorithm "main" (one
 *                   shift-and-invert iteration with oversampling).  1: the
 *                   adaptive partitioning of Algorithm "main" (Section 3.2):
 *                   intervals s..q found one after another on the deflated
 *                   matrix, by plain subspace iteration where Algorithm
 *                   "largeDetect" finds a multiplicative gap, else by
 *                   shift-and-invert iteration split by Algorithm
 *                   "deltaDetect"; lr_report lists the intervals.  Dense X,
 *                   LR_PREC_F64 and no replay only (LR_EINVAL otherwise).
 *   norm            the norm xi of the guarantee ||X - Pi X||_xi <= (1 + eps)
 *                   ||X - X_k||_xi (Corollary "mainResult"): 0 Frobenius
 *                   (default), 1 spectral.  eps is rescaled by mu, a rough
 *                   bound on ||X||_xi / ||X - X_k||_xi from the estimate
 *                   phase (lr_report.mu_F holds the mu used).
 *   accel           1: accelerated inner solver (the accelerated variant the
 *                   paper cites with Theorem "svrgSolve"): an outer
 *                   proximal-point loop, each step one SVRG epoch on
 *                   ((lambda + kappa) I - XX^T) W = S + kappa Y from the last
 *                   iterate, Y extrapolated with momentum beta; kappa and beta
 *                   are reported in lr_report.  An outer step counts as
 *                   an epoch; a solve may take max_epochs ceil(1 / sqrt(q))
 *                   of them, q = mu / (mu + kappa).  0 (default): plain SVRG
 *                   epochs.  Not with a replay schedule.
 *   fill_workspace  1: when the plan is made, fill its whole device workspace
 *                   with the byte 0xFF (a NaN in every floating-point type the
 *                   library uses) by a kernel, so that any read of workspace
 *                   memory the solve has not written first changes the result.
 *                   For testing; 0 (default) leaves the workspace as found.
 *   shift_start     > 0: Algorithm "shiftTune" starts from lambda = shift_start
 *                   (with the strong-convexity estimate max(lambda - theta_1 -
 *                   ||r_1||, Delta/30)) instead of the start shift_mode names;
 *                   0 (default): shift_mode decides. */
typedef enum {
  LR_PREC_F64 = 0,
  LR_PREC_BF16_STEPS = 1,
  LR_PREC_F32_STEPS = 2,
  LR_PREC_MC_PASS = 3,
  LR_PREC_MC = 4
} lr_precision;

typedef struct lr_options {
  uint64_t seed;
  int32_t shift_mode;
  int32_t est_iters, max_outer, max_epochs, max_shift_rounds, polish;
  int64_t batch;
  double eta_scale, tau_shift;
  const lr_schedule* replay;
  int32_t timing;
  int32_t precision;      /* lr_precision */
  int32_t adaptive;
  int32_t norm;
  int32_t accel;
  int32_t fill_workspace;
  double shift_start;
} lr_options;

/* What a solve did.  Host struct filled by lowrank_solve. */
typedef struct lr_report {
  double theta_est[LR_MAX_P];     /* estimate-phase Ritz values of XX^T, descending */
  double res_est[LR_MAX_P];       /* their residual norms ||A s_i - theta_i s_i|| */
  double fro2;                    /* ||X||_F^2 */
  double mu_F;                    /* the eps rescaling mu: ||X||_F / sqrt(||X||_F^2 -
                                     sum_{i<=k} theta_i), or sqrt(theta_1 / theta_{k+1})
                                     for the spectral norm */
  int32_t shift_rounds;
  double shift_lambda[LR_MAX_SHIFT_ROUNDS];   /* lambda tried in each round */
  double shift_gap[LR_MAX_SHIFT_ROUNDS];      /* its estimate 1/nu_1 of lambda - lambda_1 */
  int32_t outer;
  int64_t total_epochs, passes, steps;
  double last_change;             /* last outer-iteration subspace change */
  double ms_pass_total;           /* timing = 1: summed duration of all passes */
  double ms_steps_total;          /* timing = 1: summed duration of all inner-step loops */
  int64_t timed_passes, timed_steps;
  double ms_sample_dot_probe;     /* timing = 1: summed execution time of one sampled-dot
                                     kernel per epoch (step m/2), from start/stop events
                                     attached to that launch */
  double ms_update_probe;         /* timing = 1: same for one update kernel per epoch */
  int64_t probes;                 /* number of epochs probed */
  /* adaptive = 1: the intervals s..q (1-based) in the order they were found,
   * branch 0 = plain subspace iteration, 1 = shift-and-invert; cols = block
   * width; iters = plain iterations or outer shift-and-invert iterations */
  int32_t n_intervals;
  int32_t interval_s[LR_MAX_P], interval_q[LR_MAX_P], interval_branch[LR_MAX_P];
  int32_t interval_cols[LR_MAX_P], interval_iters[LR_MAX_P];
  double accel_kappa, accel_beta; /* accel = 1: kappa and beta of the last solve's schedule */
  int64_t mc_passes;              /* passes run on matrix cores (LR_PREC_MC_PASS, LR_PREC_MC) */
} lr_report;

typedef struct lr_plan_s* lr_plan;

const char* lowrank_status_string(lr_status s);
const char* lowrank_last_error(void);
void lowrank_options_default(lr_options* opt);

/* Validate sizes and allocate the plan's workspace on the current device.
 * hip_stream: a hipStream_t (NULL = default stream).  Fails with LR_EINVAL on
 * bad sizes or pointers, LR_ENOMEM if the workspace cannot be allocated. */
lr_status lowrank_plan(lr_plan* out, const lr_matrix* X, int k, int p, double eps,
                       const lr_options* opt, void* hip_stream);

/* Run the whole method on the plan's X.
 *   U_out      device, d x k FP64 column-major: orthonormal U_k, each column's
 *              largest-magnitude entry positive (may be NULL)
 *   theta_out  host, k FP64: Ritz values sigma_hat_i^2, descending (may be NULL)
 *   rep        host report (may be NULL) */
lr_status lowrank_solve(lr_plan plan, double* U_out, double* theta_out, lr_report* rep);

/* Copy the schedule of the last solve.  out->epochs / out->n_epochs give a
 * caller-owned host buffer and its capacity (may be NULL / 0). */
lr_status lowrank_get_schedule(lr_plan plan, lr_schedule* out);

void lowrank_destroy(lr_plan plan);

/* Device workspace in bytes that lowrank_plan (or a server) keeps for this
 * problem: the n-length sampling table, the n x pad16(p) block X^T W, the d x p
 * iterates and the minibatch staging; for LR_CSC also the row-ordered copy of
 * X and its chunk tables, plus the buffers of the inner step's sorted scatter,
 * which depend on the largest column and are bounded from above here (plan
 * creation needs about 12 nnz + sort-scratch bytes more while it builds the
 * row-ordered copy).  Same checks as lowrank_plan, done on the host only. */
lr_status lowrank_plan_bytes(const lr_matrix* X, int k, int p, const lr_options* opt,
                             size_t* bytes);

/* Device workspace that lowrank_solve_noalloc can hold: 64 MiB. */
#define LR_NOALLOC_MAX_BYTES (64u * 1024u * 1024u)

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, tight serving loops, harnesses that forbid allocation): one whole
 * solve, as lowrank_plan + lowrank_solve + lowrank_destroy, with no device
 * allocation.  The workspace is a fixed array of LR_NOALLOC_MAX_BYTES in the
 * library's device image (each device holds its own copy for the life of the
 * process); host-side staging is per calling thread.
 *   X, k, p, eps, opt, hip_stream  as for lowrank_plan; dense X only
 *   U_out, theta_out, rep          as for lowrank_solve
 * Returns the lowrank_solve status, or LR_ENOMEM (nothing run) when
 * lowrank_plan_bytes exceeds LR_NOALLOC_MAX_BYTES, LR_EINVAL for compressed-
 * column X (its plan builds a row-ordered copy) or opt->timing != 0 (timing
 * needs events).  The solve does not depend on what the array holds when it
 * starts.  Every call on one device uses the same array: calls that overlap on
 * one device (other threads, other streams) race and give wrong results;
 * serialise them. */
lr_status lowrank_solve_noalloc(const lr_matrix* X, int k, int p, double eps,
                                const lr_options* opt, void* hip_stream, double* U_out,
                                double* theta_out, lr_report* rep);

/* ---- Single steps of the path, on a plan's X and stream (for testing and
 * measurement).  All matrices FP64 device, column-major, leading dim d. ---- */

/* Y = X (X^T W) for a d x ncols block W (ncols <= p); A = XX^T is never
 * formed (Section 2.2.1, footnote).  Computed as the plan's solves compute
 * their passes: on matrix cores for LR_PREC_MC_PASS and LR_PREC_MC, else FP64.
 * lowrank_op_svrg_solve and lowrank_op_acc_svrg_solve likewise. */
lr_status lowrank_op_apply_A(lr_plan plan, const double* W, double* Y, int ncols);

/* Plan step a0: column squared norms w (n), quantised cumulative table
 * cdf (n+1, uint64), ||X||_F^2 (host). */
lr_status lowrank_op_prepare(lr_plan plan, double* w_out, uint64_t* cdf_out, double* fro2_out);

/* The b column indices and weights 1/(b pi_i) of inner step `step` of epoch
 * `epoch` of solve `solve` (requires lowrank_op_prepare or a solve first). */
lr_status lowrank_op_sample(lr_plan plan, int32_t solve, int32_t epoch, int32_t step, int64_t b,
                            int32_t* idx_out, double* scale_out);

/* d x p' Gaussian block of stream `tag` (1 estimate, 2 shift-and-invert) and
 * solve index `solve`, as used for the random start of the subspace
 * iteration (Algorithm "subspace iteration", Section 2.2.1). */
lr_status lowrank_op_gaussian(lr_plan plan, int32_t tag, int32_t solve, int ncols, double* S_out);

/* S = W R^{-1} with R the Cholesky factor of W^T W, applied twice. */
lr_status lowrank_op_cholqr2(lr_plan plan, const double* W, double* S_out, int ncols);

/* Symmetric eigendecomposition of an m x m matrix (m <= LR_MAX_P), descending,
 * eigenvector columns with their largest-magnitude entry positive. */
lr_status lowrank_op_eigh(lr_plan plan, const double* H, int m, double* vals_out,
                          double* vecs_out);

/* Algorithm "musco" (Section 2.4) on A = XX^T with a block of ncols columns
 * (2 <= ncols <= p): `iters` plain subspace-iteration steps from the Gaussian
 * block of stream (tag 1, stream_index), each followed by Cholesky-QR2, then
 * Rayleigh-Ritz (Algorithm "second stage" with C = A).
 *   theta_out  host, ncols: Ritz values, descending
 *   res_out    host, ncols: residual norms ||A v_i - theta_i v_i|| (may be NULL)
 *   V_out      device, d x ncols: the Ritz vectors v_i (may be NULL) */
lr_status lowrank_op_estimate(lr_plan plan, int ncols, int iters, int32_t stream_index,
                              double* theta_out, double* res_out, double* V_out);

/* Plain subspace iteration (Algorithm "subspace iteration", Section 2.2.1,
 * with C = A = XX^T, no shift): S_in (device, d x ncols, full column rank) is
 * orthonormalised by Cholesky-QR2, then at most max_iters steps
 * S <- CholQR2(A S), stopping early once the block's span moves by at most tol
 * in one step (tol = 0: all steps).  S_out: device, d x ncols; iters_out,
 * change_out: host (may be NULL), steps taken and the last step's
 * sin(largest principal angle). */
lr_status lowrank_op_power(lr_plan plan, const double* S_in, int ncols, int max_iters,
                           double tol, double* S_out, int32_t* iters_out, double* change_out);

/* One inner solve of (lambda I - XX^T) W = S with a fixed number of epochs
 * (requires lowrank_op_prepare or a solve first).  res_out: host, epochs+1
 * residual norms ||G~||_F (may be NULL). */
lr_status lowrank_op_svrg_solve(lr_plan plan, const double* S, double lambda, double eta,
                                int64_t m, int64_t b, int32_t solve, int32_t epochs,
                                double* W_out, double* res_out);

/* One accelerated inner solve of (lambda I - XX^T) W = S (the proximal-point
 * loop of lr_options.accel; the plan must have been made with accel = 1) with a
 * fixed number of outer steps, each one epoch of m minibatch steps of size b
 * and step size eta at the shift lambda + kappa, followed by extrapolation
 * with momentum beta.  kappa = 0 gives the plain solver.  res_out: host,
 * epochs+1 residual norms ||S - (lambda I - XX^T) W||_F of the original system
 * (may be NULL); W_out: device, d x p. */
lr_status lowrank_op_acc_svrg_solve(lr_plan plan, const double* S, double lambda, double kappa,
                                    double beta, double eta, int64_t m, int64_t b, int32_t solve,
                                    int32_t epochs, double* W_out, double* res_out);


/* ---- Request server: continuous batching of independent problems ----
 *
 * Many low-rank problems of mixed d, n, k, p and storage type are solved
 * concurrently on the current device.  Requests queue in submission order; the
 * request at the head of the queue is admitted as soon as a worker slot is idle
 * and its whole workspace (lowrank_plan_bytes) fits in the unused part of the
 * server's HBM budget.  Each slot owns a host thread and a HIP stream, so
 * admitted requests overlap on the device; each one runs the same kernels in
 * the same order as lowrank_solve on a plan of its own, so its results are
 * bitwise the same alone and in any mix.  Requests use the method of
 * lowrank_solve (Section 3.2, Algorithm "main", q = k branch); the server adds
 * no approximation.
 *
 * Ownership: the caller owns X, U_out and theta_out of every request and keeps
 * them valid and X unchanged until lowrank_poll or lowrank_wait reports the
 * request finished.  X must be complete on the device when lowrank_submit is
 * called (the server's streams do not wait on the caller's).  The server owns
 * the HBM budget block (allocated once in lowrank_server_create), the slot
 * streams and threads.  All functions are thread-safe. */
typedef struct lr_server_s* lr_server;

typedef struct lr_ticket_info {
  double t_submit, t_admit, t_done;  /* seconds since the server was created */
  int32_t slot;                      /* worker slot that ran the request */
  int32_t reserved;
  uint64_t workspace_bytes;          /* HBM the request held while running */
} lr_ticket_info;

typedef struct lr_server_stats {
  int64_t submitted, completed, queued, running;
  uint64_t budget_bytes, bytes_in_use, peak_bytes;
  int32_t slots, peak_running;
  double elapsed;                    /* seconds since the server was created */
} lr_server_stats;

/* Allocate an HBM budget of hbm_budget_bytes on the current device and start
 * `slots` worker slots (1..LR_MAX_SLOTS).  LR_ENOMEM if the budget cannot be
 * allocated, LR_EDEVICE if streams, events or threads cannot be created. */
lr_status lowrank_server_create(lr_server* out, size_t hbm_budget_bytes, int slots);

/* Queue one problem.  X, k, p, eps, opt as for lowrank_plan (opt may be NULL;
 * a replay schedule in opt is copied).  U_out: device, d x k FP64 (may be
 * NULL); theta_out: host, k FP64 (may be NULL).  *ticket identifies the
 * request.  LR_EINVAL on bad arguments, LR_ENOMEM if the request's workspace
 * alone exceeds the budget. */
lr_status lowrank_submit(lr_server srv, const lr_matrix* X, int k, int p, double eps,
                         const lr_options* opt, double* U_out, double* theta_out,
                         uint64_t* ticket);

/* LR_EBUSY while the request is queued or running.  Once it has finished:
 * its lowrank_solve status (LR_OK or the error, with lowrank_last_error set on
 * this thread), rep and info filled (each may be NULL), and the ticket is
 * forgotten (a later poll returns LR_EINVAL). */
lr_status lowrank_poll(lr_server srv, uint64_t ticket, lr_report* rep, lr_ticket_info* info);

/* Block until the request has finished, then as lowrank_poll. */
lr_status lowrank_wait(lr_server srv, uint64_t ticket, lr_report* rep, lr_ticket_info* info);

lr_status lowrank_server_stats(lr_server srv, lr_server_stats* out);

/* Finish every queued and running request, then release the server. */
void lowrank_server_destroy(lr_server srv);

#ifdef __cplusplus
}
#endif
#endif /* LOWRANK_H */
