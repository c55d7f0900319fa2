/*
 * qpk: a primal-dual interior point method for convex QPs whose Newton
 * systems are solved by Jacobi-preconditioned conjugate gradients on the
 * doubly augmented KKT matrix, for one AMD MI355X (gfx950).
 *
 * Method: Liu, Fredriksson, Markidis, "Krylov Solvers for Interior Point
 * Methods with Applications in Radiation Therapy and Support Vector Machines"
 * (arXiv 2308.00637).  Section and equation numbers below refer to it:
 *   eq. (1)  the QP; eq. (3) perturbed optimality conditions (residuals);
 *   eq. (7)  the full Newton system; eq. (8) the 2x2 augmented system;
 *   eq. (9)  the doubly augmented SPD system solved by PCG (Section 3.1);
 *   eq. (10) the ratio test; Algorithm 1 the IPM loop (Section 3.2).
 *
 * Problem solved (eq. (1), variable bounds kept apart as in Section 3.1):
 *     min 1/2 x^T H x + c^T x   s.t.  lA <= A x <= uA,  C x = b,  lx <= x <= ux
 * Infinite bound entries (+-INFINITY) mean "no bound on that side"; only finite
 * sides carry a slack/multiplier pair.
 *
 * Conventions
 *  - Every function returns a qp_status; 0 is success, negative values are
 *    errors.  No C++ exception crosses this boundary.  After an error,
 *    qp_last_error(h) returns a message (valid until the next call on h).
 *  - qp_desc pointers are HOST pointers.  qp_create copies and converts all of
 *    them into library-owned device buffers; the caller may free them on
 *    return.
 *  - Every other double* argument is a DEVICE pointer (e.g. a torch tensor's
 *    data_ptr()) unless documented as host.  Device arguments must not alias
 *    each other.  All device work is ordered on the stream given to qp_create
 *    (or qp_set_stream); functions that return host values synchronise it.
 *  - Layouts of the iterate (device, float64):
 *      x   : n
 *      lam : me + 2m + 2n = [lam_e (me) | lam_lA (m) | lam_uA (m) | lam_lx (n) | lam_ux (n)]
 *      s   : 2m + 2n      = [s_lA (m) | s_uA (m) | s_lx (n) | s_ux (n)]
 *    Entries of absent (infinite) sides are ignored on input and written as 0.
 *  - Layout of a doubly augmented vector (eq. (9)), N = n + me + 2m:
 *      [x-part (n) | lam_e-part (me) | lam_lA-part (m) | lam_uA-part (m)]
 *    Rows of absent sides are identity rows of K (their entries stay 0).
 *  - Layout of the residual stack (eq. (3)/(7) right-hand side), 5n + me + 4m:
 *      [r_H (n) | r_e (me) | r_lA (m) | r_uA (m) | r_lx (n) | r_ux (n) |
 *       r_c1 (m) | r_c2 (m) | r_c3 (n) | r_c4 (n)]
 *  - A handle is not thread-safe; calls on one handle must be serialised.
 */
#ifndef QPK_H
#define QPK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qp_handle_s* qp_handle;

typedef enum {
  QP_OK = 0,
  QP_ERR_ARG = -1,         /* invalid argument or problem data */
  QP_ERR_ALLOC = -2,       /* device or host allocation failed */
  QP_ERR_HIP = -3,         /* a HIP runtime call failed */
  QP_ERR_NOT_SPD = -4,     /* PCG met p^T K p <= 0: H not convex or state broken */
  QP_ERR_NUMERIC = -5,     /* NaN or Inf met in a reduction */
  QP_ERR_STATE = -6,       /* call made in the wrong state (e.g. backward before solve) */
  QP_ERR_UNSUPPORTED = -7  /* valid request this build does not implement */
} qp_status;

typedef enum { QP_H_DENSE = 0, QP_H_LOWRANK = 1, QP_H_PTWP = 2 } qp_h_kind;
typedef enum { QP_A_NONE = 0, QP_A_DENSE = 1, QP_A_CSR = 2 } qp_a_kind;
/* Precision of the PCG matvec only.  Residuals, right-hand sides, the Jacobi
 * diagonal, every inner product, the PCG vectors, the ratio test and the
 * iterate stay float64 in all modes; reduced-precision solves replace the
 * residual by its float64 value periodically and accept a solve only on the
 * float64 residual. */
typedef enum {
  QP_PREC_FP64 = 0,        /* every operation in float64 */
  QP_PREC_FP32 = 1,        /* matvec values stored and accumulated in float32 */
  QP_PREC_BF16 = 2,        /* matvec values stored in bfloat16, float32 accumulation */
  QP_PREC_FP32_ACC64 = 3,  /* values stored in float32, float64 accumulation */
  QP_PREC_BF16_ACC64 = 4   /* values stored in bfloat16, float64 accumulation */
} qp_precision;

/* Problem description (all pointers HOST, read only during qp_create). */
typedef struct {
  int64_t n;                 /* variables, >= 1 */
  int64_t m;                 /* general rows of A, >= 0 */
  int64_t me;                /* equality rows of C, 0 <= me <= 64 */
  int32_t h_kind;            /* qp_h_kind */
  /* QP_H_DENSE: H symmetric, n*n row-major. */
  const double* H;
  /* QP_H_LOWRANK: H = diag(h0) + U diag(wd) U^T, the quasi-Newton form
   * H0 + U W U^T of Section 2.2 (and the linear-kernel SVM Gram matrix).
   * U is n*k row-major; 1 <= k <= 1024. */
  int64_t k;
  const double* h0;          /* n */
  const double* U;           /* n*k */
  const double* wd;          /* k */
  /* QP_H_PTWP: H = P^T diag(w) P with P sparse (p_rows x n, CSR), and the
   * objective's linear term becomes c - P^T diag(w) d, i.e. the objective is
   * 1/2 sum_v w_v (P_v x - d_v)^2 + c^T x up to a constant. */
  int64_t p_rows;
  const int64_t* p_rowptr;   /* p_rows + 1 */
  const int32_t* p_col;      /* nnz, each in [0, n) */
  const double* p_val;       /* nnz */
  const double* p_w;         /* p_rows, w_v > 0 */
  const double* p_d;         /* p_rows, or NULL for zeros */
  const double* c;           /* n */
  int32_t a_kind;            /* qp_a_kind; QP_A_NONE requires m == 0 */
  const double* A;           /* QP_A_DENSE: m*n row-major */
  const int64_t* a_rowptr;   /* QP_A_CSR: m + 1 */
  const int32_t* a_col;
  const double* a_val;
  const double* lA;          /* m, entries may be -INFINITY */
  const double* uA;          /* m, entries may be +INFINITY; lA <= uA */
  const double* C;           /* me*n row-major */
  const double* b;           /* me */
  const double* lx;          /* n or NULL (all -INFINITY) */
  const double* ux;          /* n or NULL (all +INFINITY); lx < ux where both finite */
  int32_t precision;         /* qp_precision */
} qp_desc;

/* PCG settings (Section 5.1: tolerance 1e-7 on the unpreconditioned residual,
 * relative to ||rhs||_2; at most 5000 iterations; start from 0). */
typedef struct {
  double tol;                /* default 1e-7 */
  int32_t maxit;             /* default 5000 */
  int32_t check_every;       /* iterations between host polls of the stop flag; default 8 */
  int32_t rr_period;         /* reduced precision only: replace r by the float64 residual
                              * rhs - K x every rr_period iterations (search direction kept);
                              * default 0 = only when the stop test fires */
  int32_t spectrum;          /* 1: estimate the extreme eigenvalues of the preconditioned
                              * matrix (diag(K)^-1 K, or K itself with no_precond = 1) from
                              * the CG coefficients (the Lanczos tridiagonal matrix that CG
                              * builds implicitly), reported in pcg_info; the condition
                              * number diagnostic of Section 5.3.  Float64 solves without
                              * restarts only.  Default 0 */
  int32_t no_precond;        /* 1: plain CG (z = r) instead of the Jacobi preconditioner
                              * z = r / diag(K) of Section 3.1, e.g. to estimate the
                              * spectrum of K itself.  Default 0 */
} pcg_options;

typedef struct {
  int32_t iterations;
  int32_t converged;         /* 1 if ||r|| <= tol ||rhs|| */
  int32_t status;            /* qp_status of the solve */
  double rel_residual;       /* final ||rhs - K sol|| / ||rhs|| (float64 operator) */
  double rhs_norm;
  int32_t escalated;         /* reduced precision only: 1 if the solve failed with the
                              * reduced-precision operator (iteration cap, NaN, or lost
                              * positive definiteness) and was redone in float64;
                              * iterations then counts both attempts */
  double lambda_min;         /* spectrum = 1: smallest and largest Ritz value of the */
  double lambda_max;         /* CG tridiagonal matrix (inside the spectrum of diag(K)^-1 K,
                              * or of K with no_precond, converging to its ends); 0 when
                              * not estimated */
} pcg_info;

/* Algorithm 1 settings.  gamma of eq. (10); mu is divided by mu_div when the
 * stacked residual norm falls below mu, and the solve returns when that
 * happens with mu < mu_tol (Section 3.2). */
typedef struct {
  double gamma;              /* 0.99 */
  double mu0;                /* 1.0 */
  double mu_tol;             /* 1e-6 */
  double mu_div;             /* 10 */
  int32_t max_iter;          /* 200 */
  int32_t warm_start;        /* 0: default start point; 1: current handle state and mu */
  pcg_options pcg;
  /* optional per-iteration log (HOST arrays of log_capacity entries each, or NULL) */
  int32_t log_capacity;
  double* log_mu;
  double* log_rnorm;
  double* log_primal;
  double* log_dual;
  double* log_compl;
  double* log_alpha_x;
  double* log_alpha_lam;
  int32_t* log_cg_iters;
  double* log_cg_relres;
  double* log_kappa;         /* lambda_max / lambda_min of each Newton system (needs
                              * pcg.spectrum = 1), or NULL */
  double* log_kappa_plain;   /* the same for K itself (no preconditioner), or NULL: each
                              * Newton system is then also solved by plain CG (spectrum on,
                              * the pcg tolerance and cap), for this log only (the iterate
                              * does not use it; its time counts in time_ms, not in
                              * pcg_time_ms or total_cg_iters).  Float64 handles */
  /* The barrier parameter's rule.  QP_MU_PAPER (0, the default): Algorithm 1,
   * mu divided by mu_div whenever the stacked residual is below mu, stop once
   * mu < mu_tol.  QP_MU_MEHROTRA (1): the predictor-corrector rule that
   * Sections 5.2 and 7 leave to future work (Mehrotra 1992), on the same
   * Newton system eq. (9): mu = lam^T s / N_c (N_c finite sides), also the
   * equality rows' penalty; a predictor solve for complementarity target 0,
   * its largest steps to the boundary (gamma = 1), sigma = min(1, (mu_aff /
   * mu)^3) with mu_aff the complementarity average after those steps; a
   * corrector solve for target max(sigma mu, mu_tol / (2 mu_div)) with the
   * predictor's dlam * ds added to each complementarity residual; the step
   * with gamma.  Two PCG solves per iteration (total_cg_iters counts both).
   * It stops when mu and the primal and dual residuals (target 0) are below
   * mu_tol / mu_div; mu0 and warm_start's mu are not used.  With no
   * inequality constraints the paper's rule runs.  log_rnorm, log_compl and
   * ipm_info's residuals are those of the new point for its own mu (target
   * and penalty), as under the paper's rule. */
  int32_t mu_rule;
  double* log_sigma;         /* QP_MU_MEHROTRA: sigma of each iteration, or NULL */
} ipm_options;

enum { QP_MU_PAPER = 0, QP_MU_MEHROTRA = 1 };

typedef enum { QP_IPM_CONVERGED = 0, QP_IPM_MAX_ITER = 1 } qp_ipm_result;

typedef struct {
  int32_t result;            /* qp_ipm_result */
  int32_t iterations;        /* IPM iterations taken */
  int64_t total_cg_iters;
  int32_t cg_maxiter_hits;   /* Newton steps whose PCG stopped at maxit */
  int32_t cg_escalations;    /* Newton steps redone with the float64 operator */
  double mu_final;
  double rnorm;              /* stacked residual norm at the returned point */
  double primal, dual, compl_; /* infeasibilities of Section 5.2 */
  double objective;          /* 1/2 x^T H x + (linear term)^T x */
  double time_ms;            /* wall time of the solve (stream-synchronised) */
  double pcg_time_ms;        /* part of it inside PCG */
} ipm_info;

void qp_default_pcg_options(pcg_options* o);
void qp_default_ipm_options(ipm_options* o);
const char* qp_status_string(int32_t status);
const char* qp_last_error(qp_handle h);

/* Create a handle: validates d (QP_ERR_ARG on n <= 0, lA > uA, lx >= ux,
 * non-finite data, bad CSR), copies it into device layouts, and precomputes
 * the constant parts (diag(H), the linear term).  stream is a hipStream_t
 * (NULL = default stream).  On error *out is NULL.
 *
 * Launch-shape overrides, read here from the environment (for tuning and
 * tests; the defaults are the measured best): QPK_CHUNK_COLS_R / _X (columns
 * per LDS chunk of the row / column side, 1024..20224), QPK_LPR_R / _X (lanes
 * per row, 4..64), QPK_KV_R / _X (0: chunk staged through registers, 1:
 * straight into LDS), QPK_ALTERNATE (0: every product walks rows first to
 * last), QPK_XCD_MAP (0: work item i on block i), QPK_FOLD_A (0: keep A in
 * the blocked passes even when every row of A repeats its own row of P; by
 * default such an A is folded into P's rows).  QPK_KV_*, QPK_ALTERNATE and
 * QPK_XCD_MAP leave K v bitwise unchanged; chunk widths, lanes per row and
 * QPK_FOLD_A change the order in which sums are taken. */
qp_status qp_create(const qp_desc* d, void* stream, qp_handle* out);
void qp_destroy(qp_handle h);
qp_status qp_set_stream(qp_handle h, void* stream);

/* Sizes of the device layouts above. */
qp_status qp_sizes(qp_handle h, int64_t* n_x, int64_t* n_lam, int64_t* n_s,
                   int64_t* n_kkt, int64_t* n_res);

/* Iterate I/O.  qp_set_state copies a caller iterate (QP_ERR_ARG if a present
 * slack or multiplier is <= 0 or not finite).  qp_init_state loads the
 * default starting point: x at the middle of two-sided bounds, one unit inside
 * one-sided ones, 0 if free; bound slacks exact; row slacks max(distance, 1);
 * inequality multipliers 1; lam_e 0. */
qp_status qp_set_state(qp_handle h, const double* x, const double* lam,
                       const double* s, double mu);
qp_status qp_get_state(qp_handle h, double* x, double* lam, double* s,
                       double* mu /* host, may be NULL */);
qp_status qp_init_state(qp_handle h, double mu);

/* Residual stack of eq. (3)/(7) at the current state and mu (step a1).
 * r: device, 5n+me+4m, or NULL.  norms: HOST double[4] =
 * {stacked ||r||_2, primal, dual, complementarity} (Section 5.2), or NULL. */
qp_status qp_residuals(qp_handle h, double* r, double* norms);

/* Right-hand side of eq. (9) and diag(K) (the Jacobi preconditioner of
 * Section 3.1) at the current state (steps a2, a3).  Device, N each; either
 * may be NULL. */
qp_status qp_newton_rhs(qp_handle h, double* rhs, double* jacobi_diag);

/* y = K v for the doubly augmented K of eq. (9) at the current state, applied
 * matrix-free as in Section 3.2 (step a4, float64 operator).  Device, N each. */
qp_status qp_kkt_matvec(qp_handle h, const double* v, double* y);

/* Solve K sol = rhs by Jacobi PCG at the current state (step a5).  rhs, sol:
 * device, N.  o may be NULL for defaults; info (host) may be NULL.  Returns
 * QP_ERR_NOT_SPD if a curvature p^T K p <= 0 is met. */
qp_status kkt_pcg_solve(qp_handle h, const double* rhs, double* sol,
                        const pcg_options* o, pcg_info* info);

/* Full Newton direction at the current state (steps a1-a6): residuals,
 * eq. (9) by PCG, then the eliminated unknowns (slack steps from the primal
 * rows of eq. (7), bound-multiplier steps from its complementarity rows).
 * dx (n), dlam (me+2m+2n), ds (2m+2n): device, iterate layouts. */
qp_status qp_newton_direction(qp_handle h, const pcg_options* o, double* dx,
                              double* dlam, double* ds, pcg_info* info);

/* Ratio test of eq. (10) (step a7) for a direction in iterate layout.
 * alpha_x / alpha_lam: HOST. */
qp_status qp_step_lengths(qp_handle h, const double* dlam, const double* ds,
                          double gamma, double* alpha_x, double* alpha_lam);

/* x += alpha_x dx, s += alpha_x ds, every multiplier += alpha_lam dlam
 * (Algorithm 1, step a8). */
qp_status qp_take_step(qp_handle h, const double* dx, const double* dlam,
                       const double* ds, double alpha_x, double alpha_lam);

/* Algorithm 1 (steps a1-a9).  x, lam, s: device outputs in iterate layouts,
 * each may be NULL (the result stays in the handle, see qp_get_state).
 * o may be NULL for defaults; info (host) must not be NULL. */
qp_status ipm_solve(qp_handle h, const ipm_options* o, double* x, double* lam,
                    double* s, ipm_info* info);

/* Adjoint of the solution (not in the paper): for a loss L(x*) with gradient
 * grad_x (device, n), returns dL/dc (n), dL/dlA (m), dL/duA (m), dL/db (me)
 * and, for QP_H_PTWP, dL/dw (p_rows), each a device pointer or NULL.  It
 * differentiates the perturbed optimality conditions at the returned point
 * and mu, which needs one PCG solve with the same K as the last Newton step:
 * K u = (grad_x, 0); dL/dc = -u_x, dL/dlA = -u_lamlA, dL/duA = u_lamuA,
 * dL/db = -u_lame, dL/dw_v = -(P_v u_x)(P_v x - d_v).  Entries for absent
 * sides are 0.  QP_ERR_STATE unless ipm_solve has completed on this handle. */
qp_status qp_backward(qp_handle h, const double* grad_x, double* grad_c,
                      double* grad_lA, double* grad_uA, double* grad_b,
                      double* grad_w, const pcg_options* o, pcg_info* info);

/* ---- Batches of independent QPs (one persistent launch) ----
 * qp_batch_create copies `count` problem descriptions (HOST pointers, as for
 * qp_create) into one device pool.  Supported per instance: H dense or low
 * rank, A dense (or m = 0), any row and variable bounds, no equality rows
 * (me = 0); precision QP_PREC_FP64 or QP_PREC_FP32 (operator storage, same
 * for all instances; vectors and reductions stay float64).  Other inputs give
 * QP_ERR_UNSUPPORTED; invalid data QP_ERR_ARG (see qp_batch_last_error(NULL)).
 * ipm_solve_batch runs Algorithm 1 for every instance in one kernel launch:
 * `workgroups` (<= 0: 512) workgroups of 1024 threads take instances from a
 * queue, largest first, and each solves its instances start to finish (same
 * steps, readings and defaults as ipm_solve; per-iteration logs are not
 * kept; of o->pcg only tol and maxit are read: always Jacobi, no spectrum;
 * mu_rule must be QP_MU_PAPER, else QP_ERR_UNSUPPORTED).
 * infos: HOST array of `count`, each time_ms is the whole launch.
 * Returns QP_ERR_NOT_SPD / QP_ERR_NUMERIC if an instance stopped on one
 * (the others are still solved).  qp_batch_get_solution copies instance i's
 * iterate (DEVICE pointers, layouts as for a single handle with me = 0). */
typedef struct qp_batch_s* qp_batch;
qp_status qp_batch_create(const qp_desc* descs, int32_t count, void* stream, qp_batch* out);
void qp_batch_destroy(qp_batch b);
qp_status ipm_solve_batch(qp_batch b, const ipm_options* o, int32_t workgroups, ipm_info* infos);
/* Teams of workgroups for large instances.  team_size (HOST, one entry per
 * instance, each a power of two from 1 to 64; NULL: all 1) sets how many
 * workgroups solve each instance together: its rows, columns and vector
 * entries are spread over the team, whose phases meet at device-wide team
 * barriers and whose reductions combine the members' partials in rank order
 * (so results differ from a team of one by rounding only).  With any size
 * above 1, ipm_solve_batch makes one cooperative launch of at most the
 * co-resident workgroups (and at most `workgroups` when positive): each team
 * size gets its own queue of instances, longest first, and a number of teams
 * in proportion to its instances' workgroup time (the autotuner's estimates
 * when qp_batch_autotune set the sizes, else their operator work); a team
 * whose queue is empty then takes instances from
 * the queues of smaller team sizes (which team solves an instance, and so
 * its rounding, can differ between launches).  A team whose members cannot
 * all be resident is reported as QP_ERR_HIP rather than waited for.
 * qp_batch_launch_shape returns the last launch's workgroups and teams (HOST
 * outs, may be NULL). */
qp_status qp_batch_set_teams(qp_batch b, const int32_t* team_size);
/* Sets team sizes from measured times (then as qp_batch_set_teams).  The
 * instances are classed by precision, H kind and the binary order of
 * magnitude of the bytes one PCG iteration reads; each class's largest
 * instance is timed alone with teams of 1, 2, 4, ... up to max_team (<= 0:
 * 64) workgroups (one IPM iteration of at most 24 PCG iterations; the
 * instance's iterate is overwritten, a later solve starts afresh).  The
 * times are appended to the text table at table_path (HOST string, may be
 * NULL: nothing read or kept), one line per measurement: device
 * architecture, float32 storage (0/1), H kind, class, team size,
 * microseconds per PCG iteration; measurements found there are not taken
 * again.  An instance's iteration time is taken as the larger of its
 * class's time (scaled by its work) and its operator bytes over its team's
 * share of 5.5 TB/s among the co-resident workgroups (a workgroup alone
 * streams faster than beside all the others).  Starting from teams of one,
 * the instance with the longest PCG iteration gets twice the team while
 * that lowers the estimated makespan (the larger of the slowest iteration
 * and the total workgroup time over the co-resident workgroups).  HOST
 * outs, may be NULL: team_out (one per
 * instance), probes_out (measurements taken by this call). */
qp_status qp_batch_autotune(qp_batch b, const char* table_path, int32_t max_team, int32_t* team_out,
                            int32_t* probes_out);
qp_status qp_batch_launch_shape(qp_batch b, int32_t* workgroups, int32_t* teams);
/* Per instance of the last completed ipm_solve_batch: when its team started
 * and finished it, in ms from the earliest start (the device's constant-rate
 * wall clock), and the workgroups of the team that solved it (a team whose
 * queue ran out may have taken it from another queue).  HOST arrays of
 * `count`, each may be NULL.  QP_ERR_ARG before any completed solve. */
qp_status qp_batch_instance_times(qp_batch b, double* start_ms, double* end_ms, int32_t* team);
qp_status qp_batch_get_solution(qp_batch b, int32_t i, double* x, double* lam, double* s);
const char* qp_batch_last_error(qp_batch b);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one dense QP
 *     min 1/2 x^T H x + c^T x  s.t.  lA <= A x <= uA,  lx <= x <= ux
 * solved by the batched solver's kernel (the same steps and defaults as
 * ipm_solve_batch on a batch of this one instance, float64 operators), with
 * every workspace in a fixed device array of the library: 16 MiB per GPU,
 * set aside until the process ends, which holds problems whose 29 n + 31 m
 * float64 values of workspace fit in it (n = m = 34,000 does; larger sizes
 * give QP_ERR_ARG before anything is launched).  The
 * call allocates nothing.  Inputs are DEVICE pointers read in place: H (n*n
 * row-major), c (n), A (m*n row-major), lA, uA (m; A, lA, uA may be NULL when
 * m = 0), lx, ux (n, or NULL for no bounds); bounds are checked on the device
 * (QP_ERR_ARG), NaN or Inf in H, A or c gives QP_ERR_NUMERIC.  Outputs x (n),
 * lam, s (2m + 2n, layouts as for a handle with me = 0) are DEVICE pointers,
 * each may be NULL; info (HOST) must not be NULL, and filling it synchronises
 * the stream (hipStream_t, NULL = default).  Of o only the IPM constants and
 * pcg.tol / pcg.maxit are read; warm_start and QP_MU_MEHROTRA are not
 * supported (QP_ERR_UNSUPPORTED).  Every call on
 * one GPU uses that GPU's array: calls that overlap on a GPU (other host
 * threads, other streams) race.  Error messages: qp_batch_last_error(NULL). */
qp_status ipm_solve_dense_noalloc(int64_t n, int64_t m, const double* H, const double* c,
                                  const double* A, const double* lA, const double* uA,
                                  const double* lx, const double* ux, const ipm_options* o,
                                  double* x, double* lam, double* s, ipm_info* info, void* stream);

/* Replace problem data in place (DEVICE pointers, NULL = keep): the linear
 * term c (n), the row bounds lA, uA (m, +-INFINITY allowed, with the same
 * finite/infinite pattern as at creation), the equality right-hand side b
 * (me), and for QP_H_PTWP the voxel weights w (p_rows, positive).  The
 * derived constants (diag(H), c - P^T W d) are recomputed on the device.
 * Invalidates any completed solve (qp_backward then needs a new ipm_solve).
 * For the differentiable wrapper, which changes only these parameters. */
qp_status qp_update_data(qp_handle h, const double* c, const double* lA, const double* uA,
                         const double* b, const double* w);

/* Kernel timing with HIP events on the handle's stream (instrumentation, not
 * part of the method).  qp_profile_begin(h, max_launches, every) pre-creates
 * events for up to max_launches timed dispatches per category; until
 * qp_profile_end one dispatch in `every` of each PCG kernel is launched with
 * its own event pair bound to that dispatch (hipExtLaunchKernelGGL), so a
 * category's time is kernel execution only, comparable to a profiler's kernel
 * trace.  A timed dispatch costs a few microseconds of queue time around it;
 * every > 1 keeps that out of all but a sample.  qp_profile_end synchronises
 * and returns, per category, the number of timed dispatches, their summed
 * duration in ms, and the number of dispatches made while profiling, timed
 * or not (HOST arrays of QP_PROF_COUNT entries; any may be NULL), then frees the
 * events.  Categories (one kernel each): */
enum {
  QP_PROF_ROWPASS = 0,    /* row-side operator kernel of K v (rows of P and A) */
  QP_PROF_COLPASS = 1,    /* column-side operator kernel of K v (x-part) */
  QP_PROF_TSREDUCE = 2,   /* dense low-rank reduction U^T v, C v */
  QP_PROF_EPILOGUE = 3,   /* sum of per-chunk partials, either side (multi-chunk only) */
  QP_PROF_CGUPDATE = 4,   /* PCG: alpha, x, r, z, r.z */
  QP_PROF_CGPUPDATE = 5,  /* PCG: beta, p */
  QP_PROF_FUSED = 6,      /* fused single-read operator kernel of K v (see qp_fused_layout) */
  QP_PROF_COUNT = 7
};
qp_status qp_profile_begin(qp_handle h, int32_t max_launches, int32_t every);
qp_status qp_profile_end(qp_handle h, int64_t* launches, double* total_ms, int64_t* dispatches);

/* Bytes of the stored operators (HOST out): row-side CSR, column-side CSR,
 * dense low-rank factor, each in the precision the PCG matvec reads, plus
 * the nonzero counts of the two CSR structures. */
qp_status qp_operator_bytes(qp_handle h, int64_t* row_bytes, int64_t* col_bytes,
                            int64_t* dense_bytes, int64_t* row_nnz, int64_t* col_nnz);

/* Blocked layout of the two sparse operators (HOST out arrays of 2 entries,
 * [0] row side, [1] column side; any may be NULL): column chunks staged in LDS
 * per work item (0 when that side runs the unblocked kernel), work items (=
 * blocks) per pass, and columns per chunk.  With more than one chunk a pass
 * writes per-chunk partials that a second kernel adds up. */
qp_status qp_operator_layout(qp_handle h, int32_t* chunks, int32_t* work_items,
                             int32_t* chunk_cols);

/* The fused single-read product of K v for H = P^T W P (matrix-free as in
 * Section 3.2; a layout choice of this library, not of the paper).  Every
 * contribution of a row of P (or of A) to K v depends only on that row's
 * own dot, so one pass over the rows, each entry read once, forms the whole
 * product.  Its columns are cut in two halves, each row range is handled by
 * a pair of blocks that exchange the half dots of their rows through device
 * memory; sums of the scatter are taken in a run-dependent order, so results
 * agree with the two-pass kernels to rounding, not bitwise.  qp_create builds
 * it when H = P^T W P, n <= 20,208 and the operator has at least 2^22
 * entries (QPK_FUSED=0: never; QPK_FUSED=1: whenever the shape allows);
 * then every product of the handle uses it.  A pair whose partner never runs
 * alongside (its wait is bounded by QPK_FUSED_SPIN polls, default 2^21)
 * invalidates the product; the library then switches the handle to the
 * two-pass kernels and redoes that product or PCG solve, and reports it here.
 * HOST outs, any may be NULL: active (1 while products use it), row ranges
 * (block pairs), columns in the first half, stored entries (with the
 * even-length padding), and failed (1 after such a switch). */
/* PCG iterations replayed from a HIP graph.  Float64 PCG solves (kkt_pcg_solve,
 * and those of ipm_solve and qp_backward) with an even pcg_options.check_every
 * queue their iterations in chunks of check_every: the first chunk's launches
 * (product, update, direction update, each of which reads the stop flag) are
 * captured once into a graph on a stream of the library's own, and every full
 * chunk then replays it on the handle's stream.  The graph is captured again
 * when a pointer, option or mu it was built with changes (each Newton system
 * with a new mu); it holds kernels only.  Reduced-precision and profiled
 * solves launch kernel by kernel, and so does every solve with QPK_GRAPH=0 in
 * the environment when the handle was created.  HOST outs, may be NULL: the
 * handle's captures and replays so far. */
qp_status qp_graph_stats(qp_handle h, int64_t* captures, int64_t* replays);

qp_status qp_fused_layout(qp_handle h, int32_t* active, int32_t* ranges, int32_t* half_cols,
                          int64_t* stored, int32_t* failed);

#ifdef __cplusplus
}
#endif

#endif /* QPK_H */
