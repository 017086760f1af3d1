/*
 * dynscreen.h - C-ABI of the MI355X dynamic-screening Lasso / Group-Lasso library.
 *
 * Problem (paper eq. (1)):  x* = argmin_x 1/2 ||D x - y||_2^2 + lambda * Omega(x)
 *   Lasso       (eq. (lasso)):        Omega(x) = ||x||_1
 *   Group-Lasso (eq. (group-lasso)):  Omega(x) = sum_g w_g ||x_g||_2, G a partition of the atoms
 * solved by Algorithm 3 ("general algorithm with dynamic screening") with the ISTA
 * or FISTA update of Table 1, and a safe sphere test re-evaluated at every iteration:
 *   Lasso:       SAFE (Lemma 1) or DST3 (Lemma 2)
 *   Group-Lasso: GSAFE (Lemma 4) or DGST3 (Lemma 5), through the group sphere test (Lemma 6).
 *
 * Conventions shared by every entry point
 *   - D is column-major, N x K, leading dimension ldd >= N, in DEVICE memory.  Atom i
 *     is the ldd-strided column i.  Storage type: DS_F64 (double), DS_F32 (float),
 *     DS_BF16 (bfloat16 bit patterns, uint16).  The stored values define the problem.
 *   - Vectors y, x live in DEVICE memory.  Their element type is double for DS_F64 and
 *     float for DS_F32 and DS_BF16.
 *   - Host arrays (group offsets, weights, lambdas, info) are read or written before
 *     the call returns; the library keeps no pointer to caller memory after a call.
 *   - `stream` is a hipStream_t (NULL: the default stream).  Solves are blocking with
 *     respect to the host: on return every output has been written.
 *   - Errors: a ds_status code.  Arguments are validated before any device work; a
 *     rejected call leaves outputs untouched.  ds_last_error() returns a thread-local
 *     message describing the last failure.
 *   - Thread safety: calls may come from several host threads; the library serialises
 *     device work per device internally.
 */
#ifndef DYNSCREEN_H
#define DYNSCREEN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DS_OK = 0,             /* solved; for gap_tol > 0 the gap certificate met the tolerance */
  DS_PENDING = 1,        /* serving: request not finished yet */
  DS_NOT_CONVERGED = 2,  /* max_iter reached with gap_tol > 0 and the gap above tolerance;
                            outputs and info are still filled in */
  DS_EINVAL = -1,        /* invalid argument (nothing was launched) */
  DS_ENOMEM = -2,        /* device allocation failed, or a request can never fit the budget */
  DS_EDEVICE = -3,       /* a HIP call failed */
  DS_ENOTFOUND = -4,     /* unknown request / dictionary id */
  DS_EBUSY = -5          /* serving: queue full */
} ds_status;

typedef enum { DS_F64 = 0, DS_F32 = 1, DS_BF16 = 2 } ds_dtype;

/* First-order update of Table 1.  DS_SPARSA is ISTA whose L_t follows the Barzilai-Borwein
 * rule (the SpaRSA row of Table 1): after an accepted step d = x' - p, L becomes
 * ||D d||^2 / ||d||^2 (clamped to [1e-30, 1e30]; kept when d = 0), and a step is accepted
 * when phi(x') <= max(memory) - (bb_sigma / 2) L ||d||^2, phi the primal objective and the
 * memory its values at the current primal point and the bb_memory iterates before it;
 * phi(x') - phi(p) is formed as theta^T D d + ||D d||^2 / 2 + lambda (Omega(x') - Omega(p))
 * with the Omega difference taken unit by unit.  A rejected step is undone and L multiplied
 * by bt_eta, as for DS_STEP_BACKTRACK.  Single-signal and served solves; step_rule must be
 * DS_STEP_CONSTANT, and the batched bfloat16 path returns DS_EINVAL. */
typedef enum { DS_ISTA = 0, DS_FISTA = 1, DS_SPARSA = 2, DS_CP = 3 } ds_rule;
/* DS_CP is the Chambolle-Pock update of Table 1: the dual iterate is carried,
 * theta_t = (theta_{t-1} + sigma (D u_{t-1} - y)) / (1 + sigma), x_t = prox(x_{t-1} -
 * tau D^T theta_t, lambda tau), u_t = x_t + phi (x_t - x_{t-1}) with phi = 1/sqrt(1 +
 * 2 gamma tau), then tau <- phi tau, sigma <- sigma / phi (cp_tau, cp_sigma, cp_gamma).
 * The screening and the gap use theta_t's dual point; the gap's primal point is u_{t-1},
 * and that point is what the solve returns.  Single-signal and served solves; step_rule
 * must be DS_STEP_CONSTANT (step_L is the bound L >= ||D||_2^2 that sets the default
 * steps), and the batched bfloat16 path returns DS_EINVAL. */

/* Screening test.  For Group-Lasso problems SAFE means GSAFE (Lemma 4) and DST3 means
 * DGST3 (Lemma 5).  DS_TEST_DOME is the dynamic Dome test (the dome lemma: the SAFE ball
 * B(y/lambda, ||y/lambda - v_t||) cut by the half-space d_*^T theta <= 1 of the atom
 * attaining lambda_*); Lasso only (glasso_solve returns DS_EINVAL).  DS_TEST_NONE runs the
 * plain, unscreened algorithm. */
typedef enum { DS_TEST_NONE = 0, DS_TEST_SAFE = 1, DS_TEST_DST3 = 2, DS_TEST_DOME = 3 } ds_test;

/* How `lambdas` is read: absolute penalties, or ratios lambda / lambda_* where
 * lambda_* = ||D^T y||_inf (Lasso) or max_g ||D_g^T y|| / w_g (eq. (gstar)) is
 * computed on the device for each signal. */
typedef enum { DS_LAMBDA_ABSOLUTE = 0, DS_LAMBDA_RELATIVE = 1 } ds_lambda_mode;

typedef struct {
  ds_dtype dtype;
  int64_t N;                 /* signal dimension, >= 1 */
  int64_t K;                 /* number of atoms, >= 1 */
                             /* Single-signal, multi-signal FP32/FP64 and served solves cover
                                N <= 262144 * e rows, e = 16 bytes / element size when D and
                                ldd * element size are 16-byte aligned (else e = 1), and at
                                most 262144 atoms (Lasso) or 131072 groups; a larger problem
                                returns DS_EINVAL before any device work. */
  int64_t ldd;               /* leading dimension of D, >= N */
  const void* D;             /* device pointer, column-major N x K */
  int64_t G;                 /* 0: Lasso.  > 0: Group-Lasso with G groups */
  const int64_t* group_ptr;  /* host, G+1 offsets: group g = atoms [group_ptr[g], group_ptr[g+1]);
                                group_ptr[0] = 0, group_ptr[G] = K, strictly increasing.
                                Any partition is reached by permuting the columns of D. */
  const double* w;           /* host, G positive weights; NULL means w_g = sqrt(|g|) */
} ds_problem;

/* Screening mode: DS_DYNAMIC runs the test at every iteration (Algorithm 3); DS_STATIC
 * runs it once, with the dual point of the first iteration (Algorithms 1 and 4: the static
 * SAFE / ST3 / Dome rules). */
typedef enum { DS_DYNAMIC = 0, DS_STATIC = 1 } ds_mode;

/* Step size L_t of the proximal update (Table 1). */
typedef enum { DS_STEP_CONSTANT = 0, DS_STEP_BACKTRACK = 1 } ds_step_rule;

typedef struct {
  ds_rule rule;
  ds_test test;
  ds_lambda_mode lambda_mode;
  double step_L;     /* DS_STEP_CONSTANT: > 0: constant step 1/step_L, must be >= ||D||_2^2;
                        <= 0: the library estimates ||D||_2^2 (ds_spectral_norm_sq).
                        DS_STEP_BACKTRACK and DS_SPARSA: > 0: L_0; <= 0: L_0 = the largest
                        squared atom norm (Lasso) or ||D_g||_2^2 (Group-Lasso). */
  double gap_tol;    /* > 0: stop once the duality-gap certificate <= gap_tol * ||y||^2.
                        0: run exactly max_iter iterations. */
  int32_t max_iter;  /* >= 1 */
  ds_mode screening; /* 0: dynamic (Algorithm 3: the test is re-run at every iteration).
                        1: static (Algorithms 1 and 4: the test is run once, with the dual
                        point of the first iteration, i.e. the static SAFE / ST3 rules). */
  int32_t step_rule; /* ds_step_rule.  DS_STEP_BACKTRACK: the rule of Beck and Teboulle that
                        Table 1 names for ISTA and FISTA.  The proximal point x' of an
                        iteration is kept when ||D (x' - p)||^2 <= L ||x' - p||^2 (for the
                        quadratic data term, F(x') <= Q_L(x', p)); otherwise the iteration is
                        repeated from the same p with L multiplied by bt_eta (the rejected pass
                        still counts as an iteration and still screens).  Single-signal and
                        served solves; the batched bfloat16 path returns DS_EINVAL. */
  double bt_eta;     /* backtracking and SpaRSA growth factor of L, > 1; 0 selects 2 */
  int32_t bb_memory; /* DS_SPARSA: earlier iterates in the acceptance memory, 0..15
                        (0: monotone) */
  double bb_sigma;   /* DS_SPARSA: sufficient-decrease constant, >= 0; 0 selects 1e-5 */
  double cp_tau;     /* DS_CP: initial primal step tau_0 > 0; 0 selects 1/sqrt(L) */
  double cp_sigma;   /* DS_CP: initial dual step sigma_0 > 0; 0 selects 1/(tau_0 L).  The
                        method needs tau_0 sigma_0 ||D||_2^2 <= 1 (checked against step_L
                        when both steps and step_L are given) */
  double cp_gamma;   /* DS_CP: acceleration gamma >= 0 (0: constant steps) */
  const void* x0;    /* optional initial point X_0, the input of Algorithm 3 (NULL: x_0 = 0).
                        Element type as x.  lasso_solve / glasso_solve / ds_solve_batch: DEVICE,
                        K x B with the leading dimension ldx of X; ds_solve_one: DEVICE, K
                        values; ds_submit / lasso_submit: HOST, K values, copied at submit.
                        The first iteration then starts from x_0 = u_0 = X_0 (l_0 = 1; the
                        Chambolle-Pock dual iterate still starts at 0).  A non-finite entry
                        makes the solve return DS_EINVAL.  The batched bfloat16 path (B > 1,
                        DS_BF16 Lasso) returns DS_EINVAL when x0 is given. */
  double obj_tol;    /* >= 0.  > 0: also stop once the primal objective of the certified point
                        changes by at most obj_tol relative between two consecutive iterations
                        (|P_{t-1} - P_t| <= obj_tol P_t), the stopping rule of the paper's
                        experiments section (there with 1e-7 and max_iter = 200).  Such a
                        stop returns DS_OK.  The batched bfloat16 path returns DS_EINVAL. */
  int32_t batch_slots; /* batched bfloat16 path: signals resident on the device at once
                        (0: min(B, 512)).  When B exceeds it, the other signals wait and take
                        the slots of finished ones (continuous batching); results do not depend
                        on it.  Ignored elsewhere; must be >= 0. */
} ds_params;

/* Per-signal result.  The gap certificate of iteration t pairs the primal point at which
 * theta_t = D p - y was evaluated (x_{t-1} for ISTA, u_{t-1} for FISTA) with the dual
 * point v_t = mu_t theta_t obtained by dual scaling (Lemma 7); the returned x_t has an
 * objective no larger than that primal point's. */
typedef struct {
  int32_t status;      /* ds_status of this signal */
  int32_t iters;       /* iterations run (0 when lambda >= lambda_*, where x = 0) */
  int32_t n_active;    /* atoms not screened when the solve ended */
  int32_t nnz;         /* non-zeros of the returned x */
  double lambda;       /* absolute penalty used */
  double lambda_max;   /* lambda_* */
  double primal;       /* P(p) at the last iteration */
  double dual;         /* dual objective at v_T (eq. (dual) / (dual_glasso)) */
  double gap;          /* primal - dual */
  double radius;       /* smallest sphere radius reached (r_min) */
  double mu;           /* dual-scaling factor of the last iteration */
  double L;            /* step constant used (backtracking: the last L_t) */
  double radius_slack; /* rounding slack added to the radius (>= 0) */
  double queue_ms;     /* served requests: submit -> start of the solve; else 0 */
  double run_ms;       /* served requests: start -> end of the solve; else 0 */
} ds_info;

/* lasso_solve / glasso_solve
 *   Solve B independent problems sharing D: column b of Y (N x B, leading dim ldy >= N)
 *   with penalty lambdas[b] (host array of B values > 0, read per lambda_mode), writing
 *   column b of X (K x B, leading dim ldx >= K, device) and info[b] (host).
 *   lasso_solve requires problem->G == 0; glasso_solve requires problem->G > 0.
 *   B = 1 runs the single-signal streaming path (one GEMV per iteration); B > 1 with
 *   DS_BF16 storage runs the batched MFMA path (Lasso and Group-Lasso); other B > 1 cases
 *   run B single solves,
 *   up to four at a time on streams of the library's own (each waits for the work queued
 *   on `stream` before the call; each column's result equals its B = 1 solve bit for bit).
 *   The call returns when every column is written.
 *   Returns DS_OK if every signal reached its tolerance (or ran max_iter when gap_tol = 0),
 *   DS_NOT_CONVERGED if some did not (see info[b].status), or an error code. */
ds_status lasso_solve(const ds_problem* problem, const void* Y, int64_t B, int64_t ldy,
                      const double* lambdas, const ds_params* params, void* X, int64_t ldx,
                      ds_info* info, void* stream);
ds_status glasso_solve(const ds_problem* problem, const void* Y, int64_t B, int64_t ldy,
                       const double* lambdas, const ds_params* params, void* X, int64_t ldx,
                       ds_info* info, void* stream);

/* One iteration record of a single-signal solve: the quantities the paper's flops model
 * records per iteration (dictionary size |I^c_t| and ||x_t||_0), plus radius and gap. */
typedef struct {
  int32_t n_active;   /* atoms in the (screened) dictionary used by iteration t */
  int32_t n_units;    /* active atoms (Lasso) or active groups (Group-Lasso) */
  int32_t n_support;  /* non-zeros of the primal point theta_t was evaluated at */
  int32_t nnz;        /* non-zeros of x_t */
  double radius;      /* sphere radius r_t of iteration t (no slack; +inf without a test) */
  double gap;         /* gap certificate of iteration t */
} ds_trace;

/* Single-signal solve with optional diagnostic outputs (Lasso if problem->G == 0, else
 * Group-Lasso).  y, x as in lasso_solve with B = 1.  `screened` (DEVICE, K bytes, may be
 * NULL) receives 1 for every atom of the final screened set I_T and 0 otherwise, in the
 * original atom order.  `trace` (HOST, may be NULL) receives min(iters, trace_cap)
 * records, one per iteration. */
ds_status ds_solve_one(const ds_problem* problem, const void* y, double lambda,
                       const ds_params* params, void* x, uint8_t* screened, ds_trace* trace,
                       int32_t trace_cap, ds_info* info, void* stream);

/* lasso_solve (glasso_solve when problem->G > 0) with a diagnostic output: `screened`
 * (DEVICE, K x B bytes, column b at offset b * K, may be NULL) receives 1 for every atom of
 * signal b's final screened set (groups: every atom of a screened group) and 0 otherwise.
 * For B > 1 with DS_BF16 storage (the batched MFMA path)
 * the correlations that drive the iteration are FP32-accumulated on the matrix cores;
 * the sphere radius carries their rounding bound (reported in info[b].radius_slack) and
 * the gap that ends each solve is recomputed in FP64 at that iteration's primal point.
 * Other cases run single-signal solves.  Return value and errors as lasso_solve. */
ds_status ds_solve_batch(const ds_problem* problem, const void* Y, int64_t B, int64_t ldy,
                         const double* lambdas, const ds_params* params, void* X, int64_t ldx,
                         ds_info* info, uint8_t* screened, void* stream);

/* For callers that cannot allocate device memory (code being captured into a HIP graph,
 * serving loops and harnesses that forbid allocation): ds_solve_one without the trace,
 * whose workspace is a fixed library-owned device array of DS_NOALLOC_SCRATCH_MB MiB per
 * device (held from library load until the process ends) and whose state is read back
 * through a static host buffer, so the call allocates nothing.  Arguments, outputs and
 * results are those of ds_solve_one (the same kernels run), with two restrictions:
 *   - a constant step (DS_STEP_CONSTANT with DS_ISTA, DS_FISTA or DS_CP) needs step_L > 0
 *     (estimating ||D||_2^2 would need a workspace of its own): else DS_EINVAL;
 *   - the problem's workspace must fit the array (for the Lasso about 140 bytes per
 *     atom, 8 N ceil(K / 512) bytes, 40 bytes per iteration of max_iter and 1.2 MB): a
 *     larger problem gets DS_EINVAL before any device work, with the size it needs in
 *     ds_last_error().
 * All calls on one device share the array: they are serialised inside the library, and the
 * array keeps the last call's contents (each solve clears what must start at zero).  Calls
 * on one device issued from separate processes, or re-entered from a stream callback,
 * would race on it. */
#define DS_NOALLOC_SCRATCH_MB 64
ds_status ds_solve_one_noalloc(const ds_problem* problem, const void* y, double lambda,
                               const ds_params* params, void* x, uint8_t* screened,
                               ds_info* info, void* stream);

/* lambda_* of a single signal y (device, length N) and the first index attaining it
 * (atom index for the Lasso, group index for the Group-Lasso); FP64 accumulation. */
ds_status ds_lambda_max(const ds_problem* problem, const void* y, double* lambda_max,
                        int64_t* argmax, void* stream);

/* Estimate of ||D||_2^2 (largest eigenvalue of D D^T) by FP64 power iteration with a
 * Krylov-Weinstein residual bound added, so the value is an upper estimate.  Cost:
 * 2 * iters GEMV passes over D. iters <= 0 selects 200. */
ds_status ds_spectral_norm_sq(const ds_problem* problem, int32_t iters, double* L,
                              void* stream);

/* ---------------------------------------------------------------- serving ---------
 * Continuous-batching request loop.  Dictionaries are copied into library-owned device
 * memory at registration; requests carry y on the host, are admitted when their device
 * footprint fits the HBM budget and a slot is free, and run interleaved with other
 * requests on the device.
 * With batch_slots > 0, every bfloat16 dictionary also gets a batched engine (the
 * matrix-core path of lasso_solve / glasso_solve): a request for it whose parameters that
 * path supports
 * (ISTA or FISTA, constant step, SAFE / DST3 / Dome / no test, no x0, obj_tol = 0) joins the
 * engine's resident signals at the next graph-replay boundary where a slot is free, and
 * leaves as soon as it has finished; requests with the same parameters share a run (a
 * request with other parameters is overtaken at no more than 16 slot refills, then the run drains
 * and the next one starts with it).  Its result equals the batched result of lasso_solve
 * (glasso_solve) for the same y and lambda bit for bit, alone or in any mix.  Other
 * requests run as single-signal solves on the worker slots. */
typedef struct {
  int32_t device;           /* HIP device ordinal */
  int32_t max_slots;        /* single-signal requests resident on the device at once (>= 1) */
  size_t hbm_budget_bytes;  /* device memory the server may use for requests (> 0) */
  int32_t max_queue;        /* maximum pending requests before DS_EBUSY (>= 1) */
  int32_t batch_slots;      /* 0: no batched engines; else signals resident in each
                               bfloat16 dictionary's batched engine (<= 32768) */
} ds_server_config;

/* Starts max_slots worker threads.  Failure-path testing: when the environment variable
 * DS_SERVE_FAIL_REQUEST holds a request id at creation, that request's slot is marked
 * failed once its solve has run; lasso_poll then returns DS_EDEVICE for it (no x), while
 * every other request completes as it would have (host side only, no device fault). */
ds_status ds_server_create(const ds_server_config* config, void** server);
/* Copies D (device or host pointer, detected) into server memory, converting to `store`
 * precision (DS_F32 or DS_BF16 from DS_F32 input; same type otherwise), and computes and
 * caches ||D||_2^2 (used as the step constant unless a request sets step_L > 0).  The
 * dictionary stays resident until ds_server_destroy; it is not charged to the budget. */
ds_status ds_server_add_dict(void* server, const ds_problem* problem, ds_dtype store,
                             int32_t* dict_id);
/* Queue a solve of y (HOST pointer, N floats, or doubles for a DS_F64 dictionary) with
 * penalty `lambda` (read per params->lambda_mode).  Returns immediately.  Errors:
 * DS_ENOTFOUND (unknown dictionary), DS_EBUSY (max_queue requests already waiting),
 * DS_ENOMEM (the request's device footprint exceeds the whole budget), DS_EINVAL. */
ds_status ds_submit(void* server, int32_t dict_id, const void* y_host, double lambda,
                    const ds_params* params, uint64_t* request_id);
/* Lasso-named alias of ds_submit (the dictionary decides Lasso or Group-Lasso). */
ds_status lasso_submit(void* server, int32_t dict_id, const void* y_host, double lambda,
                       const ds_params* params, uint64_t* request_id);
/* DS_PENDING while queued or running; otherwise copies x (K values, HOST) and info,
 * forgets the request and returns its final status.  x_host may be NULL to discard x.
 * DS_ENOTFOUND for an unknown (or already collected) request id. */
ds_status lasso_poll(void* server, uint64_t request_id, void* x_host, ds_info* info);
/* Stops the workers (requests still queued are dropped, running ones finish first) and
 * frees the server's device memory. */
ds_status ds_server_destroy(void* server);

/* ---------------------------------------------------------------- diagnostics ------ */
typedef struct {
  int64_t launches;   /* kernel launches accounted */
  double ms;          /* summed execution time of those launches: device wall clock from the
                         first workgroup's start to the last workgroup's end, read inside
                         the kernel */
  double bytes;       /* summed algorithmic HBM bytes */
  double flops;       /* summed algorithmic flops */
  double ms_event;    /* summed time between HIP events carried by the same dispatches
                         (includes the command processor's dispatch overhead) */
} ds_kernel_stat;

/* CORR: single-signal correlation pass; RESID: single-signal residual pass; SETUP:
 * setup passes; BATCH: batched Z = D^T Theta GEMM with the fused update; BATCH_THETA:
 * batched Theta = D U GEMM; ITER: one single-signal iteration (its correlation and the
 * residual pass after it). */
enum { DS_STAT_CORR = 0, DS_STAT_RESID = 1, DS_STAT_SETUP = 2, DS_STAT_BATCH = 3,
       DS_STAT_BATCH_THETA = 4, DS_STAT_ITER = 5, DS_STAT_COUNT = 6 };

/* One launch record of an instrumented single-signal solve: DS_STAT_CORR (a correlation
 * pass: its execution time on the device wall clock, as ds_kernel_stat.ms, and its
 * algorithmic bytes), DS_STAT_RESID (the residual pass after it: time between the HIP
 * events of its dispatch, bytes of the support columns it streams) or DS_STAT_ITER (the
 * two together: the sum of their event times).  n_atoms is the correlation's active atoms
 * |I^c_t| in all three. */
typedef struct {
  int32_t kernel;     /* DS_STAT_CORR, DS_STAT_RESID or DS_STAT_ITER */
  int32_t n_atoms;    /* active atoms |I^c_t| of the iteration */
  double bytes;       /* algorithmic bytes (0 for DS_STAT_ITER) */
  double ms;          /* execution time */
} ds_launch_stat;

/* When enabled, each launch of the instrumented kernels is bracketed by HIP events on
 * its stream and its algorithmic bytes/flops are added to the counters. */
void ds_stats_enable(int on);
void ds_stats_reset(void);
/* Copies min(n, DS_STAT_COUNT) counters into out; returns the number copied. */
int ds_stats_read(ds_kernel_stat* out, int n);
/* Copies up to n per-launch records (correlation, residual, iteration) accounted since the
 * last ds_stats_reset (the first 2^20 are kept, in launch order); returns the number
 * copied. */
int ds_stats_launches(ds_launch_stat* out, int n);

/* Block shape of the batched path's Z = D^T Theta kernel in the last batched solve on the
 * current device: its index, and (when the pointers are non-NULL) the atoms and signals a
 * block covers.  The shape is chosen per (N, K, B) by timing every eligible one once (the
 * results do not depend on it); DS_BATCH_TILE=<index> forces one, and DS_AUTOTUNE_CACHE
 * names a file that keeps the choices across processes.  -1 before any batched solve. */
int ds_batch_shape(int* atoms, int* signals);

const char* ds_last_error(void);
const char* ds_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DYNSCREEN_H */
