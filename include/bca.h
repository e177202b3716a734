/*
 * bca.h -- C ABI of the MI355X Bi-cADMM library (libbca.so).
 *
 * Bi-cADMM (Olama, Lundell, Kronqvist, Ahmadi, Camponogara, "A GPU-Accelerated
 * Bi-linear ADMM Algorithm for Distributed Sparse Machine Learning") solves the
 * sparse machine-learning problem of Sec. 2,
 *
 *     min_x  sum_i l_i(A_i x; b_i) + ||x||^2 / (2 gamma)   s.t.  ||x||_0 <= kappa,
 *
 * over N sample partitions (the paper's computational nodes), each split into M
 * feature blocks (the paper's GPUs of a node, Sec. 3.1).  On one GPU every
 * partition and block lives in device memory and all of Algorithms 1 and 2 runs
 * in this library's HIP kernels.
 *
 * Conventions
 *   - Every function returns int: BCA_OK (0) or a negative BCA_E_* code; no
 *     function throws across the ABI.  bca_last_error() gives a thread-local
 *     message for the last failure on the calling thread.
 *   - The caller owns every buffer it passes.  bca_set_data copies A and b into
 *     library-owned device memory and keeps no caller pointer.  All device state
 *     is owned by the problem handle and released by bca_destroy.
 *   - All device work is enqueued on the HIP stream given to bca_create (NULL =
 *     the null stream).  Functions that return host data synchronise that stream.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Vectors of length n x C are stored feature-major: element (k, c) at k*C + c.
 */
#ifndef BCA_H
#define BCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bca_problem_s* bca_problem;
typedef struct bca_server_s* bca_server;

/* Return codes. */
enum {
  BCA_OK = 0,
  BCA_E_INVALID = -1,   /* bad argument or parameter */
  BCA_E_OOM = -2,       /* device allocation failed */
  BCA_E_STATE = -3,     /* call out of order (e.g. step before finalize) */
  BCA_E_NONFINITE = -4, /* NaN/Inf in the data or in the iterates */
  BCA_E_DEVICE = -5,    /* HIP runtime error */
  BCA_E_BUDGET = -6,    /* request exceeds a memory budget */
  BCA_E_NOTFOUND = -7,  /* unknown ticket or index */
  BCA_E_CANCELLED = -8  /* request was cancelled */
};

/* Loss functions l_i (Sec. 2 lists sparse linear, logistic and softmax
 * regression; the experimental section fixes the squared loss without 1/2; the
 * introduction also names sparse SVMs, without a formulation):
 *   SQUARED   l(q; b) = sum_k (q_k - b_k)^2,          b real
 *   LOGISTIC  l(q; b) = sum_k log(1 + exp(-b_k q_k)),  b_k in {-1, +1}
 *   SOFTMAX   l(Q; y) = sum_k LSE(Q_k) - Q_{k, y_k},   y_k in {0..C-1};
 *             the sparsity then counts rows of the n x C coefficient matrix
 *   HINGE     l(q; b) = sum_k max(0, 1 - b_k q_k),     b_k in {-1, +1}
 *             (the sparse SVM, with the same ridge term 1/(2 gamma) ||x||^2). */
enum { BCA_LOSS_SQUARED = 0, BCA_LOSS_LOGISTIC = 1, BCA_LOSS_SOFTMAX = 2, BCA_LOSS_HINGE = 3 };

/* Storage precision of A.  F64: FP64 arithmetic throughout.  F32: FP32
 * products with FP64 long sums.  BF16: BF16 storage, FP32 products, FP64 long
 * sums.  The Cholesky factors, the iterates, the global step and the residuals
 * are FP64 for every storage precision. */
enum { BCA_F64 = 0, BCA_F32 = 1, BCA_BF16 = 2 };

/* Where a buffer passed to the library lives. */
enum { BCA_MEM_HOST = 0, BCA_MEM_DEVICE = 1 };

/* Solver parameters.  The names follow the paper: gamma is the ridge weight of
 * the SML problem (Sec. 2), rho_c the consensus penalty, rho_b the penalty of
 * the bilinear constraint x^T s = t (Sec. 3), rho_l the penalty of the
 * feature-split sub-solver (Sec. 3.1).  kappa bounds ||x||_0 (rows for softmax). */
typedef struct {
  int32_t loss;          /* BCA_LOSS_* */
  int32_t n_features;    /* n >= 1 */
  int32_t n_classes;     /* C: 1 unless softmax (2..64) */
  int32_t n_partitions;  /* N >= 1 sample partitions */
  int32_t n_blocks;      /* M >= 1 feature blocks per partition, M <= n */
  int32_t kappa;         /* 1 <= kappa <= n */
  const int64_t* rows;   /* host array of N entries: m_i >= 1; read by bca_create only */
  double gamma, rho_c, rho_b, rho_l;   /* all > 0 */
  int32_t inner_iters;   /* K_in >= 1 inner (Algorithm 2) iterations per outer iteration */
  int32_t max_iters;     /* K >= 1: cap on outer iterations for bca_solve; size of the residual history */
  double tol_p, tol_d, tol_b;          /* bca_solve stops when p_r <= tol_p, d_r <= tol_d, b_r <= tol_b */
  int32_t a_dtype;       /* BCA_F64 / BCA_F32 / BCA_BF16 */
  int32_t check_every;   /* bca_solve reads the residuals back every this many iterations (0 = 10) */
  uint32_t flags;        /* BCA_FLAG_* bits, 0 for the paper's method as written */
} bca_params;

/* Variant of the x-update (Sec. 3.1).  EXACT_X, squared or logistic loss: the
 * x-update of every partition is solved exactly -- the limit of Algorithm 2's
 * inner loop -- instead of by inner_iters warm-started inner iterations; n_blocks
 * is then ignored (one block of n features) and the omega-bar / nu state stays
 * zero.  Squared loss: x_i = H_i^-1 (2 A_i^T b_i + rho_c (z - u_i)) with
 * H_i = 2 A_i^T A_i + (1/(N gamma) + rho_c) I; H_i^-1 is formed once at finalize
 * (n x n per partition, FP64) and A_i^T b_i is streamed once, so an outer
 * iteration reads no A at all.  Logistic loss: Newton's method on the whole
 * subproblem, each direction by conjugate gradients preconditioned with the
 * cached (A_i^T A_i / 4 + (1/(N gamma) + rho_c) I)^-1 and stopped by an inexact-
 * Newton forcing term; every CG iteration is one pass over A (Hessian-vector
 * product), the step length an Armijo search over stored row values; the Newton
 * iteration stops once the step is below 1e-13 (FP64 data) or 1e-8 (FP32, BF16)
 * of max|x_i|, or after 12 Newton iterations of at most 100 CG iterations each;
 * needs N <= 256.  Not available in the batched and serving forms. */
enum { BCA_FLAG_EXACT_X = 1 };

/* WOODBURY, one-class losses (squared, logistic, hinge): the same iteration
 * (Algorithm 2's x_ij-step, inner_iters per outer iteration) computed in the
 * sample space, for blocks with fewer rows than columns (m_i < n_j).  By the
 * matrix inversion lemma the x_ij-step's new block prediction is
 * p+ = d - shift S_ij^-1 d + rho_c S_ij^-1 A_ij (z_j - u_ij) with
 * S_ij = rho_l A_ij A_ij^T + shift I (m_i x m_i, shift = 1/(N gamma) + rho_c)
 * and d = p_ij + e, so the inner iterations read only the cached S_ij^-1
 * (m_i^2 / 2 FP64 entries per block, formed once at finalize from FP64 sums)
 * and A is read twice per outer iteration: once for A_ij (z_j - u_ij) and
 * p_ij = A_ij x_ij (d is re-derived from the state at every outer iteration),
 * once for x_ij = (rho_l / shift) A_ij^T (d - p+) + (rho_c / shift)(z_j - u_ij).  Results
 * equal those of the default form up to rounding.  Device memory: N M
 * ceil(mw/64) (ceil(mw/64) + 1) / 2 tiles of 32 KB, mw = max_i m_i, instead of
 * the n_j x n_j inverses.  bca_get_inverse then fails with BCA_E_STATE; not
 * available with EXACT_X, softmax, or in the batched and serving forms. */
enum { BCA_FLAG_WOODBURY = 2 };

/* Create a problem: validates the parameters and allocates device memory for
 * the data and the ADMM state.  hip_stream is a hipStream_t (may be NULL).
 * Errors: BCA_E_INVALID (parameter out of range), BCA_E_OOM, BCA_E_DEVICE. */
int bca_create(const bca_params* params, void* hip_stream, bca_problem* out);

/* Load partition `part` (0 <= part < N): A_i is m_i x n in the problem's a_dtype
 * (row-major, row stride `ld` elements >= n; BF16 as uint16 bit patterns), b_i
 * holds m_i doubles (squared: targets; logistic: labels -1/+1) or m_i int32
 * class ids (softmax).  `mem` says whether A and b are host or device pointers;
 * both are copied before the call returns (the copy is ordered on the problem's
 * stream and the call synchronises it).  A partition may be loaded again until
 * bca_finalize.
 * Errors: BCA_E_INVALID (bad index, ld < n, label out of range),
 * BCA_E_NONFINITE (NaN/Inf in A or b), BCA_E_STATE (after finalize). */
int bca_set_data(bca_problem p, int32_t part, const void* A, int64_t ld, const void* b, int32_t mem);

/* Setup of Sec. 3.1's x_ij-step, once per problem: for every partition i and
 * block j the Gram matrix A_ij^T A_ij (MFMA), K_ij = rho_l A_ij^T A_ij +
 * (1/(N gamma) + rho_c) I, its FP64 Cholesky factor L_ij, W_ij = L_ij^-1 and the
 * cached inverse K_ij^-1 = W_ij^T W_ij (FP64, tiled), which every x_ij-step then
 * applies as one symmetric matrix-vector product.  With BCA_FLAG_EXACT_X the same
 * is done once per partition for H_i = 2 A_i^T A_i + (1/(N gamma) + rho_c) I
 * (squared loss) or the preconditioner A_i^T A_i / 4 + (1/(N gamma) + rho_c) I
 * (logistic loss); with BCA_FLAG_WOODBURY for S_ij = rho_l A_ij A_ij^T +
 * (1/(N gamma) + rho_c) I.  Also allocates the batched form's partial sums for
 * problems within its limits.  The Gram and factor work space comes from the
 * stream-ordered allocator on the problem's stream (hipMallocAsync) and is
 * released before the call returns.  Resets the ADMM state to zero.
 * Errors: BCA_E_STATE (a partition was never loaded), BCA_E_NONFINITE (K_ij not
 * positive definite in FP64), BCA_E_DEVICE. */
int bca_finalize(bca_problem p);

/* Run `outer_iters` outer iterations of Algorithm 1: per partition K_in inner
 * iterations of Algorithm 2 (x_ij ridge solves with the cached factors, block
 * predictions averaged over the blocks, per-sample omega-bar prox, nu update),
 * then the consensus average, the (z,t) step, the top-kappa s-step, the v- and
 * u-updates and the residuals p_r, d_r, b_r (Sec. 3, Termination).  Enqueued
 * asynchronously; *iters_done (may be NULL) gets the total outer iteration count.
 * Errors: BCA_E_STATE (before finalize), BCA_E_INVALID. */
int bca_step(bca_problem p, int32_t outer_iters, int32_t* iters_done);

/* Iterate until p_r <= tol_p, d_r <= tol_d and b_r <= tol_b (tested every
 * check_every iterations) or max_iters outer iterations in total.
 * *converged = 1 if the tolerances were met.  Errors as bca_step, plus
 * BCA_E_NONFINITE when an iterate became NaN/Inf. */
int bca_solve(bca_problem p, int32_t* iters_done, int32_t* converged);

/* The support T_kappa(z): the kappa largest |z_k| (row norms for softmax), ties
 * to the lower index, ascending.  idx receives kappa int32 (host memory);
 * *count = kappa. */
int bca_get_support(bca_problem p, int32_t* idx, int32_t* count);

/* The model x_hat = z restricted to T_kappa(z), zero elsewhere: n*C doubles
 * (host memory, feature-major). */
int bca_get_coef(bca_problem p, double* x);

/* Residuals of the last outer iteration and its number (0 before any). */
int bca_get_residuals(bca_problem p, double* pr, double* dr, double* br, int32_t* iter);

/* Residual history: up to `cap` rows of (p_r, d_r, b_r), oldest first (host). */
int bca_get_history(bca_problem p, double* hist, int32_t cap, int32_t* count);

/* Objective of the SML problem (Sec. 2) at x_hat, in FP64. */
int bca_get_objective(bca_problem p, double* f);

/* Which state vector bca_get_vector / bca_set_vector address. */
enum {
  BCA_VEC_X = 0,      /* x_i, n*C, per partition */
  BCA_VEC_U = 1,      /* u_i, n*C, per partition */
  BCA_VEC_Z = 2,      /* z, n*C */
  BCA_VEC_S = 3,      /* s, n (rows for softmax) */
  BCA_VEC_OMEGA = 4,  /* omega-bar_i, m_i*C, per partition */
  BCA_VEC_NU = 5,     /* nu_i, m_i*C, per partition */
  BCA_VEC_TV = 6      /* the scalars (t, v): 2 doubles */
};

/* Copy one FP64 state vector to host memory (`part` ignored for global ones). */
int bca_get_vector(bca_problem p, int32_t which, int32_t part, double* out);

/* Overwrite one FP64 state vector from host memory.  After the last set, the
 * next bca_step re-derives the cached block predictions from the new state. */
int bca_set_vector(bca_problem p, int32_t which, int32_t part, const double* in);

/* Checkpoint / resume of the whole ADMM state (x, u, z, s, t, v, omega-bar,
 * nu, iteration count, residual history).  With buf == NULL, *bytes receives
 * the size needed.  Resuming and continuing gives the same bits as an
 * uninterrupted run. */
int bca_get_state(bca_problem p, void* buf, size_t* bytes);
int bca_set_state(bca_problem p, const void* buf, size_t bytes);

/* The cached inverse P_ij = K_ij^-1 of block (part, block) (Sec. 3.1: the
 * matrix of the x_ij-step's regularised least-squares problem, K_ij =
 * rho_l A_ij^T A_ij + (1/(N gamma) + rho_c) I), written dense row-major
 * n_j x n_j to host memory owned by the caller.  It is formed once at finalize
 * in FP64 from the Cholesky factor: P_ij = W_ij^T W_ij with W_ij = L_ij^-1.
 * For tests of the setup: P_ij K_ij = I. */
int bca_get_inverse(bca_problem p, int32_t part, int32_t block, double* Kinv);

/* Kernel timing with HIP events on the problem's stream (off by default).
 * Classes: 0 = A-streaming pass (block matvecs, prox, duals), 1 = block
 * solves, 2 = global step, 3 = Gram, 4 = factorisation. */
enum { BCA_KC_STREAM = 0, BCA_KC_SOLVE = 1, BCA_KC_GLOBAL = 2, BCA_KC_GRAM = 3, BCA_KC_FACTOR = 4 };
int bca_set_timing(bca_problem p, int32_t on);
int bca_get_timing(bca_problem p, int32_t kernel_class, int32_t* launches, double* total_ms);

/* Release all device memory of the handle (NULL is accepted). */
int bca_destroy(bca_problem p);

/* Thread-local message of the last error on this thread ("" if none). */
const char* bca_last_error(void);

/* ---------------------------------------------------------------- batched form
 * Many independent problems (each created, loaded and finalized as above)
 * advanced together in ONE persistent launch on hip_stream: every outer
 * iteration of every problem is Algorithm 2's K_in inner iterations followed by
 * the global step of Algorithm 1, exactly as bca_step computes it (to rounding:
 * the batched streaming pass sums in a different order).  A problem's results do
 * not depend on which other problems share the batch.  Limits: one-class losses
 * (squared, logistic, hinge), FP32 or FP64 storage, n_j <= 1024, n <= 2048 (FP32)
 * or 1024 (FP64).  The launch is cooperative, with a grid that fills every CU, and
 * its grid barriers need all of its workgroups resident: kernels that other
 * streams run at the same time can stall it (a server whose materialiser ran
 * kernels beside it made no progress for minutes), so run nothing else on the
 * device during the call.  The call synchronises hip_stream.
 * Errors: BCA_E_INVALID (a problem outside the limits), BCA_E_STATE (not
 * finalized), BCA_E_NONFINITE (a problem's iterates became NaN/Inf; every problem
 * of the batch has still advanced, and the others' results are valid),
 * BCA_E_DEVICE. */

/* Advance every problem by min(outer_iters, its remaining max_iters) outer iterations. */
int bca_batch_step(bca_problem* probs, int32_t count, int32_t outer_iters, void* hip_stream);

/* Run every problem to its own max_iters. */
int bca_batch_solve(bca_problem* probs, int32_t count, void* hip_stream);

/* bca_batch_step without device allocation, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc): same arguments, kernels and results (bit for bit) as
 * bca_batch_step.  The launch's descriptors, item lists, phase counters and
 * gathered status flags live in a fixed scratch array of 16 MiB in the library's
 * device code (one copy per
 * GPU, held until the process ends); every problem must already hold its batched
 * partial sums, which bca_finalize allocates for every problem within the
 * batched form's limits (bca_batch_set_shape and bca_batch_autotune resize them).
 * Calls in one process are serialised, since they share the scratch array; the
 * array keeps the last call's contents, and what must start at zero is cleared
 * by each call.  Synchronises hip_stream.
 * Errors: as bca_batch_step; BCA_E_INVALID also when the batch needs more than
 * the 16 MiB of scratch (too many problems or items, or too many outer
 * iterations for the phase counters); BCA_E_STATE when a problem lacks its
 * batched partial sums. */
int bca_batch_step_noalloc(bca_problem* probs, int32_t count, int32_t outer_iters, void* hip_stream);

/* Phase tracing of the batched launches (bca_batch_step, bca_batch_solve,
 * bca_batch_step_noalloc; not the autotuner's timing launches).  While on, every
 * launch records when each of its phases ends -- one timestamp per grid barrier,
 * taken by one thread from the GPU's 100 MHz real-time counter -- and the
 * microseconds are summed per phase kind: the re-derivation pass of problems
 * whose partial sums are stale (PRIME), and per inner iteration the right-hand
 * sides (RHS), the symmetric products (SYMV), the x update (XUPD) and the
 * streaming pass (STREAM), and the global steps (GLOBAL).  A phase's time
 * includes the grid barrier that ends it.  Turning tracing on clears the sums.
 * Tracing needs (phases + 1) x 8 more bytes of launch scratch. */
enum { BCA_BP_PRIME = 0, BCA_BP_RHS = 1, BCA_BP_SYMV = 2, BCA_BP_XUPD = 3, BCA_BP_STREAM = 4,
       BCA_BP_GLOBAL = 5, BCA_BP_KINDS = 6 };
int bca_batch_set_tracing(int32_t on);
/* Summed microseconds per phase kind into us[0 .. count - 1] (count <= BCA_BP_KINDS)
 * and the number of traced launches.  Errors: BCA_E_INVALID. */
int bca_batch_get_tracing(double* us, int32_t count, int64_t* launches);

/* Tile-shape autotuner of the batched streaming pass: groups the problems by
 * (storage type, row length, rows per partition), times every candidate shape
 * (rows per wavefront tile 1/2/4, and 8 for rows of at most 64 16-byte chunks,
 * x rows per work item 16/32/64/256/1024; a work item is one wavefront's chunk of rows)
 * on each group with state-preserving streaming passes (the fastest of three), and
 * keeps per group, among the shapes within 3 % of the fastest, the one with the
 * most rows per item, then per tile.  The ADMM state is not modified. */
int bca_batch_autotune(bca_problem* probs, int32_t count, void* hip_stream);

/* Explicit tile shape of a problem in the batched form (rows per wavefront tile
 * 1, 2, 4 or 8 -- 8 only for rows of at most 64 16-byte chunks; rows per work
 * item >= 16) and its current value.  BCA_E_INVALID if no such shape is built. */
int bca_batch_set_shape(bca_problem p, int32_t rows_per_tile, int32_t rows_per_item);
int bca_batch_get_shape(bca_problem p, int32_t* rows_per_tile, int32_t* rows_per_item);

/* ---------------------------------------------------------------- serving form
 * A request loop with continuous batching.  Each request is a complete sparse
 * fit (the problem of Sec. 2 with its own data and parameters) run for its
 * max_iters outer iterations.  A scheduler thread admits queued requests in
 * arrival order while a slot is free and the request's device footprint fits
 * hbm_budget_bytes; a materialiser thread copies each admitted request to the
 * device and factorises it on a stream of its own while the resident requests
 * keep running; the scheduler advances all resident requests together in rounds
 * of round_iters outer iterations (one-class requests in one batched persistent
 * launch, softmax requests with their own kernels on two streams of the server);
 * finished requests are retired between rounds, freeing their slot at once and
 * their memory (for waiting ones) when a releaser thread has freed it.  A request's result does not depend on the other requests it
 * shares rounds with.  Submit/poll/fetch/cancel/stats are thread-safe. */

/* Request states reported by bca_server_poll. */
enum { BCA_REQ_QUEUED = 0, BCA_REQ_RUNNING = 1, BCA_REQ_DONE = 2, BCA_REQ_FAILED = 3,
       BCA_REQ_CANCELLED = 4 };

/* Start a server (its scheduler, materialiser and releaser threads) whose rounds run on
 * hip_stream; the server creates three more non-blocking streams of its own (two
 * for softmax requests, one for materialising).  The batched launch of a round
 * runs alone on the GPU (a cooperative launch that fills every CU), so the
 * caller should not run other kernels on the device while the server is busy.
 * Errors: BCA_E_INVALID (max_slots < 1, round_iters < 1, zero budget),
 * BCA_E_DEVICE (no current device, or a stream could not be created). */
int bca_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t round_iters, void* hip_stream,
                      bca_server* out);

/* Queue a request: params as for bca_create (params->rows read here; flags 0),
 * A[i] and b[i] host pointers of partition i laid out as for bca_set_data with
 * ld = n; both are copied before the call returns.  *ticket identifies the
 * request.  Errors: BCA_E_INVALID, BCA_E_BUDGET (the request alone exceeds the
 * budget). */
int bca_server_submit(bca_server s, const bca_params* params, const void* const* A, const void* const* b,
                      uint64_t* ticket);

/* Current BCA_REQ_* state of a request.  Errors: BCA_E_NOTFOUND. */
int bca_server_poll(bca_server s, uint64_t ticket, int32_t* state);

/* Results of a finished request (host memory, any pointer may be NULL): the
 * support (kappa int32, ascending), x_hat (n*C doubles), the objective and the
 * latency from submit to retirement in seconds.
 * Errors: BCA_E_NOTFOUND, BCA_E_STATE (not finished), BCA_E_CANCELLED,
 * BCA_E_DEVICE (the request failed). */
int bca_server_fetch(bca_server s, uint64_t ticket, int32_t* idx, double* x, double* f, double* lat_s);

/* Cancel a queued or running request; its slot and memory are released at the
 * next round boundary.  Errors: BCA_E_NOTFOUND. */
int bca_server_cancel(bca_server s, uint64_t ticket);

/* Queue length, admitted requests (resident or being materialised), reserved
 * device bytes and rounds run so far. */
int bca_server_stats(bca_server s, int32_t* queued, int32_t* running, double* used_bytes, int64_t* rounds);

/* Wall-clock seconds the server's threads have spent so far, per activity, into
 * seconds[0 .. count-1] (count <= BCA_SRV_TIMES): the rounds' softmax work (issue
 * and wait), their batched launches, retiring finished requests (copying their
 * results out), materialising admitted ones, the materialiser waiting for a
 * batched launch to end, the scheduler waiting for a materialiser call to end, and
 * the releaser freeing retired requests' memory (which waits for the device).
 * Errors: BCA_E_INVALID. */
enum { BCA_SRV_SOFTMAX = 0, BCA_SRV_BATCHED = 1, BCA_SRV_RETIRE = 2, BCA_SRV_MATERIALISE = 3,
       BCA_SRV_MAT_WAIT = 4, BCA_SRV_SCHED_WAIT = 5, BCA_SRV_RELEASE = 6, BCA_SRV_TIMES = 7 };
int bca_server_timing(bca_server s, double* seconds, int32_t count);

/* Stop the scheduler and release every resident request. */
int bca_server_destroy(bca_server s);

/* The top-kappa projection of the s-step (Sec. 3), as a standalone device
 * primitive: idx (device, kappa int32) receives the indices of the kappa
 * largest |z_k| of the device vector z (n values, dtype BCA_F64 or BCA_F32),
 * ties to the lower index, -0 equal to +0, ascending.  NaN inputs are not
 * allowed.  Enqueued on hip_stream; synchronises it. */
int bca_topk(const void* z, int32_t dtype, int64_t n, int32_t kappa, int32_t* idx, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* BCA_H */
