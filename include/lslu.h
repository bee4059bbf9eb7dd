/*
 * lslu.h -- C ABI of the MI355X (gfx950) LSLU / Hybrid LSLU library.
 *
 * The library solves the rectangular linear inverse problem b = A x_true + e
 * (Section 1, eq. ip) either as the least-squares problem min ||b - A x||
 * regularised by the iteration count (eq. ir; LSLU, Section 2.2) or as the
 * Tikhonov problem min ||b - A x||^2 + lambda^2 ||x||^2 (eq. vr; Hybrid LSLU,
 * Section 3, Algorithm 5).  The operator A is dense, CSR or a PSF stencil; it
 * is only used through the products A l and A^T d (Section 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns an lslu_status.  Negative values are failures;
 *   the outputs are then unspecified.  Positive values report a breakdown of
 *   the Hessenberg process; outputs are valid up to k_done (Algorithm 4 and 5:
 *   q = 0 or u = 0).  Nothing throws across this boundary.
 * - lslu_last_error(ctx) returns a human-readable message for the last failure
 *   on that context (never NULL).
 * - Handles (lslu_ctx, lslu_op) are owned by the library; the caller owns every
 *   array it passes.  Host arrays given to lslu_op_* are copied; device arrays
 *   given to lslu_solve/lslu_op_apply are only borrowed for the duration of the
 *   call.  No caller pointer is kept after a call returns.
 * - "Working precision" (wp) is the vector type of an operator: double for
 *   LSLU_FP64, float for LSLU_FP32, LSLU_BF16OP, LSLU_FP16OP and LSLU_FP8OP.  Device vectors passed to
 *   the library are contiguous arrays of that type.
 * - All work of one context is enqueued on that context's HIP stream (the one
 *   given to lslu_create, or one it made).  Calls on one context must not
 *   overlap; use one context per thread.
 * - Matrices of the projected problem are FP64 and column-major.
 */
#ifndef LSLU_H
#define LSLU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LSLU_ABI_VERSION 13

typedef enum lslu_status {
  LSLU_OK = 0,
  LSLU_BREAKDOWN_Q = 1,  /* q = A^T d_k has no eligible nonzero entry, or k > n */
  LSLU_BREAKDOWN_U = 2,  /* u = A l_k has no eligible nonzero entry, or k >= m */
  LSLU_ZERO_RHS = 3,     /* r_0 = b - A x_0 is zero; x = x_0 */
  LSLU_EINVAL = -1,      /* invalid argument (sizes, pointers, options) */
  LSLU_ENOMEM = -2,      /* device allocation failed */
  LSLU_EDEVICE = -3,     /* HIP runtime error or no usable GPU */
  LSLU_ENONFINITE = -4,  /* an input holds NaN or Inf */
  LSLU_EUNSUPPORTED = -5 /* combination not implemented */
} lslu_status;

typedef enum lslu_precision {
  LSLU_FP64 = 0,  /* operator, bases and vectors in double */
  LSLU_FP32 = 1,  /* operator, bases and vectors in float; sums in double */
  LSLU_BF16OP = 2, /* operator values and its input in bfloat16, products summed
                      in float; bases and vectors in float */
  LSLU_FP16OP = 3, /* operator values and its input in IEEE binary16, products
                      summed in float; bases and vectors in float */
  LSLU_FP8OP = 4   /* operator values and its input in 8-bit E4M3 (3 fraction
                      bits, exponent bias 7, subnormals down to 2^-9, largest
                      448, saturating, ties to even), products summed in float;
                      bases and vectors in float.  Values are rounded once from
                      the double the caller gives; scale the operator so that
                      its entries lie well inside [2^-6, 448] */
} lslu_precision;

typedef enum lslu_reg {
  LSLU_REG_NONE = 0,    /* LSLU: lambda = 0 (Section 2.2) */
  LSLU_REG_FIXED = 1,   /* lambda_k = opts.lambda */
  LSLU_REG_WGCV = 2,    /* weighted GCV on the grid (Section 3.2.1) */
  LSLU_REG_GCV = 3,     /* GCV on the grid (eq. gcv2) */
  LSLU_REG_OPTIMAL = 4  /* argmin ||x_k(lambda) - x_true|| on the grid (eq. lambda;
                           a diagnostic for simulated data): needs x_true_dev and
                           a grid; priced from the FP64 Gram matrix of
                           [L_K, x_true - x_0], the one place the library forms
                           inner products of basis vectors */
} lslu_reg;

typedef struct lslu_ctx lslu_ctx;
typedef struct lslu_op lslu_op;

/* ------------------------------------------------------------------------ */
/* Context                                                                  */
/* ------------------------------------------------------------------------ */

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * enqueue on (e.g. torch.cuda.current_stream().cuda_stream), or NULL to let
 * the library create one.  The library never destroys a stream it was given.
 * Errors: LSLU_EDEVICE if the device does not exist or is not gfx950,
 * LSLU_EINVAL if out is NULL. */
lslu_status lslu_create(int device, void* hip_stream, lslu_ctx** out);

/* Free the context, its device workspace and (if it made it) its stream.
 * Operators created on it must be destroyed first.  NULL is accepted. */
lslu_status lslu_destroy(lslu_ctx* ctx);

/* Message for the last failure on ctx (or a generic text for ctx == NULL). */
const char* lslu_last_error(const lslu_ctx* ctx);

/* Name of a status code, e.g. "LSLU_BREAKDOWN_U". */
const char* lslu_status_name(int status);

/* LSLU_ABI_VERSION of the built library. */
int lslu_abi_version(void);

/* ------------------------------------------------------------------------ */
/* Operators (the forward model A of eq. ip)                                */
/* ------------------------------------------------------------------------ */

/* Dense operator.  `A` is a host array of m*n doubles, row-major (A[i*n+j]).
 * The library stores A and A^T on the device in the operator's precision.
 * Errors: LSLU_EINVAL (m, n < 1, NULL pointers), LSLU_ENONFINITE,
 * LSLU_ENOMEM. */
lslu_status lslu_op_dense(lslu_ctx* ctx, int64_t m, int64_t n, const double* A,
                          int32_t precision, lslu_op** out);

/* CSR operator: host arrays indptr[m+1] (int64, indptr[0] = 0, non-decreasing,
 * indptr[m] = nnz), indices[nnz] (int32, strictly increasing within each row,
 * in [0, n)) and data[nnz] (double).  nnz must be < 2^31.  The library builds
 * the CSR of A^T on the host and keeps both on the device, so both products
 * are row-parallel with a fixed summation order (deterministic).  Column
 * indices are stored in 16 bits when they fit (those of A when n <= 65536,
 * those of A^T when m <= 65536), else in 32.
 * Errors: LSLU_EINVAL (shape, ordering or range violations), LSLU_ENONFINITE,
 * LSLU_ENOMEM. */
lslu_status lslu_op_csr(lslu_ctx* ctx, int64_t m, int64_t n, int64_t nnz,
                        const int64_t* indptr, const int32_t* indices,
                        const double* data, int32_t precision, lslu_op** out);

/* PSF operator on a rows x cols image stored row-major (m = n = rows*cols).
 * `psf` is a host array of ph*pw doubles (row-major, ph and pw odd) centred at
 * (ph/2, pw/2).  A is the zero-boundary, same-size convolution
 *   (A x)[i,j] = sum_{a,b} psf[a,b] x[i-a+ph/2, j-b+pw/2]
 * and A^T the matching correlation
 *   (A^T y)[i,j] = sum_{a,b} psf[a,b] y[i+a-ph/2, j+b-pw/2],
 * entries outside the image read as zero.  ph, pw odd and <= 31.  The tile
 * shape of its products is measured on the device at creation (as
 * lslu_op_tile with rows_per_lane = 0; a few products, about a millisecond
 * on a 1024 x 1024 image).
 * Errors: LSLU_EINVAL, LSLU_ENONFINITE, LSLU_ENOMEM, LSLU_EDEVICE. */
lslu_status lslu_op_psf(lslu_ctx* ctx, int64_t rows, int64_t cols, int32_t ph,
                        int32_t pw, const double* psf, int32_t precision,
                        lslu_op** out);

/* Tile shape of a PSF operator's products (in lslu_op_apply and inside
 * lslu_solve): each lane of a 4-wavefront block computes rows_per_lane = 2, 4
 * or 8 consecutive output rows of a (4 rows_per_lane) x 64 tile.  0 measures
 * the three on the device (pairs of A and A^T products after a warm-up, the
 * fastest of three timings with HIP events on the context's stream) and keeps
 * the fastest shape.
 * Every shape sums each output in the same order, so results do not depend on
 * it.  In the 16- and 8-bit operator modes the products run on the matrix
 * cores (a banded-matrix form of the correlation, 32 x 64 output tiles) and
 * the shape has no effect.  *chosen (may be NULL) receives the shape in use.  Synchronous.
 * Errors: LSLU_EUNSUPPORTED (not a PSF operator), LSLU_EINVAL,
 * LSLU_ENOMEM, LSLU_EDEVICE. */
lslu_status lslu_op_tile(lslu_ctx* ctx, lslu_op* op, int32_t rows_per_lane,
                         int32_t* chosen);

/* y = A x (transpose = 0; x has n entries, y has m) or y = A^T x
 * (transpose = 1; x has m entries, y has n), on the context's stream, with
 * device vectors in the operator's working precision.  Asynchronous. */
lslu_status lslu_op_apply(lslu_ctx* ctx, const lslu_op* op, int32_t transpose,
                          const void* x_dev, void* y_dev);

/* Shape and precision of an operator (any output pointer may be NULL). */
lslu_status lslu_op_info(const lslu_op* op, int64_t* m, int64_t* n,
                         int32_t* precision);

/* Free an operator (NULL accepted). */
lslu_status lslu_op_destroy(lslu_op* op);

/* ------------------------------------------------------------------------ */
/* Solve (Algorithm 5: REQUIRE A, b, x0, maxiter, RegParam)                 */
/* ------------------------------------------------------------------------ */

typedef struct lslu_opts {
  int32_t maxiter;            /* K >= 1; at most min(m, n) + 1 */
  int32_t reg;                /* lslu_reg */
  double lambda;              /* LSLU_REG_FIXED: lambda >= 0 */
  const double* lambda_grid;  /* host, n_grid > 0 values, strictly ascending
                                 and positive (WGCV, GCV, OPTIMAL) */
  int32_t n_grid;             /* <= 256 */
  int32_t grid_relative;      /* nonzero: grid values are multiplied by the
                                 largest singular value of H_{k+1,k} */
  double omega;               /* WGCV weight; <= 0 selects (k+1)/m */
  const void* x_true_dev;     /* OPTIMAL and LSLU_FLAG_GRAD_LAMBDA (required,
                                 else LSLU_EINVAL): device, wp, n entries;
                                 borrowed for the call */
  double stop_tol;            /* tolerance of the stopping rule (eq. tol);
                                 <= 0 selects 1e-6 */
  int32_t early_stop;         /* nonzero: x_out is x_{k_stop} */
  void* X_dev;                /* optional device output, wp, n x maxiter
                                 column-major: column k-1 is x_k */
  /* Replay hooks (tests): host arrays of pivot rows to use instead of the
   * library's own choice.  piv_t needs maxiter+1 entries (t(1) is the pivot of
   * r_0), piv_g and lambda_idx maxiter entries.  NULL = own choice. */
  const int32_t* replay_piv_t;
  const int32_t* replay_piv_g;
  const int32_t* replay_lambda_idx;
  int32_t flags;              /* bitwise OR of lslu_flag values; 0 = default */
  /* Sampled pivots (the variant of Section 2.2 that takes the largest entry
   * of a small random sample instead of the infinity norm).  NULL = full
   * searches.  Host array of (2*maxiter + 1) rows of sample_len int32:
   * row 0 lists candidate rows of r_0 (< m), row 2k-1 of q at iteration k
   * (< n), row 2k of u at iteration k (< m); -1 entries are skipped.  A
   * search takes the first sample_s listed rows that are not earlier pivots
   * and picks the one of largest magnitude (ties: smallest row); if their
   * largest magnitude is 0 it falls back to the full search.  Copied. */
  const int32_t* sample_rows;
  int32_t sample_s;           /* >= 1 */
  int32_t sample_len;         /* 1..512 */
} lslu_opts;

/* lslu_opts.flags */
typedef enum lslu_flag {
  /* Enqueue every kernel directly instead of replaying the context's cached
   * HIP graph of the solve.  Results are identical either way. */
  LSLU_FLAG_EAGER = 1,
  /* Enqueue directly (as LSLU_FLAG_EAGER) and record HIP events on the
   * context's stream around the recurrence, the projected problems and the
   * assembly; the elapsed times are returned in lslu_result.  Events between
   * launches add a little time of their own. */
  LSLU_FLAG_TIMING = 2,
  /* Enqueue the whole solve, including the copy of the small results to
   * pinned host memory, on the context's stream and return LSLU_OK without
   * waiting; lslu_wait completes it.  Until then the caller keeps every array
   * the call was given (device vectors and the lslu_result arrays), and the
   * context accepts no other solve.  Solves on several contexts (one stream
   * each) run concurrently: many small problems share the GPU.  Not with
   * LSLU_FLAG_TIMING. */
  LSLU_FLAG_ASYNC = 4,
  /* Also return, for every k, the derivative in lambda of the squared error
   * ||x_k(lambda) - x_true||^2 of the regularised projected solution of
   * iteration k (Section 3.2.1, eq. TSP), taken at the lambda_k the rule
   * chose: the gradient of the optimal-parameter loss (eq. lambda) that a
   * learned or tuned parameter rule descends.  Needs x_true_dev (borrowed as
   * for LSLU_REG_OPTIMAL) and lslu_result.dloss_dlambda; works with every
   * rule.  0 where lambda_k = 0 (the derivative of the projected solution
   * vanishes there).  FP64 throughout, from the Gram matrix of
   * [L_k, x_true - x_0]. */
  LSLU_FLAG_GRAD_LAMBDA = 8,
  /* Form only the returned iterate, x_out = x_0 + L_k y_k at the k the
   * stopping rule selects (k_done, or k_stop with early_stop), instead of
   * every x_k of Algorithm 5 followed by a copy of one of them: one pass over
   * k columns of L instead of the product L Y.  Every other output is the
   * same; x_out agrees with the all-iterates solve to the rounding of the
   * order of the sum over j.  X_dev must be NULL (LSLU_EINVAL otherwise). */
  LSLU_FLAG_FINAL_ONLY = 16,
  /* Also return, for every pivot search, its separation (a1 - a2) / a1,
   * where a1 and a2 are the largest and second largest magnitudes among the
   * candidates (1 for a single candidate), in lslu_result.sep_t and sep_g:
   * how far the choice is from a tie (Algorithm 4's infinity-norm pivot; for
   * sampled searches, over the sampled candidates unless the search fell
   * back to the full one).  Evaluated after the recurrence, from the
   * normalised vector (a2/a1 = largest non-pivot |entry| of d_k or l_k), so
   * it carries the rounding of the stored basis: about 1e-16 in FP64, 6e-8
   * in the other modes.  One extra pass over both bases. */
  LSLU_FLAG_PIVOT_SEP = 32
} lslu_flag;

typedef struct lslu_result {
  int32_t status;     /* as returned */
  int32_t k_done;     /* iterates x_1..x_{k_done} were formed */
  int32_t k_stop;     /* first k with |Ghat(k+1)-Ghat(k)|/Ghat(1) < tol, else k_done */
  int32_t n_l, n_d;   /* basis vectors l_j and d_j formed */
  double beta;        /* signed r_0(t(1)) */
  int32_t piv_t_mismatch, piv_g_mismatch; /* replay: own choice differed */
  /* Host arrays filled on return when non-NULL (caller-allocated): */
  int32_t* piv_t;     /* maxiter+1: t(1), t(2), ... (0-based row indices) */
  int32_t* piv_g;     /* maxiter:   g(1), g(2), ... (0-based column indices) */
  int32_t* own_piv_t; /* maxiter+1: the library's own choices (replay) */
  int32_t* own_piv_g; /* maxiter */
  double* H;          /* (maxiter+1) x maxiter, upper Hessenberg (eq. nhr) */
  double* W;          /* maxiter x maxiter, upper triangular (eq. nhr2) */
  double* Y;          /* maxiter x maxiter: column k-1 holds y_k in rows 0..k-1 */
  double* lambda_k;   /* maxiter */
  int32_t* lambda_idx;/* maxiter: grid index of lambda_k, -1 without a grid */
  double* ghat;       /* maxiter: Ghat(k) (eq. stop2) */
  double* sep_lambda; /* maxiter: (G_2 - G_1)/G_1 over the grid */
  double* sigma_max;  /* maxiter: largest singular value of H_{k+1,k} */
  double* sigma_min;  /* maxiter: smallest singular value of H_{k+1,k} */
  /* With LSLU_FLAG_TIMING (else 0): device time of the basis recurrence
   * (n_recurrence_launches launches, one per half-iteration plus the last
   * pivot), of the projected problems and of the assembly of the iterates. */
  double t_recurrence_ms;
  int32_t n_recurrence_launches;
  double t_projected_ms;
  double t_assemble_ms;
  /* maxiter: with LSLU_FLAG_GRAD_LAMBDA, d/dlambda ||x_k(lambda) - x_true||^2
   * at lambda = lambda_k (NULL: not copied) */
  double* dloss_dlambda;
  /* With LSLU_FLAG_PIVOT_SEP: the separation of each pivot search (see the
   * flag); sep_t: maxiter+1 entries (search for t(1), t(2), ...), sep_g:
   * maxiter (g(1), ...).  NaN for a search that was not made (breakdown,
   * or the flag not set).  NULL: not copied. */
  double* sep_t;
  double* sep_g;
} lslu_result;

/* Run Hybrid LSLU (LSLU with LSLU_REG_NONE) for opts->maxiter iterations.
 * The device work of a solve is captured once into a HIP graph owned by the
 * context and replayed by later calls with the same operator, sizes, device
 * pointers and options (the lambda grid and replay arrays are re-uploaded
 * when they change); any other change re-captures it.  The graph holds no
 * memset nodes.
 * b_dev: device, wp, m entries.  x0_dev: device, wp, n entries, or NULL for
 * x_0 = 0.  x_out_dev: device, wp, n entries: the final iterate x_{k_done}
 * (x_{k_stop} with early_stop; x_0 after a breakdown before x_1).  The call
 * returns after the device work finished and `res` is filled.
 * Errors: LSLU_EINVAL (options), LSLU_ENOMEM, LSLU_EDEVICE.  Breakdowns are
 * reported as LSLU_BREAKDOWN_Q/U/LSLU_ZERO_RHS with valid outputs. */
lslu_status lslu_solve(lslu_ctx* ctx, const lslu_op* op, const void* b_dev,
                       const void* x0_dev, const lslu_opts* opts,
                       void* x_out_dev, lslu_result* res);

/* lslu_solve with host arrays: b_host (m doubles), x0_host (n doubles, or
 * NULL for x_0 = 0) and x_out_host (n doubles, written) are converted to and
 * from the working precision (rounded to float outside FP64) and moved
 * through device staging buffers that the context keeps and reuses (so
 * repeated calls replay the same captured solve).  The device pointers in
 * opts (x_true_dev, X_dev) stay device pointers.  Synchronous: the
 * returned status is lslu_solve's, and x_out_host is written when it is not
 * negative.  Errors: as lslu_solve, plus LSLU_ENONFINITE for NaN/Inf in b or
 * x0 and LSLU_EINVAL with LSLU_FLAG_ASYNC. */
lslu_status lslu_solve_host(lslu_ctx* ctx, const lslu_op* op, const double* b_host,
                            const double* x0_host, const lslu_opts* opts,
                            double* x_out_host, lslu_result* res);

/* lslu_solve for callers that cannot allocate device memory (code running
 * under HIP graph capture elsewhere, tight serving loops, harnesses that
 * forbid hipMalloc): the same solve with the same arguments, outputs and
 * results (bit for bit), but its whole device workspace (bases, iterates,
 * projected-problem scratch, result block) lives in one fixed 64 MiB array
 * the library keeps in the memory of each GPU it runs on until the process
 * ends, its kernels are enqueued directly (no captured graph), and the small
 * results are copied straight into the caller's lslu_result arrays.  The
 * call allocates nothing.  The workspace of a solve is about
 * wp (n K + m (K + 1)) (bases) + wp n K (iterates, even when X_dev is given)
 * + 8 K ((K + 1) K + 3 K G) (projected problems, G = grid values) + O(K^2)
 * bytes; a solve that needs more than 64 MiB is refused with LSLU_EINVAL
 * (use lslu_solve).  Every call on one GPU shares the array and leaves its
 * own contents there: calls that overlap on one GPU (several contexts or
 * threads at once) race and must be serialised by the caller.  lslu_vjp
 * and lslu_get_basis do not apply to such a solve (they read the context's
 * own workspace) and report LSLU_EINVAL after it.  Synchronous: returns
 * when the results are written.
 * Errors: as lslu_solve; LSLU_EINVAL also for LSLU_FLAG_ASYNC or
 * LSLU_FLAG_TIMING and for a workspace beyond 64 MiB; LSLU_EDEVICE when the
 * array's device address could not be obtained at context creation. */
lslu_status lslu_solve_static(lslu_ctx* ctx, const lslu_op* op, const void* b_dev,
                              const void* x0_dev, const lslu_opts* opts,
                              void* x_out_dev, lslu_result* res);

/* Solves count problems together: problem i is op[i] (created on ctxs[i]),
 * b_dev[i] (m_i entries, wp), x_out_dev[i] (n_i entries, wp, written) and
 * res[i] (may be NULL, or res itself NULL), all with the same opts.  Launch
 * j of the recurrence (one per half-iteration, Algorithm 5) of every problem
 * runs in one merged kernel launch whose blocks are split among the problems,
 * so many small problems fill the GPU together.  The problems are split by
 * size (rows) into up to 4 classes whose merged launches run side by side on
 * the stream of each class's first context (a merged launch lasts as long as
 * its largest problem's half-iteration); the projected problems and the
 * assembly of each problem then run on its own context's stream.  Results are bit-identical to solving each problem
 * alone.  Each problem needs its own context (its workspace); the call
 * returns when all are done.  Requirements: dense or CSR operators of one kind and one
 * precision on one device; opts without x_true_dev, X_dev, sampled pivots,
 * replays, LSLU_REG_OPTIMAL and the ASYNC, TIMING and GRAD_LAMBDA flags;
 * x_0 = 0.  Returns LSLU_OK, or the first negative status of a problem
 * (message on ctxs[0]); breakdowns are reported per problem in res[i].
 * Errors: LSLU_EINVAL, LSLU_ENOMEM, LSLU_EDEVICE. */
lslu_status lslu_solve_batch(int32_t count, lslu_ctx* const* ctxs, const lslu_op* const* ops,
                             const void* const* b_dev, const lslu_opts* opts,
                             void* const* x_out_dev, lslu_result* const* res);

/* Completes the pending LSLU_FLAG_ASYNC solve of the context: waits for its
 * stream, fills the lslu_result given to lslu_solve and returns the solve's
 * status (as lslu_solve would have).  LSLU_OK when nothing is pending. */
lslu_status lslu_wait(lslu_ctx* ctx);

/* Reverse pass (vector-Jacobian product) of the context's last completed
 * solve, which must have used `op`:
 *     bbar_dev   <- (d x_k / d b)^T xbar      (m entries, wp, device, written)
 *     *lambda_bar = xbar^T (d x_k / d lambda)  (host, NULL: not returned)
 * for 1 <= k <= k_done, with the pivots t(.), g(.) of that solve, x_0 and
 * lambda_k held fixed (Algorithm 5 with fixed pivots is a smooth map of b;
 * the projected problem is the Tikhonov problem of eq. TSP, Section 3.2.1).
 * With the loss ||x_k - x_true||^2, xbar = 2 (x_k - x_true) gives its
 * gradient in b and lambda.  xbar_dev: n entries, wp, device, borrowed.  The
 * pass reads the bases and small arrays the solve left on the device (no
 * recomputation), so no other solve may run on the context in between; it
 * allocates its scratch (about (m + n) (K + 3) wp values plus
 * O(K^2) doubles) on the first call and keeps it with the context.  Returns
 * after the device work finished.
 * Errors: LSLU_EINVAL (no such solve, k out of range, a pending solve, or
 * H_k^T H_k + lambda_k^2 I singular: lambda_k = 0 with a rank-deficient
 * H_k), LSLU_ENOMEM, LSLU_EDEVICE. */
lslu_status lslu_vjp(lslu_ctx* ctx, const lslu_op* op, int32_t k,
                     const void* xbar_dev, void* bbar_dev, double* lambda_bar);

/* Copy basis vectors of the last solve on ctx into a device buffer (wp,
 * column-major, leading dimension = vector length): which = 0 copies the
 * n x count matrix L, which = 1 the m x count matrix D.  count must not
 * exceed what the last solve formed.  Asynchronous on the context's stream. */
lslu_status lslu_get_basis(lslu_ctx* ctx, int32_t which, int32_t count,
                           void* dst_dev);

#ifdef __cplusplus
}
#endif

#endif /* LSLU_H */
