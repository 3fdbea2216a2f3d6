/*
 * alsncg.h -- C ABI of the MI355X (gfx950) ALS / ALS-NCG hot path.
 *
 * Method: Winlaw, Hynes, Caterini, De Sterck, "Algorithmic Acceleration of
 * Parallel ALS for Collaborative Filtering" (arXiv:1508.03110).  Section
 * II defines the loss (Eq. (1)); Section III-A the ALS row solves (Eq. (3),
 * Eq. (4), Algorithm 1); Section III-B ALS-NCG (Eq. (5), Eq. (8),
 * Algorithm 2); Section V-C the one-pass quartic line search (Algorithm 4)
 * and the gradient.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every array argument is a DEVICE pointer owned by the caller unless a
 *    parameter name ends in _host.  The library never frees, and never
 *    keeps, a caller pointer after the call returns.
 *  - Every compute call is asynchronous and stream-ordered on `stream` (a
 *    hipStream_t passed as void*; NULL = the default stream).  Outputs are
 *    valid once the stream has been synchronised.  Argument errors are
 *    detected on the host before anything is enqueued and reported through
 *    the return code; nothing is thrown across the ABI and nothing aborts.
 *  - A context holds workspace and is not thread-safe: use one context per
 *    host thread / stream.  Calls on one context must be issued on one stream
 *    (its workspace is reused call after call).
 *  - Factors are row-major: U is [n_u, ld], M is [n_m, ld], ld >= n_f; row i
 *    holds the n_f latent factors of user (or item) i (the paper's n_f x n
 *    column-per-entity matrices, same memory image).  Padding columns
 *    n_f..ld-1 are never read and never written.
 *  - The concatenated unknown x of Eq. (5) is one buffer [U; M] of
 *    n_u*ld + n_m*ld elements, so U = x and M = x + n_u*ld.
 *  - Ratings: one orientation of R as CSR (int64 indptr [n_rows+1], int32
 *    column ids [nnz], float values [nnz]); the item orientation is the CSR
 *    of R^T.  Column ids inside a row must be distinct.  Rating values are
 *    FP32 in every path (half-stars are exact); the FP64 path widens them.
 *  - Regularisation is always the paper's count-weighted lambda * n_i of
 *    Eq. (1) (n_i = number of ratings of row i); lambda >= 0.
 *  - Element type of factor and vector arguments is selected by `dt`:
 *    ALS_F64 (double), ALS_F32 (float).  ALS_BF16 (bfloat16, stored as
 *    16-bit words) appears only in the reduced-precision calls
 *    als_sweep_mixed / als_to_bf16.
 */
#ifndef ALSNCG_H
#define ALSNCG_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define ALS_API __attribute__((visibility("default")))
#else
#define ALS_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { ALS_F64 = 0, ALS_F32 = 1, ALS_BF16 = 2 } als_dtype;

typedef enum {
    ALS_OK = 0,
    ALS_E_INVAL = -1,      /* bad argument (NULL pointer, size, unsupported n_f / dtype) */
    ALS_E_HIP = -2,        /* a HIP runtime call failed */
    ALS_E_NOT_SPD = -3,    /* a row's normal equations were not positive definite */
    ALS_E_NONFINITE = -4,  /* reserved */
    ALS_E_NOMEM = -5,      /* device allocation failed */
    ALS_E_BUDGET = -6      /* request larger than the stated limit */
} als_status;

typedef struct als_ctx als_ctx;
typedef struct als_plan als_plan;

/* One orientation of the ratings matrix (device arrays). */
typedef struct {
    int64_t n_rows;          /* rows of this orientation (users for R, items for R^T) */
    int64_t n_cols;          /* columns (items for R, users for R^T) */
    int64_t nnz;             /* number of ratings */
    const int64_t *indptr;   /* device [n_rows + 1], indptr[0] = 0, non-decreasing */
    const int32_t *indices;  /* device [nnz], column ids in [0, n_cols), distinct per row */
    const float *values;     /* device [nnz], ratings */
} als_csr;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  Returns ALS_OK and *out, or an
 * error code with *out = NULL. */
ALS_API int als_ctx_create(als_ctx **out, int device);
/* Release the context and its workspace (synchronises the device first).
 * NULL is ignored. */
ALS_API void als_ctx_destroy(als_ctx *ctx);
/* Text of a status code (static storage). */
ALS_API const char *als_strerror(int status);
/* Bytes of device workspace currently held by the context. */
ALS_API size_t als_ctx_workspace_bytes(const als_ctx *ctx);

/* ---------------------------------------------------------------- row plan
 *
 * Work decomposition of one orientation of R, built once before the
 * iteration loop (the ratings are static, as the paper's routing tables are,
 * Section V-B): rows are cut into chunks of at most `chunk` ratings, chunks
 * are ordered longest first, and rows longer than `chunk` are marked for a
 * split-K second stage with a fixed-order reduction (results do not depend
 * on scheduling).  chunk = 0 picks a size from the matrix shape:
 * nnz / (8 x compute units), at least 256 and at most 8192 ratings (bounding
 * the length of each FP32 MFMA accumulation; longer rows are split).  The call
 * copies R->indptr to the host (it synchronises the device) and allocates
 * the plan's device arrays; the plan stays valid until als_plan_destroy and
 * may only be used with a CSR of the same indptr.
 */
ALS_API int als_plan_create(als_ctx *ctx, const als_csr *R, int64_t chunk, als_plan **out);
ALS_API void als_plan_destroy(als_plan *plan);
/* Launch shape of the chunk kernels that use this plan, for the half-sweep
 * (sweep_grid) and for the gradient and coefficient passes (pass_grid):
 * 0 (default) launches one 64-lane workgroup per chunk; > 0 launches
 * min(grid, chunks) persistent workgroups that stride over the chunks
 * (longest first).  Results do not depend on it (every chunk writes its own
 * partials).  Used by the tuner. */
ALS_API int als_plan_set_grid(als_plan *plan, int64_t sweep_grid, int64_t pass_grid);
/* Plan statistics: out[0]=n_rows, [1]=nnz, [2]=n_chunks, [3]=split rows,
 * [4]=split chunks, [5]=chunk size, [6]=longest row, [7]=rows in the
 * dual-form bins. */
ALS_API int als_plan_info(const als_plan *plan, int64_t out[8]);
/* Length bins of the half-sweep (Eq. (3)): rows with 1 <= n_i <= max_len
 * ratings (max_len <= 94; capped at the plan's chunk size so that they are
 * whole rows) are solved by als_sweep in the dual form
 *     x_i = Y_I^T (Y_I Y_I^T + lambda n_i I)^{-1} r_i,
 * an n_i x n_i system instead of n_f x n_f, which for lambda > 0 is the same
 * solution (push-through identity (A^T A + c I)^{-1} A^T = A^T (A A^T + c I)^{-1}).
 * The rows are binned by ceil((n_i + 2) / 16), the number of 16-wide tiles
 * of their system (one kernel instance per bin); the others keep the
 * n_f x n_f form.  max_len = 0 (the default) turns the bins off; with
 * lambda = 0 als_sweep ignores them (the primal system is then singular for
 * n_i < n_f and is reported as not positive definite).  Reorders the
 * plan's chunks on the host and device (synchronises the device first);
 * results of every other call do not depend on the order.  Used by the tuner. */
ALS_API int als_plan_set_dual(als_plan *plan, int64_t max_len);
/* FP32 half-sweep of this plan (Eq. (3)/(4)) over a split copy of the fixed
 * side: als_sweep first writes, once per call, the two-term FP16 split of
 * every row of Y (the values its Gram loop otherwise forms for every
 * gathered rating) into a context-owned device buffer (grown as needed,
 * like the workspace; calls on one context that overlap on different
 * streams race on it), and the Gram loop gathers the split rows: fewer
 * instructions per rating, rows of 64 * ceil(NB / 4) * 4 bytes with
 * NB = ceil((n_f + 1) / 16) instead of 4 ld.  Results are bitwise the same
 * either way.  mode 1: on; 0: off; -1 (default): on when the split rows are
 * no wider than the factor rows.  Not used for the dual-form bins, for FP64,
 * for fold-in or the server, or when the copy would exceed 4 GiB.  Used by
 * the tuner. */
ALS_API int als_plan_set_split_copy(als_plan *plan, int mode);
/* Plan of R for the gradient pass (Section V-C "Gradient Evaluation": the
 * per-rating terms of a row summed over the row's ratings) with each row cut
 * at n_slices column-slice boundaries, chosen so that every slice holds about
 * nnz / n_slices ratings.  Every non-empty segment of a row is a piece of its
 * own (segments longer than `chunk` are cut further, chunk = 0 as in
 * als_plan_create), summed by the fixed-order split stage.  Pieces are laid
 * out so that, with one workgroup per piece and workgroups handed to the
 * device's 8 accelerator dies in turn, slice s runs on die s mod 8, slices
 * s and s + 8 one after the other: each die then gathers rows of the other
 * factor from one slice at a time, a table 8 / n_slices of the whole, which
 * its own L2 can hold.  Slots of the layout that a slice does not fill are
 * empty pieces.  Requires ascending column ids within every row (checked);
 * copies R->indptr and R->indices to the host (synchronises the device).
 * n_slices in [1, 4096].  Accepted as plan_R or plan_Rt by ncg_gradient
 * only (ALS_E_INVAL elsewhere, and from als_plan_set_dual); results agree
 * with those of an als_plan_create plan to rounding (another summation
 * order), and are bitwise reproducible for a given plan. */
ALS_API int als_plan_create_sliced(als_ctx *ctx, const als_csr *R, int64_t chunk, int64_t n_slices,
                                   als_plan **out);

/* ---------------------------------------------------------------- hot path */

/*
 * ALS half-sweep, Eq. (3) (Eq. (4) when R is the CSR of R^T; Algorithm 1
 * runs one half-sweep per orientation).  For every row i of R with n_i > 0:
 *     A_i = sum_{j in I_i} y_j y_j^T + lambda n_i I,   v_i = sum_{j in I_i} r_ij y_j,
 *     X[i] = A_i^{-1} v_i   (Cholesky factorisation, Section V-B),
 * where y_j = Y[j] is a row of the fixed factor Y [R->n_cols, ld].  Rows with
 * n_i = 0 get X[i] = 0.  X [R->n_rows, ld] is overwritten.
 *   grad_out (may be NULL): [R->n_rows, ld]; receives 2 (A_i x_i - v_i)
 *     with x_i = X_at[i], i.e. the gradient block of Eq. (1) for the rows of
 *     R at the point (X_at, Y) (Section V-C), taken from the same Gram
 *     matrices at no extra pass.  X_at (may be NULL: the contents of X before
 *     this call) is [R->n_rows, ld] and may not overlap grad_out.  Rows with
 *     n_i = 0 get 0.
 *   bad_row (may be NULL): device int64; set to the smallest row whose A_i
 *     was not numerically SPD, or INT64_MAX when every row was SPD.  Such
 *     rows are written as NaN.
 * n_f: 1..143 for ALS_F32, 1..95 for ALS_F64.  Y and X must not overlap.
 */
ALS_API int als_sweep(als_ctx *ctx, const als_plan *plan, const als_csr *R, const void *Y, void *X,
                      int n_f, int ld, double lambda, als_dtype dt, const void *X_at,
                      void *grad_out, int64_t *bad_row, void *stream);

/*
 * Reduced-precision ALS half-sweep: the row solve of Eq. (3) (Eq. (4) for
 * R^T) with the fixed factor read from a BF16 copy.  For every row i:
 *     A~_i = sum_j y~_j y~_j^T + lambda n_i I,  v~_i = sum_j bf16(r_ij) y~_j,
 *     x0 = A~_i^{-1} v~_i        (y~_j = Y16[j]; Gram on BF16 MFMA with FP32
 *                                 accumulation, Cholesky and solves in FP32)
 * and, when refine != 0, one step of iterative refinement with the residual
 * of the FP32 normal equations (y_j = Y32[j], FP32 ratings):
 *     x1 = x0 + A~_i^{-1} ( sum_j (r_ij - y_j . x0) y_j - lambda n_i x0 ).
 * The result is written to X32 [R->n_rows, ld] (float) and, when X16 is not
 * NULL, rounded to nearest even into X16 [R->n_rows, ld] (bfloat16 words).
 *   Y16: [R->n_cols, ld] bfloat16 words (the BF16 copy of the fixed factor);
 *   Y32: [R->n_cols, ld] float, the same factor in FP32 (required when
 *        refine != 0, else may be NULL).
 *   bad_row: as in als_sweep.  Rows with n_i = 0 get 0.
 * Loads are 16-byte vectors when ld is a multiple of 8 and Y16 is 16-byte
 * aligned (element loads otherwise).  n_f: 1..143.  A plan is required.  The
 * outputs must not overlap the inputs.
 */
ALS_API int als_sweep_mixed(als_ctx *ctx, const als_plan *plan, const als_csr *R, const void *Y16,
                            const float *Y32, float *X32, void *X16, int n_f, int ld,
                            double lambda, int refine, int64_t *bad_row, void *stream);

/* y[k] = bf16(x[k]) (round to nearest even) for k < n; x float, y bfloat16
 * words; the BF16 copy of a factor read by als_sweep_mixed. */
ALS_API int als_to_bf16(als_ctx *ctx, int64_t n, const float *x, void *y, void *stream);

/*
 * Gradient of Eq. (1) (Section III-A; Section V-C, gradient evaluation):
 *   g_ui = 2 lambda n_ui u_i + 2 sum_{j in I_i} m_j (u_i^T m_j - r_ij),
 *   g_mj = 2 lambda n_mj m_j + 2 sum_{i in I_j} u_i (u_i^T m_j - r_ij),
 * by one pass over R (U block) and one over R^T (M block).  gU [n_u, ld] /
 * gM [n_m, ld] may each be NULL to skip that block.  out2 (device double
 * [2], may be NULL): out2[0] = f(U, M) of Eq. (1), out2[1] = ||gU||^2 +
 * ||gM||^2 over the blocks requested; both reduced in FP64 in a fixed order.
 * When out2 is given both passes run (f needs the data term of the R pass
 * and the item regulariser of the R^T pass) even if gU or gM is NULL.
 */
ALS_API int ncg_gradient(als_ctx *ctx, const als_plan *plan_R, const als_csr *R, const als_plan *plan_Rt,
                 const als_csr *Rt, const void *U, const void *M, int n_f, int ld, double lambda,
                 als_dtype dt, void *gU, void *gM, double *out2, void *stream);

/*
 * Coefficients of the line-search quartic (Section V-C): with
 * u_i = U[i] + alpha pU[i] and m_j = M[j] + alpha pM[j],
 *     f(x + alpha p) = sum_{n=0..4} coeffs[n] alpha^n,
 * computed in ONE pass over the ratings of R (user-major, gathering the item
 * side), per-rating dot products in the factor type and all accumulation in
 * FP64 (fixed reduction order).  coeffs: device double [5].  The item
 * regulariser needs the item counts n_mj, taken from Rt->indptr (Rt is the
 * CSR of R^T; only its indptr is read).  coeffs[1] equals g^T p.
 */
ALS_API int linesearch_coeffs(als_ctx *ctx, const als_plan *plan_R, const als_csr *R, const als_csr *Rt,
                      const void *U, const void *M, const void *pU, const void *pM, int n_f,
                      int ld, double lambda, als_dtype dt, double *coeffs, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same
 * coefficients as linesearch_coeffs, from the same kernels in the same order
 * (bitwise equal results), with the per-chunk partial sums kept in a fixed
 * scratch array of 2^22 doubles (32 MiB) that the library holds on every
 * device it runs on until the process ends; no device memory is allocated
 * or freed.  Plans of more than linesearch_coeffs_noalloc_max_chunks() chunks
 * are refused with ALS_E_BUDGET (nothing is launched).  Every call on one
 * device shares that device's array and the last call leaves its contents
 * there: calls that overlap on one device (different streams, or different
 * contexts on one device) race and must be ordered by the caller.  Other
 * arguments, outputs and errors as linesearch_coeffs.
 */
ALS_API int linesearch_coeffs_noalloc(als_ctx *ctx, const als_plan *plan_R, const als_csr *R,
                                      const als_csr *Rt, const void *U, const void *M,
                                      const void *pU, const void *pM, int n_f, int ld,
                                      double lambda, als_dtype dt, double *coeffs, void *stream);

/* Largest plan (in row chunks) that linesearch_coeffs_noalloc accepts. */
ALS_API size_t linesearch_coeffs_noalloc_max_chunks(void);

/*
 * Exact line search on the same quartic (a stronger search than Algorithm 4,
 * like the one the paper's serial runs use): alpha_out = the global minimiser
 * over alpha > 0 of Q(alpha) = sum coeffs[n] alpha^n, from the real roots of
 * Q' (bracketed by the roots of Q'', bisected to full FP64 precision), kept
 * when it passes the sufficient-decrease test of Algorithm 4 with constant c.
 * trials_out (device int32, may be NULL): 0, or -1 (alpha_out = 0) when
 * coeffs[1] >= 0, Q has no minimiser on alpha > 0, or the test fails.
 * q_out (device double, may be NULL): Q(alpha_out) = f(x + alpha p) by
 * Horner's rule, no fused multiply-adds; NaN on failure.
 */
ALS_API int ncg_linesearch_exact(als_ctx *ctx, const double *coeffs, double c, double *alpha_out,
                                 int32_t *trials_out, double *q_out, void *stream);

/*
 * Backtracking line search, Algorithm 4, evaluated on the device from the
 * quartic coefficients (no data pass): alpha = alpha0 tau^n for the first
 * n = 0, 1, ..., max_trials-1 with
 *     (1 - c) C1 + alpha (C2 + alpha (C3 + alpha C4)) <= 0,
 * which is f(x + alpha p) - f(x) <= alpha c g^T p divided by alpha > 0.
 * alpha_out (device double): the step, or 0 when no trial passed or C1 >= 0
 * (not a descent direction); trials_out (device int32, may be NULL): n, or
 * -1 on failure.  q_out (device double, may be NULL): Q(alpha) = f(x +
 * alpha p) of the accepted step by Horner's rule, no fused multiply-adds;
 * NaN on failure.  Section V-C uses tau = 0.9, c = 0.5, alpha0 = 10.
 */
ALS_API int ncg_backtrack(als_ctx *ctx, const double *coeffs, double alpha0, double tau, double c,
                  int max_trials, double *alpha_out, int32_t *trials_out, double *q_out,
                  void *stream);

/*
 * x <- x + alpha p over n elements, alpha read from device memory (Algorithm
 * 2, x_{k+1} = x_k + alpha_k p_k).  The FP32 path forms x + alpha p in FP64
 * and rounds once.
 */
ALS_API int ncg_axpy(als_ctx *ctx, int64_t n, void *x, const void *p, const double *alpha, als_dtype dt,
             void *stream);

/*
 * y <- a x + b y over n elements with host scalars a, b (FP64 arithmetic,
 * one rounding).  Used by Algorithm 2's restarts: p = -gbar (a = -1, b = 0)
 * and the ALS step x = x - gbar = P(x) (a = -1, b = 1).  With b = 0 the old
 * contents of y are not read.
 */
ALS_API int ncg_axpby(als_ctx *ctx, int64_t n, double a, const void *x, double b, void *y,
                      als_dtype dt, void *stream);

/*
 * Preconditioned direction update of Algorithm 2 with beta of Eq. (8), over
 * the flat vectors of Eq. (5) (n elements each):
 *     gbar_new = x - xbar                 (xbar = P(x), one ALS iteration)
 *     beta     = gbar_new^T (g_new - g_old) / den     (den = gbar_old^T g_old)
 *     p        <- -gbar_new + beta p
 * and the FP64 scalars scal (device double [4], read and written):
 *     in : scal[0] = den of the previous iteration
 *     out: scal[0] = gbar_new^T g_new (the next den), scal[1] = beta,
 *          scal[2] = ||g_new||^2, scal[3] = gbar_new^T (g_new - g_old).
 * beta is 0 when restart != 0 (p = -gbar_new, the start p_0 = -gbar_0 of
 * Algorithm 2), when den is 0 or not finite, or when beta is not finite;
 * pr_plus != 0 clamps beta at 0.  g_old may be NULL when restart != 0.
 * xbar is overwritten with gbar_new.
 */
ALS_API int ncg_direction(als_ctx *ctx, int64_t n, const void *x, void *xbar, const void *g_new,
                  const void *g_old, void *p, double *scal, int restart, int pr_plus,
                  als_dtype dt, void *stream);

/*
 * Fold-in: a batch of n_req new users, each solved against the FIXED item
 * factors M [n_items, ld] by the row solve of Eq. (3):
 *     U_out[q] = (M_I^T M_I + lambda n_q I)^{-1} M_I^T r_q,
 * for request q with ratings (req_items, req_vals)[req_indptr[q] ..
 * req_indptr[q+1]) (device arrays).  Each request is independent: its result
 * does not depend on the other requests in the batch.  req_status (device
 * int32 [n_req], may be NULL): 0, ALS_E_INVAL for an empty request (output
 * 0), ALS_E_NOT_SPD (output NaN).  One wavefront solves one request.
 */
ALS_API int fold_in(als_ctx *ctx, const void *M, int64_t n_items, int n_f, int ld, double lambda,
            als_dtype dt, int64_t n_req, const int64_t *req_indptr, const int32_t *req_items,
            const float *req_vals, void *U_out, int32_t *req_status, void *stream);

/* ---------------------------------------------------------------- device-side step control
 *
 * The two calls below run one step of Algorithm 2 with every decision taken
 * on the device, so that a whole iteration is a fixed sequence of launches
 * with no host read (it may be captured as one HIP graph).
 */

/*
 * Line search and update of Algorithm 2 (Section V-C, Algorithm 4) with the
 * restart and ALS-point safeguards, on the flat vectors x, p of Eq. (5)
 * ([U; M] with U = x, M = x + R->n_rows * ld):
 *   1. C = coefficients of f(x + alpha p) (one pass, as linesearch_coeffs);
 *      alpha by backtracking (search = 0: alpha0, tau, c, max_trials as
 *      ncg_backtrack) or by the exact minimiser (search = 1: as
 *      ncg_linesearch_exact; alpha0, tau, max_trials unused);
 *   2. if C1 >= 0 or no trial passed: p = -gbar and step 1 again (restart);
 *   3. if that fails too: the ALS point x = x - gbar (= x + p) is taken
 *      (safeguard; the next direction must restart), else x = x + alpha p.
 * gbar: the preconditioned gradient x - P(x) (what ncg_direction leaves in
 * its xbar argument).  state: device double[32], caller-owned, zeroed before
 * the first step; after the call
 *   state[16..20] accepted C0..C4, [21] step applied (alpha, or 1 for the ALS
 *   point), [22] trials (-1 after a safeguard), [23] 1 if p was restarted,
 *   [24] 1 if the ALS point was taken, [25] f(x_new) = Q(alpha) (NaN after a
 *   safeguard), [26] restarts so far, [27] safeguards so far, [28] steps so far;
 *   [0..15] hold the two coefficient sets and trial results.
 * The second coefficient pass is launched in every case and returns at once
 * unless the restart flag is set.  Errors as linesearch_coeffs.
 */
ALS_API int ncg_linesearch_step(als_ctx *ctx, const als_plan *plan_R, const als_csr *R,
                                const als_csr *Rt, void *x, void *p, const void *gbar, int n_f,
                                int ld, double lambda, als_dtype dt, int search, double alpha0,
                                double tau, double c, int max_trials, double *state, void *stream);

/*
 * ncg_direction with the restart decided on the device: beta = 0 when
 * *restart_flag != 0 (device double, e.g. state + 24 of ncg_linesearch_step),
 * else Eq. (8).  g_old must be valid.  Same outputs as ncg_direction.
 */
ALS_API int ncg_direction_dev(als_ctx *ctx, int64_t n, const void *x, void *xbar,
                              const void *g_new, const void *g_old, void *p, double *scal,
                              const double *restart_flag, int pr_plus, als_dtype dt, void *stream);

/* ---------------------------------------------------------------- ranking accuracy
 *
 * Section IV measures how close a solution is to the converged one by the
 * top-t rankings of every user: a modified Kendall tau distance counts the
 * adjacent swaps that bring the converged solution's top t items, in order,
 * to the front of the current ranking, normalised by its largest value.
 *
 * A user's ranking lists all items by decreasing predicted rating
 * U[i] . M[j], formed in FP64 (FP32 factors are widened), equal ratings by
 * increasing item id.  U: [n_u, ld], M: [n_m, ld] (device, element type dt =
 * ALS_F32 or ALS_F64); 1 <= n_f <= 128, ld >= n_f; 1 <= t <= 32, t <= n_m.
 * Factors must be finite.
 */

/* top (device int32 [n_u, t], row-major, caller-owned): the first t items of
 * every user's ranking, best first.  n_u = 0 does nothing.  Errors:
 * ALS_E_INVAL for a NULL pointer or a size outside the limits above. */
ALS_API int rank_top_t(als_ctx *ctx, const void *U, const void *M, int64_t n_u, int64_t n_m,
                       int n_f, int ld, als_dtype dt, int t, int32_t *top, void *stream);

/* Ranking accuracy of (U, M) against reference lists top [n_u, t] (distinct
 * item ids per row, e.g. rank_top_t of the converged factors): for user i,
 * s_i = the number of adjacent swaps that move the reference items
 * top[i][0], top[i][1], ... one after the other to places 1, 2, ... of the
 * current ranking (Section IV), and q_i = 1 - s_i / s_max with
 * s_max = t (2 n_m - t - 1) / 2.  swaps (device int64 [n_u], may be NULL)
 * receives s_i; mean_q (device double [1], may be NULL) the mean of q_i,
 * computed as 1 - (sum_i s_i) / (n_u s_max) from the exact integer sum.
 * Needs n_u >= 1 and n_m >= 2; uses 8 bytes of context workspace.  Errors as
 * rank_top_t. */
ALS_API int rank_accuracy(als_ctx *ctx, const void *U, const void *M, int64_t n_u, int64_t n_m,
                          int n_f, int ld, als_dtype dt, int t, const int32_t *top,
                          int64_t *swaps, double *mean_q, void *stream);

/* ---------------------------------------------------------------- serving
 *
 * Fold-in server: new users (requests) are solved against fixed item factors
 * by the row solve of Eq. (3), with continuous batching.  Requests wait in a
 * FIFO queue; whenever one of `max_inflight` batch slots is free, every queued
 * request that fits the slot is admitted into one batch, which is copied to
 * the device, solved (long requests split over several wavefronts, fixed-order
 * reduction) and copied back on the slot's own stream, so batches overlap on
 * the device while new requests keep arriving.  Device memory is bounded by
 * `hbm_budget_bytes` (split evenly over the slots); a request too large for a
 * slot is answered with ALS_E_BUDGET, never dropped.  A request's result does
 * not depend on which other requests share its batch.  One server per host
 * thread; M must stay valid and unchanged while the server lives.
 */
typedef struct als_server als_server;

typedef struct {
    int64_t hbm_budget_bytes; /* device bytes for all slots (inputs, plans, results, workspace) */
    int32_t max_inflight;     /* batch slots (each with its own stream), >= 1 */
    int32_t max_batch;        /* requests per batch, >= 1 (1 = one request per launch) */
    int32_t split;            /* ratings per wavefront for long requests (0: one wavefront each) */
} als_server_config;

/* Create a server solving against M [n_items, ld] (device, FP32 or FP64). */
ALS_API int als_server_create(als_ctx *ctx, const void *M, int64_t n_items, int n_f, int ld,
                              double lambda, als_dtype dt, const als_server_config *cfg,
                              als_server **out);
/* Waits for in-flight batches, then frees everything.  NULL is ignored. */
ALS_API void als_server_destroy(als_server *srv);

/* Queue n requests (host arrays, copied by the call): request q has id
 * ids[q] and ratings (items[k], vals[k]) for k in [indptr[q], indptr[q+1]),
 * item ids in [0, n_items), distinct within a request. */
ALS_API int als_server_submit(als_server *srv, int64_t n, const int64_t *ids, const int64_t *indptr,
                              const int32_t *items, const float *vals);

/* Non-blocking progress: harvest finished batches and admit queued requests
 * into free slots.  Reports at most max_done finished requests: done_ids,
 * done_status (0, ALS_E_INVAL for an empty request, ALS_E_NOT_SPD,
 * ALS_E_BUDGET) and their solutions in done_U (host, row-major
 * [max_done, n_f], element type dt); *n_done receives the count. */
ALS_API int als_server_poll(als_server *srv, int64_t max_done, int64_t *done_ids,
                            int32_t *done_status, void *done_U, int64_t *n_done);

/* Number of requests queued or in flight. */
ALS_API int64_t als_server_pending(const als_server *srv);

/* Open-loop replay for latency measurement: arrival q carries request
 * pool_row[q] of a request pool (host CSR pool_indptr [n_pool+1], pool_items,
 * pool_vals) and becomes visible to the server arrival_ns[q] nanoseconds
 * after the call starts (non-decreasing); the call spins on the server's
 * admission and harvesting until every arrival is answered.  completion_ns[q]
 * receives the time its result was visible on the host, status[q] (may be
 * NULL) its status, U_out (host [n, n_f], may be NULL) its solution.  The
 * server must be idle (nothing queued or in flight). */
ALS_API int als_server_replay(als_server *srv, int64_t n, const int64_t *arrival_ns,
                              const int32_t *pool_row, int64_t n_pool, const int64_t *pool_indptr,
                              const int32_t *pool_items, const float *pool_vals,
                              int64_t *completion_ns, int32_t *status, void *U_out);

#ifdef __cplusplus
}
#endif
#endif /* ALSNCG_H */
