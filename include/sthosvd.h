/*
 * sthosvd.h -- C ABI of the MI355X (gfx950) st-HOSVD library.
 *
 * Sequentially truncated HOSVD of a dense tensor (Alg. 2 of the a-Tucker
 * paper, arXiv 2010.10131): for each mode n, form the mode-n Gram matrix
 * without explicit matricization and take its R_n leading eigenvectors
 * (EIG branch), or run the ALS factor solver (ALS branch, Alg. 3); then shrink
 * the working tensor with a matricization-free TTM.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Layout.  Tensors are dense and column-major: the first index varies fastest
 *   (Sec. II-A, Sec. V).  For dims I_1..I_N the element (i_1..i_N) sits at
 *   offset sum_k i_k * prod_{m<k} I_m.  For mode n the library views a tensor
 *   as (L, I_n, M) with L = prod_{m<n} I_m and M = prod_{m>n} I_m; nothing is
 *   ever transposed or copied into a matricized form.  Factors U^(n) are
 *   I_n x R_n column-major FP64; the core is R_1 x ... x R_N column-major.
 *   Modes are 0-based in this API (mode 0 is the paper's mode 1).
 * Data types.  A tensor is either FP64 or FP32 (sth_dtype).  Factors,
 *   eigenvalues and Gram matrices are always FP64.
 * Memory.  Every pointer named "device" is device memory allocated by the
 *   caller (for instance through PyTorch); the library never allocates,
 *   frees or retains caller memory.  Host arrays (dims, ranks, pointer
 *   arrays) are read during the call only.  A plan owns host memory only.
 * Streams.  sth_stream_t is a hipStream_t (NULL = the null stream).  Entry
 *   points that launch work are enqueue-only: they return once the kernels are
 *   queued, without synchronizing, unless stated otherwise.
 * Errors.  Every call returns sth_status.  Arguments are validated before any
 *   launch; on error nothing is launched and sth_last_error() returns a
 *   thread-local description.  No C++ exception crosses this interface.
 *   Numerical failures detected on the device (NaN/Inf input, eigensolver
 *   sweep cap) are recorded in the workspace and reported by
 *   sthosvd_check().
 */
#ifndef STHOSVD_H
#define STHOSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *sth_stream_t; /* a hipStream_t */

typedef enum {
    STH_OK = 0,
    STH_ERR_INVALID = 1,     /* bad order, dims, ranks, mode, enum value or NULL pointer */
    STH_ERR_LAYOUT = 2,      /* misaligned pointer (device pointers must be 16-byte aligned) */
    STH_ERR_NOMEM = 3,       /* workspace smaller than required, or over the plan's cap */
    STH_ERR_HIP = 4,         /* a HIP runtime call or kernel launch failed */
    STH_ERR_NUMERIC = 5,     /* NaN/Inf met, or the eigensolver hit its sweep cap */
    STH_ERR_UNSUPPORTED = 6  /* a valid request this build does not implement */
} sth_status;

typedef enum { STH_F64 = 0, STH_F32 = 1 } sth_dtype;

/* Arithmetic of a contraction (Gram, TTT or TTM).  Products are formed as
 * stated.  Gram and TTT accumulate in FP32 within a chunk of at most 128
 * contraction steps, then in FP64 across chunks.  The TTM accumulates each
 * output in FP32 over its whole contraction (K = I_n terms; the K-split
 * kernel of contiguous rows with 256 < K <= 512: K / 8 terms per wave, then
 * the eight partial sums in FP32), and rounds it to the data type.  FP64:
 * FP64 throughout.
 *   STH_PREC_FP64   FP64 products (FP32 data is widened exactly)
 *   STH_PREC_FP32   FP32 products on the FP32 matrix cores
 *   STH_PREC_BF16X3 x = hi + mid (two bf16, round to nearest even);
 *                   x*y ~ hi*hi' + hi*mid' + mid*hi' on the bf16 matrix cores
 *   STH_PREC_BF16X6 x = hi + mid + lo; the six products of order <= 2^-16
 * FP64 data accepts only STH_PREC_FP64. */
typedef enum {
    STH_PREC_FP64 = 0,
    STH_PREC_FP32 = 1,
    STH_PREC_BF16X3 = 2,
    STH_PREC_BF16X6 = 3
} sth_prec;

/* Solver for a mode (Alg. 2: method 0 = EIG, otherwise ALS). */
typedef enum {
    STH_SOLVER_EIG = 0,   /* Gram + FP64 eigensolver + TTM (Alg. 2 EIG branch) */
    STH_SOLVER_ALS = 1,   /* Alg. 3 + QR + TTM (Alg. 2 ALS branch) */
    STH_SOLVER_AUTO = 2,  /* per-mode choice by the learned cost model (Sec. IV analogue) */
    STH_SOLVER_AUTO_TREE = 3   /* per-mode choice by the decision tree of Sec. IV-B */
} sth_solver;

/* Description of one decomposition.  Zero-initialize and fill. */
typedef struct {
    int32_t order;             /* N, 1..8 */
    const int64_t *dims;       /* host, N entries: I_1..I_N (>= 1) */
    const int64_t *ranks;      /* host, N entries: 1 <= R_n <= I_n */
    const int32_t *mode_order; /* host, N entries, a permutation of 0..N-1; NULL = 0,1,..,N-1 */
    int32_t dtype;             /* sth_dtype of X, the working tensor and the core */
    int32_t gram_prec;         /* sth_prec of the Gram / TTT contractions */
    int32_t ttm_prec;          /* sth_prec of the TTM contractions */
    int32_t solver;            /* sth_solver for every mode */
    const int32_t *per_mode;   /* host, N entries of sth_solver (EIG/ALS) overriding solver; or NULL */
    int32_t als_iters;         /* ALS sweeps (Alg. 3 loop count); 0 = 5 */
    int32_t eig_max_sweeps;    /* Jacobi sweep cap; 0 = 60 */
    int64_t workspace_cap;     /* bytes; 0 = no cap.  Plans needing more fail with STH_ERR_NOMEM */
    const float *mlp_weights;  /* host, selector weights (sth_selector_num_params floats); NULL = built in */
} sth_desc;

typedef struct sth_plan_s sth_plan;
typedef struct sth_batch_plan_s sth_batch_plan;

/* Thread-local text of the last error (never NULL). */
const char *sth_last_error(void);

/* Library version string. */
const char *sth_version(void);

/* ---------------------------------------------------------------------------
 * Whole decomposition (Alg. 2).
 * ------------------------------------------------------------------------- */

/* Validates d, fixes the per-mode shapes (L_n, I_n, M_n, J_n on the current
 * working tensor), the solver of every mode (the learned selector runs here,
 * on the host, for STH_SOLVER_AUTO and STH_SOLVER_AUTO_TREE) and the workspace
 * layout.  Host work only.
 * *plan receives a new plan (free with sthosvd_plan_destroy); *workspace_bytes
 * the device workspace sthosvd_run needs. */
sth_status sthosvd_plan(const sth_desc *d, sth_plan **plan, size_t *workspace_bytes);

/* Solver chosen for each mode of a plan (N entries of sth_solver, indexed by
 * mode, not by step). */
sth_status sthosvd_plan_solvers(const sth_plan *plan, int32_t *solvers_out);

void sthosvd_plan_destroy(sth_plan *plan);

/* Runs the decomposition of X (device, dims of the plan, plan dtype; read
 * only).  core: device, prod R_n elements of the plan dtype.  U: host array of
 * N device pointers, U[n] receives I_n x R_n FP64 (orthonormal columns).
 * eigvals: NULL, or host array of N device pointers (entries may be NULL);
 * for an EIG mode eigvals[n] receives the R_n leading eigenvalues of the
 * mode-n Gram in descending order (FP64); untouched for ALS modes.
 * als_init: NULL, or host array of N device pointers to I_n x R_n FP64 initial
 * guesses L_0 for ALS modes (Alg. 3 input); NULL entries use a Gaussian guess
 * drawn on the device from the counter-based generator seeded by
 * (seed, mode).  workspace: device, >= the plan's workspace_bytes.
 * Enqueue-only; the eigenvectors carry the sign convention "largest-magnitude
 * entry positive".  The EIG solver takes the R_n leading eigenvectors by
 * Jacobi up to I_n = 96 and by subspace iteration with Rayleigh-Ritz above
 * (block R_n + 16 rounded up to 8, at most 128 with at least 4 guard
 * vectors, and within the Gram's rank bound; Jacobi otherwise); FP32 data
 * also takes the subspace iteration for I_n = 49..96 when the block is at
 * most I_n / 2.  The iteration yields the leading subspace to working
 * accuracy when the spectrum has a gap after R_n. */
sth_status sthosvd_run(const sth_plan *plan, const void *X, void *core, double *const *U,
                       double *const *eigvals, const double *const *als_init, uint64_t seed,
                       void *workspace, size_t workspace_bytes, sth_stream_t stream);

/* Higher-order orthogonal iteration (HOOI; Sec. II-B names it beside
 * st-HOSVD as the Tucker algorithm st-HOSVD usually initializes): sweeps
 * times, for n = 1..N, Y = X x_m U_m^T for every m != n (increasing m) and
 * U_n <- the R_n leading eigenvectors of the mode-n Gram of Y (the EIG
 * solver of sthosvd_run, same routing and sign rule); then core = X x_1
 * U_1^T ... x_N U_N^T.  order >= 2, 1 <= R_n <= I_n <= 512.  X: device,
 * column-major, dtype (STH_F32 / STH_F64); U: host array of N device
 * pointers to I_n x R_n FP64 factors with orthonormal columns, read as the
 * starting point (e.g. st-HOSVD's) and overwritten; core: device R_1 x ...
 * x R_N of dtype; sweeps >= 0 (0: the core of the given factors only);
 * gram_prec / ttm_prec as in sthosvd_desc.  workspace: device, >=
 * sth_hooi_workspace(...) bytes (0 for invalid arguments).  Enqueue-only;
 * sth_hooi_check reports numerical failures.  Errors: STH_ERR_INVALID,
 * STH_ERR_UNSUPPORTED (I_n > 512), STH_ERR_NOMEM, STH_ERR_HIP. */
size_t sth_hooi_workspace(int32_t order, const int64_t *dims, const int64_t *ranks, int32_t dtype,
                          int32_t ttm_prec);
sth_status sth_hooi(int32_t order, const int64_t *dims, const int64_t *ranks, int32_t dtype,
                    int32_t gram_prec, int32_t ttm_prec, const void *X, double *const *U, void *core,
                    int32_t sweeps, void *workspace, size_t workspace_bytes, sth_stream_t stream);
/* Synchronizes the stream and reports the numerical flag of the last
 * sth_hooi on this workspace (as sthosvd_check), then clears it. */
sth_status sth_hooi_check(void *workspace, sth_stream_t stream);

/* Synchronizes the stream and reports numerical failures recorded in the
 * workspace by the last run on it (STH_ERR_NUMERIC), then clears them. */
sth_status sthosvd_check(const sth_plan *plan, void *workspace, sth_stream_t stream);

/* ---------------------------------------------------------------------------
 * Batched decomposition: count independent FP32 tensors of one order, EIG
 * branch in mode order 1..N, every R_n <= 64 (each tensor follows Alg. 2
 * exactly as a single run would).  One launch per phase of a mode step
 * covers the whole batch; the run is enqueue-only and may be captured in a
 * HIP graph.  The plan owns pinned host memory holding the shape/offset
 * tables, allocated and filled when the plan is made on a machine with a
 * usable device (a run then allocates nothing; without one the first run
 * makes it) and copied into the workspace by every run; a captured graph
 * reads that memory, so it must not outlive its plan.  The eigen phase runs
 * the library's direct solver for every order (exact leading eigenpairs on
 * every spectrum, R_n above the Gram's rank included).
 * ------------------------------------------------------------------------- */
sth_status sthosvd_plan_batched(const sth_desc *descs, int32_t count, sth_batch_plan **plan,
                                size_t *workspace_bytes);

/* Tile choices of the batched kernels; a zero field takes its default.  They
 * change the work split only: the TTM results are bit-identical for every
 * choice; the Gram's split (workgroups per CU, tile width) changes which
 * products each FP32 accumulator sums before its FP64 flush and the order of
 * the FP64 partial sums, so Grams agree to the rounding of the product
 * precision and decompositions within its tolerance (reconstructions within
 * 1e-5 of each other and of the FP64 oracle for split-bf16 recipes).  Modes
 * with I_n <= 160 always take the skinny class (whole triangles per
 * workgroup), whatever gram_wt_max says.
 *   gram_wg_per_cu    Gram workgroups aimed at per compute unit over the
 *                     whole batch (split-K depth), 1..64, default 4
 *   gram_wt_max       largest Gram output tile, in units of 32 rows: 1, 2
 *                     or 4, default 4
 *   ttm_rows_per_wave TTM row blocks per wave of a workgroup, 1..64,
 *                     default 4 */
typedef struct sth_batch_tiles {
    int32_t gram_wg_per_cu;
    int32_t gram_wt_max;
    int32_t ttm_rows_per_wave;
    int32_t reserved; /* must be 0 */
} sth_batch_tiles;

/* sthosvd_plan_batched with explicit tile choices (tiles may be NULL: the
 * defaults).  STH_ERR_INVALID for an out-of-range field. */
sth_status sthosvd_plan_batched_tiles(const sth_desc *descs, int32_t count,
                                      const sth_batch_tiles *tiles, sth_batch_plan **plan,
                                      size_t *workspace_bytes);
void sthosvd_plan_batched_destroy(sth_batch_plan *plan);
/* X_dev: device array of count device pointers to the inputs; core_dev:
 * device array of count device pointers to the cores; U_dev: device array of
 * count * N device pointers, U_dev[t * N + n] receives tensor t's I_n x R_n
 * FP64 factor.  workspace: device, >= workspace_bytes of the plan. */
sth_status sthosvd_run_batched(const sth_batch_plan *plan, const void *const *X_dev,
                               void *const *core_dev, double *const *U_dev, void *workspace,
                               size_t workspace_bytes, sth_stream_t stream);
/* Synchronizes, reports the device-side numerical flag of the batched runs
 * since the last check (non-finite values met: STH_ERR_NUMERIC) and clears it. */
sth_status sthosvd_check_batched(const sth_batch_plan *plan, void *workspace, sth_stream_t stream);

/* ---------------------------------------------------------------------------
 * Building blocks.  All act on one tensor Y with order/dims as above and
 * mode n (0-based).
 * ------------------------------------------------------------------------- */

/* Device workspace (bytes) needed by gram_mode_n / ttt_mode_n for this shape. */
size_t gram_mode_n_workspace(int32_t order, const int64_t *dims, int32_t n, int32_t other_rows);

/* Mode-n Gram S = Y_(n) Y_(n)^T (Alg. 2 EIG branch; the special case
 * TTT(Y, Y) of Eq. 3) without matricization.  Y: device, dtype.  S: device,
 * I_n x I_n FP64, the full symmetric matrix is written.  ws: device scratch
 * of gram_mode_n_workspace(order, dims, n, 0) bytes. */
sth_status gram_mode_n(int32_t order, const int64_t *dims, int32_t n, int32_t dtype,
                       int32_t prec, const void *Y, double *S, void *ws, size_t ws_bytes,
                       sth_stream_t stream);

/* Mode-n TTT (Eq. 3, read as a contraction over every mode but n):
 * P = Y_(n) Z_(n)^T where Z has the dims of Y with dims[n] replaced by R.
 * Y, Z: device, dtype.  P: device, I_n x R FP64.  ws: device scratch of
 * gram_mode_n_workspace(order, dims, n, R) bytes. */
sth_status ttt_mode_n(int32_t order, const int64_t *dims, int32_t n, int64_t R, int32_t dtype,
                      int32_t prec, const void *Y, const void *Z, double *P, void *ws,
                      size_t ws_bytes, sth_stream_t stream);

/* Device workspace (bytes) needed by ttm_mode_n for an I_n x R factor. */
size_t ttm_mode_n_workspace(int64_t I, int64_t R);

/* Mode-n TTM with the transpose of an I_n x R factor (Eq. 2 with the
 * R x I_n matrix U^T; the core update of Alg. 2):
 *   Z(a, r, b) = sum_i U(i, r) Y(a, i, b),
 * Z has the dims of Y with dims[n] replaced by R, in the same column-major
 * layout.  Y: device, dtype.  U: device, I_n x R FP64.  Z: device, dtype.
 * ws: device scratch of ttm_mode_n_workspace(I_n, R) bytes.  transpose_u = 1
 * takes U as R x I_n instead and applies it as is (Z = Y x_n U), which is the
 * expansion step of the Tucker reconstruction. */
sth_status ttm_mode_n(int32_t order, const int64_t *dims, int32_t n, int64_t R, int32_t dtype,
                      int32_t prec, const void *Y, const double *U, int32_t transpose_u, void *Z,
                      void *ws, size_t ws_bytes, sth_stream_t stream);

/* ttm_mode_n for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * kernels and the same bits as ttm_mode_n, with the pre-split factor kept in
 * a scratch array inside the library instead of a caller workspace.  The
 * library allocates nothing here; each device it runs on holds one array of
 * ttm_mode_n_noalloc_max_bytes() bytes (4 MiB) until the process ends.  A
 * factor whose split needs more (ttm_factor_bytes(I_n, R, prec)) is
 * STH_ERR_NOMEM with nothing launched.  All calls on one device share that
 * array: calls that can overlap on one device (several streams or host
 * threads) race and must be serialized by the caller.  Other arguments and
 * errors as in ttm_mode_n. */
size_t ttm_mode_n_noalloc_max_bytes(void);
sth_status ttm_mode_n_noalloc(int32_t order, const int64_t *dims, int32_t n, int64_t R,
                              int32_t dtype, int32_t prec, const void *Y, const double *U,
                              int32_t transpose_u, void *Z, sth_stream_t stream);

/* Device bytes of a prepared (pre-split) I_n x R factor for precision prec. */
size_t ttm_factor_bytes(int64_t I, int64_t R, int32_t prec);

/* Splits the FP64 factor U (device, I_n x R, or R x I_n with transpose_u = 1,
 * as in ttm_mode_n) once into the matrix-core operand layout that the TTM
 * kernels read for precision prec (one FP64 or FP32 value, or the two or
 * three bf16 pieces of the split precisions, per entry; the split is this
 * library's precision recipe, the contraction is Eq. 2).  out: device buffer
 * of ttm_factor_bytes(I, R, prec) bytes, owned by the caller, opaque; it stays
 * valid for any tensor whose mode n has I_n entries, as long as U does not
 * change.  For callers that apply one factor to many tensors.  Errors:
 * STH_ERR_INVALID (sizes, prec, NULL), STH_ERR_LAYOUT (unaligned pointer),
 * STH_ERR_NOMEM (out_bytes too small). */
sth_status ttm_factor_prepare(int64_t I, int64_t R, int32_t prec, const double *U,
                              int32_t transpose_u, void *out, size_t out_bytes,
                              sth_stream_t stream);

/* ttm_mode_n with a factor prepared by ttm_factor_prepare for the same I_n,
 * R and prec: one kernel launch, no workspace.  Gives the same bits as
 * ttm_mode_n with the unprepared factor.  uprep_bytes below
 * ttm_factor_bytes(I_n, R, prec) is STH_ERR_INVALID. */
sth_status ttm_mode_n_prepared(int32_t order, const int64_t *dims, int32_t n, int64_t R,
                               int32_t dtype, int32_t prec, const void *Y, const void *Uprep,
                               size_t uprep_bytes, void *Z, sth_stream_t stream);

/* R leading eigenpairs of a symmetric n x n FP64 matrix S (device), in FP64
 * (Alg. 2, EIG branch, line 7: the leading eigenvectors of the mode-n Gram):
 * U (device, n x R FP64, orthonormal, largest-magnitude entry of each column
 * positive) and lam (device, R values, descending; may be NULL).
 * n <= 128: parallel cyclic Jacobi on S (relative accuracy; max_sweeps caps
 * its sweeps, 0 = 60).  n > 128: subspace iteration on a seeded Gaussian
 * block of p = R + 16 (rounded up to 8, at most 128) columns with
 * Rayleigh-Ritz, accepted only when every Ritz residual
 * ||S u - theta u|| <= max(16 sqrt(n) eps, s_unit) |theta_1|; otherwise (and
 * when no such block exists) the direct solver of the library
 * (tridiagonalization, bisection, inverse iteration) runs on S, so the
 * result is the leading eigenpairs on every spectrum.  eig_leading_ex takes
 * s_unit, the unit roundoff with which S was formed (0 for exact data, e.g.
 * 2^-24 for a Gram of FP32 products), so that the iteration is not asked to
 * resolve S beyond its own accuracy; eig_leading uses s_unit = 0.
 * ws: device scratch of eig_leading_workspace(n) bytes; the first 8 bytes
 * receive a non-zero int64 when Jacobi hit its sweep cap (1) or S was not
 * finite (3); bytes 8..15 count the direct solves that replaced the subspace
 * iteration (a diagnostic, not an error).  s_unit outside [0, 1) is
 * STH_ERR_INVALID. */
size_t eig_leading_workspace(int64_t n);
sth_status eig_leading(int64_t n, int64_t R, const double *S, double *U, double *lam,
                       int32_t max_sweeps, void *ws, size_t ws_bytes, sth_stream_t stream);
sth_status eig_leading_ex(int64_t n, int64_t R, const double *S, double *U, double *lam,
                          int32_t max_sweeps, double s_unit, void *ws, size_t ws_bytes,
                          sth_stream_t stream);

/* Tucker reconstruction X^ = G x_1 U1 x_2 ... x_N UN (Sec. II-B).
 * G: device, prod ranks, dtype.  U: host array of N device pointers to
 * I_n x R_n FP64.  Xhat: device, prod dims, dtype.  ws: device scratch of
 * tucker_reconstruct_workspace(...) bytes. */
size_t tucker_reconstruct_workspace(int32_t order, const int64_t *dims, const int64_t *ranks,
                                    int32_t dtype);
sth_status tucker_reconstruct(int32_t order, const int64_t *dims, const int64_t *ranks,
                              int32_t dtype, int32_t prec, const void *G, const double *const *U,
                              void *Xhat, void *ws, size_t ws_bytes, sth_stream_t stream);

/* Relative-error terms of a decomposition (Sec. VI-B metric): writes
 * out[0] = ||X - X^||_F^2 and out[1] = ||X||_F^2 (device, 2 FP64), both
 * accumulated in FP64 in a fixed order, with X^ the reconstruction of
 * (G, U) (each value rounded to dtype, as tucker_reconstruct stores it).
 * The expansions of modes 1 .. N-1 run as in tucker_reconstruct; the last
 * one is fused with the sums, so X^ is never stored and X is read once.
 * ws: tucker_reconstruct_workspace bytes plus the fused step's partial sums
 * (tucker_error_workspace). */
size_t tucker_error_workspace(int32_t order, const int64_t *dims, const int64_t *ranks,
                              int32_t dtype);
sth_status tucker_error(int32_t order, const int64_t *dims, const int64_t *ranks, int32_t dtype,
                        int32_t prec, const void *X, const void *G, const double *const *U,
                        double *out, void *ws, size_t ws_bytes, sth_stream_t stream);

/* ---------------------------------------------------------------------------
 * One mode of Alg. 2 (the loop body: EIG branch, lines 6-8, or ALS branch,
 * lines 10-13 with Alg. 3) on a working tensor Y with the given dims:
 * Z (device, dims with dims[n] replaced by R, dtype) receives the shrunk
 * tensor, U (device, dims[n] x R FP64) the factor, eigvals (device, R FP64,
 * may be NULL; EIG only) the leading eigenvalues.  als_init: NULL or device
 * dims[n] x R FP64 initial guess (ALS only; NULL = seeded Gaussian).
 * solver: STH_SOLVER_EIG or STH_SOLVER_ALS.  Used to time both solvers per
 * mode for the selector's training data (Sec. IV-B).
 * ------------------------------------------------------------------------- */
size_t sthosvd_mode_step_workspace(int32_t order, const int64_t *dims, int32_t n, int64_t R,
                                   int32_t dtype, int32_t gram_prec, int32_t ttm_prec,
                                   int32_t solver, int32_t als_iters);
sth_status sthosvd_mode_step(int32_t order, const int64_t *dims, int32_t n, int64_t R,
                             int32_t dtype, int32_t gram_prec, int32_t ttm_prec, int32_t solver,
                             int32_t als_iters, const void *Y, void *Z, double *U, double *eigvals,
                             const double *als_init, uint64_t seed, void *ws, size_t ws_bytes,
                             sth_stream_t stream);

/* ---------------------------------------------------------------------------
 * Exhaustive solver selection (Sec. IV-B: timing both solvers per mode, the
 * choice the learned selector and the decision tree stand in for).  For
 * n = 1..N on the working tensor (X, then the kept step's output), the EIG
 * and the ALS step of the mode (sthosvd_mode_step, ALS only where it can run)
 * are each run once untimed and once timed with HIP events on the stream;
 * a step that raises the numerical flag does not count; the faster step is
 * kept and its output is the next mode's input.  dims/ranks: host, order
 * entries; X: device, column-major, dtype; gram_prec, ttm_prec, als_iters
 * as in sthosvd_desc.  solvers_out: host, order entries (STH_SOLVER_EIG or
 * STH_SOLVER_ALS), usable as sthosvd_desc.per_mode; ms_out: host, 2 * order
 * floats (EIG, ALS time per mode; -1 where the step did not count) or NULL.
 * workspace: device, >= sthosvd_choose_exhaustive_workspace(...) bytes (0
 * for invalid arguments); X is not modified.  Synchronizes the stream (it
 * reads the timings), so it is a planning call, not part of a captured run.
 * Errors: STH_ERR_INVALID, STH_ERR_UNSUPPORTED (no EIG step for a mode),
 * STH_ERR_NOMEM, STH_ERR_NUMERIC (the EIG step raised the flag), STH_ERR_HIP.
 * ------------------------------------------------------------------------- */
size_t sthosvd_choose_exhaustive_workspace(int32_t order, const int64_t *dims, const int64_t *ranks,
                                           int32_t dtype, int32_t gram_prec, int32_t ttm_prec,
                                           int32_t als_iters);
sth_status sthosvd_choose_exhaustive(int32_t order, const int64_t *dims, const int64_t *ranks,
                                     int32_t dtype, int32_t gram_prec, int32_t ttm_prec,
                                     int32_t als_iters, const void *X, int32_t *solvers_out,
                                     float *ms_out, void *workspace, size_t workspace_bytes,
                                     sth_stream_t stream);

/* ---------------------------------------------------------------------------
 * Learned solver selector (the role of the Sec. IV decision tree, with a
 * small MLP cost model).  Features are the ten Table I quantities of a mode
 * (I_n, R_n, J_n, I_n^2, R_n^2, I_n R_n, R_n^2/I_n, R_n^2/J_n, I_n/J_n,
 * R_n/J_n), log-scaled; the network 10 -> 32 -> 32 -> 2 (tanh hidden layers)
 * predicts (log t_EIG, log t_ALS) and the selector takes the smaller.
 * Parameters are packed floats: W1 (32x10 column-major), b1, W2 (32x32), b2,
 * W3 (2x32), b3, then the feature mean (10) and inverse std (10).
 * ------------------------------------------------------------------------- */
int32_t sth_selector_num_params(void);    /* all packed floats */
int32_t sth_selector_num_trainable(void); /* leading floats that training updates */
/* Host: the ten log-scaled features of a mode (out10: host, 10 floats). */
sth_status sth_selector_features(int64_t I, int64_t R, int64_t J, float *out10);
/* Host inference: out2 (host) = predicted (log t_EIG, log t_ALS); weights
 * (host) NULL = the built-in weights. */
sth_status sth_selector_predict(const float *weights, int64_t I, int64_t R, int64_t J, float *out2);
/* Host: the solver sthosvd_plan picks for a mode under STH_SOLVER_AUTO
 * (solver_out: STH_SOLVER_EIG or STH_SOLVER_ALS): the smaller predicted
 * time, then the solvers' limits (EIG needs I_n <= 512, ALS R_n <= 128; above
 * order 128 with R_n in 125..128, where EIG would run cyclic Jacobi on the
 * whole Gram, ALS). */
sth_status sth_selector_choose(const float *weights, int64_t I, int64_t R, int64_t J, int32_t *solver_out);

/* Host: the solver sthosvd_plan picks for a mode under STH_SOLVER_AUTO_TREE:
 * the class of the compiled-in decision tree (Sec. IV-B: CART on the Table I
 * features, depth and class weights by cross-validated grid search, trained
 * on the same timing database as the MLP), then the same solver limits and
 * whole-Gram rule as sth_selector_choose.  I, R, J >= 1, R <= I, else
 * STH_ERR_INVALID. */
sth_status sth_selector_tree_choose(int64_t I, int64_t R, int64_t J, int32_t *solver_out);

/* Device training kernels.  X: device, 10 x B features (column per sample);
 * T: device, 2 x B targets; params: device packed floats; ws: device scratch
 * of sth_mlp_workspace(B) bytes. */
size_t sth_mlp_workspace(int64_t B);
/* Y (device, 2 x B) = network(X). */
sth_status sth_mlp_forward(const float *params, int64_t B, const float *X, float *Y, void *ws,
                           size_t ws_bytes, sth_stream_t stream);
/* grad (device, num_params floats; the normalization entries are zero) =
 * gradient of L = 0.5/B sum (Y - T)^2; loss (device, 1 float, may be NULL)
 * = L.  Sums over samples run in sample order (deterministic). */
sth_status sth_mlp_loss_grad(const float *params, int64_t B, const float *X, const float *T,
                             float *grad, float *loss, void *ws, size_t ws_bytes,
                             sth_stream_t stream);
/* One Adam step (Kingma & Ba, 2015) on the first count parameters, step >= 1;
 * m and v (device, count floats) are the moment estimates, zero at step 1. */
sth_status sth_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t count,
                        float lr, float beta1, float beta2, float eps, int32_t step,
                        sth_stream_t stream);

/* FP64 sum of squares of a device array of count elements (Eq. 1 squared):
 * out (device, 1 FP64). ws: 8 * 1024 bytes. */
sth_status sth_sumsq(int32_t dtype, const void *x, int64_t count, double *out, void *ws,
                     size_t ws_bytes, sth_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* STHOSVD_H */
