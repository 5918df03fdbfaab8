/*
 * rqlp.h -- C ABI of the MI355X (gfx950) randomized unpivoted QLP library.
 *
 * The library factors a real m x n matrix A as A ~ Q L V^T, where Q (m x d)
 * and V (n x d) have orthonormal columns, L (d x d) is lower triangular, and
 * d = k + p (target rank k plus oversampling p).  The steps follow the paper
 * "Randomized Rank-Revealing QLP for Low-Rank Matrix Decomposition",
 * Algorithm 1 (Section III-A) with the power iteration of Algorithm 2
 * (Section III-B), applied in the column-sketch orientation:
 *
 *   Omega = randn(n, d)           Gaussian test matrix (Section III-A, the sketch)
 *   Q     = orth(A Omega)         sketch and orthonormal basis
 *   q times: W = orth(A^T Q); Q = orth(A W)        (Algorithm 2)
 *   B^T   = A^T Q                 projection (Section III-A, the product with A)
 *   [V, Rt] = qr(B^T);  L = Rt^T  unpivoted QR; the L-values diag(L) reveal
 *                                 the numerical rank (Theorem 1, Corollary 1)
 *
 * orth() and qr() are the unpivoted QR with a positive diagonal in R,
 * computed by CholeskyQR2 with a float64 Gram matrix and Cholesky factor.
 * A basis inside the power iteration that only feeds the next product (Q
 * before the last step, and W) takes the first CholeskyQR pass alone: it is
 * the orthonormal factor times an upper-triangular matrix, which leaves the
 * next orthonormal factor, and so every returned factor, unchanged in exact
 * arithmetic.  The returned Q and the final qr() take both passes.
 *
 * Conventions for every entry point:
 *  - Matrices are row-major with an explicit leading dimension (elements).
 *  - Pointers named A, Q, L, V, X, Y, rowptr, colidx, vals, workspace are
 *    DEVICE pointers owned by the caller; the library never frees them and
 *    keeps no reference after the call returns.
 *  - `stream` is a hipStream_t passed as void*; NULL means the default
 *    stream.  All work is enqueued on it; calls return before it finishes.
 *  - `workspace` may be NULL: the context then uses (and grows) a device
 *    buffer of its own, kept until rqlp_destroy.  Otherwise it must hold at
 *    least the bytes the matching *_workspace_size function reports.
 *  - Argument errors are returned synchronously and enqueue nothing.
 *  - Numerical events (rank-deficient sketches completed with fresh random
 *    columns, non-finite values) are recorded on the device; read them with
 *    rqlp_get_info after synchronizing the stream.
 *  - Calls on one context must not overlap in time (the info record and the
 *    internal workspace belong to the context).  Use one context per stream.
 */
#ifndef RQLP_H
#define RQLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RQLP_OK = 0,
  RQLP_ERR_INVALID_ARG = 1,   /* bad sizes, null pointers, bad enum       */
  RQLP_ERR_UNSUPPORTED = 2,   /* valid request this build does not cover  */
  RQLP_ERR_OUT_OF_MEMORY = 3, /* workspace too small or allocation failed */
  RQLP_ERR_HIP = 4,           /* a HIP runtime call failed                */
  RQLP_ERR_NUMERICAL = 5      /* non-finite values met (rqlp_get_info)    */
} rqlp_status;

/* Working precision.  A, Q, L, V (and X, Y of the step entry points) are
 * double for RQLP_FP64 and float otherwise.  Gram matrices, Cholesky
 * factors and the first CholeskyQR pass are always float64.
 * RQLP_BF16_REFINED (dense rqlp_decompose only; UNSUPPORTED elsewhere): A
 * is float; every product with A rounds A and its right-hand factor to
 * bfloat16 (round to nearest even) and accumulates in float32 on the matrix
 * cores; the orthonormalizations are the same float64-Gram CholeskyQR as
 * for RQLP_FP32, whose second pass (returned Q, final qr()) restores
 * orthogonality.  Results are
 * float.  Its workspace also holds bfloat16 copies of A and A^T. */
typedef enum {
  RQLP_FP64 = 0,
  RQLP_FP32 = 1,
  RQLP_BF16_REFINED = 2
} rqlp_precision;

/* A context holds the device info record, an internal workspace, event
 * pools, batch streams and the autotuned plan table.  Use each context from
 * one host thread at a time (calls on one context are not synchronized with
 * each other); separate contexts are independent. */
typedef struct rqlp_ctx rqlp_ctx;

/* Device-side record of the last call on a context. */
typedef struct {
  int32_t status;          /* RQLP_OK or RQLP_ERR_NUMERICAL                  */
  int32_t completed_cols;  /* columns replaced by random completion (all QRs) */
  int32_t breakdown_pass;  /* 1-based index of the first QR that completed a
                              column (0 if none)                             */
  int32_t nonfinite;       /* 1 if a Gram matrix held NaN or Inf             */
} rqlp_info;

/* Create a context on HIP device `device` (its ordinal).  Allocates a small
 * device buffer for the info record.  *ctx is set to NULL on failure. */
rqlp_status rqlp_create(rqlp_ctx** ctx, int device);

/* Destroy a context and free its internal buffers.  Synchronizes the device
 * first.  NULL is accepted. */
rqlp_status rqlp_destroy(rqlp_ctx* ctx);

/* Bytes of workspace rqlp_decompose needs; 0 if the arguments are invalid. */
size_t rqlp_workspace_size(int64_t m, int64_t n, int k, int p, int q, rqlp_precision prec);

/* Bytes of workspace rqlp_decompose_csr needs; 0 if invalid. */
size_t rqlp_workspace_size_csr(int64_t m, int64_t n, int64_t nnz, int k, int p, int q,
                               rqlp_precision prec);

/* RU-QLP of a dense A (Algorithms 1 and 2; see the top of this file).
 *  A    : m x n, row-major, leading dimension lda >= n.
 *  k, p : target rank (k >= 1) and oversampling (p >= 0); d = k + p must
 *         satisfy d <= min(m, n) and d <= 544 in this build (d <= 256 for
 *         the CSR form).
 *  q    : number of power iterations (q >= 0), each two more passes over A.
 *  seed : key of the Gaussian test matrix (Philox4x64-10, see rqlp_gaussian).
 *  Q    : m x d output, leading dimension d.
 *  L    : d x d output, lower triangular, leading dimension d.
 *  V    : n x d output, leading dimension d.
 * Rank-deficient sketches are completed with fresh random orthonormal
 * columns; their L-values are exactly zero. */
rqlp_status rqlp_decompose(rqlp_ctx* ctx, const void* A, int64_t m, int64_t n, int64_t lda,
                           int k, int p, int q, rqlp_precision prec, uint64_t seed,
                           void* Q, void* L, void* V, void* workspace, size_t ws_bytes,
                           void* stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * rqlp_decompose with the workspace taken from a fixed device array of
 * RQLP_NOALLOC_SCRATCH_BYTES bytes that the library holds on every GPU it
 * runs on until the process ends (the array is located once per device by
 * rqlp_create).  The call allocates nothing and calls no allocating
 * routine; event timing (rqlp_set_timing) is ignored for it.  Arguments and
 * results as for rqlp_decompose (the same launch sequence, so the same
 * bits).  Returns RQLP_ERR_OUT_OF_MEMORY, enqueuing nothing, when the
 * problem's workspace (rqlp_workspace_size) exceeds the array.  Every call
 * on a GPU uses that GPU's one array: calls whose work overlaps on the
 * device (other streams, other contexts, other host threads) race and give
 * undefined results; calls ordered on one stream are safe.  The array keeps
 * the last call's contents; nothing in the method reads workspace it has
 * not written in the same call. */
#define RQLP_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
rqlp_status rqlp_decompose_noalloc(rqlp_ctx* ctx, const void* A, int64_t m, int64_t n, int64_t lda, int k, int p,
                                   int q, rqlp_precision prec, uint64_t seed, void* Q, void* L, void* V,
                                   void* stream);

/* RU-QLP of a CSR matrix A (m x n) with nnz stored entries (Section III-D:
 * O(nnz d) work per pass).  rowptr: m+1 int32, colidx: nnz int32 (column
 * indices, no duplicates within a row), vals: nnz values in the working
 * precision.  Builds the CSR of A^T once in the workspace.  Other arguments
 * as for rqlp_decompose. */
rqlp_status rqlp_decompose_csr(rqlp_ctx* ctx, const int32_t* rowptr, const int32_t* colidx,
                               const void* vals, int64_t m, int64_t n, int64_t nnz, int k, int p,
                               int q, rqlp_precision prec, uint64_t seed, void* Q, void* L,
                               void* V, void* workspace, size_t ws_bytes, void* stream);

/* Copy the info record of the last call to *out (host).  Synchronizes with
 * the device copy; valid once the call's stream has been synchronized. */
rqlp_status rqlp_get_info(rqlp_ctx* ctx, rqlp_info* out);

/* Static English description of a status code. */
const char* rqlp_status_string(rqlp_status s);

/* ---- Step entry points: each runs one step of the path on its own ---- */

/* Gaussian test matrix (the sketch of Section III-A; randn of Section II-A).
 * out: rows x cols, leading dimension ldo >= cols; entries in columns
 * [cols, ldo) are set to zero.  Entry (i, j) has logical index
 * l = j*rows + i; block c = l / 4 is Philox4x64-10 at counter (c, 0, 0, 0)
 * with key (seed, 0x52514C50 + stream_id); its words (w0, w1) give the
 * values for l = 4c and 4c+1, (w2, w3) those for 4c+2 and 4c+3, through
 * u1 = ((w >> 11) + 1) 2^-53, u2 = (w' >> 11) 2^-53 and Box-Muller
 * z = sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2), evaluated in float64 and
 * rounded to the working precision. */
rqlp_status rqlp_gaussian(rqlp_ctx* ctx, uint64_t seed, uint32_t stream_id, int64_t rows,
                          int64_t cols, rqlp_precision prec, void* out, int64_t ldo, void* stream);

/* Dense product with A (Algorithm 1: the sketch A*Omega and the projection
 * A^T Q; Algorithm 2: the power steps).
 *  trans = 0: Y (m x d) = A X,   X is n x d;   trans = 1: Y (n x d) = A^T X,
 *  X is m x d.  A is m x n row-major (lda).  X, Y leading dims ldx, ldy
 *  >= d; d <= 544.  A, X, Y are double for RQLP_FP64, float otherwise; with
 *  RQLP_BF16_REFINED, A and X are rounded to bfloat16 (into the workspace)
 *  and the products accumulated in float32. */
size_t rqlp_gemm_workspace_size(int trans, int64_t m, int64_t n, int d, rqlp_precision prec);
rqlp_status rqlp_gemm(rqlp_ctx* ctx, int trans, const void* A, int64_t m, int64_t n, int64_t lda,
                      const void* X, int64_t ldx, int d, void* Y, int64_t ldy,
                      rqlp_precision prec, void* workspace, size_t ws_bytes, void* stream);

/* Unpivoted QR of a tall matrix, Y = Q R with diag(R) >= 0 (Section II-B;
 * orth() of Section II-A), by CholeskyQR2 with float64 Gram and Cholesky.
 *  Y: rows x d (ldy), not modified.  Q: rows x d output (ldq).  R: optional
 *  d x d output (row-major, leading dimension d, working precision), NULL to
 *  skip.  Columns found linearly dependent (relative residual below about
 *  sqrt(64 d eps64)) are replaced by random unit columns; their diagonal
 *  entry of R is zero (and their whole R row when no independent column
 *  follows them).  Requires d <= rows and d <= 544. */
size_t rqlp_orth_workspace_size(int64_t rows, int d, rqlp_precision prec);
rqlp_status rqlp_orth(rqlp_ctx* ctx, const void* Y, int64_t rows, int d, int64_t ldy, void* Q,
                      int64_t ldq, void* R, rqlp_precision prec, uint64_t seed, void* workspace,
                      size_t ws_bytes, void* stream);

/* CSR times dense (Section III-D, sparse A): Y (rows x d) = A X with A a
 * rows x cols CSR matrix and X cols x d (ldx).  Working precision only. */
rqlp_status rqlp_spmm(rqlp_ctx* ctx, const int32_t* rowptr, const int32_t* colidx,
                      const void* vals, int64_t rows, int64_t cols, int64_t nnz, const void* X,
                      int64_t ldx, int d, void* Y, int64_t ldy, rqlp_precision prec, void* stream);

/* CSR transpose: CSR(A) (m x n, nnz entries) -> CSR(A^T) (n x m).  Entries
 * of each output row are ordered by increasing input row, so the result is
 * unique.  rowptr_t: n+1, colidx_t: nnz, vals_t: nnz (device, caller-owned).
 * Bit-exact and deterministic. */
size_t rqlp_csr_transpose_workspace_size(int64_t m, int64_t n, int64_t nnz);
rqlp_status rqlp_csr_transpose(rqlp_ctx* ctx, const int32_t* rowptr, const int32_t* colidx,
                               const void* vals, int64_t m, int64_t n, int64_t nnz,
                               rqlp_precision prec, int32_t* rowptr_t, int32_t* colidx_t,
                               void* vals_t, void* workspace, size_t ws_bytes, void* stream);

/* RU-QLP in the paper's own orientation (Algorithm 1 as printed, with
 * Algorithm 2 for P-bar), computed as rqlp_decompose's method on A^T (its
 * Gaussian is then m x d, drawn with the same generator and key; its basis
 * is P-bar and its right-hand factor the paper's Q) followed by the d x d
 * unpivoted QR of its L, which gives P-tilde and R-tilde: P = P-bar P-tilde,
 * L = R-tilde^T, so that A ~ Q L P^T = A P-bar P-bar^T.  The unpivoted QRs
 * are the same CholeskyQR2 as elsewhere.  Arguments as for rqlp_decompose
 * with P (n x d, leading dimension d) in place of V; RQLP_FP64 or
 * RQLP_FP32, dense A. */
size_t rqlp_workspace_size_paper(int64_t m, int64_t n, int k, int p, int q, rqlp_precision prec);
rqlp_status rqlp_decompose_paper(rqlp_ctx* ctx, const void* A, int64_t m, int64_t n, int64_t lda, int k, int p,
                                 int q, rqlp_precision prec, uint64_t seed, void* Q, void* L, void* P,
                                 void* workspace, size_t ws_bytes, void* stream);

/* ---- Autotuning of the products' plans (tile shape and split-K) ---- */

/* Time the candidate plans of the two products a dense decomposition of
 * this shape issues (Y = A X and Y = A^T X with d columns, float32 or
 * float64 kernel; the sketch and projection products of Section III-A) and
 * keep the fastest per product shape in the context's plan table; later
 * calls on the context (decompositions, batches, servers, rqlp_gemm) use
 * it.  A plan is a row tile (128 rows per workgroup, two workgroups per CU;
 * for float32 also 256 rows, one workgroup per CU) and a split-K count (the
 * default plan fills about two workgroups per CU; candidates go up to
 * four).  A (m x n, lda >= n) is only read; scratch comes from the context's
 * internal workspace.  Synchronizes `stream`.  The chosen split counts are
 * returned in *nsplit_nn and *nsplit_tn (either may be NULL).  The split
 * count changes the summation order of a product (the row tile does not),
 * so results are reproducible bit for bit for a given plan table, not
 * across tables. */
rqlp_status rqlp_autotune(rqlp_ctx* ctx, const void* A, int64_t m, int64_t n, int64_t lda, int d,
                          rqlp_precision prec, void* stream, int* nsplit_nn, int* nsplit_tn);
/* Forget every tuned plan. */
rqlp_status rqlp_autotune_clear(rqlp_ctx* ctx);
/* Number of tuned product shapes in the table. */
rqlp_status rqlp_autotune_count(rqlp_ctx* ctx, int* count);
/* Write the plan table to a text file ("rqlp-plans 2", then one line
 * "gemm <element bytes> <trans> <M> <N> <K> <nsplit> <mb>" per shape, mb = 2
 * for 128-row and 4 for 256-row tiles), or merge one read from such a file
 * into the table (version 1 files, without the mb field, are read as 128-row
 * tiles; RQLP_ERR_INVALID_ARG, table unchanged, on a malformed file or a
 * 256-row tile for float64). */
rqlp_status rqlp_autotune_save(rqlp_ctx* ctx, const char* path);
rqlp_status rqlp_autotune_load(rqlp_ctx* ctx, const char* path);

/* ---- The SVD-like form (Remark 1 of Section III-B) ---- */

/* SVD of a small square matrix, M = U diag(S) V^T (Remark 1: an SVD of the
 * d x d middle factor).  M, U, V: d x d row-major device matrices with
 * leading dimensions ldm, ldu, ldv >= d (M is read only); S: d device
 * values.  d <= 544; RQLP_FP64 or RQLP_FP32 (the iteration is float64 in
 * both).  Conventions: S descending; each pair of singular vectors signed so
 * that the entry of largest magnitude of the V column is positive (the
 * first on ties); the U column of a singular value that is exactly zero is
 * zero.  One-sided Jacobi; when it has not converged within 40 sweeps the
 * info record's status is RQLP_ERR_NUMERICAL.  Workspace as elsewhere
 * (rqlp_svd_workspace_size bytes, or NULL). */
size_t rqlp_svd_workspace_size(int d);
rqlp_status rqlp_svd_small(rqlp_ctx* ctx, const void* M, int d, int64_t ldm, void* U, int64_t ldu, void* S,
                           void* V, int64_t ldv, rqlp_precision prec, void* workspace, size_t ws_bytes,
                           void* stream);

/* RU-QLP in its SVD-like form (Remark 1): A ~ Q L V^T as by rqlp_decompose,
 * then L = U-bar diag(S) V-bar^T (rqlp_svd_small's conventions), U = Q U-bar
 * (m x d) and W = V V-bar (n x d), so that A ~ U diag(S) W^T.  U, W: leading
 * dimension d; S: d values.  Precisions as for rqlp_decompose (the bfloat16
 * form computes the SVD and the two products in float32); dense A. */
size_t rqlp_workspace_size_svd(int64_t m, int64_t n, int k, int p, int q, rqlp_precision prec);
rqlp_status rqlp_decompose_svd(rqlp_ctx* ctx, const void* A, int64_t m, int64_t n, int64_t lda, int k, int p,
                               int q, rqlp_precision prec, uint64_t seed, void* U, void* S, void* W,
                               void* workspace, size_t ws_bytes, void* stream);

/* ---- Batches of dense decompositions ---- */

/* One decomposition of a batch: A (m x n, lda >= n, device), k, p, q and
 * seed as for rqlp_decompose, outputs Q (m x d), L (d x d), V (n x d) with
 * leading dimension d = k + p. */
typedef struct {
  const void* A;
  int64_t m, n, lda;
  int k, p, q;
  uint64_t seed;
  void* Q;
  void* L;
  void* V;
} rqlp_problem;

/* Workspace bytes of rqlp_decompose_batched (the sum of the problems' own
 * workspaces); 0 when a problem is invalid. */
size_t rqlp_workspace_size_batched(int count, const rqlp_problem* problems, rqlp_precision prec);

/* Batched RU-QLP (the compute side of serving many uneven requests): every
 * problem is decomposed as by rqlp_decompose, with the same precision
 * (RQLP_FP64, RQLP_FP32 or RQLP_BF16_REFINED; dense A only) and its own
 * slice of the workspace.  With grouping on (the default,
 * rqlp_set_batch_grouping) and RQLP_FP64 or RQLP_FP32, every problem's
 * launch sequence is recorded once on the host and the batch runs as
 * grouped launches: the problems, ordered by work, are cut into three
 * groups of about equal work, and each group advances in lockstep on its
 * own stream (forked from and joined back into `stream`): phase by phase
 * (each Cholesky factorization is a phase of its own), one launch per
 * kernel variant runs that step for all the group's problems, each
 * workgroup working on its problem exactly as in the problem's own launch.  The argument tables of a batch are kept in device
 * memory and reused when the same batch (descriptors and workspace) comes
 * again.  With grouping off, or for RQLP_BF16_REFINED, the problems' launch
 * sequences are spread over eight internal streams forked from and joined
 * back into `stream`.  Either way each result is bitwise the result of
 * rqlp_decompose on the same problem.  With rqlp_set_graphs enabled, a
 * batch takes the lane form, and a batch submitted twice in a row with
 * identical descriptors and workspace is captured into a HIP graph on its
 * second submission and replayed on later ones.  The info record covers the whole batch.  `problems` is read
 * during the call only. */
rqlp_status rqlp_decompose_batched(rqlp_ctx* ctx, int count, const rqlp_problem* problems,
                                   rqlp_precision prec, void* workspace, size_t ws_bytes, void* stream);

/* Turn graph capture and replay of repeated batches on (1) or off (0). */
rqlp_status rqlp_set_graphs(rqlp_ctx* ctx, int enabled);

/* Turn grouped batches on (1, default) or off (0: every problem's launch
 * sequence runs on a lane stream unchanged).  The results are the same bits
 * either way. */
rqlp_status rqlp_set_batch_grouping(rqlp_ctx* ctx, int enabled);

/* ---- Serving: continuous batching of requests ---- */

/* A server owns an HBM budget (one device allocation of hbm_budget bytes,
 * sub-allocated first-fit for the requests' workspaces) and `slots` tick
 * streams at the default priority.  Requests (rqlp_problem, caller-owned
 * device buffers, precision fixed per server) are queued by submit; poll
 * reports finished requests and, for every free tick stream, admits queued
 * requests in arrival order (the head waits until its workspace fits) and
 * launches them together as one tick; the queue is shared out over the free
 * tick streams (a tick takes about queued / free slots requests, at most
 * rqlp_server_set_tick's limit), so requests run alone while the queue is
 * short and are grouped when a backlog builds up.  A tick runs the grouped
 * launches of rqlp_decompose_batched (RQLP_FP64, RQLP_FP32) or the requests' own
 * sequences (RQLP_BF16_REFINED) on the tick's stream.  Requests admitted
 * while earlier ticks run overlap with them on the device.  Each result is
 * bitwise the rqlp_decompose result of the same request.  Single-threaded
 * use; the context must outlive the server; its info record accumulates
 * over everything the server runs. */
typedef struct rqlp_server rqlp_server;

rqlp_status rqlp_server_create(rqlp_server** server, rqlp_ctx* ctx, size_t hbm_budget, int slots,
                               rqlp_precision prec);
rqlp_status rqlp_server_destroy(rqlp_server* server);

/* Largest number of requests admitted into one tick (1 .. 1024; default
 * 64).  A tick of one request runs its own launch sequence. */
rqlp_status rqlp_server_set_tick(rqlp_server* server, int max_requests);

/* Workspace bytes a request takes from the budget (0 when invalid). */
size_t rqlp_server_request_bytes(const rqlp_problem* request, rqlp_precision prec);

/* Queue a request; *ticket identifies it in poll's reports.  An event is
 * recorded on `stream` (a hipStream_t as void*, NULL for the default
 * stream) and the request's launches wait on it, so work the caller
 * enqueued on that stream before submitting (such as writing A) is complete
 * before the request reads its inputs.  A request whose workspace exceeds
 * the whole budget is refused (RQLP_ERR_OUT_OF_MEMORY). */
rqlp_status rqlp_server_submit(rqlp_server* server, const rqlp_problem* request, void* stream, int64_t* ticket);

/* Report finished tickets (whole ticks, at most max_done), then admit and
 * launch queued requests.  done[i] is a ticket; status[i] (status may be NULL) is RQLP_OK
 * when its outputs are complete on the device, or the error its launch
 * returned (the request then ran partly or not at all, and its outputs are
 * undefined; its workspace was released only after its stream drained).
 * inflight (requests in running ticks) and queued (may be NULL) receive the
 * counts after the call. */
rqlp_status rqlp_server_poll(rqlp_server* server, int64_t* done, int32_t* status, int max_done, int* ndone,
                             int* inflight, int* queued);

/* ---- Timing hooks (benchmarking) ---- */

/* Kernel classes whose launches can be timed with HIP events recorded on
 * the call's stream around each launch. */
typedef enum {
  RQLP_KT_GEMM_NN = 0,   /* dense A X product, split-K reduction included   */
  RQLP_KT_GEMM_TN = 1,   /* dense A^T X product, split-K reduction included */
  RQLP_KT_SPMM = 2,      /* CSR times dense            */
  RQLP_KT_GRAM = 3,      /* float64 Gram partials      */
  RQLP_KT_CHOL = 4,      /* float64 Cholesky           */
  RQLP_KT_APPLY = 5,     /* triangular solve Q = Y R^-1 */
  RQLP_KT_COUNT = 6
} rqlp_kernel_class;

/* Turn per-launch event timing on (1) or off (0) for every class; resets
 * the totals.  Each timed launch adds two event records to the stream. */
rqlp_status rqlp_set_timing(rqlp_ctx* ctx, int enabled);

/* The same for a subset of classes: bit k of mask enables class k. */
rqlp_status rqlp_set_timing_mask(rqlp_ctx* ctx, uint32_t mask);

/* After synchronizing: total milliseconds and launch count of a class since
 * timing was enabled (all recorded event pairs are resolved). */
rqlp_status rqlp_get_timing(rqlp_ctx* ctx, rqlp_kernel_class cls, double* total_ms,
                            int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* RQLP_H */
