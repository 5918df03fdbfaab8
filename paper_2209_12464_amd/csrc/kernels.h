// Host-side launch functions of the gfx950 kernels (one translation unit per
// kernel family).  Every launcher enqueues on `s` and returns the launch
// status; none synchronizes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rqlp {

// ---- Gaussian test matrix (k_gaussian.hip) ----
template <typename T>
hipError_t launch_gaussian(uint64_t seed, uint64_t key1, int64_t rows, int64_t cols, T* out,
                           int64_t ldo, hipStream_t s);
template <typename T>
hipError_t launch_zero_cols(T* out, int64_t rows, int64_t c0, int64_t c1, int64_t ld, hipStream_t s);

// ---- dense products (k_gemm.hip) ----
template <typename T>
struct GemmArgs {
  const T* A;      // NN: M x K (lda); TN: K x M (lda)
  int64_t lda;
  const T* B;      // K x N (ldb)
  int64_t ldb;
  int M, N, K;     // output M x N, reduction K
  int trans;       // 0: Y = A B, 1: Y = A^T B
  int mtiles;      // ceil(M / gemm_block_rows(mb))
  int nsplit;      // split-K count
  int kchunk;      // reduction length per split (multiple of 16)
  bool avec;       // A rows 16-byte aligned: vector loads
  bool bvec;       // X rows padded to the tile width with zeros: vector loads
  int mb = 2;      // row tile: 16 mb rows per wave, 64 mb per workgroup (4: float only)
};
// Rows of one workgroup's slab for row-tile parameter mb (128 or 256).
template <typename T> int gemm_block_rows(int mb);
template <typename T> int gemm_block_cols(int N);
// Y (M x nst, ldy) = op(A) B; columns [N, nst) of Y are written as zero.
// P: partial buffer of nsplit * M * nst elements (unused when nsplit == 1).
// ev0/ev1 (may be null) are recorded around the product and its reduction.
template <typename T>
hipError_t launch_gemm(GemmArgs<T> g, T* Y, int64_t ldy, int nst, T* P, hipStream_t s,
                       hipEvent_t ev0, hipEvent_t ev1);

// Y (M x nst, ldy) = sum over s of P[s] (M x nst slabs, ld nst), fixed order.
hipError_t launch_splitk_reduce_f32(const float* P, int nsplit, int M, int nst, float* Y, int64_t ldy,
                                    hipStream_t s);

// ---- bfloat16 products, float32 accumulation (k_bf16.hip) ----
// Ab (m x ldb) = bf16(A) and, if At is not null, At (n x ldt) = bf16(A)^T,
// for A (m x n float, lda); padding columns are written as zero.
hipError_t launch_cvt_bf16(const float* A, int64_t lda, int64_t m, int64_t n, uint16_t* Ab, int64_t ldb,
                           uint16_t* At, int64_t ldt, hipStream_t s);
// Xt (N x ldt) = bf16(X)^T for X (K x N float, ldx); columns [K, ldt) zero.
hipError_t launch_cvt_bf16_t(const float* X, int64_t ldx, int64_t K, int64_t N, uint16_t* Xt, int64_t ldt,
                             hipStream_t s);
// Y (M x nst, ldy) = A Xt^T with A (M x K bf16, lda) and Xt (N x K bf16,
// ldx), both k-contiguous, K a multiple of 32 with zero padding, lda and ldx
// multiples of 8.  P: split-K partials (gemm_bf16_partial_elems).
hipError_t launch_gemm_bf16(const uint16_t* A, int64_t lda, const uint16_t* Xt, int64_t ldx, int M, int N, int K,
                            float* Y, int64_t ldy, int nst, float* P, hipStream_t s, hipEvent_t ev0,
                            hipEvent_t ev1);
size_t gemm_bf16_partial_elems(int M, int K, int dp);

// ---- float64 Gram matrix (k_gram.hip) ----
// G (dp x dp, ld dp, float64, full symmetric) = Y^T Y over rows [0, rows),
// columns [0, d) of Y (ldy); entries outside d x d are zero.  Partials:
// nchunks * dp * dp doubles in P.  Sets info->nonfinite on NaN/Inf.  esq
// (gram_reduce_blocks(dp) doubles) receives block partial sums of
// ||G - I||_F^2 over the d x d part.
template <typename T>
hipError_t launch_gram(const T* Y, int64_t ldy, int64_t rows, int d, int dp, double* P,
                       int nchunks, double* G, double* esq, void* info, hipStream_t s,
                       hipEvent_t ev0, hipEvent_t ev1);
// The same with float32 arithmetic (Y rounded to float, float32 MFMA within
// a row chunk, chunk partials and their sum in float64): for a basis that
// is orthonormal to working accuracy (the bfloat16 form's second pass).
hipError_t launch_gram_f32c(const double* Y, int64_t ldy, int64_t rows, int d, int dp, double* P, int nchunks,
                            double* G, double* esq, void* info, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
int gram_chunks(int64_t rows, int dp);

// X = R^-1 (dp x dp, row-major; the blocks on and above the diagonal are
// written) from the upper Cholesky factor R and its diagonal-block
// inverses; does nothing when *mode == 2 (the fast path wrote its own
// inverse).
hipError_t launch_trinv(const double* R, const double* Rinv16, int dp, const int32_t* mode, double* X,
                        hipStream_t s);
// The same for the nT x nT block upper-triangular R (row stride ld, as X).
hipError_t launch_trinv_block(const double* R, const double* Rinv16, int ld, int nT, const int32_t* mode,
                              double* X, hipStream_t s);
int gram_reduce_blocks(int dp);

// ---- float64 Cholesky (k_chol.hip) ----
// G = R^T R for the d x d leading block of G (ld dp).  Writes R (upper,
// dp x dp, ld dp, identity beyond d; rows of dependent columns are e_j^T),
// Rinv16 (inverses of the dp/16 diagonal 16x16 blocks of R, row-major
// 16x16 each), flags[j] = 1 for dependent columns (j < dp).  Updates info.
// fast_tol > 0: when ||G - I||_F < fast_tol (from the nesq partial sums in
// esq written by launch_gram), use R = I + F (first order)
// and write the explicit inverse I - F to Xfull (dp x dp); *mode is set to
// 2 in that case.  After a full factorization *mode is 1, or 0 when a column
// was dependent; launch_trinv then forms Xfull = R^-1 in both cases.  For dp > 256 the
// factorization is blocked: it overwrites G's trailing blocks, uses Xfull
// as scratch, and keeps the original diagonal in gd0 (dp doubles).
hipError_t launch_chol(double* G, int d, int dp, double* R, double* Rinv16, int32_t* flags,
                       void* info, int pass_id, double fast_tol, const double* esq, int nesq,
                       int32_t* mode, double* Xfull, double* gd0, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);

// Register-slot class (7, 14 or 17 tiles per wave) of a dp <= 256 factorization.
int chol_slot_class(int dp);

// ---- SVD of the small factor (k_svd.hip) ----
// M (d x d, row-major, ld ldm, d <= 544) = U diag(S) V^T: S descending, U
// (ld ldu) and V (ld ldv) row-major d x d, each pair of singular vectors
// signed so that the entry of largest magnitude of the V column is
// positive; U columns of zero singular values are zero.  ws: svd_ws_bytes(d)
// bytes of device memory.  info->status is set to 5 (numerical) when the
// Jacobi iteration has not converged in kSvSweeps sweeps (one cooperative
// launch runs them all).
constexpr int kSvSweeps = 40;
inline int svd_padded(int d) { return (d + 15) / 16 * 16; }
size_t svd_ws_bytes(int d);
template <typename T>
hipError_t launch_svd_small(const T* M, int64_t ldm, int d, T* U, int64_t ldu, T* S, T* V, int64_t ldv, void* ws,
                            void* info, hipStream_t s);

// ---- triangular solve Q = Y R^-1 (k_apply.hip) ----
// Y: rows x dp (ldy, type Tin); out1 (ld1, first `ncols1` columns, type
// Tout) and optional out2 (ld2, first `ncols2` columns).  Dependent columns (flags) are replaced
// by Gaussian columns of stream (seed, key1) divided by sqrt(rows) when
// *mode == 0 (device, from launch_chol: a column was dependent); the others
// are Q = Y Xfull (Xfull = R^-1 from launch_trinv or the fast path).
template <typename Tin, typename Tout>
hipError_t launch_apply(const Tin* Y, int64_t ldy, int64_t rows, int d, int dp, const int32_t* flags,
                        const int32_t* mode, const double* Xfull, Tout* out1, int64_t ld1, int ncols1, Tout* out2,
                        int64_t ld2, int ncols2, uint64_t seed, uint64_t key1, hipStream_t s,
                        hipEvent_t ev0, hipEvent_t ev1);
// The same, but when the Cholesky took its fast path (*mode == 2: Xfull =
// I - F with F small) Y and Xfull are rounded to float and multiplied with
// float32 MFMA (the product is within float32 rounding of Y itself);
// otherwise as launch_apply.
hipError_t launch_apply_f32fast(const double* Y, int64_t ldy, int64_t rows, int d, int dp, const int32_t* flags,
                                const int32_t* mode, const double* Xfull, float* out1, int64_t ld1, int ncols1,
                                float* out2, int64_t ld2, int ncols2, uint64_t seed, uint64_t key1, hipStream_t s,
                                hipEvent_t ev0, hipEvent_t ev1);

// ---- small d x d helpers (k_small.hip) ----
// L (d x d, ld ldl, type T) = (R2 * R1')^T where R1' is R1 with the rows of
// dependent columns (flags1) zeroed; R2, R1 upper, ld dp.
template <typename T>
hipError_t launch_form_l(const double* R2, const double* R1, const int32_t* flags1, int d, int dp,
                         T* L, int64_t ldl, hipStream_t s);
// R (d x d, ld d, type T) = R2 * R1' (upper triangular)
template <typename T>
hipError_t launch_form_r(const double* R2, const double* R1, const int32_t* flags1, int d, int dp,
                         T* R, int64_t ldr, hipStream_t s);
hipError_t launch_info_reset(void* info, hipStream_t s);

// ---- CSR (k_csr.hip) ----
template <typename T>
hipError_t launch_spmm(const int32_t* rowptr, const int32_t* colidx, const T* vals, int64_t rows,
                       const T* X, int64_t ldx, int d, T* Y, int64_t ldy, int nst, hipStream_t s,
                       hipEvent_t ev0, hipEvent_t ev1);
size_t csr_transpose_scratch_bytes(int64_t m, int64_t n, int64_t nnz);
template <typename T>
hipError_t launch_csr_transpose(const int32_t* rowptr, const int32_t* colidx, const T* vals,
                                int64_t m, int64_t n, int64_t nnz, int32_t* rowptr_t,
                                int32_t* colidx_t, T* vals_t, void* scratch, hipStream_t s);

}  // namespace rqlp
