// Cholesky factor of the float64 Gram matrix, G = R^T R (R upper), for
// d <= 256: the middle step of each CholeskyQR pass (orth() and qr() of the
// paper, computed as an unpivoted QR with a positive diagonal in R).
//
// One workgroup of 8 waves, right-looking over 16-column blocks k.  The
// lower triangle of G is cut into 16 x 16 tiles held in registers (MFMA
// 16x16x4 accumulator layout: lane l holds rows l/16 + 4 s, column l % 16),
// dealt round-robin to the waves.  Per block column k:
//   A. the owner of tile (k,k) factors it in registers and, in the same
//      sweep, forms the inverse of the 16 x 16 factor.  The trailing part
//      is kept symmetric so that each lane finds the multiplier of its own
//      column in row j; per pivot the lanes exchange data by one readlane
//      (the pivot), one cross-lane shuffle (row j) and DPP row broadcasts
//      (column j), and 1/sqrt is a hardware estimate plus Newton steps;
//   B. owners of tiles (i,k), i > k, form L_ik = G_ik L_kk^-T (4 MFMAs) and
//      publish them in an LDS panel;
//   C. owners of tiles (i,j), k < j <= i, update G_ij -= L_ik L_jk^T (MFMA).
// Columns whose pivot is <= tol * (their original squared norm) are marked
// dependent: their L column is zero, their R diagonal is 1 (so R stays
// invertible for the solve) and the caller replaces the matching columns of
// Q with random directions.
//
// Fast path for the second CholeskyQR pass: G = I + E with E small.  The
// upper-triangular F with F + F^T = E (F = triu(E, 1) + diag(E) / 2) gives
// R = I + F with R^T R = G + F^T F, so Q = Q1 R^-1 is orthonormal up to
// ~||F||_2^2 <= ||E||_F^2 / 4.  The host passes the largest ||E||_F that keeps
// this below the output precision; then R = I + F, R^-1 = I - F (to the same
// order) is written explicitly and the solve becomes a plain product.
#include "common.h"
#include "kernels.h"

namespace rqlp {

constexpr double kFastPathTol = 0x1p-30;

__device__ inline double bcast(double x, int lane) {
  // value of x in lane `lane` (wave-uniform index), as a scalar broadcast
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

__device__ inline void tile_of(int t, int& i, int& j) {
  // t = i (i + 1) / 2 + j, 0 <= j <= i
  int ii = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
  while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
  while (ii * (ii + 1) / 2 > t) --ii;
  i = ii;
  j = t - ii * (ii + 1) / 2;
}


// 1/sqrt(x) to float64 accuracy: hardware estimate and two Newton steps.
__device__ inline double rsqrt_f64(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double r = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, r, y);
  }
  return y;
}

// Value of x in lane N of this lane's 16-lane row (DPP row_newbcast).
template <int N>
__device__ inline double row_bcast(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x150 + N, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x150 + N, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// One pivot step of the 16 x 16 diagonal-tile factorization.  The tile is in
// the MFMA accumulator layout (lane (g, c) = (l / 16, l % 16) holds rows
// g + 4 r of column c) and is kept symmetric, so S[J][c] = S[c][J] gives
// every lane the multiplier of its own column.  x accumulates L^-1 by rows.
template <int J>
__device__ inline void pivot_step(doublex4& a, doublex4& x, int lr, int lc, const double* gd, double tol,
                                  int& depmask) {
  constexpr int kSlot = J >> 2;
  const double piv = bcast(a[kSlot], J + 16 * (J & 3));  // S[J][J]
  const int src = lc + 16 * (J & 3);
  const double sjc = __shfl(a[kSlot], src);             // S[J][c]
  const double xj = __shfl(x[kSlot], src);              // running X[J][c]
  const double orig = gd[J];
  const bool dep = !(piv > tol * orig);
  const double inv = dep ? 1.0 : rsqrt_f64(piv);
  const double ljj = dep ? 1.0 : piv * inv;
  const double lcj = dep ? 0.0 : sjc * inv;              // L[c][J]
  const double xjc = xj * inv;                           // X[J][c]
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double colj = row_bcast<J>(a[r]);              // S[g + 4 r][J]
    const int row = lr + 4 * r;
    const double lrj = dep ? 0.0 : colj * inv;           // L[g + 4 r][J]
    if (lc > J) a[r] -= lrj * lcj;
    else if (lc == J) a[r] = (row > J) ? lrj : (row == J ? ljj : 0.0);
    if (row == J) x[r] = xjc;
    else if (row > J) x[r] -= lrj * xjc;
  }
  depmask |= dep ? (1 << J) : 0;
}

template <int J>
__device__ inline void factor_tile(doublex4& a, doublex4& x, int lr, int lc, const double* gd, double tol,
                                   int& depmask) {
  pivot_step<J>(a, x, lr, lc, gd, tol, depmask);
  if constexpr (J + 1 < kTile) factor_tile<J + 1>(a, x, lr, lc, gd, tol, depmask);
}

template <int NW, int SLOTS>
__global__ __launch_bounds__(NW * 64) void chol_kernel(const double* __restrict__ G, int d, int dp,
                                                    double* __restrict__ R,
                                                    double* __restrict__ Rinv16,
                                                    int32_t* __restrict__ flags, DevInfo* info,
                                                    int pass_id, double tol, double fast_tol,
                                                    const double* __restrict__ esq, int nesq,
                                                    int32_t* __restrict__ mode,
                                                    double* __restrict__ Xfull) {
  __shared__ double Pn[kDMax / kTile][kTile][kTile + 1];  // panel tiles L_ik
  __shared__ double Di[kTile][kTile + 1];                  // inverse of the diagonal factor
  __shared__ double Gdiag[kDMax];
  __shared__ int defl[kDMax];
  constexpr int kCholWaves = NW;
  __shared__ double red[kCholWaves];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int T = dp / kTile;
  const int lr = lane >> 4, lc = lane & 15;  // MFMA accumulator layout: row lr + 4 r, col lc

  // ---------------- fast path: G close to the identity ----------------
  // ||G - I||_F^2 comes as per-block partial sums from the Gram reduction;
  // every workgroup adds them in the same fixed order.
  if (fast_tol > 0.0) {
    double ss = 0.0;
    for (int e = tid; e < nesq; e += blockDim.x) ss += esq[e];
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    double tot = 0.0;
    for (int w = 0; w < kCholWaves; ++w) tot += red[w];
    if (tot < fast_tol * fast_tol) {  // false for NaN
      // all workgroups write their share of R = I + F, R^-1 = I - F
      for (int e = blockIdx.x * blockDim.x + tid; e < dp * dp; e += gridDim.x * blockDim.x) {
        const int i = e / dp, j = e - (e / dp) * dp;
        double f = 0.0;  // F[i][j]
        if (i < d && j < d && i <= j) {
          const double g = G[(int64_t)i * dp + j];
          f = (i < j) ? g : 0.5 * (g - 1.0);
        }
        const double id = (i == j) ? 1.0 : 0.0;
        R[(int64_t)i * dp + j] = id + f;
        Xfull[(int64_t)i * dp + j] = id - f;
        if ((i >> 4) == (j >> 4))
          Rinv16[(int64_t)(i >> 4) * kTile * kTile + (i & 15) * kTile + (j & 15)] = id - f;
      }
      for (int i = blockIdx.x * blockDim.x + tid; i < dp; i += gridDim.x * blockDim.x) flags[i] = 0;
      if (blockIdx.x == 0 && tid == 0) *mode = 1;
      return;
    }
    __syncthreads();
  }
  if (blockIdx.x != 0) return;  // the factorization runs in one workgroup
  if (tid == 0) *mode = 0;

  // ---------------- full factorization ----------------
  for (int i = tid; i < dp; i += blockDim.x) {
    Gdiag[i] = (i < d) ? G[(int64_t)i * dp + i] : 1.0;
    defl[i] = 0;
  }
  const int ntiles = T * (T + 1) / 2;
  doublex4 tile[SLOTS];
  int ti[SLOTS], tj[SLOTS];
#pragma unroll
  for (int sl = 0; sl < SLOTS; ++sl) {
    const int t = wave + kCholWaves * sl;
    ti[sl] = -1;
    tj[sl] = -1;
    if (t < ntiles) tile_of(t, ti[sl], tj[sl]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = 0.0;
      if (t < ntiles) {
        const int row = ti[sl] * kTile + lr + 4 * r, col = tj[sl] * kTile + lc;
        v = (row < d && col < d) ? G[(int64_t)row * dp + col] : (row == col ? 1.0 : 0.0);
      }
      tile[sl][r] = v;
    }
  }
  int ndep_total = 0;
  __syncthreads();

  for (int k = 0; k < T; ++k) {
    const int tkk = k * (k + 1) / 2 + k;
    // ---------------- A: factor the diagonal tile ----------------
    if (wave == tkk % kCholWaves) {
      const int sk = tkk / kCholWaves;
      doublex4 a = tile[0];
#pragma unroll
      for (int sl = 1; sl < SLOTS; ++sl)
        if (sl == sk) a = tile[sl];
      doublex4 x;  // running inverse, starts as I
#pragma unroll
      for (int r = 0; r < 4; ++r) x[r] = (lr + 4 * r == lc) ? 1.0 : 0.0;
      int depmask = 0;
      factor_tile<0>(a, x, lr, lc, &Gdiag[k * kTile], tol, depmask);
      // a = L_kk (lower; rows lr + 4 r of column lc), x = L_kk^-1
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = lr + 4 * r;
        Di[row][lc] = x[r];
        // R block = L_kk^T, inverse of the R block = (L_kk^-1)^T
        R[(int64_t)(k * kTile + lc) * dp + k * kTile + row] = a[r];
        Rinv16[(int64_t)k * kTile * kTile + lc * kTile + row] = x[r];
      }
      if (lane < kTile) {
        const int dep_c = (depmask >> lane) & 1;
        defl[k * kTile + lane] = dep_c;
        flags[k * kTile + lane] = dep_c;
      }
      ndep_total += __popc(depmask);
    }
    __syncthreads();
    // ---------------- B: panel L_ik = G_ik L_kk^-T ----------------
#pragma unroll
    for (int sl = 0; sl < SLOTS; ++sl) {
      if (tj[sl] == k && ti[sl] > k) {
        const int i = ti[sl];
#pragma unroll
        for (int r = 0; r < 4; ++r) Pn[i][lr + 4 * r][lc] = tile[sl][r];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        doublex4 acc = Mfma<double>::zero();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int kk = ks * 4 + lr;
          acc = Mfma<double>::mma(Pn[i][lc][kk], Di[lc][kk], acc);  // B[kk][n] = X[n][kk]
        }
        const bool zc = defl[k * kTile + lc] != 0;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int r = 0; r < 4; ++r) Pn[i][lr + 4 * r][lc] = zc ? 0.0 : acc[r];
      }
    }
    __syncthreads();
    // publish the panel: R = L^T above the diagonal block row k, zero below
    for (int e = tid; e < (T - 1 - k) * kTile * kTile; e += blockDim.x) {
      const int i = k + 1 + e / (kTile * kTile), row = (e / kTile) % kTile, col = e % kTile;
      R[(int64_t)(k * kTile + col) * dp + i * kTile + row] = Pn[i][row][col];
      R[(int64_t)(i * kTile + row) * dp + k * kTile + col] = 0.0;
    }
    // ---------------- C: trailing update ----------------
#pragma unroll
    for (int sl = 0; sl < SLOTS; ++sl) {
      if (tj[sl] > k) {
        const int i = ti[sl], j = tj[sl];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int kk = ks * 4 + lr;
          tile[sl] = Mfma<double>::mma(-Pn[i][lc][kk], Pn[j][lc][kk], tile[sl]);  // B[kk][n] = L_jk[n][kk]
        }
      }
    }
  }
  if (lane == 0 && ndep_total > 0) {
    atomicAdd(&info->completed_cols, ndep_total);
    atomicCAS(&info->breakdown_pass, 0, pass_id);
  }
}

hipError_t launch_chol(const double* G, int d, int dp, double* R, double* Rinv16, int32_t* flags,
                       void* info, int pass_id, double fast_tol, const double* esq, int nesq,
                       int32_t* mode, double* Xfull, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const double tol = 64.0 * (double)d * 2.220446049250313e-16;
  if (ev0) (void)hipEventRecord(ev0, s);
  const int T = dp / kTile;
  // register slots per wave for the T (T + 1) / 2 lower tiles (waves x
  // slots chosen so that tiles and the diagonal-block code fit in registers)
  const int tiles = T * (T + 1) / 2;
  const unsigned grid = fast_tol > 0.0 ? 16 : 1;  // extra workgroups only help the fast path
  if (tiles <= 8 * 7)
    hipLaunchKernelGGL((chol_kernel<8, 7>), dim3(grid), dim3(8 * kWave), 0, s, G, d, dp, R, Rinv16, flags,
                       (DevInfo*)info, pass_id, tol, fast_tol, esq, nesq, mode, Xfull);
  else if (tiles <= 8 * 14)
    hipLaunchKernelGGL((chol_kernel<8, 14>), dim3(grid), dim3(8 * kWave), 0, s, G, d, dp, R, Rinv16, flags,
                       (DevInfo*)info, pass_id, tol, fast_tol, esq, nesq, mode, Xfull);
  else
    hipLaunchKernelGGL((chol_kernel<8, 17>), dim3(grid), dim3(8 * kWave), 0, s, G, d, dp, R, Rinv16, flags,
                       (DevInfo*)info, pass_id, tol, fast_tol, esq, nesq, mode, Xfull);
  if (ev1) (void)hipEventRecord(ev1, s);
  return hipGetLastError();
}

}  // namespace rqlp
