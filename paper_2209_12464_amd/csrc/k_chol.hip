// Cholesky factor of the float64 Gram matrix, G = R^T R (R upper), for
// d <= 256, in one workgroup of 16 waves.  This is the middle step of each
// CholeskyQR pass (orth() and qr() of the paper, computed as an unpivoted
// QR with positive diagonal).
//
// The lower triangle of G is cut into 16 x 16 tiles held in registers, in
// the accumulator layout of the float64 MFMA 16x16x4, spread over the 16
// waves.  Right-looking blocked algorithm, per block column k:
//   A. the owner of tile (k,k) factors it in LDS (unblocked, one wave) and
//      forms the inverse of the 16 x 16 factor;
//   B. owners of tiles (i,k), i > k, form L_ik = G_ik L_kk^-T (4 MFMAs) and
//      publish them in an LDS panel;
//   C. owners of tiles (i,j), k < j <= i, update G_ij -= L_ik L_jk^T (MFMA).
// Columns whose pivot falls to tol * (their original squared norm) or below
// are marked dependent: their factor column is zero and their diagonal is 1
// in R (so R stays invertible for the solve), and the caller replaces the
// matching columns of Q with fresh random directions.
#include "common.h"
#include "kernels.h"

namespace rqlp {

constexpr int kCholWaves = 16;
constexpr int kMaxT = kDMax / kTile;                                   // 16
constexpr int kSlots = (kMaxT * (kMaxT + 1) / 2 + kCholWaves - 1) / kCholWaves;  // 9

__device__ inline void tile_of(int t, int& i, int& j) {
  // t = i (i + 1) / 2 + j, 0 <= j <= i
  int ii = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
  while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
  while (ii * (ii + 1) / 2 > t) --ii;
  i = ii;
  j = t - ii * (ii + 1) / 2;
}

__global__ __launch_bounds__(1024) void chol_kernel(const double* __restrict__ G, int d, int dp,
                                                    double* __restrict__ R,
                                                    double* __restrict__ Rinv16,
                                                    int32_t* __restrict__ flags, DevInfo* info,
                                                    int pass_id, double tol) {
  __shared__ double Dg[kTile][kTile + 1];
  __shared__ double Di[kTile][kTile + 1];
  __shared__ double Pn[kMaxT][kTile][kTile + 1];
  __shared__ double Gdiag[kDMax];
  __shared__ int defl[kDMax];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const int T = dp / kTile;
  const int ntiles = T * (T + 1) / 2;
  const int lr = lane >> 4, lc = lane & 15;  // accumulator layout: row lr + 4 r, col lc

  for (int i = tid; i < dp; i += blockDim.x) {
    Gdiag[i] = (i < d) ? G[(int64_t)i * dp + i] : 1.0;
    defl[i] = 0;
  }

  doublex4 tile[kSlots];
  int ti[kSlots], tj[kSlots];
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    const int t = wave + kCholWaves * s;
    ti[s] = -1;
    tj[s] = -1;
    if (t < ntiles) tile_of(t, ti[s], tj[s]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = 0.0;
      if (t < ntiles) {
        const int row = ti[s] * kTile + lr + 4 * r, col = tj[s] * kTile + lc;
        v = (row < d && col < d) ? G[(int64_t)row * dp + col] : (row == col ? 1.0 : 0.0);
      }
      tile[s][r] = v;
    }
  }
  __syncthreads();

  for (int k = 0; k < T; ++k) {
    const int tkk = k * (k + 1) / 2 + k;
    // ---------------- A: factor the diagonal tile ----------------
    if (wave == tkk % kCholWaves) {
      const int sk = tkk / kCholWaves;
#pragma unroll
      for (int s = 0; s < kSlots; ++s)
        if (s == sk)
#pragma unroll
          for (int r = 0; r < 4; ++r) Dg[lr + 4 * r][lc] = tile[s][r];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      int ndep = 0;
#pragma unroll 1
      for (int c = 0; c < kTile; ++c) {
        const double piv = Dg[c][c];
        const double orig = Gdiag[k * kTile + c];
        const bool dep = !(piv > tol * orig);
        const double lcc = dep ? 1.0 : sqrt(piv);
        const double inv = 1.0 / lcc;
        __builtin_amdgcn_wave_barrier();
        if (lane > c && lane < kTile) Dg[lane][c] = dep ? 0.0 : Dg[lane][c] * inv;
        if (lane == 0) {
          Dg[c][c] = lcc;
          if (dep) defl[k * kTile + c] = 1;
        }
        ndep += dep ? 1 : 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll 1
        for (int e = lane; e < kTile * kTile; e += kWave) {
          const int r = e >> 4, j = e & 15;
          if (j > c && r >= j) Dg[r][j] -= Dg[r][c] * Dg[j][c];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
      // inverse of the lower-triangular factor; lane c < 16 forms column c in
      // LDS by forward substitution (its own column only: no cross-lane reads)
      if (lane < kTile) {
        const int c = lane;
#pragma unroll 1
        for (int i = 0; i < kTile; ++i) {
          double s = (i == c) ? 1.0 : 0.0;
#pragma unroll 1
          for (int t = c; t < i; ++t) s -= Dg[i][t] * Di[t][c];
          Di[i][c] = (i >= c) ? s / Dg[i][i] : 0.0;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      // R diagonal block = L_kk^T; inverse of the R block = (L_kk^-1)^T
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = lr + 4 * r, b = lc;  // element (a, b) of the block
        R[(int64_t)(k * kTile + a) * dp + k * kTile + b] = (b >= a) ? Dg[b][a] : 0.0;
        Rinv16[(int64_t)k * kTile * kTile + a * kTile + b] = (b >= a) ? Di[b][a] : 0.0;
      }
      if (lane < kTile) flags[k * kTile + lane] = defl[k * kTile + lane];
      // dependent columns beyond d are impossible (identity padding)
      if (lane == 0 && ndep > 0) {
        atomicAdd(&info->completed_cols, ndep);
        atomicCAS(&info->breakdown_pass, 0, pass_id);
      }
    }
    __syncthreads();
    // ---------------- B: panel L_ik = G_ik L_kk^-T ----------------
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      if (tj[s] == k && ti[s] > k) {
        const int i = ti[s];
#pragma unroll
        for (int r = 0; r < 4; ++r) Pn[i][lr + 4 * r][lc] = tile[s][r];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        doublex4 acc = Mfma<double>::zero();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int kk = ks * 4 + (lane >> 4);
          const double a = Pn[i][lc][kk];
          const double b = Di[lc][kk];  // B[kk][n] = (L_kk^-1)^T[kk][n]
          acc = Mfma<double>::mma(a, b, acc);
        }
        const bool zc = defl[k * kTile + lc] != 0;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double v = zc ? 0.0 : acc[r];
          const int row = lr + 4 * r;
          Pn[i][row][lc] = v;
          R[(int64_t)(k * kTile + lc) * dp + i * kTile + row] = v;   // R = L^T
          R[(int64_t)(i * kTile + row) * dp + k * kTile + lc] = 0.0; // below the diagonal
        }
      }
    }
    __syncthreads();
    // ---------------- C: trailing update ----------------
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      if (tj[s] > k) {
        const int i = ti[s], j = tj[s];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int kk = ks * 4 + (lane >> 4);
          const double a = -Pn[i][lc][kk];
          const double b = Pn[j][lc][kk];  // B[kk][n] = L_jk^T[kk][n]
          tile[s] = Mfma<double>::mma(a, b, tile[s]);
        }
      }
    }
  }
}

hipError_t launch_chol(const double* G, int d, int dp, double* R, double* Rinv16, int32_t* flags,
                       void* info, int pass_id, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const double tol = 64.0 * (double)d * 2.220446049250313e-16;
  if (ev0) hipEventRecord(ev0, s);
  hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(kCholWaves * kWave), 0, s, G, d, dp, R, Rinv16, flags,
                     (DevInfo*)info, pass_id, tol);
  if (ev1) hipEventRecord(ev1, s);
  return hipGetLastError();
}

}  // namespace rqlp
