// Explicit inverse X = R^-1 of the upper-triangular Cholesky factor R (dp x
// dp, 16 x 16 blocks), so that the CholeskyQR solve Q = Y R^-1 becomes a
// plain product with no chain across column blocks.  Column blocks of X are
// independent: workgroup J forms X[:, J] by block back substitution,
//     X_JJ = R_JJ^-1,   X_IJ = -R_II^-1 sum_{t = I+1..J} R_It X_tJ   (I < J),
// right-looking: as soon as X_{I+1,J} is known every pending block row
// I' <= I adds R_{I',I+1} X_{I+1,J} to its accumulator (float64 MFMA), and the
// owner of row I finishes it with R_II^-1.  Rows are dealt to the 8 waves
// round-robin; X_{I+1,J} is passed through LDS (double buffered, one
// workgroup barrier per block row).  The diagonal-block inverses come from
// the Cholesky.  Nothing is done when the Cholesky marked a dependent column
// (the solve then substitutes instead).
#include "common.h"
#include "kernels.h"

namespace rqlp {

constexpr int kInvWaves = 8;
constexpr int kInvRows = kDMax / kTile / kInvWaves;  // block rows per wave

__global__ __launch_bounds__(kInvWaves * 64) void trinv_kernel(const double* __restrict__ R,
                                                               const double* __restrict__ Rinv16, int dp,
                                                               const int32_t* __restrict__ mode,
                                                               double* __restrict__ X) {
  __shared__ double Zs[2][kTile][kTile + 1];
  if (*mode != 1) return;
  const int J = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane >> 4, lc = lane & 15;

  // X_JJ = R_JJ^-1 (row-major 16 x 16 block of Rinv16)
  for (int e = tid; e < kTile * kTile; e += blockDim.x) {
    const int r = e / kTile, c = e % kTile;
    const double v = Rinv16[(int64_t)J * kTile * kTile + e];
    Zs[0][r][c] = v;
    X[(int64_t)(J * kTile + r) * dp + J * kTile + c] = v;
  }
  doublex4 S[kInvRows];  // accumulators of block rows wave + 8 s
#pragma unroll
  for (int s = 0; s < kInvRows; ++s) S[s] = Mfma<double>::zero();
  __syncthreads();

  int buf = 0;
  for (int I = J - 1; I >= 0; --I) {
    const int t = I + 1;  // X_tJ is in Zs[buf]
    // S_I' += R_I't X_tJ for the pending rows I' <= I of this wave
#pragma unroll
    for (int s = 0; s < kInvRows; ++s) {
      const int Ip = wave + kInvWaves * s;
      if (Ip <= I) {
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int kk = ks * 4 + lr;
          const double a = R[(int64_t)(Ip * kTile + lc) * dp + t * kTile + kk];  // A[m][kk] = R_I't[m][kk]
          S[s] = Mfma<double>::mma(a, Zs[buf][kk][lc], S[s]);                  // B[kk][n] = X_tJ[kk][n]
        }
      }
    }
    // the owner of row I finishes X_IJ = -R_II^-1 S_I
    if (wave == I % kInvWaves) {
      const int so = I / kInvWaves;
      doublex4 z = Mfma<double>::zero();
#pragma unroll
      for (int s = 0; s < kInvRows; ++s)
        if (s == so) {
#pragma unroll
          for (int ks = 0; ks < 4; ++ks)  // the accumulator layout is the B operand layout
            z = Mfma<double>::mma(-Rinv16[(int64_t)I * kTile * kTile + lc * kTile + ks * 4 + lr], S[s][ks], z);
        }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = lr + 4 * r;
        Zs[buf ^ 1][row][lc] = z[r];
        X[(int64_t)(I * kTile + row) * dp + J * kTile + lc] = z[r];
      }
    }
    __syncthreads();
    buf ^= 1;
  }
}

hipError_t launch_trinv(const double* R, const double* Rinv16, int dp, const int32_t* mode, double* X,
                        hipStream_t s) {
  hipLaunchKernelGGL(trinv_kernel, dim3((unsigned)(dp / kTile)), dim3(kInvWaves * kWave), 0, s, R, Rinv16, dp,
                     mode, X);
  return hipGetLastError();
}

}  // namespace rqlp
