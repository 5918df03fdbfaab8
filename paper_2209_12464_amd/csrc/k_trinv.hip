// Explicit inverse X = R^-1 of the upper-triangular Cholesky factor R (dp x
// dp, 16 x 16 blocks), so that the CholeskyQR solve Q = Y R^-1 becomes a
// plain product with no chain across column blocks.  Column blocks of X are
// independent: workgroup J forms X[:, J] by block back substitution,
//     X_JJ = R_JJ^-1,   X_IJ = -R_II^-1 sum_{t = I+1..J} R_It X_tJ   (I < J),
// right-looking: as soon as X_{I+1,J} is known every pending block row
// I' <= I adds R_{I',I+1} X_{I+1,J} to its accumulator (float64 MFMA), and the
// owner of row I finishes it with R_II^-1.  Rows are dealt to the waves
// round-robin; X_{I+1,J} is passed through LDS (double buffered, one
// workgroup barrier per block row).  The step loop is unrolled so that the
// R tiles of each step can be loaded into a register ring several steps
// before they are used.  The diagonal-block inverses come from
// the Cholesky.  Nothing is done after the Cholesky's fast path, which
// writes its own inverse.  A dependent column has a unit row in R, so the
// inverse exists and its other columns do not involve it.
#include "common.h"
#include "grouped.h"
#include "kernels.h"

#include <utility>

namespace rqlp {

// kInvWaves waves; up to kInvT block rows (grid = number of block rows,
// dp is the row stride of R and X); R tiles are loaded kInvAhead steps
// before they are used.
// The body is shared by the one-matrix kernel and the grouped kernel
// (J: the column block this workgroup forms).
template <int kInvWaves, int kInvT, int kInvAhead>
__device__ __attribute__((always_inline)) inline void trinv_body(const double* __restrict__ R,
                                                               const double* __restrict__ Rinv16, int dp,
                                                               const int32_t* __restrict__ mode,
                                                               double* __restrict__ X, const int J) {
  constexpr int kInvRows = (kInvT + kInvWaves - 1) / kInvWaves;  // block rows per wave
  __shared__ double Zs[2][kTile][kTile + 1];
  if (*mode == 2) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane >> 4, lc = lane & 15;

  // A operands of R_{I', t} for this wave's rows I' = wave + 8 s, step I = t - 1:
  // ring[I % kInvAhead][s][ks] (float64 MFMA A layout: A[m][kk] = R_I't[m][kk])
  double ring[kInvAhead][kInvRows][4];
  auto load_step = [&](auto Ic) {
    constexpr int I = decltype(Ic)::value;
    constexpr int t = I + 1;
#pragma unroll
    for (int s = 0; s < kInvRows; ++s) {
      const int Ip = wave + kInvWaves * s;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        ring[I % kInvAhead][s][ks] =
            (Ip <= I) ? R[(int64_t)(Ip * kTile + lc) * dp + t * kTile + ks * 4 + lr] : 0.0;
    }
  };
  // -R_I'I'^-1 as A operands for the rows this wave finishes
  double rinv[kInvRows][4];
#pragma unroll
  for (int s = 0; s < kInvRows; ++s) {
    const int Ip = wave + kInvWaves * s;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
      rinv[s][ks] = (Ip < J) ? -Rinv16[(int64_t)Ip * kTile * kTile + lc * kTile + ks * 4 + lr] : 0.0;
  }
  // the first kInvAhead steps (I = J-1 down to J-kInvAhead)
  [&]<int... Is>(std::integer_sequence<int, Is...>) {
    ((Is < J && Is >= J - kInvAhead ? load_step(std::integral_constant<int, Is>{}) : void()), ...);
  }(std::make_integer_sequence<int, kInvT>{});

  // X_JJ = R_JJ^-1 (row-major 16 x 16 block of Rinv16)
  for (int e = tid; e < kTile * kTile; e += blockDim.x) {
    const int r = e / kTile, c = e % kTile;
    const double v = Rinv16[(int64_t)J * kTile * kTile + e];
    Zs[0][r][c] = v;
    X[(int64_t)(J * kTile + r) * dp + J * kTile + c] = v;
  }
  doublex4 S[kInvRows];  // accumulators of block rows wave + kInvWaves s
#pragma unroll
  for (int s = 0; s < kInvRows; ++s) S[s] = Mfma<double>::zero();
  __syncthreads();

  // steps I = J-1 down to 0, unrolled so that the ring slots are fixed
  auto step = [&](auto Ic) {
    constexpr int I = decltype(Ic)::value;
    if (I >= J) return;
    const int buf = (J - 1 - I) & 1;  // X_{I+1,J} is in Zs[buf]
    // S_I' += R_{I',I+1} X_{I+1,J} for the pending rows I' <= I of this wave
#pragma unroll
    for (int s = 0; s < kInvRows; ++s) {
      const int Ip = wave + kInvWaves * s;
      if (Ip <= I) {
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
          S[s] = Mfma<double>::mma(ring[I % kInvAhead][s][ks], Zs[buf][ks * 4 + lr][lc], S[s]);
      }
    }
    // this step's ring slot is free again: fetch the tiles of step I - kInvAhead
    if constexpr (I >= kInvAhead) load_step(std::integral_constant<int, I - kInvAhead>{});
    // the owner of row I finishes X_IJ = -R_II^-1 S_I
    if (wave == I % kInvWaves) {
      constexpr int so = I / kInvWaves;
      doublex4 z = Mfma<double>::zero();
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)  // the accumulator layout is the B operand layout
        z = Mfma<double>::mma(rinv[so][ks], S[so][ks], z);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = lr + 4 * r;
        Zs[buf ^ 1][row][lc] = z[r];
        X[(int64_t)(I * kTile + row) * dp + J * kTile + lc] = z[r];
      }
    }
    __syncthreads();
  };
  [&]<int... Is>(std::integer_sequence<int, Is...>) {
    (step(std::integral_constant<int, kInvT - 1 - Is>{}), ...);
  }(std::make_integer_sequence<int, kInvT>{});
}

template <int kInvWaves, int kInvT, int kInvAhead>
__global__ __launch_bounds__(kInvWaves * 64) void trinv_kernel(const double* __restrict__ R,
                                                               const double* __restrict__ Rinv16, int dp,
                                                               const int32_t* __restrict__ mode,
                                                               double* __restrict__ X) {
  trinv_body<kInvWaves, kInvT, kInvAhead>(R, Rinv16, dp, mode, X, blockIdx.x);
}

// Many matrices in one launch (argument table in device memory):
// workgroups start[p] .. start[p + 1] - 1 form the column blocks of matrix p.
struct TrinvRecArgs {
  const double* R;
  const double* Rinv16;
  const int32_t* mode;
  double* X;
  int ld;
};

template <int W, int T, int AH>
__global__ __launch_bounds__(W * 64) void trinv_grouped(const TrinvRecArgs* __restrict__ a,
                                                        const int* __restrict__ start, int count) {
  const int p = group_find(start, count, blockIdx.x);
  const TrinvRecArgs g = a[p];
  trinv_body<W, T, AH>(g.R, g.Rinv16, g.ld, g.mode, g.X, (int)blockIdx.x - start[p]);
}

template <int W, int T, int AH>
void trinv_grouped_launch(const void* args, const int* start, int count, unsigned blocks, hipStream_t s) {
  hipLaunchKernelGGL((trinv_grouped<W, T, AH>), dim3(blocks), dim3(W * kWave), 0, s, (const TrinvRecArgs*)args, start,
                     count);
}

hipError_t launch_trinv(const double* R, const double* Rinv16, int dp, const int32_t* mode, double* X,
                        hipStream_t s) {
  return launch_trinv_block(R, Rinv16, dp, dp / kTile, mode, X, s);
}

hipError_t launch_trinv_block(const double* R, const double* Rinv16, int ld, int nT, const int32_t* mode,
                              double* X, hipStream_t s) {
  const TrinvRecArgs a{R, Rinv16, mode, X, ld};
  if (nT <= kCholRegMax / kTile) {
    if (!record_launch(&trinv_grouped_launch<8, kCholRegMax / kTile, 4>, a, (unsigned)nT))
      hipLaunchKernelGGL((trinv_kernel<8, kCholRegMax / kTile, 4>), dim3((unsigned)nT), dim3(8 * kWave), 0, s, R,
                         Rinv16, ld, mode, X);
  } else {
    if (!record_launch(&trinv_grouped_launch<16, kDMax / kTile, 2>, a, (unsigned)nT))
      hipLaunchKernelGGL((trinv_kernel<16, kDMax / kTile, 2>), dim3((unsigned)nT), dim3(16 * kWave), 0, s, R,
                         Rinv16, ld, mode, X);
  }
  return hipGetLastError();
}

}  // namespace rqlp
