// Q = Y R^-1 for the upper-triangular Cholesky factor R (float64), the last
// step of each CholeskyQR pass.  Rows are independent: one wave owns 16
// rows and walks the 16-column blocks J in order,
//     acc   = Y[:, J] - sum_{t < J} Q[:, t] R[t, J]      (float64 MFMA)
//     Q[:,J] = acc * inv(R[J, J])                        (4 MFMAs)
// keeping its finished Q blocks in LDS as the A operand of later blocks.
// Arithmetic is float64 whatever the storage type of Y and Q.
// Columns the Cholesky marked dependent are replaced by N(0,1)/sqrt(rows)
// columns from a Philox stream of their own (completion of a rank-deficient
// basis); their R rows are zero, so later columns do not depend on them.
// When the Cholesky took its fast path it also wrote R^-1 explicitly; then
// every 16 x 16 output block is an independent sum, Q[:,J] = sum_t Y[:,t]
// X[t,J], and the grid's second dimension splits the column blocks into
// groups of four so that four times as many waves share the work.
#include "common.h"
#include "kernels.h"

namespace rqlp {

template <typename Tin, typename Tout>
__global__ __launch_bounds__(64) void apply_kernel(const Tin* __restrict__ Y, int64_t ldy, int64_t rows,
                                                   int d, int dp, const double* __restrict__ R,
                                                   const double* __restrict__ Rinv16,
                                                   const int32_t* __restrict__ flags,
                                                   const int32_t* __restrict__ mode,
                                                   const double* __restrict__ Xfull,
                                                   Tout* __restrict__ out1, int64_t ld1, int ncols1,
                                                   Tout* __restrict__ out2, int64_t ld2, int ncols2,
                                                   uint64_t seed, uint64_t key1, double inv_sqrt_rows) {
  extern __shared__ double Qs[];  // [16][dp + 1]
  const int lane = threadIdx.x;
  const int lr = lane >> 4, lc = lane & 15;
  const int S = dp + 1;
  const int64_t r0 = (int64_t)blockIdx.x * kTile;
  const int T = dp / kTile;

  if (*mode == 1) {
    // explicit inverse: column blocks J in [4 g, 4 g + 4)
    const int g = blockIdx.y;
    const int J0 = 4 * g;
    if (J0 >= T) return;
    const int J1 = min(T, J0 + 4);
    doublex4 acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = Mfma<double>::zero();
    const int64_t arow = r0 + lc;
    for (int t = 0; t < J1; ++t) {
      double a[4];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int col = t * kTile + ks * 4 + lr;
        a[ks] = (arow < rows && col < d) ? (double)Y[arow * ldy + col] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int J = J0 + u;
        if (J < J1 && t <= J) {
#pragma unroll
          for (int ks = 0; ks < 4; ++ks)
            acc[u] = Mfma<double>::mma(a[ks], Xfull[(int64_t)(t * kTile + ks * 4 + lr) * dp + J * kTile + lc],
                                       acc[u]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int col = (J0 + u) * kTile + lc;
      if (J0 + u >= J1) break;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + lr + 4 * r;
        if (row < rows) {
          if (col < ncols1) out1[row * ld1 + col] = (Tout)acc[u][r];
          if (out2 && col < ncols2) out2[row * ld2 + col] = (Tout)acc[u][r];
        }
      }
    }
    return;
  }
  if (blockIdx.y != 0) return;

  for (int J = 0; J < T; ++J) {
    doublex4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + lr + 4 * r;
      const int col = J * kTile + lc;
      acc[r] = (row < rows && col < d) ? (double)Y[row * ldy + col] : 0.0;
    }
    // acc -= Q[:, t-block] R[t-block, J-block]: all R fragments of column
    // block J are requested first (one memory latency per block), and the
    // sum is split over two accumulators to shorten the dependent chain.
    double b[kDMax / kTile][4];
#pragma unroll
    for (int t = 0; t < kDMax / kTile; ++t)
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        b[t][ks] = (t < J) ? R[(int64_t)(t * kTile + ks * 4 + lr) * dp + J * kTile + lc] : 0.0;
    doublex4 acc2 = Mfma<double>::zero();
#pragma unroll
    for (int t = 0; t < kDMax / kTile; ++t) {
      if (t < J) {
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const double a = -Qs[lc * S + t * kTile + ks * 4 + lr];
          if (t & 1) acc2 = Mfma<double>::mma(a, b[t][ks], acc2);
          else acc = Mfma<double>::mma(a, b[t][ks], acc);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] += acc2[r];
    // stage acc as an A operand, then multiply by inv(R[J, J])
#pragma unroll
    for (int r = 0; r < 4; ++r) Qs[(lr + 4 * r) * S + J * kTile + lc] = acc[r];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    doublex4 q = Mfma<double>::zero();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const double a = Qs[lc * S + J * kTile + ks * 4 + lr];
      const double b = Rinv16[(int64_t)J * kTile * kTile + (ks * 4 + lr) * kTile + lc];
      q = Mfma<double>::mma(a, b, q);
    }
    const int col = J * kTile + lc;
    const bool dep = (col < d) && flags[col] != 0;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + lr + 4 * r;
      double v = q[r];
      if (dep) v = (row < rows) ? gaussian_at(seed, key1, (uint64_t)col * rows + row) * inv_sqrt_rows : 0.0;
      Qs[(lr + 4 * r) * S + col] = v;
      if (row < rows) {
        if (col < ncols1) out1[row * ld1 + col] = (Tout)v;
        if (out2 && col < ncols2) out2[row * ld2 + col] = (Tout)v;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

template <typename Tin, typename Tout>
hipError_t launch_apply(const Tin* Y, int64_t ldy, int64_t rows, int d, int dp, const double* R,
                        const double* Rinv16, const int32_t* flags, const int32_t* mode,
                        const double* Xfull, Tout* out1, int64_t ld1, int ncols1, Tout* out2,
                        int64_t ld2, int ncols2, uint64_t seed, uint64_t key1, hipStream_t s,
                        hipEvent_t ev0, hipEvent_t ev1) {
  if (rows <= 0) return hipSuccess;
  const size_t shmem = (size_t)kTile * (dp + 1) * sizeof(double);
  const double isr = 1.0 / sqrt((double)rows);
  const unsigned groups = (unsigned)ceil_div(dp / kTile, 4);
  if (ev0) (void)hipEventRecord(ev0, s);
  hipLaunchKernelGGL((apply_kernel<Tin, Tout>), dim3((unsigned)ceil_div(rows, kTile), groups), dim3(64), shmem, s,
                     Y, ldy, rows, d, dp, R, Rinv16, flags, mode, Xfull, out1, ld1, ncols1, out2, ld2, ncols2,
                     seed, key1, isr);
  if (ev1) (void)hipEventRecord(ev1, s);
  return hipGetLastError();
}

#define RQLP_APPLY_INST(TI, TO)                                                                       \
  template hipError_t launch_apply<TI, TO>(const TI*, int64_t, int64_t, int, int, const double*,     \
                                           const double*, const int32_t*, const int32_t*, const double*, \
                                           TO*, int64_t, int, TO*, int64_t,                               \
                                           int, uint64_t, uint64_t, hipStream_t, hipEvent_t, hipEvent_t);
RQLP_APPLY_INST(float, double)
RQLP_APPLY_INST(double, double)
RQLP_APPLY_INST(double, float)
#undef RQLP_APPLY_INST

}  // namespace rqlp
