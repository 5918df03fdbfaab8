// Small d x d steps: combining the two CholeskyQR factors into the R factor
// of the unpivoted QR (R = R2 R1), forming L = R^T of the last QR (the
// L-values of the method), and resetting the info record.
#include "common.h"
#include "grouped.h"
#include "kernels.h"

#include <type_traits>

namespace rqlp {

// R = R2 * R1' (R1' = R1 with the rows of dependent columns zeroed, R2 with
// its own dependent rows zeroed), one 16 x 16 output tile per wave with the
// float64 MFMA; written as R (transpose = 0) or as L = R^T (transpose = 1).
template <typename T>
__device__ __attribute__((always_inline)) inline void form_r_body(const double* __restrict__ R2,
                                                                  const double* __restrict__ R1,
                                                                  const int32_t* __restrict__ f1,
                                                                  const int32_t* __restrict__ f2, int d, int dp,
                                                                  T* __restrict__ out, int64_t ldo, int transpose,
                                                                  int bid) {
  const int nT = dp / kTile;
  const int I = bid / nT, J = bid % nT;  // output tile of R
  const int lane = threadIdx.x, lr = lane >> 4, lc = lane & 15;
  doublex4 acc = Mfma<double>::zero();
  // The operands of kFB block columns t are fetched into registers one
  // batch ahead of their products (two batches alternate), so the chain of
  // products waits for a load once per batch rather than once per t; the
  // products run in the order t = I..J, ks = 0..3 all the same.
  constexpr int kFB = 8;
  double pa[2][kFB][4], pb[2][kFB][4];
  auto fetch = [&](auto Bc, int tb) {
    constexpr int B = decltype(Bc)::value;
#pragma unroll
    for (int i = 0; i < kFB; ++i) {
      const int t = tb + i;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int kk = t * kTile + ks * 4 + lr;
        double a = 0.0, b = 0.0;
        if (t <= J) {
          a = R2[(int64_t)(I * kTile + lc) * dp + kk];  // A[m][kk], m = lc
          const double r = R1[(int64_t)kk * dp + J * kTile + lc];
          b = f1[kk] ? 0.0 : r;
        }
        pa[B][i][ks] = a;
        pb[B][i][ks] = b;
      }
    }
  };
  auto run = [&](auto Bc, int tb) {
    constexpr int B = decltype(Bc)::value;
#pragma unroll
    for (int i = 0; i < kFB; ++i) {
      if (tb + i > J) break;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) acc = Mfma<double>::mma(pa[B][i][ks], pb[B][i][ks], acc);
    }
  };
  if (I <= J) {
    using B0 = std::integral_constant<int, 0>;
    using B1 = std::integral_constant<int, 1>;
    fetch(B0{}, I);
    for (int tb = I; tb <= J; tb += 2 * kFB) {
      if (tb + kFB <= J) fetch(B1{}, tb + kFB);
      run(B0{}, tb);
      if (tb + 2 * kFB <= J) fetch(B0{}, tb + 2 * kFB);
      if (tb + kFB <= J) run(B1{}, tb + kFB);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = I * kTile + lr + 4 * r, col = J * kTile + lc;
    if (row < d && col < d) {
      const double v = (row <= col && !f2[row]) ? acc[r] : 0.0;
      if (transpose) out[(int64_t)col * ldo + row] = (T)v;
      else out[(int64_t)row * ldo + col] = (T)v;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(64) void form_r_kernel(const double* __restrict__ R2, const double* __restrict__ R1,
                                                    const int32_t* __restrict__ f1, const int32_t* __restrict__ f2,
                                                    int d, int dp, T* __restrict__ out, int64_t ldo, int transpose) {
  form_r_body<T>(R2, R1, f1, f2, d, dp, out, ldo, transpose, blockIdx.x);
}

struct FormRArgs {
  const double* R2;
  const double* R1;
  const int32_t* f1;
  const int32_t* f2;
  void* out;
  int64_t ldo;
  int d, dp, transpose;
};

template <typename T>
__global__ __launch_bounds__(64) void form_r_grouped(const FormRArgs* __restrict__ a, const int* __restrict__ start,
                                                     int count) {
  const int p = group_find(start, count, blockIdx.x);
  const FormRArgs g = a[p];
  form_r_body<T>(g.R2, g.R1, g.f1, g.f2, g.d, g.dp, (T*)g.out, g.ldo, g.transpose, (int)blockIdx.x - start[p]);
}

template <typename T>
void form_r_grouped_launch(const void* args, const int* start, int count, unsigned blocks, hipStream_t s) {
  hipLaunchKernelGGL(form_r_grouped<T>, dim3(blocks), dim3(64), 0, s, (const FormRArgs*)args, start, count);
}

template <typename T>
hipError_t launch_form_l(const double* R2, const double* R1, const int32_t* flags1, int d, int dp,
                         T* L, int64_t ldl, hipStream_t s) {
  // flags of the second pass follow the first pass's dp flags in memory
  const int nT = dp / kTile;
  const unsigned blocks = (unsigned)(nT * nT);
  if (!record_launch(&form_r_grouped_launch<T>, FormRArgs{R2, R1, flags1, flags1 + dp, L, ldl, d, dp, 1}, blocks))
    hipLaunchKernelGGL(form_r_kernel<T>, dim3(blocks), dim3(64), 0, s, R2, R1, flags1, flags1 + dp, d, dp, L, ldl, 1);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_form_r(const double* R2, const double* R1, const int32_t* flags1, int d, int dp,
                         T* R, int64_t ldr, hipStream_t s) {
  const int nT = dp / kTile;
  hipLaunchKernelGGL(form_r_kernel<T>, dim3(nT * nT), dim3(64), 0, s, R2, R1, flags1, flags1 + dp, d, dp, R,
                     ldr, 0);
  return hipGetLastError();
}
template hipError_t launch_form_l<float>(const double*, const double*, const int32_t*, int, int, float*, int64_t, hipStream_t);
template hipError_t launch_form_l<double>(const double*, const double*, const int32_t*, int, int, double*, int64_t, hipStream_t);
template hipError_t launch_form_r<float>(const double*, const double*, const int32_t*, int, int, float*, int64_t, hipStream_t);
template hipError_t launch_form_r<double>(const double*, const double*, const int32_t*, int, int, double*, int64_t, hipStream_t);

__global__ void info_reset_kernel(DevInfo* info) {
  if (threadIdx.x == 0) {
    info->status = 0;
    info->completed_cols = 0;
    info->breakdown_pass = 0;
    info->nonfinite = 0;
  }
}

hipError_t launch_info_reset(void* info, hipStream_t s) {
  hipLaunchKernelGGL(info_reset_kernel, dim3(1), dim3(64), 0, s, (DevInfo*)info);
  return hipGetLastError();
}

}  // namespace rqlp
