// Small d x d steps: combining the two CholeskyQR factors into the R factor
// of the unpivoted QR (R = R2 R1), forming L = R^T of the last QR (the
// L-values of the method), and resetting the info record.
#include "common.h"
#include "kernels.h"

namespace rqlp {

// Entry (a, b), a <= b < d, of R2 * R1' (R1' = R1 with dependent rows zero).
__device__ inline double r_entry(const double* R2, const double* R1, const int32_t* f1,
                                 const int32_t* f2, int dp, int a, int b) {
  if (f2[a]) return 0.0;
  double s = 0.0;
  for (int t = a; t <= b; ++t)
    if (!f1[t]) s += R2[(int64_t)a * dp + t] * R1[(int64_t)t * dp + b];
  return s;
}

template <typename T>
__global__ __launch_bounds__(256) void form_l_kernel(const double* __restrict__ R2,
                                                     const double* __restrict__ R1,
                                                     const int32_t* __restrict__ f1,
                                                     const int32_t* __restrict__ f2, int d, int dp,
                                                     T* __restrict__ L, int64_t ldl, int transpose) {
  const int64_t total = (int64_t)d * d;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / d), j = (int)(e % d);
    double v = 0.0;
    if (transpose) {  // L[i][j] = R[j][i], lower triangular
      if (j <= i) v = r_entry(R2, R1, f1, f2, dp, j, i);
    } else {          // R[i][j], upper triangular
      if (i <= j) v = r_entry(R2, R1, f1, f2, dp, i, j);
    }
    L[(int64_t)i * ldl + j] = (T)v;
  }
}

template <typename T>
hipError_t launch_form_l(const double* R2, const double* R1, const int32_t* flags1, int d, int dp,
                         T* L, int64_t ldl, hipStream_t s) {
  // flags of the second pass follow the first pass's dp flags in memory
  const int64_t g = ceil_div((int64_t)d * d, 256);
  hipLaunchKernelGGL(form_l_kernel<T>, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(256), 0, s, R2, R1,
                     flags1, flags1 + dp, d, dp, L, ldl, 1);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_form_r(const double* R2, const double* R1, const int32_t* flags1, int d, int dp,
                         T* R, int64_t ldr, hipStream_t s) {
  const int64_t g = ceil_div((int64_t)d * d, 256);
  hipLaunchKernelGGL(form_l_kernel<T>, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(256), 0, s, R2, R1,
                     flags1, flags1 + dp, d, dp, R, ldr, 0);
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
