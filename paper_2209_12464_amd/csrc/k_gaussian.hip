// Gaussian test matrix: out[i][j] (rows x cols, leading dimension ldo) is the
// normal with logical index l = j*rows + i of the Philox stream
// (seed, key1); columns [cols, ldo) are zeroed.  One thread per Philox block
// (four consecutive logical indices).
#include "common.h"
#include "kernels.h"

namespace rqlp {

template <typename T>
__global__ __launch_bounds__(256) void gaussian_kernel(uint64_t seed, uint64_t key1, int64_t rows,
                                                       int64_t cols, T* __restrict__ out,
                                                       int64_t ldo) {
  const int64_t total = rows * cols;
  const int64_t nblk = (total + 3) >> 2;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nblk;
       c += (int64_t)gridDim.x * blockDim.x) {
    u64x4 ctr = {(uint64_t)c, 0, 0, 0};
    const u64x4 w = philox4x64_10(ctr, seed, key1);
    double z[4];
    box_muller(w.x0, w.x1, z[0], z[1]);
    box_muller(w.x2, w.x3, z[2], z[3]);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t l = 4 * c + t;
      if (l < total) {
        const int64_t j = l / rows, i = l - j * rows;
        out[i * ldo + j] = (T)z[t];
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void zero_cols_kernel(T* __restrict__ out, int64_t rows,
                                                        int64_t c0, int64_t c1, int64_t ld) {
  const int64_t w = c1 - c0;
  const int64_t total = rows * w;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / w, j = c0 + (e - i * w);
    out[i * ld + j] = (T)0;
  }
}

template <typename T>
hipError_t launch_gaussian(uint64_t seed, uint64_t key1, int64_t rows, int64_t cols, T* out,
                           int64_t ldo, hipStream_t s) {
  const int64_t nblk = (rows * cols + 3) / 4;
  if (nblk > 0) {
    const int64_t g = ceil_div(nblk, 256);
    hipLaunchKernelGGL(gaussian_kernel<T>, dim3((unsigned)(g < 65536 ? g : 65536)), dim3(256), 0, s,
                       seed, key1, rows, cols, out, ldo);
  }
  if (ldo > cols && rows > 0) {
    const int64_t tot = rows * (ldo - cols);
    const int64_t g = ceil_div(tot, 256);
    hipLaunchKernelGGL(zero_cols_kernel<T>, dim3((unsigned)(g < 65536 ? g : 65536)), dim3(256), 0, s,
                       out, rows, cols, ldo, ldo);
  }
  return hipGetLastError();
}

template hipError_t launch_gaussian<float>(uint64_t, uint64_t, int64_t, int64_t, float*, int64_t, hipStream_t);
template hipError_t launch_gaussian<double>(uint64_t, uint64_t, int64_t, int64_t, double*, int64_t, hipStream_t);

template <typename T>
hipError_t launch_zero_cols(T* out, int64_t rows, int64_t c0, int64_t c1, int64_t ld, hipStream_t s) {
  if (c1 <= c0 || rows <= 0) return hipSuccess;
  const int64_t g = ceil_div(rows * (c1 - c0), 256);
  hipLaunchKernelGGL(zero_cols_kernel<T>, dim3((unsigned)(g < 65536 ? g : 65536)), dim3(256), 0, s,
                     out, rows, c0, c1, ld);
  return hipGetLastError();
}
template hipError_t launch_zero_cols<float>(float*, int64_t, int64_t, int64_t, int64_t, hipStream_t);
template hipError_t launch_zero_cols<double>(double*, int64_t, int64_t, int64_t, int64_t, hipStream_t);

}  // namespace rqlp
