// Gaussian test matrix: out[i][j] (rows x cols, leading dimension ldo) is the
// normal with logical index l = j*rows + i of the Philox stream
// (seed, key1); columns [cols, ldo) are zeroed.  Each Philox block gives
// four consecutive logical indices, i.e. four consecutive rows of one
// column.  A workgroup takes a 64 x 16 tile: it computes the blocks that
// cover the tile's columns (a block straddling two tiles is computed by
// both and each keeps its part) into LDS, then writes the tile row by row,
// 16 consecutive columns per row, so the stores are coalesced.
#include "common.h"
#include "grouped.h"
#include "kernels.h"

namespace rqlp {

struct GaussianArgs {
  uint64_t seed, key1;
  int64_t rows, cols, ldo;
  void* out;
};

constexpr int kGsR = 64, kGsC = 16;  // tile rows x columns
constexpr int kGsB = kGsR / 4 + 1;    // Philox blocks that can touch one column of a tile

template <typename T>
__device__ __attribute__((always_inline)) inline void gaussian_body(uint64_t seed, uint64_t key1, int64_t rows,
                                                                    int64_t cols, T* __restrict__ out, int64_t ldo,
                                                                    int bid, int nblk_grid) {
  __shared__ double tile[kGsR][kGsC + 1];
  const int tid = threadIdx.x;
  const int64_t ntr = (rows + kGsR - 1) / kGsR, ntc = (ldo + kGsC - 1) / kGsC;
  for (int64_t tb = bid; tb < ntr * ntc; tb += nblk_grid) {
    const int64_t tc = tb % ntc, tr = tb / ntc;  // neighbouring workgroups share rows
    const int64_t i0 = tr * kGsR, j0 = tc * kGsC;
    const int64_t i1 = i0 + kGsR < rows ? i0 + kGsR : rows;
    for (int q = tid; q < kGsC * kGsB; q += blockDim.x) {
      const int jj = q / kGsB, kb = q - jj * kGsB;
      const int64_t j = j0 + jj;
      if (j >= cols) continue;
      const int64_t l0 = j * rows + i0, l1 = j * rows + i1;  // this column's logical indices in the tile
      const int64_t c = (l0 >> 2) + kb;
      if (4 * c >= l1) continue;
      u64x4 ctr = {(uint64_t)c, 0, 0, 0};
      const u64x4 w = philox4x64_10(ctr, seed, key1);
      double z[4];
      box_muller(w.x0, w.x1, z[0], z[1]);
      box_muller(w.x2, w.x3, z[2], z[3]);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t l = 4 * c + t;
        if (l >= l0 && l < l1) tile[l - l0][jj] = z[t];
      }
    }
    __syncthreads();
    const int jj = tid & (kGsC - 1);
    const int64_t j = j0 + jj;
    for (int r = tid / kGsC; r < kGsR; r += blockDim.x / kGsC) {
      const int64_t i = i0 + r;
      if (i < rows && j < ldo) out[i * ldo + j] = (j < cols) ? (T)tile[r][jj] : (T)0;
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(256) void gaussian_kernel(uint64_t seed, uint64_t key1, int64_t rows, int64_t cols,
                                                       T* __restrict__ out, int64_t ldo) {
  gaussian_body<T>(seed, key1, rows, cols, out, ldo, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ __launch_bounds__(256) void gaussian_grouped(const GaussianArgs* __restrict__ a,
                                                        const int* __restrict__ start, int count) {
  const int p = group_find(start, count, blockIdx.x);
  const GaussianArgs g = a[p];
  gaussian_body<T>(g.seed, g.key1, g.rows, g.cols, (T*)g.out, g.ldo, blockIdx.x - start[p], start[p + 1] - start[p]);
}

template <typename T>
void gaussian_grouped_launch(const void* args, const int* start, int count, unsigned blocks, hipStream_t s) {
  hipLaunchKernelGGL(gaussian_grouped<T>, dim3(blocks), dim3(256), 0, s, (const GaussianArgs*)args, start, count);
}

struct ZeroColsArgs {
  int64_t rows, c0, c1, ld;
  void* out;
};

template <typename T>
__device__ __attribute__((always_inline)) inline void zero_cols_body(T* __restrict__ out, int64_t rows, int64_t c0,
                                                                     int64_t c1, int64_t ld, int bid, int nblk) {
  const int64_t w = c1 - c0;
  const int64_t total = rows * w;
  for (int64_t e = bid * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)nblk * blockDim.x) {
    const int64_t i = e / w, j = c0 + (e - i * w);
    out[i * ld + j] = (T)0;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void zero_cols_kernel(T* __restrict__ out, int64_t rows, int64_t c0, int64_t c1,
                                                        int64_t ld) {
  zero_cols_body<T>(out, rows, c0, c1, ld, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ __launch_bounds__(256) void zero_cols_grouped(const ZeroColsArgs* __restrict__ a,
                                                         const int* __restrict__ start, int count) {
  const int p = group_find(start, count, blockIdx.x);
  const ZeroColsArgs g = a[p];
  zero_cols_body<T>((T*)g.out, g.rows, g.c0, g.c1, g.ld, blockIdx.x - start[p], start[p + 1] - start[p]);
}

template <typename T>
void zero_cols_grouped_launch(const void* args, const int* start, int count, unsigned blocks, hipStream_t s) {
  hipLaunchKernelGGL(zero_cols_grouped<T>, dim3(blocks), dim3(256), 0, s, (const ZeroColsArgs*)args, start, count);
}

template <typename T>
static void zero_cols_dispatch(T* out, int64_t rows, int64_t c0, int64_t c1, int64_t ld, hipStream_t s) {
  const int64_t g = ceil_div(rows * (c1 - c0), 256);
  const unsigned blocks = (unsigned)(g < 65536 ? g : 65536);
  if (!record_launch(&zero_cols_grouped_launch<T>, ZeroColsArgs{rows, c0, c1, ld, out}, blocks))
    hipLaunchKernelGGL(zero_cols_kernel<T>, dim3(blocks), dim3(256), 0, s, out, rows, c0, c1, ld);
}

template <typename T>
hipError_t launch_gaussian(uint64_t seed, uint64_t key1, int64_t rows, int64_t cols, T* out,
                           int64_t ldo, hipStream_t s) {
  if (rows > 0 && cols > 0) {  // the tiles cover [0, ldo): padding columns are written as zero
    const int64_t g = ceil_div(rows, kGsR) * ceil_div(ldo, kGsC);
    const unsigned blocks = (unsigned)(g < 65536 ? g : 65536);
    if (!record_launch(&gaussian_grouped_launch<T>, GaussianArgs{seed, key1, rows, cols, ldo, out}, blocks))
      hipLaunchKernelGGL(gaussian_kernel<T>, dim3(blocks), dim3(256), 0, s, seed, key1, rows, cols, out, ldo);
  } else if (ldo > cols && rows > 0) {
    zero_cols_dispatch<T>(out, rows, cols, ldo, ldo, s);
  }
  return hipGetLastError();
}

template hipError_t launch_gaussian<float>(uint64_t, uint64_t, int64_t, int64_t, float*, int64_t, hipStream_t);
template hipError_t launch_gaussian<double>(uint64_t, uint64_t, int64_t, int64_t, double*, int64_t, hipStream_t);

template <typename T>
hipError_t launch_zero_cols(T* out, int64_t rows, int64_t c0, int64_t c1, int64_t ld, hipStream_t s) {
  if (c1 <= c0 || rows <= 0) return hipSuccess;
  zero_cols_dispatch<T>(out, rows, c0, c1, ld, s);
  return hipGetLastError();
}
template hipError_t launch_zero_cols<float>(float*, int64_t, int64_t, int64_t, int64_t, hipStream_t);
template hipError_t launch_zero_cols<double>(double*, int64_t, int64_t, int64_t, int64_t, hipStream_t);

}  // namespace rqlp
