// Sparse A in CSR form (Section III-D: a pass costs O(nnz d)).
//
// SpMM Y = A X: one wave per row of A.  For each stored entry the wave
// gathers one row of X (d values, coalesced across lanes) and accumulates
// in the working precision, entries taken in storage order, so results are
// deterministic.  Four entries are loaded ahead to keep gathers in flight.
//
// Transpose CSR(A) -> CSR(A^T), done once per decomposition: column
// histogram (integer atomics), one-workgroup exclusive scan, scatter with
// per-column cursors (order within a column depends on timing), then each
// output row is put in increasing order of the original row index by
// ranking (keys are unique), which makes the result unique and bit-exact.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace rqlp {

constexpr int kSpmmWaves = 4;
constexpr int kSpmmCols = 4;  // columns per lane: d <= 256

template <typename T>
__global__ __launch_bounds__(kSpmmWaves * 64) void spmm_kernel(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
    const T* __restrict__ vals, int64_t rows, const T* __restrict__ X, int64_t ldx, int d,
    T* __restrict__ Y, int64_t ldy, int nst) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * kSpmmWaves + (threadIdx.x >> 6);
  if (row >= rows) return;
  const int e0 = rowptr[row], e1 = rowptr[row + 1];
  T acc[kSpmmCols];
#pragma unroll
  for (int j = 0; j < kSpmmCols; ++j) acc[j] = (T)0;
  int e = e0;
  for (; e + 4 <= e1; e += 4) {
    int c[4];
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      c[u] = colidx[e + u];
      v[u] = vals[e + u];
    }
    T x[4][kSpmmCols];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < kSpmmCols; ++j) {
        const int col = lane + 64 * j;
        x[u][j] = (col < d) ? X[(int64_t)c[u] * ldx + col] : (T)0;
      }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < kSpmmCols; ++j) acc[j] += v[u] * x[u][j];
  }
  for (; e < e1; ++e) {
    const int c = colidx[e];
    const T v = vals[e];
#pragma unroll
    for (int j = 0; j < kSpmmCols; ++j) {
      const int col = lane + 64 * j;
      if (col < d) acc[j] += v * X[(int64_t)c * ldx + col];
    }
  }
#pragma unroll
  for (int j = 0; j < kSpmmCols; ++j) {
    const int col = lane + 64 * j;
    if (col < nst) Y[row * ldy + col] = (col < d) ? acc[j] : (T)0;
  }
}

template <typename T>
hipError_t launch_spmm(const int32_t* rowptr, const int32_t* colidx, const T* vals, int64_t rows,
                       const T* X, int64_t ldx, int d, T* Y, int64_t ldy, int nst, hipStream_t s,
                       hipEvent_t ev0, hipEvent_t ev1) {
  if (rows <= 0) return hipSuccess;
  if (ev0) (void)hipEventRecord(ev0, s);
  hipLaunchKernelGGL(spmm_kernel<T>, dim3((unsigned)ceil_div(rows, kSpmmWaves)), dim3(kSpmmWaves * 64), 0, s,
                     rowptr, colidx, vals, rows, X, ldx, d, Y, ldy, nst);
  if (ev1) (void)hipEventRecord(ev1, s);
  return hipGetLastError();
}
template hipError_t launch_spmm<float>(const int32_t*, const int32_t*, const float*, int64_t, const float*,
                                       int64_t, int, float*, int64_t, int, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_spmm<double>(const int32_t*, const int32_t*, const double*, int64_t, const double*,
                                        int64_t, int, double*, int64_t, int, hipStream_t, hipEvent_t, hipEvent_t);

// ---------------------------------------------------------------------------
// transpose

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ __launch_bounds__(256) void col_count_kernel(const int32_t* __restrict__ colidx, int64_t nnz,
                                                        int32_t* __restrict__ cnt) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&cnt[colidx[e]], 1);
}

// rowptr_t[0] = 0, rowptr_t[j+1] = cnt[0] + ... + cnt[j]; one workgroup.
__global__ __launch_bounds__(1024) void excl_scan_kernel(const int32_t* __restrict__ cnt, int64_t n,
                                                         int32_t* __restrict__ out) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = ceil_div(n, 1024);
  const int64_t b = t * per, e = min(n, b + per);
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += cnt[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t v = (t >= off) ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = (t == 0) ? 0 : part[t - 1];
  if (t == 0) out[0] = 0;
  for (int64_t i = b; i < e; ++i) {
    run += cnt[i];
    out[i + 1] = (int32_t)run;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void scatter_kernel(const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ colidx,
                                                      const T* __restrict__ vals, int64_t m,
                                                      const int32_t* __restrict__ rowptr_t,
                                                      int32_t* __restrict__ cursor,
                                                      int32_t* __restrict__ tmp_idx, T* __restrict__ tmp_val) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      const int c = colidx[e];
      const int pos = rowptr_t[c] + atomicAdd(&cursor[c], 1);
      tmp_idx[pos] = (int32_t)i;
      tmp_val[pos] = vals[e];
    }
  }
}

// One wave per output row: entry with key k goes to position
// (number of keys in the row smaller than k).
template <typename T>
__global__ __launch_bounds__(256) void rank_sort_kernel(const int32_t* __restrict__ rowptr_t, int64_t n,
                                                        const int32_t* __restrict__ tmp_idx,
                                                        const T* __restrict__ tmp_val,
                                                        int32_t* __restrict__ colidx_t, T* __restrict__ vals_t) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  const int b = rowptr_t[j], e = rowptr_t[j + 1];
  for (int p = b + lane; p < e; p += 64) {
    const int key = tmp_idx[p];
    int rank = 0;
    for (int f = b; f < e; ++f) rank += (tmp_idx[f] < key) ? 1 : 0;
    colidx_t[b + rank] = key;
    vals_t[b + rank] = tmp_val[p];
  }
}

size_t csr_transpose_scratch_bytes(int64_t m, int64_t n, int64_t nnz) {
  (void)m;
  return (size_t)round_up(2 * n * sizeof(int32_t), 256) + (size_t)round_up(nnz * sizeof(int32_t), 256) +
         (size_t)round_up(nnz * sizeof(double), 256);
}

template <typename T>
hipError_t launch_csr_transpose(const int32_t* rowptr, const int32_t* colidx, const T* vals,
                                int64_t m, int64_t n, int64_t nnz, int32_t* rowptr_t,
                                int32_t* colidx_t, T* vals_t, void* scratch, hipStream_t s) {
  char* p = (char*)scratch;
  int32_t* cnt = (int32_t*)p;            // n
  int32_t* cursor = cnt + n;             // n
  p += round_up(2 * n * sizeof(int32_t), 256);
  int32_t* tmp_idx = (int32_t*)p;
  p += round_up(nnz * sizeof(int32_t), 256);
  T* tmp_val = (T*)p;
  const unsigned gn = (unsigned)std::min<int64_t>(ceil_div(2 * n, 256), 65535);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(gn > 0 ? gn : 1), dim3(256), 0, s, cnt, 2 * n, 0);
  if (nnz > 0) {
    const unsigned ge = (unsigned)std::min<int64_t>(ceil_div(nnz, 256), 65535);
    hipLaunchKernelGGL(col_count_kernel, dim3(ge), dim3(256), 0, s, colidx, nnz, cnt);
  }
  hipLaunchKernelGGL(excl_scan_kernel, dim3(1), dim3(1024), 0, s, cnt, n, rowptr_t);
  if (nnz > 0) {
    const unsigned gm = (unsigned)std::min<int64_t>(ceil_div(m, 256), 65535);
    hipLaunchKernelGGL(scatter_kernel<T>, dim3(gm), dim3(256), 0, s, rowptr, colidx, vals, m, rowptr_t,
                       cursor, tmp_idx, tmp_val);
    hipLaunchKernelGGL(rank_sort_kernel<T>, dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, s, rowptr_t, n,
                       tmp_idx, tmp_val, colidx_t, vals_t);
  }
  return hipGetLastError();
}
template hipError_t launch_csr_transpose<float>(const int32_t*, const int32_t*, const float*, int64_t, int64_t,
                                                int64_t, int32_t*, int32_t*, float*, void*, hipStream_t);
template hipError_t launch_csr_transpose<double>(const int32_t*, const int32_t*, const double*, int64_t, int64_t,
                                                 int64_t, int32_t*, int32_t*, double*, void*, hipStream_t);

}  // namespace rqlp
