// Sparse A in CSR form (Section III-D: a pass costs O(nnz d)).
//
// SpMM Y = A X: one wave per row of A.  For each stored entry the wave
// gathers one row of X (d values, coalesced across lanes) and accumulates
// in the working precision, entries taken in storage order, so results are
// deterministic.  Four entries are loaded ahead to keep gathers in flight.
//
// Transpose CSR(A) -> CSR(A^T), done once per decomposition, as a stable
// radix sort of the entries by column (see below); bit-exact.
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
// transpose: a stable LSD radix sort of the entries by column index
//
// The entries are visited in CSR order (row-major, rising columns within a
// row).  A stable sort by column therefore leaves the entries of each
// column in rising row order, which is CSR(A^T) with sorted indices, unique
// and bit-exact.  Keys need ceil(log2 n) bits, 8 per pass (two passes for
// n <= 65536).  Each pass: per-tile digit histograms (LDS atomics; counts
// do not depend on order), a scan over (digit, tile), and a scatter in
// which every entry's position is fixed by its digit, its tile and its rank
// among equal digits before it in the tile (wave ballots), so no position
// depends on timing.

constexpr int kRxThreads = 256;
constexpr int kRxItems = 16;                       // per thread
constexpr int kRxTile = kRxThreads * kRxItems;     // entries per tile
constexpr int kRxWaveItems = kRxTile / (kRxThreads / 64);

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// rowid[e] = i for the entries e of row i (one wave per row)
__global__ __launch_bounds__(256) void expand_rows_kernel(const int32_t* __restrict__ rowptr, int64_t m,
                                                          int32_t* __restrict__ rowid) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= m) return;
  const int lane = threadIdx.x & 63;
  for (int e = rowptr[i] + lane; e < rowptr[i + 1]; e += 64) rowid[e] = (int32_t)i;
}

// hist[digit * ntiles + tile] = number of entries of the tile with that digit
__global__ __launch_bounds__(kRxThreads) void radix_hist_kernel(const int32_t* __restrict__ keys, int64_t nnz,
                                                                 int shift, int ntiles, int32_t* __restrict__ hist) {
  __shared__ int32_t h[256];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRxTile;
#pragma unroll
  for (int i = 0; i < kRxItems; ++i) {
    const int64_t e = base + i * kRxThreads + tid;
    if (e < nnz) atomicAdd(&h[(keys[e] >> shift) & 255], 1);
  }
  __syncthreads();
  hist[(int64_t)tid * ntiles + blockIdx.x] = h[tid];
}

// Exclusive scan of hist in (digit, tile) order.  Pass 1 (one workgroup per
// digit): scan of the digit's tiles in place, total to tot[digit].
__global__ __launch_bounds__(256) void radix_scan_tiles_kernel(int32_t* __restrict__ hist, int ntiles,
                                                               int32_t* __restrict__ tot) {
  __shared__ int32_t part[256];
  int32_t* h = hist + (int64_t)blockIdx.x * ntiles;
  const int tid = threadIdx.x;
  int32_t carry = 0;
  for (int c0 = 0; c0 < ntiles; c0 += 256) {
    const int i = c0 + tid;
    const int32_t v = (i < ntiles) ? h[i] : 0;
    part[tid] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int32_t u = (tid >= off) ? part[tid - off] : 0;
      __syncthreads();
      part[tid] += u;
      __syncthreads();
    }
    if (i < ntiles) h[i] = carry + part[tid] - v;
    carry += part[255];
    __syncthreads();
  }
  if (tid == 0) tot[blockIdx.x] = carry;
}

// Pass 2: base[digit] = exclusive scan of tot (one workgroup of 256).
__global__ __launch_bounds__(256) void radix_scan_digits_kernel(const int32_t* __restrict__ tot,
                                                                int32_t* __restrict__ base) {
  __shared__ int32_t part[256];
  const int tid = threadIdx.x;
  const int32_t v = tot[tid];
  part[tid] = v;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int32_t u = (tid >= off) ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += u;
    __syncthreads();
  }
  base[tid] = part[tid] - v;
}

// Stable scatter of one pass.  Wave w of a tile owns entries
// [w * kRxWaveItems, (w + 1) * kRxWaveItems) of the tile and walks them in
// rounds of 64 consecutive entries; within a round a lane's rank among the
// lanes with the same digit comes from eight ballots.  The tile is then
// reordered by digit in LDS, so that the global writes of each digit's run
// come from consecutive threads (coalesced) instead of from scattered lanes.
template <typename T>
__global__ __launch_bounds__(kRxThreads) void radix_scatter_kernel(
    const int32_t* __restrict__ kin, const int32_t* __restrict__ rin, const T* __restrict__ vin, int64_t nnz,
    int shift, int ntiles, const int32_t* __restrict__ hist, const int32_t* __restrict__ base,
    int32_t* __restrict__ kout, int32_t* __restrict__ rout, T* __restrict__ vout) {
  __shared__ int32_t cnt[kRxThreads / 64][256];
  __shared__ int32_t tdo[256];   // exclusive offset of each digit within the tile
  __shared__ int32_t gofs[256];  // global position of each digit's run
  __shared__ int32_t sk[kRxTile], sr[kRxTile];
  __shared__ T sv[kRxTile];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int i = tid; i < (kRxThreads / 64) * 256; i += kRxThreads) (&cnt[0][0])[i] = 0;
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * kRxTile;
  const int64_t e0 = t0 + (int64_t)wave * kRxWaveItems;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int32_t key[kRxItems], row[kRxItems], rank[kRxItems];
  T val[kRxItems];
#pragma unroll
  for (int r = 0; r < kRxItems; ++r) {
    const int64_t e = e0 + r * 64 + lane;
    const bool ok = e < nnz;
    key[r] = ok ? kin[e] : 0;
    row[r] = ok ? rin[e] : 0;
    val[r] = ok ? vin[e] : (T)0;
  }
#pragma unroll
  for (int r = 0; r < kRxItems; ++r) {
    const bool ok = e0 + r * 64 + lane < nnz;
    const int dg = (key[r] >> shift) & 255;
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bb = __ballot((dg >> b) & 1);
      peers &= ((dg >> b) & 1) ? bb : ~bb;
    }
    const int pre = cnt[wave][dg];  // entries of this digit in earlier rounds
    rank[r] = pre + __popcll(peers & below);
    __builtin_amdgcn_wave_barrier();
    if (ok && (peers & below) == 0) cnt[wave][dg] = pre + __popcll(peers);  // the group's first lane
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  int32_t total;
  {  // per digit (thread tid): exclusive prefix over the waves, and the tile total
    int32_t run = 0;
#pragma unroll
    for (int w = 0; w < kRxThreads / 64; ++w) {
      const int32_t c = cnt[w][tid];
      cnt[w][tid] = run;
      run += c;
    }
    total = run;
    tdo[tid] = total;
  }
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {  // inclusive scan of the totals over digits
    const int32_t u = (tid >= off) ? tdo[tid - off] : 0;
    __syncthreads();
    tdo[tid] += u;
    __syncthreads();
  }
  tdo[tid] -= total;  // exclusive
  gofs[tid] = base[tid] + hist[(int64_t)tid * ntiles + blockIdx.x];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRxItems; ++r) {
    if (e0 + r * 64 + lane < nnz) {
      const int dg = (key[r] >> shift) & 255;
      const int lp = tdo[dg] + cnt[wave][dg] + rank[r];
      sk[lp] = key[r];
      sr[lp] = row[r];
      sv[lp] = val[r];
    }
  }
  __syncthreads();
  const int n_tile = (int)min((int64_t)kRxTile, nnz - t0);
  for (int j = tid; j < n_tile; j += kRxThreads) {
    const int32_t k = sk[j];
    const int dg = (k >> shift) & 255;
    const int64_t pos = (int64_t)gofs[dg] + (j - tdo[dg]);
    kout[pos] = k;
    rout[pos] = sr[j];
    vout[pos] = sv[j];
  }
}

// rowptr_t from the sorted keys: rowptr_t[c] = first position with key >= c.
__global__ __launch_bounds__(256) void rowptr_from_keys_kernel(const int32_t* __restrict__ keys, int64_t nnz,
                                                               int64_t n, int32_t* __restrict__ rowptr_t) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p <= nnz; p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t lo = (p == 0) ? -1 : keys[p - 1];
    const int64_t hi = (p == nnz) ? n : keys[p];
    // clamped to [0, n]: column indices outside [0, n) cannot write out of bounds
    for (int64_t c = max(lo + 1, (int64_t)0); c <= min(hi, n); ++c) rowptr_t[c] = (int32_t)p;
  }
}

static int radix_passes(int64_t n) {
  int bits = 0;
  while (bits < 31 && ((int64_t)1 << bits) < n) ++bits;
  return std::max(1, (bits + 7) / 8);
}

size_t csr_transpose_scratch_bytes(int64_t m, int64_t n, int64_t nnz) {
  (void)m;
  (void)n;
  const int64_t ntiles = std::max<int64_t>(1, ceil_div(nnz, kRxTile));
  const size_t a = (size_t)round_up(nnz * sizeof(int32_t), 256);
  const size_t v = (size_t)round_up(nnz * sizeof(double), 256);
  return 5 * a + 2 * v + (size_t)round_up(256 * ntiles * sizeof(int32_t), 256) + 2 * 256 * sizeof(int32_t) + 256;
}

template <typename T>
hipError_t launch_csr_transpose(const int32_t* rowptr, const int32_t* colidx, const T* vals,
                                int64_t m, int64_t n, int64_t nnz, int32_t* rowptr_t,
                                int32_t* colidx_t, T* vals_t, void* scratch, hipStream_t s) {
  if (nnz <= 0) {
    const unsigned g = (unsigned)std::min<int64_t>(std::max<int64_t>(1, ceil_div(n + 1, 256)), 65535);
    hipLaunchKernelGGL(fill_i32_kernel, dim3(g), dim3(256), 0, s, rowptr_t, n + 1, 0);
    return hipGetLastError();
  }
  const int64_t ntiles = ceil_div(nnz, kRxTile);
  char* p = (char*)scratch;
  auto take = [&](size_t bytes) { void* q = p; p += round_up(bytes, 256); return q; };
  int32_t* rowid = (int32_t*)take(nnz * sizeof(int32_t));
  int32_t* kA = (int32_t*)take(nnz * sizeof(int32_t));
  int32_t* rA = (int32_t*)take(nnz * sizeof(int32_t));
  T* vA = (T*)take(nnz * sizeof(double));
  int32_t* kB = (int32_t*)take(nnz * sizeof(int32_t));
  int32_t* rB = (int32_t*)take(nnz * sizeof(int32_t));
  T* vB = (T*)take(nnz * sizeof(double));
  int32_t* hist = (int32_t*)take(256 * ntiles * sizeof(int32_t));
  int32_t* tot = (int32_t*)p;
  int32_t* base = tot + 256;

  hipLaunchKernelGGL(expand_rows_kernel, dim3((unsigned)ceil_div(m, 4)), dim3(256), 0, s, rowptr, m, rowid);
  const int P = radix_passes(n);
  const int32_t* kin = colidx;
  const int32_t* rin = rowid;
  const T* vin = vals;
  for (int pass = 0; pass < P; ++pass) {
    const bool last = pass == P - 1;
    int32_t* kout = (pass & 1) ? kB : kA;
    int32_t* rout = last ? colidx_t : ((pass & 1) ? rB : rA);
    T* vout = last ? vals_t : ((pass & 1) ? vB : vA);
    const int shift = 8 * pass;
    hipLaunchKernelGGL(radix_hist_kernel, dim3((unsigned)ntiles), dim3(kRxThreads), 0, s, kin, nnz, shift,
                       (int)ntiles, hist);
    hipLaunchKernelGGL(radix_scan_tiles_kernel, dim3(256), dim3(256), 0, s, hist, (int)ntiles, tot);
    hipLaunchKernelGGL(radix_scan_digits_kernel, dim3(1), dim3(256), 0, s, tot, base);
    hipLaunchKernelGGL((radix_scatter_kernel<T>), dim3((unsigned)ntiles), dim3(kRxThreads), 0, s, kin, rin, vin,
                       nnz, shift, (int)ntiles, hist, base, kout, rout, vout);
    kin = kout;
    rin = rout;
    vin = vout;
  }
  const unsigned gp = (unsigned)std::min<int64_t>(ceil_div(nnz + 1, 256), 65535);
  hipLaunchKernelGGL(rowptr_from_keys_kernel, dim3(gp), dim3(256), 0, s, kin, nnz, n, rowptr_t);
  return hipGetLastError();
}
template hipError_t launch_csr_transpose<float>(const int32_t*, const int32_t*, const float*, int64_t, int64_t,
                                                int64_t, int32_t*, int32_t*, float*, void*, hipStream_t);
template hipError_t launch_csr_transpose<double>(const int32_t*, const int32_t*, const double*, int64_t, int64_t,
                                                 int64_t, int32_t*, int32_t*, double*, void*, hipStream_t);

}  // namespace rqlp
