// Gram matrix G = Y^T Y in float64, the first step of each CholeskyQR pass.
// Float inputs are widened to double: a product of two floats is exact in
// double, so only the summation rounds.  A float32-arithmetic variant
// (inputs rounded to float, float32 MFMA within a row chunk, chunk sums in
// float64) serves the second pass of the bfloat16 form, whose basis is
// orthonormal to working accuracy (G = I + E, E small), so that float32
// rounding of the Gram entries is far below the form's own error.  The d x d upper triangle is cut
// into 64 x 64 tiles and the rows of Y into chunks; each workgroup forms one
// tile over one chunk with the float64 MFMA (16x16x4), and a second kernel
// adds the chunk partials in a fixed order (deterministic) and mirrors the
// result into the lower triangle.
#include "common.h"
#include "grouped.h"
#include "kernels.h"

#include <algorithm>

namespace rqlp {

constexpr int kGT = 64;   // output tile side
constexpr int kGK = 32;   // rows of Y per LDS step

__device__ inline void tile_pair(int p, int& I, int& J) {
  // p enumerates (I, J), I <= J, row by row of the upper triangle of a t x t grid
  // via J = floor((sqrt(8p+1)-1)/2): pairs are listed as J-major.
  int j = (int)((sqrtf(8.0f * p + 1.0f) - 1.0f) * 0.5f);
  while ((j + 1) * (j + 2) / 2 <= p) ++j;
  while (j * (j + 1) / 2 > p) --j;
  J = j;
  I = p - j * (j + 1) / 2;
}

template <typename T, typename C>
__device__ __attribute__((always_inline)) inline void gram_partial_body(const T* __restrict__ Y, int64_t ldy,
                                                                        int64_t rows, int d, int dp,
                                                                        int64_t chunk_rows, int npairs,
                                                                        double* __restrict__ P, int bid) {
  // rows of kGT + 1 doubles, or kGT + 16 floats: the two k-rows one operand
  // read touches fall in disjoint banks
  constexpr int LS = sizeof(C) == 8 ? kGT + 1 : kGT + 16;
  __shared__ C YI[2][kGK][LS];
  __shared__ C YJ[2][kGK][LS];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int pair = bid % npairs;
  const int chunk = bid / npairs;
  int I, J;
  tile_pair(pair, I, J);
  const int64_t r0 = (int64_t)chunk * chunk_rows;
  const int64_t r1 = min(rows, r0 + chunk_rows);
  const int wi = wave >> 1, wj = wave & 1;
  typename Mfma<C>::acc_t acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<C>::zero();

  // The prefetch registers hold the raw inputs: widening to double happens
  // at the LDS store, so the loads stay in flight across the MFMA loop.
  constexpr int PER = kGK * kGT / 256;  // elements per thread per tile
  T ri[PER], rj[PER];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = tid + 256 * i;
      const int kr = idx / kGT, c = idx % kGT;
      const int64_t r = k0 + kr;
      const int ci = I * kGT + c, cj = J * kGT + c;
      ri[i] = (r < r1 && ci < d) ? Y[r * ldy + ci] : (T)0;
      rj[i] = (r < r1 && cj < d) ? Y[r * ldy + cj] : (T)0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = tid + 256 * i;
      YI[buf][idx / kGT][idx % kGT] = (C)ri[i];
      YJ[buf][idx / kGT][idx % kGT] = (C)rj[i];
    }
  };

  if (r0 < r1) {
    load(r0);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int64_t k0 = r0; k0 < r1; k0 += kGK) {
      const bool more = k0 + kGK < r1;
      if (more) load(k0 + kGK);
#pragma unroll
      for (int ks = 0; ks < kGK / 4; ++ks) {
        C a[2], b[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          a[t] = YI[buf][ks * 4 + lane / 16][wi * 32 + t * 16 + (lane & 15)];
          b[t] = YJ[buf][ks * 4 + lane / 16][wj * 32 + t * 16 + (lane & 15)];
        }
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) acc[x][y] = Mfma<C>::mma(a[x], b[y], acc[x][y]);
      }
      if (more) store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
  double* Pc = P + (int64_t)chunk * dp * dp;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = I * kGT + wi * 32 + x * 16 + Mfma<C>::row(lane, r);
        const int col = J * kGT + wj * 32 + y * 16 + Mfma<C>::col(lane);
        if (row < dp && col < dp) Pc[(int64_t)row * dp + col] = (double)acc[x][y][r];
      }
}

template <typename T, typename C>
__global__ __launch_bounds__(256) void gram_partial_kernel(const T* __restrict__ Y, int64_t ldy, int64_t rows, int d,
                                                           int dp, int64_t chunk_rows, int npairs,
                                                           double* __restrict__ P) {
  gram_partial_body<T, C>(Y, ldy, rows, d, dp, chunk_rows, npairs, P, blockIdx.x);
}

struct GramPartialArgs {
  const void* Y;
  double* P;
  int64_t ldy, rows, chunk_rows;
  int d, dp, npairs;
};

template <typename T, typename C>
__global__ __launch_bounds__(256) void gram_partial_grouped(const GramPartialArgs* __restrict__ a,
                                                            const int* __restrict__ start, int count) {
  const int p = group_find(start, count, blockIdx.x);
  const GramPartialArgs g = a[p];
  gram_partial_body<T, C>((const T*)g.Y, g.ldy, g.rows, g.d, g.dp, g.chunk_rows, g.npairs, g.P,
                          (int)blockIdx.x - start[p]);
}

template <typename T, typename C>
void gram_partial_grouped_launch(const void* args, const int* start, int count, unsigned blocks, hipStream_t s) {
  hipLaunchKernelGGL((gram_partial_grouped<T, C>), dim3(blocks), dim3(256), 0, s, (const GramPartialArgs*)args,
                     start, count);
}

// G[i][j] = G[j][i] = sum over chunks of P[c][i][j] for i <= j (fixed order).
// Each block also writes esq[block] = its share of ||G - I||_F^2 over the
// d x d part (fixed-order reduction; NaN propagates), which the Cholesky
// sums in a fixed order to decide on its fast path.
__device__ __attribute__((always_inline)) inline void gram_reduce_body(const double* __restrict__ P, int nchunks,
                                                                       int d, int dp, double* __restrict__ G,
                                                                       double* __restrict__ esq, DevInfo* info,
                                                                       int bid, int nblk) {
  __shared__ double red[4];
  const int64_t total = (int64_t)dp * dp;
  bool bad = false;
  double e2 = 0.0;
  for (int64_t e = bid * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)nblk * blockDim.x) {
    const int i = (int)(e / dp), j = (int)(e % dp);
    if (i > j) continue;
    // (i, j) lies in tile (i/64, j/64) with i/64 <= j/64: written by every chunk
    double s = 0.0;
    const double* p = P + e;
    int c = 0;
    for (; c + 8 <= nchunks; c += 8) {  // loads first, then the ordered adds
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(c + u) * total];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; c < nchunks; ++c) s += p[(int64_t)c * total];
    if (!isfinite(s)) bad = true;
    G[(int64_t)i * dp + j] = s;
    G[(int64_t)j * dp + i] = s;
    if (j < d) {
      const double v = s - (i == j ? 1.0 : 0.0);
      e2 += (i == j ? 1.0 : 2.0) * v * v;
    }
  }
  if (bad) atomicOr(&info->nonfinite, 1);
  for (int off = 32; off > 0; off >>= 1) e2 += __shfl_xor(e2, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e2;
  __syncthreads();
  if (threadIdx.x == 0) esq[bid] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(256) void gram_reduce_kernel(const double* __restrict__ P, int nchunks, int d, int dp,
                                                          double* __restrict__ G, double* __restrict__ esq,
                                                          DevInfo* info) {
  gram_reduce_body(P, nchunks, d, dp, G, esq, info, blockIdx.x, gridDim.x);
}

struct GramReduceArgs {
  const double* P;
  double* G;
  double* esq;
  DevInfo* info;
  int nchunks, d, dp;
};

__global__ __launch_bounds__(256) void gram_reduce_grouped(const GramReduceArgs* __restrict__ a,
                                                           const int* __restrict__ start, int count) {
  const int p = group_find(start, count, blockIdx.x);
  const GramReduceArgs g = a[p];
  gram_reduce_body(g.P, g.nchunks, g.d, g.dp, g.G, g.esq, g.info, (int)blockIdx.x - start[p], start[p + 1] - start[p]);
}

void gram_reduce_grouped_launch(const void* args, const int* start, int count, unsigned blocks, hipStream_t s) {
  hipLaunchKernelGGL(gram_reduce_grouped, dim3(blocks), dim3(256), 0, s, (const GramReduceArgs*)args, start, count);
}

int gram_reduce_blocks(int dp) { return (int)ceil_div((int64_t)dp * dp, 256); }

int gram_chunks(int64_t rows, int dp) {
  // about 512 workgroups in total, two per CU, so that one workgroup's
  // MFMAs cover the other's load latency; for wide Gram matrices (21 or
  // more tile pairs, dp > 320) about 1024, four per CU: their long
  // per-chunk MFMA work hides more latency with more workgroups, while for
  // narrow ones the extra partial slabs cost more than they gain (measured)
  const int t = (int)ceil_div(dp, kGT);
  const int npairs = t * (t + 1) / 2;
  // (chunks of at least 128 rows, so that a short matrix is not cut into
  // slivers: in a batch the other problems fill the GPU)
  int64_t chunks = ceil_div(npairs >= 21 ? 1024 : 512, npairs);
  const int64_t maxc = ceil_div(rows, kGK);
  if (chunks > maxc) chunks = maxc;
  if (chunks < 1) chunks = 1;
  const int64_t chunk_rows = std::max<int64_t>(128, round_up(ceil_div(rows, chunks), kGK));
  return (int)ceil_div(rows, chunk_rows);
}

template <typename T, typename C>
hipError_t launch_gram_c(const T* Y, int64_t ldy, int64_t rows, int d, int dp, double* P,
                         int nchunks, double* G, double* esq, void* info, hipStream_t s,
                         hipEvent_t ev0, hipEvent_t ev1) {
  const int t = (int)ceil_div(dp, kGT);
  const int npairs = t * (t + 1) / 2;
  const int64_t chunk_rows = std::max<int64_t>(128, round_up(ceil_div(rows, nchunks), kGK));
  if (ev0) (void)hipEventRecord(ev0, s);
  const unsigned pb = (unsigned)(npairs * nchunks);
  if (!record_launch(&gram_partial_grouped_launch<T, C>, GramPartialArgs{Y, P, ldy, rows, chunk_rows, d, dp, npairs},
                     pb))
    hipLaunchKernelGGL((gram_partial_kernel<T, C>), dim3(pb), dim3(256), 0, s, Y, ldy, rows, d, dp, chunk_rows, npairs,
                       P);
  if (ev1) (void)hipEventRecord(ev1, s);
  const unsigned rb = (unsigned)gram_reduce_blocks(dp);
  if (!record_launch(&gram_reduce_grouped_launch, GramReduceArgs{P, G, esq, (DevInfo*)info, nchunks, d, dp}, rb))
    hipLaunchKernelGGL(gram_reduce_kernel, dim3(rb), dim3(256), 0, s, P, nchunks, d, dp, G, esq, (DevInfo*)info);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_gram(const T* Y, int64_t ldy, int64_t rows, int d, int dp, double* P, int nchunks, double* G,
                       double* esq, void* info, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  return launch_gram_c<T, double>(Y, ldy, rows, d, dp, P, nchunks, G, esq, info, s, ev0, ev1);
}
template hipError_t launch_gram<float>(const float*, int64_t, int64_t, int, int, double*, int,
                                       double*, double*, void*, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_gram<double>(const double*, int64_t, int64_t, int, int, double*, int,
                                        double*, double*, void*, hipStream_t, hipEvent_t, hipEvent_t);

hipError_t launch_gram_f32c(const double* Y, int64_t ldy, int64_t rows, int d, int dp, double* P, int nchunks,
                            double* G, double* esq, void* info, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  return launch_gram_c<double, float>(Y, ldy, rows, d, dp, P, nchunks, G, esq, info, s, ev0, ev1);
}

}  // namespace rqlp
