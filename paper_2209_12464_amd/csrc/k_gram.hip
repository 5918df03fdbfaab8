// Gram matrix G = Y^T Y in float64, the first step of each CholeskyQR pass.
// Float inputs are widened to double: a product of two floats is exact in
// double, so only the summation rounds.  The d x d upper triangle is cut
// into 64 x 64 tiles and the rows of Y into chunks; each workgroup forms one
// tile over one chunk with the float64 MFMA (16x16x4), and a second kernel
// adds the chunk partials in a fixed order (deterministic) and mirrors the
// result into the lower triangle.
#include "common.h"
#include "kernels.h"

namespace rqlp {

constexpr int kGT = 64;   // output tile side
constexpr int kGK = 16;   // rows of Y per LDS step

__device__ inline void tile_pair(int p, int& I, int& J) {
  // p enumerates (I, J), I <= J, row by row of the upper triangle of a t x t grid
  // via J = floor((sqrt(8p+1)-1)/2): pairs are listed as J-major.
  int j = (int)((sqrtf(8.0f * p + 1.0f) - 1.0f) * 0.5f);
  while ((j + 1) * (j + 2) / 2 <= p) ++j;
  while (j * (j + 1) / 2 > p) --j;
  J = j;
  I = p - j * (j + 1) / 2;
}

template <typename T>
__global__ __launch_bounds__(256) void gram_partial_kernel(const T* __restrict__ Y, int64_t ldy,
                                                           int64_t rows, int d, int dp,
                                                           int64_t chunk_rows, int npairs,
                                                           double* __restrict__ P) {
  __shared__ double YI[kGK][kGT + 1];
  __shared__ double YJ[kGK][kGT + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int pair = blockIdx.x % npairs;
  const int chunk = blockIdx.x / npairs;
  int I, J;
  tile_pair(pair, I, J);
  const int64_t r0 = (int64_t)chunk * chunk_rows;
  const int64_t r1 = min(rows, r0 + chunk_rows);
  const int wi = wave >> 1, wj = wave & 1;
  doublex4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<double>::zero();

  for (int64_t k0 = r0; k0 < r1; k0 += kGK) {
#pragma unroll
    for (int i = 0; i < kGK * kGT / 256; ++i) {
      const int idx = tid + 256 * i;
      const int kr = idx / kGT, c = idx % kGT;
      const int64_t r = k0 + kr;
      const int ci = I * kGT + c, cj = J * kGT + c;
      YI[kr][c] = (r < r1 && ci < d) ? (double)Y[r * ldy + ci] : 0.0;
      YJ[kr][c] = (r < r1 && cj < d) ? (double)Y[r * ldy + cj] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kGK / 4; ++ks) {
      double a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = YI[ks * 4 + lane / 16][wi * 32 + t * 16 + (lane & 15)];
        b[t] = YJ[ks * 4 + lane / 16][wj * 32 + t * 16 + (lane & 15)];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = Mfma<double>::mma(a[x], b[y], acc[x][y]);
    }
    __syncthreads();
  }
  double* Pc = P + (int64_t)chunk * dp * dp;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = I * kGT + wi * 32 + x * 16 + Mfma<double>::row(lane, r);
        const int col = J * kGT + wj * 32 + y * 16 + Mfma<double>::col(lane);
        if (row < dp && col < dp) Pc[(int64_t)row * dp + col] = acc[x][y][r];
      }
}

// G[i][j] = G[j][i] = sum over chunks of P[c][i][j] for i <= j (fixed order).
__global__ __launch_bounds__(256) void gram_reduce_kernel(const double* __restrict__ P, int nchunks,
                                                          int dp, double* __restrict__ G,
                                                          DevInfo* info) {
  const int64_t total = (int64_t)dp * dp;
  bool bad = false;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / dp), j = (int)(e % dp);
    if (i > j) continue;
    // (i, j) lies in tile (i/64, j/64) with i/64 <= j/64: written by every chunk
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += P[(int64_t)c * total + e];
    if (!isfinite(s)) bad = true;
    G[(int64_t)i * dp + j] = s;
    G[(int64_t)j * dp + i] = s;
  }
  if (bad) atomicOr(&info->nonfinite, 1);
}

int gram_chunks(int64_t rows, int dp) {
  const int t = (int)ceil_div(dp, kGT);
  const int npairs = t * (t + 1) / 2;
  int64_t chunks = ceil_div(512, npairs);
  const int64_t maxc = ceil_div(rows, kGK);
  if (chunks > maxc) chunks = maxc;
  if (chunks < 1) chunks = 1;
  const int64_t chunk_rows = round_up(ceil_div(rows, chunks), kGK);
  return (int)ceil_div(rows, chunk_rows);
}

template <typename T>
hipError_t launch_gram(const T* Y, int64_t ldy, int64_t rows, int d, int dp, double* P,
                       int nchunks, double* G, void* info, hipStream_t s, hipEvent_t ev0,
                       hipEvent_t ev1) {
  const int t = (int)ceil_div(dp, kGT);
  const int npairs = t * (t + 1) / 2;
  const int64_t chunk_rows = round_up(ceil_div(rows, nchunks), kGK);
  if (ev0) hipEventRecord(ev0, s);
  hipLaunchKernelGGL(gram_partial_kernel<T>, dim3(npairs * nchunks), dim3(256), 0, s, Y, ldy, rows, d,
                     dp, chunk_rows, npairs, P);
  if (ev1) hipEventRecord(ev1, s);
  const int64_t g = ceil_div((int64_t)dp * dp, 256);
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)g), dim3(256), 0, s, P, nchunks, dp, G,
                     (DevInfo*)info);
  return hipGetLastError();
}
template hipError_t launch_gram<float>(const float*, int64_t, int64_t, int, int, double*, int,
                                       double*, void*, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_gram<double>(const double*, int64_t, int64_t, int, int, double*, int,
                                        double*, void*, hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace rqlp
