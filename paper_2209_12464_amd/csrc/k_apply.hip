// Q = Y R^-1 for the upper-triangular Cholesky factor R (float64), the last
// step of each CholeskyQR pass.  Arithmetic is float64 whatever the storage
// type of Y and Q.  R^-1 = X is explicit (the Cholesky's fast path, or the
// inverse kernel after a full factorization), and every 16 x 16 output block
// is an independent sum Q[:, J] = sum_{t <= J} Y[:, t] X[t, J]: workgroups
// take 64 RF rows x 4 column blocks with LDS-staged tiles, each wave RF
// 16-row fragments (RF = 2 for tall inputs, so that a wave issues 32 MFMAs
// per staged block row).
// Columns the Cholesky marked dependent are written as N(0,1)/sqrt(rows)
// columns from a Philox stream of their own (completion of a rank-deficient
// basis).  Their rows of R are zero (with a unit diagonal), so the other
// columns of Y R^-1 do not involve them.
#include "common.h"
#include "grouped.h"
#include "kernels.h"

#include <utility>

namespace rqlp {

constexpr int kApCols = 4 * kTile;    // columns per workgroup (4 blocks)
constexpr int kApXS = kApCols + 16;   // LDS row stride of the X tile (doubles): rows 32 banks apart
constexpr int kApYS = kTile + 1;      // LDS row stride of the Y tile (doubles)

__host__ __device__ inline size_t apply_lds_doubles(int rf) {
  return 2 * (size_t)(kTile * kApXS + 64 * rf * kApYS);
}

// Workgroup (bx, by): rows bx * 64 RF .. and column blocks J0 .. J0 + 3,
// J0 = 4 (G - 1 - by) for G = ceil(T / 4) column groups.
template <typename Tin, typename Tout, int RF, typename C = double>
__device__ __attribute__((always_inline)) inline void apply_body(const Tin* __restrict__ Y, int64_t ldy, int64_t rows,
                                                                 int d, int dp, const int32_t* __restrict__ flags,
                                                                 const int32_t* __restrict__ mode,
                                                                 const double* __restrict__ Xfull,
                                                                 Tout* __restrict__ out1, int64_t ld1, int ncols1,
                                                                 Tout* __restrict__ out2, int64_t ld2, int ncols2,
                                                                 uint64_t seed, uint64_t key1, double inv_sqrt_rows,
                                                                 int bx, int by) {
  constexpr int kApRows = 64 * RF;  // rows per workgroup (16 RF per wave)
  extern __shared__ double smem_raw[];
  C* smem = reinterpret_cast<C*>(smem_raw);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane >> 4, lc = lane & 15;
  const int64_t r0 = (int64_t)bx * kApRows;
  const int T = dp / kTile;

  // out[:, J] = sum_{t <= J} Y[:, t] X[t, J] for column blocks J0..J1-1;
  // per block row t the X tile (16 x 64) and the Y tile (64 x 16, widened
  // to double) are staged in LDS, double buffered, while the tiles of the
  // next kDepth block rows are in flight into a register ring (slot t mod
  // kDepth).  Narrow row blocks (RF = 1: short, latency-bound chains) keep
  // two block rows in flight; RF = 2 keeps one, which leaves room for more
  // resident waves (measured faster for it).
  // column groups in reverse of the dispatch order: the long triangular
  // loops of the last column groups start first, the short ones fill in
  const int J0 = 4 * ((T + 3) / 4 - 1 - by);
  if (J0 < 0 || J0 >= T) return;
  const int J1 = min(T, J0 + 4);
  constexpr int kDepth = RF == 1 ? 2 : 1;
  C* Xs = smem;                                // [2][16][kApXS]
  C* Ys = smem + 2 * kTile * kApXS;            // [2][64 RF][kApYS]
  double xr[kDepth][4];
  Tin yr[kDepth][4 * RF];
  auto load = [&](auto Sc, int t) {
    constexpr int S = decltype(Sc)::value;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int kr = e >> 6, c = e & 63;       // X[t*16 + kr][J0*16 + c]
      const int col = J0 * kTile + c;
      xr[S][q] = (col < J1 * kTile) ? Xfull[(int64_t)(t * kTile + kr) * dp + col] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4 * RF; ++q) {
      const int e = tid + 256 * q;
      const int rr = e >> 4, cc = e & 15;      // Y[r0 + rr][t*16 + cc]
      const int64_t row = r0 + rr;
      const int ycol = t * kTile + cc;
      yr[S][q] = (row < rows && ycol < d) ? Y[row * ldy + ycol] : (Tin)0;
    }
  };
  auto store = [&](auto Sc, int buf) {
    constexpr int S = decltype(Sc)::value;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      Xs[buf * kTile * kApXS + (e >> 6) * kApXS + (e & 63)] = (C)xr[S][q];
    }
#pragma unroll
    for (int q = 0; q < 4 * RF; ++q) {
      const int e = tid + 256 * q;
      Ys[buf * kApRows * kApYS + (e >> 4) * kApYS + (e & 15)] = (C)yr[S][q];
    }
  };
  typename Mfma<C>::acc_t acc[RF][4];
#pragma unroll
  for (int f = 0; f < RF; ++f)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[f][u] = Mfma<C>::zero();
  auto compute = [&](int t) {
    const int buf = t & 1;
    const C* xs = Xs + buf * kTile * kApXS;
    const C* ys = Ys + buf * kApRows * kApYS + (wave * kTile * RF + lc) * kApYS;
    C a[RF][4];
#pragma unroll
    for (int f = 0; f < RF; ++f)
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)  // A[m][k] = Y[16 (RF w + f) + m][t*16 + k]
        a[f][ks] = ys[f * kTile * kApYS + ks * 4 + lr];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (J0 + u >= t && J0 + u < J1) {
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const C b = xs[(ks * 4 + lr) * kApXS + u * kTile + lc];
#pragma unroll
          for (int f = 0; f < RF; ++f) acc[f][u] = Mfma<C>::mma(a[f][ks], b, acc[f][u]);
        }
      }
    }
  };
  using S0 = std::integral_constant<int, 0>;
  if constexpr (kDepth == 1) {
    // one block row in flight: row t + 1 is fetched while row t is used
    load(S0{}, 0);
    store(S0{}, 0);
    __syncthreads();
    for (int t = 0; t < J1; ++t) {
      const bool more = t + 1 < J1;
      if (more) load(S0{}, t + 1);
      compute(t);
      if (more) store(S0{}, (t + 1) & 1);
      __syncthreads();
    }
  } else {
    // block rows 0 .. kDepth-1 in flight, row 0 staged, row kDepth into its slot
    [&]<int... Ss>(std::integer_sequence<int, Ss...>) {
      ((Ss < J1 ? load(std::integral_constant<int, Ss>{}, Ss) : void()), ...);
    }(std::make_integer_sequence<int, kDepth>{});
    store(S0{}, 0);
    if (kDepth < J1) load(S0{}, kDepth);
    __syncthreads();
    // block row t = t0 + S (S = t mod kDepth): its products, then row t + 1
    // staged from slot (S + 1) mod kDepth, which then takes row t + 1 + kDepth
    auto sub = [&](auto Sc, int t) {
      constexpr int S = decltype(Sc)::value;
      constexpr int N = (S + 1) % kDepth;
      if (t >= J1) return;
      compute(t);
      if (t + 1 < J1) {
        store(std::integral_constant<int, N>{}, (t + 1) & 1);
        if (t + 1 + kDepth < J1) load(std::integral_constant<int, N>{}, t + 1 + kDepth);
      }
      __syncthreads();
    };
    for (int t0 = 0; t0 < J1; t0 += kDepth) {
      [&]<int... Ss>(std::integer_sequence<int, Ss...>) {
        (sub(std::integral_constant<int, Ss>{}, t0 + Ss), ...);
      }(std::make_integer_sequence<int, kDepth>{});
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    if (J0 + u >= J1) break;
#pragma unroll
    for (int f = 0; f < RF; ++f)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + (wave * RF + f) * kTile + Mfma<C>::row(lane, r);
        const int cc = (J0 + u) * kTile + Mfma<C>::col(lane);
        if (row < rows) {
          if (cc < ncols1) out1[row * ld1 + cc] = (Tout)acc[f][u][r];
          if (out2 && cc < ncols2) out2[row * ld2 + cc] = (Tout)acc[f][u][r];
        }
      }
  }
  // dependent columns (mode 0 only): the same places again, now with the
  // completion values (one rolled loop, so the generator is inlined once)
  if (*mode != 0) return;
  for (int e = 0; e < 4 * RF * 4; ++e) {
    const int u = e / (RF * 4), f = (e / 4) % RF, r = e % 4;
    const int col = (J0 + u) * kTile + lc;
    if (J0 + u >= J1 || col >= d || flags[col] == 0) continue;
    const int64_t row = r0 + (wave * RF + f) * kTile + lr + 4 * r;
    if (row >= rows) continue;
    const double v = gaussian_at(seed, key1, (uint64_t)col * rows + row) * inv_sqrt_rows;
    if (col < ncols1) out1[row * ld1 + col] = (Tout)v;
    if (out2 && col < ncols2) out2[row * ld2 + col] = (Tout)v;
  }
}

template <typename Tin, typename Tout, int RF>
__global__ __launch_bounds__(256) void apply_kernel(const Tin* __restrict__ Y, int64_t ldy, int64_t rows, int d, int dp,
                                                    const int32_t* __restrict__ flags, const int32_t* __restrict__ mode,
                                                    const double* __restrict__ Xfull, Tout* __restrict__ out1,
                                                    int64_t ld1, int ncols1, Tout* __restrict__ out2, int64_t ld2,
                                                    int ncols2, uint64_t seed, uint64_t key1, double inv_sqrt_rows) {
  apply_body<Tin, Tout, RF>(Y, ldy, rows, d, dp, flags, mode, Xfull, out1, ld1, ncols1, out2, ld2, ncols2, seed, key1,
                            inv_sqrt_rows, blockIdx.x, blockIdx.y);
}

struct ApplyArgs {
  const void* Y;
  const int32_t* flags;
  const int32_t* mode;
  const double* X;
  void* out1;
  void* out2;
  int64_t ldy, rows, ld1, ld2;
  uint64_t seed, key1;
  double isr;
  int d, dp, ncols1, ncols2, gx;
};

template <typename Tin, typename Tout, int RF>
__global__ __launch_bounds__(256) void apply_grouped(const ApplyArgs* __restrict__ a, const int* __restrict__ start,
                                                     int count) {
  const int p = group_find(start, count, blockIdx.x);
  const ApplyArgs g = a[p];
  const int b = (int)blockIdx.x - start[p];
  apply_body<Tin, Tout, RF>((const Tin*)g.Y, g.ldy, g.rows, g.d, g.dp, g.flags, g.mode, g.X, (Tout*)g.out1, g.ld1,
                            g.ncols1, (Tout*)g.out2, g.ld2, g.ncols2, g.seed, g.key1, g.isr, b % g.gx, b / g.gx);
}

template <typename Tin, typename Tout, int RF>
void apply_grouped_launch(const void* args, const int* start, int count, unsigned blocks, hipStream_t s) {
  hipLaunchKernelGGL((apply_grouped<Tin, Tout, RF>), dim3(blocks), dim3(256), apply_lds_doubles(RF) * sizeof(double),
                     s, (const ApplyArgs*)args, start, count);
}

template <typename Tin, typename Tout>
hipError_t launch_apply(const Tin* Y, int64_t ldy, int64_t rows, int d, int dp, const int32_t* flags,
                        const int32_t* mode, const double* Xfull, Tout* out1, int64_t ld1, int ncols1, Tout* out2,
                        int64_t ld2, int ncols2, uint64_t seed, uint64_t key1, hipStream_t s,
                        hipEvent_t ev0, hipEvent_t ev1) {
  if (rows <= 0) return hipSuccess;
  const double isr = 1.0 / sqrt((double)rows);
  const unsigned groups = (unsigned)ceil_div(dp / kTile, 4);
  // two row fragments per wave for wide R (five or more column groups, whose
  // workgroups run long triangular loops) once that still gives about four
  // workgroups per CU; narrow R keeps one (measured faster there)
  const int rf = (groups >= 5 && ceil_div(rows, 128) * groups >= 1024) ? 2 : 1;
  const size_t shmem = apply_lds_doubles(rf) * sizeof(double);  // at most 55 KB
  if (ev0) (void)hipEventRecord(ev0, s);
  const unsigned gx = (unsigned)ceil_div(rows, 64 * rf);
  const ApplyArgs a{Y, flags, mode, Xfull, out1, out2, ldy, rows, ld1, ld2, seed, key1, isr, d, dp, ncols1, ncols2,
                    (int)gx};
  if (rf == 2) {
    if (!record_launch(&apply_grouped_launch<Tin, Tout, 2>, a, gx * groups))
      hipLaunchKernelGGL((apply_kernel<Tin, Tout, 2>), dim3(gx, groups), dim3(256), shmem, s, Y, ldy, rows, d, dp,
                         flags, mode, Xfull, out1, ld1, ncols1, out2, ld2, ncols2, seed, key1, isr);
  } else {
    if (!record_launch(&apply_grouped_launch<Tin, Tout, 1>, a, gx * groups))
      hipLaunchKernelGGL((apply_kernel<Tin, Tout, 1>), dim3(gx, groups), dim3(256), shmem, s, Y, ldy, rows, d, dp,
                         flags, mode, Xfull, out1, ld1, ncols1, out2, ld2, ncols2, seed, key1, isr);
  }
  if (ev1) (void)hipEventRecord(ev1, s);
  return hipGetLastError();
}

// Second pass of the bfloat16 form: float32 arithmetic when the Cholesky
// took its fast path (X = I - F), float64 otherwise.
template <int RF>
__device__ __attribute__((always_inline)) inline void apply_f32fast_body(
    const double* __restrict__ Y, int64_t ldy, int64_t rows, int d, int dp, const int32_t* __restrict__ flags,
    const int32_t* __restrict__ mode, const double* __restrict__ Xfull, float* __restrict__ out1, int64_t ld1,
    int ncols1, float* __restrict__ out2, int64_t ld2, int ncols2, uint64_t seed, uint64_t key1,
    double inv_sqrt_rows, int bx, int by) {
  if (*mode == 2)
    apply_body<double, float, RF, float>(Y, ldy, rows, d, dp, flags, mode, Xfull, out1, ld1, ncols1, out2, ld2,
                                         ncols2, seed, key1, inv_sqrt_rows, bx, by);
  else
    apply_body<double, float, RF, double>(Y, ldy, rows, d, dp, flags, mode, Xfull, out1, ld1, ncols1, out2, ld2,
                                          ncols2, seed, key1, inv_sqrt_rows, bx, by);
}

template <int RF>
__global__ __launch_bounds__(256) void apply_f32fast_kernel(const double* __restrict__ Y, int64_t ldy, int64_t rows,
                                                            int d, int dp, const int32_t* __restrict__ flags,
                                                            const int32_t* __restrict__ mode,
                                                            const double* __restrict__ Xfull,
                                                            float* __restrict__ out1, int64_t ld1, int ncols1,
                                                            float* __restrict__ out2, int64_t ld2, int ncols2,
                                                            uint64_t seed, uint64_t key1, double inv_sqrt_rows) {
  apply_f32fast_body<RF>(Y, ldy, rows, d, dp, flags, mode, Xfull, out1, ld1, ncols1, out2, ld2, ncols2, seed, key1,
                         inv_sqrt_rows, blockIdx.x, blockIdx.y);
}

template <int RF>
__global__ __launch_bounds__(256) void apply_f32fast_grouped(const ApplyArgs* __restrict__ a,
                                                             const int* __restrict__ start, int count) {
  const int p = group_find(start, count, blockIdx.x);
  const ApplyArgs g = a[p];
  const int b = (int)blockIdx.x - start[p];
  apply_f32fast_body<RF>((const double*)g.Y, g.ldy, g.rows, g.d, g.dp, g.flags, g.mode, g.X, (float*)g.out1, g.ld1,
                         g.ncols1, (float*)g.out2, g.ld2, g.ncols2, g.seed, g.key1, g.isr, b % g.gx, b / g.gx);
}

template <int RF>
void apply_f32fast_grouped_launch(const void* args, const int* start, int count, unsigned blocks, hipStream_t s) {
  hipLaunchKernelGGL((apply_f32fast_grouped<RF>), dim3(blocks), dim3(256), apply_lds_doubles(RF) * sizeof(double), s,
                     (const ApplyArgs*)args, start, count);
}

hipError_t launch_apply_f32fast(const double* Y, int64_t ldy, int64_t rows, int d, int dp, const int32_t* flags,
                                const int32_t* mode, const double* Xfull, float* out1, int64_t ld1, int ncols1,
                                float* out2, int64_t ld2, int ncols2, uint64_t seed, uint64_t key1, hipStream_t s,
                                hipEvent_t ev0, hipEvent_t ev1) {
  if (rows <= 0) return hipSuccess;
  const double isr = 1.0 / sqrt((double)rows);
  const unsigned groups = (unsigned)ceil_div(dp / kTile, 4);
  const int rf = (groups >= 5 && ceil_div(rows, 128) * groups >= 1024) ? 2 : 1;  // as launch_apply
  const size_t shmem = apply_lds_doubles(rf) * sizeof(double);
  if (ev0) (void)hipEventRecord(ev0, s);
  const unsigned gx = (unsigned)ceil_div(rows, 64 * rf);
  const ApplyArgs a{Y, flags, mode, Xfull, out1, out2, ldy, rows, ld1, ld2, seed, key1, isr, d, dp, ncols1, ncols2,
                    (int)gx};
  if (rf == 2) {
    if (!record_launch(&apply_f32fast_grouped_launch<2>, a, gx * groups))
      hipLaunchKernelGGL((apply_f32fast_kernel<2>), dim3(gx, groups), dim3(256), shmem, s, Y, ldy, rows, d, dp, flags,
                         mode, Xfull, out1, ld1, ncols1, out2, ld2, ncols2, seed, key1, isr);
  } else {
    if (!record_launch(&apply_f32fast_grouped_launch<1>, a, gx * groups))
      hipLaunchKernelGGL((apply_f32fast_kernel<1>), dim3(gx, groups), dim3(256), shmem, s, Y, ldy, rows, d, dp, flags,
                         mode, Xfull, out1, ld1, ncols1, out2, ld2, ncols2, seed, key1, isr);
  }
  if (ev1) (void)hipEventRecord(ev1, s);
  return hipGetLastError();
}

#define RQLP_APPLY_INST(TI, TO)                                                                       \
  template hipError_t launch_apply<TI, TO>(const TI*, int64_t, int64_t, int, int, const int32_t*,    \
                                           const int32_t*, const double*,                                 \
                                           TO*, int64_t, int, TO*, int64_t,                               \
                                           int, uint64_t, uint64_t, hipStream_t, hipEvent_t, hipEvent_t);
RQLP_APPLY_INST(float, double)
RQLP_APPLY_INST(double, double)
RQLP_APPLY_INST(double, float)
RQLP_APPLY_INST(float, float)
#undef RQLP_APPLY_INST

}  // namespace rqlp
