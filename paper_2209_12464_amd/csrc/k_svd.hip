// SVD of the small d x d factor (Remark 1 of Section III-B: an SVD of the
// middle factor turns RU-QLP into an SVD-like decomposition), float64,
// d <= 544, by one-sided (Hestenes) Jacobi with column blocks.
//
// The columns of X = M are rotated in pairs until they are mutually
// orthogonal: X V-bar = U-bar Sigma, with V-bar the product of the
// rotations.  A rotation of columns p, q zeroes their inner product:
//     zeta = (||x_q||^2 - ||x_p||^2) / (2 x_p.x_q),
//     t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),  c = 1 / sqrt(1 + t^2),  s = c t,
//     x_p <- c x_p - s x_q,   x_q <- s x_p + c x_q.
// Each column carries its column of V-bar below it (length 2 dp: x_j, then
// v_j, starting from e_j), so that one rotation moves both and V-bar needs
// no pass of its own.  The padded columns (dp a multiple of 16) are split
// into blocks of 8.  One step pairs every block with another (a round-robin
// tournament over the blocks, so a sweep of nb - 1 steps meets every pair of
// blocks); the workgroup of a block pair (8 waves) holds its 16 columns in
// LDS and rotates them, one pair per wave and round: at a sweep's first step
// every pair of the 16 columns (15 rounds of 8), at later steps only the 64
// pairs across the two blocks (8 rounds), so that a sweep visits every pair
// of columns once or twice.  The squared column norms are computed at the
// start of a step and then carried through its rotations
// (||x_p||^2 -= t x_p.x_q, ||x_q||^2 += t x_p.x_q), so that a round needs one
// inner product.  A pair is rotated only when
// |x_p.x_q| > dp eps ||x_p|| ||x_q||; a sweep without a rotation ends the
// iteration.  All sweeps run in one cooperative launch (nb / 2 workgroups,
// a grid barrier after every step).  Finally sigma_j = ||x_j||, the
// columns are sorted by descending sigma (stable), u_j = x_j / sigma_j (zero
// when sigma_j = 0), and each pair of vectors is signed so that the entry of
// largest magnitude of v_j is positive (the first such entry on ties).
#include <hip/hip_cooperative_groups.h>

#include "common.h"
#include "kernels.h"

namespace rqlp {

constexpr int kSvW = 8;               // columns per block
constexpr int kSvCols = 2 * kSvW;     // columns of a block pair
constexpr int kSvThreads = 64 * kSvW; // one wave per rotation of a round
constexpr int kSvRows = (kDMax + 63) / 64;  // rows of each half per lane, at most

inline size_t svd_align(size_t b) { return (b + 255) & ~(size_t)255; }

// v moved across lanes by a DPP pattern; lanes outside row_mask get 0.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_take(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, kCtrl, kRowMask, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, kRowMask, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the 64 lanes, the same value in every lane (lane 63's): row
// sums by rotations within each row of 16 lanes, then rows 1 and 3 add the
// row before them (row_bcast:15) and rows 2 and 3 the first two rows
// (row_bcast:31), which leaves the total in row 3.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_take<0x128, 0xf>(v);  // row_ror:8
  v += dpp_take<0x124, 0xf>(v);  // row_ror:4
  v += dpp_take<0x122, 0xf>(v);  // row_ror:2
  v += dpp_take<0x121, 0xf>(v);  // row_ror:1
  v += dpp_take<0x142, 0xa>(v);  // row_bcast:15
  v += dpp_take<0x143, 0xc>(v);  // row_bcast:31
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// 1/x and 1/sqrt(x) for finite positive (rsqrt) or nonzero (rcp) x: the
// hardware estimates (relative error about 2^-24) with one third-order
// correction each, y (1 + e + e^2) with e = 1 - x y for the reciprocal and
// y (1 + e/2 + 3 e^2/8) with e = 1 - x y^2 for the reciprocal square root,
// within an ulp or two like two Newton steps but with a shorter dependent
// chain on the critical path of every rotation (instead of the longer
// correctly rounded sequences).
__device__ __forceinline__ double rcp_nr(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, y, 1.0);
  return fma(y, fma(e, e, e), y);
}
__device__ __forceinline__ double rsqrt_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(0.375, e, 0.5), y);
}

// XV: dp columns of length 2 dp, column j = (M[:, j] zero-padded, e_j).
template <typename T>
__global__ __launch_bounds__(256) void svd_init_kernel(const T* __restrict__ M, int64_t ldm, int d, int dp,
                                                       double* __restrict__ XV, int32_t* __restrict__ flags,
                                                       int nflags) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (int64_t)dp * 2 * dp) {
    const int j = (int)(e / (2 * dp)), r = (int)(e % (2 * dp));
    XV[e] = r < dp ? ((j < d && r < d) ? (double)M[(int64_t)r * ldm + j] : 0.0) : (r - dp == j ? 1.0 : 0.0);
  }
  if (e < nflags) flags[e] = 0;
}

// One step of a sweep for this workgroup's block pair; flags[sweep] = 1
// when the step rotated a pair.  R = ceil(dp / 64) rows of each half per
// lane.
template <int R>
__device__ __attribute__((always_inline)) inline void svd_step(double* __restrict__ XV, int dp, int nb, int step,
                                                              int sweep, int32_t* __restrict__ flags, double tol,
                                                              double* Xs, double* nrm, int& rotated) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int len = 2 * dp;
  // position 0 of the tournament holds block 0; the others rotate by step
  const int pa = blockIdx.x, pb = nb - 1 - (int)blockIdx.x;
  const int ba = pa == 0 ? 0 : 1 + (pa - 1 + step) % (nb - 1);
  const int bb = 1 + (pb - 1 + step) % (nb - 1);
  // the two blocks' columns are contiguous runs of kSvW * len values
  const int64_t base_a = (int64_t)ba * kSvW * len, base_b = (int64_t)bb * kSvW * len;
  const int half = kSvW * len;
  // batches of kLd values per thread and block, all loads of a batch in
  // flight before their LDS stores
  constexpr int kLd = 8;
  for (int e0 = tid; e0 < half; e0 += kLd * kSvThreads) {
    double va[kLd], vb[kLd];
#pragma unroll
    for (int j = 0; j < kLd; ++j) {
      const int e = e0 + j * kSvThreads;
      va[j] = e < half ? XV[base_a + e] : 0.0;
      vb[j] = e < half ? XV[base_b + e] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kLd; ++j) {
      const int e = e0 + j * kSvThreads;
      if (e < half) {
        Xs[e] = va[j];
        Xs[half + e] = vb[j];
      }
    }
  }
  if (tid == 0) rotated = 0;
  __syncthreads();
  // squared norms of the pair's columns: wave w takes columns w and w + kSvW
  // (both sums side by side)
  {
    static_assert(kSvCols == 2 * (kSvThreads / 64), "two columns per wave");
    const double* x0 = Xs + wave * len;
    const double* x1 = Xs + (wave + kSvW) * len;
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int r = lane + 64 * i;
      if (r < dp) {
        a0 = fma(x0[r], x0[r], a0);
        a1 = fma(x1[r], x1[r], a1);
      }
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    if (lane == 0) {
      nrm[wave] = a0;
      nrm[wave + kSvW] = a1;
    }
  }
  __syncthreads();

  // The rotation of a pair with squared norms a, b and inner product g
  // (false when the pair is already orthogonal to working accuracy).
  auto params = [&](double a, double b, double g, double& t, double& cs, double& sn) {
    if (!(g * g > tol * tol * (a * b))) return false;
    const double zeta = (b - a) * rcp_nr(2.0 * g);
    if (fabs(zeta) > 1e150) {
      t = 0.5 * rcp_nr(zeta);
    } else {
      const double w = fma(zeta, zeta, 1.0);
      t = copysign(rcp_nr(fabs(zeta) + w * rsqrt_nr(w)), zeta);
    }
    cs = rsqrt_nr(fma(t, t, 1.0));
    sn = cs * t;
    return true;
  };

  if (step == 0) {
    // round-robin over all the pair's columns, every column through LDS
    for (int rnd = 0; rnd < kSvCols - 1; ++rnd) {
      const int p = wave == 0 ? 0 : 1 + (wave - 1 + rnd) % (kSvCols - 1);
      const int q = 1 + (kSvCols - 2 - wave + rnd) % (kSvCols - 1);
      double* xp = Xs + p * len;
      double* xq = Xs + q * len;
      const double a = nrm[p], b = nrm[q];
      // this lane's rows of x_p and x_q and of their v halves, all loaded
      // before the first use (the v halves are needed only for a rotation,
      // but reading them here takes their latency off the rotation's chain)
      double u[R], v[R], pu[R], pv[R];
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int r = lane + 64 * i;
        u[i] = r < dp ? xp[r] : 0.0;
        v[i] = r < dp ? xq[r] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int r = dp + lane + 64 * i;
        pu[i] = r < len ? xp[r] : 0.0;
        pv[i] = r < len ? xq[r] : 0.0;
      }
      double g = 0.0;
#pragma unroll
      for (int i = 0; i < R; ++i) g = fma(u[i], v[i], g);
      g = wave_sum(g);  // uniform across the wave: all rows see one rotation
      double t, cs, sn;
      if (params(a, b, g, t, cs, sn)) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const int r = lane + 64 * i;
          if (r < dp) {
            xp[r] = cs * u[i] - sn * v[i];
            xq[r] = sn * u[i] + cs * v[i];
            xp[dp + r] = cs * pu[i] - sn * pv[i];
            xq[dp + r] = sn * pu[i] + cs * pv[i];
          }
        }
        if (lane == 0) {
          nrm[p] = a - t * g;
          nrm[q] = b + t * g;
          rotated = 1;
        }
      }
      __syncthreads();
    }
  } else {
    // column p = wave of the first block meets every column of the second,
    // q = kSvW + (wave + round) mod kSvW: p (both halves) and its squared
    // norm stay in this wave's registers for the whole step, and only the
    // q columns pass through LDS from round to round
    const int p = wave;
    double* xp = Xs + p * len;
    double u[R], pu[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int r = lane + 64 * i;
      u[i] = r < dp ? xp[r] : 0.0;
      pu[i] = r < dp ? xp[dp + r] : 0.0;
    }
    double a = nrm[p];
    for (int rnd = 0; rnd < kSvW; ++rnd) {
      const int q = kSvW + (wave + rnd) % kSvW;
      double* xq = Xs + q * len;
      const double b = nrm[q];
      double v[R], pv[R];
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int r = lane + 64 * i;
        v[i] = r < dp ? xq[r] : 0.0;
        pv[i] = r < dp ? xq[dp + r] : 0.0;
      }
      double g = 0.0;
#pragma unroll
      for (int i = 0; i < R; ++i) g = fma(u[i], v[i], g);
      g = wave_sum(g);
      double t, cs, sn;
      if (params(a, b, g, t, cs, sn)) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const int r = lane + 64 * i;
          const double nu = cs * u[i] - sn * v[i], npu = cs * pu[i] - sn * pv[i];
          if (r < dp) {
            xq[r] = sn * u[i] + cs * v[i];
            xq[dp + r] = sn * pu[i] + cs * pv[i];
          }
          u[i] = nu;
          pu[i] = npu;
        }
        a = a - t * g;
        if (lane == 0) {
          nrm[q] = b + t * g;
          rotated = 1;
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int r = lane + 64 * i;
      if (r < dp) {
        xp[r] = u[i];
        xp[dp + r] = pu[i];
      }
    }
    __syncthreads();
  }

  // columns no rotation touched are already in XV as they are; otherwise
  // batches of kLd values per thread and block, read from LDS before their
  // stores
  if (rotated) {
    for (int e0 = tid; e0 < half; e0 += kLd * kSvThreads) {
      double va[kLd], vb[kLd];
#pragma unroll
      for (int j = 0; j < kLd; ++j) {
        const int e = e0 + j * kSvThreads;
        va[j] = e < half ? Xs[e] : 0.0;
        vb[j] = e < half ? Xs[half + e] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < kLd; ++j) {
        const int e = e0 + j * kSvThreads;
        if (e < half) {
          XV[base_a + e] = va[j];
          XV[base_b + e] = vb[j];
        }
      }
    }
    if (tid == 0) flags[sweep] = 1;
  }
}

// Every sweep, in one cooperative launch of nb / 2 workgroups.
template <int R>
__global__ __launch_bounds__(kSvThreads) void svd_sweeps_kernel(double* __restrict__ XV, int dp, int nb,
                                                                int32_t* __restrict__ flags, int max_sweeps,
                                                                double tol) {
  extern __shared__ double svd_smem[];  // kSvCols columns of length 2 dp
  __shared__ double nrm[kSvCols];        // squared norms of the x parts
  __shared__ int rotated;
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    for (int step = 0; step < nb - 1; ++step) {
      svd_step<R>(XV, dp, nb, step, sweep, flags, tol, svd_smem, nrm, rotated);
      grid.sync();  // the next step reads columns other workgroups wrote
    }
    if (flags[sweep] == 0) break;  // the same value for every workgroup after the barrier
  }
}

// sigma_j, the sign of each pair and the descending order (one workgroup):
// sig[o], src[o] (the column that goes to place o) and sgn[o].
__global__ __launch_bounds__(1024) void svd_order_kernel(const double* __restrict__ XV, int d, int dp, const int32_t* __restrict__ flags,
                                                         int nflags, double* __restrict__ sig_out,
                                                         int32_t* __restrict__ src, double* __restrict__ sgn_out,
                                                         DevInfo* __restrict__ info) {
  __shared__ double sig[kDMax];
  __shared__ double sgn[kDMax];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = wave; j < d; j += 16) {
    const double* X = XV + (int64_t)j * 2 * dp;  // x_j, then v_j
    double ss = 0.0, best = -1.0;
    int bi = 0;
    for (int r = lane; r < d; r += 64) {
      const double x = X[r];
      ss = fma(x, x, ss);
      const double v = fabs(X[dp + r]);
      if (v > best) { best = v; bi = r; }  // first index of the lane's largest
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      ss += __shfl_xor(ss, off);
      const double ob = __shfl_xor(best, off);
      const int oi = __shfl_xor(bi, off);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    ss = __shfl(ss, 0);
    bi = __shfl(bi, 0);
    if (lane == 0) {
      sig[j] = sqrt(ss);
      sgn[j] = X[dp + bi] < 0.0 ? -1.0 : 1.0;
    }
  }
  __syncthreads();
  for (int j = tid; j < d; j += blockDim.x) {
    const double sj = sig[j];
    int rank = 0;
    for (int i = 0; i < d; ++i) rank += (sig[i] > sj) || (sig[i] == sj && i < j);
    sig_out[rank] = sj;
    src[rank] = j;
    sgn_out[rank] = sgn[j];
  }
  if (tid == 0 && flags[nflags - 1] != 0) info->status = 5;  // no convergence in nflags sweeps
}

// U[r][o] = sgn x_j[r] / sigma_j (0 if sigma_j = 0), V[r][o] = sgn v_j[r],
// S[o] = sigma_j with j = src[o]; row-major outputs.
template <typename T>
__global__ __launch_bounds__(256) void svd_out_kernel(const double* __restrict__ XV, int d, int dp, const double* __restrict__ sig,
                                                      const int32_t* __restrict__ src,
                                                      const double* __restrict__ sgn, T* __restrict__ U,
                                                      int64_t ldu, T* __restrict__ S, T* __restrict__ V,
                                                      int64_t ldv) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)d * d) return;
  const int o = (int)(e / d), r = (int)(e % d);  // consecutive threads: consecutive rows of one column
  const double* X = XV + (int64_t)src[o] * 2 * dp;  // x_j, then v_j
  const double s = sig[o], g = sgn[o];
  U[(int64_t)r * ldu + o] = (T)(s > 0.0 ? g * X[r] / s : 0.0);
  V[(int64_t)r * ldv + o] = (T)(g * X[dp + r]);
  if (r == 0) S[o] = (T)s;
}

size_t svd_ws_bytes(int d) {
  const int dp = svd_padded(d);
  return svd_align((size_t)dp * 2 * dp * sizeof(double)) + svd_align(kSvSweeps * sizeof(int32_t)) +
         svd_align((size_t)d * sizeof(double)) * 2 + svd_align((size_t)d * sizeof(int32_t));
}

template <typename T>
hipError_t launch_svd_small(const T* M, int64_t ldm, int d, T* U, int64_t ldu, T* S, T* V, int64_t ldv, void* ws,
                            void* info, hipStream_t s) {
  if (d < 1 || d > kDMax) return hipErrorInvalidValue;
  const int dp = svd_padded(d), nb = dp / kSvW;
  char* p = (char*)ws;
  double* XV = (double*)p;
  p += svd_align((size_t)dp * 2 * dp * sizeof(double));
  int32_t* flags = (int32_t*)p;
  p += svd_align(kSvSweeps * sizeof(int32_t));
  double* sig = (double*)p;
  p += svd_align((size_t)d * sizeof(double));
  double* sgn = (double*)p;
  p += svd_align((size_t)d * sizeof(double));
  int32_t* src = (int32_t*)p;
  const int64_t tot = (int64_t)dp * 2 * dp;
  hipLaunchKernelGGL((svd_init_kernel<T>), dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, M, ldm, d, dp, XV,
                     flags, kSvSweeps);
  const size_t shmem = (size_t)kSvCols * 2 * dp * sizeof(double);
  // R = ceil(dp / 64) rows of each column half per lane (1 .. kSvRows)
  const void* fn = nullptr;
  switch ((dp + 63) / 64) {
    case 1: fn = reinterpret_cast<const void*>(svd_sweeps_kernel<1>); break;
    case 2: fn = reinterpret_cast<const void*>(svd_sweeps_kernel<2>); break;
    case 3: fn = reinterpret_cast<const void*>(svd_sweeps_kernel<3>); break;
    case 4: fn = reinterpret_cast<const void*>(svd_sweeps_kernel<4>); break;
    case 5: fn = reinterpret_cast<const void*>(svd_sweeps_kernel<5>); break;
    case 6: fn = reinterpret_cast<const void*>(svd_sweeps_kernel<6>); break;
    case 7: fn = reinterpret_cast<const void*>(svd_sweeps_kernel<7>); break;
    case 8: fn = reinterpret_cast<const void*>(svd_sweeps_kernel<8>); break;
    default: fn = reinterpret_cast<const void*>(svd_sweeps_kernel<kSvRows>); break;
  }
  if (shmem > 65536) {  // more than 64 KB of LDS for the columns of wide pairs
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
  }
  double tol = (double)dp * 1.1102230246251565e-16;
  int max_sweeps = kSvSweeps;
  void* args[] = {&XV, (void*)&dp, (void*)&nb, &flags, &max_sweeps, &tol};
  // at most 34 workgroups of one CU each: the whole grid is resident at once
  const hipError_t e = hipLaunchCooperativeKernel(fn, dim3((unsigned)(nb / 2)), dim3(kSvThreads), args,
                                                  (unsigned)shmem, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(svd_order_kernel, dim3(1), dim3(1024), 0, s, XV, d, dp, flags, kSvSweeps, sig, src, sgn,
                     (DevInfo*)info);
  hipLaunchKernelGGL((svd_out_kernel<T>), dim3((unsigned)ceil_div((int64_t)d * d, 256)), dim3(256), 0, s, XV, d, dp,
                     sig, src, sgn, U, ldu, S, V, ldv);
  return hipGetLastError();
}

template hipError_t launch_svd_small<float>(const float*, int64_t, int, float*, int64_t, float*, float*, int64_t,
                                            void*, void*, hipStream_t);
template hipError_t launch_svd_small<double>(const double*, int64_t, int, double*, int64_t, double*, double*,
                                             int64_t, void*, void*, hipStream_t);

}  // namespace rqlp
