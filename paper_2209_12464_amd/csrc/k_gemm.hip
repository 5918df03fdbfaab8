// Dense products with A on the matrix cores: Y = A X (NN) and Y = A^T X (TN),
// the sketch, power-step and projection products of Algorithms 1 and 2.
//
// The output is tall and skinny (d columns), so one workgroup owns a BM-row
// slab of Y and all of its columns up to 256 (wider outputs take equal
// column passes): A is streamed from HBM once per product and pass.  To fill 256 CUs the reduction dimension is split
// (split-K); each split writes a partial slab and a second kernel sums the
// partials in a fixed order, so results are bitwise reproducible.
// Workgroup ids are remapped so that an XCD works on a contiguous range of
// (split, slab) pairs: the X chunk of a split then stays in that XCD's L2.
//
// Tiles: 8 waves as 4 (rows) x 2 (columns); each wave owns 16 MB rows and
// half of the BN = 32 * NBW columns, i.e. MB x NBW blocks of 16 x 16
// accumulated with the 16x16x4 MFMA (float or double).  MB = 2 (128-row
// slabs, two workgroups per CU) is the default shape; MB = 4 (256-row slabs,
// float only, one workgroup per CU, fewer LDS operand reads per MFMA) is the
// alternative the autotuner may pick per product shape.  BK = 16 along the
// reduction.  A and X tiles are staged through LDS, double buffered with
// register prefetch, one barrier per K step.
#include "common.h"
#include "grouped.h"
#include "kernels.h"

#include <algorithm>

namespace rqlp {

constexpr int kGemmThreads = 512;
constexpr int kBK = 16;

// One workgroup's share: tile `logical` = split * mtiles + slab.
template <typename T, int NBW, bool TRANS, bool AVEC, bool BVEC, int MB>
__device__ __attribute__((always_inline)) inline void gemm_body(
    const T* __restrict__ A, int64_t lda, const T* __restrict__ B, int64_t ldb,
    T* __restrict__ C, int64_t ldc, int64_t cslice, int M, int N, int K, int kchunk, int mtiles,
    int nst, int logical) {
  typedef Mfma<T> MF;
  constexpr int BM = 64 * MB;              // 4 row groups x 16 MB rows
  constexpr int BN = 32 * NBW;             // 2 column halves x NBW blocks of 16
  constexpr int VEC = 16 / sizeof(T);
  // LDS row strides of 16 (mod 32) words: the two k-rows an operand read
  // touches in one 32-lane half then fall in disjoint banks
  constexpr int AS = BM + 16;              // A tile, k-major
  constexpr int BS = BN + 16;              // X tile
  constexpr int A_ELEMS = BM * kBK / kGemmThreads;   // 2 MB per thread
  static_assert(MB == 2 || MB == 4, "row tile of 128 or 256 rows");
  constexpr int A_VECS = A_ELEMS / VEC;
  constexpr int B_VECS = (kBK * BN / VEC + kGemmThreads - 1) / kGemmThreads;
  constexpr int B_ELEMS = BVEC ? B_VECS * VEC : (kBK * BN + kGemmThreads - 1) / kGemmThreads;

  __shared__ __attribute__((aligned(16))) T As[2][kBK][AS];
  __shared__ __attribute__((aligned(16))) T Bs[2][kBK][BS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave & 3, wn = wave >> 2;
  const int split = logical / mtiles;
  const int mt = logical - split * mtiles;
  const int m0 = mt * BM;
  const int kbeg = split * kchunk;
  const int kend = min(K, kbeg + kchunk);

  T areg[A_ELEMS];
  T breg[B_ELEMS];

  auto load_tile = [&](int k0) {
    if constexpr (!TRANS) {
      // A tile rows m0..m0+BM, cols k0..k0+BK (A is M x K)
      if constexpr (AVEC) {
#pragma unroll
        for (int v = 0; v < A_VECS; ++v) {
          const int idx = tid + kGemmThreads * v;
          const int r = idx / (kBK / VEC), kv = idx % (kBK / VEC);
          const int gr = m0 + r, gk = k0 + kv * VEC;
          if (gr < M && gk + VEC <= kend) {
            const T* p = A + (int64_t)gr * lda + gk;
            if constexpr (VEC == 4) {
              const floatx4 x = *reinterpret_cast<const floatx4*>(p);
#pragma unroll
              for (int e = 0; e < VEC; ++e) areg[v * VEC + e] = x[e];
            } else {
              const double2 x = *reinterpret_cast<const double2*>(p);
              areg[v * VEC + 0] = x.x;
              areg[v * VEC + 1] = x.y;
            }
          } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e)
              areg[v * VEC + e] = (gr < M && gk + e < kend) ? A[(int64_t)gr * lda + gk + e] : (T)0;
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < A_ELEMS; ++i) {
          const int idx = tid + kGemmThreads * i;
          const int r = idx / kBK, kk = idx % kBK;
          const int gr = m0 + r, gk = k0 + kk;
          areg[i] = (gr < M && gk < kend) ? A[(int64_t)gr * lda + gk] : (T)0;
        }
      }
    } else {
      // A^T tile: rows k0..k0+BK of A (K x M), cols m0..m0+BM
      if constexpr (AVEC) {
#pragma unroll
        for (int v = 0; v < A_VECS; ++v) {
          const int idx = tid + kGemmThreads * v;
          const int kk = idx / (BM / VEC), rv = idx % (BM / VEC);
          const int gk = k0 + kk, gc = m0 + rv * VEC;
          if (gk < kend && gc + VEC <= M) {
            const T* p = A + (int64_t)gk * lda + gc;
            if constexpr (VEC == 4) {
              const floatx4 x = *reinterpret_cast<const floatx4*>(p);
#pragma unroll
              for (int e = 0; e < VEC; ++e) areg[v * VEC + e] = x[e];
            } else {
              const double2 x = *reinterpret_cast<const double2*>(p);
              areg[v * VEC + 0] = x.x;
              areg[v * VEC + 1] = x.y;
            }
          } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e)
              areg[v * VEC + e] = (gk < kend && gc + e < M) ? A[(int64_t)gk * lda + gc + e] : (T)0;
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < A_ELEMS; ++i) {
          const int idx = tid + kGemmThreads * i;
          const int kk = idx / BM, r = idx % BM;
          const int gk = k0 + kk, gc = m0 + r;
          areg[i] = (gk < kend && gc < M) ? A[(int64_t)gk * lda + gc] : (T)0;
        }
      }
    }
    if constexpr (BVEC) {
      // X rows are BN wide with zero padding beyond N (internal buffers)
#pragma unroll
      for (int v = 0; v < B_VECS; ++v) {
        const int idx = tid + kGemmThreads * v;
        const int kk = idx / (BN / VEC), nv = idx % (BN / VEC);
        const int gk = k0 + kk;
        const bool ok = idx < kBK * BN / VEC && gk < kend;
        if constexpr (VEC == 4) {
          floatx4 x = {0.f, 0.f, 0.f, 0.f};
          if (ok) x = *reinterpret_cast<const floatx4*>(B + (int64_t)gk * ldb + nv * VEC);
#pragma unroll
          for (int e = 0; e < VEC; ++e) breg[v * VEC + e] = x[e];
        } else {
          double2 x = {0.0, 0.0};
          if (ok) x = *reinterpret_cast<const double2*>(B + (int64_t)gk * ldb + nv * VEC);
          breg[v * VEC + 0] = x.x;
          breg[v * VEC + 1] = x.y;
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < B_ELEMS; ++i) {
        const int idx = tid + kGemmThreads * i;
        const int kk = idx / BN, n = idx % BN;
        const int gk = k0 + kk;
        breg[i] = (idx < kBK * BN && gk < kend && n < N) ? B[(int64_t)gk * ldb + n] : (T)0;
      }
    }
  };

  auto store_tile = [&](int buf) {
    if constexpr (!TRANS) {
      if constexpr (AVEC) {
#pragma unroll
        for (int v = 0; v < A_VECS; ++v) {
          const int idx = tid + kGemmThreads * v;
          const int r = idx / (kBK / VEC), kv = idx % (kBK / VEC);
#pragma unroll
          for (int e = 0; e < VEC; ++e) As[buf][kv * VEC + e][r] = areg[v * VEC + e];
        }
      } else {
#pragma unroll
        for (int i = 0; i < A_ELEMS; ++i) {
          const int idx = tid + kGemmThreads * i;
          As[buf][idx % kBK][idx / kBK] = areg[i];
        }
      }
    } else {
      if constexpr (AVEC) {
#pragma unroll
        for (int v = 0; v < A_VECS; ++v) {
          const int idx = tid + kGemmThreads * v;
          const int kk = idx / (BM / VEC), rv = idx % (BM / VEC);
#pragma unroll
          for (int e = 0; e < VEC; ++e) As[buf][kk][rv * VEC + e] = areg[v * VEC + e];
        }
      } else {
#pragma unroll
        for (int i = 0; i < A_ELEMS; ++i) {
          const int idx = tid + kGemmThreads * i;
          As[buf][idx / BM][idx % BM] = areg[i];
        }
      }
    }
    if constexpr (BVEC) {
#pragma unroll
      for (int v = 0; v < B_VECS; ++v) {
        const int idx = tid + kGemmThreads * v;
        if (idx < kBK * BN / VEC) {
          const int kk = idx / (BN / VEC), nv = idx % (BN / VEC);
#pragma unroll
          for (int e = 0; e < VEC; ++e) Bs[buf][kk][nv * VEC + e] = breg[v * VEC + e];
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < B_ELEMS; ++i) {
        const int idx = tid + kGemmThreads * i;
        if (idx < kBK * BN) Bs[buf][idx / BN][idx % BN] = breg[i];
      }
    }
  };

  typename MF::acc_t acc[MB][NBW];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb) acc[mb][nb] = MF::zero();

  const int arow = wm * 16 * MB + (lane & 15);
  const int bcol = wn * (BN / 2) + (lane & 15);
  if (kbeg < kend) {
    load_tile(kbeg);
    store_tile(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = kbeg; k0 < kend; k0 += kBK) {
      const bool more = k0 + kBK < kend;
      if (more) load_tile(k0 + kBK);
      __builtin_amdgcn_s_setprio(1);
      // The operands of step ks + 1 are read from LDS while the MFMAs of
      // step ks issue, and the wave's priority is raised for the MFMA loop
      // so that the co-resident workgroup's loads and stores fill its gaps.
      T aa[2][MB], bb[2][NBW];
      {
        const int kr = (lane >> 4);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) aa[0][mb] = As[buf][kr][arow + 16 * mb];
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb) bb[0][nb] = Bs[buf][kr][bcol + nb * 16];
      }
#pragma unroll
      for (int ks = 0; ks < kBK / 4; ++ks) {
        const int cur = ks & 1, nxt = cur ^ 1;
        if (ks + 1 < kBK / 4) {
          const int kr = (ks + 1) * 4 + (lane >> 4);
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) aa[nxt][mb] = As[buf][kr][arow + 16 * mb];
#pragma unroll
          for (int nb = 0; nb < NBW; ++nb) bb[nxt][nb] = Bs[buf][kr][bcol + nb * 16];
        }
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb)
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) acc[mb][nb] = MF::mma(aa[cur][mb], bb[cur][nb], acc[mb][nb]);
        __builtin_amdgcn_sched_barrier(0);
      }
      __builtin_amdgcn_s_setprio(0);
      if (more) store_tile(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }

  // ---- epilogue: write the slab (or this split's partial slab) ----
  T* Cs = C + (int64_t)split * cslice;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb) {
      const int col = wn * (BN / 2) + nb * 16 + MF::col(lane);
#pragma unroll
      for (int r = 0; r < MF::NACC; ++r) {
        const int row = m0 + wm * 16 * MB + mb * 16 + MF::row(lane, r);
        if (row < M && col < nst) Cs[(int64_t)row * ldc + col] = acc[mb][nb][r];
      }
    }
}

template <typename T, int NBW, bool TRANS, bool AVEC, bool BVEC, int MB>
__global__ __launch_bounds__(kGemmThreads) void gemm_kernel(
    const T* __restrict__ A, int64_t lda, const T* __restrict__ B, int64_t ldb,
    T* __restrict__ C, int64_t ldc, int64_t cslice, int M, int N, int K, int kchunk, int mtiles,
    int nst) {
  gemm_body<T, NBW, TRANS, AVEC, BVEC, MB>(A, lda, B, ldb, C, ldc, cslice, M, N, K, kchunk, mtiles, nst,
                                           xcd_remap(blockIdx.x, gridDim.x));
}

struct GemmRecArgs {
  const void* A;
  const void* B;
  void* C;
  int64_t lda, ldb, ldc, cslice;
  int M, N, K, kchunk, mtiles, nst;
};

template <typename T, int NBW, bool TRANS, bool AVEC, bool BVEC, int MB>
__global__ __launch_bounds__(kGemmThreads) void gemm_grouped(const GemmRecArgs* __restrict__ a,
                                                             const int* __restrict__ start, int count) {
  const int p = group_find(start, count, blockIdx.x);
  const GemmRecArgs g = a[p];
  gemm_body<T, NBW, TRANS, AVEC, BVEC, MB>((const T*)g.A, g.lda, (const T*)g.B, g.ldb, (T*)g.C, g.ldc, g.cslice,
                                           g.M, g.N, g.K, g.kchunk, g.mtiles, g.nst, (int)blockIdx.x - start[p]);
}

template <typename T, int NBW, bool TRANS, bool AVEC, bool BVEC, int MB>
void gemm_grouped_launch(const void* args, const int* start, int count, unsigned blocks, hipStream_t s) {
  hipLaunchKernelGGL((gemm_grouped<T, NBW, TRANS, AVEC, BVEC, MB>), dim3(blocks), dim3(kGemmThreads), 0, s,
                     (const GemmRecArgs*)args, start, count);
}

// Y[i][j] = sum_s P[s][i][j] in order s = 0..nsplit-1 (i < M, j < nst).
template <typename T>
__device__ __attribute__((always_inline)) inline void splitk_reduce_body(const T* __restrict__ P, int64_t ldp,
                                                                         int64_t pslice, int nsplit,
                                                                         T* __restrict__ Y, int64_t ldy, int M,
                                                                         int nst, int bid, int nblk) {
  const int64_t total = (int64_t)M * nst;
  for (int64_t e = bid * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)nblk * blockDim.x) {
    const int64_t i = e / nst, j = e - i * nst;
    T s = P[i * ldp + j];
    for (int t = 1; t < nsplit; ++t) s += P[t * pslice + i * ldp + j];
    Y[i * ldy + j] = s;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const T* __restrict__ P, int64_t ldp, int64_t pslice,
                                                            int nsplit, T* __restrict__ Y, int64_t ldy, int M,
                                                            int nst) {
  splitk_reduce_body<T>(P, ldp, pslice, nsplit, Y, ldy, M, nst, blockIdx.x, gridDim.x);
}

// The same sum, four consecutive outputs per thread with 16-byte accesses
// (float; rows of P and Y 16-byte aligned, nst a multiple of 4).  The
// additions run in the same order, so the results are the same bits.
__device__ __attribute__((always_inline)) inline void splitk_reduce4_body(const float* __restrict__ P, int64_t ldp,
                                                                          int64_t pslice, int nsplit,
                                                                          float* __restrict__ Y, int64_t ldy, int M,
                                                                          int nst, int bid, int nblk) {
  const int64_t total = (int64_t)M * (nst / 4);
  for (int64_t e = bid * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)nblk * blockDim.x) {
    const int64_t i = e / (nst / 4), j = (e - i * (nst / 4)) * 4;
    floatx4 s = *reinterpret_cast<const floatx4*>(P + i * ldp + j);
    for (int t = 1; t < nsplit; ++t) {
      const floatx4 v = *reinterpret_cast<const floatx4*>(P + t * pslice + i * ldp + j);
#pragma unroll
      for (int c = 0; c < 4; ++c) s[c] += v[c];
    }
    *reinterpret_cast<floatx4*>(Y + i * ldy + j) = s;
  }
}

__global__ __launch_bounds__(256) void splitk_reduce4_kernel(const float* __restrict__ P, int64_t ldp,
                                                             int64_t pslice, int nsplit, float* __restrict__ Y,
                                                             int64_t ldy, int M, int nst) {
  splitk_reduce4_body(P, ldp, pslice, nsplit, Y, ldy, M, nst, blockIdx.x, gridDim.x);
}

struct SplitkArgs {
  const void* P;
  void* Y;
  int64_t ldp, pslice, ldy;
  int nsplit, M, nst;
};

template <typename T, bool V4>
__global__ __launch_bounds__(256) void splitk_grouped(const SplitkArgs* __restrict__ a, const int* __restrict__ start,
                                                      int count) {
  const int p = group_find(start, count, blockIdx.x);
  const SplitkArgs g = a[p];
  const int bid = (int)blockIdx.x - start[p], nb = start[p + 1] - start[p];
  if constexpr (V4)
    splitk_reduce4_body((const float*)g.P, g.ldp, g.pslice, g.nsplit, (float*)g.Y, g.ldy, g.M, g.nst, bid, nb);
  else
    splitk_reduce_body<T>((const T*)g.P, g.ldp, g.pslice, g.nsplit, (T*)g.Y, g.ldy, g.M, g.nst, bid, nb);
}

template <typename T, bool V4>
void splitk_grouped_launch(const void* args, const int* start, int count, unsigned blocks, hipStream_t s) {
  hipLaunchKernelGGL((splitk_grouped<T, V4>), dim3(blocks), dim3(256), 0, s, (const SplitkArgs*)args, start, count);
}

// The ordered reduction of nsplit slabs (4-wide when the layout allows).
template <typename T>
static void splitk_dispatch(const T* P, int nsplit, int M, int nst, T* Y, int64_t ldy, hipStream_t s) {
  const bool vec4 = sizeof(T) == 4 && nst % 4 == 0 && ldy % 4 == 0 && ((uintptr_t)Y & 15) == 0 &&
                    ((uintptr_t)P & 15) == 0;
  const int64_t total = (int64_t)M * (vec4 ? nst / 4 : nst);
  const int64_t gr = ceil_div(total, 256);
  // every output is summed by one thread in a fixed order, so the block
  // count only sets how many outputs a thread takes in turn
  const unsigned blocks = (unsigned)(gr < 2048 ? gr : 2048);
  const SplitkArgs a{P, Y, (int64_t)nst, (int64_t)M * nst, ldy, nsplit, M, nst};
  if (vec4) {
    if (!record_launch(&splitk_grouped_launch<float, true>, a, blocks))
      hipLaunchKernelGGL(splitk_reduce4_kernel, dim3(blocks), dim3(256), 0, s, (const float*)P, (int64_t)nst,
                         (int64_t)M * nst, nsplit, (float*)Y, ldy, M, nst);
  } else {
    if (!record_launch(&splitk_grouped_launch<T, false>, a, blocks))
      hipLaunchKernelGGL(splitk_reduce_kernel<T>, dim3(blocks), dim3(256), 0, s, P, (int64_t)nst, (int64_t)M * nst,
                         nsplit, Y, ldy, M, nst);
  }
}

template <typename T, int NBW, bool TRANS, int MB>
static void launch_nb(const GemmArgs<T>& g, hipStream_t s, int grid, T* C, int64_t ldc,
                      int64_t cslice, int nst) {
#define RQLP_GEMM_LAUNCH(AV, BV)                                                                                 \
  do {                                                                                                             \
    if (!record_launch(&gemm_grouped_launch<T, NBW, TRANS, AV, BV, MB>,                                            \
                       GemmRecArgs{g.A, g.B, C, g.lda, g.ldb, ldc, cslice, g.M, g.N, g.K, g.kchunk, g.mtiles, nst}, \
                       (unsigned)grid))                                                                            \
      hipLaunchKernelGGL((gemm_kernel<T, NBW, TRANS, AV, BV, MB>), dim3(grid), dim3(kGemmThreads), 0, s, g.A,       \
                         g.lda, g.B, g.ldb, C, ldc, cslice, g.M, g.N, g.K, g.kchunk, g.mtiles, nst);               \
  } while (0)
  if (g.avec && g.bvec) RQLP_GEMM_LAUNCH(true, true);
  else if (g.avec) RQLP_GEMM_LAUNCH(true, false);
  else if (g.bvec) RQLP_GEMM_LAUNCH(false, true);
  else RQLP_GEMM_LAUNCH(false, false);
#undef RQLP_GEMM_LAUNCH
}

template <typename T, bool TRANS, int MB>
static void dispatch_nb_mb(const GemmArgs<T>& g, hipStream_t s, int grid, T* C, int64_t ldc,
                           int64_t cslice, int nst) {
  switch (gemm_block_cols<T>(g.N) / 32) {
    case 1: launch_nb<T, 1, TRANS, MB>(g, s, grid, C, ldc, cslice, nst); break;
    case 2: launch_nb<T, 2, TRANS, MB>(g, s, grid, C, ldc, cslice, nst); break;
    case 3: launch_nb<T, 3, TRANS, MB>(g, s, grid, C, ldc, cslice, nst); break;
    case 4: launch_nb<T, 4, TRANS, MB>(g, s, grid, C, ldc, cslice, nst); break;
    case 5: launch_nb<T, 5, TRANS, MB>(g, s, grid, C, ldc, cslice, nst); break;
    case 6: launch_nb<T, 6, TRANS, MB>(g, s, grid, C, ldc, cslice, nst); break;
    case 7: launch_nb<T, 7, TRANS, MB>(g, s, grid, C, ldc, cslice, nst); break;
    default: launch_nb<T, 8, TRANS, MB>(g, s, grid, C, ldc, cslice, nst); break;
  }
}

template <typename T, bool TRANS>
static void dispatch_nb(const GemmArgs<T>& g, hipStream_t s, int grid, T* C, int64_t ldc,
                        int64_t cslice, int nst) {
  if constexpr (sizeof(T) == 4) {
    if (g.mb == 4) {
      dispatch_nb_mb<T, TRANS, 4>(g, s, grid, C, ldc, cslice, nst);
      return;
    }
  }
  dispatch_nb_mb<T, TRANS, 2>(g, s, grid, C, ldc, cslice, nst);
}

template <typename T>
int gemm_block_rows(int mb) { return 64 * ((sizeof(T) == 4 && mb == 4) ? 4 : 2); }
template int gemm_block_rows<float>(int);
template int gemm_block_rows<double>(int);

template <typename T>
int gemm_block_cols(int N) { return (int)round_up(N, 32); }
template int gemm_block_cols<float>(int);
template int gemm_block_cols<double>(int);

// Widest column tile of one pass; wider outputs are cut into equal passes
// of at most this many columns (A is then streamed once per pass).
constexpr int kGemmMaxCols = 256;

// Launch the main kernel (into C directly when nsplit == 1, else into the
// partial buffer P) once per column pass and, for nsplit > 1, the ordered
// reduction over the full width.
template <typename T>
hipError_t launch_gemm(GemmArgs<T> g, T* Y, int64_t ldy, int nst, T* P, hipStream_t s,
                       hipEvent_t ev0, hipEvent_t ev1) {
  if (g.M <= 0 || nst <= 0) return hipSuccess;
  const int grid = g.mtiles * g.nsplit;
  const int npass = (int)ceil_div(round_up(g.N, 32), kGemmMaxCols);
  const int cw = (int)round_up(ceil_div(g.N, npass), 32);
  if (ev0) (void)hipEventRecord(ev0, s);
  for (int c0 = 0; c0 < g.N; c0 += cw) {
    GemmArgs<T> gc = g;
    gc.B = g.B + c0;
    gc.N = std::min(cw, g.N - c0);
    // the last pass also writes the zero columns [N, nst)
    const int nst_c = (c0 + cw >= g.N) ? nst - c0 : cw;
    if (g.nsplit == 1) {
      if (g.trans) dispatch_nb<T, true>(gc, s, grid, Y + c0, ldy, 0, nst_c);
      else dispatch_nb<T, false>(gc, s, grid, Y + c0, ldy, 0, nst_c);
    } else {
      const int64_t ldp = nst;
      const int64_t pslice = (int64_t)g.M * ldp;
      if (g.trans) dispatch_nb<T, true>(gc, s, grid, P + c0, ldp, pslice, nst_c);
      else dispatch_nb<T, false>(gc, s, grid, P + c0, ldp, pslice, nst_c);
    }
  }
  if (g.nsplit > 1) splitk_dispatch<T>(P, g.nsplit, g.M, nst, Y, ldy, s);
  // the timed interval covers the product and its split-K reduction
  if (ev1) (void)hipEventRecord(ev1, s);
  return hipGetLastError();
}
hipError_t launch_splitk_reduce_f32(const float* P, int nsplit, int M, int nst, float* Y, int64_t ldy,
                                    hipStream_t s) {
  splitk_dispatch<float>(P, nsplit, M, nst, Y, ldy, s);
  return hipGetLastError();
}

template hipError_t launch_gemm<float>(GemmArgs<float>, float*, int64_t, int, float*, hipStream_t,
                                       hipEvent_t, hipEvent_t);
template hipError_t launch_gemm<double>(GemmArgs<double>, double*, int64_t, int, double*,
                                        hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace rqlp
