// BFloat16 products with float32 accumulation (the reduced-precision form of
// the sketch, power-step and projection products of Algorithms 1 and 2):
// A is rounded to bfloat16 once per decomposition, each right-hand factor
// (Omega, Q, W) once per product, and the matrix cores accumulate the exact
// bfloat16 products in float32.  Everything after the product (Gram matrix,
// Cholesky factor, inverse, solve) stays as in the float32 form.
//
// The 16x16x32 bf16 MFMA takes 8 consecutive reduction indices per lane, so
// both operands are kept k-contiguous: A as stored (row-major m x n) for
// A X, a transposed copy of A for A^T X (both made by one conversion pass),
// and the right-hand factor transposed (d x K) by a small conversion kernel.
// The product kernel is then a single "NT" form, Y = A_op X^T_op: 128-row
// slabs with all columns per workgroup (A read once), split-K with the
// ordered float32 reduction.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace rqlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));

// s_waitcnt immediate that waits until at most n vector memory operations
// are outstanding (expcnt and lgkmcnt left at their no-wait maxima)
constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }

// float -> bfloat16 bits, round to nearest with ties to even (NaN stays NaN)
__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------------------
// conversions: 64 x 64 tiles through LDS

constexpr int kCvT = 64;

// A (m x n float, lda) -> Ab (m x ldb, bf16) and, if At != null, At (n x
// ldt, bf16) = A^T.  Columns [n, ldb) of Ab and [m, ldt) of At are zero.
__global__ __launch_bounds__(256) void cvt_bf16_kernel(const float* __restrict__ A, int64_t lda, int64_t m,
                                                       int64_t n, uint16_t* __restrict__ Ab, int64_t ldb,
                                                       uint16_t* __restrict__ At, int64_t ldt, bool vec) {
  __shared__ uint16_t tile[kCvT][kCvT + 2];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.y * kCvT, c0 = (int64_t)blockIdx.x * kCvT;
  const int cl = (tid & 15) * 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int rl = (tid >> 4) + 16 * i;
    const int64_t r = r0 + rl;
    u16x4 v;
    if (vec && r < m && c0 + cl + 4 <= n) {  // one 16-byte load
      const floatx4 x = *reinterpret_cast<const floatx4*>(A + r * lda + c0 + cl);
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = f2bf(x[j]);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t c = c0 + cl + j;
        v[j] = (r < m && c < n) ? f2bf(A[r * lda + c]) : (uint16_t)0;
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) tile[rl][cl + j] = v[j];
    if (r < m && c0 + cl < ldb) {
      if (c0 + cl + 4 <= ldb) {
        *reinterpret_cast<u16x4*>(Ab + r * ldb + c0 + cl) = v;
      } else {
        for (int j = 0; j < 4 && c0 + cl + j < ldb; ++j) Ab[r * ldb + c0 + cl + j] = v[j];
      }
    }
  }
  if (!At) return;
  __syncthreads();
  // At[c][r] for the tile: thread writes 4 consecutive r of one c
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int ccl = (tid >> 4) + 16 * i;
    const int rl = (tid & 15) * 4;
    const int64_t c = c0 + ccl;
    if (c >= n) continue;
    u16x4 v;
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = tile[rl + j][ccl];
    const int64_t r = r0 + rl;
    if (r < ldt) {
      if (r + 4 <= ldt) {
        *reinterpret_cast<u16x4*>(At + c * ldt + r) = v;
      } else {
        for (int j = 0; j < 4 && r + j < ldt; ++j) At[c * ldt + r + j] = v[j];
      }
    }
  }
}

hipError_t launch_cvt_bf16(const float* A, int64_t lda, int64_t m, int64_t n, uint16_t* Ab, int64_t ldb,
                           uint16_t* At, int64_t ldt, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  // the grid covers the padded extents so that the zero padding is written
  const int64_t cols = std::max<int64_t>(ldb, n), rows = At ? std::max<int64_t>(ldt, m) : m;
  dim3 grid((unsigned)ceil_div(cols, kCvT), (unsigned)ceil_div(rows, kCvT));
  const bool vec = lda % 4 == 0 && ((uintptr_t)A & 15) == 0;  // rows 16-byte aligned: vector loads
  hipLaunchKernelGGL(cvt_bf16_kernel, grid, dim3(256), 0, s, A, lda, m, n, Ab, ldb, At, ldt, vec);
  return hipGetLastError();
}

// X (K x N float, ldx) -> Xt (N x ldt bf16) = X^T, columns [K, ldt) zero.
hipError_t launch_cvt_bf16_t(const float* X, int64_t ldx, int64_t K, int64_t N, uint16_t* Xt, int64_t ldt,
                             hipStream_t s) {
  if (K <= 0 || N <= 0) return hipSuccess;
  // only the transposed copy is wanted: Ab is written to a null-sized target
  dim3 grid((unsigned)ceil_div(N, kCvT), (unsigned)ceil_div(std::max<int64_t>(ldt, K), kCvT));
  const bool vec = ldx % 4 == 0 && ((uintptr_t)X & 15) == 0;
  hipLaunchKernelGGL(cvt_bf16_kernel, grid, dim3(256), 0, s, X, ldx, K, N, (uint16_t*)nullptr, (int64_t)0, Xt,
                     ldt, vec);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// the product: C (M x nst slab of split `split`) = A[M x K] Xt[N x K]^T
//
// 8 waves as 2 (row groups of 64) x 4 (column groups of 16 NF); a
// workgroup owns a 128-row slab and all BN = 64 NF <= 576 columns, so A is
// read once per product.  Per 32-wide reduction step a wave issues 4 NF
// MFMAs (4 row fragments x NF column fragments).  Operand tiles go straight
// from global memory to LDS (16 bytes per lane, no register staging)
// through a ring of three stages: the tiles of step i + 2 are requested
// while step i computes, one barrier per step.  A tile row is 64 bytes (32
// bf16); its four 16-byte chunks are stored XOR-swizzled by (row / 2) mod
// 4, so that the 8 lanes the LDS serves together (8 consecutive rows of
// one chunk column) cover all 128 bytes of a bank cycle once (the (row /
// 4) mod 4 swizzle left two-way conflicts: six times the conflict cycles).  K is a multiple of 32 (zero padded) and so is every split, so no
// step needs masking; rows past M or N are read clamped (their results are
// not stored, or stored as zero).

constexpr int kBfThreads = 512;
constexpr int kBfBK = 32;                 // one bf16 MFMA step; 64-byte tile rows
constexpr int kBfBM = 128;
constexpr int kBfMaxNF = 9;               // up to 576 columns per workgroup
constexpr int kBfStages = 3;

typedef __attribute__((address_space(3))) void* lds_ptr_t;

__device__ inline int bf_swz(int row, int chunk) { return chunk ^ ((row >> 1) & 3); }

template <int NF>
__global__ __launch_bounds__(kBfThreads) void gemm_bf16_kernel(const uint16_t* __restrict__ A, int64_t lda,
                                                               const uint16_t* __restrict__ Xt, int64_t ldx,
                                                               float* __restrict__ C, int64_t ldc, int64_t cslice,
                                                               int M, int N, int K, int kchunk, int mtiles,
                                                               int nst) {
  constexpr int BM = kBfBM, BN = 64 * NF;
  constexpr int ROWS = BM + BN;                 // tile rows per stage (A rows, then Xt rows)
  constexpr int NLOADS = ROWS / 16;             // 1 KB wave loads per stage
  constexpr int LMIN = NLOADS / 8;              // loads per step of the waves that issue fewest
  __shared__ __attribute__((aligned(1024))) uint16_t tiles[kBfStages][ROWS * kBfBK];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave & 1, wn = wave >> 1;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int split = logical / mtiles;
  const int mt = logical - split * mtiles;
  const int m0 = mt * BM;
  const int kbeg = split * kchunk;
  const int kend = min(K, kbeg + kchunk);
  const int nsteps = kend > kbeg ? (kend - kbeg) / kBfBK : 0;

  // wave load j covers tile rows 16 j .. 16 j + 15; lane i fills the i-th
  // 16-byte slot: row 16 j + i / 4, stored chunk i % 4, logical chunk
  // bf_swz(row, i % 4)
  auto issue = [&](int st, int k0) {
#pragma unroll
    for (int u = 0; u < (NLOADS + 7) / 8; ++u) {
      const int j = wave + 8 * u;
      if (j < NLOADS) {
        const int row = 16 * j + (lane >> 2);
        const int ch = bf_swz(row, lane & 3);
        const uint16_t* src;
        if (row < BM) {
          const int gr = min(m0 + row, M - 1);
          src = A + (int64_t)gr * lda + k0 + ch * 8;
        } else {
          const int gn = min(row - BM, N - 1);
          src = Xt + (int64_t)gn * ldx + k0 + ch * 8;
        }
        __builtin_amdgcn_global_load_lds(src, (lds_ptr_t)&tiles[st][16 * j * kBfBK], 16, 0, 0);
      }
    }
  };

  floatx4 acc[4][NF];
#pragma unroll
  for (int rf = 0; rf < 4; ++rf)
#pragma unroll
    for (int cf = 0; cf < NF; ++cf) acc[rf][cf] = (floatx4)0.0f;
  const int kc = lane >> 4;  // this lane's 8-element chunk of the 32-wide step
  // Per step: the four A fragments and the first G column fragments are
  // read, then the column fragments go in groups of G: the reads of group
  // g + 1 are issued right after the first product of group g (whose
  // operands the compiler waits for; with direct-to-LDS loads in flight it
  // can only wait for all outstanding LDS reads), so they complete under the
  // other 4 G - 1 products of the group.  The scheduling barriers keep that
  // order.
  auto compute = [&](int st) {
    const uint16_t* T = tiles[st];
    constexpr int G = 3, NG = (NF + G - 1) / G;
    __builtin_amdgcn_s_setprio(1);
    bf16x8 a[4], b[NF];
    auto frag = [&](int row) {
      return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&T[row * kBfBK + bf_swz(row, kc) * 8]));
    };
#pragma unroll
    for (int rf = 0; rf < 4; ++rf) a[rf] = frag(wm * 64 + rf * 16 + (lane & 15));
#pragma unroll
    for (int cf = 0; cf < G && cf < NF; ++cf) b[cf] = frag(BM + wn * 16 * NF + cf * 16 + (lane & 15));
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int c0 = g * G;
      acc[0][c0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[c0], acc[0][c0], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int cf = c0 + G; cf < c0 + 2 * G && cf < NF; ++cf) b[cf] = frag(BM + wn * 16 * NF + cf * 16 + (lane & 15));
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int cf = c0; cf < c0 + G && cf < NF; ++cf)
#pragma unroll
        for (int rf = 0; rf < 4; ++rf)
          if (cf != c0 || rf != 0)
            acc[rf][cf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rf], b[cf], acc[rf][cf], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
    __builtin_amdgcn_s_setprio(0);
  };

  if (nsteps > 0) issue(0, kbeg);
  if (nsteps > 1) issue(1, kbeg + kBfBK);
  int st = 0;
  for (int i = 0; i < nsteps; ++i) {
    // this wave's loads of step i are done once at most those of step i + 1 are pending
    if (i + 1 < nsteps) __builtin_amdgcn_s_waitcnt(vmcnt_imm(LMIN));
    else __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
    // every wave's step-i tiles are in, and every wave has consumed its
    // step i - 1 operands, so that stage may be refilled.  A plain barrier
    // (a compiler memory barrier, no fence): a fence would also wait for the
    // loads of step i + 1 still in flight.
    asm volatile("s_barrier" ::: "memory");
    if (i + 2 < nsteps) issue(st == 0 ? 2 : st - 1, kbeg + (i + 2) * kBfBK);
    compute(st);
    st = (st == kBfStages - 1) ? 0 : st + 1;
  }
  float* Cs = C + (int64_t)split * cslice;
#pragma unroll
  for (int rf = 0; rf < 4; ++rf)
#pragma unroll
    for (int cf = 0; cf < NF; ++cf) {
      const int col = wn * 16 * NF + cf * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 64 + rf * 16 + 4 * (lane >> 4) + r;
        if (row < M && col < nst) Cs[(int64_t)row * ldc + col] = (col < N) ? acc[rf][cf][r] : 0.0f;
      }
    }
}

// One workgroup per CU (registers and LDS), 256 CUs.  Large M: the split-K
// count s in 1..4 that fills whole rounds of 256 workgroups best (fewest
// splits on ties, since every split adds a partial slab to write and sum).
// Small M: enough splits to reach about 256 workgroups, each with a
// reduction chunk of at least 256.
void plan_gemm_bf16(int M, int K, int* mtiles, int* nsplit, int* kchunk) {
  *mtiles = (int)ceil_div(M, kBfBM);
  const int64_t kmax = std::max<int64_t>(1, ceil_div(K, 256));
  int64_t ns = 1;
  if (*mtiles >= 128) {
    double best = 0.0;
    for (int sc = 1; sc <= 4 && sc <= kmax; ++sc) {
      const int64_t wgs = (int64_t)*mtiles * sc;
      const double eff = (double)wgs / (256.0 * (double)ceil_div(wgs, 256));
      if (eff > best + 0.02) {
        best = eff;
        ns = sc;
      }
    }
  } else {
    ns = std::min<int64_t>(std::max(1, 256 / *mtiles), kmax);
  }
  *kchunk = (int)round_up(ceil_div(std::max(K, 1), ns), kBfBK);
  *nsplit = (int)ceil_div(std::max(K, 1), *kchunk);
}

size_t gemm_bf16_partial_elems(int M, int K, int dp) {
  int mt, ns, kc;
  plan_gemm_bf16(M, K, &mt, &ns, &kc);
  return ns > 1 ? (size_t)ns * M * dp : 0;
}

hipError_t launch_gemm_bf16(const uint16_t* A, int64_t lda, const uint16_t* Xt, int64_t ldx, int M, int N, int K,
                            float* Y, int64_t ldy, int nst, float* P, hipStream_t s, hipEvent_t ev0,
                            hipEvent_t ev1) {
  if (M <= 0 || nst <= 0) return hipSuccess;
  if (K % kBfBK != 0 || lda % 8 != 0 || ldx % 8 != 0 || N < 1) return hipErrorInvalidValue;
  int mtiles, nsplit, kchunk;
  plan_gemm_bf16(M, K, &mtiles, &nsplit, &kchunk);
  const int grid = mtiles * nsplit;
  float* C = nsplit == 1 ? Y : P;
  const int64_t ldc = nsplit == 1 ? ldy : nst;
  const int64_t cslice = nsplit == 1 ? 0 : (int64_t)M * nst;
  // outputs wider than 576 columns take equal column passes (A is streamed once per pass)
  const int npass = (int)ceil_div(round_up(N, 64), 64 * kBfMaxNF);
  const int cw = (int)round_up(ceil_div(N, npass), 64);
  if (ev0) (void)hipEventRecord(ev0, s);
#define RQLP_BF_LAUNCH(NF)                                                                                   \
  hipLaunchKernelGGL(gemm_bf16_kernel<NF>, dim3(grid), dim3(kBfThreads), 0, s, A, lda, Xt + (int64_t)c0 * ldx, ldx, \
                     C + c0, ldc, cslice, M, nc, K, kchunk, mtiles, nst_c)
  for (int c0 = 0; c0 < N; c0 += cw) {
    const int nc = std::min(cw, N - c0);
    const int nst_c = (c0 + cw >= N) ? nst - c0 : cw;  // the last pass also writes the zero columns
    switch ((int)ceil_div(nst_c, 64)) {
      case 1: RQLP_BF_LAUNCH(1); break;
      case 2: RQLP_BF_LAUNCH(2); break;
      case 3: RQLP_BF_LAUNCH(3); break;
      case 4: RQLP_BF_LAUNCH(4); break;
      case 5: RQLP_BF_LAUNCH(5); break;
      case 6: RQLP_BF_LAUNCH(6); break;
      case 7: RQLP_BF_LAUNCH(7); break;
      case 8: RQLP_BF_LAUNCH(8); break;
      default: RQLP_BF_LAUNCH(9); break;
    }
  }
#undef RQLP_BF_LAUNCH
  if (nsplit > 1) {
    const hipError_t e = launch_splitk_reduce_f32(P, nsplit, M, nst, Y, ldy, s);
    if (e != hipSuccess) return e;
  }
  // the timed interval covers the product and its split-K reduction
  if (ev1) (void)hipEventRecord(ev1, s);
  return hipGetLastError();
}

}  // namespace rqlp
