// Host runtime behind include/rqlp.h: argument checks, workspace planning,
// split-K planning and the launch sequence of the method (Algorithm 1 with
// the power iteration of Algorithm 2, column-sketch orientation).  All work
// goes on the caller's stream; nothing here synchronizes except
// rqlp_destroy, rqlp_get_info and rqlp_get_timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <fstream>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <new>
#include <vector>

#include "rqlp.h"
#include "common.h"
#include "grouped.h"
#include "kernels.h"

using namespace rqlp;

namespace rqlp {
LaunchRecorder*& launch_recorder();
}

struct rqlp_ctx {
  int device = 0;
  DevInfo* info = nullptr;      // device record
  void* ws_own = nullptr;       // internal workspace (grown on demand)
  size_t ws_own_bytes = 0;
  uint32_t timing = 0;          // bit k: time launches of kernel class k
  struct Pair { hipEvent_t a, b; };
  std::vector<Pair> recorded[RQLP_KT_COUNT];
  std::vector<hipEvent_t> pool;
  double total_ms[RQLP_KT_COUNT] = {0};
  int64_t launches[RQLP_KT_COUNT] = {0};
  // batches: decompositions spread over lanes (streams at the default
  // priority), forked from and joined back into the caller's stream
  static constexpr int kLanes = 8;
  // lockstep groups of a grouped batch (64 uneven requests: 13.9 ms with 3
  // groups; 16.8 / 14.7 / 15.2 / 15.1 / 14.3 / 16.5 ms with 1 / 2 / 4 / 5 / 6
  // / 8; 16.3 ms for sub-batches of identical launch sequences on 8 lanes)
  static constexpr int kLockGroups = 3;
  hipStream_t lanes[kLanes] = {};
  hipStream_t cap = nullptr;  // origin stream of graph captures
  hipEvent_t fork = nullptr, join[kLanes] = {};
  bool graphs = false;        // capture a repeated batch once, then replay it
  bool reset_info = true;     // off inside a batch (reset once for the whole batch)
  struct GraphEntry { std::vector<uint8_t> key; hipGraphExec_t exec; };
  std::vector<GraphEntry> graph_cache;
  std::vector<uint8_t> last_key;  // the last batch run eagerly
  // Grouped batches: every problem's launch sequence is recorded once (host
  // only), then replayed phase by phase as grouped launches whose argument
  // tables live in device memory; plans are cached per batch descriptor.
  struct GroupedLaunch { GroupedFn fn; size_t args_off, start_off; int count; unsigned blocks; int lane; };
  struct GroupedPlan {
    std::vector<uint8_t> key;
    void* dev = nullptr;  // argument tables and block offsets
    std::vector<GroupedLaunch> launches;
    int lanes = 1;  // streams the launches are spread over (lane 0: the caller's)
  };
  std::vector<GroupedPlan> plans;
  bool lockstep = true;  // grouped batches (else every problem on its lane stream)
  // autotuned product plans: (element bytes, trans, M, N, K) -> (split-K
  // count, row tile parameter mb)
  std::map<std::tuple<int, int, int, int, int>, std::pair<int, int>> plan;
};

namespace {


#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return RQLP_ERR_HIP;          \
  } while (0)

// ---- timing ---------------------------------------------------------------
struct EvPair { hipEvent_t a = nullptr, b = nullptr; };

hipEvent_t take_event(rqlp_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

EvPair timer(rqlp_ctx* c, rqlp_kernel_class k) {
  EvPair p;
  if (!(c->timing >> (int)k & 1u)) return p;
  p.a = take_event(c);
  p.b = take_event(c);
  if (p.a && p.b) c->recorded[k].push_back({p.a, p.b});
  return p;
}

void resolve_timing(rqlp_ctx* c) {
  for (int k = 0; k < RQLP_KT_COUNT; ++k) {
    for (auto& pr : c->recorded[k]) {
      float ms = 0.f;
      if (hipEventSynchronize(pr.b) == hipSuccess && hipEventElapsedTime(&ms, pr.a, pr.b) == hipSuccess) {
        c->total_ms[k] += ms;
        c->launches[k] += 1;
      }
      c->pool.push_back(pr.a);
      c->pool.push_back(pr.b);
    }
    c->recorded[k].clear();
  }
}

// ---- planning -------------------------------------------------------------
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

int padded_d(int d) { return (int)round_up(d, 32); }

int env_int(const char* name, int dflt) {
  const char* v = getenv(name);
  if (!v || !*v) return dflt;
  return atoi(v);
}

template <typename T>
GemmArgs<T> plan_gemm(int trans, const T* A, int64_t lda, const T* B, int64_t ldb, int M, int N, int K) {
  GemmArgs<T> g;
  g.A = A;
  g.lda = lda;
  g.B = B;
  g.ldb = ldb;
  g.M = M;
  g.N = N;
  g.K = K;
  g.trans = trans;
  g.mb = 2;
  g.mtiles = (int)ceil_div(M, gemm_block_rows<T>(g.mb));
  // Resident workgroup slots: two 4-wave workgroups per CU (register
  // limited), 256 CUs.  Split K so that all slabs x splits fit in one round.
  const int target = std::max(1, env_int("RQLP_GEMM_TARGET_WGS", 512));
  // at least 512 reduction steps per split: a small product is not cut into
  // many slivers (a batch of them fills the GPU anyway), a large one still
  // takes about two workgroups per CU
  const int64_t kmin = std::max(16, env_int("RQLP_GEMM_MIN_KCHUNK", 512));
  int64_t ns = target / g.mtiles;
  ns = std::min<int64_t>(ns, std::max<int64_t>(1, ceil_div(K, kmin)));
  ns = std::max<int64_t>(1, ns);
  g.kchunk = (int)round_up(ceil_div(std::max(K, 1), ns), 16);
  g.nsplit = (int)ceil_div(std::max(K, 1), g.kchunk);
  const int vec = 16 / (int)sizeof(T);
  g.avec = (lda % vec == 0) && (((uintptr_t)A & 15) == 0);
  g.bvec = false;
  return g;
}

// Largest split-K count a plan may take (default or autotuned): enough
// splits for about four workgroups per CU, none shorter than 256.
int splitk_cap(int M, int K) {
  const int64_t mt = ceil_div(M, 128);
  return (int)std::max<int64_t>(1, std::min<int64_t>(1024 / mt, ceil_div(std::max(K, 1), 256)));
}

// Row tile of 128 (mb = 2) or, for float, 256 (mb = 4) rows per workgroup.
template <typename T>
void set_tile(GemmArgs<T>& g, int mb) {
  g.mb = (sizeof(T) == 4 && mb == 4) ? 4 : 2;
  g.mtiles = (int)ceil_div(g.M, gemm_block_rows<T>(g.mb));
}

// Split the reduction into (about) ns parts of whole 16-element chunks.
template <typename T>
void set_split(GemmArgs<T>& g, int ns) {
  g.kchunk = (int)round_up(ceil_div(std::max(g.K, 1), std::max(ns, 1)), 16);
  g.nsplit = (int)ceil_div(std::max(g.K, 1), g.kchunk);
}

// Partial-slab capacity of the workspaces: enough for any plan up to the cap.
template <typename T>
size_t gemm_partial_elems(int M, int K, int dp) {
  GemmArgs<T> g = plan_gemm<T>(0, (const T*)nullptr, 16, (const T*)nullptr, dp, M, dp, K);
  const int ns = std::max(g.nsplit, splitk_cap(M, K));
  return ns > 1 ? (size_t)ns * M * dp : 0;
}

// Layout of the dense / CSR decomposition workspace.
struct Layout {
  size_t om, yb, qi, q1, part, gp, g, r1, r2, rinv, flags, xf, esq, csr_rt, csr_ct, csr_vt, csr_scr;
  size_t ab, at, xt;  // bfloat16 products: A, A^T and the transposed right-hand factor
  size_t total;
};

// leading dimension of a k-contiguous bfloat16 operand of reduction length K
// (the product kernel takes whole 32-wide reduction steps; padding is zero)
int64_t bf16_ld(int64_t K) { return round_up(K, 32); }

template <typename T>
Layout layout(int64_t m, int64_t n, int d, bool sparse, int64_t nnz, bool bf16 = false) {
  const int dp = padded_d(d);
  const int64_t mx = std::max(m, n);
  Layout L;
  size_t off = 0;
  auto put = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  L.om = put((size_t)n * dp * sizeof(T));
  L.yb = put((size_t)mx * dp * sizeof(T));
  L.qi = put((size_t)m * dp * sizeof(T));
  L.q1 = put((size_t)mx * dp * sizeof(double));
  size_t pe = 0;
  if (!sparse) pe = std::max(gemm_partial_elems<T>((int)m, (int)n, dp), gemm_partial_elems<T>((int)n, (int)m, dp));
  if (!sparse)  // the paper orientation's P = P-bar P-tilde (reduction over d)
    pe = std::max({pe, gemm_partial_elems<T>((int)m, d, dp), gemm_partial_elems<T>((int)n, d, dp)});
  if (bf16) pe = std::max(gemm_bf16_partial_elems((int)m, (int)bf16_ld(n), dp),
                          gemm_bf16_partial_elems((int)n, (int)bf16_ld(m), dp));
  L.part = put(pe * sizeof(T));
  const int gc = std::max(gram_chunks(m, dp), gram_chunks(n, dp));
  L.gp = put((size_t)gc * dp * dp * sizeof(double));
  L.g = put((size_t)dp * dp * sizeof(double));
  L.r1 = put((size_t)dp * dp * sizeof(double));
  L.r2 = put((size_t)dp * dp * sizeof(double));
  L.rinv = put((size_t)dp * kTile * sizeof(double));
  L.flags = put((size_t)(2 * dp + 2) * sizeof(int32_t));
  L.xf = put((size_t)dp * dp * sizeof(double));
  L.esq = put((size_t)(gram_reduce_blocks(dp) + dp) * sizeof(double));  // + the original diagonal
  if (sparse) {
    L.csr_rt = put((size_t)(n + 1) * sizeof(int32_t));
    L.csr_ct = put((size_t)nnz * sizeof(int32_t));
    L.csr_vt = put((size_t)nnz * sizeof(T));
    L.csr_scr = put(csr_transpose_scratch_bytes(m, n, nnz));
  } else {
    L.csr_rt = L.csr_ct = L.csr_vt = L.csr_scr = 0;
  }
  if (bf16) {
    L.ab = put((size_t)m * bf16_ld(n) * 2);
    L.at = put((size_t)n * bf16_ld(m) * 2);
    L.xt = put((size_t)dp * bf16_ld(mx) * 2);
  } else {
    L.ab = L.at = L.xt = 0;
  }
  L.total = off + 256;
  return L;
}

rqlp_status get_workspace(rqlp_ctx* c, void* ws, size_t ws_bytes, size_t need, char** base) {
  if (ws) {
    if (ws_bytes < need) return RQLP_ERR_OUT_OF_MEMORY;
    *base = (char*)ws;
  } else {
    if (c->ws_own_bytes < need) {
      if (c->ws_own) {
        if (hipDeviceSynchronize() != hipSuccess) return RQLP_ERR_HIP;
        hipFree(c->ws_own);
        c->ws_own = nullptr;
        c->ws_own_bytes = 0;
      }
      if (hipMalloc(&c->ws_own, need) != hipSuccess) return RQLP_ERR_OUT_OF_MEMORY;
      c->ws_own_bytes = need;
    }
    *base = (char*)c->ws_own;
  }
  // 256-byte alignment of the base
  *base = (char*)(((uintptr_t)*base + 255) & ~(uintptr_t)255);
  return RQLP_OK;
}

struct Bufs {
  double *q1, *gp, *g, *r1, *r2, *rinv, *xf, *esq;
  int32_t* flags;  // 2 dp dependent-column flags, then the two pass modes
};

// Largest ||Q1^T Q1 - I||_F for which the first-order second-pass factor is
// used: its orthogonality error ~||E||_F^2 / 4 stays below the output's
// rounding (2^-52 for float64, far below 2^-24 for float32).
double fast_tol_for(bool fp64) { return fp64 ? 0x1p-26 : 0x1p-18; }

// Key of the completion stream of one CholeskyQR pass.
uint64_t completion_key(int orth_index, int pass) {
  return kSketchKey1 + 1 + 2 * (uint64_t)orth_index + (uint64_t)pass;
}

// R = chol(G) and its explicit inverse for one CholeskyQR pass (R: r1 or r2,
// flags and mode of that pass).  While a batch is being recorded, the
// factorization forms a phase of its own, so that the factorizations of all
// problems of the batch are grouped together.
hipError_t factor(rqlp_ctx* c, const Bufs& b, double* R, int32_t* flags, int d, int dp, int orth_index,
                  double ftol, int32_t* mode, int nesq, hipStream_t s) {
  LaunchRecorder* rec = launch_recorder();
  if (rec) ++rec->cur_phase;
  EvPair t = timer(c, RQLP_KT_CHOL);
  hipError_t e = launch_chol(b.g, d, dp, R, b.rinv, flags, c->info, orth_index, ftol, b.esq, nesq, mode, b.xf,
                             b.esq + nesq, s, t.a, t.b);
  if (e == hipSuccess) e = launch_trinv(R, b.rinv, dp, mode, b.xf, s);
  if (rec) ++rec->cur_phase;
  return e;
}

// orth()/qr() of a rows x d matrix Y (ld ldy) by CholeskyQR2.  Pass 1 writes
// the float64 basis Q1; pass 2 writes out1 (ld1, ncols1 columns) and
// optionally out2.  R1, R2 and the flags of both passes stay in `b`.
// single: the basis only feeds the next product of a power iteration, and
// pass 1 writes it to out1 at once.  The second pass would only multiply it
// by an upper-triangular factor (Q1 = Q R2), which leaves the next
// orthonormalization's Q factor unchanged (the QR of A^T Q R2 is Z (S R2) when
// A^T Q = Z S), and pass 1 keeps Q1 well conditioned (its Gram matrix is
// within c cond(Y)^2 u of I), so only rounding differs.
template <typename T>
rqlp_status cholqr2(rqlp_ctx* c, const T* Y, int64_t ldy, int64_t rows, int d, const Bufs& b,
                    T* out1, int64_t ld1, int ncols1, T* out2, int64_t ld2, int ncols2,
                    uint64_t seed, int orth_index, hipStream_t s, bool lowp2 = false, bool single = false) {
  const int dp = padded_d(d);
  const int gch = gram_chunks(rows, dp);
  const double ftol = fast_tol_for(sizeof(T) == 8);
  int32_t* mode = b.flags + 2 * dp;
  const int nesq = gram_reduce_blocks(dp);
  EvPair t = timer(c, RQLP_KT_GRAM);
  HIP_TRY(launch_gram<T>(Y, ldy, rows, d, dp, b.gp, gch, b.g, b.esq, c->info, s, t.a, t.b));
  HIP_TRY(factor(c, b, b.r1, b.flags, d, dp, orth_index, 0.0, mode, nesq, s));
  t = timer(c, RQLP_KT_APPLY);
  if (single) {
    HIP_TRY((launch_apply<T, T>(Y, ldy, rows, d, dp, b.flags, mode, b.xf, out1, ld1, ncols1, out2, ld2, ncols2, seed,
                                completion_key(orth_index, 0), s, t.a, t.b)));
    return RQLP_OK;
  }
  HIP_TRY((launch_apply<T, double>(Y, ldy, rows, d, dp, b.flags, mode, b.xf, b.q1, dp, dp, nullptr, 0, 0, seed,
                                   completion_key(orth_index, 0), s, t.a, t.b)));
  // second pass: Q1 is orthonormal to working accuracy.  For float output
  // the product on the fast path (X = I - F, ||F||_F below 2^-19) takes
  // float32 arithmetic, which changes Q by less than its own rounding; with
  // lowp2 (the bfloat16 form) so does the Gram matrix.
  t = timer(c, RQLP_KT_GRAM);
  if (lowp2 && sizeof(T) == 4)
    HIP_TRY(launch_gram_f32c(b.q1, dp, rows, d, dp, b.gp, gch, b.g, b.esq, c->info, s, t.a, t.b));
  else
    HIP_TRY(launch_gram<double>(b.q1, dp, rows, d, dp, b.gp, gch, b.g, b.esq, c->info, s, t.a, t.b));
  HIP_TRY(factor(c, b, b.r2, b.flags + dp, d, dp, orth_index, ftol, mode + 1, nesq, s));
  t = timer(c, RQLP_KT_APPLY);
  if constexpr (sizeof(T) == 4)
    HIP_TRY(launch_apply_f32fast(b.q1, dp, rows, d, dp, b.flags + dp, mode + 1, b.xf, out1, ld1, ncols1, out2, ld2,
                                 ncols2, seed, completion_key(orth_index, 1), s, t.a, t.b));
  else
    HIP_TRY((launch_apply<double, T>(b.q1, dp, rows, d, dp, b.flags + dp, mode + 1, b.xf, out1, ld1, ncols1, out2,
                                     ld2, ncols2, seed, completion_key(orth_index, 1), s, t.a, t.b)));
  return RQLP_OK;
}

template <typename T>
rqlp_status gemm(rqlp_ctx* c, int trans, const T* A, int64_t lda, int64_t m, int64_t n, const T* X,
                 int64_t ldx, int d, T* Y, int64_t ldy, int nst, T* P, hipStream_t s, bool padded_x) {
  // trans = 0: Y (m x nst) = A X (K = n); trans = 1: Y (n x nst) = A^T X (K = m)
  const int M = (int)(trans ? n : m), K = (int)(trans ? m : n);
  GemmArgs<T> g = plan_gemm<T>(trans, A, lda, X, ldx, M, d, K);
  auto it = c->plan.find(std::make_tuple((int)sizeof(T), trans, M, d, K));
  if (it != c->plan.end()) {
    set_tile(g, it->second.second);
    set_split(g, std::min(it->second.first, splitk_cap(M, K)));
  }
  // internal operands have ld = dp and zero padding columns: vector loads
  const int vec = 16 / (int)sizeof(T);
  g.bvec = padded_x && ldx == gemm_block_cols<T>(d) && ldx % vec == 0 && (((uintptr_t)X & 15) == 0);
  EvPair t = timer(c, trans ? RQLP_KT_GEMM_TN : RQLP_KT_GEMM_NN);
  HIP_TRY(launch_gemm<T>(g, Y, ldy, nst, P, s, t.a, t.b));
  return RQLP_OK;
}

bool valid_prec(rqlp_precision p) { return p == RQLP_FP64 || p == RQLP_FP32 || p == RQLP_BF16_REFINED; }

rqlp_status check_common(int64_t m, int64_t n, int k, int p, int q, rqlp_precision prec) {
  if (m < 1 || n < 1 || k < 1 || p < 0 || q < 0 || !valid_prec(prec)) return RQLP_ERR_INVALID_ARG;
  const int64_t d = (int64_t)k + p;
  if (d > std::min(m, n)) return RQLP_ERR_INVALID_ARG;
  if (m > INT32_MAX || n > INT32_MAX) return RQLP_ERR_UNSUPPORTED;
  if (d > kDMax) return RQLP_ERR_UNSUPPORTED;
  return RQLP_OK;
}

// The method's launch sequence for dense (mulA = GEMM) or CSR (mulA = SpMM)
// A: Algorithm 1 with Algorithm 2 in the column-sketch orientation.  Q (ld d)
// may be null (the basis then stays in the internal Q buffer, ld dp); L is
// written with leading dimension ldl (d when ldl <= 0).
template <typename T, typename MulA, typename MulAt>
rqlp_status run_method(rqlp_ctx* c, char* base, const Layout& Lo, int64_t m, int64_t n, int k, int p,
                       int q, uint64_t seed, T* Q, T* Lout, T* V, hipStream_t s, MulA mulA, MulAt mulAt,
                       int ldl = 0, bool lowp2 = false) {
  const int d = k + p, dp = padded_d(d);
  T* om = (T*)(base + Lo.om);
  T* yb = (T*)(base + Lo.yb);
  T* qi = (T*)(base + Lo.qi);
  Bufs b;
  b.q1 = (double*)(base + Lo.q1);
  b.gp = (double*)(base + Lo.gp);
  b.g = (double*)(base + Lo.g);
  b.r1 = (double*)(base + Lo.r1);
  b.r2 = (double*)(base + Lo.r2);
  b.rinv = (double*)(base + Lo.rinv);
  b.flags = (int32_t*)(base + Lo.flags);
  b.xf = (double*)(base + Lo.xf);
  b.esq = (double*)(base + Lo.esq);
  rqlp_status st;
  if (c->reset_info) HIP_TRY(launch_info_reset(c->info, s));
  // Omega (n x d, ld dp), then Y = A Omega and Q = orth(Y)
  HIP_TRY(launch_gaussian<T>(seed, kSketchKey1, n, d, om, dp, s));
  if ((st = mulA(om, yb)) != RQLP_OK) return st;
  // the bases that only feed the next product of the power iteration take
  // one CholeskyQR pass (see cholqr2); the returned Q and the final QR two
  int oi = 1;
  if ((st = cholqr2<T>(c, yb, dp, m, d, b, qi, dp, dp, q == 0 ? Q : nullptr, d, d, seed, oi++, s, lowp2, q > 0)) !=
      RQLP_OK)
    return st;
  for (int it = 1; it <= q; ++it) {
    // W = orth(A^T Q) (stored in the Omega buffer), Q = orth(A W)
    if ((st = mulAt(qi, yb)) != RQLP_OK) return st;
    if ((st = cholqr2<T>(c, yb, dp, n, d, b, om, dp, dp, nullptr, 0, 0, seed, oi++, s, lowp2, true)) != RQLP_OK)
      return st;
    if ((st = mulA(om, yb)) != RQLP_OK) return st;
    if ((st = cholqr2<T>(c, yb, dp, m, d, b, qi, dp, dp, it == q ? Q : nullptr, d, d, seed, oi++, s, lowp2,
                         it < q)) != RQLP_OK)
      return st;
  }
  // B^T = A^T Q; [V, R] = qr(B^T); L = R^T
  if ((st = mulAt(qi, yb)) != RQLP_OK) return st;
  if ((st = cholqr2<T>(c, yb, dp, n, d, b, V, d, d, nullptr, 0, 0, seed, oi++, s, lowp2)) != RQLP_OK) return st;
  HIP_TRY(launch_form_l<T>(b.r2, b.r1, b.flags, d, dp, Lout, ldl > 0 ? ldl : d, s));
  return RQLP_OK;
}

// The paper's own orientation (Algorithm 1 as printed, with Algorithm 2):
// the column-sketch method applied to A^T (its Gaussian is then m x d, its
// basis the paper's P-bar, its right factor the paper's Q and its L the
// transposed R of the paper's QR), followed by the d x d QR of that L and
// P = P-bar P-tilde.  Lo is the layout of the n x m problem.
template <typename T, typename MulA, typename MulAt>
rqlp_status run_method_paper(rqlp_ctx* c, char* base, const Layout& Lo, int64_t m, int64_t n, int k, int p, int q,
                             uint64_t seed, T* Q, T* Lout, T* P, hipStream_t s, MulA mulA, MulAt mulAt) {
  const int d = k + p, dp = padded_d(d);
  T* rt = (T*)(base + Lo.om);  // R^T (d x dp), after the method on A^T
  T* pt = (T*)(base + Lo.yb);  // P-tilde (d x dp)
  T* pb = (T*)(base + Lo.qi);  // P-bar (n x dp), the basis of the method on A^T
  T* part = (T*)(base + Lo.part);
  rqlp_status st = run_method<T>(c, base, Lo, n, m, k, p, q, seed, nullptr, rt, Q, s, mulAt, mulA, dp);
  if (st != RQLP_OK) return st;
  Bufs b;
  b.q1 = (double*)(base + Lo.q1);
  b.gp = (double*)(base + Lo.gp);
  b.g = (double*)(base + Lo.g);
  b.r1 = (double*)(base + Lo.r1);
  b.r2 = (double*)(base + Lo.r2);
  b.rinv = (double*)(base + Lo.rinv);
  b.flags = (int32_t*)(base + Lo.flags);
  b.xf = (double*)(base + Lo.xf);
  b.esq = (double*)(base + Lo.esq);
  // [P-tilde, R-tilde] = qr(R^T) (the QR after the 2q + 2 of the method); L = R-tilde^T
  if ((st = cholqr2<T>(c, rt, dp, d, d, b, pt, dp, dp, nullptr, 0, 0, seed, 2 * q + 3, s)) != RQLP_OK) return st;
  HIP_TRY(launch_form_l<T>(b.r2, b.r1, b.flags, d, dp, Lout, d, s));
  return gemm<T>(c, 0, pb, dp, n, d, pt, dp, d, P, d, d, part, s, true);
}

template <typename T>
rqlp_status decompose_dense(rqlp_ctx* c, const T* A, int64_t m, int64_t n, int64_t lda, int k, int p, int q,
                            uint64_t seed, T* Q, T* L, T* V, void* ws, size_t ws_bytes, hipStream_t s) {
  const int d = k + p, dp = padded_d(d);
  const Layout Lo = layout<T>(m, n, d, false, 0);
  char* base = nullptr;
  rqlp_status st = get_workspace(c, ws, ws_bytes, Lo.total, &base);
  if (st != RQLP_OK) return st;
  T* part = (T*)(base + Lo.part);
  auto mulA = [&](const T* X, T* Y) { return gemm<T>(c, 0, A, lda, m, n, X, dp, d, Y, dp, dp, part, s, true); };
  auto mulAt = [&](const T* X, T* Y) { return gemm<T>(c, 1, A, lda, m, n, X, dp, d, Y, dp, dp, part, s, true); };
  return run_method<T>(c, base, Lo, m, n, k, p, q, seed, Q, L, V, s, mulA, mulAt);
}

template <typename T>
rqlp_status decompose_paper(rqlp_ctx* c, const T* A, int64_t m, int64_t n, int64_t lda, int k, int p, int q,
                            uint64_t seed, T* Q, T* L, T* P, void* ws, size_t ws_bytes, hipStream_t s) {
  const int d = k + p, dp = padded_d(d);
  const Layout Lo = layout<T>(n, m, d, false, 0);
  char* base = nullptr;
  rqlp_status st = get_workspace(c, ws, ws_bytes, Lo.total, &base);
  if (st != RQLP_OK) return st;
  T* part = (T*)(base + Lo.part);
  auto mulA = [&](const T* X, T* Y) { return gemm<T>(c, 0, A, lda, m, n, X, dp, d, Y, dp, dp, part, s, true); };
  auto mulAt = [&](const T* X, T* Y) { return gemm<T>(c, 1, A, lda, m, n, X, dp, d, Y, dp, dp, part, s, true); };
  return run_method_paper<T>(c, base, Lo, m, n, k, p, q, seed, Q, L, P, s, mulA, mulAt);
}

// RQLP_BF16_REFINED: A (float) is rounded to bfloat16 once, in both layouts;
// every product rounds its right-hand factor to bfloat16 and accumulates in
// float32; the rest of the method is the float32 form, except that the
// second CholeskyQR pass (of the orthonormalizations that take two: the
// returned basis and the final QR) runs its Gram matrix and (on its fast
// path) its product in float32 arithmetic.
rqlp_status decompose_dense_bf16(rqlp_ctx* c, const float* A, int64_t m, int64_t n, int64_t lda, int k, int p,
                                 int q, uint64_t seed, float* Q, float* L, float* V, void* ws, size_t ws_bytes,
                                 hipStream_t s) {
  const int d = k + p, dp = padded_d(d);
  const Layout Lo = layout<float>(m, n, d, false, 0, true);
  char* base = nullptr;
  rqlp_status st = get_workspace(c, ws, ws_bytes, Lo.total, &base);
  if (st != RQLP_OK) return st;
  float* part = (float*)(base + Lo.part);
  uint16_t* ab = (uint16_t*)(base + Lo.ab);
  uint16_t* at = (uint16_t*)(base + Lo.at);
  uint16_t* xt = (uint16_t*)(base + Lo.xt);
  const int64_t ldn = bf16_ld(n), ldm = bf16_ld(m);
  HIP_TRY(launch_cvt_bf16(A, lda, m, n, ab, ldn, at, ldm, s));
  auto mulA = [&](const float* X, float* Y) -> rqlp_status {  // Y (m x dp) = A X, X n x dp
    HIP_TRY(launch_cvt_bf16_t(X, dp, n, dp, xt, ldn, s));
    EvPair t = timer(c, RQLP_KT_GEMM_NN);
    HIP_TRY(launch_gemm_bf16(ab, ldn, xt, ldn, (int)m, dp, (int)ldn, Y, dp, dp, part, s, t.a, t.b));
    return RQLP_OK;
  };
  auto mulAt = [&](const float* X, float* Y) -> rqlp_status {  // Y (n x dp) = A^T X, X m x dp
    HIP_TRY(launch_cvt_bf16_t(X, dp, m, dp, xt, ldm, s));
    EvPair t = timer(c, RQLP_KT_GEMM_TN);
    HIP_TRY(launch_gemm_bf16(at, ldm, xt, ldm, (int)n, dp, (int)ldm, Y, dp, dp, part, s, t.a, t.b));
    return RQLP_OK;
  };
  // the second CholeskyQR pass in float32 arithmetic where that is within
  // the form's own accuracy (bfloat16 operands)
  return run_method<float>(c, base, Lo, m, n, k, p, q, seed, Q, L, V, s, mulA, mulAt, 0, true);
}

template <typename T>
rqlp_status decompose_csr(rqlp_ctx* c, const int32_t* rowptr, const int32_t* colidx, const T* vals, int64_t m,
                          int64_t n, int64_t nnz, int k, int p, int q, uint64_t seed, T* Q, T* L, T* V, void* ws,
                          size_t ws_bytes, hipStream_t s) {
  const int d = k + p, dp = padded_d(d);
  const Layout Lo = layout<T>(m, n, d, true, nnz);
  char* base = nullptr;
  rqlp_status st = get_workspace(c, ws, ws_bytes, Lo.total, &base);
  if (st != RQLP_OK) return st;
  int32_t* rt = (int32_t*)(base + Lo.csr_rt);
  int32_t* ct = (int32_t*)(base + Lo.csr_ct);
  T* vt = (T*)(base + Lo.csr_vt);
  HIP_TRY(launch_csr_transpose<T>(rowptr, colidx, vals, m, n, nnz, rt, ct, vt, base + Lo.csr_scr, s));
  auto mulA = [&](const T* X, T* Y) -> rqlp_status {
    EvPair t = timer(c, RQLP_KT_SPMM);
    HIP_TRY(launch_spmm<T>(rowptr, colidx, vals, m, X, dp, d, Y, dp, dp, s, t.a, t.b));
    return RQLP_OK;
  };
  auto mulAt = [&](const T* X, T* Y) -> rqlp_status {
    EvPair t = timer(c, RQLP_KT_SPMM);
    HIP_TRY(launch_spmm<T>(rt, ct, vt, n, X, dp, d, Y, dp, dp, s, t.a, t.b));
    return RQLP_OK;
  };
  return run_method<T>(c, base, Lo, m, n, k, p, q, seed, Q, L, V, s, mulA, mulAt);
}

size_t orth_ws_bytes(int64_t rows, int d, rqlp_precision prec) {
  const int dp = padded_d(d);
  size_t off = 0;
  auto put = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  put((size_t)rows * dp * sizeof(double));                        // q1
  put((size_t)gram_chunks(rows, dp) * dp * dp * sizeof(double));  // gp
  put((size_t)dp * dp * sizeof(double) * 3);                      // g, r1, r2
  put((size_t)dp * kTile * sizeof(double));                       // rinv
  put((size_t)(2 * dp + 2) * sizeof(int32_t));                    // flags, modes
  put((size_t)dp * dp * sizeof(double));                          // explicit inverse
  put((size_t)(gram_reduce_blocks(dp) + dp) * sizeof(double));    // ||G - I||^2 partials, diagonal
  put((size_t)rows * dp * (prec == RQLP_FP64 ? 8 : 4));           // padded copy of the output
  (void)prec;
  return off + 256;
}


// ---- batches ---------------------------------------------------------------

size_t problem_ws_bytes(const rqlp_problem& P, rqlp_precision prec) {
  const int d = P.k + P.p;
  if (prec == RQLP_FP64) return align256(layout<double>(P.m, P.n, d, false, 0).total);
  return align256(layout<float>(P.m, P.n, d, false, 0, prec == RQLP_BF16_REFINED).total);
}

rqlp_status check_problem(const rqlp_problem& P, rqlp_precision prec) {
  if (!P.A || !P.Q || !P.L || !P.V || P.lda < P.n) return RQLP_ERR_INVALID_ARG;
  return check_common(P.m, P.n, P.k, P.p, P.q, prec);
}

rqlp_status make_lanes(rqlp_ctx* c) {
  if (c->fork) return RQLP_OK;
  for (int l = 0; l < rqlp_ctx::kLanes; ++l) {
    HIP_TRY(hipStreamCreateWithFlags(&c->lanes[l], hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&c->join[l], hipEventDisableTiming));
  }
  HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&c->fork, hipEventDisableTiming));
  return RQLP_OK;
}

// One problem of a batch, decomposed on `s` with its workspace slice `ws`.
rqlp_status run_problem(rqlp_ctx* c, const rqlp_problem& P, rqlp_precision prec, char* ws, size_t need,
                        hipStream_t s) {
  if (prec == RQLP_FP64)
    return decompose_dense<double>(c, (const double*)P.A, P.m, P.n, P.lda, P.k, P.p, P.q, P.seed, (double*)P.Q,
                                   (double*)P.L, (double*)P.V, ws, need, s);
  if (prec == RQLP_BF16_REFINED)
    return decompose_dense_bf16(c, (const float*)P.A, P.m, P.n, P.lda, P.k, P.p, P.q, P.seed, (float*)P.Q,
                                (float*)P.L, (float*)P.V, ws, need, s);
  return decompose_dense<float>(c, (const float*)P.A, P.m, P.n, P.lda, P.k, P.p, P.q, P.seed, (float*)P.Q,
                                (float*)P.L, (float*)P.V, ws, need, s);
}

// Enqueue the batch on `origin`, every problem's launch sequence on its own
// lane stream (problem i on lane i % kLanes, own workspace slice), forked
// from and joined back into `origin`.
rqlp_status run_batch_lanes(rqlp_ctx* c, int count, const rqlp_problem* probs, rqlp_precision prec, char* base,
                            hipStream_t origin) {
  HIP_TRY(launch_info_reset(c->info, origin));
  HIP_TRY(hipEventRecord(c->fork, origin));
  const int nl = std::min(count, (int)rqlp_ctx::kLanes);
  for (int l = 0; l < nl; ++l) HIP_TRY(hipStreamWaitEvent(c->lanes[l], c->fork, 0));
  const uint32_t timing = c->timing;
  c->timing = 0;
  c->reset_info = false;
  rqlp_status st = RQLP_OK;
  size_t off = 0;
  for (int i = 0; i < count && st == RQLP_OK; ++i) {
    const size_t need = problem_ws_bytes(probs[i], prec);
    st = run_problem(c, probs[i], prec, base + off, need, c->lanes[i % rqlp_ctx::kLanes]);
    off += need;
  }
  c->reset_info = true;
  c->timing = timing;
  for (int l = 0; l < nl; ++l) {
    HIP_TRY(hipEventRecord(c->join[l], c->lanes[l]));
    HIP_TRY(hipStreamWaitEvent(origin, c->join[l], 0));
  }
  return st;
}

LaunchRecorder*& recorder_slot() {
  static thread_local LaunchRecorder* r = nullptr;
  return r;
}

// Record every problem's launch sequence (host only) and lay the launches
// out as grouped launches: phase by phase (the factorizations form phases of
// their own), position by position within a phase, problems in batch order.
// Each problem's own launches keep their order, so its results are the bits
// of its solo run.  The argument tables and block offsets are uploaded once
// into device memory.
// Within a group of problems, every position takes one grouped launch per
// kernel variant present (the variants follow from d, alignment and the
// split-K plans), so the group's problems advance in lockstep.  With nlanes
// > 1 the problems are split into that many groups of about equal work,
// each on a lane stream of its own, so that the groups' launches run side by
// side.
rqlp_status layout_plan(rqlp_ctx* c, int count, const rqlp_problem* probs, const size_t* offs,
                        rqlp_precision prec, char* base, hipStream_t s, rqlp_ctx::GroupedPlan* plan,
                        std::vector<uint8_t>& table, int nlanes = 1) {
  std::vector<LaunchRecorder> recs((size_t)count);
  const uint32_t timing = c->timing;
  c->timing = 0;
  c->reset_info = false;
  rqlp_status st = RQLP_OK;
  size_t off = 0;
  for (int i = 0; i < count && st == RQLP_OK; ++i) {
    const size_t need = problem_ws_bytes(probs[i], prec);
    if (offs) off = offs[i];
    recorder_slot() = &recs[(size_t)i];
    st = run_problem(c, probs[i], prec, base + off, need, s);
    recorder_slot() = nullptr;
    off += need;
  }
  c->reset_info = true;
  c->timing = timing;
  if (st != RQLP_OK) return st;
  // positions: (phase, index within the phase) of every recorded launch
  int nphase = 0;
  for (auto& r : recs) nphase = std::max(nphase, r.cur_phase + 1);
  std::vector<std::vector<std::pair<size_t, size_t>>> spans((size_t)count);  // per problem: [begin, end) per phase
  size_t maxlen = 0;
  for (int i = 0; i < count; ++i) {
    const LaunchRecorder& r = recs[(size_t)i];
    spans[(size_t)i].assign((size_t)nphase, {0, 0});
    for (size_t k = 0; k < r.seq.size();) {
      size_t e = k;
      while (e < r.seq.size() && r.phase[e] == r.phase[k]) ++e;
      spans[(size_t)i][(size_t)r.phase[k]] = {k, e};
      maxlen = std::max(maxlen, e - k);
      k = e;
    }
  }
  table.clear();
  auto reserve = [&](size_t bytes) {
    const size_t o = (table.size() + 15) & ~(size_t)15;
    table.resize(o + bytes);
    return o;
  };
  plan->launches.clear();
  plan->lanes = 1;
  // one grouped launch of the given records (one kernel, same position)
  auto emit = [&](const std::vector<const LaunchRec*>& items, int lane) -> rqlp_status {
    const size_t asz = items[0]->size;
    const size_t aoff = reserve(asz * items.size());
    const size_t soff = reserve(sizeof(int) * (items.size() + 1));
    int total = 0;
    for (size_t t = 0; t < items.size(); ++t) {
      std::memcpy(table.data() + aoff + t * asz, items[t]->args, asz);
      std::memcpy(table.data() + soff + t * sizeof(int), &total, sizeof(int));
      if ((int64_t)total + items[t]->blocks > INT32_MAX) return RQLP_ERR_UNSUPPORTED;
      total += (int)items[t]->blocks;
    }
    std::memcpy(table.data() + soff + items.size() * sizeof(int), &total, sizeof(int));
    plan->launches.push_back({items[0]->fn, aoff, soff, (int)items.size(), (unsigned)total, lane});
    return RQLP_OK;
  };
  // all members in lockstep on one lane: per (phase, position) one grouped
  // launch per kernel variant present among them
  auto emit_lockstep = [&](const std::vector<int>& mem, int lane) -> rqlp_status {
    for (int ph = 0; ph < nphase; ++ph) {
      for (size_t j = 0; j < maxlen; ++j) {
        std::vector<GroupedFn> fns;
        for (int i : mem) {
          const auto sp = spans[(size_t)i][(size_t)ph];
          if (sp.first + j >= sp.second) continue;
          const LaunchRec& x = recs[(size_t)i].seq[sp.first + j];
          if (x.blocks > 0 && std::find(fns.begin(), fns.end(), x.fn) == fns.end()) fns.push_back(x.fn);
        }
        for (GroupedFn fn : fns) {
          std::vector<const LaunchRec*> items;
          for (int i : mem) {
            const auto sp = spans[(size_t)i][(size_t)ph];
            if (sp.first + j >= sp.second) continue;
            const LaunchRec& x = recs[(size_t)i].seq[sp.first + j];
            if (x.fn == fn && x.blocks > 0) items.push_back(&x);
          }
          const rqlp_status es = emit(items, lane);
          if (es != RQLP_OK) return es;
        }
      }
    }
    return RQLP_OK;
  };
  if (nlanes > 1) {
    // groups of problems in lockstep, one lane each: problems by work,
    // largest first, cut into contiguous runs of about equal work, so that
    // problems of similar size share a lane (lockstep makes a lane's
    // problems wait for its largest one at every position)
    std::vector<std::pair<double, int>> byw;
    double total = 0.0;
    for (int i = 0; i < count; ++i) {
      double w = 0.0;
      for (const auto& x : recs[(size_t)i].seq) w += x.blocks;
      byw.push_back({w, i});
      total += w;
    }
    std::stable_sort(byw.begin(), byw.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
    const int nl = std::max(1, std::min(nlanes, count));
    std::vector<std::vector<int>> groups((size_t)nl);
    double acc = 0.0;
    int g = 0;
    for (const auto& e : byw) {
      if (g < nl - 1 && acc >= total * (g + 1) / nl && !groups[(size_t)g].empty()) ++g;
      groups[(size_t)g].push_back(e.second);
      acc += e.first;
    }
    int used = 0;
    for (auto& mem : groups) {
      if (mem.empty()) continue;
      std::sort(mem.begin(), mem.end());  // batch order within a lane
      const rqlp_status es = emit_lockstep(mem, used);
      if (es != RQLP_OK) return es;
      ++used;
    }
    plan->lanes = std::max(used, 1);
    if (table.empty()) table.resize(16);
    return RQLP_OK;
  }
  std::vector<int> all((size_t)count);
  for (int i = 0; i < count; ++i) all[(size_t)i] = i;
  const rqlp_status es = emit_lockstep(all, 0);
  if (es != RQLP_OK) return es;
  if (table.empty()) table.resize(16);
  return RQLP_OK;
}

// layout_plan, then the tables into a device allocation of the plan's own.
rqlp_status build_plan(rqlp_ctx* c, int count, const rqlp_problem* probs, rqlp_precision prec, char* base,
                       hipStream_t s, rqlp_ctx::GroupedPlan* plan) {
  std::vector<uint8_t> table;
  rqlp_status st = layout_plan(c, count, probs, nullptr, prec, base, s, plan, table, rqlp_ctx::kLockGroups);
  if (st != RQLP_OK) return st;
  if (hipMalloc(&plan->dev, table.size()) != hipSuccess) {
    plan->dev = nullptr;
    return RQLP_ERR_OUT_OF_MEMORY;
  }
  if (hipMemcpy(plan->dev, table.data(), table.size(), hipMemcpyHostToDevice) != hipSuccess) return RQLP_ERR_HIP;
  return RQLP_OK;
}

// The grouped launches of a plan: lane 0 on `s`, the other lanes on the
// context's lane streams, forked from and joined back into `s`.
rqlp_status launch_plan(rqlp_ctx* c, const rqlp_ctx::GroupedPlan& plan, hipStream_t s) {
  HIP_TRY(launch_info_reset(c->info, s));
  const int nl = std::min(plan.lanes, (int)rqlp_ctx::kLanes);
  if (nl > 1) {
    HIP_TRY(hipEventRecord(c->fork, s));
    for (int l = 1; l < nl; ++l) HIP_TRY(hipStreamWaitEvent(c->lanes[l], c->fork, 0));
  }
  const char* dev = (const char*)plan.dev;
  for (const auto& L : plan.launches)
    L.fn(dev + L.args_off, (const int*)(dev + L.start_off), L.count, L.blocks, L.lane == 0 ? s : c->lanes[L.lane]);
  HIP_TRY(hipGetLastError());
  for (int l = 1; l < nl; ++l) {
    HIP_TRY(hipEventRecord(c->join[l], c->lanes[l]));
    HIP_TRY(hipStreamWaitEvent(s, c->join[l], 0));
  }
  return RQLP_OK;
}

void free_plan(rqlp_ctx::GroupedPlan& p) {
  if (p.dev) hipFree(p.dev);
  p.dev = nullptr;
}

std::vector<uint8_t> batch_key(int count, const rqlp_problem* probs, rqlp_precision prec, const void* ws,
                               size_t ws_bytes) {
  std::vector<uint8_t> key(sizeof(int) * 2 + sizeof(void*) + sizeof(size_t) + sizeof(rqlp_problem) * count);
  uint8_t* k = key.data();
  const int pr = (int)prec;
  std::memcpy(k, &count, sizeof(int)); k += sizeof(int);
  std::memcpy(k, &pr, sizeof(int)); k += sizeof(int);
  std::memcpy(k, &ws, sizeof(void*)); k += sizeof(void*);
  std::memcpy(k, &ws_bytes, sizeof(size_t)); k += sizeof(size_t);
  std::memcpy(k, probs, sizeof(rqlp_problem) * count);
  return key;
}

// ---- the SVD-like form (Remark 1) ------------------------------------------

// Workspace after the decomposition's own: the factors Q, L, V, the small
// SVD's buffers, U-bar, V-bar and the partial slabs of the two products.
struct SvdLayout { size_t q, l, v, svd, ub, vb, part, total; };

SvdLayout svd_layout(int64_t m, int64_t n, int d, rqlp_precision prec) {
  const size_t es = prec == RQLP_FP64 ? 8 : 4;
  const int dp = padded_d(d);
  SvdLayout L;
  size_t off = 0;
  auto put = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  L.q = put((size_t)m * d * es);
  L.l = put((size_t)d * d * es);
  L.v = put((size_t)n * d * es);
  L.svd = put(svd_ws_bytes(d));
  L.ub = put((size_t)d * d * es);
  L.vb = put((size_t)d * d * es);
  const size_t pe = prec == RQLP_FP64
                        ? std::max(gemm_partial_elems<double>((int)m, d, dp), gemm_partial_elems<double>((int)n, d, dp))
                        : std::max(gemm_partial_elems<float>((int)m, d, dp), gemm_partial_elems<float>((int)n, d, dp));
  L.part = put(pe * es);
  L.total = off;
  return L;
}

// L = U-bar diag(S) V-bar^T, then U = Q U-bar and W = V V-bar.
template <typename T>
rqlp_status svd_like(rqlp_ctx* c, const SvdLayout& Ly, char* b, int64_t m, int64_t n, int d, T* U, T* S, T* W,
                     hipStream_t s) {
  T* Q = (T*)(b + Ly.q);
  T* L = (T*)(b + Ly.l);
  T* V = (T*)(b + Ly.v);
  T* Ub = (T*)(b + Ly.ub);
  T* Vb = (T*)(b + Ly.vb);
  T* part = (T*)(b + Ly.part);
  HIP_TRY(launch_svd_small<T>(L, d, d, Ub, d, S, Vb, d, b + Ly.svd, c->info, s));
  rqlp_status st = gemm<T>(c, 0, Q, d, m, d, Ub, d, d, U, d, d, part, s, false);
  if (st != RQLP_OK) return st;
  return gemm<T>(c, 0, V, d, n, d, Vb, d, d, W, d, d, part, s, false);
}

// ---- autotuner --------------------------------------------------------------

// Time every candidate plan of one product shape (Y = op(A) X with d
// columns, as the decomposition issues it: X and Y with ld dp, zero padding):
// each row tile (128 rows; for float also 256) with each split-K count, and
// keep the fastest in the context's plan table.  Synchronizes.
template <typename T>
rqlp_status autotune_product(rqlp_ctx* c, int trans, const T* A, int64_t lda, int64_t m, int64_t n, int d, T* X,
                             T* Y, T* P, hipStream_t s, int* best_out) {
  const int dp = padded_d(d);
  const int M = (int)(trans ? n : m), K = (int)(trans ? m : n);
  GemmArgs<T> g0 = plan_gemm<T>(trans, A, lda, X, dp, M, d, K);
  const int vec = 16 / (int)sizeof(T);
  g0.bvec = dp == gemm_block_cols<T>(d) && dp % vec == 0 && (((uintptr_t)X & 15) == 0);
  const int cap = splitk_cap(M, K);
  std::vector<int> cand = {g0.nsplit};
  for (int ns : {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64})
    if (ns <= cap) cand.push_back(ns);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    return RQLP_ERR_HIP;
  }
  float best_ms = 0.f;
  int best = g0.nsplit, best_mb = g0.mb;
  bool any = false;
  rqlp_status st = RQLP_OK;
  std::vector<std::pair<int, int>> tried;
  std::vector<int> tiles = {2};
  if (sizeof(T) == 4) tiles.push_back(4);
  for (int mb : tiles)
  for (int ns : cand) {
    GemmArgs<T> g = g0;
    set_tile(g, mb);
    set_split(g, ns);
    const std::pair<int, int> key{g.mb, g.nsplit};
    if (std::find(tried.begin(), tried.end(), key) != tried.end()) continue;  // a plan already timed
    tried.push_back(key);
    float ms = 0.f, t = 0.f;
    bool ok = true;
    for (int r = 0; r < 7 && ok; ++r) {  // two warm-ups, then the fastest of five
      ok = hipEventRecord(e0, s) == hipSuccess && launch_gemm<T>(g, Y, dp, dp, P, s, nullptr, nullptr) == hipSuccess &&
           hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
           hipEventElapsedTime(&t, e0, e1) == hipSuccess;
      if (r >= 2) ms = (r == 2) ? t : std::min(ms, t);
    }
    if (!ok) { st = RQLP_ERR_HIP; break; }
    if (!any || ms < best_ms) {
      best_ms = ms;
      best = g.nsplit;
      best_mb = g.mb;
      any = true;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != RQLP_OK) return st;
  c->plan[std::make_tuple((int)sizeof(T), trans, M, d, K)] = {best, best_mb};
  if (best_out) *best_out = best;
  return RQLP_OK;
}

template <typename T>
rqlp_status autotune_dense(rqlp_ctx* c, const T* A, int64_t m, int64_t n, int64_t lda, int d, hipStream_t s,
                           int* best_nn, int* best_tn) {
  const int dp = padded_d(d);
  const size_t pe = std::max(gemm_partial_elems<T>((int)m, (int)n, dp), gemm_partial_elems<T>((int)n, (int)m, dp));
  const size_t xb = align256((size_t)std::max(m, n) * dp * sizeof(T));
  char* base = nullptr;
  rqlp_status st = get_workspace(c, nullptr, 0, 2 * xb + align256(pe * sizeof(T)) + 256, &base);
  if (st != RQLP_OK) return st;
  T* X = (T*)base;
  T* Y = (T*)(base + xb);
  T* P = (T*)(base + 2 * xb);
  HIP_TRY(hipMemsetAsync(X, 0, xb, s));  // operand values do not change the timing
  if ((st = autotune_product<T>(c, 0, A, lda, m, n, d, X, Y, P, s, best_nn)) != RQLP_OK) return st;
  return autotune_product<T>(c, 1, A, lda, m, n, d, X, Y, P, s, best_tn);
}

}  // namespace

// ---- scratch memory of the no-allocation entry point -------------------------
// One copy of this array lives on every GPU the library runs on, from the
// first use of this file's code object on that GPU until the process ends.
// Host code never uses the array's name as an address (on the host it is
// only a stand-in): the device address of each GPU's copy is looked up once
// per device at rqlp_create and kept in g_scratch.
static __device__ __align__(256) char scratch[RQLP_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Resolve this device's copy of `scratch` (the device must be current).
rqlp_status scratch_setup(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return RQLP_ERR_UNSUPPORTED;
  if (g_scratch[device]) return RQLP_OK;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return RQLP_ERR_HIP;
  g_scratch[device] = ptr;
  return RQLP_OK;
}

void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch[device] : nullptr;
}

}  // namespace

// ===========================================================================
extern "C" {

rqlp_status rqlp_create(rqlp_ctx** ctx, int device) {
  if (!ctx) return RQLP_ERR_INVALID_ARG;
  *ctx = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) return RQLP_ERR_HIP;
  if (device < 0 || device >= count) return RQLP_ERR_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return RQLP_ERR_HIP;
  const rqlp_status sst = scratch_setup(device);
  if (sst != RQLP_OK) return sst;
  rqlp_ctx* c = new (std::nothrow) rqlp_ctx();
  if (!c) return RQLP_ERR_OUT_OF_MEMORY;
  c->device = device;
  if (hipMalloc(&c->info, sizeof(DevInfo)) != hipSuccess) {
    delete c;
    return RQLP_ERR_OUT_OF_MEMORY;
  }
  if (hipMemset(c->info, 0, sizeof(DevInfo)) != hipSuccess) {
    hipFree(c->info);
    delete c;
    return RQLP_ERR_HIP;
  }
  *ctx = c;
  return RQLP_OK;
}

rqlp_status rqlp_destroy(rqlp_ctx* c) {
  if (!c) return RQLP_OK;
  hipSetDevice(c->device);
  hipDeviceSynchronize();
  resolve_timing(c);
  for (hipEvent_t e : c->pool) hipEventDestroy(e);
  for (auto& e : c->graph_cache) hipGraphExecDestroy(e.exec);
  for (auto& p : c->plans) free_plan(p);
  for (int l = 0; l < rqlp_ctx::kLanes; ++l) {
    if (c->lanes[l]) hipStreamDestroy(c->lanes[l]);
    if (c->join[l]) hipEventDestroy(c->join[l]);
  }
  if (c->cap) hipStreamDestroy(c->cap);
  if (c->fork) hipEventDestroy(c->fork);
  if (c->ws_own) hipFree(c->ws_own);
  if (c->info) hipFree(c->info);
  delete c;
  return RQLP_OK;
}

size_t rqlp_workspace_size(int64_t m, int64_t n, int k, int p, int q, rqlp_precision prec) {
  if (check_common(m, n, k, p, q, prec) != RQLP_OK) return 0;
  return prec == RQLP_FP64 ? layout<double>(m, n, k + p, false, 0).total
                           : layout<float>(m, n, k + p, false, 0, prec == RQLP_BF16_REFINED).total;
}

size_t rqlp_workspace_size_csr(int64_t m, int64_t n, int64_t nnz, int k, int p, int q, rqlp_precision prec) {
  if (check_common(m, n, k, p, q, prec) != RQLP_OK || nnz < 0 || nnz > INT32_MAX) return 0;
  if (prec == RQLP_BF16_REFINED || k + p > kDMaxCsr) return 0;
  return prec == RQLP_FP64 ? layout<double>(m, n, k + p, true, nnz).total
                           : layout<float>(m, n, k + p, true, nnz).total;
}

rqlp_status rqlp_decompose(rqlp_ctx* c, const void* A, int64_t m, int64_t n, int64_t lda, int k, int p, int q,
                           rqlp_precision prec, uint64_t seed, void* Q, void* L, void* V, void* ws,
                           size_t ws_bytes, void* stream) {
  if (!c || !A || !Q || !L || !V) return RQLP_ERR_INVALID_ARG;
  rqlp_status st = check_common(m, n, k, p, q, prec);
  if (st != RQLP_OK) return st;
  if (lda < n) return RQLP_ERR_INVALID_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return RQLP_ERR_HIP;
  hipStream_t s = (hipStream_t)stream;
  if (prec == RQLP_FP64)
    return decompose_dense<double>(c, (const double*)A, m, n, lda, k, p, q, seed, (double*)Q, (double*)L,
                                   (double*)V, ws, ws_bytes, s);
  if (prec == RQLP_BF16_REFINED)
    return decompose_dense_bf16(c, (const float*)A, m, n, lda, k, p, q, seed, (float*)Q, (float*)L, (float*)V, ws,
                                ws_bytes, s);
  return decompose_dense<float>(c, (const float*)A, m, n, lda, k, p, q, seed, (float*)Q, (float*)L, (float*)V,
                                ws, ws_bytes, s);
}

rqlp_status rqlp_decompose_noalloc(rqlp_ctx* c, const void* A, int64_t m, int64_t n, int64_t lda, int k, int p,
                                   int q, rqlp_precision prec, uint64_t seed, void* Q, void* L, void* V,
                                   void* stream) {
  if (!c || !A || !Q || !L || !V) return RQLP_ERR_INVALID_ARG;
  rqlp_status st = check_common(m, n, k, p, q, prec);
  if (st != RQLP_OK) return st;
  if (lda < n) return RQLP_ERR_INVALID_ARG;
  const size_t need = prec == RQLP_FP64 ? layout<double>(m, n, k + p, false, 0).total
                                        : layout<float>(m, n, k + p, false, 0, prec == RQLP_BF16_REFINED).total;
  if (need > RQLP_NOALLOC_SCRATCH_BYTES) return RQLP_ERR_OUT_OF_MEMORY;
  if (hipSetDevice(c->device) != hipSuccess) return RQLP_ERR_HIP;
  void* ws = scratch_ptr(c->device);
  if (!ws) return RQLP_ERR_HIP;
  // the same launch sequence as rqlp_decompose on the scratch array; event
  // timing (which may create events) is off for the call
  const uint32_t timing = c->timing;
  c->timing = 0;
  hipStream_t s = (hipStream_t)stream;
  if (prec == RQLP_FP64)
    st = decompose_dense<double>(c, (const double*)A, m, n, lda, k, p, q, seed, (double*)Q, (double*)L, (double*)V,
                                 ws, RQLP_NOALLOC_SCRATCH_BYTES, s);
  else if (prec == RQLP_BF16_REFINED)
    st = decompose_dense_bf16(c, (const float*)A, m, n, lda, k, p, q, seed, (float*)Q, (float*)L, (float*)V, ws,
                              RQLP_NOALLOC_SCRATCH_BYTES, s);
  else
    st = decompose_dense<float>(c, (const float*)A, m, n, lda, k, p, q, seed, (float*)Q, (float*)L, (float*)V, ws,
                                RQLP_NOALLOC_SCRATCH_BYTES, s);
  c->timing = timing;
  return st;
}

size_t rqlp_workspace_size_batched(int count, const rqlp_problem* probs, rqlp_precision prec) {
  if (count < 1 || !probs || !valid_prec(prec)) return 0;
  size_t total = 0;
  for (int i = 0; i < count; ++i) {
    if (check_problem(probs[i], prec) != RQLP_OK) return 0;
    total += problem_ws_bytes(probs[i], prec);
  }
  return total + 256;
}

rqlp_status rqlp_decompose_batched(rqlp_ctx* c, int count, const rqlp_problem* probs, rqlp_precision prec,
                                   void* ws, size_t ws_bytes, void* stream) {
  if (!c || count < 1 || !probs || !valid_prec(prec)) return RQLP_ERR_INVALID_ARG;
  size_t need = 0;
  for (int i = 0; i < count; ++i) {
    rqlp_status st = check_problem(probs[i], prec);
    if (st != RQLP_OK) return st;
    need += problem_ws_bytes(probs[i], prec);
  }
  need += 256;
  if (hipSetDevice(c->device) != hipSuccess) return RQLP_ERR_HIP;
  rqlp_status st = make_lanes(c);
  if (st != RQLP_OK) return st;
  char* base = nullptr;
  if ((st = get_workspace(c, ws, ws_bytes, need, &base)) != RQLP_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  // the bfloat16 form's conversion and product kernels have no grouped form:
  // its batches run every problem's sequence on a lane stream
  if (!c->lockstep || prec == RQLP_BF16_REFINED) {
    if (!c->graphs) return run_batch_lanes(c, count, probs, prec, base, s);
  }
  std::vector<uint8_t> key = batch_key(count, probs, prec, base, need);
  if (c->graphs) {
    for (auto& e : c->graph_cache)
      if (e.key == key) {
        HIP_TRY(hipGraphLaunch(e.exec, s));
        return RQLP_OK;
      }
  }
  // Graph capture takes the ungrouped form: a grouped batch has not been run
  // under stream capture in this build (an earlier grouped design ended the
  // host process under capture, with no cause found), so it runs eagerly.
  const bool grouped = c->lockstep && prec != RQLP_BF16_REFINED && !c->graphs;
  rqlp_ctx::GroupedPlan* plan = nullptr;
  if (grouped) {
    for (auto& p : c->plans)
      if (p.key == key) plan = &p;
    if (!plan) {
      rqlp_ctx::GroupedPlan np;
      np.key = key;
      st = build_plan(c, count, probs, prec, base, s, &np);
      if (st != RQLP_OK) {
        free_plan(np);
        return st;
      }
      if (c->plans.size() >= 8) {  // the oldest plan may still be read by queued work
        HIP_TRY(hipDeviceSynchronize());
        free_plan(c->plans.front());
        c->plans.erase(c->plans.begin());
      }
      c->plans.push_back(std::move(np));
      plan = &c->plans.back();
    }
  }
  // graphs: a batch seen for the second time in a row (same problems,
  // buffers and workspace) is captured once and replayed from then on
  if (!c->graphs || key != c->last_key) {
    c->last_key = key;
    return grouped ? launch_plan(c, *plan, s) : run_batch_lanes(c, count, probs, prec, base, s);
  }
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  st = grouped ? launch_plan(c, *plan, c->cap) : run_batch_lanes(c, count, probs, prec, base, c->cap);
  const hipError_t e_end = hipStreamEndCapture(c->cap, &g);
  if (st != RQLP_OK) {
    if (g) hipGraphDestroy(g);
    return st;
  }
  if (e_end != hipSuccess || !g) return RQLP_ERR_HIP;
  hipGraphExec_t exec = nullptr;
  const hipError_t e_inst = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e_inst != hipSuccess) return RQLP_ERR_HIP;
  if (c->graph_cache.size() >= 8) {
    hipGraphExecDestroy(c->graph_cache.front().exec);
    c->graph_cache.erase(c->graph_cache.begin());
  }
  c->graph_cache.push_back({key, exec});
  HIP_TRY(hipGraphLaunch(exec, s));
  return RQLP_OK;
}

rqlp_status rqlp_set_graphs(rqlp_ctx* c, int enabled) {
  if (!c) return RQLP_ERR_INVALID_ARG;
  c->graphs = enabled != 0;
  c->last_key.clear();
  return RQLP_OK;
}

rqlp_status rqlp_set_batch_grouping(rqlp_ctx* c, int enabled) {
  if (!c) return RQLP_ERR_INVALID_ARG;
  c->lockstep = enabled != 0;
  c->last_key.clear();
  return RQLP_OK;
}

rqlp_status rqlp_autotune(rqlp_ctx* c, const void* A, int64_t m, int64_t n, int64_t lda, int d,
                          rqlp_precision prec, void* stream, int* nsplit_nn, int* nsplit_tn) {
  if (!c || !A || m < 1 || n < 1 || d < 1 || lda < n || (prec != RQLP_FP64 && prec != RQLP_FP32))
    return RQLP_ERR_INVALID_ARG;
  if (d > kDMax || d > std::min(m, n)) return d > kDMax ? RQLP_ERR_UNSUPPORTED : RQLP_ERR_INVALID_ARG;
  if (m > INT32_MAX || n > INT32_MAX) return RQLP_ERR_UNSUPPORTED;
  if (hipSetDevice(c->device) != hipSuccess) return RQLP_ERR_HIP;
  hipStream_t s = (hipStream_t)stream;
  if (prec == RQLP_FP64)
    return autotune_dense<double>(c, (const double*)A, m, n, lda, d, s, nsplit_nn, nsplit_tn);
  return autotune_dense<float>(c, (const float*)A, m, n, lda, d, s, nsplit_nn, nsplit_tn);
}

rqlp_status rqlp_autotune_clear(rqlp_ctx* c) {
  if (!c) return RQLP_ERR_INVALID_ARG;
  c->plan.clear();
  return RQLP_OK;
}

rqlp_status rqlp_autotune_save(rqlp_ctx* c, const char* path) {
  if (!c || !path) return RQLP_ERR_INVALID_ARG;
  std::ofstream f(path);
  if (!f) return RQLP_ERR_INVALID_ARG;
  f << "rqlp-plans 2\n";
  for (const auto& e : c->plan) {
    const auto& k = e.first;
    f << "gemm " << std::get<0>(k) << ' ' << std::get<1>(k) << ' ' << std::get<2>(k) << ' ' << std::get<3>(k) << ' '
      << std::get<4>(k) << ' ' << e.second.first << ' ' << e.second.second << "\n";
  }
  return f.good() ? RQLP_OK : RQLP_ERR_INVALID_ARG;
}

rqlp_status rqlp_autotune_load(rqlp_ctx* c, const char* path) {
  if (!c || !path) return RQLP_ERR_INVALID_ARG;
  std::ifstream f(path);
  if (!f) return RQLP_ERR_INVALID_ARG;
  std::string tag;
  int version = 0;
  if (!(f >> tag >> version) || tag != "rqlp-plans" || (version != 1 && version != 2)) return RQLP_ERR_INVALID_ARG;
  std::map<std::tuple<int, int, int, int, int>, std::pair<int, int>> plan;
  std::string kind;
  while (f >> kind) {
    int es, trans, M, N, K, ns, mb = 2;  // version 1 files hold no row tile (128 rows)
    if (kind != "gemm" || !(f >> es >> trans >> M >> N >> K >> ns) || (version == 2 && !(f >> mb)) ||
        (es != 4 && es != 8) || (trans != 0 && trans != 1) || M < 1 || N < 1 || K < 1 || ns < 1 ||
        (mb != 2 && mb != 4) || (mb == 4 && es != 4))
      return RQLP_ERR_INVALID_ARG;
    plan[std::make_tuple(es, trans, M, N, K)] = {ns, mb};
  }
  for (const auto& e : plan) c->plan[e.first] = e.second;
  return RQLP_OK;
}

rqlp_status rqlp_autotune_count(rqlp_ctx* c, int* count) {
  if (!c || !count) return RQLP_ERR_INVALID_ARG;
  *count = (int)c->plan.size();
  return RQLP_OK;
}

size_t rqlp_svd_workspace_size(int d) {
  if (d < 1 || d > kDMax) return 0;
  return svd_ws_bytes(d) + 256;
}

rqlp_status rqlp_svd_small(rqlp_ctx* c, const void* M, int d, int64_t ldm, void* U, int64_t ldu, void* S, void* V,
                           int64_t ldv, rqlp_precision prec, void* ws, size_t ws_bytes, void* stream) {
  if (!c || !M || !U || !S || !V || d < 1 || ldm < d || ldu < d || ldv < d ||
      (prec != RQLP_FP64 && prec != RQLP_FP32))
    return RQLP_ERR_INVALID_ARG;
  if (d > kDMax) return RQLP_ERR_UNSUPPORTED;
  if (hipSetDevice(c->device) != hipSuccess) return RQLP_ERR_HIP;
  char* base = nullptr;
  rqlp_status st = get_workspace(c, ws, ws_bytes, svd_ws_bytes(d) + 256, &base);
  if (st != RQLP_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_info_reset(c->info, s));
  if (prec == RQLP_FP64)
    HIP_TRY(launch_svd_small<double>((const double*)M, ldm, d, (double*)U, ldu, (double*)S, (double*)V, ldv, base,
                                     c->info, s));
  else
    HIP_TRY(launch_svd_small<float>((const float*)M, ldm, d, (float*)U, ldu, (float*)S, (float*)V, ldv, base, c->info,
                                    s));
  return RQLP_OK;
}

size_t rqlp_workspace_size_svd(int64_t m, int64_t n, int k, int p, int q, rqlp_precision prec) {
  const size_t dec = rqlp_workspace_size(m, n, k, p, q, prec);
  if (!dec) return 0;
  return align256(dec) + svd_layout(m, n, k + p, prec).total + 256;
}

rqlp_status rqlp_decompose_svd(rqlp_ctx* c, const void* A, int64_t m, int64_t n, int64_t lda, int k, int p, int q,
                               rqlp_precision prec, uint64_t seed, void* U, void* S, void* W, void* ws,
                               size_t ws_bytes, void* stream) {
  if (!c || !A || !U || !S || !W) return RQLP_ERR_INVALID_ARG;
  rqlp_status st = check_common(m, n, k, p, q, prec);
  if (st != RQLP_OK) return st;
  if (lda < n) return RQLP_ERR_INVALID_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return RQLP_ERR_HIP;
  const int d = k + p;
  const size_t dec = align256(rqlp_workspace_size(m, n, k, p, q, prec));
  const SvdLayout Ly = svd_layout(m, n, d, prec);
  char* base = nullptr;
  if ((st = get_workspace(c, ws, ws_bytes, dec + Ly.total + 256, &base)) != RQLP_OK) return st;
  char* sb = base + dec;
  hipStream_t s = (hipStream_t)stream;
  if (prec == RQLP_FP64) {
    if ((st = decompose_dense<double>(c, (const double*)A, m, n, lda, k, p, q, seed, (double*)(sb + Ly.q),
                                      (double*)(sb + Ly.l), (double*)(sb + Ly.v), base, dec, s)) != RQLP_OK)
      return st;
    return svd_like<double>(c, Ly, sb, m, n, d, (double*)U, (double*)S, (double*)W, s);
  }
  if (prec == RQLP_BF16_REFINED)
    st = decompose_dense_bf16(c, (const float*)A, m, n, lda, k, p, q, seed, (float*)(sb + Ly.q), (float*)(sb + Ly.l),
                              (float*)(sb + Ly.v), base, dec, s);
  else
    st = decompose_dense<float>(c, (const float*)A, m, n, lda, k, p, q, seed, (float*)(sb + Ly.q),
                                (float*)(sb + Ly.l), (float*)(sb + Ly.v), base, dec, s);
  if (st != RQLP_OK) return st;
  return svd_like<float>(c, Ly, sb, m, n, d, (float*)U, (float*)S, (float*)W, s);
}

size_t rqlp_workspace_size_paper(int64_t m, int64_t n, int k, int p, int q, rqlp_precision prec) {
  if (check_common(m, n, k, p, q, prec) != RQLP_OK || prec == RQLP_BF16_REFINED) return 0;
  return prec == RQLP_FP64 ? layout<double>(n, m, k + p, false, 0).total : layout<float>(n, m, k + p, false, 0).total;
}

rqlp_status rqlp_decompose_paper(rqlp_ctx* c, const void* A, int64_t m, int64_t n, int64_t lda, int k, int p, int q,
                                 rqlp_precision prec, uint64_t seed, void* Q, void* L, void* P, void* ws,
                                 size_t ws_bytes, void* stream) {
  if (!c || !A || !Q || !L || !P) return RQLP_ERR_INVALID_ARG;
  rqlp_status st = check_common(m, n, k, p, q, prec);
  if (st != RQLP_OK) return st;
  if (lda < n) return RQLP_ERR_INVALID_ARG;
  if (prec == RQLP_BF16_REFINED) return RQLP_ERR_UNSUPPORTED;
  if (hipSetDevice(c->device) != hipSuccess) return RQLP_ERR_HIP;
  hipStream_t s = (hipStream_t)stream;
  if (prec == RQLP_FP64)
    return decompose_paper<double>(c, (const double*)A, m, n, lda, k, p, q, seed, (double*)Q, (double*)L, (double*)P,
                                   ws, ws_bytes, s);
  return decompose_paper<float>(c, (const float*)A, m, n, lda, k, p, q, seed, (float*)Q, (float*)L, (float*)P, ws,
                                ws_bytes, s);
}

rqlp_status rqlp_decompose_csr(rqlp_ctx* c, const int32_t* rowptr, const int32_t* colidx, const void* vals,
                               int64_t m, int64_t n, int64_t nnz, int k, int p, int q, rqlp_precision prec,
                               uint64_t seed, void* Q, void* L, void* V, void* ws, size_t ws_bytes,
                               void* stream) {
  if (!c || !rowptr || !Q || !L || !V) return RQLP_ERR_INVALID_ARG;
  if (nnz < 0 || nnz > INT32_MAX) return RQLP_ERR_INVALID_ARG;
  if (nnz > 0 && (!colidx || !vals)) return RQLP_ERR_INVALID_ARG;
  rqlp_status st = check_common(m, n, k, p, q, prec);
  if (st != RQLP_OK) return st;
  if (prec == RQLP_BF16_REFINED || k + p > kDMaxCsr) return RQLP_ERR_UNSUPPORTED;
  if (hipSetDevice(c->device) != hipSuccess) return RQLP_ERR_HIP;
  hipStream_t s = (hipStream_t)stream;
  if (prec == RQLP_FP64)
    return decompose_csr<double>(c, rowptr, colidx, (const double*)vals, m, n, nnz, k, p, q, seed, (double*)Q,
                                 (double*)L, (double*)V, ws, ws_bytes, s);
  return decompose_csr<float>(c, rowptr, colidx, (const float*)vals, m, n, nnz, k, p, q, seed, (float*)Q,
                              (float*)L, (float*)V, ws, ws_bytes, s);
}

rqlp_status rqlp_get_info(rqlp_ctx* c, rqlp_info* out) {
  if (!c || !out) return RQLP_ERR_INVALID_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return RQLP_ERR_HIP;
  DevInfo h;
  if (hipMemcpy(&h, c->info, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return RQLP_ERR_HIP;
  out->completed_cols = h.completed_cols;
  out->breakdown_pass = h.breakdown_pass;
  out->nonfinite = h.nonfinite;
  out->status = h.nonfinite ? RQLP_ERR_NUMERICAL : RQLP_OK;
  return RQLP_OK;
}

const char* rqlp_status_string(rqlp_status s) {
  switch (s) {
    case RQLP_OK: return "success";
    case RQLP_ERR_INVALID_ARG: return "invalid argument";
    case RQLP_ERR_UNSUPPORTED: return "unsupported by this build";
    case RQLP_ERR_OUT_OF_MEMORY: return "workspace too small or allocation failed";
    case RQLP_ERR_HIP: return "HIP runtime error";
    case RQLP_ERR_NUMERICAL: return "non-finite values encountered";
  }
  return "unknown status";
}

// ---- step entry points ----------------------------------------------------

rqlp_status rqlp_gaussian(rqlp_ctx* c, uint64_t seed, uint32_t stream_id, int64_t rows, int64_t cols,
                          rqlp_precision prec, void* out, int64_t ldo, void* stream) {
  if (!c || !out || rows < 0 || cols < 0 || ldo < cols || !valid_prec(prec)) return RQLP_ERR_INVALID_ARG;
  if (prec == RQLP_BF16_REFINED) return RQLP_ERR_UNSUPPORTED;
  if (hipSetDevice(c->device) != hipSuccess) return RQLP_ERR_HIP;
  hipStream_t s = (hipStream_t)stream;
  const uint64_t key1 = kSketchKey1 + stream_id;
  if (prec == RQLP_FP64) HIP_TRY(launch_gaussian<double>(seed, key1, rows, cols, (double*)out, ldo, s));
  else HIP_TRY(launch_gaussian<float>(seed, key1, rows, cols, (float*)out, ldo, s));
  return RQLP_OK;
}

size_t rqlp_gemm_workspace_size(int trans, int64_t m, int64_t n, int d, rqlp_precision prec) {
  if (m < 1 || n < 1 || d < 1 || d > kDMax || m > INT32_MAX || n > INT32_MAX || !valid_prec(prec)) return 0;
  const int dp = padded_d(d);
  const int M = (int)(trans ? n : m), K = (int)(trans ? m : n);
  if (prec == RQLP_BF16_REFINED) {
    // bf16 copy of op(A) (M x K, k-contiguous), of X^T (d x K), partial slabs
    const int64_t kp = bf16_ld(K);
    return align256((size_t)M * kp * 2) + align256((size_t)d * kp * 2) +
           align256(gemm_bf16_partial_elems(M, (int)kp, d) * 4) + 512;
  }
  const size_t e = prec == RQLP_FP64 ? gemm_partial_elems<double>(M, K, dp) * 8 : gemm_partial_elems<float>(M, K, dp) * 4;
  return e + 512;
}

rqlp_status rqlp_gemm(rqlp_ctx* c, int trans, const void* A, int64_t m, int64_t n, int64_t lda, const void* X,
                      int64_t ldx, int d, void* Y, int64_t ldy, rqlp_precision prec, void* ws, size_t ws_bytes,
                      void* stream) {
  if (!c || !A || !X || !Y || m < 1 || n < 1 || d < 1 || lda < n || ldx < d || ldy < d || !valid_prec(prec) ||
      (trans != 0 && trans != 1))
    return RQLP_ERR_INVALID_ARG;
  if (d > kDMax || m > INT32_MAX || n > INT32_MAX) return RQLP_ERR_UNSUPPORTED;
  if (hipSetDevice(c->device) != hipSuccess) return RQLP_ERR_HIP;
  const size_t need = rqlp_gemm_workspace_size(trans, m, n, d, prec);
  char* base = nullptr;
  rqlp_status st = get_workspace(c, ws, ws_bytes, need, &base);
  if (st != RQLP_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (prec == RQLP_BF16_REFINED) {
    const int M = (int)(trans ? n : m), K = (int)(trans ? m : n);
    const int64_t kp = bf16_ld(K);
    uint16_t* ab = (uint16_t*)base;
    uint16_t* xt = (uint16_t*)(base + align256((size_t)M * kp * 2));
    float* part = (float*)((char*)xt + align256((size_t)d * kp * 2));
    if (trans) HIP_TRY(launch_cvt_bf16((const float*)A, lda, m, n, ab, 0, ab, kp, s));  // A^T only
    else HIP_TRY(launch_cvt_bf16((const float*)A, lda, m, n, ab, kp, nullptr, 0, s));
    HIP_TRY(launch_cvt_bf16_t((const float*)X, ldx, K, d, xt, kp, s));
    EvPair t = timer(c, trans ? RQLP_KT_GEMM_TN : RQLP_KT_GEMM_NN);
    HIP_TRY(launch_gemm_bf16(ab, kp, xt, kp, M, d, (int)kp, (float*)Y, ldy, d, part, s, t.a, t.b));
    return RQLP_OK;
  }
  // the partial buffer is laid out with row length d here (nst = d)
  if (prec == RQLP_FP64)
    return gemm<double>(c, trans, (const double*)A, lda, m, n, (const double*)X, ldx, d, (double*)Y, ldy, d,
                        (double*)base, s, false);
  return gemm<float>(c, trans, (const float*)A, lda, m, n, (const float*)X, ldx, d, (float*)Y, ldy, d,
                     (float*)base, s, false);
}

size_t rqlp_orth_workspace_size(int64_t rows, int d, rqlp_precision prec) {
  if (rows < 1 || d < 1 || d > rows || d > kDMax || !valid_prec(prec)) return 0;
  return orth_ws_bytes(rows, d, prec);
}

rqlp_status rqlp_orth(rqlp_ctx* c, const void* Y, int64_t rows, int d, int64_t ldy, void* Q, int64_t ldq,
                      void* R, rqlp_precision prec, uint64_t seed, void* ws, size_t ws_bytes, void* stream) {
  if (!c || !Y || !Q || rows < 1 || d < 1 || d > rows || ldy < d || ldq < d || !valid_prec(prec))
    return RQLP_ERR_INVALID_ARG;
  if (d > kDMax || prec == RQLP_BF16_REFINED) return RQLP_ERR_UNSUPPORTED;
  if (hipSetDevice(c->device) != hipSuccess) return RQLP_ERR_HIP;
  const size_t need = orth_ws_bytes(rows, d, prec);
  char* base = nullptr;
  rqlp_status st = get_workspace(c, ws, ws_bytes, need, &base);
  if (st != RQLP_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const int dp = padded_d(d);
  size_t off = 0;
  auto take = [&](size_t bytes) { char* p = base + off; off += align256(bytes); return p; };
  Bufs b;
  b.q1 = (double*)take((size_t)rows * dp * sizeof(double));
  b.gp = (double*)take((size_t)gram_chunks(rows, dp) * dp * dp * sizeof(double));
  char* gr = take((size_t)dp * dp * sizeof(double) * 3);
  b.g = (double*)gr;
  b.r1 = b.g + (size_t)dp * dp;
  b.r2 = b.r1 + (size_t)dp * dp;
  b.rinv = (double*)take((size_t)dp * kTile * sizeof(double));
  b.flags = (int32_t*)take((size_t)(2 * dp + 2) * sizeof(int32_t));
  b.xf = (double*)take((size_t)dp * dp * sizeof(double));
  b.esq = (double*)take((size_t)(gram_reduce_blocks(dp) + dp) * sizeof(double));
  HIP_TRY(launch_info_reset(c->info, s));
  if (prec == RQLP_FP64) {
    st = cholqr2<double>(c, (const double*)Y, ldy, rows, d, b, (double*)Q, ldq, d, nullptr, 0, 0, seed, 1, s);
    if (st == RQLP_OK && R) HIP_TRY(launch_form_r<double>(b.r2, b.r1, b.flags, d, dp, (double*)R, d, s));
  } else {
    st = cholqr2<float>(c, (const float*)Y, ldy, rows, d, b, (float*)Q, ldq, d, nullptr, 0, 0, seed, 1, s);
    if (st == RQLP_OK && R) HIP_TRY(launch_form_r<float>(b.r2, b.r1, b.flags, d, dp, (float*)R, d, s));
  }
  return st;
}

rqlp_status rqlp_spmm(rqlp_ctx* c, const int32_t* rowptr, const int32_t* colidx, const void* vals, int64_t rows,
                      int64_t cols, int64_t nnz, const void* X, int64_t ldx, int d, void* Y, int64_t ldy,
                      rqlp_precision prec, void* stream) {
  if (!c || !rowptr || !X || !Y || rows < 0 || cols < 1 || nnz < 0 || d < 1 || ldx < d || ldy < d ||
      !valid_prec(prec) || (nnz > 0 && (!colidx || !vals)))
    return RQLP_ERR_INVALID_ARG;
  if (d > kDMaxCsr || prec == RQLP_BF16_REFINED || nnz > INT32_MAX) return RQLP_ERR_UNSUPPORTED;
  if (hipSetDevice(c->device) != hipSuccess) return RQLP_ERR_HIP;
  hipStream_t s = (hipStream_t)stream;
  EvPair t = timer(c, RQLP_KT_SPMM);
  if (prec == RQLP_FP64)
    HIP_TRY(launch_spmm<double>(rowptr, colidx, (const double*)vals, rows, (const double*)X, ldx, d, (double*)Y,
                                ldy, d, s, t.a, t.b));
  else
    HIP_TRY(launch_spmm<float>(rowptr, colidx, (const float*)vals, rows, (const float*)X, ldx, d, (float*)Y, ldy,
                               d, s, t.a, t.b));
  return RQLP_OK;
}

size_t rqlp_csr_transpose_workspace_size(int64_t m, int64_t n, int64_t nnz) {
  if (m < 0 || n < 1 || nnz < 0) return 0;
  return csr_transpose_scratch_bytes(m, n, nnz) + 256;
}

rqlp_status rqlp_csr_transpose(rqlp_ctx* c, const int32_t* rowptr, const int32_t* colidx, const void* vals,
                               int64_t m, int64_t n, int64_t nnz, rqlp_precision prec, int32_t* rowptr_t,
                               int32_t* colidx_t, void* vals_t, void* ws, size_t ws_bytes, void* stream) {
  if (!c || !rowptr || !rowptr_t || m < 0 || n < 1 || nnz < 0 || !valid_prec(prec) ||
      (nnz > 0 && (!colidx || !vals || !colidx_t || !vals_t)))
    return RQLP_ERR_INVALID_ARG;
  if (prec == RQLP_BF16_REFINED || nnz > INT32_MAX || m > INT32_MAX || n > INT32_MAX) return RQLP_ERR_UNSUPPORTED;
  if (hipSetDevice(c->device) != hipSuccess) return RQLP_ERR_HIP;
  char* base = nullptr;
  rqlp_status st = get_workspace(c, ws, ws_bytes, rqlp_csr_transpose_workspace_size(m, n, nnz), &base);
  if (st != RQLP_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (prec == RQLP_FP64)
    HIP_TRY(launch_csr_transpose<double>(rowptr, colidx, (const double*)vals, m, n, nnz, rowptr_t, colidx_t,
                                         (double*)vals_t, base, s));
  else
    HIP_TRY(launch_csr_transpose<float>(rowptr, colidx, (const float*)vals, m, n, nnz, rowptr_t, colidx_t,
                                        (float*)vals_t, base, s));
  return RQLP_OK;
}

rqlp_status rqlp_set_timing_mask(rqlp_ctx* c, uint32_t mask) {
  if (!c) return RQLP_ERR_INVALID_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return RQLP_ERR_HIP;
  resolve_timing(c);
  for (int k = 0; k < RQLP_KT_COUNT; ++k) {
    c->total_ms[k] = 0;
    c->launches[k] = 0;
  }
  c->timing = mask & ((1u << RQLP_KT_COUNT) - 1);
  return RQLP_OK;
}

rqlp_status rqlp_set_timing(rqlp_ctx* c, int enabled) {
  return rqlp_set_timing_mask(c, enabled ? (1u << RQLP_KT_COUNT) - 1 : 0u);
}

rqlp_status rqlp_get_timing(rqlp_ctx* c, rqlp_kernel_class cls, double* total_ms, int64_t* launches) {
  if (!c || !total_ms || !launches || (int)cls < 0 || (int)cls >= RQLP_KT_COUNT) return RQLP_ERR_INVALID_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return RQLP_ERR_HIP;
  resolve_timing(c);
  *total_ms = c->total_ms[cls];
  *launches = c->launches[cls];
  return RQLP_OK;
}

}  // extern "C"

// ---- serving -----------------------------------------------------------------
// Continuous batching at request granularity: a request is admitted as soon
// as a slot (a stream of its own) is free and its workspace fits into the
// free part of the HBM budget; admitted requests run concurrently on their
// slots' streams, so requests arriving while others are on the GPU overlap
// with them.  Completion is observed with events by rqlp_server_poll.

struct rqlp_server {
  rqlp_ctx* ctx = nullptr;
  rqlp_precision prec = RQLP_FP32;
  char* pool = nullptr;
  size_t budget = 0;
  // A tick: the requests admitted together, launched as one grouped batch on
  // the tick's stream and completed together.
  struct Slot {
    hipStream_t s = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<int64_t> tickets;
    std::vector<std::pair<size_t, size_t>> ranges;  // workspace (offset, bytes) per request
    void* table_dev = nullptr;                      // grouped argument tables of the tick
    size_t table_bytes = 0;
    std::vector<uint8_t> table_host;                // kept until the tick completes
    rqlp_ctx::GroupedPlan plan;
  };
  // A queued request and the event recorded on the submitter's stream at
  // submit: the tick stream waits on it, so work the caller enqueued before
  // submitting (writing A, say) is complete before the request reads it.
  struct Queued {
    int64_t ticket;
    rqlp_problem prob;
    hipEvent_t ready;
  };
  int max_tick = 64;  // requests per tick
  std::vector<Slot> slots;
  std::deque<Queued> queue;
  std::vector<hipEvent_t> event_pool;
  std::deque<std::pair<int64_t, rqlp_status>> failed;  // launches that failed, reported by poll
  std::map<size_t, size_t> free_ranges;  // offset -> bytes, coalesced
  int64_t next_ticket = 0;
};

namespace {

bool pool_alloc(rqlp_server* sv, size_t bytes, size_t* off) {
  for (auto it = sv->free_ranges.begin(); it != sv->free_ranges.end(); ++it) {
    if (it->second >= bytes) {  // first fit
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t roff = it->first + bytes;
      sv->free_ranges.erase(it);
      if (rest) sv->free_ranges[roff] = rest;
      return true;
    }
  }
  return false;
}

void pool_free(rqlp_server* sv, size_t off, size_t bytes) {
  auto it = sv->free_ranges.emplace(off, bytes).first;
  auto nx = std::next(it);
  if (nx != sv->free_ranges.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    sv->free_ranges.erase(nx);
  }
  if (it != sv->free_ranges.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      sv->free_ranges.erase(it);
    }
  }
}

// Launch the requests `rq` (workspace offsets in the pool already taken) as
// one tick on slot `sl`: the grouped batch executor's launches (every result
// the bits of the request's solo run), or, for the bfloat16 form, every
// request's own sequence, all on the tick stream.
// A tick of one request runs the request's own sequence (no tables to build).
rqlp_status launch_tick(rqlp_server* sv, rqlp_server::Slot& sl, const std::vector<rqlp_server::Queued>& rq) {
  rqlp_ctx* c = sv->ctx;
  for (const auto& q : rq) HIP_TRY(hipStreamWaitEvent(sl.s, q.ready, 0));
  std::vector<rqlp_problem> probs;
  std::vector<size_t> offs;
  for (size_t i = 0; i < rq.size(); ++i) {
    probs.push_back(rq[i].prob);
    offs.push_back(sl.ranges[i].first);
  }
  const uint32_t timing = c->timing;
  rqlp_status st = RQLP_OK;
  if (sv->prec != RQLP_BF16_REFINED && probs.size() > 1) {
    st = layout_plan(c, (int)probs.size(), probs.data(), offs.data(), sv->prec, sv->pool, sl.s, &sl.plan,
                     sl.table_host);
    if (st != RQLP_OK) return st;
    if (sl.table_bytes < sl.table_host.size()) {
      if (sl.table_dev) hipFree(sl.table_dev);
      sl.table_dev = nullptr;
      sl.table_bytes = 0;
      if (hipMalloc(&sl.table_dev, sl.table_host.size()) != hipSuccess) return RQLP_ERR_OUT_OF_MEMORY;
      sl.table_bytes = sl.table_host.size();
    }
    HIP_TRY(hipMemcpyAsync(sl.table_dev, sl.table_host.data(), sl.table_host.size(), hipMemcpyHostToDevice, sl.s));
    sl.plan.dev = sl.table_dev;
    c->timing = 0;
    const char* dev = (const char*)sl.table_dev;
    for (const auto& L : sl.plan.launches)
      L.fn(dev + L.args_off, (const int*)(dev + L.start_off), L.count, L.blocks, sl.s);
    sl.plan.dev = nullptr;  // owned by the slot
    c->timing = timing;
    HIP_TRY(hipGetLastError());
  } else {
    c->timing = 0;
    c->reset_info = false;
    for (size_t i = 0; i < probs.size() && st == RQLP_OK; ++i)
      st = run_problem(c, probs[i], sv->prec, sv->pool + offs[i], sl.ranges[i].second, sl.s);
    c->reset_info = true;
    c->timing = timing;
    if (st != RQLP_OK) return st;
  }
  HIP_TRY(hipEventRecord(sl.done, sl.s));
  return RQLP_OK;
}

hipEvent_t take_server_event(rqlp_server* sv) {
  if (!sv->event_pool.empty()) {
    hipEvent_t e = sv->event_pool.back();
    sv->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

extern "C" {

rqlp_status rqlp_server_create(rqlp_server** out, rqlp_ctx* c, size_t hbm_budget, int slots,
                               rqlp_precision prec) {
  if (!out || !c || hbm_budget < 4096 || slots < 1 || slots > 64 || !valid_prec(prec)) return RQLP_ERR_INVALID_ARG;
  *out = nullptr;
  if (hipSetDevice(c->device) != hipSuccess) return RQLP_ERR_HIP;
  rqlp_server* sv = new (std::nothrow) rqlp_server();
  if (!sv) return RQLP_ERR_OUT_OF_MEMORY;
  sv->ctx = c;
  sv->prec = prec;
  sv->budget = hbm_budget & ~(size_t)255;
  if (hipMalloc(&sv->pool, sv->budget) != hipSuccess) {
    delete sv;
    return RQLP_ERR_OUT_OF_MEMORY;
  }
  sv->free_ranges[0] = sv->budget;
  sv->slots.resize(slots);
  for (auto& sl : sv->slots) {
    if (hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
      rqlp_server_destroy(sv);
      return RQLP_ERR_HIP;
    }
  }
  // one reset of the shared info record for everything the server runs
  if (launch_info_reset(c->info, sv->slots[0].s) != hipSuccess ||
      hipStreamSynchronize(sv->slots[0].s) != hipSuccess) {
    rqlp_server_destroy(sv);
    return RQLP_ERR_HIP;
  }
  *out = sv;
  return RQLP_OK;
}

rqlp_status rqlp_server_destroy(rqlp_server* sv) {
  if (!sv) return RQLP_OK;
  hipSetDevice(sv->ctx->device);
  for (auto& sl : sv->slots) {
    if (sl.s) hipStreamSynchronize(sl.s);
    if (sl.done) hipEventDestroy(sl.done);
    if (sl.s) hipStreamDestroy(sl.s);
    if (sl.table_dev) hipFree(sl.table_dev);
  }
  for (auto& rq : sv->queue) hipEventDestroy(rq.ready);
  for (hipEvent_t e : sv->event_pool) hipEventDestroy(e);
  if (sv->pool) hipFree(sv->pool);
  delete sv;
  return RQLP_OK;
}

rqlp_status rqlp_server_set_tick(rqlp_server* sv, int max_requests) {
  if (!sv || max_requests < 1 || max_requests > 1024) return RQLP_ERR_INVALID_ARG;
  sv->max_tick = max_requests;
  return RQLP_OK;
}

size_t rqlp_server_request_bytes(const rqlp_problem* req, rqlp_precision prec) {
  if (!req || !valid_prec(prec) || check_problem(*req, prec) != RQLP_OK) return 0;
  return problem_ws_bytes(*req, prec);
}

rqlp_status rqlp_server_submit(rqlp_server* sv, const rqlp_problem* req, void* stream, int64_t* ticket) {
  if (!sv || !req || !ticket) return RQLP_ERR_INVALID_ARG;
  rqlp_status st = check_problem(*req, sv->prec);
  if (st != RQLP_OK) return st;
  if (problem_ws_bytes(*req, sv->prec) > sv->budget) return RQLP_ERR_OUT_OF_MEMORY;
  if (hipSetDevice(sv->ctx->device) != hipSuccess) return RQLP_ERR_HIP;
  hipEvent_t ready = take_server_event(sv);
  if (!ready) return RQLP_ERR_HIP;
  if (hipEventRecord(ready, (hipStream_t)stream) != hipSuccess) {
    sv->event_pool.push_back(ready);
    return RQLP_ERR_HIP;
  }
  *ticket = sv->next_ticket++;
  sv->queue.push_back({*ticket, *req, ready});
  return RQLP_OK;
}

rqlp_status rqlp_server_poll(rqlp_server* sv, int64_t* done, int32_t* status, int max_done, int* ndone,
                             int* inflight, int* queued) {
  if (!sv || !ndone || (max_done > 0 && !done)) return RQLP_ERR_INVALID_ARG;
  if (hipSetDevice(sv->ctx->device) != hipSuccess) return RQLP_ERR_HIP;
  *ndone = 0;
  // requests whose launch failed earlier, then completions (up to max_done
  // per call; the rest on later calls)
  while (!sv->failed.empty() && *ndone < max_done) {
    if (status) status[*ndone] = (int32_t)sv->failed.front().second;
    done[(*ndone)++] = sv->failed.front().first;
    sv->failed.pop_front();
  }
  for (auto& sl : sv->slots) {
    if (!sl.busy || *ndone + (int)sl.tickets.size() > max_done) continue;
    const hipError_t q = hipEventQuery(sl.done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return RQLP_ERR_HIP;
    sl.busy = false;
    for (const auto& r : sl.ranges) pool_free(sv, r.first, r.second);
    for (const int64_t t : sl.tickets) {
      if (status) status[*ndone] = RQLP_OK;
      done[(*ndone)++] = t;
    }
    sl.tickets.clear();
    sl.ranges.clear();
  }
  // admissions, in arrival order (the head waits until its workspace fits),
  // one tick per free slot: the queue is shared out over the free slots, so
  // that requests run alone while the queue is short and are grouped (at most
  // max_tick per tick) only when a backlog builds up
  int free_slots = 0;
  for (auto& sl : sv->slots) free_slots += sl.busy ? 0 : 1;
  for (auto& sl : sv->slots) {
    if (sl.busy) continue;
    if (sv->queue.empty()) break;
    const int share = (int)std::min<int64_t>(sv->max_tick, ceil_div((int64_t)sv->queue.size(), std::max(free_slots, 1)));
    --free_slots;
    std::vector<rqlp_server::Queued> tick;
    while (!sv->queue.empty() && (int)tick.size() < share) {
      const rqlp_server::Queued& rq = sv->queue.front();
      const size_t need = problem_ws_bytes(rq.prob, sv->prec);
      size_t off = 0;
      if (!pool_alloc(sv, need, &off)) break;
      sl.ranges.emplace_back(off, need);
      sl.tickets.push_back(rq.ticket);
      tick.push_back(rq);
      sv->queue.pop_front();
    }
    if (tick.empty()) break;
    const rqlp_status st = launch_tick(sv, sl, tick);
    for (const auto& q : tick) sv->event_pool.push_back(q.ready);  // the tick's waits are enqueued
    if (st != RQLP_OK) {
      // part of the tick may already be on its stream: let it drain before
      // the workspace goes back to the pool, and report the tickets as failed
      if (hipStreamSynchronize(sl.s) != hipSuccess) return RQLP_ERR_HIP;
      for (const auto& r : sl.ranges) pool_free(sv, r.first, r.second);
      for (const int64_t t : sl.tickets) sv->failed.emplace_back(t, st);
      sl.tickets.clear();
      sl.ranges.clear();
      continue;
    }
    sl.busy = true;
  }
  int nb = 0;
  for (auto& sl : sv->slots) nb += sl.busy ? (int)sl.tickets.size() : 0;
  if (inflight) *inflight = nb;
  if (queued) *queued = (int)sv->queue.size();
  return RQLP_OK;
}

}  // extern "C"

namespace rqlp {
// The launch recorder of the calling thread (see grouped.h).
LaunchRecorder*& launch_recorder() { return recorder_slot(); }
}  // namespace rqlp
