// Cholesky factor of the float64 Gram matrix, G = R^T R (R upper): the
// middle step of each CholeskyQR pass (orth() and qr() of the paper,
// computed as an unpivoted QR with a positive diagonal in R).
//
// For d <= 256, one workgroup of 8 waves, right-looking over 16-column blocks k.  The
// lower triangle of G is cut into 16 x 16 tiles held in registers (MFMA
// 16x16x4 accumulator layout: lane l holds rows l/16 + 4 s, column l % 16),
// dealt round-robin to the waves.  Per block column k:
//   A. the owner of tile (k,k) factors it in four steps of 4 pivots: a
//      4 x 4 factorization on wave-uniform scalars, then MFMAs for the
//      panel, the rank-4 trailing update and the running inverse of the
//      16 x 16 factor;
//   B. owners of tiles (i,k), i > k, form L_ik = G_ik L_kk^-T (4 MFMAs) and
//      publish them in an LDS panel;
//   C. owners of tiles (i,j), k < j <= i, update G_ij -= L_ik L_jk^T (MFMA).
// Columns whose pivot is <= tol * (their original squared norm) are marked
// dependent: their L column is zero, their R diagonal is 1 (so R stays
// invertible for the solve) and the caller replaces the matching columns of
// Q with random directions.
//
// Fast path for the second CholeskyQR pass: G = I + E with E small.  The
// upper-triangular F with F + F^T = E (F = triu(E, 1) + diag(E) / 2) gives
// R = I + F with R^T R = G + F^T F, so Q = Q1 R^-1 is orthonormal up to
// ~||F||_2^2 <= ||E||_F^2 / 4.  The host passes the largest ||E||_F that keeps
// this below the output precision; then R = I + F, R^-1 = I - F (to the same
// order) is written explicitly and the solve becomes a plain product.
#include "common.h"
#include "grouped.h"
#include "kernels.h"

#include <algorithm>

namespace rqlp {

__device__ inline double bcast(double x, int lane) {
  // value of x in lane `lane` (wave-uniform index), as a scalar broadcast
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

__device__ inline void tile_of(int t, int& i, int& j) {
  // t = i (i + 1) / 2 + j, 0 <= j <= i
  int ii = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
  while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
  while (ii * (ii + 1) / 2 > t) --ii;
  i = ii;
  j = t - ii * (ii + 1) / 2;
}

// 1/sqrt(x) to float64 accuracy: the hardware estimate (relative error
// about 2^-24) and one third-order correction, y (1 + e/2 + 3 e^2/8) with
// e = 1 - x y^2, which leaves a truncation error near 5 e^3 / 16 and is as
// accurate as two Newton steps (about an ulp) with four dependent
// operations instead of six on the pivot chain.
__device__ inline double rsqrt_f64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(0.375, e, 0.5), y);
}

// One 4-pivot step of the 16 x 16 diagonal-tile factorization S = L L^T,
// pivots j0..j0+3 (j0 = 4 B), with the tile in the MFMA accumulator layout
// (lane (g, c) = (l / 16, l % 16) holds rows g + 4 r of column c, so
// register B of lane (g, c) is S[j0 + g][c]) and X = L^-1 carried along in
// the same layout:
//   1. the 4 x 4 block D = S[j0.., j0..] is read as wave-uniform scalars and
//      factored, D = L_D L_D^T, with M = L_D^-1 (dependent pivots get a unit
//      column in L_D); the pivots' Schur updates use the L_D entries, so the
//      chain from one pivot to the next is one 1/sqrt and one FMA;
//   2. C = M S[j0..j0+3, :] (one MFMA; the B operand is register B as it
//      stands) holds L^T's rows j0..j0+3: the panel L_P^T right of the block
//      and, by symmetry, L_D^T inside it;
//   3. S -= L_P L_P^T on the trailing block and X[j0.., :] = M X[j0.., :],
//      X[below, :] -= L_P X[j0.., :] (three MFMAs; A and B of the rank-4
//      update are the same register, zero outside the trailing part).
// R = L^T's rows j0..j0+3 of the tile are written to Rt (row stride dp).
template <int B>
__device__ inline void diag_step4(doublex4& a, doublex4& x, int lane, int lr, int lc, double gdl, double tol,
                                  int& depmask, double* __restrict__ Rt, int dp) {
  constexpr int j0 = 4 * B;
  double W[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) W[i][j] = bcast(a[B], 16 * i + j0 + j);  // S[j0 + i][j0 + j]
  double Ld[4][4], inv[4];
  int dm = 0;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const double piv = W[p][p];
    const bool dep = !(piv > tol * bcast(gdl, j0 + p));
    inv[p] = dep ? 1.0 : rsqrt_f64(piv);
    Ld[p][p] = dep ? 1.0 : piv * inv[p];
#pragma unroll
    for (int i = p + 1; i < 4; ++i) Ld[i][p] = dep ? 0.0 : W[i][p] * inv[p];
#pragma unroll
    for (int i = p + 1; i < 4; ++i)
#pragma unroll
      for (int j = p + 1; j <= i; ++j) W[i][j] = fma(-Ld[i][p], Ld[j][p], W[i][j]);
    dm |= dep ? (1 << p) : 0;
  }
  // M = L_D^-1 (lower), M[i][i] = 1 / L_D[i][i]
  double M[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    M[i][i] = inv[i];
#pragma unroll
    for (int j = 0; j < i; ++j) {
      double t = 0.0;
#pragma unroll
      for (int q = j; q < i; ++q) t = fma(Ld[i][q], M[q][j], t);
      M[i][j] = -t * inv[i];
    }
  }
  // A operand: lane (k, m) supplies M[m][k] (rows m >= 4 are zero); every
  // lane holds the uniform M, so each picks its entry by selects
  double am = 0.0;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int k = 0; k <= m; ++k) am = (lc == m && lr == k) ? M[m][k] : am;
  const doublex4 z = Mfma<double>::zero();
  const doublex4 c = Mfma<double>::mma(am, a[B], z);   // c[0] = (M S[j0.., :])[lr][lc]
  const doublex4 xn = Mfma<double>::mma(am, x[B], z);  // xn[0] = new X[j0 + lr][lc]
  const bool depg = (dm >> lr) & 1;
  // L_P^T[lr][lc] = L[lc][j0 + lr] right of the block (zero for a dependent pivot)
  const double lp = (lc > j0 + 3 && !depg) ? c[0] : 0.0;
  double rv = lp;  // R[j0 + lr][lc]
  if (lc < j0 + lr) rv = 0.0;
  else if (lc <= j0 + 3) rv = depg ? (lc == j0 + lr ? 1.0 : 0.0) : c[0];
  Rt[(int64_t)(j0 + lr) * dp + lc] = rv;
  x[B] = xn[0];
  a = Mfma<double>::mma(-lp, lp, a);     // S[m][n] -= sum_k L_P[m][k] L_P[n][k]
  x = Mfma<double>::mma(-lp, x[B], x);   // X[m][:] -= sum_k L_P[m][k] X[j0 + k][:]
  depmask |= dm << j0;
}

// Fast path of the second CholeskyQR pass: when ||G - I||_F < fast_tol
// (from the nesq partial sums the Gram reduction wrote; every workgroup adds
// them in the same fixed order), all workgroups write their share of
// R = I + F and R^-1 = I - F, and the call returns true.
__device__ inline bool chol_fast_path(const double* __restrict__ G, int d, int dp, double* __restrict__ R,
                                      double* __restrict__ Rinv16, int32_t* __restrict__ flags, double fast_tol,
                                      const double* __restrict__ esq, int nesq, int32_t* __restrict__ mode,
                                      double* __restrict__ Xfull, double* red, int nw, int bid, int nblk) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  double ss = 0.0;
  for (int e = tid; e < nesq; e += blockDim.x) ss += esq[e];
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
  if (lane == 0) red[wave] = ss;
  __syncthreads();
  double tot = 0.0;
  for (int w = 0; w < nw; ++w) tot += red[w];
  if (tot < fast_tol * fast_tol) {  // false for NaN
    for (int e = bid * blockDim.x + tid; e < dp * dp; e += nblk * blockDim.x) {
      const int i = e / dp, j = e - (e / dp) * dp;
      double f = 0.0;  // F[i][j]
      if (i < d && j < d && i <= j) {
        const double g = G[(int64_t)i * dp + j];
        f = (i < j) ? g : 0.5 * (g - 1.0);
      }
      const double id = (i == j) ? 1.0 : 0.0;
      R[(int64_t)i * dp + j] = id + f;
      Xfull[(int64_t)i * dp + j] = id - f;
      if ((i >> 4) == (j >> 4))
        Rinv16[(int64_t)(i >> 4) * kTile * kTile + (i & 15) * kTile + (j & 15)] = id - f;
    }
    for (int i = bid * blockDim.x + tid; i < dp; i += nblk * blockDim.x) flags[i] = 0;
    if (bid == 0 && tid == 0) *mode = 2;  // explicit inverse already written
    return true;
  }
  __syncthreads();
  return false;
}

// G (dp x dp block, row stride ld; R the same) is factored in registers.
// Standalone (block = 0): the whole matrix, with the fast path, and *mode
// set to 1 or 0.  As a diagonal block of a larger factorization (block =
// 1): nothing is done when *mode == 2, the dependence test takes the
// original diagonal from gdiag0, and *mode is only lowered to 0.
// The body is shared by the one-matrix kernel and the grouped kernel that
// factors many matrices in one launch (bid, nblk: this workgroup's index
// and the workgroup count of its matrix).
template <int NW, int SLOTS>
__device__ __attribute__((always_inline)) inline void chol_body(const double* __restrict__ G, int ld, int d, int dp,
                                                    double* __restrict__ R,
                                                    double* __restrict__ Rinv16,
                                                    int32_t* __restrict__ flags, DevInfo* info,
                                                    int pass_id, double tol, double fast_tol,
                                                    const double* __restrict__ esq, int nesq,
                                                    int32_t* __restrict__ mode,
                                                    double* __restrict__ Xfull,
                                                    const double* __restrict__ gdiag0, int block, int bid, int nblk) {
  __shared__ double Pn[kCholRegMax / kTile][kTile][kTile + 1];  // panel tiles L_ik of column k
  __shared__ double Di[kTile][kTile + 1];                        // inverse of the diagonal factor
  __shared__ double Gdiag[kCholRegMax];
  __shared__ int defl[kCholRegMax];
  __shared__ double red[NW];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int T = dp / kTile;
  const int lr = lane >> 4, lc = lane & 15;  // MFMA accumulator layout: row lr + 4 r, col lc

  if (block) {
    if (*mode == 2) return;
  } else if (fast_tol > 0.0 &&
             chol_fast_path(G, d, dp, R, Rinv16, flags, fast_tol, esq, nesq, mode, Xfull, red, NW, bid, nblk)) {
    return;
  }
  if (bid != 0) return;  // the factorization runs in one workgroup

  // ---------------- full factorization ----------------
  for (int i = tid; i < dp; i += blockDim.x) {
    Gdiag[i] = (i < d) ? (gdiag0 ? gdiag0[i] : G[(int64_t)i * ld + i]) : 1.0;
    defl[i] = 0;
  }
  const int ntiles = T * (T + 1) / 2;
  // slot sl of this wave holds tile t = wave + NW sl of the lower triangle,
  // (i, j) packed as i + 256 (j + 1) (a free slot has j = -1)
  doublex4 tile[SLOTS];
  int tij[SLOTS];
#pragma unroll
  for (int sl = 0; sl < SLOTS; ++sl) {
    const int t = wave + NW * sl;
    int i0 = 0, j0 = -1;
    if (t < ntiles) tile_of(t, i0, j0);
    tij[sl] = __builtin_amdgcn_readfirstlane(i0 + 256 * (j0 + 1));
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = 0.0;
      if (t < ntiles) {
        const int row = i0 * kTile + lr + 4 * r, col = j0 * kTile + lc;
        v = (row < d && col < d) ? G[(int64_t)row * ld + col] : (row == col ? 1.0 : 0.0);
      }
      tile[sl][r] = v;
    }
  }
  int ndep_total = 0;
  __syncthreads();

  // A: the owner of tile (k,k) factors it in four 4-pivot steps and
  // publishes Di = L_kk^-1, the R block L_kk^T, its inverse and the
  // dependent-column flags.
  auto factor_diag = [&](int k, int sk) {
    doublex4 t = Mfma<double>::zero();
#pragma unroll
    for (int sl = 0; sl < SLOTS; ++sl)
      if (sl == sk) t = tile[sl];
    doublex4 x;
#pragma unroll
    for (int r = 0; r < 4; ++r) x[r] = (lr + 4 * r == lc) ? 1.0 : 0.0;
    const double gdl = Gdiag[k * kTile + lc];
    int depmask = 0;
    double* Rt = R + (int64_t)k * kTile * ld + k * kTile;
    // the diagonal factorization is the latency chain of the whole
    // factorization: its wave takes issue priority over the co-resident
    // waves' trailing updates while it runs
    __builtin_amdgcn_s_setprio(3);
    diag_step4<0>(t, x, lane, lr, lc, gdl, tol, depmask, Rt, ld);
    diag_step4<1>(t, x, lane, lr, lc, gdl, tol, depmask, Rt, ld);
    diag_step4<2>(t, x, lane, lr, lc, gdl, tol, depmask, Rt, ld);
    diag_step4<3>(t, x, lane, lr, lc, gdl, tol, depmask, Rt, ld);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = lr + 4 * r;
      Di[row][lc] = x[r];                                              // X[row][c]
      Rinv16[(int64_t)k * kTile * kTile + lc * kTile + row] = x[r];    // (L^-1)^T
    }
    __builtin_amdgcn_s_setprio(0);
    if (lane < kTile) {
      const int dep_c = (depmask >> lane) & 1;
      defl[k * kTile + lane] = dep_c;
      flags[k * kTile + lane] = dep_c;
    }
    ndep_total += __popc(depmask);
  };

  // G_ij -= L_ik L_jk^T for a tile of the trailing matrix (k < j <= i)
  auto update_g = [&](doublex4& t, int i, int j) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kk = ks * 4 + lr;
      t = Mfma<double>::mma(-Pn[i][lc][kk], Pn[j][lc][kk], t);  // B[kk][n] = L_jk[n][kk]
    }
  };

  {  // A for k = 0
    const int t0 = 0;
    if (wave == t0 % NW) factor_diag(0, t0 / NW);
  }
  for (int k = 0; k < T; ++k) {
    // Opaque to the optimizer: otherwise the LDS addresses of every slot are
    // hoisted out of this loop and held in vector registers the tiles need.
#pragma unroll
    for (int sl = 0; sl < SLOTS; ++sl) asm volatile("" : "+s"(tij[sl]));
    __syncthreads();
    // ---------------- B: panel L_ik = G_ik L_kk^-T ----------------
#pragma unroll
    for (int sl = 0; sl < SLOTS; ++sl) {
      const int i = tij[sl] & 255, j = (tij[sl] >> 8) - 1;
      if (j == k && i > k) {
#pragma unroll
        for (int r = 0; r < 4; ++r) Pn[i][lr + 4 * r][lc] = tile[sl][r];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        doublex4 acc = Mfma<double>::zero();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int kk = ks * 4 + lr;
          acc = Mfma<double>::mma(Pn[i][lc][kk], Di[lc][kk], acc);  // B[kk][n] = X[n][kk]
        }
        const bool zc = defl[k * kTile + lc] != 0;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int r = 0; r < 4; ++r) Pn[i][lr + 4 * r][lc] = zc ? 0.0 : acc[r];
      }
    }
    __syncthreads();
    // ---------------- C: trailing update, with the next A looked ahead ----------------
    // The owner of tile (k+1, k+1) updates it first and factors it at once;
    // the other waves publish the panel (R = L^T above the diagonal block
    // row k, zero below) and go on with their updates meanwhile.
    const int kn = k + 1;
    const int tn = kn * (kn + 1) / 2 + kn;
    const int own = tn % NW;
    const bool ahead = kn < T && wave == own;
    const int sn = tn / NW;
    if (ahead) {
      __builtin_amdgcn_s_setprio(3);  // the update of tile (k+1, k+1) is on the chain too
#pragma unroll
      for (int sl = 0; sl < SLOTS; ++sl)
        if (sl == sn) update_g(tile[sl], kn, kn);
      factor_diag(kn, sn);
    } else {
      const int nt = (kn < T) ? NW - 1 : NW;                 // publishing waves
      const int pw = (kn < T && wave > own) ? wave - 1 : wave;  // rank among them
      for (int e = pw * kWave + lane; e < (T - 1 - k) * kTile * kTile; e += nt * kWave) {
        const int i = k + 1 + e / (kTile * kTile), row = (e / kTile) % kTile, col = e % kTile;
        R[(int64_t)(k * kTile + col) * ld + i * kTile + row] = Pn[i][row][col];
        R[(int64_t)(i * kTile + row) * ld + k * kTile + col] = 0.0;
      }
    }
#pragma unroll
    for (int sl = 0; sl < SLOTS; ++sl) {
      if (ahead && sl == sn) continue;
      const int i = tij[sl] & 255, j = (tij[sl] >> 8) - 1;
      if (j > k) update_g(tile[sl], i, j);
    }
  }
  // the explicit R^-1 (formed next by the inverse kernel) serves the solve
  // unless a column was dependent
  int anydep = 0;
  for (int i = tid; i < dp; i += blockDim.x) anydep |= defl[i];
  anydep = __syncthreads_or(anydep);
  if (tid == 0) {
    if (!block) *mode = anydep ? 0 : 1;
    else if (anydep) *mode = 0;
  }
  if (lane == 0 && ndep_total > 0) {
    atomicAdd(&info->completed_cols, ndep_total);
    atomicCAS(&info->breakdown_pass, 0, pass_id);
  }
}

template <int NW, int SLOTS>
__global__ __launch_bounds__(NW * 64) void chol_kernel(const double* __restrict__ G, int ld, int d, int dp,
                                                    double* __restrict__ R, double* __restrict__ Rinv16,
                                                    int32_t* __restrict__ flags, DevInfo* info, int pass_id,
                                                    double tol, double fast_tol, const double* __restrict__ esq,
                                                    int nesq, int32_t* __restrict__ mode,
                                                    double* __restrict__ Xfull, const double* __restrict__ gdiag0,
                                                    int block) {
  chol_body<NW, SLOTS>(G, ld, d, dp, R, Rinv16, flags, info, pass_id, tol, fast_tol, esq, nesq, mode, Xfull, gdiag0,
                       block, blockIdx.x, gridDim.x);
}

// Many independent matrices in one launch (argument table in device
// memory): workgroups start[p] .. start[p + 1] - 1 belong to matrix p.
struct CholRecArgs {
  const double* G;
  double* R;
  double* Rinv16;
  int32_t* flags;
  DevInfo* info;
  const double* esq;
  int32_t* mode;
  double* Xfull;
  const double* gdiag0;
  double tol, fast_tol;
  int ld, d, dp, pass_id, nesq, block;
};

template <int NW, int SLOTS>
__global__ __launch_bounds__(NW * 64) void chol_grouped(const CholRecArgs* __restrict__ a,
                                                        const int* __restrict__ start, int count) {
  const int p = group_find(start, count, blockIdx.x);
  const CholRecArgs g = a[p];
  chol_body<NW, SLOTS>(g.G, g.ld, g.d, g.dp, g.R, g.Rinv16, g.flags, g.info, g.pass_id, g.tol, g.fast_tol, g.esq,
                       g.nesq, g.mode, g.Xfull, g.gdiag0, g.block, (int)blockIdx.x - start[p], start[p + 1] - start[p]);
}

template <int NW, int SLOTS>
void chol_grouped_launch(const void* args, const int* start, int count, unsigned blocks, hipStream_t s) {
  hipLaunchKernelGGL((chol_grouped<NW, SLOTS>), dim3(blocks), dim3(NW * kWave), 0, s, (const CholRecArgs*)args,
                     start, count);
}

// ---------------- d > 256: blocked over register-sized diagonal blocks ----------------
// The matrix is cut into nb diagonal blocks of at most 256 columns.  For
// each block b in turn: R_bb = chol(G_bb) (chol_kernel in block mode), then,
// unless b is the last block, X_bb = R_bb^-1 (inverse kernel),
// R_b,r = X_bb^T G_b,r for the columns r after the block (rows of dependent
// columns zero), and the trailing update G_r,r -= R_b,r^T R_b,r (both
// triangles, in place).  The panel and update spread over many workgroups;
// only the diagonal blocks run in one.

// Fast path of the second pass (all workgroups), else the original diagonal
// into gd0 (for the dependence test of later blocks) and *mode = 1.
__device__ __attribute__((always_inline)) inline void chol_prep_body(const double* __restrict__ G, int d, int dp,
                                                                     double* __restrict__ R,
                                                                     double* __restrict__ Rinv16,
                                                                     int32_t* __restrict__ flags, double fast_tol,
                                                                     const double* __restrict__ esq, int nesq,
                                                                     int32_t* __restrict__ mode,
                                                                     double* __restrict__ Xfull,
                                                                     double* __restrict__ gd0, int bid, int nblk) {
  __shared__ double red[16];
  if (fast_tol > 0.0 && chol_fast_path(G, d, dp, R, Rinv16, flags, fast_tol, esq, nesq, mode, Xfull, red, 16, bid, nblk))
    return;
  if (bid != 0) return;
  for (int i = threadIdx.x; i < dp; i += blockDim.x) gd0[i] = (i < d) ? G[(int64_t)i * dp + i] : 1.0;
  if (threadIdx.x == 0) *mode = 1;
}

__global__ __launch_bounds__(1024) void chol_prep_kernel(const double* __restrict__ G, int d, int dp,
                                                      double* __restrict__ R, double* __restrict__ Rinv16,
                                                      int32_t* __restrict__ flags, double fast_tol,
                                                      const double* __restrict__ esq, int nesq,
                                                      int32_t* __restrict__ mode, double* __restrict__ Xfull,
                                                      double* __restrict__ gd0) {
  chol_prep_body(G, d, dp, R, Rinv16, flags, fast_tol, esq, nesq, mode, Xfull, gd0, blockIdx.x, gridDim.x);
}

struct CholPrepArgs {
  const double* G;
  double* R;
  double* Rinv16;
  int32_t* flags;
  const double* esq;
  int32_t* mode;
  double* Xfull;
  double* gd0;
  double fast_tol;
  int d, dp, nesq;
};

__global__ __launch_bounds__(1024) void chol_prep_grouped(const CholPrepArgs* __restrict__ a,
                                                       const int* __restrict__ start, int count) {
  const int p = group_find(start, count, blockIdx.x);
  const CholPrepArgs g = a[p];
  chol_prep_body(g.G, g.d, g.dp, g.R, g.Rinv16, g.flags, g.fast_tol, g.esq, g.nesq, g.mode, g.Xfull, g.gd0,
                 (int)blockIdx.x - start[p], start[p + 1] - start[p]);
}

void chol_prep_grouped_launch(const void* args, const int* start, int count, unsigned blocks, hipStream_t s) {
  hipLaunchKernelGGL(chol_prep_grouped, dim3(blocks), dim3(1024), 0, s, (const CholPrepArgs*)args, start, count);
}

// R[b, r] = X_bb^T G[b, r] (one wave per 16 x 16 output tile, float64 MFMA)
// and R[r, b] = 0; X_bb is upper triangular, so tile row I needs only the
// first 16 (I + 1) rows of X_bb and G.
__device__ __attribute__((always_inline)) inline void chol_panel_body(const double* __restrict__ G, int ld, int off,
                                                                      int db, int rest, const double* __restrict__ X,
                                                                      double* __restrict__ R,
                                                                      const int32_t* __restrict__ flags,
                                                                      const int32_t* __restrict__ mode, int bid) {
  if (*mode == 2) return;
  const int nI = db / kTile;
  const int I = bid % nI, J = bid / nI;
  const int lane = threadIdx.x, lr = lane >> 4, lc = lane & 15;
  const double* Xb = X + (int64_t)off * ld + off;
  const double* Gb = G + (int64_t)off * ld + off + db;
  doublex4 acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = Mfma<double>::zero();
  const int kend = (I + 1) * kTile;
  for (int t0 = 0; t0 < kend; t0 += kTile) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {  // A[m][kk] = X_bb[t][I*16+m], B[kk][n] = G_b,r[t][J*16+n]
      const int t = t0 + 4 * u + lr;
      acc[u] = Mfma<double>::mma(Xb[(int64_t)t * ld + I * kTile + lc], Gb[(int64_t)t * ld + J * kTile + lc],
                                 acc[u]);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = I * kTile + lr + 4 * r, col = J * kTile + lc;
    const double v = ((acc[0][r] + acc[1][r]) + acc[2][r]) + acc[3][r];
    R[(int64_t)(off + row) * ld + off + db + col] = flags[off + row] ? 0.0 : v;
    R[(int64_t)(off + db + col) * ld + off + row] = 0.0;
  }
}

__global__ __launch_bounds__(64) void chol_panel_kernel(const double* __restrict__ G, int ld, int off, int db,
                                                     int rest, const double* __restrict__ X,
                                                     double* __restrict__ R, const int32_t* __restrict__ flags,
                                                     const int32_t* __restrict__ mode) {
  chol_panel_body(G, ld, off, db, rest, X, R, flags, mode, blockIdx.x);
}

struct CholPanelArgs {
  const double* G;
  const double* X;
  double* R;
  const int32_t* flags;
  const int32_t* mode;
  int ld, off, db, rest;
};

__global__ __launch_bounds__(64) void chol_panel_grouped(const CholPanelArgs* __restrict__ a,
                                                      const int* __restrict__ start, int count) {
  const int p = group_find(start, count, blockIdx.x);
  const CholPanelArgs g = a[p];
  chol_panel_body(g.G, g.ld, g.off, g.db, g.rest, g.X, g.R, g.flags, g.mode, (int)blockIdx.x - start[p]);
}

void chol_panel_grouped_launch(const void* args, const int* start, int count, unsigned blocks, hipStream_t s) {
  hipLaunchKernelGGL(chol_panel_grouped, dim3(blocks), dim3(64), 0, s, (const CholPanelArgs*)args, start, count);
}

// G[r, r] -= R[b, r]^T R[b, r] (one wave per 16 x 16 tile of the square
// trailing block, K = db)
__device__ __attribute__((always_inline)) inline void chol_syrk_body(double* __restrict__ G, int ld, int off, int db,
                                                                     int rest, const double* __restrict__ R,
                                                                     const int32_t* __restrict__ mode, int bid) {
  if (*mode == 2) return;
  const int nI = rest / kTile;
  const int I = bid % nI, J = bid / nI;
  const int lane = threadIdx.x, lr = lane >> 4, lc = lane & 15;
  const double* Rb = R + (int64_t)off * ld + off + db;
  doublex4 acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = Mfma<double>::zero();
  for (int t0 = 0; t0 < db; t0 += kTile) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = t0 + 4 * u + lr;
      acc[u] = Mfma<double>::mma(Rb[(int64_t)t * ld + I * kTile + lc], Rb[(int64_t)t * ld + J * kTile + lc],
                                 acc[u]);
    }
  }
  double* Gt = G + (int64_t)(off + db + I * kTile) * ld + off + db + J * kTile;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    Gt[(int64_t)(lr + 4 * r) * ld + lc] -= ((acc[0][r] + acc[1][r]) + acc[2][r]) + acc[3][r];
}

__global__ __launch_bounds__(64) void chol_syrk_kernel(double* __restrict__ G, int ld, int off, int db, int rest,
                                                    const double* __restrict__ R, const int32_t* __restrict__ mode) {
  chol_syrk_body(G, ld, off, db, rest, R, mode, blockIdx.x);
}

struct CholSyrkArgs {
  double* G;
  const double* R;
  const int32_t* mode;
  int ld, off, db, rest;
};

__global__ __launch_bounds__(64) void chol_syrk_grouped(const CholSyrkArgs* __restrict__ a,
                                                     const int* __restrict__ start, int count) {
  const int p = group_find(start, count, blockIdx.x);
  const CholSyrkArgs g = a[p];
  chol_syrk_body(g.G, g.ld, g.off, g.db, g.rest, g.R, g.mode, (int)blockIdx.x - start[p]);
}

void chol_syrk_grouped_launch(const void* args, const int* start, int count, unsigned blocks, hipStream_t s) {
  hipLaunchKernelGGL(chol_syrk_grouped, dim3(blocks), dim3(64), 0, s, (const CholSyrkArgs*)args, start, count);
}

// register slots per wave for the t (t + 1) / 2 lower tiles of a block of t
// tile columns (8 waves; slots chosen so that tiles and the diagonal-block
// code fit in registers)
static hipError_t launch_chol_reg(const double* G, int ld, int d, int db, double* R, double* Rinv16,
                                  int32_t* flags, void* info, int pass_id, double tol, double fast_tol,
                                  const double* esq, int nesq, int32_t* mode, double* Xfull, const double* gdiag0,
                                  int block, hipStream_t s) {
  const int T = db / kTile;
  const int tiles = T * (T + 1) / 2;
  const unsigned grid = (!block && fast_tol > 0.0) ? 16 : 1;  // extra workgroups only help the fast path
  const CholRecArgs a{G, R, Rinv16, flags, (DevInfo*)info, esq, mode, Xfull, gdiag0, tol, fast_tol, ld, d, db, pass_id,
                      nesq, block};
#define RQLP_CHOL_LAUNCH(S)                                                                                        \
  do {                                                                                                             \
    if (!record_launch(&chol_grouped_launch<8, S>, a, grid))                                                       \
      hipLaunchKernelGGL((chol_kernel<8, S>), dim3(grid), dim3(8 * kWave), 0, s, G, ld, d, db, R, Rinv16, flags,    \
                         (DevInfo*)info, pass_id, tol, fast_tol, esq, nesq, mode, Xfull, gdiag0, block);             \
  } while (0)
  if (tiles <= 8 * 7) RQLP_CHOL_LAUNCH(7);
  else if (tiles <= 8 * 14) RQLP_CHOL_LAUNCH(14);
  else RQLP_CHOL_LAUNCH(17);
#undef RQLP_CHOL_LAUNCH
  return hipGetLastError();
}

hipError_t launch_chol(double* G, int d, int dp, double* R, double* Rinv16, int32_t* flags,
                       void* info, int pass_id, double fast_tol, const double* esq, int nesq,
                       int32_t* mode, double* Xfull, double* gd0, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const double tol = 64.0 * (double)d * 2.220446049250313e-16;
  if (ev0) (void)hipEventRecord(ev0, s);
  hipError_t e = hipSuccess;
  if (dp <= kCholRegMax) {
    e = launch_chol_reg(G, dp, d, dp, R, Rinv16, flags, info, pass_id, tol, fast_tol, esq, nesq, mode, Xfull,
                        nullptr, 0, s);
  } else {
    const unsigned pg = fast_tol > 0.0 ? 16 : 1;
    if (!record_launch(&chol_prep_grouped_launch,
                       CholPrepArgs{G, R, Rinv16, flags, esq, mode, Xfull, gd0, fast_tol, d, dp, nesq}, pg))
      hipLaunchKernelGGL(chol_prep_kernel, dim3(pg), dim3(1024), 0, s, G, d, dp, R, Rinv16, flags, fast_tol, esq, nesq,
                         mode, Xfull, gd0);
    const int T = dp / kTile;
    const int nb = (int)ceil_div(T, kCholRegMax / kTile);
    int t0 = 0;
    for (int b = 0; b < nb && e == hipSuccess; ++b) {
      const int tb = (T - t0) / (nb - b);  // equal shares, the larger ones first
      const int tbs = tb + ((T - t0) % (nb - b) ? 1 : 0);
      const int off = t0 * kTile, db = tbs * kTile, rest = dp - off - db;
      const int dl = std::max(0, std::min(d - off, db));
      e = launch_chol_reg(G + (int64_t)off * dp + off, dp, dl, db, R + (int64_t)off * dp + off,
                          Rinv16 + (int64_t)t0 * kTile * kTile, flags + off, info, pass_id, tol, 0.0, esq, nesq,
                          mode, Xfull, gd0 + off, 1, s);
      if (e == hipSuccess && rest > 0) {
        e = launch_trinv_block(R + (int64_t)off * dp + off, Rinv16 + (int64_t)t0 * kTile * kTile, dp, tbs, mode,
                               Xfull + (int64_t)off * dp + off, s);
        if (e != hipSuccess) break;
        const unsigned npb = (unsigned)(tbs * (rest / kTile)), nsb = (unsigned)((rest / kTile) * (rest / kTile));
        if (!record_launch(&chol_panel_grouped_launch, CholPanelArgs{G, Xfull, R, flags, mode, dp, off, db, rest}, npb))
          hipLaunchKernelGGL(chol_panel_kernel, dim3(npb), dim3(kWave), 0, s, G, dp, off, db, rest, Xfull, R, flags,
                             mode);
        if (!record_launch(&chol_syrk_grouped_launch, CholSyrkArgs{G, R, mode, dp, off, db, rest}, nsb))
          hipLaunchKernelGGL(chol_syrk_kernel, dim3(nsb), dim3(kWave), 0, s, G, dp, off, db, rest, R, mode);
        e = hipGetLastError();
      }
      t0 += tbs;
    }
  }
  if (ev1) (void)hipEventRecord(ev1, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

int chol_slot_class(int dp) {
  const int T = dp / kTile;
  const int tiles = T * (T + 1) / 2;
  return tiles <= 8 * 7 ? 7 : (tiles <= 8 * 14 ? 14 : 17);
}

}  // namespace rqlp
