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
#include "kernels.h"

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

// 1/sqrt(x) to float64 accuracy: hardware estimate and two Newton steps.
__device__ inline double rsqrt_f64(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double r = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, r, y);
  }
  return y;
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
                                  int& depmask, double* __restrict__ Rt, int dp, double* Mb) {
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
  // A operand: lane (k, m) supplies M[m][k] (rows m >= 4 are zero), handed
  // out through LDS from lane 0's copy of the uniform values
  if (lane == 0) {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int k = 0; k < 4; ++k) Mb[4 * m + k] = (k <= m) ? M[m][k] : 0.0;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const double am = (lc < 4) ? Mb[4 * lc + lr] : 0.0;
  __builtin_amdgcn_wave_barrier();
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
                                      double* __restrict__ Xfull, double* red, int nw) {
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
    for (int e = blockIdx.x * blockDim.x + tid; e < dp * dp; e += gridDim.x * blockDim.x) {
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
    for (int i = blockIdx.x * blockDim.x + tid; i < dp; i += gridDim.x * blockDim.x) flags[i] = 0;
    if (blockIdx.x == 0 && tid == 0) *mode = 2;  // explicit inverse already written
    return true;
  }
  __syncthreads();
  return false;
}

template <int NW, int SLOTS>
__global__ __launch_bounds__(NW * 64) void chol_kernel(const double* __restrict__ G, int d, int dp,
                                                    double* __restrict__ R,
                                                    double* __restrict__ Rinv16,
                                                    int32_t* __restrict__ flags, DevInfo* info,
                                                    int pass_id, double tol, double fast_tol,
                                                    const double* __restrict__ esq, int nesq,
                                                    int32_t* __restrict__ mode,
                                                    double* __restrict__ Xfull) {
  __shared__ double Pn[kCholRegMax / kTile][kTile][kTile + 1];  // panel tiles L_ik of column k
  __shared__ double Di[kTile][kTile + 1];                        // inverse of the diagonal factor
  __shared__ double Gdiag[kCholRegMax];
  __shared__ int defl[kCholRegMax];
  __shared__ double red[NW];
  __shared__ double Mb[16];  // 4 x 4 inverse of the current diagonal block step

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int T = dp / kTile;
  const int lr = lane >> 4, lc = lane & 15;  // MFMA accumulator layout: row lr + 4 r, col lc

  if (fast_tol > 0.0 && chol_fast_path(G, d, dp, R, Rinv16, flags, fast_tol, esq, nesq, mode, Xfull, red, NW))
    return;
  if (blockIdx.x != 0) return;  // the factorization runs in one workgroup

  // ---------------- full factorization ----------------
  for (int i = tid; i < dp; i += blockDim.x) {
    Gdiag[i] = (i < d) ? G[(int64_t)i * dp + i] : 1.0;
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
        v = (row < d && col < d) ? G[(int64_t)row * dp + col] : (row == col ? 1.0 : 0.0);
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
    double* Rt = R + (int64_t)k * kTile * dp + k * kTile;
    diag_step4<0>(t, x, lane, lr, lc, gdl, tol, depmask, Rt, dp, Mb);
    diag_step4<1>(t, x, lane, lr, lc, gdl, tol, depmask, Rt, dp, Mb);
    diag_step4<2>(t, x, lane, lr, lc, gdl, tol, depmask, Rt, dp, Mb);
    diag_step4<3>(t, x, lane, lr, lc, gdl, tol, depmask, Rt, dp, Mb);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = lr + 4 * r;
      Di[row][lc] = x[r];                                              // X[row][c]
      Rinv16[(int64_t)k * kTile * kTile + lc * kTile + row] = x[r];    // (L^-1)^T
    }
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
#pragma unroll
      for (int sl = 0; sl < SLOTS; ++sl)
        if (sl == sn) update_g(tile[sl], kn, kn);
      factor_diag(kn, sn);
    } else {
      const int nt = (kn < T) ? NW - 1 : NW;                 // publishing waves
      const int pw = (kn < T && wave > own) ? wave - 1 : wave;  // rank among them
      for (int e = pw * kWave + lane; e < (T - 1 - k) * kTile * kTile; e += nt * kWave) {
        const int i = k + 1 + e / (kTile * kTile), row = (e / kTile) % kTile, col = e % kTile;
        R[(int64_t)(k * kTile + col) * dp + i * kTile + row] = Pn[i][row][col];
        R[(int64_t)(i * kTile + row) * dp + k * kTile + col] = 0.0;
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
  if (tid == 0) *mode = anydep ? 0 : 1;
  if (lane == 0 && ndep_total > 0) {
    atomicAdd(&info->completed_cols, ndep_total);
    atomicCAS(&info->breakdown_pass, 0, pass_id);
  }
}

// Cholesky for dp > kCholRegMax: the same right-looking algorithm, with the
// lower tiles of the trailing matrix kept in G itself (updated in place,
// 2.4 MB at d = 544, resident in L2) instead of registers, and 16 waves.
// A tile is only ever read and written by its owner wave (tile t =
// i (i + 1) / 2 + j belongs to wave t % NW), and by the same lane for the
// same element, so no synchronisation beyond the per-step barriers is
// needed.  Rows and columns in [d, dp) are read as the identity.
template <int NW>
__global__ __launch_bounds__(NW * 64) void chol_big_kernel(double* __restrict__ G, int d, int dp,
                                                        double* __restrict__ R, double* __restrict__ Rinv16,
                                                        int32_t* __restrict__ flags, DevInfo* info, int pass_id,
                                                        double tol, double fast_tol, const double* __restrict__ esq,
                                                        int nesq, int32_t* __restrict__ mode,
                                                        double* __restrict__ Xfull) {
  __shared__ double Pn[kDMax / kTile][kTile][kTile + 1];  // panel tiles L_ik of column k
  __shared__ double Di[kTile][kTile + 1];                  // inverse of the diagonal factor
  __shared__ double Gdiag[kDMax];
  __shared__ int defl[kDMax];
  __shared__ double red[NW];
  __shared__ double Mb[16];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int T = dp / kTile;
  const int lr = lane >> 4, lc = lane & 15;

  if (fast_tol > 0.0 && chol_fast_path(G, d, dp, R, Rinv16, flags, fast_tol, esq, nesq, mode, Xfull, red, NW))
    return;
  if (blockIdx.x != 0) return;

  for (int i = tid; i < dp; i += blockDim.x) {
    Gdiag[i] = (i < d) ? G[(int64_t)i * dp + i] : 1.0;
    defl[i] = 0;
  }
  int ndep_total = 0;
  __syncthreads();

  auto load_tile = [&](int i, int j) {
    doublex4 v;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = i * kTile + lr + 4 * r, col = j * kTile + lc;
      const double g = G[(int64_t)row * dp + col];
      v[r] = (row < d && col < d) ? g : (row == col ? 1.0 : 0.0);
    }
    return v;
  };
  auto store_tile = [&](int i, int j, const doublex4& v) {
#pragma unroll
    for (int r = 0; r < 4; ++r) G[(int64_t)(i * kTile + lr + 4 * r) * dp + j * kTile + lc] = v[r];
  };
  auto factor_diag = [&](int k, doublex4 t) {
    doublex4 x;
#pragma unroll
    for (int r = 0; r < 4; ++r) x[r] = (lr + 4 * r == lc) ? 1.0 : 0.0;
    const double gdl = Gdiag[k * kTile + lc];
    int depmask = 0;
    double* Rt = R + (int64_t)k * kTile * dp + k * kTile;
    diag_step4<0>(t, x, lane, lr, lc, gdl, tol, depmask, Rt, dp, Mb);
    diag_step4<1>(t, x, lane, lr, lc, gdl, tol, depmask, Rt, dp, Mb);
    diag_step4<2>(t, x, lane, lr, lc, gdl, tol, depmask, Rt, dp, Mb);
    diag_step4<3>(t, x, lane, lr, lc, gdl, tol, depmask, Rt, dp, Mb);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = lr + 4 * r;
      Di[row][lc] = x[r];
      Rinv16[(int64_t)k * kTile * kTile + lc * kTile + row] = x[r];
    }
    if (lane < kTile) {
      const int dep_c = (depmask >> lane) & 1;
      defl[k * kTile + lane] = dep_c;
      flags[k * kTile + lane] = dep_c;
    }
    ndep_total += __popc(depmask);
  };
  auto update_g = [&](doublex4& t, int i, int j) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kk = ks * 4 + lr;
      t = Mfma<double>::mma(-Pn[i][lc][kk], Pn[j][lc][kk], t);
    }
  };
  // first column j >= j0 of row i whose tile this wave owns
  auto first_owned = [&](int i, int j0) {
    const int base = i * (i + 1) / 2;
    return j0 + ((wave - (base + j0)) % NW + NW) % NW;
  };

  if (wave == 0) factor_diag(0, load_tile(0, 0));
  for (int k = 0; k < T; ++k) {
    __syncthreads();
    // ---------------- B: panel L_ik = G_ik L_kk^-T, two tiles at a time ----------------
    {
      int i = k + 1;
      while (i < T && (i * (i + 1) / 2 + k) % NW != wave) ++i;
      while (i < T) {
        int i2 = i + 1;
        while (i2 < T && (i2 * (i2 + 1) / 2 + k) % NW != wave) ++i2;
        const doublex4 t1 = load_tile(i, k);
        const doublex4 t2 = (i2 < T) ? load_tile(i2, k) : Mfma<double>::zero();
        const int ni = (i2 < T) ? 2 : 1;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          if (u >= ni) break;
          const int ii = u ? i2 : i;
          const doublex4& tt = u ? t2 : t1;
#pragma unroll
          for (int r = 0; r < 4; ++r) Pn[ii][lr + 4 * r][lc] = tt[r];
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          doublex4 acc = Mfma<double>::zero();
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) {
            const int kk = ks * 4 + lr;
            acc = Mfma<double>::mma(Pn[ii][lc][kk], Di[lc][kk], acc);
          }
          const bool zc = defl[k * kTile + lc] != 0;
          __builtin_amdgcn_wave_barrier();
#pragma unroll
          for (int r = 0; r < 4; ++r) Pn[ii][lr + 4 * r][lc] = zc ? 0.0 : acc[r];
        }
        i = i2 + 1;
        while (i < T && (i * (i + 1) / 2 + k) % NW != wave) ++i;
      }
    }
    __syncthreads();
    // ---------------- C: trailing update, with the next A looked ahead ----------------
    const int kn = k + 1;
    const int own = (kn * (kn + 1) / 2 + kn) % NW;
    const bool ahead = kn < T && wave == own;
    if (ahead) {
      doublex4 t = load_tile(kn, kn);
      update_g(t, kn, kn);
      factor_diag(kn, t);
    } else {
      const int nt = (kn < T) ? NW - 1 : NW;
      const int pw = (kn < T && wave > own) ? wave - 1 : wave;
      for (int e = pw * kWave + lane; e < (T - 1 - k) * kTile * kTile; e += nt * kWave) {
        const int i = k + 1 + e / (kTile * kTile), row = (e / kTile) % kTile, col = e % kTile;
        R[(int64_t)(k * kTile + col) * dp + i * kTile + row] = Pn[i][row][col];
        R[(int64_t)(i * kTile + row) * dp + k * kTile + col] = 0.0;
      }
    }
    // owned tiles (i, j), kn <= j <= i, row by row, four loads in flight
    int ci = kn, cj = (kn < T) ? first_owned(kn, kn) : 0;
    auto advance = [&]() {
      cj += NW;
      while (ci < T && cj > ci) {
        ++ci;
        if (ci < T) cj = first_owned(ci, kn);
      }
    };
    while (ci < T && cj > ci) {  // the first row may hold no owned tile
      ++ci;
      if (ci < T) cj = first_owned(ci, kn);
    }
    while (ci < T) {
      int bi[4], bj[4], nb = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        bi[u] = ci;
        bj[u] = cj;
        if (ci < T) {
          ++nb;
          advance();
        }
      }
      doublex4 tb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) tb[u] = (u < nb) ? load_tile(bi[u], bj[u]) : Mfma<double>::zero();
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (u < nb && !(ahead && bi[u] == kn && bj[u] == kn)) {
          update_g(tb[u], bi[u], bj[u]);
          store_tile(bi[u], bj[u], tb[u]);
        }
      }
    }
  }
  int anydep = 0;
  for (int i = tid; i < dp; i += blockDim.x) anydep |= defl[i];
  anydep = __syncthreads_or(anydep);
  if (tid == 0) *mode = anydep ? 0 : 1;
  if (lane == 0 && ndep_total > 0) {
    atomicAdd(&info->completed_cols, ndep_total);
    atomicCAS(&info->breakdown_pass, 0, pass_id);
  }
}

hipError_t launch_chol(double* G, int d, int dp, double* R, double* Rinv16, int32_t* flags,
                       void* info, int pass_id, double fast_tol, const double* esq, int nesq,
                       int32_t* mode, double* Xfull, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const double tol = 64.0 * (double)d * 2.220446049250313e-16;
  if (ev0) (void)hipEventRecord(ev0, s);
  const int T = dp / kTile;
  // register slots per wave for the T (T + 1) / 2 lower tiles (waves x
  // slots chosen so that tiles and the diagonal-block code fit in registers)
  const int tiles = T * (T + 1) / 2;
  const unsigned grid = fast_tol > 0.0 ? 16 : 1;  // extra workgroups only help the fast path
  if (dp > kCholRegMax)
    hipLaunchKernelGGL((chol_big_kernel<16>), dim3(grid), dim3(16 * kWave), 0, s, G, d, dp, R, Rinv16, flags,
                       (DevInfo*)info, pass_id, tol, fast_tol, esq, nesq, mode, Xfull);
  else if (tiles <= 8 * 7)
    hipLaunchKernelGGL((chol_kernel<8, 7>), dim3(grid), dim3(8 * kWave), 0, s, G, d, dp, R, Rinv16, flags,
                       (DevInfo*)info, pass_id, tol, fast_tol, esq, nesq, mode, Xfull);
  else if (tiles <= 8 * 14)
    hipLaunchKernelGGL((chol_kernel<8, 14>), dim3(grid), dim3(8 * kWave), 0, s, G, d, dp, R, Rinv16, flags,
                       (DevInfo*)info, pass_id, tol, fast_tol, esq, nesq, mode, Xfull);
  else
    hipLaunchKernelGGL((chol_kernel<8, 17>), dim3(grid), dim3(8 * kWave), 0, s, G, d, dp, R, Rinv16, flags,
                       (DevInfo*)info, pass_id, tol, fast_tol, esq, nesq, mode, Xfull);
  if (ev1) (void)hipEventRecord(ev1, s);
  return hipGetLastError();
}

}  // namespace rqlp
