// Cholesky factor of the float64 Gram matrix, G = R^T R (R upper), for
// d <= 256: the middle step of each CholeskyQR pass (orth() and qr() of the
// paper, computed as an unpivoted QR with a positive diagonal in R).
//
// One workgroup of 8 waves, right-looking over 16-column blocks k.  The
// lower triangle of G is cut into 16 x 16 tiles held in registers (MFMA
// 16x16x4 accumulator layout: lane l holds rows l/16 + 4 s, column l % 16),
// dealt round-robin to the waves.  Per block column k:
//   A. the owner of tile (k,k) moves it to one column per lane and factors
//      it there, forming the inverse of the 16 x 16 factor in the same
//      sweep (every cross-lane value is a readlane broadcast);
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

constexpr double kFastPathTol = 0x1p-30;

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

// 1/x to float64 accuracy: hardware estimate and two Newton steps.
__device__ inline double rcp_f64(double x) {
  double y = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
  }
  return y;
}

// Factor the 16 x 16 diagonal tile S = L L^T in column-per-lane form and
// form X = L^-1 in the same sweep.  Lane c < 16 holds column c of S in v[]
// (both triangles, S symmetric); lane 16 + c holds column c of X (starting
// as the identity).  Per pivot J every value another lane needs is column J
// of S, read from lane J as wave-uniform scalars, and both halves apply the
// same update v[r] -= S[r][J] * coef for r > J, with coef = S[J][c] / S[J][J]
// (lanes c > J of S) or X[J][c] / S[J][J] (X), before row J is scaled by
// 1 / sqrt(S[J][J]).  The chain from one pivot to the next is a reciprocal
// and one FMA; 1/sqrt runs beside it.  On return lane c holds row c of L
// (column c of R = L^T, zero below the diagonal) and lane 16 + c column c of
// X; depmask has bit J set for each dependent pivot.  Lanes 32..63 repeat
// lanes 0..31.
__device__ inline void factor_diag_tile(double (&v)[kTile], int lane, double gdl, double tol,
                                        int& depmask) {
  // gdl: lane c holds the original squared norm of column c (the pivot test)
  int c = lane & 15;
  // opaque to the optimizer: keeps the per-step lane masks from being
  // hoisted out of the block loop, where they would pin scalar registers
  asm volatile("" : "+v"(c));
  const bool xs = (lane & 16) != 0;  // this lane holds a column of X
#pragma unroll
  for (int J = 0; J < kTile; ++J) {
    const double piv = bcast(v[J], J);  // S[J][J]
    const bool dep = !(piv > tol * bcast(gdl, J));
    // both chains are computed unconditionally (no branch) and selected
    const double rp = dep ? 0.0 : rcp_f64(piv);
    const double inv = dep ? 1.0 : rsqrt_f64(piv);
    const bool upd = xs || c > J;
    const double vj = v[J];  // S[J][c] or X[J][c]
    const double coef = upd ? vj * rp : 0.0;
#pragma unroll
    for (int r = J + 1; r < kTile; ++r) v[r] = fma(-bcast(v[r], J), coef, v[r]);
    double nv = upd ? vj * inv : vj;       // X[J][c], or L[c][J] for c > J
    if (!xs && c > J && dep) nv = 0.0;
    if (!xs && c == J) nv = dep ? 1.0 : piv * inv;  // L[J][J]
    v[J] = nv;
    depmask |= dep ? (1 << J) : 0;
    __builtin_amdgcn_sched_barrier(0);  // keep the steps apart: bounds the live scalars
  }
  // lane c of S: entries below the diagonal of R = L^T are zero
  if (!xs) {
#pragma unroll
    for (int r = 0; r < kTile; ++r)
      if (r > c) v[r] = 0.0;
  }
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
  __shared__ double Pn[kDMax / kTile][kTile][kTile + 1];  // panel tiles L_ik of column k
  __shared__ double Di[kTile][kTile + 1];                  // inverse of the diagonal factor
  __shared__ double Gdiag[kDMax];
  __shared__ int defl[kDMax];
  __shared__ double red[NW];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int T = dp / kTile;
  const int lr = lane >> 4, lc = lane & 15;  // MFMA accumulator layout: row lr + 4 r, col lc

  // ---------------- fast path: G close to the identity ----------------
  // ||G - I||_F^2 comes as per-block partial sums from the Gram reduction;
  // every workgroup adds them in the same fixed order.
  if (fast_tol > 0.0) {
    double ss = 0.0;
    for (int e = tid; e < nesq; e += blockDim.x) ss += esq[e];
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    double tot = 0.0;
    for (int w = 0; w < NW; ++w) tot += red[w];
    if (tot < fast_tol * fast_tol) {  // false for NaN
      // all workgroups write their share of R = I + F, R^-1 = I - F
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
      return;
    }
    __syncthreads();
  }
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

  // A: the owner of tile (k,k) factors it (column per lane) and publishes
  // Di = L_kk^-1, the R block L_kk^T, its inverse and the dependent-column
  // flags.
  auto factor_diag = [&](int k, int sk) {
#pragma unroll
    for (int sl = 0; sl < SLOTS; ++sl)
      if (sl == sk) {
#pragma unroll
        for (int r = 0; r < 4; ++r) Di[lr + 4 * r][lc] = tile[sl][r];
      }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const bool xs = (lane & 16) != 0;
    double v[kTile];
#pragma unroll
    for (int r = 0; r < kTile; ++r) v[r] = xs ? (r == lc ? 1.0 : 0.0) : Di[r][lc];
    const double gdl = Gdiag[k * kTile + lc];
    __builtin_amdgcn_wave_barrier();
    int depmask = 0;
    factor_diag_tile(v, lane, gdl, tol, depmask);
    if (lane < kTile) {
#pragma unroll
      for (int r = 0; r < kTile; ++r) R[(int64_t)(k * kTile + r) * dp + k * kTile + lc] = v[r];  // R[r][c]
      const int dep_c = (depmask >> lc) & 1;
      defl[k * kTile + lc] = dep_c;
      flags[k * kTile + lc] = dep_c;
    } else if (lane < 2 * kTile) {
#pragma unroll
      for (int r = 0; r < kTile; ++r) {
        Di[r][lc] = v[r];                                            // X[r][c]
        Rinv16[(int64_t)k * kTile * kTile + lc * kTile + r] = v[r];  // (L^-1)^T
      }
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

hipError_t launch_chol(const double* G, int d, int dp, double* R, double* Rinv16, int32_t* flags,
                       void* info, int pass_id, double fast_tol, const double* esq, int nesq,
                       int32_t* mode, double* Xfull, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const double tol = 64.0 * (double)d * 2.220446049250313e-16;
  if (ev0) (void)hipEventRecord(ev0, s);
  const int T = dp / kTile;
  // register slots per wave for the T (T + 1) / 2 lower tiles (waves x
  // slots chosen so that tiles and the diagonal-block code fit in registers)
  const int tiles = T * (T + 1) / 2;
  const unsigned grid = fast_tol > 0.0 ? 16 : 1;  // extra workgroups only help the fast path
  if (tiles <= 8 * 7)
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
