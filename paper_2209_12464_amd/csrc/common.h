// Shared device helpers for the gfx950 kernels: vector types, MFMA traits,
// the XCD-aware block remap and the counter-based Gaussian generator.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rqlp {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;
constexpr int kXcds = 8;       // MI355X: 8 accelerator complex dies, 32 CUs each
constexpr int kDMax = 544;        // largest d = k + p (dense inputs)
constexpr int kDMaxCsr = 256;     // largest d = k + p for sparse (CSR) inputs
constexpr int kCholRegMax = 256;  // up to this d the Cholesky holds G in registers
constexpr int kTile = 16;      // side of the float64 Cholesky / solve tiles

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// Workgroups are dealt to the XCDs round-robin (block b runs on XCD b % 8).
// Remap so that each XCD gets a contiguous range of logical tile ids, which
// keeps tiles that share an operand chunk in the same L2.
__device__ inline int xcd_remap(int b, int nblocks) {
  const int q = nblocks / kXcds, r = nblocks % kXcds;
  const int x = b % kXcds, j = b / kXcds;
  return x * q + (x < r ? x : r) + j;
}

// ---------------------------------------------------------------------------
// MFMA shapes.  Operand layouts (verified on gfx950):
//   A operand: lane l supplies A[m = l % TM][k = l / TM] (TM * TK = 64)
//   B operand: lane l supplies B[k = l / TN][n = l % TN]
//   f32 16x16x4: acc[r] = C[4 (l/16) + r][l % 16]
//   f64 16x16x4: acc[r] = C[l/16 + 4 r][l % 16]
template <typename T> struct Mfma;

template <> struct Mfma<float> {
  static constexpr int TM = 16, TN = 16, TK = 4, NACC = 4;
  typedef floatx4 acc_t;
  __device__ static inline acc_t zero() { acc_t z; for (int i = 0; i < 4; ++i) z[i] = 0.f; return z; }
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
  __device__ static inline int col(int lane) { return lane & 15; }
};

template <> struct Mfma<double> {
  static constexpr int TM = 16, TN = 16, TK = 4, NACC = 4;
  typedef doublex4 acc_t;
  __device__ static inline acc_t zero() { acc_t z; for (int i = 0; i < 4; ++i) z[i] = 0.0; return z; }
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
  __device__ static inline int col(int lane) { return lane & 15; }
};

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller.
constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;
constexpr uint64_t kSketchKey1 = 0x52514C50ull;  // "RQLP"

struct u64x4 { uint64_t x0, x1, x2, x3; };

__device__ inline u64x4 philox4x64_10(u64x4 c, uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t lo0 = kPhiloxM0 * c.x0, hi0 = __umul64hi(kPhiloxM0, c.x0);
    const uint64_t lo1 = kPhiloxM1 * c.x2, hi1 = __umul64hi(kPhiloxM1, c.x2);
    u64x4 n;
    n.x0 = hi1 ^ c.x1 ^ k0;
    n.x1 = lo1;
    n.x2 = hi0 ^ c.x3 ^ k1;
    n.x3 = lo0;
    c = n;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  return c;
}

// Two N(0,1) values from two 64-bit words (top 53 bits of each).
__device__ inline void box_muller(uint64_t w0, uint64_t w1, double& z0, double& z1) {
  const double u1 = ((double)(w0 >> 11) + 1.0) * 0x1p-53;
  const double u2 = (double)(w1 >> 11) * 0x1p-53;
  const double r = sqrt(-2.0 * log(u1));
  const double t = (2.0 * 3.141592653589793) * u2;
  double s, c;
  sincos(t, &s, &c);
  z0 = r * c;
  z1 = r * s;
}

// The Gaussian with logical index l of stream (seed, key1).
__device__ inline double gaussian_at(uint64_t seed, uint64_t key1, uint64_t l) {
  u64x4 c = {l >> 2, 0, 0, 0};
  const u64x4 w = philox4x64_10(c, seed, key1);
  const int t = (int)(l & 3);
  double z0, z1;
  if (t < 2) box_muller(w.x0, w.x1, z0, z1);
  else box_muller(w.x2, w.x3, z0, z1);
  return (t & 1) ? z1 : z0;
}

// Device-side info record (mirrors rqlp_info).
struct DevInfo {
  int32_t status;
  int32_t completed_cols;
  int32_t breakdown_pass;
  int32_t nonfinite;
};

}  // namespace rqlp
