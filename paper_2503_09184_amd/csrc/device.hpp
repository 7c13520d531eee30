// device.hpp -- types and device arithmetic shared by the gfx950 kernels.
//
// Residues are uint64 below primes q < 2^62.  gfx950 has no 64-bit integer
// multiplier: every 64x64 product is assembled from 32-bit mul_lo/mul_hi
// (v_mad_u64_u32), so the kernels use
//   * Shoup's precomputed-quotient product for a constant operand w
//     (w' = floor(w 2^64 / q); result lazily in [0, 2q)), and
//   * a Barrett reduction with mu = floor(2^128 / q) for full 128-bit values
//     (lazy sums of products), result exact in [0, q).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfhe {

typedef uint64_t u64;
typedef int64_t i64;
typedef uint32_t u32;

constexpr int kMaxBasis = 16;   // data + special primes
constexpr int kCdtLen = 20;     // |e| <= 19

// Per-prime constants (host-computed) and device table pointers.
struct PrimeDev {
  u64 q;
  u64 mu_hi, mu_lo;       // floor(2^128 / q)
  u64 ninv, ninv_s;       // N^-1 mod q and its Shoup quotient
  const u64* tw;          // psi^brv(m), m < N
  const u64* tws;         // Shoup quotients of tw
  const u64* itw;         // psi^-brv(m)
  const u64* itws;
  const double* twd;       // tw and itw as doubles (exact below 2^53)
  const double* itwd;
};

struct DevParams {
  int N, logN, L, alpha, dnum, nb;
  PrimeDev pr[kMaxBasis];
};

// ---------------------------------------------------------------- 128-bit
struct U128 {
  u64 lo, hi;
};

__device__ __forceinline__ U128 mul_wide(u64 a, u64 b) {
  U128 r;
  r.lo = a * b;
  r.hi = __umul64hi(a, b);
  return r;
}

__device__ __forceinline__ void add_wide(U128& acc, U128 x) {
  u64 lo = acc.lo + x.lo;
  acc.hi += x.hi + (lo < x.lo ? 1ull : 0ull);
  acc.lo = lo;
}

// x mod q for any 128-bit x.  qhat = x_hi mu_hi + hi(x_hi mu_lo) + hi(x_lo mu_hi)
// drops the low partial products (at most 2 below floor(x mu / 2^128)), which
// is itself at most 1 below floor(x / q); so x - qhat q, computed mod 2^64,
// lies in [0, 4q) and two conditional subtractions finish.
__device__ __forceinline__ u64 reduce_wide(U128 x, u64 q, u64 mu_hi, u64 mu_lo) {
  u64 qhat = x.hi * mu_hi + __umul64hi(x.hi, mu_lo) + __umul64hi(x.lo, mu_hi);
  u64 r = x.lo - qhat * q;
  r = r >= 2 * q ? r - 2 * q : r;
  r = r >= q ? r - q : r;
  return r;
}

__device__ __forceinline__ u64 mul_mod(u64 a, u64 b, const PrimeDev& P) {
  return reduce_wide(mul_wide(a, b), P.q, P.mu_hi, P.mu_lo);
}

// Shoup: x * w mod q for a constant w < q, any x < 2^64; result in [0, 2q).
__device__ __forceinline__ u64 mul_shoup_lazy(u64 x, u64 w, u64 ws, u64 q) {
  u64 qh = __umul64hi(x, ws);
  return x * w - qh * q;
}
__device__ __forceinline__ u64 mul_shoup(u64 x, u64 w, u64 ws, u64 q) {
  u64 r = mul_shoup_lazy(x, w, ws, q);
  return r >= q ? r - q : r;
}

__device__ __forceinline__ u64 add_mod(u64 a, u64 b, u64 q) {
  u64 s = a + b;
  return s >= q ? s - q : s;
}
__device__ __forceinline__ u64 sub_mod(u64 a, u64 b, u64 q) {
  return a >= b ? a - b : a + q - b;
}
// a signed value with |v| < 2^63 reduced mod q via the Barrett path
__device__ __forceinline__ u64 signed_mod(i64 v, const PrimeDev& P) {
  if (v >= 0) return reduce_wide(U128{(u64)v, 0}, P.q, P.mu_hi, P.mu_lo);
  u64 r = reduce_wide(U128{(u64)(-v), 0}, P.q, P.mu_hi, P.mu_lo);
  return r == 0 ? 0 : P.q - r;
}

// Exact conversions between integers below 2^52 and fp64 through the
// mantissa of 2^52: one integer op and one fp64 op each way.
__device__ __forceinline__ double u52_to_f64(u64 x) {
  return __longlong_as_double((long long)(x | 0x4330000000000000ull)) - 4503599627370496.0;
}
__device__ __forceinline__ u64 f64_to_u52(double r) {   // r an integer in [0, 2^52)
  return (u64)__double_as_longlong(r + 4503599627370496.0) & 0x000FFFFFFFFFFFFFull;
}

// ---------------------------------------------------------------- randomness
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) used as a counter-based
// generator: stream key k = mix(seed + (tag+1) G), then k = mix(k + (f+1) G)
// for each field f; word n of the stream is mix(k + (n+1) G).
constexpr u64 kGolden = 0x9E3779B97F4A7C15ull;

__host__ __device__ __forceinline__ u64 sm_mix(u64 z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ __forceinline__ u64 sm_key(u64 seed, u64 tag) { return sm_mix(seed + (tag + 1) * kGolden); }
__host__ __device__ __forceinline__ u64 sm_field(u64 key, u64 f) { return sm_mix(key + (f + 1) * kGolden); }
__host__ __device__ __forceinline__ u64 sm_word(u64 key, u64 n) { return sm_mix(key + (n + 1) * kGolden); }

// stream tags
enum : u64 { kTagSecret = 1, kTagRlkA = 2, kTagRlkE = 3, kTagEncA = 4, kTagEncE = 5 };

// uniform residue of coefficient t: (w(2t) 2^64 + w(2t+1)) mod q
__device__ __forceinline__ u64 uniform_residue(u64 key, u64 t, const PrimeDev& P) {
  U128 x{sm_word(key, 2 * t + 1), sm_word(key, 2 * t)};
  return reduce_wide(x, P.q, P.mu_hi, P.mu_lo);
}

// discrete Gaussian magnitude by cumulative table (63-bit uniform), sign from bit 63
__device__ __forceinline__ i64 cdt_sample(const u64* T, u64 w) {
  u64 u = w & 0x7FFFFFFFFFFFFFFFull;
  int mag = kCdtLen - 1;
#pragma unroll
  for (int k = kCdtLen - 1; k >= 0; --k) mag = (u < T[k]) ? k : mag;
  return (w >> 63) ? -(i64)mag : (i64)mag;
}

}  // namespace sfhe
