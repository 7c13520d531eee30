// fparith.hpp -- exact residue arithmetic in fp64 for primes below 2^42,
// shared by the kernels that multiply residues without a transform around
// them (the ct x ct tensor and the plaintext-weight product).
#pragma once
#include "internal.hpp"

namespace sfhe {

// fp64 residue product: a*b - k*q exactly, with k = rint(a*b/q); |result| <= 1.5 q.
// Exact for integers a, b < 2^44 and q < 2^42 (2Prod via fma; h - k q and
// the sum with the rounding error are integers below 2^53).
__device__ __forceinline__ double fp_mulmod_lazy(double a, double b, double q, double qinv) {
  const double h = a * b;
  const double l = fma(a, b, -h);
  const double k = rint(h * qinv);
  return fma(-k, q, h) + l;
}
// reduce an exact integer-valued double |x| < 2^53 to [0, q)
__device__ __forceinline__ u64 fp_final(double x, double q, double qinv) {
  const double k = floor(x * qinv);
  double r = fma(-k, q, x);
  r = r < 0.0 ? r + q : r;
  r = r >= q ? r - q : r;
  return f64_to_u52(r);
}
// |x| < 2^53 exact integer -> congruent value of magnitude <= q / 2 + 1
__device__ __forceinline__ double fp_fold(double x, double q, double qinv) { return fma(-rint(x * qinv), q, x); }

struct FpLimb {
  int limb;
  double q, qinv;
};

struct FpLimbs {
  int n;
  FpLimb l[kMaxBasis];
};

}  // namespace sfhe
