// hostmath.hpp -- host-side number theory for building the parameter tables:
// 64-bit modular arithmetic, primality, roots of unity, Shoup quotients.
#pragma once
#include <stdint.h>

#include <vector>

namespace sfhe {
namespace hostmath {

typedef unsigned __int128 u128;

inline uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

inline uint64_t powmod(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  b %= m;
  for (; e; e >>= 1) {
    if (e & 1) r = mulmod(r, b, m);
    b = mulmod(b, b, m);
  }
  return r;
}

inline uint64_t invmod(uint64_t a, uint64_t p) { return powmod(a % p, p - 2, p); }  // p prime

// floor(w * 2^64 / q) for w < q
inline uint64_t shoup(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }

// floor(2^128 / q) as (hi, lo); q odd so (2^128 - 1) / q has the same floor
inline void barrett128(uint64_t q, uint64_t* hi, uint64_t* lo) {
  u128 mu = (~(u128)0) / q;
  *hi = (uint64_t)(mu >> 64);
  *lo = (uint64_t)mu;
}

// Miller-Rabin with the seven bases of J. Sinclair, deterministic below 2^64.
inline bool probable_prime_base(uint64_t n, uint64_t a, uint64_t d, int s) {
  a %= n;
  if (a == 0) return true;
  uint64_t x = powmod(a, d, n);
  if (x == 1 || x == n - 1) return true;
  for (int i = 1; i < s; ++i) {
    x = mulmod(x, x, n);
    if (x == n - 1) return true;
  }
  return false;
}
inline bool is_prime(uint64_t n) {
  if (n < 2) return false;
  static const uint64_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (uint64_t p : small) {
    if (n % p == 0) return n == p;
  }
  uint64_t d = n - 1;
  int s = 0;
  while (!(d & 1)) { d >>= 1; ++s; }
  static const uint64_t bases[] = {2, 325, 9375, 28178, 450775, 9780504, 1795265022};
  for (uint64_t a : bases)
    if (!probable_prime_base(n, a, d, s)) return false;
  return true;
}

// The smallest primitive 2N-th root of unity modulo q (q = 1 mod 2N): any
// quadratic non-residue g gives h = g^((q-1)/2N) of order exactly 2N, and the
// primitive 2N-th roots are the odd powers of h.
inline uint64_t smallest_primitive_root_2n(uint64_t q, uint64_t two_n) {
  uint64_t g = 2;
  while (powmod(g, (q - 1) / 2, q) != q - 1) ++g;
  uint64_t h = powmod(g, (q - 1) / two_n, q);
  uint64_t h2 = mulmod(h, h, q);
  uint64_t best = h, x = h;
  for (uint64_t k = 1; k < two_n / 2; ++k) {
    x = mulmod(x, h2, q);
    if (x < best) best = x;
  }
  return best;
}

}  // namespace hostmath
}  // namespace sfhe
