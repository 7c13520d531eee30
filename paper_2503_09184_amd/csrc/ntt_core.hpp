// ntt_core.hpp -- the in-LDS negacyclic transform shared by the NTT kernels
// and the fused key-switching kernels.
//
// One workgroup transforms one row of N residues (N <= 2^14) held in LDS.
// Forward: Cooley-Tukey with the psi twist merged into the twiddles (Longa
// and Naehrig 2016), bit-reversed output, so index k holds a(psi^(2 brv(k)+1)).
// Inverse: Gentleman-Sande; N^-1 is applied by the caller.
//
// The log2 N butterfly stages run in passes of up to four: a thread holds 16
// residues x0 + u * t (u < 16) in registers, performs the pass's four stages
// on them, and the pass ends with one LDS exchange and one barrier (4 passes
// instead of 14 for N = 2^14).  LDS rows are padded by one word every 16, so
// every pass's access pattern hits each bank at most four times per wave.
//
// Two arithmetics: primes below 2^42 run the butterflies in exact fp64
// (products a*b - k*q via fma; forward values grow by at most 1.5 q per stage
// and need no reduction before the end, inverse values are folded after each
// pass); larger primes use Harvey's lazy integer butterflies with Shoup
// quotients (forward values in [0, 4q), inverse in [0, 2q)).
#pragma once
#include "internal.hpp"

namespace sfhe {

constexpr int kMaxRows = 2 * kMaxBasis;   // rows per group: both polys of a ciphertext
constexpr int kPadShift = 4;

struct NttRows {
  u64* base;
  int64_t bstride;
  int nrow;
  int pos[kMaxRows];
  int prime[kMaxRows];
  // N = 2^15 only: twiddle tables of the two 2^14-point halves,
  // [prime][direction][half][2^14] (values, Shoup companions, fp64 values)
  const u64* sub;
  const u64* sub_s;
  const double* subd;
};

__device__ __forceinline__ int lpos(int x) { return x + (x >> kPadShift); }

// exact fp64 a*b mod q up to a multiple of q: |result| <= 1.5 q for |a*b| < 2^92, q < 2^42
__device__ __forceinline__ double fmm(double a, double b, double q, double qinv) {
  const double h = a * b;
  const double l = fma(a, b, -h);
  const double k = rint(h * qinv);
  return fma(-k, q, h) + l;
}
__device__ __forceinline__ u64 fp_to_residue(double x, double q, double qinv) {
  const double k = floor(x * qinv);
  double r = fma(-k, q, x);
  r = r < 0.0 ? r + q : r;
  r = r >= q ? r - q : r;
  return f64_to_u52(r);
}

struct NttInt {
  typedef u64 Val;
  u64 q, q2;
  const u64 *w, *ws;
  __device__ NttInt(const PrimeDev& P, bool inv) : q(P.q), q2(2 * P.q), w(inv ? P.itw : P.tw), ws(inv ? P.itws : P.tws) {}
  __device__ Val in(u64 x) const { return x; }
  __device__ void ct(Val& X, Val& Y, int idx) const {
    const u64 x = X >= q2 ? X - q2 : X;
    const u64 T = mul_shoup_lazy(Y, w[idx], ws[idx], q);
    X = x + T;
    Y = x - T + q2;
  }
  __device__ void gs(Val& X, Val& Y, int idx) const {
    u64 S = X + Y;
    S = S >= q2 ? S - q2 : S;
    const u64 D = X - Y + q2;
    X = S;
    Y = mul_shoup_lazy(D, w[idx], ws[idx], q);
  }
  __device__ void fold(Val&) const {}
  __device__ u64 out_fwd(Val x) const {
    x = x >= q2 ? x - q2 : x;
    return x >= q ? x - q : x;
  }
  __device__ u64 fwd_res(Val x) const { return out_fwd(x); }
  __device__ u64 inv_res(Val x, const PrimeDev& P) const { return out_inv(x, P); }
  __device__ u64 out_inv(Val x, const PrimeDev& P) const {
    const u64 v = mul_shoup_lazy(x, P.ninv, P.ninv_s, q);
    return v >= q ? v - q : v;
  }
  // inverse output times a constant w in [0, q) (Shoup companion ws) that
  // already holds N^-1
  __device__ u64 out_mul(Val x, u64 w, u64 ws) const {
    const u64 v = mul_shoup_lazy(x, w, ws, q);
    return v >= q ? v - q : v;
  }
};

struct NttFp {
  typedef double Val;
  double q, qinv;
  const double* w;
  __device__ NttFp(const PrimeDev& P, bool inv) : q((double)P.q), qinv(1.0 / (double)P.q), w(inv ? P.itwd : P.twd) {}
  __device__ Val in(u64 x) const { return u52_to_f64(x); }   // x < q < 2^42
  __device__ void ct(Val& X, Val& Y, int idx) const {
    const double T = fmm(w[idx], Y, q, qinv);
    const double x = X;
    X = x + T;
    Y = x - T;
  }
  __device__ void gs(Val& X, Val& Y, int idx) const {
    const double S = X + Y, D = X - Y;
    X = S;
    Y = fmm(w[idx], D, q, qinv);
  }
  __device__ void fold(Val& x) const { x = fma(-rint(x * qinv), q, x); }
  __device__ u64 out_fwd(Val x) const { return fp_to_residue(x, q, qinv); }
  __device__ u64 fwd_res(Val x) const { return out_fwd(x); }
  __device__ u64 inv_res(Val x, const PrimeDev& P) const { return out_inv(x, P); }
  __device__ u64 out_inv(Val x, const PrimeDev& P) const {
    return fp_to_residue(fmm(x, (double)P.ninv, q, qinv), q, qinv);
  }
  __device__ u64 out_mul(Val x, u64 w, u64) const { return fp_to_residue(fmm(x, (double)w, q, qinv), q, qinv); }
};

// one forward pass of P stages s0 .. s0+P-1 over all units of this thread;
// reads from gsrc (a row in HBM) when non-null, else from LDS
template <int P, typename Ar>
__device__ __forceinline__ void fwd_pass(const Ar& ar, typename Ar::Val* sh, const u64* gsrc, int N, int logN, int s0) {
  typedef typename Ar::Val Val;
  constexpr int R = 1 << P;
  const int ltP = logN - s0 - P;
  const int tP = 1 << ltP;
  for (int th = threadIdx.x; th < (N >> P); th += blockDim.x) {
    const int g = th >> ltP, r = th & (tP - 1);
    const int x0 = (g << (ltP + P)) + r;
    Val v[R];
#pragma unroll
    for (int u = 0; u < R; ++u) v[u] = gsrc ? ar.in(gsrc[x0 + u * tP]) : sh[lpos(x0 + u * tP)];
#pragma unroll
    for (int qq = 0; qq < P; ++qq) {
      const int dq = 1 << (P - 1 - qq);
      const int m = 1 << (s0 + qq);
#pragma unroll
      for (int u = 0; u < R; ++u)
        if (!(u & dq)) ar.ct(v[u], v[u + dq], m + (g << qq) + (u >> (P - qq)));
    }
#pragma unroll
    for (int u = 0; u < R; ++u) sh[lpos(x0 + u * tP)] = v[u];
  }
}

// one inverse pass of P stages with distances t0, 2 t0, ..., 2^(P-1) t0;
// writes the scaled residues to gdst (a row in HBM) when non-null, else folds
// them back into LDS
template <int P, typename Ar>
__device__ __forceinline__ void inv_pass(const Ar& ar, typename Ar::Val* sh, u64* gdst, const PrimeDev& Pr, int N,
                                         int logN, int lt0) {
  typedef typename Ar::Val Val;
  constexpr int R = 1 << P;
  const int t0 = 1 << lt0;
  for (int th = threadIdx.x; th < (N >> P); th += blockDim.x) {
    const int g = th >> lt0, r = th & (t0 - 1);
    const int x0 = (g << (lt0 + P)) + r;
    Val v[R];
#pragma unroll
    for (int u = 0; u < R; ++u) v[u] = sh[lpos(x0 + u * t0)];
#pragma unroll
    for (int qq = 0; qq < P; ++qq) {
      const int dq = 1 << qq;
      const int h = N >> (lt0 + qq + 1);
#pragma unroll
      for (int u = 0; u < R; ++u)
        if (!(u & dq)) ar.gs(v[u], v[u + dq], h + (g << (P - 1 - qq)) + (u >> (qq + 1)));
    }
    if (gdst) {
#pragma unroll
      for (int u = 0; u < R; ++u) gdst[x0 + u * t0] = ar.out_inv(v[u], Pr);
    } else {
#pragma unroll
      for (int u = 0; u < R; ++u) {
        ar.fold(v[u]);
        sh[lpos(x0 + u * t0)] = v[u];
      }
    }
  }
}


// whole transforms, LDS to LDS (the caller has filled sh and synchronised;
// on return sh holds the transformed row and all threads are synchronised)
template <typename Ar>
__device__ __forceinline__ void fwd_lds(const Ar& ar, typename Ar::Val* sh, int N, int logN) {
  int s0 = 0;
  while (s0 < logN) {
    const int np = min(4, logN - s0);
    if (np == 4) fwd_pass<4>(ar, sh, nullptr, N, logN, s0);
    else if (np == 3) fwd_pass<3>(ar, sh, nullptr, N, logN, s0);
    else if (np == 2) fwd_pass<2>(ar, sh, nullptr, N, logN, s0);
    else fwd_pass<1>(ar, sh, nullptr, N, logN, s0);
    __syncthreads();
    s0 += np;
  }
}
// inverse without the N^-1 factor (Ar::inv_res applies it)
template <typename Ar>
__device__ __forceinline__ void inv_lds(const Ar& ar, typename Ar::Val* sh, const PrimeDev& P, int N, int logN) {
  int lt0 = 0;
  while (lt0 < logN) {
    const int np = min(4, logN - lt0);
    if (np == 4) inv_pass<4>(ar, sh, nullptr, P, N, logN, lt0);
    else if (np == 3) inv_pass<3>(ar, sh, nullptr, P, N, logN, lt0);
    else if (np == 2) inv_pass<2>(ar, sh, nullptr, P, N, logN, lt0);
    else inv_pass<1>(ar, sh, nullptr, P, N, logN, lt0);
    __syncthreads();
    lt0 += np;
  }
}

}  // namespace sfhe
