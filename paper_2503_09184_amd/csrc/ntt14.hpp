// ntt14.hpp -- the negacyclic transform for N = 2^14 with 32 residues per
// thread and half the row in LDS, so that two workgroups share a CU.
//
// Same transform as ntt_core.hpp (forward Cooley-Tukey with the psi twist in
// the twiddles, bit-reversed output; inverse Gentleman-Sande without N^-1),
// organised for occupancy: 512 threads hold the 16384 residues in registers
// and run the 14 stages in three register passes of 5, 5 and 4 stages:
//
//   pass A  stages 0-4   x = (u << 9) | a(t)              u = register 0..31
//   pass B  stages 5-9   x = b(t) | (u << 4)
//   pass C  stages 10-13 x = (k << 13) | c(t) | v        register k*16 + v
//
// a, b, c place the thread bits t0..t8 on the x bits a pass does not own.
// Between passes the residues move through LDS in two rounds, each over one
// half of the row (66.5 KiB with padding instead of 133 KiB).  The half is
// chosen by an x bit that every participating thread owns entirely in both
// distributions and that sits on a wave-uniform thread bit: x bit 3 = t8
// between A and B, x bit 12 = t7 between B and C.  So in each round whole
// waves write all 32 of their residues and then read all 32 of their new
// ones, and no register is needed twice.  The LDS index of a half-row word
// is y + (y >> 6), which keeps every exchange pattern at the minimum number
// of lanes per bank (2 of 64 lanes per 64-bank row).
//
// Storage orders.  Coefficient-domain rows at the boundary are in natural
// order (pass A order, read or written in 64-byte runs).  NTT-domain rows
// are stored in pass C's register-major order: the value of NTT index
// xc(t, r) sits at position r * 512 + t (pos_c), so every access of a pass C
// register by a wave is one contiguous 512-byte run.  Rows private to the
// fused key switch that stay in the coefficient domain use the same idea for
// pass A (pos_a = u * 512 + t).  Every kernel that touches NTT-domain data at
// N = 2^14 works position-wise or through these two maps.
#pragma once
#include "ntt_core.hpp"

namespace sfhe {

namespace n14 {

constexpr int kLogN = 14;
constexpr int kN = 1 << kLogN;
constexpr int kThreads = 512;
constexpr int kLdsWords = 8319;   // lp(8191) + 1

__device__ __forceinline__ int bit(int t, int i) { return (t >> i) & 1; }
// thread -> x bits of each distribution (see above)
__device__ __forceinline__ int a_of(int t) { return (t & 7) | (bit(t, 8) << 3) | (((t >> 3) & 31) << 4); }
__device__ __forceinline__ int b_of(int t) {
  return (t & 7) | (bit(t, 8) << 3) | (((t >> 3) & 7) << 9) | (bit(t, 7) << 12) | (bit(t, 6) << 13);
}
__device__ __forceinline__ int c_of(int t) { return ((t & 63) << 4) | (bit(t, 6) << 10) | (bit(t, 8) << 11) | (bit(t, 7) << 12); }
__device__ __forceinline__ int xa(int t, int u) { return (u << 9) | a_of(t); }
__device__ __forceinline__ int xb(int t, int u) { return b_of(t) | (u << 4); }
__device__ __forceinline__ int xc(int t, int r) { return ((r >> 4) << 13) | c_of(t) | (r & 15); }
// half-row word index: drop the split bit, then pad
__device__ __forceinline__ int lp(int y) { return y + (y >> 6); }
__device__ __forceinline__ int half_ab(int x) { return lp(((x >> 4) << 3) | (x & 7)); }
__device__ __forceinline__ int half_bc(int x) { return lp(((x >> 13) << 12) | (x & 4095)); }
// Each index above is its value at register 0 plus a constant of the
// register (the split and pad leave no carries), so a thread needs one base
// per pattern and the LDS instructions take the rest as immediate offsets:
//   half_ab(xa(t,u)) = half_ab(xa(t,0)) + 260 u
//   half_ab(xb(t,u)) = half_ab(xb(t,0)) + 8 u + (u >> 3)
//   half_bc(xb(t,u)) = half_bc(xb(t,0)) + 16 u + (u >> 2)
//   half_bc(xc(t,r)) = half_bc(xc(t,0)) + 4160 (r >> 4) + (r & 15)
//   xa(t,u) = xa(t,0) + 512 u,  xc(t,r) = xc(t,0) + 8192 (r >> 4) + (r & 15)
__device__ __forceinline__ constexpr int off_ab_a(int u) { return 260 * u; }
__device__ __forceinline__ constexpr int off_ab_b(int u) { return 8 * u + (u >> 3); }
__device__ __forceinline__ constexpr int off_bc_b(int u) { return 16 * u + (u >> 2); }
__device__ __forceinline__ constexpr int off_bc_c(int r) { return 4160 * (r >> 4) + (r & 15); }
__device__ __forceinline__ constexpr int off_a(int u) { return 512 * u; }
// register-major storage positions (see above)
__device__ __forceinline__ constexpr int pos_c(int t, int r) { return r * kThreads + t; }
__device__ __forceinline__ constexpr int pos_a(int t, int u) { return u * kThreads + t; }
__device__ __forceinline__ constexpr int off_c(int r) { return 8192 * (r >> 4) + (r & 15); }

// The thread index as a value the compiler cannot hoist: index arithmetic
// derived from it is redone where it is used instead of being kept live
// (dozens of registers) across the transforms.
__device__ __forceinline__ int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// The thread index made to depend on two registers of a finished transform:
// loads addressed from it cannot be issued before the transform's last
// stages, which keeps an epilogue's loads from being hoisted into the
// transform and spilled.
template <typename Val>
__device__ __forceinline__ int after(int x, const Val& a, const Val& b) {
  asm volatile("" : "+v"(x) : "v"(a), "v"(b));
  return x;
}

// ---------------------------------------------------------------- exchanges
// A -> B (forward) or B -> A (inverse): rounds over x bit 3 = t8
template <typename Val, bool A_TO_B>
__device__ __forceinline__ void exchange_ab(Val (&v)[32], Val* sh, int t) {
  const int me = bit(t, 8);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (me == h) {
      const int tt = opaque(t);
      Val* w = sh + (A_TO_B ? half_ab(xa(tt, 0)) : half_ab(xb(tt, 0)));
#pragma unroll
      for (int u = 0; u < 32; ++u) w[A_TO_B ? off_ab_a(u) : off_ab_b(u)] = v[u];
    }
    __syncthreads();
    if (me == h) {
      const int tt = opaque(t);
      const Val* rd = sh + (A_TO_B ? half_ab(xb(tt, 0)) : half_ab(xa(tt, 0)));
#pragma unroll
      for (int u = 0; u < 32; ++u) v[u] = rd[A_TO_B ? off_ab_b(u) : off_ab_a(u)];
    }
    __syncthreads();
  }
}

// B -> C (forward) or C -> B (inverse): rounds over x bit 12 = t7
template <typename Val, bool B_TO_C>
__device__ __forceinline__ void exchange_bc(Val (&v)[32], Val* sh, int t) {
  const int me = bit(t, 7);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (me == h) {
      const int tt = opaque(t);
      Val* w = sh + (B_TO_C ? half_bc(xb(tt, 0)) : half_bc(xc(tt, 0)));
#pragma unroll
      for (int u = 0; u < 32; ++u) w[B_TO_C ? off_bc_b(u) : off_bc_c(u)] = v[u];
    }
    __syncthreads();
    if (me == h) {
      const int tt = opaque(t);
      const Val* rd = sh + (B_TO_C ? half_bc(xc(tt, 0)) : half_bc(xb(tt, 0)));
#pragma unroll
      for (int u = 0; u < 32; ++u) v[u] = rd[B_TO_C ? off_bc_c(u) : off_bc_b(u)];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- passes
// A stage is 16 butterflies; its twiddles (two words each on the integer
// path) are loaded in groups of 8 butterflies, scheduled apart, so that the
// loads of a whole stage never hold 64 registers at once.
__device__ __forceinline__ void bfly_fence(int u, int d) {
  // the butterfly ordinal of lower index u at distance d is (u / (2d)) * d + u % d
  const int n = (u / (2 * d)) * d + (u % d);
  if ((n & 7) == 7) __builtin_amdgcn_sched_barrier(0);
}
// forward stage s pairs x and x + 2^(13-s); its twiddle is w[2^s + (x >> (14-s))]
template <typename Ar>
__device__ __forceinline__ void fwd_a(const Ar& ar, typename Ar::Val (&v)[32]) {
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    const int d = 1 << (4 - s);
#pragma unroll
    for (int u = 0; u < 32; ++u)
      if (!(u & d)) {
        ar.ct(v[u], v[u + d], (1 << s) + (u >> (5 - s)));
        bfly_fence(u, d);
      }
  }
}
template <typename Ar>
__device__ __forceinline__ void fwd_b(const Ar& ar, typename Ar::Val (&v)[32], int t) {
  const int hb = b_of(opaque(t)) & ~15;
#pragma unroll
  for (int s = 5; s < 10; ++s) {
    const int d = 1 << (9 - s);
    const int base = (1 << s) + (hb >> (14 - s));
#pragma unroll
    for (int u = 0; u < 32; ++u)
      if (!(u & d)) {
        ar.ct(v[u], v[u + d], base + (u >> (10 - s)));
        bfly_fence(u, d);
      }
  }
}
template <typename Ar>
__device__ __forceinline__ void fwd_c(const Ar& ar, typename Ar::Val (&v)[32], int t) {
  const int ct = c_of(opaque(t));
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int xk = (k << 13) | ct;
#pragma unroll
    for (int s = 10; s < 14; ++s) {
      const int d = 1 << (13 - s);
      const int base = (1 << s) + (xk >> (14 - s));
#pragma unroll
      for (int r = 0; r < 16; ++r)
        if (!(r & d)) {
          ar.ct(v[k * 16 + r], v[k * 16 + r + d], base + (r >> (14 - s)));
          bfly_fence(r, d);
        }
    }
  }
}
// inverse stage with distance 2^dd pairs x and x + 2^dd; twiddle iw[N/2^(dd+1) + (x >> (dd+1))]
template <typename Ar>
__device__ __forceinline__ void inv_c(const Ar& ar, typename Ar::Val (&v)[32], int t) {
  const int ct = c_of(opaque(t));
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int xk = (k << 13) | ct;
#pragma unroll
    for (int dd = 0; dd < 4; ++dd) {
      const int d = 1 << dd;
      const int base = (kN >> (dd + 1)) + (xk >> (dd + 1));
#pragma unroll
      for (int r = 0; r < 16; ++r)
        if (!(r & d)) {
          ar.gs(v[k * 16 + r], v[k * 16 + r + d], base + (r >> (dd + 1)));
          bfly_fence(r, d);
        }
    }
  }
}
template <typename Ar>
__device__ __forceinline__ void inv_b(const Ar& ar, typename Ar::Val (&v)[32], int t) {
  const int hb = b_of(opaque(t)) & ~15;
#pragma unroll
  for (int dd = 4; dd < 9; ++dd) {
    const int d = 1 << (dd - 4);
    const int base = (kN >> (dd + 1)) + (hb >> (dd + 1));
#pragma unroll
    for (int u = 0; u < 32; ++u)
      if (!(u & d)) {
        ar.gs(v[u], v[u + d], base + (u >> (dd - 3)));
        bfly_fence(u, d);
      }
  }
}
template <typename Ar>
__device__ __forceinline__ void inv_a(const Ar& ar, typename Ar::Val (&v)[32]) {
#pragma unroll
  for (int dd = 9; dd < 14; ++dd) {
    const int d = 1 << (dd - 9);
#pragma unroll
    for (int u = 0; u < 32; ++u)
      if (!(u & d)) {
        ar.gs(v[u], v[u + d], (kN >> (dd + 1)) + (u >> (dd - 8)));
        bfly_fence(u, d);
      }
  }
}
template <typename Ar>
__device__ __forceinline__ void fold_all(const Ar& ar, typename Ar::Val (&v)[32]) {
#pragma unroll
  for (int u = 0; u < 32; ++u) ar.fold(v[u]);
}

// Whole transforms on registers.  forward: v in A order on entry, C order on
// exit.  inverse: C order on entry, A order on exit (N^-1 not applied).  The
// caller synchronises before sh is reused.
template <typename Ar>
__device__ __forceinline__ void forward(const Ar& ar, typename Ar::Val (&v)[32], typename Ar::Val* sh, int t) {
  fwd_a(ar, v);
  exchange_ab<typename Ar::Val, true>(v, sh, t);
  fwd_b(ar, v, t);
  exchange_bc<typename Ar::Val, true>(v, sh, t);
  fwd_c(ar, v, t);
}
template <typename Ar>
__device__ __forceinline__ void inverse(const Ar& ar, typename Ar::Val (&v)[32], typename Ar::Val* sh, int t) {
  inv_c(ar, v, t);
  fold_all(ar, v);
  exchange_bc<typename Ar::Val, false>(v, sh, t);
  inv_b(ar, v, t);
  fold_all(ar, v);
  exchange_ab<typename Ar::Val, false>(v, sh, t);
  inv_a(ar, v);
}

}  // namespace n14
}  // namespace sfhe
