// ks14.hip -- relinearisation and rescale of the lazy sums at N = 2^14,
// fused around the register transforms of ntt14.hpp (the key-switch and
// rescale steps of Algorithm 1, applied once per output).
//
// For a slice of n outputs at level lev (data primes q_0..q_lev, special
// primes p_0..p_{alpha-1}, digits D_j of alpha consecutive data primes) with
// D[b] = (d0, d1, d2) in the NTT domain, these kernels compute
// C[b] = Rescale((d0, d1) + KeySwitch(d2)):
//
//  K1 (b, i)    y_i = [iNTT(d2_i) (D_j/q_i)^-1]_{q_i}: ModUp's pre-scale,
//               with N^-1 folded into the constant.
//  BConv (b, j, e, x)  ext_{j,e} = sum_{i in D_j} y_i [D_j/q_i]_e (y_i
//               centered) for every digit j and every prime e outside it
//               (element-wise).
//  K2 (b, e)    x_j = NTT(ext_{j,e}) for the digits j not holding e, and the
//               key products acc_p = sum_j x_j rlk_j,p[e] (+ d2_e rlk_own,p[e]
//               when e is a data prime of digit own).  Data prime: acc_p is
//               kept (NTT domain).  Special prime p_k: acc_p goes back to
//               coefficients times (P/p_k)^-1, ModDown's pre-scale yP_k.
//  K3a (b, p)   the last prime of the key-switched sum, in coefficients:
//               r = iNTT(acc_lev P^-1 + d_lev) - z_lev P^-1 with
//               z_i = sum_k yP_k [P/p_k]_{q_i}.
//  K3b (b, p, i), i < lev:  C_i = (acc_i P^-1 + d_i - NTT(w_i)) q_lev^-1,
//               with the lift w_i = z_i P^-1 + [centered r]_{q_i} computed
//               as the row is loaded.
//
// Every identity is exact modular arithmetic, so the result is the same, bit
// for bit, as key switching with centered fast base conversions followed by
// an exactly rounded rescale.  Per output this takes 4 L + 4 + (the base
// conversions') transforms -- 32 at L = 5, alpha = 3, dnum = 2 -- instead of
// the 42 of the separate steps.  The transform kernels load, transform and
// store with light arithmetic on either side; ModUp's base conversion, whose
// rows are each read by several target primes' transforms spread over the
// chip, is an element-wise kernel of its own, while ModDown's (the lift)
// is taken by K3b as it loads.
//
// Without the rescale (a rotation's key switch: D = (c0, 0, c1) after the
// automorphism) K3a is skipped, the lift is w_i = z_i P^-1 for every
// i <= lev and K3b writes acc_i P^-1 + d_i - NTT(w_i) itself.
//
// Each transform block has 512 threads and 66.5 KiB of LDS, two blocks per
// CU.  NTT-domain rows are in the register-major order pos_c of ntt14.hpp,
// the private coefficient rows (y, ext, yP, r, w) in pos_a, so every access
// of a register by a wave is one contiguous 512-byte run.
#include "ntt14.hpp"

namespace sfhe {

namespace {

using n14::kN;
using n14::pos_a;
using n14::pos_c;
using n14::after;

// keeps the scheduler from hoisting the loads of all 32 element-wise steps
// at once (which would spill): every group of G steps is scheduled apart
template <int G>
__device__ __forceinline__ void group_fence(int u) {
  if ((u % G) == G - 1) __builtin_amdgcn_sched_barrier(0);
}

struct Ks14Args {
  const u64* D;          // [n] x dw words: d0, d1, d2 rows of nl primes (NTT domain)
  int64_t dw;
  u64* y;                // [n][nl][N]          ModUp inputs, coefficients
  u64* ext;              // [n][next][N]        base-converted digits, coefficients
  int next;              // rows of ext per output: sum over digits of (ne - digit size)
  u64* accQ;             // [n][2][nl][N]       key products on the data primes, NTT domain
  u64* part;             // [n][alpha][2][N]    key products on the special primes so far, NTT domain
  u64* yP;               // [n][2][alpha][N]    ModDown inputs, coefficients
  u64* r;                // [n][2][N]           last prime of the key-switched sum, coefficients
  const u64* rlk;        // [dnum][2][nb][N]
  const u64* rlk_s;      // Shoup companions of rlk
  const ModUpConst* mu;  // [dnum] at this level
  const ModDownConst* md;
  const RescaleConst* rs;
  int lev, nl, n;
};

// row of ext holding digit j converted to extended-basis position e (e outside the digit)
__device__ __forceinline__ int ext_slot(const ModUpConst* mu, int ne, int j, int e) {
  int base = 0;
  for (int jj = 0; jj < j; ++jj) base += ne - (mu[jj].hi - mu[jj].lo);
  return base + (e < mu[j].lo ? e : e - (mu[j].hi - mu[j].lo));
}

template <typename Ar>
__device__ __forceinline__ void load_a(const Ar& ar, typename Ar::Val (&v)[32], const u64* row, int t) {
#pragma unroll
  for (int u = 0; u < 32; ++u) v[u] = ar.in(row[pos_a(t, u)]);
}
template <typename Ar>
__device__ __forceinline__ void load_c(const Ar& ar, typename Ar::Val (&v)[32], const u64* row, int t) {
#pragma unroll
  for (int r = 0; r < 32; ++r) v[r] = ar.in(row[pos_c(t, r)]);
}

// ---------------------------------------------------------------- K1
template <typename Ar>
__device__ __forceinline__ void k1_body(const Ks14Args& a, const DevParams& dp, int b, int i, void* lds) {
  typedef typename Ar::Val Val;
  const int t = threadIdx.x;
  const PrimeDev& P = dp.pr[i];
  const Ar ar(P, true);
  Val v[32];
  load_c(ar, v, a.D + (int64_t)b * a.dw + (int64_t)(2 * a.nl + i) * kN, t);
  n14::inverse(ar, v, reinterpret_cast<Val*>(lds), t);
  const ModUpConst& m = a.mu[i / dp.alpha];
  const u64 w = m.inv_n[i - m.lo], ws = m.inv_n_s[i - m.lo];
  u64* dst = a.y + ((int64_t)b * a.nl + i) * kN;
#pragma unroll
  for (int u = 0; u < 32; ++u) {
    dst[pos_a(t, u)] = ar.out_mul(v[u], w, ws);
    group_fence<8>(u);
  }
}

__global__ void __launch_bounds__(n14::kThreads, 4) ks14_k1_kernel(Ks14Args a, DevParams dp) {
  extern __shared__ u64 lds[];
  const int b = blockIdx.x / a.nl, i = blockIdx.x % a.nl;
  if (dp.pr[i].q < (1ull << 42))
    k1_body<NttFp>(a, dp, b, i, lds);
  else
    k1_body<NttInt>(a, dp, b, i, lds);
}

// ---------------------------------------------------------------- BConv
// Element-wise kernels take kEwPer positions per thread (strided by the
// block size), so that the per-block scalar set-up is amortised and each
// thread has kEwPer independent loads in flight.
constexpr int kEwThreads = 256, kEwPer = 8, kEwSpan = kEwThreads * kEwPer;

// grid (N / kEwSpan, n * next): block row (b, slot), slot enumerating
// (digit j, position e outside j) as ext_slot does
__global__ void __launch_bounds__(kEwThreads) ks14_bconv_kernel(Ks14Args a, DevParams dp) {
  const int x0 = blockIdx.x * kEwSpan + threadIdx.x;
  const int b = blockIdx.y / a.next, slot = blockIdx.y % a.next;
  const int ne = a.nl + dp.alpha;
  int j = 0, rem = slot;
  while (rem >= ne - (a.mu[j].hi - a.mu[j].lo)) {
    rem -= ne - (a.mu[j].hi - a.mu[j].lo);
    ++j;
  }
  const ModUpConst& mc = a.mu[j];
  const int e = rem < mc.lo ? rem : rem + (mc.hi - mc.lo);
  const u64 q = dp.pr[mc.basis[e]].q;
  const u64* yb = a.y + (int64_t)b * a.nl * kN + x0;
  u64 s[kEwPer], neg[kEwPer];   // centered conversion: residues above (q_i - 1) / 2 stand for y_i - q_i
#pragma unroll
  for (int m = 0; m < kEwPer; ++m) s[m] = neg[m] = 0;
  for (int i = mc.lo; i < mc.hi; ++i) {
    const u64 c = mc.conv[i - mc.lo][e], cs = mc.conv_s[i - mc.lo][e], h = (dp.pr[i].q - 1) / 2;
#pragma unroll
    for (int m = 0; m < kEwPer; ++m) {
      const u64 y = yb[(int64_t)i * kN + m * kEwThreads];
      s[m] = add_mod(s[m], mul_shoup(y, c, cs, q), q);
      neg[m] += y > h;
    }
  }
#pragma unroll
  for (int m = 0; m < kEwPer; ++m) s[m] = sub_mod(s[m], mul_shoup(neg[m], mc.dmod[e], mc.dmod_s[e], q), q);
  u64* o = a.ext + ((int64_t)b * a.next + slot) * kN + x0;
#pragma unroll
  for (int m = 0; m < kEwPer; ++m) o[m * kEwThreads] = s[m];
}

// ---------------------------------------------------------------- K2
// the key rows one digit multiplies: rlk_j,0[e] and its Shoup companions (the
// p = 1 rows are `next` words further), and the same for e's own digit
struct KeyRows {
  const u64 *k, *ks, *ok, *oks;
  int64_t next;
};

// key products of one transformed digit:
// s_p = X rlk_p (+ o_p unless FIRST) (+ d2_e rlk_own,p if OWN); s_1 goes to o1,
// s_0 to o0, or back into v for the inverse transform if KEEP0
template <bool FIRST, bool OWN, bool KEEP0, typename Ar>
__device__ __forceinline__ void k2_products(const Ar& ar, typename Ar::Val (&v)[32], const KeyRows& kr, const u64* d2e,
                                            u64* o0, u64* o1, u64 q, int t) {
  const int tt = after(t, v[15], v[31]);
#pragma unroll
  for (int r = 0; r < 32; ++r) {
    const int x = pos_c(tt, r);
    const u64 X = ar.fwd_res(v[r]);
    u64 s0 = mul_shoup(X, kr.k[x], kr.ks[x], q);
    u64 s1 = mul_shoup(X, kr.k[kr.next + x], kr.ks[kr.next + x], q);
    if (!FIRST) {
      s0 = add_mod(s0, o0[x], q);
      s1 = add_mod(s1, o1[x], q);
    }
    if (OWN) {
      const u64 d = d2e[x];
      s0 = add_mod(s0, mul_shoup(d, kr.ok[x], kr.oks[x], q), q);
      s1 = add_mod(s1, mul_shoup(d, kr.ok[kr.next + x], kr.oks[kr.next + x], q), q);
    }
    if (KEEP0) v[r] = ar.in(s0);
    else o0[x] = s0;
    o1[x] = s1;
    group_fence<4>(r);
  }
}

// a special prime's key products from two transformed digits: X0 (the first
// digit, stored in o0 by this thread at the same positions) and X1 (in v):
// s_p = X0 rlk_{j0},p + X1 rlk_{j1},p; s_0 stays in v for the inverse
// transform, s_1 goes to o1.  The two digits' partial sums never make a round
// trip through memory; only X0 does.
template <typename Ar>
__device__ __forceinline__ void k2_products_two(const Ar& ar, typename Ar::Val (&v)[32], const KeyRows& k0,
                                                const KeyRows& k1, const u64* x0, u64* o1, u64 q, int t) {
  const int tt = after(t, v[15], v[31]);
#pragma unroll
  for (int r = 0; r < 32; ++r) {
    const int x = pos_c(tt, r);
    const u64 X1 = ar.fwd_res(v[r]);
    const u64 X0 = x0[x];
    const u64 s0 = add_mod(mul_shoup(X0, k0.k[x], k0.ks[x], q), mul_shoup(X1, k1.k[x], k1.ks[x], q), q);
    const u64 s1 = add_mod(mul_shoup(X0, k0.k[k0.next + x], k0.ks[k0.next + x], q),
                           mul_shoup(X1, k1.k[k1.next + x], k1.ks[k1.next + x], q), q);
    v[r] = ar.in(s0);
    o1[x] = s1;
    group_fence<2>(r);
  }
}

// step IT of the digit loop of k2_body, unrolled at compile time
template <int IT, int NT, bool SPECIAL, typename Ar>
__device__ __forceinline__ void k2_steps(const Ar& ar, typename Ar::Val (&v)[32], typename Ar::Val* sh, const Ks14Args& a,
                                         const int (&js)[NT], int b, int e, int ne, int re, int nb, int64_t okrow,
                                         const u64* d2e, u64* o0, u64* o1, u64 q, int t) {
  if constexpr (IT < NT) {
    const int j = js[IT];
    load_a(ar, v, a.ext + ((int64_t)b * a.next + ext_slot(a.mu, ne, j, e)) * kN, t);
    n14::forward(ar, v, sh, t);
    const int64_t krow = ((int64_t)j * 2 * nb + re) * kN;   // rlk_j,0[re]; rlk_j,1[re] is nb rows further
    const KeyRows kr{a.rlk + krow, a.rlk_s + krow, a.rlk + okrow, a.rlk_s + okrow, (int64_t)nb * kN};
    k2_products<IT == 0, !SPECIAL && IT == NT - 1, SPECIAL && IT == NT - 1>(ar, v, kr, d2e, o0, o1, q, t);
    k2_steps<IT + 1, NT, SPECIAL>(ar, v, sh, a, js, b, e, ne, re, nb, okrow, d2e, o0, o1, q, t);
  }
}

// The NT digits needing a transform (those not holding prime e) are taken
// one at a time; each adds its key products into the destination rows (accQ
// for a data prime, part for a special one), the same words the same thread
// wrote before, so no synchronisation is needed.  The digit holding a data
// prime e needs no transform and is folded into the last pass.  For a special
// prime the last pass keeps acc_0 in registers for the inverse transform; with
// two digits the first digit's transformed row is kept instead of its two key
// products (one row written and read back instead of two), and both digits'
// products are formed in the second pass.  NT is a template argument so that
// no transform sits inside a run-time loop.
template <int NT, bool SPECIAL, typename Ar>
__device__ __forceinline__ void k2_body(const Ks14Args& a, const DevParams& dp, int b, int e, void* lds) {
  typedef typename Ar::Val Val;
  Val* sh = reinterpret_cast<Val*>(lds);
  const int t = threadIdx.x, nb = dp.nb, ne = a.nl + dp.alpha;
  const int re = a.mu[0].basis[e];
  const PrimeDev& P = dp.pr[re];
  const u64 q = P.q;
  const int k = e - a.nl;
  u64* o0 = SPECIAL ? a.part + (((int64_t)b * dp.alpha + k) * 2 + 0) * kN
                    : a.accQ + (((int64_t)b * 2 + 0) * a.nl + e) * kN;
  u64* o1 = SPECIAL ? a.part + (((int64_t)b * dp.alpha + k) * 2 + 1) * kN
                    : a.accQ + (((int64_t)b * 2 + 1) * a.nl + e) * kN;
  int js[NT];
  int own = 0, n = 0;
  for (int j = 0; j < dp.dnum; ++j) {
    const ModUpConst& mc = a.mu[j];
    if (mc.lo >= mc.hi) break;
    if (re >= mc.lo && re < mc.hi) own = j;
    else if (n < NT) js[n++] = j;
  }
  const int64_t okrow = ((int64_t)own * 2 * nb + re) * kN;
  const u64* d2e = a.D + (int64_t)b * a.dw + (int64_t)(2 * a.nl + (SPECIAL ? 0 : re)) * kN;
  const Ar ar(P, false);
  Val v[32];
  if constexpr (SPECIAL && NT == 2) {
    // the first digit's transform is kept (one row) until the second's is done
    load_a(ar, v, a.ext + ((int64_t)b * a.next + ext_slot(a.mu, ne, js[0], e)) * kN, t);
    n14::forward(ar, v, sh, t);
    {
      const int tt = after(t, v[15], v[31]);
#pragma unroll
      for (int r = 0; r < 32; ++r) {
        o0[pos_c(tt, r)] = ar.fwd_res(v[r]);
        group_fence<8>(r);
      }
    }
    load_a(ar, v, a.ext + ((int64_t)b * a.next + ext_slot(a.mu, ne, js[1], e)) * kN, t);
    n14::forward(ar, v, sh, t);
    const int64_t kr0 = ((int64_t)js[0] * 2 * nb + re) * kN, kr1 = ((int64_t)js[1] * 2 * nb + re) * kN;
    const KeyRows K0{a.rlk + kr0, a.rlk_s + kr0, nullptr, nullptr, (int64_t)nb * kN};
    const KeyRows K1{a.rlk + kr1, a.rlk_s + kr1, nullptr, nullptr, (int64_t)nb * kN};
    k2_products_two(ar, v, K0, K1, o0, o1, q, t);
  } else {
    k2_steps<0, NT, SPECIAL>(ar, v, sh, a, js, b, e, ne, re, nb, okrow, d2e, o0, o1, q, t);
  }
  if (!SPECIAL) return;
  // special prime p_k: both sums back to coefficients, times (P/p_k)^-1 N^-1
  const Ar ai(P, true);
  const u64 w = a.md->pinv_n[k], ws = a.md->pinv_n_s[k];
  n14::inverse(ai, v, sh, t);
  u64* y0 = a.yP + (((int64_t)b * 2 + 0) * dp.alpha + k) * kN;
#pragma unroll
  for (int u = 0; u < 32; ++u) {
    y0[pos_a(t, u)] = ai.out_mul(v[u], w, ws);
    group_fence<8>(u);
  }
  load_c(ai, v, o1, t);
  n14::inverse(ai, v, sh, t);
  u64* y1 = a.yP + (((int64_t)b * 2 + 1) * dp.alpha + k) * kN;
#pragma unroll
  for (int u = 0; u < 32; ++u) {
    y1[pos_a(t, u)] = ai.out_mul(v[u], w, ws);
    group_fence<8>(u);
  }
}

// Workgroups are dispatched to the 8 XCDs round robin (block i to XCD i mod
// 8), and each XCD has its own L2.  This maps block i to a work index so that
// each XCD takes one contiguous range of [0, G): consecutive work indices
// share their key rows, so an XCD's key working set stays within its L2.
__device__ __forceinline__ int xcd_range_index(int i, int G) {
  const int per = G >> 3, rem = G & 7, x = i & 7, s = i >> 3;
  return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + s;
}

// blocks (e, b), prime-major: e over the special primes (SPECIAL) or the
// data primes; every output b of one prime multiplies the same key rows
template <int NT, bool SPECIAL>
__global__ void __launch_bounds__(n14::kThreads, 4) ks14_k2_kernel(Ks14Args a, DevParams dp) {
  extern __shared__ u64 lds[];
  const int w = xcd_range_index(blockIdx.x, gridDim.x);
  const int f = w / a.n, b = w % a.n;
  const int e = SPECIAL ? a.nl + f : f;
  const int re = a.mu[0].basis[e];
  if (dp.pr[re].q < (1ull << 42))
    k2_body<NT, SPECIAL, NttFp>(a, dp, b, e, lds);
  else
    k2_body<NT, SPECIAL, NttInt>(a, dp, b, e, lds);
}

// a single digit holds every data prime: their key products need no transform
__global__ void __launch_bounds__(256) ks14_k2own_kernel(Ks14Args a, DevParams dp) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int b = blockIdx.y / a.nl, e = blockIdx.y % a.nl;
  const u64 q = dp.pr[e].q;
  const int64_t nbN = (int64_t)dp.nb * kN;
  const int64_t krow = (int64_t)e * kN + x;   // digit 0: rows rlk_0,p[e]
  const u64 d = a.D[(int64_t)b * a.dw + (int64_t)(2 * a.nl + e) * kN + x];
  a.accQ[(((int64_t)b * 2 + 0) * a.nl + e) * kN + x] = mul_shoup(d, a.rlk[krow], a.rlk_s[krow], q);
  a.accQ[(((int64_t)b * 2 + 1) * a.nl + e) * kN + x] = mul_shoup(d, a.rlk[krow + nbN], a.rlk_s[krow + nbN], q);
}

// ---------------------------------------------------------------- K3a
// z P^-1 mod q_i at one position (yb = yP rows of (b, p) at it), z = sum_k
// yP_k [P/p_k]_{q_i} with yP_k centered: the uncentered sum with P^-1 folded
// into the constants, minus the count of yP_k above (p_k - 1) / 2 (each such
// term stands for yP_k - p_k, and p_k [P/p_k] P^-1 = 1)
template <int ALPHA>
__device__ __forceinline__ u64 moddown_zp(const u64* yb, const ModDownConst* md, int i, u64 q, const DevParams& dp) {
  u64 z = 0, neg = 0;
#pragma unroll
  for (int k = 0; k < ALPHA; ++k) {
    const u64 y = yb[(int64_t)k * kN];
    z = add_mod(z, mul_shoup(y, md->convp[k][i], md->convp_s[k][i], q), q);
    neg += y > (dp.pr[dp.L + k].q - 1) / 2;
  }
  return sub_mod(z, neg, q);
}

// K3a's epilogue for register U and the ones after it, unrolled at compile
// time (a loop of this length is not always unrolled, and a run-time index
// would put v in scratch)
template <int U, int ALPHA, typename Ar>
__device__ __forceinline__ void k3a_out(const Ar& ar, const typename Ar::Val (&v)[32], const u64* yb, u64* o,
                                        const ModDownConst* md, int lev, const PrimeDev& P, const DevParams& dp, int tt) {
  if constexpr (U < 32) {
    const int x = pos_a(tt, U);
    const u64 z = moddown_zp<ALPHA>(yb + x, md, lev, P.q, dp);
    o[x] = sub_mod(ar.out_inv(v[U], P), z, P.q);
    group_fence<4>(U);
    k3a_out<U + 1, ALPHA>(ar, v, yb, o, md, lev, P, dp, tt);
  }
}

// instantiated per alpha: a run-time trip count inside the unrolled
// per-register code would keep the row's addresses live
template <int ALPHA, typename Ar>
__device__ __forceinline__ void k3a_body(const Ks14Args& a, const DevParams& dp, int b, int p, void* lds) {
  typedef typename Ar::Val Val;
  const int t = threadIdx.x, lev = a.lev;
  const PrimeDev& P = dp.pr[lev];
  const u64 q = P.q;
  const Ar ar(P, true);
  const u64 Pi = a.md->Pinv[lev], Pis = a.md->Pinv_s[lev];
  const u64* acc = a.accQ + (((int64_t)b * 2 + p) * a.nl + lev) * kN;
  const u64* d = a.D + (int64_t)b * a.dw + (int64_t)(p * a.nl + lev) * kN;
  Val v[32];
#pragma unroll
  for (int r = 0; r < 32; ++r) {
    const int x = pos_c(t, r);
    v[r] = ar.in(add_mod(mul_shoup(acc[x], Pi, Pis, q), d[x], q));
    group_fence<8>(r);
  }
  n14::inverse(ar, v, reinterpret_cast<Val*>(lds), t);
  const int tt = after(t, v[15], v[31]);
  u64* o = a.r + ((int64_t)b * 2 + p) * kN;
  const u64* yb = a.yP + ((int64_t)b * 2 + p) * ALPHA * kN;
  k3a_out<0, ALPHA>(ar, v, yb, o, a.md, lev, P, dp, tt);
}

template <int ALPHA>
__global__ void __launch_bounds__(n14::kThreads, 4) ks14_k3a_kernel(Ks14Args a, DevParams dp) {
  extern __shared__ u64 lds[];
  const int b = blockIdx.x >> 1, p = blockIdx.x & 1;
  if (dp.pr[a.lev].q < (1ull << 42))
    k3a_body<ALPHA, NttFp>(a, dp, b, p, lds);
  else
    k3a_body<ALPHA, NttInt>(a, dp, b, p, lds);
}

// ---------------------------------------------------------------- Lift
// w_i at the positions pos_a(t, u) of thread t, taken while K3b loads its
// row: z_i P^-1, plus the centered last prime r reduced mod q_i with the
// rescale (RS).  The lift reads the same ALPHA + 1 coefficient rows of (b, p)
// for every target prime i; K3b's blocks of one (b, p) run back to back on
// one XCD, so those rows come from its L2 after the first block.
template <int ALPHA>
struct LiftConsts {
  const u64 *yb, *rb;            // yP rows and r row of (b, p)
  u64 q, ql, mu_hi, mu_lo;
  u64 cv[ALPHA], cs[ALPHA], ph[ALPHA];   // [P/p_k]_{q_i} P^-1 with companions; (p_k - 1) / 2
};

template <int ALPHA, bool RS>
__device__ __forceinline__ u64 lift_one(const LiftConsts<ALPHA>& lc, int x) {
  const u64 q = lc.q;
  u64 z = 0, above = 0;   // centered conversion: residues above (p_k - 1) / 2 stand for y - p_k
#pragma unroll
  for (int k = 0; k < ALPHA; ++k) {
    const u64 y = lc.yb[(int64_t)k * kN + x];
    z = add_mod(z, mul_shoup(y, lc.cv[k], lc.cs[k], q), q);
    above += y > lc.ph[k];
  }
  u64 w = sub_mod(z, above, q);
  if (RS) {   // centered lift of the last prime, reduced mod q_i
    const u64 c = lc.rb[x];
    const bool neg = c > (lc.ql - 1) / 2;
    const u64 mag = neg ? lc.ql - c : c;
    u64 r = reduce_wide(U128{mag, 0}, q, lc.mu_hi, lc.mu_lo);
    r = (neg && r) ? q - r : r;
    w = add_mod(w, r, q);
  }
  return w;
}

// register U and the ones after it, unrolled at compile time (a loop this
// long is not always unrolled, and a run-time index would put v in scratch)
template <int U, int ALPHA, bool RS, typename Ar>
__device__ __forceinline__ void lift_steps(const Ar& ar, typename Ar::Val (&v)[32], const LiftConsts<ALPHA>& lc, int t) {
  if constexpr (U < 32) {
    v[U] = ar.in(lift_one<ALPHA, RS>(lc, pos_a(t, U)));
    group_fence<4>(U);
    lift_steps<U + 1, ALPHA, RS>(ar, v, lc, t);
  }
}

template <int ALPHA, bool RS, typename Ar>
__device__ __forceinline__ void load_lift(const Ar& ar, typename Ar::Val (&v)[32], const Ks14Args& a,
                                          const DevParams& dp, int bp, int i, int t) {
  LiftConsts<ALPHA> lc;
  const PrimeDev& P = dp.pr[i];
  lc.yb = a.yP + (int64_t)bp * ALPHA * kN;
  lc.rb = a.r + (int64_t)bp * kN;
  lc.q = P.q;
  lc.ql = dp.pr[a.lev].q;
  lc.mu_hi = P.mu_hi;
  lc.mu_lo = P.mu_lo;
#pragma unroll
  for (int k = 0; k < ALPHA; ++k) {
    lc.cv[k] = a.md->convp[k][i];
    lc.cs[k] = a.md->convp_s[k][i];
    lc.ph[k] = (dp.pr[dp.L + k].q - 1) / 2;
  }
  lift_steps<0, ALPHA, RS>(ar, v, lc, t);
}

// ---------------------------------------------------------------- K3b
// RS: C_i = (acc_i P^-1 + d_i - NTT(w_i)) q_lev^-1 for i < lev; else the
// key-switched sum itself, acc_i P^-1 + d_i - NTT(w_i) for i <= lev (limb-major
// output rows only)
template <int ALPHA, typename Ar, bool RS>
__device__ __forceinline__ void k3b_body(const Ks14Args& a, const DevParams& dp, const OutLayout& ol, int b, int p, int i,
                                         void* lds) {
  typedef typename Ar::Val Val;
  const int t = threadIdx.x, lev = a.lev;
  const PrimeDev& P = dp.pr[i];
  const u64 q = P.q;
  const Ar ar(P, false);
  const u64 Pi = a.md->Pinv[i], Pis = a.md->Pinv_s[i];
  Val v[32];
  const int rows = RS ? lev : lev + 1;
  load_lift<ALPHA, RS>(ar, v, a, dp, b * 2 + p, i, t);
  n14::forward(ar, v, reinterpret_cast<Val*>(lds), t);
  const u64* acc = a.accQ + (((int64_t)b * 2 + p) * a.nl + i) * kN;
  const u64* d = a.D + (int64_t)b * a.dw + (int64_t)(p * a.nl + i) * kN;
  const u64 qi = a.rs->qinv[i], qis = a.rs->qinv_s[i];
  const int tt = after(t, v[15], v[31]);
  if (!RS) {
    u64* dst = ol.base + (int64_t)b * ol.stride + ((int64_t)p * rows + i) * kN;
#pragma unroll
    for (int r = 0; r < 32; ++r) {
      const int x = pos_c(tt, r);
      dst[x] = sub_mod(add_mod(mul_shoup(acc[x], Pi, Pis, q), d[x], q), ar.fwd_res(v[r]), q);
      group_fence<4>(r);
    }
    return;
  }
  // the two destination layouts in loops of their own (a select of the
  // address inside one loop spills registers)
  if (ol.chunked) {
#pragma unroll
    for (int r = 0; r < 32; ++r) {
      const int x = pos_c(tt, r);
      const u64 s = sub_mod(add_mod(mul_shoup(acc[x], Pi, Pis, q), d[x], q), ar.fwd_res(v[r]), q);
      ol.base[chunk_index(ol.elem_base + b, p, i, x, ol.n_ct, kN >> 6)] = mul_shoup(s, qi, qis, q);
      group_fence<4>(r);
    }
  } else {
    u64* dst = ol.base + (int64_t)b * ol.stride + ((int64_t)p * lev + i) * kN;
#pragma unroll
    for (int r = 0; r < 32; ++r) {
      const int x = pos_c(tt, r);
      const u64 s = sub_mod(add_mod(mul_shoup(acc[x], Pi, Pis, q), d[x], q), ar.fwd_res(v[r]), q);
      dst[x] = mul_shoup(s, qi, qis, q);
      group_fence<4>(r);
    }
  }
}

// blocks (b, p, i), i fastest, in XCD ranges: the target primes of one
// (b, p) share the lift's source rows through one L2
template <int ALPHA, bool RS>
__global__ void __launch_bounds__(n14::kThreads, 4) ks14_k3b_kernel(Ks14Args a, OutLayout ol, DevParams dp) {
  extern __shared__ u64 lds[];
  const int rows = RS ? a.lev : a.lev + 1;
  const int w = xcd_range_index(blockIdx.x, gridDim.x);
  const int b = w / (2 * rows);
  const int rem = w % (2 * rows);
  const int p = rem / rows, i = rem % rows;
  if (dp.pr[i].q < (1ull << 42))
    k3b_body<ALPHA, NttFp, RS>(a, dp, ol, b, p, i, lds);
  else
    k3b_body<ALPHA, NttInt, RS>(a, dp, ol, b, p, i, lds);
}

template <int NT>
int launch_k2(const sfhe_ctx* c, const Ks14Args& a, int64_t n, size_t lds, hipStream_t s) {
  constexpr int NTD = NT > 1 ? NT - 1 : 1;   // transforms per data prime
  static bool attr = false;
  if (!attr) {
    SFHE_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&ks14_k2_kernel<NT, true>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    SFHE_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&ks14_k2_kernel<NTD, false>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = true;
  }
  const dim3 blk(n14::kThreads);
  hipLaunchKernelGGL((ks14_k2_kernel<NT, true>), dim3((unsigned)(n * c->alpha)), blk, lds, s, a, c->dp);
  SFHE_HIP(hipGetLastError());
  if (NT > 1)
    hipLaunchKernelGGL((ks14_k2_kernel<NTD, false>), dim3((unsigned)(n * a.nl)), blk, lds, s, a, c->dp);
  else
    hipLaunchKernelGGL(ks14_k2own_kernel, dim3(kN / 256, (unsigned)(n * a.nl)), dim3(256), 0, s, a, c->dp);
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

template <int ALPHA>
int launch_ks14(sfhe_ctx* c, const Ks14Args& a, int ndig, OutLayout out, int64_t n, bool rescale, hipStream_t s) {
  const size_t lds = (size_t)n14::kLdsWords * sizeof(u64);
  static bool attr = false;
  if (!attr) {
    const void* fns[4] = {reinterpret_cast<const void*>(&ks14_k1_kernel),
                          reinterpret_cast<const void*>(&ks14_k3a_kernel<ALPHA>),
                          reinterpret_cast<const void*>(&ks14_k3b_kernel<ALPHA, true>),
                          reinterpret_cast<const void*>(&ks14_k3b_kernel<ALPHA, false>)};
    for (const void* f : fns) SFHE_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = true;
  }
  const int lev = a.lev, nl = a.nl;
  const dim3 blk(n14::kThreads);
  hipLaunchKernelGGL(ks14_k1_kernel, dim3((unsigned)(n * nl)), blk, lds, s, a, c->dp);
  SFHE_HIP(hipGetLastError());
  hipLaunchKernelGGL(ks14_bconv_kernel, dim3(kN / kEwSpan, (unsigned)(n * a.next)), dim3(kEwThreads), 0, s, a, c->dp);
  SFHE_HIP(hipGetLastError());
  int rc;
  switch (ndig) {
    case 1: rc = launch_k2<1>(c, a, n, lds, s); break;
    case 2: rc = launch_k2<2>(c, a, n, lds, s); break;
    case 3: rc = launch_k2<3>(c, a, n, lds, s); break;
    default: rc = launch_k2<4>(c, a, n, lds, s); break;
  }
  if (rc) return rc;
  if (!rescale) {   // the key-switched sum itself: no last-prime transform
    hipLaunchKernelGGL((ks14_k3b_kernel<ALPHA, false>), dim3((unsigned)(n * 2 * nl)), blk, lds, s, a, out, c->dp);
    SFHE_HIP(hipGetLastError());
    return SFHE_OK;
  }
  hipLaunchKernelGGL(ks14_k3a_kernel<ALPHA>, dim3((unsigned)(n * 2)), blk, lds, s, a, c->dp);
  SFHE_HIP(hipGetLastError());
  hipLaunchKernelGGL((ks14_k3b_kernel<ALPHA, true>), dim3((unsigned)(n * 2 * lev)), blk, lds, s, a, out, c->dp);
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

// ---------------------------------------------------------------- rescale alone
// The rescale of degree-1 sums that need no key switch (plaintext weights
// times encrypted values): RS-A (b, p) r = iNTT(d_lev), the last prime in
// coefficients; RS-B (b, p, i), i < lev: C_i = (d_i - NTT([centered r]_{q_i}))
// q_lev^-1, the lift taken while the row is loaded.
struct Rs14Args {
  const u64* D;          // [n] x dw words: d0, d1 rows of nl primes (NTT domain)
  int64_t dw;
  u64* r;                // [n][2][N] last prime in coefficients
  const RescaleConst* rs;
  int lev, nl;
};

template <typename Ar>
__device__ __forceinline__ void rsa_body(const Rs14Args& a, const DevParams& dp, int b, int p, void* lds) {
  typedef typename Ar::Val Val;
  const int t = threadIdx.x;
  const PrimeDev& P = dp.pr[a.lev];
  const Ar ar(P, true);
  Val v[32];
  load_c(ar, v, a.D + (int64_t)b * a.dw + (int64_t)(p * a.nl + a.lev) * kN, t);
  n14::inverse(ar, v, reinterpret_cast<Val*>(lds), t);
  u64* o = a.r + ((int64_t)b * 2 + p) * kN;
#pragma unroll
  for (int u = 0; u < 32; ++u) {
    o[pos_a(t, u)] = ar.out_inv(v[u], P);
    group_fence<8>(u);
  }
}

__global__ void __launch_bounds__(n14::kThreads, 4) rs14_a_kernel(Rs14Args a, DevParams dp) {
  extern __shared__ u64 lds[];
  const int b = blockIdx.x >> 1, p = blockIdx.x & 1;
  if (dp.pr[a.lev].q < (1ull << 42))
    rsa_body<NttFp>(a, dp, b, p, lds);
  else
    rsa_body<NttInt>(a, dp, b, p, lds);
}

template <typename Ar>
__device__ __forceinline__ void rsb_body(const Rs14Args& a, const DevParams& dp, const OutLayout& ol, int b, int p, int i,
                                         void* lds) {
  typedef typename Ar::Val Val;
  const int t = threadIdx.x, lev = a.lev;
  const PrimeDev& P = dp.pr[i];
  const u64 q = P.q, ql = dp.pr[lev].q;
  const Ar ar(P, false);
  const u64* rr = a.r + ((int64_t)b * 2 + p) * kN;
  Val v[32];
#pragma unroll
  for (int u = 0; u < 32; ++u) {
    // centered lift of the last prime, reduced mod q_i
    const u64 c = rr[pos_a(t, u)];
    const bool neg = c > (ql - 1) / 2;
    const u64 mag = neg ? ql - c : c;
    u64 x = mag < q ? mag : reduce_wide(U128{mag, 0}, q, P.mu_hi, P.mu_lo);
    x = (neg && x) ? q - x : x;
    v[u] = ar.in(x);
  }
  n14::forward(ar, v, reinterpret_cast<Val*>(lds), t);
  const u64* d = a.D + (int64_t)b * a.dw + (int64_t)(p * a.nl + i) * kN;
  const u64 qi = a.rs->qinv[i], qis = a.rs->qinv_s[i];
  const int tt = after(t, v[15], v[31]);
  if (ol.chunked) {
#pragma unroll
    for (int r = 0; r < 32; ++r) {
      const int x = pos_c(tt, r);
      ol.base[chunk_index(ol.elem_base + b, p, i, x, ol.n_ct, kN >> 6)] = mul_shoup(sub_mod(d[x], ar.fwd_res(v[r]), q), qi, qis, q);
      group_fence<4>(r);
    }
  } else {
    u64* dst = ol.base + (int64_t)b * ol.stride + ((int64_t)p * lev + i) * kN;
#pragma unroll
    for (int r = 0; r < 32; ++r) {
      const int x = pos_c(tt, r);
      dst[x] = mul_shoup(sub_mod(d[x], ar.fwd_res(v[r]), q), qi, qis, q);
      group_fence<4>(r);
    }
  }
}

__global__ void __launch_bounds__(n14::kThreads, 4) rs14_b_kernel(Rs14Args a, OutLayout ol, DevParams dp) {
  extern __shared__ u64 lds[];
  const int lev = a.lev;
  const int b = blockIdx.x / (2 * lev);
  const int rem = blockIdx.x % (2 * lev);
  const int p = rem / lev, i = rem % lev;
  if (dp.pr[i].q < (1ull << 42))
    rsb_body<NttFp>(a, dp, ol, b, p, i, lds);
  else
    rsb_body<NttInt>(a, dp, ol, b, p, i, lds);
}

}  // namespace

bool keyswitch_rescale_n14_supported(const sfhe_ctx* c) {
  return c->logN == n14::kLogN && c->alpha >= 1 && c->alpha <= 4 && c->dnum <= 4;
}

int rescale_n14(sfhe_ctx* c, int lev, const u64* D, int64_t dw, OutLayout out, int64_t n, hipStream_t s, u64* scratch) {
  if (n <= 0) return SFHE_OK;
  if (c->logN != n14::kLogN) { set_error("rescale_n14: N = 2^14 only"); return SFHE_E_INVALID_ARG; }
  if (lev < 1) { set_error("rescale: level 0 has no prime to drop"); return SFHE_E_LEVEL; }
  if (n * 2 * lev > 0x7FFFFFFF) { set_error("rescale: batch too large"); return SFHE_E_INVALID_ARG; }
  const size_t lds = (size_t)n14::kLdsWords * sizeof(u64);
  static bool attr = false;
  if (!attr) {
    SFHE_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&rs14_a_kernel),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    SFHE_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&rs14_b_kernel),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = true;
  }
  DevBuf<u64> r;
  if (!scratch && !r.alloc(&c->alloc, (size_t)n * 2 * kN)) { set_error("rescale: device allocation failed"); return SFHE_E_NOMEM; }
  Rs14Args a{D, dw, scratch ? scratch : r.ptr, c->d_rescale.ptr + lev, lev, lev + 1};
  const dim3 blk(n14::kThreads);
  hipLaunchKernelGGL(rs14_a_kernel, dim3((unsigned)(n * 2)), blk, lds, s, a, c->dp);
  SFHE_HIP(hipGetLastError());
  hipLaunchKernelGGL(rs14_b_kernel, dim3((unsigned)(n * 2 * lev)), blk, lds, s, a, out, c->dp);
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

// rows of each working buffer per output, in allocation order: y, ext,
// accQ, part, yP, r
static void ks14_rows(const sfhe_ctx* c, int lev, bool rescale, int64_t rows[6]) {
  const int nl = lev + 1, ne = nl + c->alpha;
  int next = 0;
  for (int j = 0; j < c->dnum; ++j) {
    const int lo = j * c->alpha, hi = std::min((j + 1) * c->alpha, nl);
    if (lo >= hi) break;
    next += ne - (hi - lo);
  }
  rows[0] = nl;
  rows[1] = next;
  rows[2] = 2 * nl;
  rows[3] = 2 * c->alpha;
  rows[4] = 2 * c->alpha;
  rows[5] = rescale ? 2 : 0;
}

int64_t keyswitch_rescale_n14_scratch_words(const sfhe_ctx* c, int lev, int64_t n) {
  int64_t rows[6], t = 0;
  ks14_rows(c, lev, true, rows);
  for (int x = 0; x < 6; ++x) t += rows[x];
  return t * n * kN;
}

static int ks14_run(sfhe_ctx* c, int lev, const u64* D, int64_t dw, OutLayout out, int64_t n, const u64* key,
                    const u64* key_s, bool rescale, hipStream_t s, u64* scratch = nullptr) {
  if (n <= 0) return SFHE_OK;
  if (!keyswitch_rescale_n14_supported(c)) {
    set_error("fused key switch: N = 2^14, 1 <= alpha <= 4 and dnum <= 4 only");
    return SFHE_E_INVALID_ARG;
  }
  if (rescale && lev < 1) { set_error("rescale: level 0 has no prime to drop"); return SFHE_E_LEVEL; }
  if (!rescale && out.chunked) { set_error("key switch: limb-major output only"); return SFHE_E_INVALID_ARG; }
  if (!key || !key_s) { set_error("keygen first"); return SFHE_E_STATE; }
  const int nl = lev + 1, ne = nl + c->alpha;
  int next = 0, ndig = 0;
  for (int j = 0; j < c->dnum; ++j) {
    const int lo = j * c->alpha, hi = std::min((j + 1) * c->alpha, nl);
    if (lo >= hi) break;
    next += ne - (hi - lo);
    ++ndig;
  }
  // grid limits of the element-wise kernels (rows in y)
  if (n * ne > 0x7FFFFFFF || n * std::max(std::max(next, 2 * nl), nl) > 65535) {
    set_error("key switch: slice too large");
    return SFHE_E_INVALID_ARG;
  }
  // working rows: from the caller's scratch (ks14_rows order), else allocated
  int64_t rows[6];
  ks14_rows(c, lev, rescale, rows);
  DevBuf<u64> bufs[6];
  u64* ptr[6];
  for (int x = 0; x < 6; ++x) {
    if (scratch) {
      ptr[x] = scratch;
      scratch += (size_t)n * rows[x] * kN;
    } else {
      if (!bufs[x].alloc(&c->alloc, (size_t)n * rows[x] * kN)) {
        set_error("key switch: device allocation failed");
        return SFHE_E_NOMEM;
      }
      ptr[x] = bufs[x].ptr;
    }
  }
  Ks14Args a;
  a.D = D;
  a.dw = dw;
  a.y = ptr[0];
  a.ext = ptr[1];
  a.next = next;
  a.accQ = ptr[2];
  a.part = ptr[3];
  a.yP = ptr[4];
  a.r = ptr[5];
  a.rlk = key;
  a.rlk_s = key_s;
  a.mu = c->d_modup.ptr + (size_t)lev * c->dnum;
  a.md = c->d_moddown.ptr + lev;
  a.rs = c->d_rescale.ptr + lev;
  a.lev = lev;
  a.nl = nl;
  a.n = (int)n;
  switch (c->alpha) {
    case 1: return launch_ks14<1>(c, a, ndig, out, n, rescale, s);
    case 2: return launch_ks14<2>(c, a, ndig, out, n, rescale, s);
    case 3: return launch_ks14<3>(c, a, ndig, out, n, rescale, s);
    default: return launch_ks14<4>(c, a, ndig, out, n, rescale, s);
  }
}

int keyswitch_rescale_n14(sfhe_ctx* c, int lev, const u64* D, int64_t dw, OutLayout out, int64_t n, hipStream_t s,
                          u64* scratch) {
  return ks14_run(c, lev, D, dw, out, n, c->d_rlk.ptr, c->d_rlk_s.ptr, true, s, scratch);
}

int keyswitch_n14(sfhe_ctx* c, int lev, const u64* D, int64_t dw, OutLayout out, int64_t n, const u64* key,
                  const u64* key_s, hipStream_t s) {
  return ks14_run(c, lev, D, dw, out, n, key, key_s, false, s);
}

}  // namespace sfhe
