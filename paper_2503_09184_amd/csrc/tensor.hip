// tensor.hip -- ciphertext tensor products in the NTT domain (the multiply
// step of Algorithm 1): d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1 per prime
// and coefficient, one product at a time (per-product form) or summed over
// every visited k of an output before any reduction (lazy form).
#include "fparith.hpp"

namespace sfhe {

// d[p][l][t] for `batch` pairs, strides in words
__global__ void tensor_pointwise_kernel(int nl, const u64* a, int64_t as, const u64* b, int64_t bs, u64* d,
                                        int64_t ds, int64_t batch, DevParams dp) {
  const int N = dp.N;
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;   // (x, l)
  if (row >= batch * nl) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t x = row / nl;
  const int l = (int)(row % nl);
  const PrimeDev& P = dp.pr[l];
  const u64* ax = a + x * as;
  const u64* bx = b + x * bs;
  const u64 a0 = ax[(int64_t)l * N + t], a1 = ax[(int64_t)(nl + l) * N + t];
  const u64 b0 = bx[(int64_t)l * N + t], b1 = bx[(int64_t)(nl + l) * N + t];
  U128 m = mul_wide(a0, b1);
  add_wide(m, mul_wide(a1, b0));
  u64* dx = d + x * ds;
  dx[(int64_t)l * N + t] = mul_mod(a0, b0, P);
  dx[(int64_t)(nl + l) * N + t] = reduce_wide(m, P.q, P.mu_hi, P.mu_lo);
  dx[(int64_t)(2 * nl + l) * N + t] = mul_mod(a1, b1, P);
}

// gathered: product x multiplies A ciphertext aidx[x] by B ciphertext bidx[x]
// (chunked matrices, top level, L primes); d limb-major
__global__ void tensor_gather_kernel(int nl, const u64* A, int64_t nA, const u64* B, int64_t nB, const int* aidx,
                                     const int* bidx, u64* d, int64_t count, DevParams dp) {
  const int N = dp.N;
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;
  if (row >= count * nl) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t x = row / nl;
  const int l = (int)(row % nl);
  const PrimeDev& P = dp.pr[l];
  const int C = N >> 6;
  const u64 a0 = A[chunk_index(aidx[x], 0, l, t, nA, C)], a1 = A[chunk_index(aidx[x], 1, l, t, nA, C)];
  const u64 b0 = B[chunk_index(bidx[x], 0, l, t, nB, C)], b1 = B[chunk_index(bidx[x], 1, l, t, nB, C)];
  U128 m = mul_wide(a0, b1);
  add_wide(m, mul_wide(a1, b0));
  u64* dx = d + x * (int64_t)3 * nl * N;
  dx[(int64_t)l * N + t] = mul_mod(a0, b0, P);
  dx[(int64_t)(nl + l) * N + t] = reduce_wide(m, P.q, P.mu_hi, P.mu_lo);
  dx[(int64_t)(2 * nl + l) * N + t] = mul_mod(a1, b1, P);
}

// ---- lazy sums over a row tile's visited k ----
// The host turns the left operand's plaintext structure (Sec. 3.3.2: every k
// for naive dense, the unmasked k for naive sparse, the CSR column list, the
// ELLPACK columns other than -1) into, for each tile of kTileRows consecutive
// output rows, the ascending union of their visited k with a bit mask of the
// rows that visit it and each such row's A ciphertext slot.  Mask tests are
// uniform across a wavefront, so a zero of A costs no multiply.
//
// Block order is XCD-aware: consecutive blocks go to the 8 XCDs in turn, so
// block b takes 64-coefficient chunk (b mod 8) of a 512-coefficient slab; a
// slab's A and B stay resident in the Infinity Cache while every output tile
// of the slab is computed, and each XCD's L2 sees one 64-coefficient chunk.

constexpr int kWavesPerBlock = 8;
constexpr int kSegEntries = 128;   // tile entries held in LDS at a time
static_assert(kTileRows == 2 * kWavesPerBlock, "each wave of the block kernel stages two tile rows");

struct ArithFp {   // q < 2^42: fp64 residues, Karatsuba middle term
  typedef double Val;
  static constexpr bool kSum = true;   // uses a0 + a1 (Karatsuba)
  struct Acc {
    double d0, d2, ss;   // sums of a0 b0, a1 b1, (a0 + a1)(b0 + b1)
  };
  double q, qinv;
  __device__ ArithFp(const FpLimb& F, const PrimeDev&) : q(F.q), qinv(F.qinv) {}
  __device__ static Val load(u64 x) { return u52_to_f64(x); }   // x < q < 2^42
  __device__ static void zero(Acc& a) { a.d0 = a.d2 = a.ss = 0.0; }
  __device__ static Val sum(Val x, Val y) { return x + y; }
  __device__ void mac(Acc& a, Val a0, Val a1, Val as, Val b0, Val b1, Val bs) const {
    a.d0 += fp_mulmod_lazy(a0, b0, q, qinv);
    a.d2 += fp_mulmod_lazy(a1, b1, q, qinv);
    a.ss += fp_mulmod_lazy(as, bs, q, qinv);
  }
  static constexpr int kFold = 1024;   // each product adds < 1.5 q to a sum: stay below 2^53
  static constexpr int kGroup = 4;     // rows whose operands are read from LDS together
  __device__ void fold(Acc& a, int = 0) const {
    a.d0 = fp_fold(a.d0, q, qinv);
    a.d2 = fp_fold(a.d2, q, qinv);
    a.ss = fp_fold(a.ss, q, qinv);
  }
  // d1 = (a0 + a1)(b0 + b1) - a0 b0 - a1 b1, formed once per output
  __device__ void final(const Acc& a, u64& d0, u64& d1, u64& d2) const {
    const double x0 = fp_fold(a.d0, q, qinv), x2 = fp_fold(a.d2, q, qinv);
    const double x1 = fp_fold(a.ss, q, qinv) - x0 - x2;
    d0 = fp_final(x0, q, qinv);
    d1 = fp_final(x1, q, qinv);
    d2 = fp_final(x2, q, qinv);
  }
};

// a*b added to a 128-bit sum, for a, b < 2^62: four 32x32 -> 64 multiply-adds
// (the high halves are below 2^30, so every partial sum stays below 2^64)
__device__ __forceinline__ void mac_wide(U128& acc, u64 a, u64 b) {
  const u32 a0 = (u32)a, a1 = (u32)(a >> 32), b0 = (u32)b, b1 = (u32)(b >> 32);
  const u64 p00 = (u64)a0 * b0;
  const u64 t = (u64)a1 * b0 + ((u64)a0 * b1 + (p00 >> 32));
  const u64 lo = (t << 32) | (p00 & 0xffffffffull);
  const u64 hi = (u64)a1 * b1 + (t >> 32);
  add_wide(acc, U128{lo, hi});
}

struct ArithInt {   // q < 2^61: 128-bit integer sums, Karatsuba middle term
  typedef u64 Val;
  static constexpr bool kSum = true;
  struct Acc {
    U128 d0, d2, ss;   // sums of a0 b0, a1 b1, (a0 + a1)(b0 + b1)
  };
  u64 q, mu_hi, mu_lo;
  __device__ ArithInt(const FpLimb&, const PrimeDev& P) : q(P.q), mu_hi(P.mu_hi), mu_lo(P.mu_lo) {}
  __device__ static Val load(u64 x) { return x; }
  __device__ static void zero(Acc& a) { a.d0 = a.d2 = a.ss = U128{0, 0}; }
  __device__ static Val sum(Val x, Val y) { return x + y; }   // < 2^62
  __device__ void mac(Acc& a, Val a0, Val a1, Val as, Val b0, Val b1, Val bs) const {
    mac_wide(a.d0, a0, b0);
    mac_wide(a.d2, a1, b1);
    mac_wide(a.ss, as, bs);
  }
  static constexpr int kFold = 16;     // 16 terms below 2^124 (plus a residue) stay below 2^128
  static constexpr int kGroup = 4;
  __device__ void fold(Acc& a, int = 0) const {
    a.d0 = U128{reduce_wide(a.d0, q, mu_hi, mu_lo), 0};
    a.d2 = U128{reduce_wide(a.d2, q, mu_hi, mu_lo), 0};
    a.ss = U128{reduce_wide(a.ss, q, mu_hi, mu_lo), 0};
  }
  // d1 = (a0 + a1)(b0 + b1) - a0 b0 - a1 b1, formed once per output
  __device__ void final(const Acc& a, u64& d0, u64& d1, u64& d2) const {
    d0 = reduce_wide(a.d0, q, mu_hi, mu_lo);
    d2 = reduce_wide(a.d2, q, mu_hi, mu_lo);
    d1 = sub_mod(sub_mod(reduce_wide(a.ss, q, mu_hi, mu_lo), d0, q), d2, q);
  }
};

// Primes q = 2^60 - c with c < 2^20 (the largest NTT primes below 2^60):
// carry-save sums without Karatsuba.  An operand x < 2^60 is staged as its
// 30-bit halves (xl, xh) in the two 32-bit words of a u64, and a product x y
// adds its partials xl yl, xl yh + xh yl, xh yh (each below 2^60) to sums L,
// M, H of weights 1, 2^30, 2^60 with one v_mad_u64_u32 each: 16 per
// ciphertext product, no carries.  Every kFold entries the sums are folded
// back: carries move up (L into M, M into H), and since 2^60 = c (mod q),
// H 2^60 = (H mod 2^32) c + t 2^32 with t = (H >> 32) c < 2^52, of which
// (H mod 2^32) c goes into L, (t mod 2^28) 4 into M and t >> 28 stays in H.
// Afterwards L < 2^53, M < 2^31, H < 2^24.  An entry adds at most 4 partials
// below 2^60 - 2^31 to a sum of d1 (two products) and at most 2 to one of d0
// or d2, so d1 is folded every kFold = 4 entries and d0, d2 every 8: no sum
// takes more than 16 partials between folds, and every sum stays below 2^64.
__device__ __forceinline__ u32 lo32(u64 x) { return (u32)x; }
__device__ __forceinline__ u32 hi32(u64 x) { return (u32)(x >> 32); }
__device__ __forceinline__ u64 madw(u32 a, u32 b, u64 acc) { return (u64)a * b + acc; }

struct ArithInt60 {
  typedef u64 Val;   // (x mod 2^30) | (x >> 30) << 32
  static constexpr bool kSum = false;
  struct Sums {
    u64 L, M, H;
  };
  struct Acc {
    Sums d0, d1, d2;
  };
  u64 q, mu_hi, mu_lo;
  u32 c;   // 2^60 - q
  __device__ ArithInt60(const FpLimb&, const PrimeDev& P)
      : q(P.q), mu_hi(P.mu_hi), mu_lo(P.mu_lo), c((u32)((1ull << 60) - P.q)) {}
  __device__ static Val load(u64 x) { return (x & 0x3fffffffull) | ((x >> 30) << 32); }
  __device__ static void zero(Acc& a) { a.d0 = a.d1 = a.d2 = Sums{0, 0, 0}; }
  __device__ static Val sum(Val x, Val) { return x; }   // no Karatsuba term
  __device__ static void mac1(Sums& s, Val x, Val y) {
    s.L = madw(lo32(x), lo32(y), s.L);
    s.M = madw(lo32(x), hi32(y), s.M);
    s.M = madw(hi32(x), lo32(y), s.M);
    s.H = madw(hi32(x), hi32(y), s.H);
  }
  __device__ void mac(Acc& a, Val a0, Val a1, Val, Val b0, Val b1, Val) const {
    mac1(a.d0, a0, b0);
    mac1(a.d1, a0, b1);
    mac1(a.d1, a1, b0);
    mac1(a.d2, a1, b1);
  }
  static constexpr int kFold = 4;   // entries between folds of d1 (twice that for d0 and d2)
  static constexpr int kGroup = 2;
  __device__ void fold1(Sums& s) const {
    s.M += s.L >> 30;
    s.H += s.M >> 30;
    const u64 t = madw(hi32(s.H), c, 0);
    s.L = madw(lo32(s.H), c, s.L & 0x3fffffffull);
    s.M = (s.M & 0x3fffffffull) + ((t & 0xfffffffull) << 2);
    s.H = t >> 28;
  }
  // the n-th fold since the start: d1 every time, d0 and d2 every other time
  __device__ void fold(Acc& a, int n = 0) const {
    fold1(a.d1);
    if ((n & 1) == 0) {
      fold1(a.d0);
      fold1(a.d2);
    }
  }
  // L + M 2^30 + H 2^60 (after a fold) as 128 bits, reduced
  __device__ u64 residue(const Sums& s) const {
    U128 v{s.L, 0};
    add_wide(v, U128{s.M << 30, s.M >> 34});
    add_wide(v, U128{s.H << 60, s.H >> 4});
    return reduce_wide(v, q, mu_hi, mu_lo);
  }
  __device__ void final(const Acc& a, u64& d0, u64& d1, u64& d2) const {
    Acc f = a;
    fold(f);
    d0 = residue(f.d0);
    d1 = residue(f.d1);
    d2 = residue(f.d2);
  }
};

// Block kernel: 8 waves share one 64-coefficient chunk of one prime and a
// tile of kTileRows output rows and kCols columns.  Each wave owns RPW rows
// and CPW columns of the tile (RPW x CPW accumulators fit the register
// budget; a wave reads RPW + CPW operands from LDS per entry for RPW * CPW
// products).  Per visited k, the A values of the
// tile rows that visit it and the B values of the block's kCols columns are
// staged once through LDS (double-buffered): each wave loads two A rows and
// one B row (a column's poly), and every wave reads what it needs from LDS,
// so each operand word is loaded from memory once per block and entry.
// Global loads run two entries ahead of the multiplies.
//
// BSP: the right operand is sparse too (tl.bslot gives the stored slot of
// B_kj, or -1 for a zero): a wave skips the columns whose B_kj is zero, so a
// product is skipped when either operand is zero.
template <typename Arith, int RPW, int CPW, bool BSP>
__global__ void __launch_bounds__(512, 4) tensor_block_kernel(TileList tl, const u64* A, const u64* B, u64* D,
                                                             FpLimbs fl, DevParams dp) {
  typedef typename Arith::Val Val;
  constexpr int kRowGroups = kTileRows / RPW;
  constexpr int kColGroups = kWavesPerBlock / kRowGroups;
  constexpr int kCols = kColGroups * CPW;
  static_assert(kRowGroups * kColGroups == kWavesPerBlock, "waves tile the block");
  __shared__ Val sa[2][kTileRows][2][64];
  __shared__ Val sb[2][kCols][2][64];              // B of the block's columns for the entry
  __shared__ int2 s_km[kSegEntries];               // (k, row mask) per entry
  __shared__ int s_es[kSegEntries][kTileRows];     // A slot per entry and row
  const int N = dp.N, L = dp.L;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: row and column choices are scalar
  // block b: XCD-aware order.  b mod 8 picks the 64-coefficient chunk of a
  // 512-coefficient slab, so one XCD works on one chunk; above that the row
  // tile varies fastest, then the column tile, then the slab: the row tiles
  // of one column tile run back to back on an XCD and reuse its B from L2.
  int g, h, li, tbase;
  {
    const int64_t b = blockIdx.x;
    const int x = (int)(b & 7);
    int64_t rest = b >> 3;
    g = (int)(rest % tl.n_row_tiles);
    rest /= tl.n_row_tiles;
    h = (int)(rest % tl.n_col_tiles);
    rest /= tl.n_col_tiles;
    const int chunks512 = N / 512;
    const int c512 = (int)(rest % chunks512);
    li = (int)(rest / chunks512);
    tbase = (c512 * 8 + x) * 64;
  }
  const FpLimb& F = fl.l[li];
  const int l = F.limb;
  const Arith ar(F, dp.pr[l]);
  const int Nc = tl.Nc;
  // chunked layout: poly 0 of ciphertext e at base + e * 64, poly 1 one n_ct * 64 further
  const int64_t cidx = (int64_t)l * (N >> 6) + (tbase >> 6);
  const u64* Ab = A + cidx * 2 * tl.nA * 64 + lane;
  const u64* Bb = B + cidx * 2 * tl.nB * 64 + lane;
  const int64_t pA = tl.nA * 64, pB = tl.nB * 64;
  const int rbase = (wave / kColGroups) * RPW;   // the wave's rows and columns within the tile
  const int cbase = (wave % kColGroups) * CPW;
  const int arow0 = 2 * wave, arow1 = 2 * wave + 1;   // the rows this wave stages
  // and the B row (column wave / 2 of the block, poly wave % 2) it stages
  const bool bload = wave < 2 * kCols;
  const int jb = h * kCols + (wave >> 1);
  const int64_t pb_off = (wave & 1) ? pB : 0;
  typename Arith::Acc acc[RPW][CPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r)
#pragma unroll
    for (int c = 0; c < CPW; ++c) Arith::zero(acc[r][c]);

  const int e0 = tl.tstart[g], e1 = tl.tstart[g + 1];
  struct Stage {
    u64 b, a00, a01, a10, a11;
    int mask;
    int cmask;   // bit c: column cbase + c has B_kj (always all ones for a dense B)
  };
  // the tile's entry list goes through LDS in segments, so that the loads two
  // entries ahead need no scalar memory round trip
  // entry metadata is the same for every lane: read it into scalar registers
  // so that the row tests below are scalar branches, not lane masks
  auto fetch = [&](int x, int xend, Stage& st) {
    st.mask = 0;
    if (x >= xend) return;
    const int2 km = s_km[x];
    const int2 sl = *reinterpret_cast<const int2*>(&s_es[x][arow0]);   // slots of rows arow0, arow0 + 1
    const int k = __builtin_amdgcn_readfirstlane(km.x);
    st.mask = __builtin_amdgcn_readfirstlane(km.y);
    st.b = 0;
    if constexpr (BSP) {
      const int* bs_k = tl.bslot + (int64_t)k * Nc;
      st.cmask = 0;
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const int jc = h * kCols + cbase + c;
        if (jc < Nc && bs_k[jc] >= 0) st.cmask |= 1 << c;
      }
      if (bload && jb < Nc) {
        const int sl = bs_k[jb];
        if (sl >= 0) st.b = Bb[(int64_t)sl * 64 + pb_off];
      }
    } else {
      st.cmask = (1 << CPW) - 1;
      if (bload && jb < Nc) st.b = Bb[((int64_t)k * Nc + jb) * 64 + pb_off];
    }
    if ((st.mask >> arow0) & 1) {
      const u64* ap = Ab + (int64_t)__builtin_amdgcn_readfirstlane(sl.x) * 64;
      st.a00 = ap[0];
      st.a01 = ap[pA];
    }
    if ((st.mask >> arow1) & 1) {
      const u64* ap = Ab + (int64_t)__builtin_amdgcn_readfirstlane(sl.y) * 64;
      st.a10 = ap[0];
      st.a11 = ap[pA];
    }
  };
  auto put = [&](const Stage& st, int bf) {
    if (bload) sb[bf][wave >> 1][wave & 1][lane] = Arith::load(st.b);
    if ((st.mask >> arow0) & 1) {
      sa[bf][arow0][0][lane] = Arith::load(st.a00);
      sa[bf][arow0][1][lane] = Arith::load(st.a01);
    }
    if ((st.mask >> arow1) & 1) {
      sa[bf][arow1][0][lane] = Arith::load(st.a10);
      sa[bf][arow1][1][lane] = Arith::load(st.a11);
    }
  };
  // the A values of groups of four rows are read from LDS before their
  // multiplies, so their latency is paid once per group; a row not visiting
  // k reads a stale word that is never used
  auto compute = [&](const Stage& st, int bf) {
    const int wmask = (st.mask >> rbase) & ((1 << RPW) - 1);
    if (!wmask) return;
    if (BSP && !st.cmask) return;
    Val b0[CPW], b1[CPW], bs[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      b0[c] = sb[bf][cbase + c][0][lane];
      b1[c] = sb[bf][cbase + c][1][lane];
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c) bs[c] = Arith::sum(b0[c], b1[c]);
    constexpr int G = RPW > Arith::kGroup ? Arith::kGroup : RPW;   // rows read from LDS together
#pragma unroll
    for (int g0 = 0; g0 < RPW; g0 += G) {
      Val a0[G], a1[G];
#pragma unroll
      for (int r = 0; r < G; ++r) {
        a0[r] = sa[bf][rbase + g0 + r][0][lane];
        a1[r] = sa[bf][rbase + g0 + r][1][lane];
      }
#pragma unroll
      for (int r = 0; r < G; ++r) {
        if (wmask & (1 << (g0 + r))) {
          const Val as = Arith::sum(a0[r], a1[r]);
#pragma unroll
          for (int c = 0; c < CPW; ++c)
            if (!BSP || ((st.cmask >> c) & 1)) ar.mac(acc[g0 + r][c], a0[r], a1[r], as, b0[c], b1[c], bs[c]);
        }
      }
    }
  };
  int cnt = 0;
  for (int sg = e0; sg < e1; sg += kSegEntries) {
    const int n = min(kSegEntries, e1 - sg);
    __syncthreads();   // the previous segment's entries are no longer read
    for (int x = threadIdx.x; x < n; x += blockDim.x) {
      s_km[x] = make_int2(tl.ek[sg + x], tl.emask[sg + x]);
    }
    for (int x = threadIdx.x; x < n * kTileRows; x += blockDim.x) s_es[x / kTileRows][x % kTileRows] = tl.eslot[(int64_t)sg * kTileRows + x];
    __syncthreads();
    Stage sA, sB;
    fetch(0, n, sA);
    fetch(1, n, sB);
    for (int x = 0; x < n; x += 2) {
      put(sA, 0);
      __syncthreads();
      const Stage cA = sA;
      fetch(x + 2, n, sA);
      compute(cA, 0);
      if (x + 1 < n) {
        put(sB, 1);
        __syncthreads();
        const Stage cB = sB;
        fetch(x + 3, n, sB);
        compute(cB, 1);
      }
      cnt += 2;
      if (cnt >= Arith::kFold) {
        cnt = 0;
#pragma unroll
        for (int r = 0; r < RPW; ++r)
#pragma unroll
          for (int c = 0; c < CPW; ++c) ar.fold(acc[r][c]);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int j = h * kCols + cbase + c;
    if (j >= Nc) continue;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int pos = g * kTileRows + rbase + r;
      if (pos >= tl.rows) continue;
      u64* dp_ = D + ((int64_t)pos * Nc + j) * (int64_t)3 * L * N + (int64_t)l * N + tbase + lane;
      u64 d0, d1, d2;
      ar.final(acc[r][c], d0, d1, d2);
      dp_[0] = d0;
      dp_[(int64_t)L * N] = d1;
      dp_[(int64_t)2 * L * N] = d2;
    }
  }
}

// Column kernel (the fp64 primes and the primes 2^60 - c): 8 waves share one
// 64-coefficient chunk of one prime, a tile of TR output rows and 8 CPW
// columns, and wave w owns columns w, w + 8, ... of the block for all TR
// rows.  Per visited k every wave multiplies the same rows (those the tile's
// entry mask marks), so the waves reach each barrier together: none idles
// while another works through more rows, which is what a split of the rows
// among waves costs at unstructured sparsity.  With CPW = 2 a row's A values,
// read once from LDS, serve two columns, and an entry's per-wave work (its
// mask and slots, its B words and their conversion) is spread over twice the
// products of a tile half as tall.
//
// Entries go in pairs.  The A values of the rows that visit the pair's two k
// (with a0 + a1, the Karatsuba operand, formed once by the staging wave:
// wave w stages row w) are staged through LDS, double-buffered, with one
// barrier per pair.  B needs no exchange: a wave is the only user of its
// columns, so it loads B[k][j] straight into registers.  Global loads run one
// pair (two entries) ahead.  The tile list has TR rows per tile (eslot
// [entries][TR]).
template <int TR, int CPW>
struct ColsEntry {
  static constexpr int kAV = 2 * TR / kWavesPerBlock < 2 ? 2 : 2 * TR / kWavesPerBlock;   // A values (row, poly) a staging wave loads
  u64 a[kAV];
  u64 b0[CPW], b1[CPW];
  int mask;
  bool bact[CPW];
};

// B's words go through a raw buffer resource: a wave-uniform base and byte
// offset in scalar registers and the lane's byte offset in one vector
// register set up once, so a load takes no vector address arithmetic (one
// (prime, chunk) slice of B is below 2^31 bytes).  The base is read through
// readfirstlane so that the resource is known to be uniform.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t slice_rsrc(const u64* base, int64_t bytes) {
  const u64 p = (u64)base;
  const u64 pu = ((u64)(u32)__builtin_amdgcn_readfirstlane((int)(p >> 32)) << 32) |
                 (u32)__builtin_amdgcn_readfirstlane((int)(u32)p);
  return __builtin_amdgcn_make_buffer_rsrc((void*)pu, (short)0, __builtin_amdgcn_readfirstlane((int)bytes), 0x00020000);
}
__device__ __forceinline__ u64 slice_load(__amdgpu_buffer_rsrc_t r, unsigned lane_off, int off) {
  const u32x2_t v = __builtin_amdgcn_raw_buffer_load_b64(r, lane_off, off, 0);
  return ((u64)v.y << 32) | v.x;
}

template <typename Arith, int TR, int CPW, bool BSP>
__global__ void __launch_bounds__(512, 4) tensor_cols_kernel(TileList tl, const u64* A, const u64* B, u64* D,
                                                            FpLimbs fl, DevParams dp) {
  typedef typename Arith::Val Val;
  constexpr int kCols = kWavesPerBlock * CPW;
  constexpr int kAV = ColsEntry<TR, CPW>::kAV;
  constexpr int kAR = kAV < 2 ? 1 : kAV / 2;         // rows each staging wave stages
  constexpr int kStagers = TR / kAR;                 // waves that stage A rows
  constexpr int kNV = Arith::kSum ? 3 : 2;           // staged values per row
  __shared__ Val sa[2][2][TR][kNV][64];              // [buffer][entry of the pair][row]: a0, a1 (, a0 + a1)
  __shared__ int2 s_km[kSegEntries];
  __shared__ int s_es[kSegEntries][TR];
  const int N = dp.N, L = dp.L;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int g, h, li, tbase;
  {
    const int64_t b = blockIdx.x;
    const int x = (int)(b & 7);
    int64_t rest = b >> 3;
    g = (int)(rest % tl.n_row_tiles);
    rest /= tl.n_row_tiles;
    h = (int)(rest % tl.n_col_tiles);
    rest /= tl.n_col_tiles;
    const int chunks512 = N / 512;
    const int c512 = (int)(rest % chunks512);
    li = (int)(rest / chunks512);
    tbase = (c512 * 8 + x) * 64;
  }
  const FpLimb& F = fl.l[li];
  const int l = F.limb;
  const Arith ar(F, dp.pr[l]);
  const int Nc = tl.Nc;
  const int64_t cidx = (int64_t)l * (N >> 6) + (tbase >> 6);
  const u64* Ab = A + cidx * 2 * tl.nA * 64 + lane;
  const __amdgpu_buffer_rsrc_t rB = slice_rsrc(B + cidx * 2 * tl.nB * 64, (int64_t)tl.nB * 1024);
  const unsigned loff = (unsigned)lane * 8u;
  const int pBb = (int)tl.nB * 512;   // byte offset of poly 1
  const int64_t pA = tl.nA * 64;
  int jc[CPW];                                       // this wave's columns
  bool jinc[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    jc[c] = h * kCols + c * kWavesPerBlock + wave;
    jinc[c] = jc[c] < Nc;
  }
  const bool jin = jinc[0];
  const bool stager = wave < kStagers;
  const int arow = stager ? wave * kAR : 0;          // first row this wave stages
  typename Arith::Acc acc[TR][CPW];
#pragma unroll
  for (int r = 0; r < TR; ++r)
#pragma unroll
    for (int c = 0; c < CPW; ++c) Arith::zero(acc[r][c]);

  typedef ColsEntry<TR, CPW> Entry;
  struct Pair {
    Entry e[2];
  };
  const int e0 = tl.tstart[g], e1 = tl.tstart[g + 1];
  auto fetch = [&](int x, int xend, Entry& st) {
    st.mask = 0;
#pragma unroll
    for (int c = 0; c < CPW; ++c) st.bact[c] = false;
    if (x >= xend) return;
    const int2 km = s_km[x];
    const int k = __builtin_amdgcn_readfirstlane(km.x);
    st.mask = __builtin_amdgcn_readfirstlane(km.y);
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      st.bact[c] = jinc[c];
      if (jinc[c]) {
        int64_t bsl = (int64_t)k * Nc + jc[c];
        if constexpr (BSP) {
          bsl = tl.bslot[(int64_t)k * Nc + jc[c]];
          st.bact[c] = bsl >= 0;
        }
        if (st.bact[c]) {
          st.b0[c] = slice_load(rB, loff, (int)bsl * 512);
          st.b1[c] = slice_load(rB, loff, (int)bsl * 512 + pBb);
        }
      }
    }
    if (!stager) return;
#pragma unroll
    for (int r = 0; r < kAR; ++r) {
      if ((st.mask >> (arow + r)) & 1) {
        const u64* ap = Ab + (int64_t)__builtin_amdgcn_readfirstlane(s_es[x][arow + r]) * 64;
        st.a[2 * r] = ap[0];
        st.a[2 * r + 1] = ap[pA];
      }
    }
  };
  auto put = [&](const Entry& st, int bf, int ep) {
    if (!stager) return;
#pragma unroll
    for (int r = 0; r < kAR; ++r) {
      if ((st.mask >> (arow + r)) & 1) {
        const Val a0 = Arith::load(st.a[2 * r]), a1 = Arith::load(st.a[2 * r + 1]);
        sa[bf][ep][arow + r][0][lane] = a0;
        sa[bf][ep][arow + r][1][lane] = a1;
        if constexpr (Arith::kSum) sa[bf][ep][arow + r][kNV - 1][lane] = Arith::sum(a0, a1);
      }
    }
  };
  // what a pair's products need besides LDS: the B words and the row masks
  // (zero for an entry whose B_kj is zero or whose column is outside B)
  struct PairB {
    u64 b0[2][CPW], b1[2][CPW];
    int m[2][CPW];
  };
  auto take_b = [&](const Pair& pr) {
    PairB q;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        q.b0[x][c] = pr.e[x].b0[c];
        q.b1[x][c] = pr.e[x].b1[c];
        q.m[x][c] = pr.e[x].bact[c] ? pr.e[x].mask : 0;
      }
    return q;
  };
  // the products of one entry of a pair (B from registers, A from LDS, read
  // once per row for the wave's CPW columns)
  auto compute1 = [&](const PairB& pb, int x, int bf) {
    int mu = 0;
#pragma unroll
    for (int c = 0; c < CPW; ++c) mu |= pb.m[x][c];
    if (!mu) return;
    Val b0[CPW], b1[CPW], bs[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      b0[c] = Arith::load(pb.b0[x][c]);
      b1[c] = Arith::load(pb.b1[x][c]);
      bs[c] = Arith::sum(b0[c], b1[c]);
    }
#pragma unroll
    for (int r = 0; r < TR; ++r) {
      if ((mu >> r) & 1) {
        const Val a0 = sa[bf][x][r][0][lane], a1 = sa[bf][x][r][1][lane];
        const Val as = sa[bf][x][r][kNV - 1][lane];
#pragma unroll
        for (int c = 0; c < CPW; ++c)
          if ((pb.m[x][c] >> r) & 1) ar.mac(acc[r][c], a0, a1, as, b0[c], b1[c], bs[c]);
      }
    }
  };
  auto compute = [&](const PairB& pb, int bf) {
    compute1(pb, 0, bf);
    compute1(pb, 1, bf);
  };
  int cnt = 0, nfold = 0;
  for (int sg = e0; sg < e1; sg += kSegEntries) {
    const int n = min(kSegEntries, e1 - sg);
    __syncthreads();   // the previous segment's entries are no longer read
    for (int x = threadIdx.x; x < n; x += blockDim.x) s_km[x] = make_int2(tl.ek[sg + x], tl.emask[sg + x]);
    for (int x = threadIdx.x; x < n * TR; x += blockDim.x) s_es[x / TR][x % TR] = tl.eslot[(int64_t)sg * TR + x];
    __syncthreads();
    // one pair in flight: pair p's A goes to LDS buffer p mod 2, its B
    // words to registers, then pair p + 1 is fetched while pair p computes
    Pair pn;
    fetch(0, n, pn.e[0]);
    fetch(1, n, pn.e[1]);
    for (int x = 0; x < n; x += 4) {
      put(pn.e[0], 0, 0);
      put(pn.e[1], 0, 1);
      const PairB cA = take_b(pn);
      __syncthreads();
      fetch(x + 2, n, pn.e[0]);
      fetch(x + 3, n, pn.e[1]);
      compute(cA, 0);
      if (x + 2 < n) {
        put(pn.e[0], 1, 0);
        put(pn.e[1], 1, 1);
        const PairB cB = take_b(pn);
        __syncthreads();
        fetch(x + 4, n, pn.e[0]);
        fetch(x + 5, n, pn.e[1]);
        compute(cB, 1);
      }
      cnt += 4;
      if (cnt >= Arith::kFold) {
        cnt = 0;
        ++nfold;
#pragma unroll
        for (int r = 0; r < TR; ++r)
#pragma unroll
          for (int c = 0; c < CPW; ++c) ar.fold(acc[r][c], nfold);
      }
    }
  }
  if (!jin) return;
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    if (!jinc[c]) continue;
#pragma unroll
    for (int r = 0; r < TR; ++r) {
      const int pos = g * TR + r;
      if (pos >= tl.rows) continue;
      u64* dp_ = D + ((int64_t)pos * Nc + jc[c]) * (int64_t)3 * L * N + (int64_t)l * N + tbase + lane;
      u64 d0, d1, d2;
      ar.final(acc[r][c], d0, d1, d2);
      dp_[0] = d0;
      dp_[(int64_t)L * N] = d1;
      dp_[(int64_t)2 * L * N] = d2;
    }
  }
}

static void grid_rows(int64_t rows, unsigned& gy, unsigned& gz) {
  if (rows < 1) rows = 1;
  gy = rows < 65535 ? (unsigned)rows : 65535u;
  gz = (unsigned)((rows + gy - 1) / gy);
}

int launch_tensor_pointwise(const sfhe_ctx* c, int lev, const u64* a, int64_t astride, const u64* b,
                            int64_t bstride, u64* d, int64_t dstride, int64_t batch, hipStream_t s) {
  if (batch <= 0) return SFHE_OK;
  const int nl = lev + 1;
  unsigned gy, gz;
  grid_rows(batch * nl, gy, gz);
  hipLaunchKernelGGL(tensor_pointwise_kernel, dim3((c->N + 255) / 256, gy, gz), dim3(256), 0, s, nl, a, astride, b,
                     bstride, d, dstride, batch, c->dp);
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

int launch_tensor_gather(const sfhe_ctx* c, int lev, const u64* A, int64_t nA, const u64* B, int64_t nB,
                         const int* d_aidx, const int* d_bidx, u64* d, int64_t count, hipStream_t s) {
  if (count <= 0) return SFHE_OK;
  const int nl = lev + 1;
  unsigned gy, gz;
  grid_rows(count * nl, gy, gz);
  hipLaunchKernelGGL(tensor_gather_kernel, dim3((c->N + 255) / 256, gy, gz), dim3(256), 0, s, nl, A, nA, B, nB,
                     d_aidx, d_bidx, d, count, c->dp);
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

template <typename Arith, int RPW, int CPW, bool BSP>
static int launch_block(const sfhe_ctx* c, const TileList& tl, const FpLimbs& fl, const u64* A, const u64* B, u64* D,
                        hipStream_t s) {
  if (fl.n == 0) return SFHE_OK;
  constexpr int kCols = kWavesPerBlock / (kTileRows / RPW) * CPW;
  TileList t2 = tl;
  t2.n_col_tiles = (tl.Nc + kCols - 1) / kCols;
  const int64_t blocks = (int64_t)fl.n * (c->N / 64) * tl.n_row_tiles * t2.n_col_tiles;
  if (blocks > 0x7FFFFFFF) { set_error("tensor: grid too large"); return SFHE_E_INVALID_ARG; }
  hipLaunchKernelGGL((tensor_block_kernel<Arith, RPW, CPW, BSP>), dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), 0, s, t2, A,
                     B, D, fl, c->dp);
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

template <typename Arith, int TR, int CPW, bool BSP>
static int launch_cols(const sfhe_ctx* c, const TileList& tl, const FpLimbs& fl, const u64* A, const u64* B, u64* D,
                       hipStream_t s) {
  if (fl.n == 0) return SFHE_OK;
  if (tl.tile_rows != TR) { set_error("tensor: tile list of another height"); return SFHE_E_INVALID_ARG; }
  // B's words are addressed by 32-bit byte offsets within one (prime, chunk) slice
  if (tl.nB * 1024 > 0x7FFFFFFF) { set_error("tensor: right operand too large"); return SFHE_E_INVALID_ARG; }
  TileList t2 = tl;
  t2.n_col_tiles = (tl.Nc + kWavesPerBlock * CPW - 1) / (kWavesPerBlock * CPW);
  const int64_t blocks = (int64_t)fl.n * (c->N / 64) * tl.n_row_tiles * t2.n_col_tiles;
  if (blocks > 0x7FFFFFFF) { set_error("tensor: grid too large"); return SFHE_E_INVALID_ARG; }
  hipLaunchKernelGGL((tensor_cols_kernel<Arith, TR, CPW, BSP>), dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), 0, s, t2, A, B,
                     D, fl, c->dp);
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

int tensor_fp_prime_count(const sfhe_ctx* c) {
  int n = 0;
  for (int l = 0; l < c->L; ++l) n += c->primes[l] < (1ull << 42);
  return n;
}

int launch_tensor_tiles(const sfhe_ctx* c, const TileList& tl, const TileList& tl_cols, const u64* A, const u64* B,
                        u64* D, hipStream_t s, hipEvent_t fp_start, hipEvent_t fp_stop) {
  if (tl.rows <= 0) return SFHE_OK;
  // primes below 2^42 use the fp64 residue arithmetic, the others 128-bit integers
  FpLimbs ffp{}, fint{}, f60{};
  for (int l = 0; l < c->L; ++l) {
    const u64 q = c->primes[l];
    FpLimb F{};
    F.limb = l;
    F.q = (double)q;
    F.qinv = 1.0 / (double)q;
    const bool near60 = q < (1ull << 60) && (1ull << 60) - q < (1ull << 20);
    FpLimbs& dst = q < (1ull << 42) ? ffp : near60 ? f60 : fint;
    dst.l[dst.n++] = F;
  }
  if (fp_start) SFHE_HIP(hipEventRecord(fp_start, s));
  const bool bsp = tl.bslot != nullptr;
  int rc = bsp ? launch_cols<ArithFp, kColTileRows, 2, true>(c, tl_cols, ffp, A, B, D, s)
               : launch_cols<ArithFp, kColTileRows, 2, false>(c, tl_cols, ffp, A, B, D, s);
  if (fp_stop) SFHE_HIP(hipEventRecord(fp_stop, s));
  if (!rc)
    rc = bsp ? launch_block<ArithInt, 4, 1, true>(c, tl, fint, A, B, D, s)
             : launch_block<ArithInt, 4, 1, false>(c, tl, fint, A, B, D, s);
  if (!rc)
    rc = bsp ? launch_cols<ArithInt60, kColTileRows, 1, true>(c, tl_cols, f60, A, B, D, s)
             : launch_cols<ArithInt60, kColTileRows, 1, false>(c, tl_cols, f60, A, B, D, s);
  return rc;
}

}  // namespace sfhe
