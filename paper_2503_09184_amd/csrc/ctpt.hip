// ctpt.hip -- plaintext weights times encrypted values (Sec. 3.3.2: a server
// that holds a layer's weights in plaintext multiplies them into the client's
// encrypted input, and the weights' zeros are skipped through the same three
// encodings as an encrypted left operand's).
//
// A weight w is the constant polynomial m = nearbyint(w * 2^sw).  A constant
// polynomial takes the same value at every root of X^N + 1, so its product
// with a ciphertext multiplies both polys, coefficient by coefficient and in
// either domain, by the residue m mod q_i.  An output is the sum of these
// products over the visited k, in the NTT domain, followed by one rescale.
// Per (output, prime, coefficient) the work is a sparse-times-dense product
// over Z_q: one multiply-add per loaded word of B and per tile row that
// visits its k.
#include "fparith.hpp"

namespace sfhe {

namespace {

constexpr int kPlainTileRows = 16;   // rows of a tile: bits of an entry's row mask
constexpr int kPlainCols = 4;        // columns of a block: one per wave

// block b: 64-coefficient chunk (b mod 8) of a 512-coefficient slab, then
// the (job, tile, column group) descriptor, the slab and the prime.  The 8
// XCDs take consecutive blocks in turn, so each XCD works on one chunk, and
// the row tiles of one column group (which read the same B words) run back
// to back on it.
struct BlockPos {
  int desc, t, li;
};
__device__ __forceinline__ BlockPos plain_block(int64_t b, int n_desc, int N) {
  BlockPos r;
  const int x = (int)(b & 7);
  int64_t rest = b >> 3;
  r.desc = (int)(rest % n_desc);
  rest /= n_desc;
  const int slabs = N >> 9;
  const int slab = (int)(rest % slabs);
  r.li = (int)(rest / slabs);
  r.t = (slab * 8 + x) * 64;
  return r;
}

// exact fp64 arithmetic, primes below 2^42: sums of lazy products
struct PlainFp {
  double q, qinv;
  __device__ PlainFp(const FpLimb& F, const PrimeDev&) : q(F.q), qinv(F.qinv) {}
  typedef double Acc;
  typedef double In;
  __device__ static In in(u64 x) { return u52_to_f64(x); }   // x < q < 2^42
  __device__ static Acc zero() { return 0.0; }
  // w: the residue's fp64 bits (the weight table holds them for these primes)
  __device__ void mac(Acc& a, In b, u64 w, u64) const { a += fp_mulmod_lazy(b, __longlong_as_double((long long)w), q, qinv); }
  static constexpr int kFold = 1024;   // each product adds < 1.5 q: stay below 2^53
  __device__ void fold(Acc& a) const { a = fp_fold(a, q, qinv); }
  __device__ u64 final(Acc a) const { return fp_final(a, q, qinv); }
};

// integer arithmetic with Shoup products, other primes (q < 2^61): the sum
// stays in [0, 2q)
struct PlainInt {
  u64 q, q2;
  __device__ PlainInt(const FpLimb&, const PrimeDev& P) : q(P.q), q2(2 * P.q) {}
  typedef u64 Acc;
  typedef u64 In;
  __device__ static In in(u64 x) { return x; }
  __device__ static Acc zero() { return 0; }
  __device__ void mac(Acc& a, In b, u64 w, u64 ws) const {
    const u64 s = a + mul_shoup_lazy(b, w, ws, q);   // < 4q < 2^63
    a = s >= q2 ? s - q2 : s;
  }
  static constexpr int kFold = 1 << 30;
  __device__ void fold(Acc&) const {}
  __device__ u64 final(Acc a) const { return a >= q ? a - q : a; }
};

// Block: 4 waves, one column each, of one job's 16-row tile, one 64-coefficient
// chunk and one prime.  Per entry (k, row mask) of the tile a wave loads the
// two words of B[k][j] for its lane's coefficient (512 contiguous bytes per
// wave and poly) once and multiplies them into the accumulators of the tile
// rows in the mask; the 16 weights of the entry and prime are scalars, read
// from the weight table in whole 32-byte loads, so a row test is a scalar
// branch.  B for the next
// entry is loaded before the current entry's products (the last entry's
// next load repeats it, so every iteration issues the same loads).
template <typename Ar>
__global__ void __launch_bounds__(64 * kPlainCols) ctpt_block_kernel(PlainBatch pb, FpLimbs fl, DevParams dp) {
  const int N = dp.N;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const BlockPos bp = plain_block(blockIdx.x, pb.n_desc, N);
  const int4 dsc = pb.desc[bp.desc];
  const PlainJob& J = pb.jobs[dsc.x];
  const int g = dsc.y;
  const int j = dsc.z * kPlainCols + wave;
  if (j >= J.Nc) return;   // no barrier in this kernel: a wave without a column leaves
  const FpLimb& F = fl.l[bp.li];
  const int l = F.limb;
  const Ar ar(F, dp.pr[l]);
  const int t = bp.t + lane;
  const int nchunk = N >> 6;
  // B word of stored ciphertext e, poly p: Bl[e * 64 + p * pstride] (chunked layout)
  const u64* Bl = J.B + ((int64_t)l * nchunk + (t >> 6)) * 2 * J.nB * 64 + lane;
  const int64_t pstride = J.nB * 64;
  const int e0 = J.tstart[g], e1 = J.tstart[g + 1];
  typename Ar::Acc acc0[kPlainTileRows], acc1[kPlainTileRows];
#pragma unroll
  for (int r = 0; r < kPlainTileRows; ++r) acc0[r] = acc1[r] = Ar::zero();
  if (e0 < e1) {
    int k = J.ek[e0];
    u64 nb0 = Bl[((int64_t)k * J.Nc + j) * 64], nb1 = Bl[((int64_t)k * J.Nc + j) * 64 + pstride];
    int cnt = 0;
    for (int e = e0; e < e1; ++e) {
      const typename Ar::In b0 = Ar::in(nb0), b1 = Ar::in(nb1);
      const int mask = J.emask[e];
      const int en = e + 1 < e1 ? e + 1 : e;
      k = J.ek[en];
      nb0 = Bl[((int64_t)k * J.Nc + j) * 64];
      nb1 = Bl[((int64_t)k * J.Nc + j) * 64 + pstride];
      // the entry's 16 weights (and companions) in whole 32-byte scalar
      // loads, waited for once: read one by one inside the row branches, each
      // visited row waited for its own scalar load
      const ulonglong4* wv = reinterpret_cast<const ulonglong4*>(J.ew + ((int64_t)e * pb.nl + l) * kPlainTileRows);
      const ulonglong4* wsv = reinterpret_cast<const ulonglong4*>(J.ews + ((int64_t)e * pb.nl + l) * kPlainTileRows);
      u64 wr[kPlainTileRows], wsr[kPlainTileRows];
#pragma unroll
      for (int g4 = 0; g4 < kPlainTileRows / 4; ++g4) {
        const ulonglong4 a4 = wv[g4], s4 = wsv[g4];
        wr[4 * g4] = a4.x;
        wr[4 * g4 + 1] = a4.y;
        wr[4 * g4 + 2] = a4.z;
        wr[4 * g4 + 3] = a4.w;
        wsr[4 * g4] = s4.x;
        wsr[4 * g4 + 1] = s4.y;
        wsr[4 * g4 + 2] = s4.z;
        wsr[4 * g4 + 3] = s4.w;
      }
#pragma unroll
      for (int r = 0; r < kPlainTileRows; ++r) {
        if ((mask >> r) & 1) {
          ar.mac(acc0[r], b0, wr[r], wsr[r]);
          ar.mac(acc1[r], b1, wr[r], wsr[r]);
        }
      }
      if (++cnt >= Ar::kFold) {
        cnt = 0;
#pragma unroll
        for (int r = 0; r < kPlainTileRows; ++r) {
          ar.fold(acc0[r]);
          ar.fold(acc1[r]);
        }
      }
    }
  }
  const int nl = pb.nl;
#pragma unroll
  for (int r = 0; r < kPlainTileRows; ++r) {
    const int pos = g * kPlainTileRows + r;
    if (pos >= J.rows) break;
    u64* d = pb.D + (J.d0 + (int64_t)pos * J.Nc + j) * 2 * nl * N + (int64_t)l * N + t;
    d[0] = ar.final(acc0[r]);
    d[(int64_t)nl * N] = ar.final(acc1[r]);
  }
}

// one product: D[p][i][t] += (w_i B[slot][p][i][t]) mod q_i over every prime
// and coefficient (the one-launch-per-product form); grid (N / 256, 2 nl)
__global__ void __launch_bounds__(256) ctpt_product_kernel(const u64* B, int64_t nB, int64_t slot, const u64* w,
                                                           const u64* ws, u64* D, int nl, DevParams dp) {
  const int N = dp.N;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= N) return;
  const int p = blockIdx.y / nl, i = blockIdx.y % nl;
  const u64 q = dp.pr[i].q;
  const u64 b = B[chunk_index(slot, p, i, t, nB, N >> 6)];
  u64& d = D[((int64_t)p * nl + i) * N + t];
  d = add_mod(d, mul_shoup(b, w[i], ws[i], q), q);
}

template <typename Ar>
int launch_plain_blocks(const sfhe_ctx* c, const PlainBatch& pb, const FpLimbs& fl, hipStream_t s) {
  if (fl.n == 0 || pb.n_desc == 0) return SFHE_OK;
  const int64_t blocks = (int64_t)8 * pb.n_desc * (c->N >> 9) * fl.n;
  if (blocks > 0x7FFFFFFF) { set_error("plaintext-weight product: grid too large"); return SFHE_E_INVALID_ARG; }
  hipLaunchKernelGGL((ctpt_block_kernel<Ar>), dim3((unsigned)blocks), dim3(64 * kPlainCols), 0, s, pb, fl, c->dp);
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

}  // namespace

int launch_plain_batch(const sfhe_ctx* c, const PlainBatch& pb, hipStream_t s) {
  if (c->N < 512) { set_error("plaintext-weight product: ring degree below 512"); return SFHE_E_UNSUPPORTED; }
  FpLimbs ffp{}, fint{};
  for (int l = 0; l < pb.nl; ++l) {
    const u64 q = c->primes[l];
    FpLimb F{};
    F.limb = l;
    F.q = (double)q;
    F.qinv = 1.0 / (double)q;
    FpLimbs& dst = q < (1ull << 42) ? ffp : fint;
    dst.l[dst.n++] = F;
  }
  int rc = launch_plain_blocks<PlainFp>(c, pb, ffp, s);
  if (!rc) rc = launch_plain_blocks<PlainInt>(c, pb, fint, s);
  return rc;
}

int launch_plain_product(const sfhe_ctx* c, const u64* B, int64_t nB, int64_t slot, const u64* w, const u64* ws,
                         u64* D, int nl, hipStream_t s) {
  hipLaunchKernelGGL(ctpt_product_kernel, dim3((unsigned)((c->N + 255) / 256), (unsigned)(2 * nl)), dim3(256), 0, s, B,
                     nB, slot, w, ws, D, nl, c->dp);
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

}  // namespace sfhe
