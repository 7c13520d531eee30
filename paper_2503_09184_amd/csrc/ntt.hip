// ntt.hip -- batched negacyclic NTT / inverse NTT for gfx950.
//
// One workgroup transforms one row of N residues (N <= 2^14) held in LDS.
// Forward: Cooley-Tukey with the psi twist merged into the twiddles (Longa
// and Naehrig 2016), bit-reversed output, so index k holds a(psi^(2 brv(k)+1)).
// Inverse: Gentleman-Sande, N^-1 applied on the way out.
//
// The log2 N butterfly stages run in passes of up to four: a thread holds 16
// residues x0 + u * t (u < 16) in registers, performs the pass's four stages
// on them, and the pass ends with one LDS exchange and one barrier (4 passes
// instead of 14 for N = 2^14).  LDS rows are padded by one word every 16, so
// every pass's access pattern hits each bank at most four times per wave.
// The forward transform reads its first pass straight from HBM (coalesced),
// the inverse writes its last pass straight to HBM.
//
// Two arithmetics: primes below 2^42 run the butterflies in exact fp64
// (products a*b - k*q via fma; forward values grow by at most 1.5 q per stage
// and need no reduction before the end, inverse values are folded after each
// pass); larger primes use Harvey's lazy integer butterflies with Shoup
// quotients (forward values in [0, 4q), inverse in [0, 2q)).
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
  return (u64)r;
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
  __device__ u64 out_inv(Val x, const PrimeDev& P) const {
    const u64 v = mul_shoup_lazy(x, P.ninv, P.ninv_s, q);
    return v >= q ? v - q : v;
  }
};

struct NttFp {
  typedef double Val;
  double q, qinv;
  const double* w;
  __device__ NttFp(const PrimeDev& P, bool inv) : q((double)P.q), qinv(1.0 / (double)P.q), w(inv ? P.itwd : P.twd) {}
  __device__ Val in(u64 x) const { return (double)x; }
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
  __device__ u64 out_inv(Val x, const PrimeDev& P) const {
    return fp_to_residue(fmm(x, (double)P.ninv, q, qinv), q, qinv);
  }
};

// one forward pass of P stages s0 .. s0+P-1 over all units of this thread
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

// one inverse pass of P stages with distances t0, 2 t0, ..., 2^(P-1) t0
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

template <bool INV, typename Ar>
__device__ __forceinline__ void ntt_row(u64* p, const PrimeDev& P, int N, int logN, void* lds) {
  typedef typename Ar::Val Val;
  Val* sh = reinterpret_cast<Val*>(lds);
  const Ar ar(P, INV);
  if (!INV) {
    int s0 = 0;
    while (s0 < logN) {
      const int np = min(4, logN - s0);
      const u64* src = s0 == 0 ? p : nullptr;
      if (np == 4) fwd_pass<4>(ar, sh, src, N, logN, s0);
      else if (np == 3) fwd_pass<3>(ar, sh, src, N, logN, s0);
      else if (np == 2) fwd_pass<2>(ar, sh, src, N, logN, s0);
      else fwd_pass<1>(ar, sh, src, N, logN, s0);
      __syncthreads();
      s0 += np;
    }
    for (int x = threadIdx.x; x < N; x += blockDim.x) p[x] = ar.out_fwd(sh[lpos(x)]);
  } else {
    for (int x = threadIdx.x; x < N; x += blockDim.x) sh[lpos(x)] = ar.in(p[x]);
    __syncthreads();
    int lt0 = 0;
    while (lt0 < logN) {
      const int np = min(4, logN - lt0);
      u64* dst = lt0 + np == logN ? p : nullptr;
      if (np == 4) inv_pass<4>(ar, sh, dst, P, N, logN, lt0);
      else if (np == 3) inv_pass<3>(ar, sh, dst, P, N, logN, lt0);
      else if (np == 2) inv_pass<2>(ar, sh, dst, P, N, logN, lt0);
      else inv_pass<1>(ar, sh, dst, P, N, logN, lt0);
      __syncthreads();
      lt0 += np;
    }
  }
}

template <bool INV>
__global__ void __launch_bounds__(1024) ntt_kernel(NttRows R, DevParams dp) {
  extern __shared__ u64 lds[];
  const int N = dp.N, logN = dp.logN;
  const int64_t g = blockIdx.x / R.nrow;
  const int r = blockIdx.x % R.nrow;
  u64* p = R.base + g * R.bstride + (int64_t)R.pos[r] * N;
  const PrimeDev& P = dp.pr[R.prime[r]];
  if (P.q < (1ull << 42))
    ntt_row<INV, NttFp>(p, P, N, logN, lds);
  else
    ntt_row<INV, NttInt>(p, P, N, logN, lds);
}

int launch_ntt(const sfhe_ctx* c, u64* base, int64_t batch, int64_t bstride, int nrow, const int* pos,
               const int* prime, bool inverse, hipStream_t s) {
  if (batch <= 0 || nrow <= 0) return SFHE_OK;
  if (nrow > kMaxRows) { set_error("ntt: too many rows per group"); return SFHE_E_INVALID_ARG; }
  NttRows R;
  R.base = base;
  R.bstride = bstride;
  R.nrow = nrow;
  for (int i = 0; i < kMaxRows; ++i) { R.pos[i] = i < nrow ? pos[i] : 0; R.prime[i] = i < nrow ? prime[i] : 0; }
  const int N = c->N;
  const int threads = N / 16 < 1024 ? N / 16 : 1024;
  const size_t lds = (size_t)(N + (N >> kPadShift)) * sizeof(u64);
  const int64_t blocks = batch * nrow;
  if (blocks > 0x7FFFFFFF) { set_error("ntt: batch too large"); return SFHE_E_INVALID_ARG; }
  static bool attr_done[2] = {false, false};
  if (!attr_done[inverse ? 1 : 0]) {
    const void* fn = inverse ? reinterpret_cast<const void*>(&ntt_kernel<true>)
                             : reinterpret_cast<const void*>(&ntt_kernel<false>);
    SFHE_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    attr_done[inverse ? 1 : 0] = true;
  }
  if (inverse)
    hipLaunchKernelGGL(ntt_kernel<true>, dim3((unsigned)blocks), dim3(threads), lds, s, R, c->dp);
  else
    hipLaunchKernelGGL(ntt_kernel<false>, dim3((unsigned)blocks), dim3(threads), lds, s, R, c->dp);
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

__global__ void zero_kernel(u64* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0;
}

int launch_zero(u64* p, int64_t n, hipStream_t s) {
  if (n <= 0) return SFHE_OK;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

// ---- layout conversions (limb-major rows <-> chunked matrix layout) ----
__global__ void to_chunked_kernel(const u64* src, int64_t sstride, int nl, int64_t count, u64* dst, int64_t n_ct,
                                  const int64_t* elem, int64_t elem_base, int N) {
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;   // (x, p, i)
  if (row >= count * 2 * nl) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t x = row / (2 * nl);
  const int pi = (int)(row % (2 * nl));
  const int p = pi / nl, i = pi % nl;
  const int64_t e = elem ? elem[x] : elem_base + x;
  dst[chunk_index(e, p, i, t, n_ct, N >> 6)] = src[x * sstride + (int64_t)pi * N + t];
}
__global__ void from_chunked_kernel(const u64* src, int64_t n_ct, int nl, int64_t count, const int64_t* elem,
                                    int64_t elem_base, u64* dst, int64_t dstride, int N) {
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;
  if (row >= count * 2 * nl) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t x = row / (2 * nl);
  const int pi = (int)(row % (2 * nl));
  const int p = pi / nl, i = pi % nl;
  const int64_t e = elem ? elem[x] : elem_base + x;
  dst[x * dstride + (int64_t)pi * N + t] = src[chunk_index(e, p, i, t, n_ct, N >> 6)];
}

static void grid_rows(int64_t rows, unsigned& gy, unsigned& gz) {
  if (rows < 1) rows = 1;
  gy = rows < 65535 ? (unsigned)rows : 65535u;
  gz = (unsigned)((rows + gy - 1) / gy);
}

int launch_to_chunked(const sfhe_ctx* c, const u64* src, int64_t sstride, int nl, int64_t count, u64* dst,
                      int64_t n_ct, const int64_t* elem, int64_t elem_base, hipStream_t s) {
  if (count <= 0) return SFHE_OK;
  unsigned gy, gz;
  grid_rows(count * 2 * nl, gy, gz);
  hipLaunchKernelGGL(to_chunked_kernel, dim3((c->N + 255) / 256, gy, gz), dim3(256), 0, s, src, sstride, nl, count,
                     dst, n_ct, elem, elem_base, c->N);
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

int launch_from_chunked(const sfhe_ctx* c, const u64* src, int64_t n_ct, int nl, int64_t count, const int64_t* elem,
                        int64_t elem_base, u64* dst, int64_t dstride, hipStream_t s) {
  if (count <= 0) return SFHE_OK;
  unsigned gy, gz;
  grid_rows(count * 2 * nl, gy, gz);
  hipLaunchKernelGGL(from_chunked_kernel, dim3((c->N + 255) / 256, gy, gz), dim3(256), 0, s, src, n_ct, nl, count,
                     elem, elem_base, dst, dstride, c->N);
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

}  // namespace sfhe
