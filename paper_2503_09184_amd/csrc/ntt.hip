// ntt.hip -- batched negacyclic NTT / inverse NTT kernels (one workgroup
// per row: the 32-residues-per-thread transform of ntt14.hpp for N = 2^14,
// the radix-16 transform of ntt_core.hpp for smaller rings), and layout
// helpers.
#include "ntt14.hpp"

namespace sfhe {

// storage position x of an N = 2^14 row -> the NTT index it holds (the
// register-major order of the 2^14 transform kernels)
__device__ __forceinline__ int ord14(int x) {
  const int r = x >> 9, t = x & 511;
  return ((r >> 4) << 13) | ((t & 63) << 4) | (((t >> 6) & 1) << 10) | (((t >> 8) & 1) << 11) |
         (((t >> 7) & 1) << 12) | (r & 15);
}

// The LDS transform with passes of at most PMAX stages (radix 2^PMAX); at
// N = 2^14 its NTT-domain side is read and written in the 2^14 kernels'
// storage order, so that either design can serve a ring.
template <bool INV, int PMAX, typename Ar>
__device__ __forceinline__ void ntt_row(u64* p, const PrimeDev& P, int N, int logN, void* lds) {
  typedef typename Ar::Val Val;
  Val* sh = reinterpret_cast<Val*>(lds);
  const Ar ar(P, INV);
  const bool perm = logN == 14;
  if (!INV) {
    int s0 = 0;
    while (s0 < logN) {
      const int np = min(PMAX, logN - s0);
      const u64* src = s0 == 0 ? p : nullptr;
      if (np == 4) fwd_pass<4>(ar, sh, src, N, logN, s0);
      else if (np == 3) fwd_pass<3>(ar, sh, src, N, logN, s0);
      else if (np == 2) fwd_pass<2>(ar, sh, src, N, logN, s0);
      else fwd_pass<1>(ar, sh, src, N, logN, s0);
      __syncthreads();
      s0 += np;
    }
    for (int x = threadIdx.x; x < N; x += blockDim.x) p[x] = ar.out_fwd(sh[lpos(perm ? ord14(x) : x)]);
  } else {
    for (int x = threadIdx.x; x < N; x += blockDim.x) sh[lpos(perm ? ord14(x) : x)] = ar.in(p[x]);
    __syncthreads();
    int lt0 = 0;
    while (lt0 < logN) {
      const int np = min(PMAX, logN - lt0);
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

template <bool INV, int PMAX>
__global__ void __launch_bounds__(1024) ntt_kernel(NttRows R, DevParams dp) {
  extern __shared__ u64 lds[];
  const int N = dp.N, logN = dp.logN;
  const int64_t g = blockIdx.x / R.nrow;
  const int r = blockIdx.x % R.nrow;
  u64* p = R.base + g * R.bstride + (int64_t)R.pos[r] * N;
  const PrimeDev& P = dp.pr[R.prime[r]];
  if (P.q < (1ull << 42))
    ntt_row<INV, PMAX, NttFp>(p, P, N, logN, lds);
  else
    ntt_row<INV, PMAX, NttInt>(p, P, N, logN, lds);
}


// one row of 2^14 residues in place: coefficients in natural order, the NTT
// domain in the register-major order of ntt14.hpp
template <bool INV, typename Ar>
__device__ __forceinline__ void ntt14_row(u64* p, const PrimeDev& P, void* lds) {
  typedef typename Ar::Val Val;
  Val* sh = reinterpret_cast<Val*>(lds);
  const int t = threadIdx.x;
  const Ar ar(P, INV);
  Val v[32];
  if (!INV) {
    const u64* src = p + n14::xa(n14::opaque(t), 0);
#pragma unroll
    for (int u = 0; u < 32; ++u) v[u] = ar.in(src[n14::off_a(u)]);
    n14::forward(ar, v, sh, t);
#pragma unroll
    for (int r = 0; r < 32; ++r) p[n14::pos_c(t, r)] = ar.out_fwd(v[r]);
  } else {
#pragma unroll
    for (int r = 0; r < 32; ++r) v[r] = ar.in(p[n14::pos_c(t, r)]);
    n14::inverse(ar, v, sh, t);
    u64* dst = p + n14::xa(n14::opaque(t), 0);
#pragma unroll
    for (int u = 0; u < 32; ++u) dst[n14::off_a(u)] = ar.out_inv(v[u], P);
  }
}

template <bool INV>
__global__ void __launch_bounds__(n14::kThreads, 4) ntt14_kernel(NttRows R, DevParams dp) {
  extern __shared__ u64 lds[];
  const int64_t g = blockIdx.x / R.nrow;
  const int r = blockIdx.x % R.nrow;
  u64* p = R.base + g * R.bstride + (int64_t)R.pos[r] * n14::kN;
  const PrimeDev& P = dp.pr[R.prime[r]];
  if (P.q < (1ull << 42))
    ntt14_row<INV, NttFp>(p, P, lds);
  else
    ntt14_row<INV, NttInt>(p, P, lds);
}

// ---- N = 2^15: the first forward stage (last inverse stage) across the two
// halves, then each half as a 2^14-point transform with its own tables ----
// grid (2^14 / 256, rows): x_i, x_{i + 2^14} -> x_i + w x_{i+2^14}, x_i - w x_{i+2^14}
__global__ void __launch_bounds__(256) ntt15_first_kernel(NttRows R, int64_t rows, DevParams dp) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;
  if (row >= rows) return;
  const int64_t g = row / R.nrow;
  const int r = (int)(row % R.nrow);
  u64* p = R.base + g * R.bstride + (int64_t)R.pos[r] * (2 * n14::kN);
  const PrimeDev& P = dp.pr[R.prime[r]];
  const u64 q = P.q;
  const u64 a = p[i], T = mul_shoup(p[i + n14::kN], P.tw[1], P.tws[1], q);
  p[i] = add_mod(a, T, q);
  p[i + n14::kN] = sub_mod(a, T, q);
}
// x_i, x_{i + 2^14} -> x_i + x_{i+2^14}, (x_i - x_{i+2^14}) w^-1 (N^-1 is
// applied by the halves' transforms)
__global__ void __launch_bounds__(256) ntt15_last_kernel(NttRows R, int64_t rows, DevParams dp) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;
  if (row >= rows) return;
  const int64_t g = row / R.nrow;
  const int r = (int)(row % R.nrow);
  u64* p = R.base + g * R.bstride + (int64_t)R.pos[r] * (2 * n14::kN);
  const PrimeDev& P = dp.pr[R.prime[r]];
  const u64 q = P.q;
  const u64 a = p[i], b = p[i + n14::kN];
  p[i] = add_mod(a, b, q);
  p[i + n14::kN] = mul_shoup(sub_mod(a, b, q), P.itw[1], P.itws[1], q);
}
// one half of a row (block = (row, half)) as a 2^14-point transform
template <bool INV>
__global__ void __launch_bounds__(n14::kThreads, 4) ntt15_half_kernel(NttRows R, DevParams dp) {
  extern __shared__ u64 lds[];
  const int64_t g = (blockIdx.x >> 1) / R.nrow;
  const int r = (blockIdx.x >> 1) % R.nrow, h = blockIdx.x & 1;
  u64* p = R.base + g * R.bstride + (int64_t)R.pos[r] * (2 * n14::kN) + (int64_t)h * n14::kN;
  const int pr = R.prime[r];
  PrimeDev P = dp.pr[pr];
  const int64_t fo = (((int64_t)pr * 2 + 0) * 2 + h) * n14::kN, io = (((int64_t)pr * 2 + 1) * 2 + h) * n14::kN;
  P.tw = R.sub + fo;
  P.tws = R.sub_s + fo;
  P.twd = R.subd + fo;
  P.itw = R.sub + io;
  P.itws = R.sub_s + io;
  P.itwd = R.subd + io;
  if (P.q < (1ull << 42))
    ntt14_row<INV, NttFp>(p, P, lds);
  else
    ntt14_row<INV, NttInt>(p, P, lds);
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
  R.sub = c->d_sub.ptr;
  R.sub_s = c->d_sub_s.ptr;
  R.subd = c->d_sub_d.ptr;
  const int N = c->N;
  const int64_t blocks = batch * nrow;
  if (blocks > 0x7FFFFFFF / 2) { set_error("ntt: batch too large"); return SFHE_E_INVALID_ARG; }
  if (c->logN == n14::kLogN + 1) {
    static bool attr15 = false;
    if (!attr15) {
      SFHE_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&ntt15_half_kernel<false>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, n14::kLdsWords * 8));
      SFHE_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&ntt15_half_kernel<true>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, n14::kLdsWords * 8));
      attr15 = true;
    }
    const size_t lds = (size_t)n14::kLdsWords * sizeof(u64);
    // element-wise grid: (2^14 / 256, rows split over y and z)
    const unsigned gy = blocks < 65535 ? (unsigned)blocks : 65535u;
    const dim3 ew(n14::kN / 256, gy, (unsigned)((blocks + gy - 1) / gy));
    if (!inverse) {
      hipLaunchKernelGGL(ntt15_first_kernel, ew, dim3(256), 0, s, R, blocks, c->dp);
      SFHE_HIP(hipGetLastError());
      hipLaunchKernelGGL(ntt15_half_kernel<false>, dim3((unsigned)(2 * blocks)), dim3(n14::kThreads), lds, s, R, c->dp);
    } else {
      hipLaunchKernelGGL(ntt15_half_kernel<true>, dim3((unsigned)(2 * blocks)), dim3(n14::kThreads), lds, s, R, c->dp);
      SFHE_HIP(hipGetLastError());
      hipLaunchKernelGGL(ntt15_last_kernel, ew, dim3(256), 0, s, R, blocks, c->dp);
    }
    SFHE_HIP(hipGetLastError());
    return SFHE_OK;
  }
  const int var = c->ntt_var[inverse ? 1 : 0];
  if (c->logN == n14::kLogN && var == kNttRegister) {
    static bool attr14 = false;
    if (!attr14) {
      SFHE_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&ntt14_kernel<false>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, n14::kLdsWords * 8));
      SFHE_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&ntt14_kernel<true>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, n14::kLdsWords * 8));
      attr14 = true;
    }
    const size_t lds = (size_t)n14::kLdsWords * sizeof(u64);
    if (inverse)
      hipLaunchKernelGGL(ntt14_kernel<true>, dim3((unsigned)blocks), dim3(n14::kThreads), lds, s, R, c->dp);
    else
      hipLaunchKernelGGL(ntt14_kernel<false>, dim3((unsigned)blocks), dim3(n14::kThreads), lds, s, R, c->dp);
    SFHE_HIP(hipGetLastError());
    return SFHE_OK;
  }
  // the LDS designs: radix 16, 8 or 4 passes, one thread per 2^PMAX residues
  const int pmax = var == kNttRadix8 ? 3 : var == kNttRadix4 ? 2 : 4;
  const int threads = std::min(N >> pmax, 1024);
  const size_t lds = (size_t)(N + (N >> kPadShift)) * sizeof(u64);
  static bool attr_done = false;
  if (!attr_done) {
    const void* fns[6] = {reinterpret_cast<const void*>(&ntt_kernel<false, 4>), reinterpret_cast<const void*>(&ntt_kernel<true, 4>),
                          reinterpret_cast<const void*>(&ntt_kernel<false, 3>), reinterpret_cast<const void*>(&ntt_kernel<true, 3>),
                          reinterpret_cast<const void*>(&ntt_kernel<false, 2>), reinterpret_cast<const void*>(&ntt_kernel<true, 2>)};
    for (const void* fn : fns) SFHE_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    attr_done = true;
  }
#define SFHE_NTT_LAUNCH(I, PM) hipLaunchKernelGGL((ntt_kernel<I, PM>), dim3((unsigned)blocks), dim3(threads), lds, s, R, c->dp)
  if (pmax == 4) { if (inverse) SFHE_NTT_LAUNCH(true, 4); else SFHE_NTT_LAUNCH(false, 4); }
  else if (pmax == 3) { if (inverse) SFHE_NTT_LAUNCH(true, 3); else SFHE_NTT_LAUNCH(false, 3); }
  else { if (inverse) SFHE_NTT_LAUNCH(true, 2); else SFHE_NTT_LAUNCH(false, 2); }
#undef SFHE_NTT_LAUNCH
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
