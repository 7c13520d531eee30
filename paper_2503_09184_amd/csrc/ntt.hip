// ntt.hip -- batched negacyclic NTT / inverse NTT for gfx950.
//
// One workgroup transforms one row of N residues held entirely in LDS
// (N <= 2^14: 128 KiB of the 160 KiB per CU).  Forward: Cooley-Tukey with the
// psi twist merged into the twiddles (Longa and Naehrig 2016), bit-reversed
// output, so index k holds a(psi^(2*brv(k)+1)).  Inverse: Gentleman-Sande with
// N^-1 applied at the end.  Butterflies are Harvey's lazy ones (2014): values
// stay in [0, 4q) (forward) or [0, 2q) (inverse) between stages, the constant
// twiddle products use Shoup quotients, and only the final store reduces to
// [0, q).
#include "internal.hpp"

namespace sfhe {

constexpr int kMaxRows = 2 * kMaxBasis;   // rows per group: both polys of a ciphertext

struct NttRows {
  u64* base;
  int64_t bstride;
  int nrow;
  int pos[kMaxRows];
  int prime[kMaxRows];
};

template <bool INV>
__global__ void __launch_bounds__(1024) ntt_lds_kernel(NttRows R, DevParams dp) {
  extern __shared__ u64 sh[];
  const int N = dp.N, logN = dp.logN;
  const int64_t g = blockIdx.x / R.nrow;
  const int r = blockIdx.x % R.nrow;
  u64* p = R.base + g * R.bstride + (int64_t)R.pos[r] * N;
  const PrimeDev& P = dp.pr[R.prime[r]];
  const u64 q = P.q, q2 = 2 * q;
  const int T = blockDim.x;
  const int half = N >> 1;

  for (int x = threadIdx.x; x < N; x += T) sh[x] = p[x];
  __syncthreads();

  if (!INV) {
    for (int lm = 0; lm < logN; ++lm) {        // m = 2^lm groups, t = N / 2m
      const int lt = logN - 1 - lm;
      const int t = 1 << lt;
      const int m = 1 << lm;
      for (int bf = threadIdx.x; bf < half; bf += T) {
        const int i = bf >> lt, j = bf & (t - 1);
        const int i1 = (i << (lt + 1)) + j, i2 = i1 + t;
        const u64 W = P.tw[m + i], Ws = P.tws[m + i];
        u64 X = sh[i1];
        const u64 Y = sh[i2];
        X = X >= q2 ? X - q2 : X;
        const u64 Tm = mul_shoup_lazy(Y, W, Ws, q);
        sh[i1] = X + Tm;
        sh[i2] = X - Tm + q2;
      }
      __syncthreads();
    }
    for (int x = threadIdx.x; x < N; x += T) {
      u64 v = sh[x];
      v = v >= q2 ? v - q2 : v;
      v = v >= q ? v - q : v;
      p[x] = v;
    }
  } else {
    for (int lm = logN - 1; lm >= 0; --lm) {   // h = 2^lm groups, t = N / 2h
      const int lt = logN - 1 - lm;
      const int t = 1 << lt;
      const int h = 1 << lm;
      for (int bf = threadIdx.x; bf < half; bf += T) {
        const int i = bf >> lt, j = bf & (t - 1);
        const int i1 = (i << (lt + 1)) + j, i2 = i1 + t;
        const u64 W = P.itw[h + i], Ws = P.itws[h + i];
        const u64 X = sh[i1], Y = sh[i2];
        u64 S = X + Y;
        S = S >= q2 ? S - q2 : S;
        sh[i1] = S;
        sh[i2] = mul_shoup_lazy(X - Y + q2, W, Ws, q);
      }
      __syncthreads();
    }
    for (int x = threadIdx.x; x < N; x += T) {
      u64 v = mul_shoup_lazy(sh[x], P.ninv, P.ninv_s, q);
      p[x] = v >= q ? v - q : v;
    }
  }
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
  const int threads = N / 2 < 1024 ? N / 2 : 1024;
  const size_t lds = (size_t)N * sizeof(u64);
  const int64_t blocks = batch * nrow;
  if (blocks > 0x7FFFFFFF) { set_error("ntt: batch too large"); return SFHE_E_INVALID_ARG; }
  static bool attr_done[2] = {false, false};
  if (!attr_done[inverse ? 1 : 0]) {
    const void* fn = inverse ? reinterpret_cast<const void*>(&ntt_lds_kernel<true>)
                             : reinterpret_cast<const void*>(&ntt_lds_kernel<false>);
    SFHE_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    attr_done[inverse ? 1 : 0] = true;
  }
  if (inverse)
    hipLaunchKernelGGL(ntt_lds_kernel<true>, dim3((unsigned)blocks), dim3(threads), lds, s, R, c->dp);
  else
    hipLaunchKernelGGL(ntt_lds_kernel<false>, dim3((unsigned)blocks), dim3(threads), lds, s, R, c->dp);
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
