// tensor.hip -- ciphertext tensor products in the NTT domain (the multiply
// step of Algorithm 1): d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1 per prime
// and coefficient.
//
// The lazy form sums the tensors of every visited k of an output before any
// reduction: 128-bit accumulators (each product < 2^122, folded every 32
// products), one Barrett reduction at the end.  The visited k come straight
// from the left operand's plaintext structure (Sec. 3.3.2): every k (naive
// dense), the k whose zero-mask bit is clear (naive sparse), the CSR column
// list of the row, or the row's ELLPACK columns other than -1.
#include "internal.hpp"

namespace sfhe {

__device__ __forceinline__ void fold(U128& a, const PrimeDev& P) { a = U128{reduce_wide(a, P.q, P.mu_hi, P.mu_lo), 0}; }

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

// gathered: product x multiplies A ciphertext aidx[x] by B ciphertext bidx[x] (top level, L limbs)
__global__ void tensor_gather_kernel(int nl, const u64* A, const u64* B, const int* aidx, const int* bidx, u64* d,
                                     int64_t count, DevParams dp) {
  const int N = dp.N;
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;
  if (row >= count * nl) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t x = row / nl;
  const int l = (int)(row % nl);
  const PrimeDev& P = dp.pr[l];
  const int64_t cts = (int64_t)2 * nl * N;
  const u64* ax = A + (int64_t)aidx[x] * cts;
  const u64* bx = B + (int64_t)bidx[x] * cts;
  const u64 a0 = ax[(int64_t)l * N + t], a1 = ax[(int64_t)(nl + l) * N + t];
  const u64 b0 = bx[(int64_t)l * N + t], b1 = bx[(int64_t)(nl + l) * N + t];
  U128 m = mul_wide(a0, b1);
  add_wide(m, mul_wide(a1, b0));
  u64* dx = d + x * (int64_t)3 * nl * N;
  dx[(int64_t)l * N + t] = mul_mod(a0, b0, P);
  dx[(int64_t)(nl + l) * N + t] = reduce_wide(m, P.q, P.mu_hi, P.mu_lo);
  dx[(int64_t)(2 * nl + l) * N + t] = mul_mod(a1, b1, P);
}

// ---- the left operand's visiting order, per encoding ----
struct LeftStruct {
  int K, cols_b;
  const int* row_ptr;    // CSR
  const int* col_idx;
  const int* ell_col;    // ELL
  int ell_w;
  const uint32_t* mask;  // naive sparse
};

template <int ENC>
struct RowIter;

template <>
struct RowIter<SFHE_ENC_DENSE> {
  int i, n, pos;
  const LeftStruct& S;
  __device__ RowIter(const LeftStruct& s, int row) : i(row), n(s.K), pos(0), S(s) {}
  __device__ bool next(int& k, int64_t& aslot) {
    if (pos >= n) return false;
    k = pos;
    aslot = (int64_t)i * S.K + pos;
    ++pos;
    return true;
  }
};

template <>
struct RowIter<SFHE_ENC_NAIVE_SPARSE> {
  int i, pos;
  const LeftStruct& S;
  __device__ RowIter(const LeftStruct& s, int row) : i(row), pos(0), S(s) {}
  __device__ bool next(int& k, int64_t& aslot) {
    while (pos < S.K) {
      const int64_t e = (int64_t)i * S.K + pos;
      const bool zero = (S.mask[e >> 5] >> (e & 31)) & 1u;
      ++pos;
      if (!zero) { k = pos - 1; aslot = e; return true; }
    }
    return false;
  }
};

template <>
struct RowIter<SFHE_ENC_CSR> {
  int p, end;
  const LeftStruct& S;
  __device__ RowIter(const LeftStruct& s, int row) : p(s.row_ptr[row]), end(s.row_ptr[row + 1]), S(s) {}
  __device__ bool next(int& k, int64_t& aslot) {
    if (p >= end) return false;
    k = S.col_idx[p];
    aslot = p;
    ++p;
    return true;
  }
};

template <>
struct RowIter<SFHE_ENC_ELL> {
  int i, s;
  const LeftStruct& S;
  __device__ RowIter(const LeftStruct& st, int row) : i(row), s(0), S(st) {}
  __device__ bool next(int& k, int64_t& aslot) {
    while (s < S.ell_w) {
      const int64_t e = (int64_t)i * S.ell_w + s;
      const int kk = S.ell_col[e];
      ++s;
      if (kk >= 0) { k = kk; aslot = e; return true; }
    }
    return false;
  }
};

// one block = one output (oi, oj), one prime l, 256 coefficients
template <int ENC>
__global__ void __launch_bounds__(256) tensor_lazy_kernel(LeftStruct S, const u64* A, const u64* B, const int* oi,
                                                          const int* oj, int64_t count, u64* d, DevParams dp) {
  const int N = dp.N, L = dp.L;
  const int64_t o = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;
  if (o >= count) return;
  const int tiles = N / 256;
  const int l = blockIdx.x / tiles;
  const int t = (blockIdx.x % tiles) * 256 + threadIdx.x;
  const PrimeDev& P = dp.pr[l];
  const int i = oi[o], j = oj[o];
  const int64_t cts = (int64_t)2 * L * N;
  U128 s0{0, 0}, s1{0, 0}, s2{0, 0};
  RowIter<ENC> it(S, i);
  int k;
  int64_t aslot;
  int n = 0;
  while (it.next(k, aslot)) {
    const u64* a = A + aslot * cts + (int64_t)l * N + t;
    const u64* b = B + ((int64_t)k * S.cols_b + j) * cts + (int64_t)l * N + t;
    const u64 a0 = a[0], a1 = a[(int64_t)L * N];
    const u64 b0 = b[0], b1 = b[(int64_t)L * N];
    add_wide(s0, mul_wide(a0, b0));
    add_wide(s1, mul_wide(a0, b1));
    add_wide(s1, mul_wide(a1, b0));
    add_wide(s2, mul_wide(a1, b1));
    if ((++n & 31) == 0) { fold(s0, P); fold(s1, P); fold(s2, P); }   // sums stay below 2^128
  }
  u64* dx = d + o * (int64_t)3 * L * N + (int64_t)l * N + t;
  dx[0] = reduce_wide(s0, P.q, P.mu_hi, P.mu_lo);
  dx[(int64_t)L * N] = reduce_wide(s1, P.q, P.mu_hi, P.mu_lo);
  dx[(int64_t)2 * L * N] = reduce_wide(s2, P.q, P.mu_hi, P.mu_lo);
}

// rows >= 1 (callers return early on empty work)
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

int launch_tensor_gather(const sfhe_ctx* c, int lev, const u64* A, const u64* B, const int* d_aidx,
                         const int* d_bidx, u64* d, int64_t count, hipStream_t s) {
  if (count <= 0) return SFHE_OK;
  const int nl = lev + 1;
  unsigned gy, gz;
  grid_rows(count * nl, gy, gz);
  hipLaunchKernelGGL(tensor_gather_kernel, dim3((c->N + 255) / 256, gy, gz), dim3(256), 0, s, nl, A, B, d_aidx,
                     d_bidx, d, count, c->dp);
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

int launch_tensor_lazy(const sfhe_ctx* c, const sfhe_mat* A, const sfhe_mat* B, const int* d_oi, const int* d_oj,
                       int64_t count, u64* d, hipStream_t s) {
  if (count <= 0) return SFHE_OK;
  LeftStruct S;
  S.K = A->cols;
  S.cols_b = B->cols;
  S.row_ptr = A->d_row_ptr.ptr;
  S.col_idx = A->d_col_idx.ptr;
  S.ell_col = A->d_ell_col.ptr;
  S.ell_w = A->ell_w;
  S.mask = A->d_mask.ptr;
  unsigned gy, gz;
  grid_rows(count, gy, gz);
  dim3 grid((unsigned)((c->N / 256) * c->L), gy, gz);
  switch (A->enc) {
    case SFHE_ENC_DENSE:
      hipLaunchKernelGGL(tensor_lazy_kernel<SFHE_ENC_DENSE>, grid, dim3(256), 0, s, S, A->data.ptr, B->data.ptr, d_oi,
                         d_oj, count, d, c->dp);
      break;
    case SFHE_ENC_NAIVE_SPARSE:
      hipLaunchKernelGGL(tensor_lazy_kernel<SFHE_ENC_NAIVE_SPARSE>, grid, dim3(256), 0, s, S, A->data.ptr,
                         B->data.ptr, d_oi, d_oj, count, d, c->dp);
      break;
    case SFHE_ENC_CSR:
      hipLaunchKernelGGL(tensor_lazy_kernel<SFHE_ENC_CSR>, grid, dim3(256), 0, s, S, A->data.ptr, B->data.ptr, d_oi,
                         d_oj, count, d, c->dp);
      break;
    case SFHE_ENC_ELL:
      hipLaunchKernelGGL(tensor_lazy_kernel<SFHE_ENC_ELL>, grid, dim3(256), 0, s, S, A->data.ptr, B->data.ptr, d_oi,
                         d_oj, count, d, c->dp);
      break;
  }
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

}  // namespace sfhe
