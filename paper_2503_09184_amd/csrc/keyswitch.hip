// keyswitch.hip -- relinearisation (hybrid key switching) and rescaling,
// the second and third steps of every ciphertext product in Algorithm 1.
//
// Key switching of a degree-2 part d2 at level lev (Q = q_0..q_lev, special
// primes P = p_0..p_{alpha-1}, digits of alpha consecutive data primes):
//   ModUp     per digit j, the centered fast base conversion of [d2]_{D_j}
//             to every other prime of Q and P, then the NTT of those rows;
//   inner     acc_p = sum_j x_j * rlk_j.p over Q u P (NTT domain);
//   ModDown   the special rows of acc back to coefficients, their centered
//             fast base conversion to Q, NTT, and (acc_i - z_i) P^-1.
// Rescale drops q_lev with exact rounding: r = centered lift of the last row,
// c_i' = (c_i - r) q_lev^-1.  Base conversions run in the coefficient domain,
// products with the key in the NTT domain.
#include "internal.hpp"

namespace sfhe {

// rows >= 1 (callers return early on empty work)
static void grid_rows(int64_t rows, unsigned& gy, unsigned& gz) {
  if (rows < 1) rows = 1;
  gy = rows < 65535 ? (unsigned)rows : 65535u;
  gz = (unsigned)((rows + gy - 1) / gy);
}

// xbuf[b][e][t] for the targets e outside the digit (coefficient domain)
__global__ void modup_kernel(const u64* d2c, int nl, const ModUpConst* __restrict__ mc, u64* xbuf, int64_t batch,
                             DevParams dp) {
  const int N = dp.N;
  const int64_t b = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;
  if (b >= batch) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int lo = mc->lo, hi = mc->hi, ne = mc->ne;
  u64 y[kMaxDigit];
  u64 neg = 0;   // centered conversion: residues above (q_i - 1) / 2 stand for y_i - q_i
#pragma unroll
  for (int i = 0; i < kMaxDigit; ++i) {
    if (lo + i < hi) {
      const u64 qi = dp.pr[lo + i].q;
      y[i] = mul_shoup(d2c[(b * nl + lo + i) * N + t], mc->inv[i], mc->inv_s[i], qi);
      neg += y[i] > (qi - 1) / 2;
    } else {
      y[i] = 0;
    }
  }
  for (int e = 0; e < ne; ++e) {
    const int r = mc->basis[e];
    if (r >= lo && r < hi) continue;
    const u64 qe = dp.pr[r].q;
    u64 acc = 0;
#pragma unroll
    for (int i = 0; i < kMaxDigit; ++i) {
      if (lo + i < hi) acc = add_mod(acc, mul_shoup(y[i], mc->conv[i][e], mc->conv_s[i][e], qe), qe);
    }
    xbuf[(b * ne + e) * N + t] = sub_mod(acc, mul_shoup(neg, mc->dmod[e], mc->dmod_s[e], qe), qe);
  }
}

// acc[b][p][e][t] (+)= x_j[e] * rlk_j.p[basis e]; x_j[e] is d2 itself on the digit's primes
__global__ void ks_inner_kernel(const u64* d2n, int64_t d2stride, const u64* xbuf, u64* acc, int j, bool first,
                                const ModUpConst* __restrict__ mc, const u64* rlk, DevParams dp, int64_t batch) {
  const int N = dp.N, nb = dp.nb;
  const int ne = mc->ne;
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;   // (b, e)
  if (row >= batch * ne) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t b = row / ne;
  const int e = (int)(row % ne);
  const int r = mc->basis[e];
  const PrimeDev& P = dp.pr[r];
  const u64 x = (r >= mc->lo && r < mc->hi) ? d2n[b * d2stride + (int64_t)r * N + t] : xbuf[(b * ne + e) * N + t];
  const u64 kb = rlk[(((int64_t)j * 2 + 0) * nb + r) * N + t];
  const u64 ka = rlk[(((int64_t)j * 2 + 1) * nb + r) * N + t];
  u64* a0 = acc + ((b * 2 + 0) * ne + e) * N + t;
  u64* a1 = acc + ((b * 2 + 1) * ne + e) * N + t;
  const u64 v0 = mul_mod(x, kb, P), v1 = mul_mod(x, ka, P);
  if (first) {
    *a0 = v0;
    *a1 = v1;
  } else {
    *a0 = add_mod(*a0, v0, P.q);
    *a1 = add_mod(*a1, v1, P.q);
  }
}

// z[b][p][i][t] = sum_k y_k [P/p_k]_{q_i}, y_k = [acc_{p_k} (P/p_k)^-1]_{p_k}
// centered (coefficient domain)
__global__ void moddown_kernel(const u64* acc, int nl, int ne, u64* z, const ModDownConst* __restrict__ md,
                               int64_t batch, DevParams dp) {
  const int N = dp.N, alpha = dp.alpha, L = dp.L;
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;   // (b, p)
  if (row >= batch * 2) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  u64 y[kMaxDigit];
  u64 neg = 0;   // residues above (p_k - 1) / 2: they stand for y_k - p_k
#pragma unroll
  for (int k = 0; k < kMaxDigit; ++k) {
    if (k < alpha) {
      const u64 pk = dp.pr[L + k].q;
      y[k] = mul_shoup(acc[(row * ne + nl + k) * N + t], md->pinv[k], md->pinv_s[k], pk);
      neg += y[k] > (pk - 1) / 2;
    } else {
      y[k] = 0;
    }
  }
  for (int i = 0; i < nl; ++i) {
    const u64 qi = dp.pr[i].q;
    u64 s = 0;
#pragma unroll
    for (int k = 0; k < kMaxDigit; ++k)
      if (k < alpha) s = add_mod(s, mul_shoup(y[k], md->conv[k][i], md->conv_s[k][i], qi), qi);
    z[(row * nl + i) * N + t] = sub_mod(s, mul_mod(neg, md->Pq[i], dp.pr[i]), qi);
  }
}

// out[b][p][i] (+)= (acc_i - z_i) P^-1  (NTT domain)
__global__ void moddown_finish_kernel(const u64* acc, int nl, int ne, const u64* z, u64* out, int64_t ostride,
                                      bool add_in, const ModDownConst* __restrict__ md, int64_t batch,
                                      DevParams dp) {
  const int N = dp.N;
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;   // (b, p, i)
  if (row >= batch * 2 * nl) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t b = row / (2 * nl);
  const int rem = (int)(row % (2 * nl));
  const int p = rem / nl, i = rem % nl;
  const u64 qi = dp.pr[i].q;
  const u64 a = acc[((b * 2 + p) * ne + i) * N + t];
  const u64 zz = z[((b * 2 + p) * nl + i) * N + t];
  const u64 v = mul_shoup(sub_mod(a, zz, qi), md->Pinv[i], md->Pinv_s[i], qi);
  u64* o = out + b * ostride + ((int64_t)p * nl + i) * N + t;
  *o = add_in ? add_mod(*o, v, qi) : v;
}

int keyswitch_batch(sfhe_ctx* c, int lev, const u64* d2, int64_t d2stride, u64* out, int64_t ostride, bool add_in,
                    int64_t batch, hipStream_t s, const u64* key, u64* scratch) {
  if (batch <= 0) return SFHE_OK;
  if (!key) key = c->d_rlk.ptr;
  const int N = c->N, nl = lev + 1, ne = nl + c->alpha;
  // working rows: d2 in coefficients, one raised digit, the key products
  // over Q and P, the ModDown conversion (every word is written before it
  // is read, so a reused scratch needs no clearing)
  DevBuf<u64> d2c_b, xbuf_b, acc_b, z_b;
  struct { u64* ptr; } d2c{}, xbuf{}, acc{}, z{};
  if (scratch) {
    d2c.ptr = scratch;
    xbuf.ptr = d2c.ptr + (size_t)batch * nl * N;
    acc.ptr = xbuf.ptr + (size_t)batch * ne * N;
    z.ptr = acc.ptr + (size_t)batch * 2 * ne * N;
  } else {
    if (!d2c_b.alloc(&c->alloc, (size_t)batch * nl * N) || !xbuf_b.alloc(&c->alloc, (size_t)batch * ne * N) ||
        !acc_b.alloc(&c->alloc, (size_t)batch * 2 * ne * N) || !z_b.alloc(&c->alloc, (size_t)batch * 2 * nl * N)) {
      set_error("keyswitch: device allocation failed");
      return SFHE_E_NOMEM;
    }
    d2c.ptr = d2c_b.ptr;
    xbuf.ptr = xbuf_b.ptr;
    acc.ptr = acc_b.ptr;
    z.ptr = z_b.ptr;
  }
  // coefficient-domain copy of d2
  SFHE_HIP(hipMemcpy2DAsync(d2c.ptr, (size_t)nl * N * sizeof(u64), d2, (size_t)d2stride * sizeof(u64),
                            (size_t)nl * N * sizeof(u64), (size_t)batch, hipMemcpyDeviceToDevice, s));
  int pos[2 * kMaxBasis], pr[2 * kMaxBasis];
  for (int r = 0; r < nl; ++r) { pos[r] = r; pr[r] = r; }
  int rc = launch_ntt(c, d2c.ptr, batch, (int64_t)nl * N, nl, pos, pr, true, s);
  if (rc) return rc;
  unsigned gy, gz;
  bool first = true;
  for (int j = 0; j < c->dnum; ++j) {
    if (j * c->alpha >= nl) break;
    const ModUpConst* mc = c->d_modup.ptr + (size_t)lev * c->dnum + j;
    grid_rows(batch, gy, gz);
    hipLaunchKernelGGL(modup_kernel, dim3((N + 255) / 256, gy, gz), dim3(256), 0, s, d2c.ptr, nl, mc, xbuf.ptr, batch,
                       c->dp);
    SFHE_HIP(hipGetLastError());
    // NTT of the converted rows
    const int lo = j * c->alpha, hi = std::min((j + 1) * c->alpha, nl);
    int np = 0;
    for (int e = 0; e < ne; ++e) {
      const int r = e < nl ? e : c->L + (e - nl);
      if (r >= lo && r < hi) continue;
      pos[np] = e;
      pr[np] = r;
      ++np;
    }
    rc = launch_ntt(c, xbuf.ptr, batch, (int64_t)ne * N, np, pos, pr, false, s);
    if (rc) return rc;
    grid_rows(batch * ne, gy, gz);
    hipLaunchKernelGGL(ks_inner_kernel, dim3((N + 255) / 256, gy, gz), dim3(256), 0, s, d2, d2stride, xbuf.ptr,
                       acc.ptr, j, first, mc, key, c->dp, batch);
    SFHE_HIP(hipGetLastError());
    first = false;
  }
  // ModDown: special rows back to coefficients
  int np = 0;
  for (int p = 0; p < 2; ++p)
    for (int k = 0; k < c->alpha; ++k) { pos[np] = p * ne + nl + k; pr[np] = c->L + k; ++np; }
  rc = launch_ntt(c, acc.ptr, batch, (int64_t)2 * ne * N, np, pos, pr, true, s);
  if (rc) return rc;
  const ModDownConst* md = c->d_moddown.ptr + lev;
  grid_rows(batch * 2, gy, gz);
  hipLaunchKernelGGL(moddown_kernel, dim3((N + 255) / 256, gy, gz), dim3(256), 0, s, acc.ptr, nl, ne, z.ptr, md, batch,
                     c->dp);
  SFHE_HIP(hipGetLastError());
  for (int r = 0; r < 2 * nl; ++r) { pos[r] = r; pr[r] = r % nl; }
  rc = launch_ntt(c, z.ptr, batch, (int64_t)2 * nl * N, 2 * nl, pos, pr, false, s);
  if (rc) return rc;
  grid_rows(batch * 2 * nl, gy, gz);
  hipLaunchKernelGGL(moddown_finish_kernel, dim3((N + 255) / 256, gy, gz), dim3(256), 0, s, acc.ptr, nl, ne, z.ptr,
                     out, ostride, add_in, md, batch, c->dp);
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

// ---------------------------------------------------------------- rescale
// last[b][p] = in[b][p][lev]
__global__ void gather_last_kernel(const u64* in, int64_t istride, int nl, int lev, u64* last, int64_t batch,
                                   DevParams dp) {
  const int N = dp.N;
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;   // (b, p)
  if (row >= batch * 2) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t b = row >> 1;
  const int p = (int)(row & 1);
  last[row * N + t] = in[b * istride + ((int64_t)p * nl + lev) * N + t];
}

// R[b][p][i][t] = centered(last[b][p][t]) mod q_i, i < lev
__global__ void rescale_lift_kernel(const u64* last, int lev, u64* R, int64_t batch, DevParams dp) {
  const int N = dp.N;
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;   // (b, p)
  if (row >= batch * 2) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const u64 ql = dp.pr[lev].q;
  const u64 v = last[row * N + t];
  const i64 r = v > (ql - 1) / 2 ? -(i64)(ql - v) : (i64)v;
  for (int i = 0; i < lev; ++i) R[(row * lev + i) * N + t] = signed_mod(r, dp.pr[i]);
}

// out[b][p][i] = (in_i - R_i) q_lev^-1
__global__ void rescale_finish_kernel(const u64* in, int64_t istride, int lev, const u64* R, OutLayout ol,
                                      const RescaleConst* __restrict__ rc, int64_t batch, DevParams dp) {
  const int N = dp.N;
  const int nl = lev + 1;
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;   // (b, p, i)
  if (row >= batch * 2 * lev) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t b = row / (2 * lev);
  const int rem = (int)(row % (2 * lev));
  const int p = rem / lev, i = rem % lev;
  const u64 qi = dp.pr[i].q;
  const u64 x = in[b * istride + ((int64_t)p * nl + i) * N + t];
  const u64 y = R[((b * 2 + p) * lev + i) * N + t];
  const u64 v = mul_shoup(sub_mod(x, y, qi), rc->qinv[i], rc->qinv_s[i], qi);
  if (ol.chunked)
    ol.base[chunk_index(ol.elem_base + b, p, i, t, ol.n_ct, N >> 6)] = v;
  else
    ol.base[b * ol.stride + ((int64_t)p * lev + i) * N + t] = v;
}

int rescale_batch(sfhe_ctx* c, int lev, const u64* in, int64_t istride, OutLayout out, int64_t batch, hipStream_t s,
                  u64* scratch) {
  if (batch <= 0) return SFHE_OK;
  if (lev < 1) { set_error("rescale: level 0 has no prime to drop"); return SFHE_E_LEVEL; }
  const int N = c->N, nl = lev + 1;
  DevBuf<u64> last_b, R_b;
  if (!scratch && (!last_b.alloc(&c->alloc, (size_t)batch * 2 * N) || !R_b.alloc(&c->alloc, (size_t)batch * 2 * lev * N))) {
    set_error("rescale: device allocation failed");
    return SFHE_E_NOMEM;
  }
  u64* last = scratch ? scratch : last_b.ptr;
  u64* R = scratch ? scratch + (size_t)batch * 2 * N : R_b.ptr;
  unsigned gy, gz;
  grid_rows(batch * 2, gy, gz);
  hipLaunchKernelGGL(gather_last_kernel, dim3((N + 255) / 256, gy, gz), dim3(256), 0, s, in, istride, nl, lev,
                     last, batch, c->dp);
  SFHE_HIP(hipGetLastError());
  int pos[2 * kMaxBasis], pr[2 * kMaxBasis];
  pos[0] = 0; pr[0] = lev;
  int rc = launch_ntt(c, last, batch * 2, N, 1, pos, pr, true, s);
  if (rc) return rc;
  hipLaunchKernelGGL(rescale_lift_kernel, dim3((N + 255) / 256, gy, gz), dim3(256), 0, s, last, lev, R, batch,
                     c->dp);
  SFHE_HIP(hipGetLastError());
  for (int r = 0; r < 2 * lev; ++r) { pos[r] = r; pr[r] = r % lev; }
  rc = launch_ntt(c, R, batch, (int64_t)2 * lev * N, 2 * lev, pos, pr, false, s);
  if (rc) return rc;
  grid_rows(batch * 2 * lev, gy, gz);
  hipLaunchKernelGGL(rescale_finish_kernel, dim3((N + 255) / 256, gy, gz), dim3(256), 0, s, in, istride, lev, R,
                     out, c->d_rescale.ptr + lev, batch, c->dp);
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

// ---------------------------------------------------------------- accumulation
// chunked out[oidx[o]] += sum_{p in seg[o]..seg[o+1]-1} t[p], t limb-major [2][nl][N]
__global__ void segment_sum_kernel(int nl, const u64* tv, u64* out, int64_t n_ct, const int* seg, const int64_t* oidx,
                                   int64_t nout, DevParams dp) {
  const int N = dp.N;
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;   // (o, p, i)
  if (row >= nout * 2 * nl) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t o = row / (2 * nl);
  const int rem = (int)(row % (2 * nl));
  const int p = rem / nl, i = rem % nl;
  const u64 q = dp.pr[i].q;
  const int64_t cw = (int64_t)2 * nl * N;
  u64* dst = out + chunk_index(oidx[o], p, i, t, n_ct, N >> 6);
  u64 acc = *dst;
  for (int x = seg[o]; x < seg[o + 1]; ++x) acc = add_mod(acc, tv[(int64_t)x * cw + (int64_t)rem * N + t], q);
  *dst = acc;
}

int launch_segment_sum(const sfhe_ctx* c, int nl, const u64* t, u64* out, int64_t n_ct, const int* d_seg,
                       const int64_t* d_oidx, int64_t nout, hipStream_t s) {
  if (nout <= 0) return SFHE_OK;
  unsigned gy, gz;
  grid_rows(nout * 2 * nl, gy, gz);
  hipLaunchKernelGGL(segment_sum_kernel, dim3((c->N + 255) / 256, gy, gz), dim3(256), 0, s, nl, t, out, n_ct, d_seg,
                     d_oidx, nout, c->dp);
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

__global__ void zero_outputs_kernel(u64* out, int64_t n_ct, int nl, const int64_t* oidx, int64_t n, int N) {
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;   // (o, p, i)
  if (row >= n * 2 * nl) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t o = row / (2 * nl);
  const int rem = (int)(row % (2 * nl));
  out[chunk_index(oidx[o], rem / nl, rem % nl, t, n_ct, N >> 6)] = 0;
}

int launch_zero_outputs(const sfhe_ctx* c, u64* out, int64_t n_ct, int nl, const int64_t* d_oidx, int64_t n,
                        hipStream_t s) {
  if (n <= 0) return SFHE_OK;
  unsigned gy, gz;
  grid_rows(n * 2 * nl, gy, gz);
  hipLaunchKernelGGL(zero_outputs_kernel, dim3((c->N + 255) / 256, gy, gz), dim3(256), 0, s, out, n_ct, nl, d_oidx, n,
                     c->N);
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

}  // namespace sfhe
