// sample.hip -- key generation, encryption and decryption kernels.
//
// Conventions (the paper fixes only the scheme, CKKS, and its parameters,
// Sec. 3.1): one value per ciphertext in slot 0 of the canonical embedding
// (chunk size c = 1, Sec. 3.2), m_t = rint(z 2 Delta / N cos(pi t / N));
// secret-key encryption c = (-a s + e + m, a) with a uniform per prime and e a
// discrete Gaussian; ternary secret; relinearisation key for hybrid key
// switching.  Randomness is drawn from counter-based SplitMix64 streams keyed
// by (seed, tag, fields), sampled in the coefficient domain.
#include "internal.hpp"
#include "hostmath.hpp"

namespace sfhe {

struct SampleArgs {
  u64 cdt[kCdtLen];
};

// ---------------------------------------------------------------- encryption
// Coefficient-domain parts of element x: c1[r] = a_r, c0[r] = e + m.
__global__ void enc_sample_kernel(u64* ct, int64_t count, const int* ei, const int* ej, const double* zv, u64 seed,
                                  u64 operand, double pow2, const double* cosv, SampleArgs sa, DevParams dp) {
  const int N = dp.N, L = dp.L;
  const int64_t x = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;
  if (x >= count) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const u64 i = (u64)ei[x], j = (u64)ej[x];
  const double sz = zv[x] * pow2;                       // exact: a power of two
  const i64 m = (i64)rint(sz * cosv[t]);
  const u64 ke = sm_field(sm_field(sm_field(sm_key(seed, kTagEncE), operand), i), j);
  const i64 e = cdt_sample(sa.cdt, sm_word(ke, (u64)t));
  const u64 ka0 = sm_field(sm_field(sm_field(sm_key(seed, kTagEncA), operand), i), j);
  u64* base = ct + x * (int64_t)(2 * L) * N;
  for (int r = 0; r < L; ++r) {
    const PrimeDev& P = dp.pr[r];
    const u64 ka = sm_field(ka0, (u64)r);
    base[(int64_t)(L + r) * N + t] = uniform_residue(ka, (u64)t, P);
    base[(int64_t)r * N + t] = signed_mod(e + m, P);
  }
}

// NTT domain: c0 <- c0 - c1 * s
__global__ void enc_finish_kernel(u64* ct, int64_t nct, const u64* s_ntt, DevParams dp) {
  const int N = dp.N, L = dp.L;
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;   // (slot, limb)
  if (row >= nct * L) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t x = row / L;
  const int r = (int)(row % L);
  const PrimeDev& P = dp.pr[r];
  u64* c0 = ct + (x * 2 * L + r) * N;
  const u64* c1 = ct + (x * 2 * L + L + r) * N;
  const u64 as = mul_mod(c1[t], s_ntt[(int64_t)r * N + t], P);
  c0[t] = sub_mod(c0[t], as, P.q);
}

// rows >= 1 (callers return early on empty work)
static void grid_rows(int64_t rows, unsigned& gy, unsigned& gz) {
  if (rows < 1) rows = 1;
  gy = rows < 65535 ? (unsigned)rows : 65535u;
  gz = (unsigned)((rows + gy - 1) / gy);
}

int encrypt_elements(sfhe_ctx* c, u64* ct, int64_t count, const int* d_ei, const int* d_ej, const double* d_z,
                     u64 seed, u64 operand, hipStream_t s) {
  const int N = c->N;
  if (count > 0) {
    SampleArgs sa;
    for (int k = 0; k < kCdtLen; ++k) sa.cdt[k] = c->cdt[k];
    const double pow2 = ldexp(1.0, (int)c->log2_scale + 1 - c->logN);
    unsigned gy, gz;
    grid_rows(count, gy, gz);
    dim3 grid((N + 255) / 256, gy, gz);
    hipLaunchKernelGGL(enc_sample_kernel, grid, dim3(256), 0, s, ct, count, d_ei, d_ej, d_z, seed, operand, pow2,
                       c->d_cos.ptr, sa, c->dp);
    SFHE_HIP(hipGetLastError());
  }
  return SFHE_OK;
}

int encrypt_finish(sfhe_ctx* c, u64* ct, int64_t nct, hipStream_t s) {
  if (nct <= 0) return SFHE_OK;
  const int N = c->N, L = c->L;
  int pos[2 * kMaxBasis], pr[2 * kMaxBasis];
  for (int r = 0; r < 2 * L; ++r) { pos[r] = r; pr[r] = r % L; }
  int rc = launch_ntt(c, ct, nct, (int64_t)2 * L * N, 2 * L, pos, pr, false, s);
  if (rc) return rc;
  unsigned gy, gz;
  grid_rows(nct * L, gy, gz);
  hipLaunchKernelGGL(enc_finish_kernel, dim3((N + 255) / 256, gy, gz), dim3(256), 0, s, ct, nct, c->d_s.ptr,
                     c->dp);
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

// ---------------------------------------------------------------- keys
// secret s_t = (word(t) mod 3) - 1, reduced mod every basis prime (coefficient domain)
__global__ void secret_kernel(u64* s_out, u64 seed, DevParams dp) {
  const int N = dp.N;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (t >= N) return;
  const u64 w = sm_word(sm_key(seed, kTagSecret), (u64)t);
  const i64 v = (i64)(w % 3) - 1;
  s_out[(int64_t)r * N + t] = signed_mod(v, dp.pr[r]);
}

// rlk digit j: slot [j][1][r] = a (uniform), slot [j][0][r] = e (coefficient domain)
__global__ void rlk_sample_kernel(u64* rlk, u64 seed, SampleArgs sa, DevParams dp) {
  const int N = dp.N, nb = dp.nb;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y, j = blockIdx.z;
  if (t >= N) return;
  const PrimeDev& P = dp.pr[r];
  const u64 ka = sm_field(sm_field(sm_key(seed, kTagRlkA), (u64)j), (u64)r);
  const u64 ke = sm_field(sm_key(seed, kTagRlkE), (u64)j);
  const i64 e = cdt_sample(sa.cdt, sm_word(ke, (u64)t));
  rlk[(((int64_t)j * 2 + 1) * nb + r) * N + t] = uniform_residue(ka, (u64)t, P);
  rlk[(((int64_t)j * 2 + 0) * nb + r) * N + t] = signed_mod(e, P);
}

// NTT domain: b = e - a s + g_jr s^2, g_jr = [P]_{q_r} on the primes of digit j
__global__ void rlk_finish_kernel(u64* rlk, const u64* s_ntt, const u64* gad, DevParams dp) {
  const int N = dp.N, nb = dp.nb;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y, j = blockIdx.z;
  if (t >= N) return;
  const PrimeDev& P = dp.pr[r];
  u64* b = rlk + (((int64_t)j * 2 + 0) * nb + r) * N;
  const u64* a = rlk + (((int64_t)j * 2 + 1) * nb + r) * N;
  const u64 sv = s_ntt[(int64_t)r * N + t];
  const u64 as = mul_mod(a[t], sv, P);
  const u64 g = gad[j * nb + r];
  const u64 gs2 = mul_mod(mul_mod(sv, sv, P), g, P);
  b[t] = add_mod(sub_mod(b[t], as, P.q), gs2, P.q);
}

int keygen_device(sfhe_ctx* c, u64 seed, hipStream_t s) {
  const int N = c->N, nb = c->nb, dnum = c->dnum;
  c->key_seed = seed;
  c->rot_keys.clear();
  c->rot_keys_s.clear();
  if (!c->d_s.alloc(&c->alloc, (size_t)nb * N) || !c->d_rlk.alloc(&c->alloc, (size_t)dnum * 2 * nb * N)) {
    set_error("keygen: device allocation failed");
    return SFHE_E_NOMEM;
  }
  hipLaunchKernelGGL(secret_kernel, dim3((N + 255) / 256, nb), dim3(256), 0, s, c->d_s.ptr, seed, c->dp);
  SFHE_HIP(hipGetLastError());
  int pos[2 * kMaxBasis], pr[2 * kMaxBasis];
  for (int r = 0; r < nb; ++r) { pos[r] = r; pr[r] = r; }
  int rc = launch_ntt(c, c->d_s.ptr, 1, 0, nb, pos, pr, false, s);
  if (rc) return rc;
  SampleArgs sa;
  for (int k = 0; k < kCdtLen; ++k) sa.cdt[k] = c->cdt[k];
  hipLaunchKernelGGL(rlk_sample_kernel, dim3((N + 255) / 256, nb, dnum), dim3(256), 0, s, c->d_rlk.ptr, seed, sa,
                     c->dp);
  SFHE_HIP(hipGetLastError());
  // NTT of every row: [dnum][2][nb]
  for (int j = 0; j < dnum; ++j) {
    rc = launch_ntt(c, c->d_rlk.ptr + (size_t)j * 2 * nb * N, 2, (int64_t)nb * N, nb, pos, pr, false, s);
    if (rc) return rc;
  }
  // gadget residues: P mod q_r for data prime r in digit j
  std::vector<u64> gad((size_t)dnum * nb, 0);
  for (int j = 0; j < dnum; ++j) {
    const int lo = j * c->alpha, hi = std::min((j + 1) * c->alpha, c->L);
    for (int r = lo; r < hi; ++r) {
      unsigned __int128 g = 1;
      for (int k = 0; k < c->alpha; ++k) g = g * (c->primes[c->L + k] % c->primes[r]) % c->primes[r];
      gad[(size_t)j * nb + r] = (u64)g;
    }
  }
  DevBuf<u64> d_gad;
  if (!d_gad.alloc(&c->alloc, gad.size())) { set_error("keygen: allocation failed"); return SFHE_E_NOMEM; }
  SFHE_HIP(hipMemcpyAsync(d_gad.ptr, gad.data(), gad.size() * sizeof(u64), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(rlk_finish_kernel, dim3((N + 255) / 256, nb, dnum), dim3(256), 0, s, c->d_rlk.ptr, c->d_s.ptr,
                     d_gad.ptr, c->dp);
  SFHE_HIP(hipGetLastError());
  SFHE_HIP(hipStreamSynchronize(s));
  // Shoup companions floor(k 2^64 / q) of every key word, for the key
  // products of the fused key switch (computed once, on the host)
  const size_t nk = (size_t)dnum * 2 * nb * N;
  std::vector<u64> key(nk);
  SFHE_HIP(hipMemcpy(key.data(), c->d_rlk.ptr, nk * sizeof(u64), hipMemcpyDeviceToHost));
  for (size_t w = 0; w < nk; ++w) key[w] = hostmath::shoup(key[w], c->primes[(w / N) % nb]);
  if (!c->d_rlk_s.alloc(&c->alloc, nk)) { set_error("keygen: device allocation failed"); return SFHE_E_NOMEM; }
  SFHE_HIP(hipMemcpy(c->d_rlk_s.ptr, key.data(), nk * sizeof(u64), hipMemcpyHostToDevice));
  return SFHE_OK;
}

// ---------------------------------------------------------------- decryption
// m = c0 + c1 s (NTT domain) for count ciphertexts at level lev
__global__ void dec_phase_kernel(const u64* ct, int64_t count, int64_t ctstride, int nl, u64* m,
                                 const u64* s_ntt, DevParams dp) {
  const int N = dp.N;
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;
  if (row >= count * nl) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t x = row / nl;
  const int r = (int)(row % nl);
  const PrimeDev& P = dp.pr[r];
  const u64* c0 = ct + x * ctstride + (int64_t)r * N;
  const u64* c1 = ct + x * ctstride + (int64_t)(nl + r) * N;
  m[(x * nl + r) * N + t] = add_mod(c0[t], mul_mod(c1[t], s_ntt[(int64_t)r * N + t], P), P.q);
}

// decode slot j = blockIdx.y: sum_t m_t cos(pi (g t mod 2N) / N) / scale,
// g = 5^j, m_t the centered integer (slot 0: g = 1).  The candidate comes
// from the largest prime's residue; every other residue must agree with it,
// else the coefficient is out of the decodable range.  Value x slots + j goes
// to out[x slots + j] when below nvals.
__global__ void __launch_bounds__(256) dec_decode_kernel(const u64* m, int nl, int big, double inv_scale,
                                                         const double* cosv, const u64* gal, int slots,
                                                         int64_t nvals, double* out, int* flag, DevParams dp) {
  __shared__ double red[256];
  const int N = dp.N;
  const int64_t x = blockIdx.x;
  const int64_t v = x * slots + blockIdx.y;
  if (v >= nvals) return;   // uniform across the block
  const u64 g = blockIdx.y ? gal[blockIdx.y] : 1, m2 = 2 * (u64)N;
  const u64* mx = m + x * nl * N;
  const u64 qb = dp.pr[big].q;
  double acc = 0.0;
  int bad = 0;
  for (int t = threadIdx.x; t < N; t += blockDim.x) {
    const u64 v = mx[(int64_t)big * N + t];
    const i64 cv = v > (qb - 1) / 2 ? -(i64)(qb - v) : (i64)v;
    for (int r = 0; r < nl; ++r)
      if (r != big && signed_mod(cv, dp.pr[r]) != mx[(int64_t)r * N + t]) bad = 1;
    const u64 e = g * (u64)t % m2;
    acc += (double)cv * (e < (u64)N ? cosv[e] : -cosv[e - N]);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (bad) atomicOr(flag, 1);
  if (threadIdx.x == 0) out[v] = red[0] * inv_scale;
}

int decrypt_values(sfhe_ctx* c, const u64* data, int64_t n_ct, int lev, double scale, double* d_out, int* d_flag,
                   hipStream_t s, int slots, int64_t nvals) {
  const int N = c->N, nl = lev + 1;
  if (nvals < 0) nvals = n_ct * slots;
  if (slots > 1 && !c->d_gal.ptr) {
    set_error("decrypt: slot table missing");
    return SFHE_E_STATE;
  }
  const int64_t chunk = 512;
  const int64_t ctw = (int64_t)2 * nl * N;
  DevBuf<u64> ct, m;
  const size_t cap = (size_t)std::min<int64_t>(chunk, n_ct);
  if (!ct.alloc(&c->alloc, cap * ctw) || !m.alloc(&c->alloc, cap * nl * N)) {
    set_error("decrypt: allocation failed");
    return SFHE_E_NOMEM;
  }
  int big = 0;
  for (int r = 1; r < nl; ++r)
    if (c->primes[r] > c->primes[big]) big = r;
  int pos[2 * kMaxBasis], pr[2 * kMaxBasis];
  for (int r = 0; r < nl; ++r) { pos[r] = r; pr[r] = r; }
  for (int64_t x0 = 0; x0 < n_ct; x0 += chunk) {
    const int64_t n = std::min(chunk, n_ct - x0);
    int rc = launch_from_chunked(c, data, n_ct, nl, n, nullptr, x0, ct.ptr, ctw, s);
    if (rc) return rc;
    unsigned gy, gz;
    grid_rows(n * nl, gy, gz);
    hipLaunchKernelGGL(dec_phase_kernel, dim3((N + 255) / 256, gy, gz), dim3(256), 0, s, ct.ptr, n, ctw, nl, m.ptr,
                       c->d_s.ptr, c->dp);
    SFHE_HIP(hipGetLastError());
    rc = launch_ntt(c, m.ptr, n, (int64_t)nl * N, nl, pos, pr, true, s);
    if (rc) return rc;
    hipLaunchKernelGGL(dec_decode_kernel, dim3((unsigned)n, (unsigned)slots), dim3(256), 0, s, m.ptr, nl, big,
                       1.0 / scale, c->d_cos.ptr, c->d_gal.ptr, slots, nvals - x0 * slots, d_out + x0 * slots, d_flag,
                       c->dp);
    SFHE_HIP(hipGetLastError());
  }
  SFHE_HIP(hipStreamSynchronize(s));
  return SFHE_OK;
}

}  // namespace sfhe
