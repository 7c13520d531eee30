// rotate.hip -- several values per ciphertext (Sec. 3.2) and the slot
// movements of Algorithm 1 (Sec. 3.3.1): encryption of value chunks, Galois
// automorphisms with their rotation keys, and the slot-zero mask.
//
// Slot j of a ciphertext holds its plaintext's value at zeta^(5^j), zeta =
// exp(i pi / N).  A rotation by r (slot j receives slot j + r) maps X to X^g,
// g = 5^r mod 2N, on both polys, then switches c1(X^g), which decrypts under
// s(X^g), back to s with the rotation key of g.  In the NTT domain X -> X^g is
// a permutation of the evaluation points: the value at psi^e moves from the
// one at psi^(g e), so the automorphism is a gather with one table per g.
#include "internal.hpp"
#include "hostmath.hpp"

namespace sfhe {

namespace {

constexpr u64 kTagRotA = 6, kTagRotE = 7;   // randomness streams of the rotation keys

struct CdtArgs {
  u64 cdt[kCdtLen];
};

void grid_rows(int64_t rows, unsigned& gy, unsigned& gz) {
  if (rows < 1) rows = 1;
  gy = rows < 65535 ? (unsigned)rows : 65535u;
  gz = (unsigned)((rows + gy - 1) / gy);
}

int brv_bits(int x, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((x >> b) & 1) << (bits - 1 - b);
  return r;
}

// NTT index held at each storage position of a row (the transform kernels'
// order: identity below N = 2^14; at N = 2^14 each thread's 16 registers are
// contiguous; at N = 2^15 each half repeats the N = 2^14 order)
std::vector<int> storage_order(int logN) {
  const int N = 1 << logN;
  std::vector<int> o(N);
  if (logN < 14) {
    for (int p = 0; p < N; ++p) o[p] = p;
    return o;
  }
  for (int h = 0; h < N >> 14; ++h)
    for (int t = 0; t < 512; ++t) {
      const int c = ((t & 63) << 4) | (((t >> 6) & 1) << 10) | (((t >> 8) & 1) << 11) | (((t >> 7) & 1) << 12);
      for (int r = 0; r < 32; ++r) o[(h << 14) + r * 512 + t] = (h << 14) | ((r >> 4) << 13) | c | (r & 15);
    }
  return o;
}

// ---------------------------------------------------------------- encryption
// Chunk x of the batch (chunk x0 + x of the matrix) holds the stored values
// z[v0 .. v0 + cnt), v0 = (x0 + x) slots, in slots 0 .. cnt - 1:
// m_t = nearbyint(sum_j z_j 2 Delta / N cos(pi (g_j t mod 2N) / N)), g_j = 5^j,
// the sum taken in slot order with every product and sum rounded on its own.
// Coefficient-domain parts: c1[r] = a_r, c0[r] = e + m; randomness keyed by
// (operand, chunk, 2^40 + cnt).
__global__ void enc_slots_kernel(u64* ct, int64_t count, int64_t x0, const double* z, int64_t nvals, int slots,
                                 const u64* gal, u64 seed, u64 operand, double pow2, const double* cosv, CdtArgs sa,
                                 DevParams dp) {
#pragma clang fp contract(off)
  const int N = dp.N, L = dp.L;
  const int64_t x = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;
  if (x >= count) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t ch = x0 + x, v0 = ch * slots;
  const int cnt = (int)(nvals - v0 < slots ? nvals - v0 : slots);
  const u64 m2 = 2 * (u64)N;
  double acc = 0.0;
  for (int j = 0; j < cnt; ++j) {
    const u64 e = (gal[j] * (u64)t) % m2;
    const double cv = e < (u64)N ? cosv[e] : -cosv[e - N];
    const double sz = z[v0 + j] * pow2;   // exact: a power of two
    const double pr = sz * cv;
    acc = acc + pr;
  }
  const i64 m = (i64)rint(acc);
  const u64 jf = (1ull << 40) + (u64)cnt;
  const u64 ke = sm_field(sm_field(sm_field(sm_key(seed, kTagEncE), operand), (u64)ch), jf);
  const i64 e = cdt_sample(sa.cdt, sm_word(ke, (u64)t));
  const u64 ka0 = sm_field(sm_field(sm_field(sm_key(seed, kTagEncA), operand), (u64)ch), jf);
  u64* base = ct + x * (int64_t)(2 * L) * N;
  for (int r = 0; r < L; ++r) {
    const PrimeDev& P = dp.pr[r];
    base[(int64_t)(L + r) * N + t] = uniform_residue(sm_field(ka0, (u64)r), (u64)t, P);
    base[(int64_t)r * N + t] = signed_mod(e + m, P);
  }
}

// ---------------------------------------------------------------- keys
// digit j of the key of g: [j][1][r] = a (uniform), [j][0][r] = e (coefficient domain)
__global__ void rot_sample_kernel(u64* key, u64 seed, u64 g, CdtArgs sa, DevParams dp) {
  const int N = dp.N, nb = dp.nb;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y, j = blockIdx.z;
  if (t >= N) return;
  const PrimeDev& P = dp.pr[r];
  const u64 ka = sm_field(sm_field(sm_field(sm_key(seed, kTagRotA), g), (u64)j), (u64)r);
  const u64 ke = sm_field(sm_field(sm_key(seed, kTagRotE), g), (u64)j);
  const i64 e = cdt_sample(sa.cdt, sm_word(ke, (u64)t));
  key[(((int64_t)j * 2 + 1) * nb + r) * N + t] = uniform_residue(ka, (u64)t, P);
  key[(((int64_t)j * 2 + 0) * nb + r) * N + t] = signed_mod(e, P);
}

// NTT domain: b = e - a s + g_jr s(X^g), s(X^g) gathered from s by the
// automorphism table; g_jr = [P]_{q_r} on the primes of digit j, else 0
__global__ void rot_finish_kernel(u64* key, const u64* s_ntt, const int* perm, const u64* gad, DevParams dp) {
  const int N = dp.N, nb = dp.nb;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y, j = blockIdx.z;
  if (t >= N) return;
  const PrimeDev& P = dp.pr[r];
  u64* b = key + (((int64_t)j * 2 + 0) * nb + r) * N;
  const u64* a = key + (((int64_t)j * 2 + 1) * nb + r) * N;
  const u64 as = mul_mod(a[t], s_ntt[(int64_t)r * N + t], P);
  const u64 gs = mul_mod(s_ntt[(int64_t)r * N + perm[t]], gad[j * nb + r], P);
  b[t] = add_mod(sub_mod(b[t], as, P.q), gs, P.q);
}

// ---------------------------------------------------------------- slot movement
// out[x] = (c0(X^g), 0) and t1[x] = c1(X^g) for n ciphertexts of nl primes (NTT domain)
__global__ void automorphism_kernel(const u64* in, int64_t istride, int nl, const int* perm, u64* out,
                                    int64_t ostride, u64* t1, int64_t n, int N) {
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;   // (x, prime)
  if (row >= n * nl) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t x = row / nl;
  const int i = (int)(row % nl);
  const int src = perm[t];
  const u64* ci = in + x * istride;
  u64* co = out + x * ostride;
  co[(int64_t)i * N + t] = ci[(int64_t)i * N + src];
  co[(int64_t)(nl + i) * N + t] = 0;
  t1[row * N + t] = ci[(int64_t)(nl + i) * N + src];
}

// D[x] = (c0(X^g), 0, c1(X^g)), rows of nl primes, stride 3 nl N: the input
// of the fused key switch (NTT domain)
__global__ void automorphism_d_kernel(const u64* in, int64_t istride, int nl, const int* perm, u64* D, int64_t n,
                                      int N) {
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;   // (x, prime)
  if (row >= n * nl) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t x = row / nl;
  const int i = (int)(row % nl);
  const int src = perm[t];
  const u64* ci = in + x * istride;
  u64* d = D + x * (int64_t)3 * nl * N;
  d[(int64_t)i * N + t] = ci[(int64_t)i * N + src];
  d[(int64_t)(nl + i) * N + t] = 0;
  d[(int64_t)(2 * nl + i) * N + t] = ci[(int64_t)(nl + i) * N + src];
}

// the same, reading ciphertext elem[x] of a chunked matrix (n_ct ciphertexts)
__global__ void automorphism_dc_kernel(const u64* src, int64_t n_ct, const int64_t* elem, int nl, const int* perm,
                                       u64* D, int64_t n, int N) {
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;   // (x, prime)
  if (row >= n * nl) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t x = row / nl;
  const int i = (int)(row % nl);
  const int sp = perm[t];
  const int64_t e = elem[x];
  u64* d = D + x * (int64_t)3 * nl * N;
  d[(int64_t)i * N + t] = src[chunk_index(e, 0, i, sp, n_ct, N >> 6)];
  d[(int64_t)(nl + i) * N + t] = 0;
  d[(int64_t)(2 * nl + i) * N + t] = src[chunk_index(e, 1, i, sp, n_ct, N >> 6)];
}

// x[b][p][i] *= mask[i] (NTT domain, pointwise) for n ciphertexts of nl primes
__global__ void mask_kernel(u64* x, int64_t stride, int nl, const u64* mask, int64_t n, DevParams dp) {
  const int N = dp.N;
  const int64_t row = blockIdx.y + (int64_t)blockIdx.z * gridDim.y;   // (b, p, i)
  if (row >= n * 2 * nl) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t b = row / (2 * nl);
  const int pi = (int)(row % (2 * nl));
  const int i = pi % nl;
  u64& v = x[b * stride + (int64_t)pi * N + t];
  v = mul_mod(v, mask[(int64_t)i * N + t], dp.pr[i]);
}

}  // namespace

u64 galois_element(const sfhe_ctx* c, int64_t r) {
  const int64_t h = c->N / 2;
  const int64_t e = ((r % h) + h) % h;
  const u64 m2 = 2 * (u64)c->N;
  u64 g = 1;
  for (int64_t x = 0; x < e; ++x) g = g * 5 % m2;
  return g;
}

const int* automorphism_table(sfhe_ctx* c, u64 g) {
  auto it = c->auto_perm.find(g);
  if (it != c->auto_perm.end()) return it->second.ptr;
  const int N = c->N, logN = c->logN;
  const std::vector<int> order = storage_order(logN);
  std::vector<int> pos(N), perm(N);
  for (int p = 0; p < N; ++p) pos[order[p]] = p;
  const u64 m2 = 2 * (u64)N;
  for (int p = 0; p < N; ++p) {
    const u64 e = 2 * (u64)brv_bits(order[p], logN) + 1;    // position p holds a(psi^e)
    const u64 ge = g * e % m2;                               // sigma_g(a)(psi^e) = a(psi^(g e))
    perm[p] = pos[brv_bits((int)((ge - 1) / 2), logN)];
  }
  DevBuf<int> d;
  if (!d.alloc(&c->alloc, N)) { set_error("automorphism table: device allocation failed"); return nullptr; }
  if (hipMemcpy(d.ptr, perm.data(), N * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("automorphism table: copy failed");
    return nullptr;
  }
  const int* p = d.ptr;
  c->auto_perm.emplace(g, std::move(d));
  return p;
}

const u64* rotation_key(sfhe_ctx* c, u64 g) {
  auto it = c->rot_keys.find(g);
  if (it != c->rot_keys.end()) return it->second.ptr;
  const int N = c->N, nb = c->nb, dnum = c->dnum;
  const int* perm = automorphism_table(c, g);
  if (!perm) return nullptr;
  DevBuf<u64> key, d_gad;
  if (!key.alloc(&c->alloc, (size_t)dnum * 2 * nb * N) || !d_gad.alloc(&c->alloc, (size_t)dnum * nb)) {
    set_error("rotation key: device allocation failed");
    return nullptr;
  }
  CdtArgs sa;
  for (int k = 0; k < kCdtLen; ++k) sa.cdt[k] = c->cdt[k];
  hipLaunchKernelGGL(rot_sample_kernel, dim3((N + 255) / 256, nb, dnum), dim3(256), 0, 0, key.ptr, c->key_seed, g, sa,
                     c->dp);
  if (hipGetLastError() != hipSuccess) { set_error("rotation key: launch failed"); return nullptr; }
  int pos[2 * kMaxBasis], pr[2 * kMaxBasis];
  for (int r = 0; r < nb; ++r) { pos[r] = r; pr[r] = r; }
  for (int j = 0; j < dnum; ++j)
    if (launch_ntt(c, key.ptr + (size_t)j * 2 * nb * N, 2, (int64_t)nb * N, nb, pos, pr, false, 0)) return nullptr;
  std::vector<u64> gad((size_t)dnum * nb, 0);
  for (int j = 0; j < dnum; ++j) {
    const int lo = j * c->alpha, hi = std::min((j + 1) * c->alpha, c->L);
    for (int r = lo; r < hi; ++r) {
      u64 v = 1;
      for (int k = 0; k < c->alpha; ++k) v = hostmath::mulmod(v, c->primes[c->L + k] % c->primes[r], c->primes[r]);
      gad[(size_t)j * nb + r] = v;
    }
  }
  if (hipMemcpy(d_gad.ptr, gad.data(), gad.size() * sizeof(u64), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("rotation key: copy failed");
    return nullptr;
  }
  hipLaunchKernelGGL(rot_finish_kernel, dim3((N + 255) / 256, nb, dnum), dim3(256), 0, 0, key.ptr, c->d_s.ptr, perm,
                     d_gad.ptr, c->dp);
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    set_error("rotation key: kernel failed");
    return nullptr;
  }
  // Shoup companions floor(k 2^64 / q) of every key word, for the fused key
  // switch (computed once, on the host)
  const size_t nk = (size_t)dnum * 2 * nb * N;
  std::vector<u64> h(nk);
  DevBuf<u64> ks;
  if (!ks.alloc(&c->alloc, nk) || hipMemcpy(h.data(), key.ptr, nk * sizeof(u64), hipMemcpyDeviceToHost) != hipSuccess) {
    set_error("rotation key: allocation or copy failed");
    return nullptr;
  }
  for (size_t w = 0; w < nk; ++w) h[w] = hostmath::shoup(h[w], c->primes[(w / N) % nb]);
  if (hipMemcpy(ks.ptr, h.data(), nk * sizeof(u64), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("rotation key: copy failed");
    return nullptr;
  }
  const u64* p = key.ptr;
  c->rot_keys.emplace(g, std::move(key));
  c->rot_keys_s.emplace(g, std::move(ks));
  return p;
}

int prepare_rotations(sfhe_ctx* c, const std::vector<int64_t>& offsets) {
  for (int64_t r : offsets) {
    const u64 g = galois_element(c, r);
    if (g == 1) continue;
    if (!rotation_key(c, g)) return SFHE_E_NOMEM;
  }
  return SFHE_OK;
}

int rotate_batch(sfhe_ctx* c, int lev, const u64* in, int64_t istride, int64_t r, u64* out, int64_t ostride,
                 int64_t n, hipStream_t s) {
  if (n <= 0) return SFHE_OK;
  const int N = c->N, nl = lev + 1;
  const u64 g = galois_element(c, r);
  if (g == 1) {   // rotation by a multiple of N/2: the identity
    SFHE_HIP(hipMemcpy2DAsync(out, (size_t)ostride * sizeof(u64), in, (size_t)istride * sizeof(u64),
                              (size_t)2 * nl * N * sizeof(u64), (size_t)n, hipMemcpyDeviceToDevice, s));
    return SFHE_OK;
  }
  const int* perm = automorphism_table(c, g);
  const u64* key = perm ? rotation_key(c, g) : nullptr;
  if (!key) return SFHE_E_NOMEM;
  if (keyswitch_rescale_n14_supported(c)) {
    // N = 2^14: the fused key switch, in slices within its grid limits
    const u64* key_s = c->rot_keys_s.at(g).ptr;
    const int64_t slice = std::min<int64_t>(n, 1024);
    DevBuf<u64> D;
    if (!D.alloc(&c->alloc, (size_t)slice * 3 * nl * N)) { set_error("rotate: device allocation failed"); return SFHE_E_NOMEM; }
    for (int64_t x0 = 0; x0 < n; x0 += slice) {
      const int64_t m = std::min(slice, n - x0);
      unsigned gy, gz;
      grid_rows(m * nl, gy, gz);
      hipLaunchKernelGGL(automorphism_d_kernel, dim3((N + 255) / 256, gy, gz), dim3(256), 0, s, in + x0 * istride, istride,
                         nl, perm, D.ptr, m, N);
      SFHE_HIP(hipGetLastError());
      const int rc = keyswitch_n14(c, lev, D.ptr, (int64_t)3 * nl * N, OutLayout{out + x0 * ostride, ostride, false, 0, 0},
                                   m, key, key_s, s);
      if (rc) return rc;
    }
    return SFHE_OK;
  }
  DevBuf<u64> t1;
  if (!t1.alloc(&c->alloc, (size_t)n * nl * N)) { set_error("rotate: device allocation failed"); return SFHE_E_NOMEM; }
  unsigned gy, gz;
  grid_rows(n * nl, gy, gz);
  hipLaunchKernelGGL(automorphism_kernel, dim3((N + 255) / 256, gy, gz), dim3(256), 0, s, in, istride, nl, perm, out,
                     ostride, t1.ptr, n, N);
  SFHE_HIP(hipGetLastError());
  return keyswitch_batch(c, lev, t1.ptr, (int64_t)nl * N, out, ostride, true, n, s, key);
}

int slot_table(sfhe_ctx* c) {
  if (c->d_gal.ptr) return SFHE_OK;
  std::vector<u64> gal(64);
  for (int j = 0; j < 64; ++j) gal[j] = galois_element(c, j);
  if (!c->d_gal.alloc(&c->alloc, gal.size())) { set_error("slot table: device allocation failed"); return SFHE_E_NOMEM; }
  SFHE_HIP(hipMemcpy(c->d_gal.ptr, gal.data(), gal.size() * sizeof(u64), hipMemcpyHostToDevice));
  return SFHE_OK;
}

int rotate_chunked(sfhe_ctx* c, int lev, const u64* src, int64_t n_ct, const int64_t* d_elem, int64_t r, u64* out,
                   int64_t ostride, int64_t n, hipStream_t s) {
  if (n <= 0) return SFHE_OK;
  if (!keyswitch_rescale_n14_supported(c)) { set_error("rotate_chunked: N = 2^14 only"); return SFHE_E_INVALID_ARG; }
  const int N = c->N, nl = lev + 1;
  const u64 g = galois_element(c, r);
  const int* perm = automorphism_table(c, g);
  const u64* key = perm ? rotation_key(c, g) : nullptr;
  if (!key) return SFHE_E_NOMEM;
  const u64* key_s = c->rot_keys_s.at(g).ptr;
  if (n > 1024) { set_error("rotate_chunked: at most 1024 ciphertexts per call"); return SFHE_E_INVALID_ARG; }
  DevBuf<u64> D;
  if (!D.alloc(&c->alloc, (size_t)n * 3 * nl * N)) { set_error("rotate: device allocation failed"); return SFHE_E_NOMEM; }
  unsigned gy, gz;
  grid_rows(n * nl, gy, gz);
  hipLaunchKernelGGL(automorphism_dc_kernel, dim3((N + 255) / 256, gy, gz), dim3(256), 0, s, src, n_ct, d_elem, nl, perm,
                     D.ptr, n, N);
  SFHE_HIP(hipGetLastError());
  return keyswitch_n14(c, lev, D.ptr, (int64_t)3 * nl * N, OutLayout{out, ostride, false, 0, 0}, n, key, key_s, s);
}

int encrypt_slots(sfhe_ctx* c, u64* tmp, int64_t count, int64_t x0, const double* d_vals, int64_t nvals, int slots,
                  u64 seed, u64 operand, hipStream_t s) {
  if (count <= 0) return SFHE_OK;
  const int N = c->N;
  int rc = slot_table(c);
  if (rc) return rc;
  CdtArgs sa;
  for (int k = 0; k < kCdtLen; ++k) sa.cdt[k] = c->cdt[k];
  const double pow2 = ldexp(1.0, (int)c->log2_scale + 1 - c->logN);
  unsigned gy, gz;
  grid_rows(count, gy, gz);
  hipLaunchKernelGGL(enc_slots_kernel, dim3((N + 255) / 256, gy, gz), dim3(256), 0, s, tmp, count, x0, d_vals, nvals,
                     slots, c->d_gal.ptr, seed, operand, pow2, c->d_cos.ptr, sa, c->dp);
  SFHE_HIP(hipGetLastError());
  return encrypt_finish(c, tmp, count, s);
}

int mask_batch(sfhe_ctx* c, int lev, u64* x, int64_t stride, int64_t n, hipStream_t s) {
  if (n <= 0) return SFHE_OK;
  const int N = c->N, L = c->L;
  if (!c->d_mask0.ptr) {
    // the plaintext of 1.0 in slot 0 at scale Delta: m_t = nearbyint(2 Delta / N cos(pi t / N))
    const double sz = ldexp(1.0, (int)c->log2_scale + 1 - c->logN);
    std::vector<u64> m((size_t)L * N);
    for (int t = 0; t < N; ++t) {
      const i64 v = (i64)nearbyint(sz * cos(M_PI * (double)t / (double)N));
      for (int r = 0; r < L; ++r) {
        const u64 q = c->primes[r];
        m[(size_t)r * N + t] = v >= 0 ? (u64)v % q : (q - (u64)(-v) % q) % q;
      }
    }
    DevBuf<u64> d;
    if (!d.alloc(&c->alloc, m.size())) { set_error("mask: device allocation failed"); return SFHE_E_NOMEM; }
    SFHE_HIP(hipMemcpy(d.ptr, m.data(), m.size() * sizeof(u64), hipMemcpyHostToDevice));
    int pos[2 * kMaxBasis], pr[2 * kMaxBasis];
    for (int r = 0; r < L; ++r) { pos[r] = r; pr[r] = r; }
    int rc = launch_ntt(c, d.ptr, 1, 0, L, pos, pr, false, 0);
    if (rc) return rc;
    SFHE_HIP(hipDeviceSynchronize());
    c->d_mask0 = std::move(d);
  }
  const int nl = lev + 1;
  unsigned gy, gz;
  grid_rows(n * 2 * nl, gy, gz);
  hipLaunchKernelGGL(mask_kernel, dim3((N + 255) / 256, gy, gz), dim3(256), 0, s, x, stride, nl, c->d_mask0.ptr, n,
                     c->dp);
  SFHE_HIP(hipGetLastError());
  return SFHE_OK;
}

}  // namespace sfhe
