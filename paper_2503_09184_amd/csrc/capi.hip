// capi.hip -- the C ABI: parameter set-up, keys, encryption of matrices under
// the encodings of Sec. 3.3, the encrypted product C = A*B in both
// accumulation orders, decryption, and the primitive steps.
#include <math.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "hostmath.hpp"
#include "internal.hpp"

namespace sfhe {

static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }

void* Alloc::get(size_t bytes) {
  if (bytes == 0) return nullptr;
  if (has_hooks) return hooks.alloc(bytes, (void*)cur, hooks.user);
  void* p = nullptr;
  if (hipMallocFromPoolAsync(&p, bytes, pool, cur) == hipSuccess) return p;
  (void)hipGetLastError();
  // the pool keeps freed blocks, which may be too small or pieces of the
  // device's memory that a large request needs whole: once the device has
  // drained (every pending free completed), give them all back and try once
  // more
  p = nullptr;
  if (hipDeviceSynchronize() == hipSuccess && hipMemPoolTrimTo(pool, 0) == hipSuccess &&
      hipMallocFromPoolAsync(&p, bytes, pool, cur) == hipSuccess)
    return p;
  (void)hipGetLastError();
  return nullptr;
}
void Alloc::put(void* p, size_t bytes, hipStream_t s) {
  if (!p) return;
  if (has_hooks)
    hooks.free(p, bytes, (void*)s, hooks.user);
  else
    (void)hipFreeAsync(p, s);
}

static int brv(int x, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
}

template <typename T>
static bool upload(sfhe_ctx* c, DevBuf<T>& buf, const std::vector<T>& v, hipStream_t s) {
  if (!buf.alloc(&c->alloc, v.size())) return false;
  if (v.empty()) return true;
  return hipMemcpyAsync(buf.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s) == hipSuccess;
}

// ---------------------------------------------------------------- timing
enum { kCatTensor = 0, kCatKeyswitch = 1, kCatRescale = 2, kCatTensorFp = 3 };

// brackets a launch group with an event pair when profiling is on
struct StepTimer {
  sfhe_ctx* c;
  hipStream_t s;
  hipEvent_t stop = nullptr;
  StepTimer(sfhe_ctx* ctx, hipStream_t st, int cat) : c(ctx), s(st) {
    if (!c->profiling || cat < 0) return;   // cat < 0: no events (launches under graph capture)
    hipEvent_t a = c->prof_event(), b = c->prof_event();
    if (!a || !b) return;
    (void)hipEventRecord(a, s);
    c->prof_cat.push_back(cat);
    stop = b;
  }
  ~StepTimer() {
    if (stop) (void)hipEventRecord(stop, s);
  }
};

}  // namespace sfhe

hipEvent_t sfhe_ctx::prof_event() {
  if (prof_used == prof_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    prof_pool.push_back(e);
  }
  return prof_pool[prof_used++];
}

namespace sfhe {

// ---------------------------------------------------------------- context
static int build_tables(sfhe_ctx* c) {
  using namespace hostmath;
  const int N = c->N, nb = c->nb;
  std::vector<u64> tab((size_t)nb * 4 * N);
  for (int r = 0; r < nb; ++r) {
    const u64 q = c->primes[r];
    const u64 psi = smallest_primitive_root_2n(q, 2 * (u64)N);
    const u64 psi_inv = invmod(psi, q);
    std::vector<u64> pw(N), ipw(N);
    pw[0] = 1;
    ipw[0] = 1;
    for (int k = 1; k < N; ++k) { pw[k] = mulmod(pw[k - 1], psi, q); ipw[k] = mulmod(ipw[k - 1], psi_inv, q); }
    u64* tw = tab.data() + ((size_t)r * 4 + 0) * N;
    u64* tws = tab.data() + ((size_t)r * 4 + 1) * N;
    u64* itw = tab.data() + ((size_t)r * 4 + 2) * N;
    u64* itws = tab.data() + ((size_t)r * 4 + 3) * N;
    for (int m = 0; m < N; ++m) {
      const int e = brv(m, c->logN);
      tw[m] = pw[e];
      tws[m] = shoup(tw[m], q);
      itw[m] = ipw[e];
      itws[m] = shoup(itw[m], q);
    }
    PrimeDev& P = c->dp.pr[r];
    P.q = q;
    barrett128(q, &P.mu_hi, &P.mu_lo);
    P.ninv = invmod((u64)N % q, q);
    P.ninv_s = shoup(P.ninv, q);
  }
  if (!c->d_tables.alloc(&c->alloc, tab.size())) return SFHE_E_NOMEM;
  SFHE_HIP(hipMemcpy(c->d_tables.ptr, tab.data(), tab.size() * sizeof(u64), hipMemcpyHostToDevice));
  std::vector<double> tabd((size_t)nb * 2 * N);
  for (int r = 0; r < nb; ++r)
    for (int m = 0; m < N; ++m) {
      tabd[((size_t)r * 2 + 0) * N + m] = (double)tab[((size_t)r * 4 + 0) * N + m];
      tabd[((size_t)r * 2 + 1) * N + m] = (double)tab[((size_t)r * 4 + 2) * N + m];
    }
  if (!c->d_tables_d.alloc(&c->alloc, tabd.size())) return SFHE_E_NOMEM;
  SFHE_HIP(hipMemcpy(c->d_tables_d.ptr, tabd.data(), tabd.size() * sizeof(double), hipMemcpyHostToDevice));
  for (int r = 0; r < nb; ++r) {
    PrimeDev& P = c->dp.pr[r];
    P.tw = c->d_tables.ptr + ((size_t)r * 4 + 0) * N;
    P.tws = c->d_tables.ptr + ((size_t)r * 4 + 1) * N;
    P.itw = c->d_tables.ptr + ((size_t)r * 4 + 2) * N;
    P.itws = c->d_tables.ptr + ((size_t)r * 4 + 3) * N;
    P.twd = c->d_tables_d.ptr + ((size_t)r * 2 + 0) * N;
    P.itwd = c->d_tables_d.ptr + ((size_t)r * 2 + 1) * N;
  }
  // N = 2^15: after the first stage (pairs x_i, x_{i + N/2}), each half is a
  // 2^14-point transform whose twiddles, indexed as a transform of its own
  // (m + g for m groups), are the full transform's (2 + h) m + g: tables
  // [prime][direction][half][2^14], forward (tw) then inverse (itw)
  if (c->logN == 15) {
    const int H = N / 2;
    std::vector<u64> sub((size_t)nb * 4 * H, 0), sub_s((size_t)nb * 4 * H, 0);
    std::vector<double> subd((size_t)nb * 4 * H, 0.0);
    for (int r = 0; r < nb; ++r)
      for (int d = 0; d < 2; ++d) {
        const u64* full = tab.data() + ((size_t)r * 4 + 2 * d) * N;
        const u64* full_s = tab.data() + ((size_t)r * 4 + 2 * d + 1) * N;
        for (int h = 0; h < 2; ++h) {
          const size_t base = (((size_t)r * 2 + d) * 2 + h) * H;
          for (int j = 1; j < H; ++j) {
            int m = 1;
            while (2 * m <= j) m *= 2;
            const int src = (2 + h) * m + (j - m);
            sub[base + j] = full[src];
            sub_s[base + j] = full_s[src];
            subd[base + j] = (double)full[src];
          }
        }
      }
    if (!c->d_sub.alloc(&c->alloc, sub.size()) || !c->d_sub_s.alloc(&c->alloc, sub_s.size()) ||
        !c->d_sub_d.alloc(&c->alloc, subd.size()))
      return SFHE_E_NOMEM;
    SFHE_HIP(hipMemcpy(c->d_sub.ptr, sub.data(), sub.size() * sizeof(u64), hipMemcpyHostToDevice));
    SFHE_HIP(hipMemcpy(c->d_sub_s.ptr, sub_s.data(), sub_s.size() * sizeof(u64), hipMemcpyHostToDevice));
    SFHE_HIP(hipMemcpy(c->d_sub_d.ptr, subd.data(), subd.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  // slot-0 decoding / encoding weights, from the host libm
  std::vector<double> cv(N);
  for (int t = 0; t < N; ++t) cv[t] = cos(M_PI * (double)t / (double)N);
  if (!c->d_cos.alloc(&c->alloc, N)) return SFHE_E_NOMEM;
  SFHE_HIP(hipMemcpy(c->d_cos.ptr, cv.data(), N * sizeof(double), hipMemcpyHostToDevice));
  // discrete Gaussian cumulative table over |e| = 0..19:
  // T[k] = floor(2^63 P(|e| <= k)), rho(x) = exp(-x^2 / (2 sigma^2))
  {
    double rho[kCdtLen];
    for (int x = 0; x < kCdtLen; ++x) rho[x] = exp(-(double)(x * x) / (2.0 * c->sigma * c->sigma));
    double total = rho[0];
    for (int x = 1; x < kCdtLen; ++x) total += 2.0 * rho[x];
    double run = rho[0];
    for (int k = 0; k < kCdtLen; ++k) {
      if (k > 0) run += 2.0 * rho[k];
      c->cdt[k] = (u64)((run / total) * 9223372036854775808.0);
    }
  }
  // base-conversion constants
  const int L = c->L, al = c->alpha, dnum = c->dnum;
  std::vector<ModUpConst> mu((size_t)L * dnum);
  std::vector<ModDownConst> md(L);
  std::vector<RescaleConst> rs(L);
  std::memset(mu.data(), 0, mu.size() * sizeof(ModUpConst));
  std::memset(md.data(), 0, md.size() * sizeof(ModDownConst));
  std::memset(rs.data(), 0, rs.size() * sizeof(RescaleConst));
  auto basis_of = [&](int lev, int e) { return e <= lev ? e : L + (e - lev - 1); };
  for (int lev = 0; lev < L; ++lev) {
    const int nl = lev + 1;
    for (int j = 0; j < dnum; ++j) {
      ModUpConst& m = mu[(size_t)lev * dnum + j];
      m.lo = j * al;
      m.hi = std::min((j + 1) * al, nl);
      m.ne = nl + al;
      for (int e = 0; e < m.ne; ++e) m.basis[e] = basis_of(lev, e);
      if (m.lo >= m.hi) continue;
      for (int i = m.lo; i < m.hi; ++i) {
        const u64 qi = c->primes[i];
        u64 dq = 1;   // (D/q_i) mod q_i
        for (int i2 = m.lo; i2 < m.hi; ++i2)
          if (i2 != i) dq = mulmod(dq, c->primes[i2] % qi, qi);
        m.inv[i - m.lo] = invmod(dq, qi);
        m.inv_s[i - m.lo] = shoup(m.inv[i - m.lo], qi);
        m.inv_n[i - m.lo] = mulmod(m.inv[i - m.lo], invmod((u64)N % qi, qi), qi);
        m.inv_n_s[i - m.lo] = shoup(m.inv_n[i - m.lo], qi);
        for (int e = 0; e < m.ne; ++e) {
          const u64 qe = c->primes[m.basis[e]];
          u64 v = 1;  // (D/q_i) mod q_e
          for (int i2 = m.lo; i2 < m.hi; ++i2)
            if (i2 != i) v = mulmod(v, c->primes[i2] % qe, qe);
          m.conv[i - m.lo][e] = v;
          m.conv_s[i - m.lo][e] = shoup(v, qe);
        }
      }
      for (int e = 0; e < m.ne; ++e) {
        const u64 qe = c->primes[m.basis[e]];
        u64 v = 1;  // D mod q_e
        for (int i2 = m.lo; i2 < m.hi; ++i2) v = mulmod(v, c->primes[i2] % qe, qe);
        m.dmod[e] = v;
        m.dmod_s[e] = shoup(v, qe);
      }
    }
    ModDownConst& d = md[lev];
    for (int k = 0; k < al; ++k) {
      const u64 pk = c->primes[L + k];
      u64 v = 1;
      for (int k2 = 0; k2 < al; ++k2)
        if (k2 != k) v = mulmod(v, c->primes[L + k2] % pk, pk);
      d.pinv[k] = invmod(v, pk);
      d.pinv_s[k] = shoup(d.pinv[k], pk);
      d.pinv_n[k] = mulmod(d.pinv[k], invmod((u64)N % pk, pk), pk);
      d.pinv_n_s[k] = shoup(d.pinv_n[k], pk);
      for (int i = 0; i < nl; ++i) {
        const u64 qi = c->primes[i];
        u64 w = 1;
        for (int k2 = 0; k2 < al; ++k2)
          if (k2 != k) w = mulmod(w, c->primes[L + k2] % qi, qi);
        d.conv[k][i] = w;
        d.conv_s[k][i] = shoup(w, qi);
      }
    }
    for (int i = 0; i < nl; ++i) {
      const u64 qi = c->primes[i];
      u64 P = 1;
      for (int k = 0; k < al; ++k) P = mulmod(P, c->primes[L + k] % qi, qi);
      d.Pinv[i] = invmod(P, qi);
      d.Pinv_s[i] = shoup(d.Pinv[i], qi);
      d.Pq[i] = P;
      for (int k = 0; k < al; ++k) {
        d.convp[k][i] = mulmod(d.conv[k][i], d.Pinv[i], qi);
        d.convp_s[k][i] = shoup(d.convp[k][i], qi);
      }
    }
    RescaleConst& rc = rs[lev];
    for (int i = 0; i < lev; ++i) {
      const u64 qi = c->primes[i];
      rc.qinv[i] = invmod(c->primes[lev] % qi, qi);
      rc.qinv_s[i] = shoup(rc.qinv[i], qi);
    }
  }
  if (!c->d_modup.alloc(&c->alloc, mu.size()) || !c->d_moddown.alloc(&c->alloc, md.size()) ||
      !c->d_rescale.alloc(&c->alloc, rs.size()))
    return SFHE_E_NOMEM;
  SFHE_HIP(hipMemcpy(c->d_modup.ptr, mu.data(), mu.size() * sizeof(ModUpConst), hipMemcpyHostToDevice));
  SFHE_HIP(hipMemcpy(c->d_moddown.ptr, md.data(), md.size() * sizeof(ModDownConst), hipMemcpyHostToDevice));
  SFHE_HIP(hipMemcpy(c->d_rescale.ptr, rs.data(), rs.size() * sizeof(RescaleConst), hipMemcpyHostToDevice));
  return SFHE_OK;
}

// Which designs can transform this ring (each gives the same bits in the
// library's storage order): the register design at N >= 2^14, the LDS
// designs at N <= 2^14 (N = 2^15 runs halves of the register design only).
static bool ntt_variant_applies(const sfhe_ctx* c, int v) {
  if (v == kNttRegister) return c->logN >= 14;
  return v >= kNttRadix16 && v <= kNttRadix4 && c->logN <= 14;
}

// Time every applicable design on a scratch batch of about 2048 rows (groups
// of one row per basis prime: enough blocks to fill the chip; 1 warm-up and
// 3 timed launches each) and keep the fastest per direction.
static int tune_ntt(sfhe_ctx* c) {
  for (int d = 0; d < 2; ++d) {
    c->ntt_var[d] = c->ntt_tuned[d] = c->logN >= 14 ? kNttRegister : kNttRadix16;
    for (int v = 0; v < 4; ++v) c->ntt_us[d][v] = -1.0;
  }
  if (c->logN > 14) return SFHE_OK;
  const int N = c->N, nb = c->nb, groups = (2048 + nb - 1) / nb, reps = 3;
  DevBuf<u64> buf;
  if (!buf.alloc(&c->alloc, (size_t)groups * nb * N)) { set_error("NTT tuning: device allocation failed"); return SFHE_E_NOMEM; }
  SFHE_HIP(hipMemset(buf.ptr, 0, (size_t)groups * nb * N * sizeof(u64)));
  int pos[2 * kMaxBasis], pr[2 * kMaxBasis];
  for (int r = 0; r < nb; ++r) { pos[r] = r; pr[r] = r; }
  hipEvent_t e0, e1;
  SFHE_HIP(hipEventCreate(&e0));
  SFHE_HIP(hipEventCreate(&e1));
  int rc = SFHE_OK;
  for (int d = 0; d < 2 && !rc; ++d) {
    double best = 1e30;
    for (int v = 0; v < 4 && !rc; ++v) {
      if (!ntt_variant_applies(c, v)) continue;
      c->ntt_var[d] = v;
      rc = launch_ntt(c, buf.ptr, groups, (int64_t)nb * N, nb, pos, pr, d == 1, 0);
      if (!rc && hipEventRecord(e0, 0) != hipSuccess) rc = SFHE_E_DEVICE;
      for (int x = 0; x < reps && !rc; ++x) rc = launch_ntt(c, buf.ptr, groups, (int64_t)nb * N, nb, pos, pr, d == 1, 0);
      float ms = 0.f;
      if (!rc && (hipEventRecord(e1, 0) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess)) {
        rc = SFHE_E_DEVICE;
        set_error("NTT tuning: event timing failed");
      }
      if (rc) break;
      const double us = (double)ms * 1e3 / reps / (groups * nb);
      c->ntt_us[d][v] = us;
      if (us < best) { best = us; c->ntt_tuned[d] = v; }
    }
    c->ntt_var[d] = c->ntt_tuned[d];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

static int gen_primes(sfhe_ctx* c, const std::vector<uint32_t>& bits) {
  const u64 two_n = 2 * (u64)c->N;
  for (size_t r = 0; r < bits.size(); ++r) {
    const u64 top = 1ull << bits[r];
    u64 cand = (top - 1) / two_n * two_n + 1;   // largest value = 1 mod 2N below 2^bits
    if (cand >= top) cand -= two_n;
    for (;;) {
      if (cand <= two_n) return SFHE_E_PARAMS;
      if (std::find(c->primes.begin(), c->primes.end(), cand) == c->primes.end() && hostmath::is_prime(cand)) break;
      cand -= two_n;
    }
    c->primes.push_back(cand);
  }
  return SFHE_OK;
}

// rows visited by row i of A under its encoding
static int64_t row_visits(const sfhe_mat* A, int i) {
  switch (A->enc) {
    case SFHE_ENC_DENSE: return A->cols;
    case SFHE_ENC_NAIVE_SPARSE: {
      int64_t n = 0;
      for (int k = 0; k < A->cols; ++k) {
        const int64_t e = (int64_t)i * A->cols + k;
        n += !((A->zero_mask[e >> 5] >> (e & 31)) & 1u);
      }
      return n;
    }
    case SFHE_ENC_CSR: return A->row_ptr[i + 1] - A->row_ptr[i];
    case SFHE_ENC_ELL: {
      int64_t n = 0;
      for (int s = 0; s < A->ell_w; ++s) n += A->ell_col[(size_t)i * A->ell_w + s] >= 0;
      return n;
    }
  }
  return 0;
}
// the (k, A slot) pairs row i visits, ascending k
static void row_pairs(const sfhe_mat* A, int i, std::vector<std::pair<int, int64_t>>& out) {
  out.clear();
  switch (A->enc) {
    case SFHE_ENC_DENSE:
      for (int k = 0; k < A->cols; ++k) out.push_back({k, (int64_t)i * A->cols + k});
      break;
    case SFHE_ENC_NAIVE_SPARSE:
      for (int k = 0; k < A->cols; ++k) {
        const int64_t e = (int64_t)i * A->cols + k;
        if (!((A->zero_mask[e >> 5] >> (e & 31)) & 1u)) out.push_back({k, e});
      }
      break;
    case SFHE_ENC_CSR:
      for (int p = A->row_ptr[i]; p < A->row_ptr[i + 1]; ++p) out.push_back({A->col_idx[p], (int64_t)p});
      break;
    case SFHE_ENC_ELL:
      for (int s = 0; s < A->ell_w; ++s) {
        const int k = A->ell_col[(size_t)i * A->ell_w + s];
        if (k >= 0) out.push_back({k, (int64_t)i * A->ell_w + s});
      }
      break;
  }
}

// stored slot of element (i, j), or -1
static int64_t slot_of(const sfhe_mat* m, int i, int j) {
  switch (m->enc) {
    case SFHE_ENC_DENSE:
    case SFHE_ENC_NAIVE_SPARSE: return (int64_t)i * m->cols + j;
    case SFHE_ENC_CSR:
      for (int p = m->row_ptr[i]; p < m->row_ptr[i + 1]; ++p)
        if (m->col_idx[p] == j) return p;
      return -1;
    case SFHE_ENC_ELL:
      for (int s = 0; s < m->ell_w; ++s)
        if (m->ell_col[(size_t)i * m->ell_w + s] == j) return (int64_t)i * m->ell_w + s;
      return -1;
  }
  return -1;
}

// The plaintext structure of encoding m->enc (Sec. 3.3.2) for the rows x cols
// matrix vals (leading dimension ld), and the storage slot of every stored
// element: push(i, j, slot) is called once per stored element.
template <typename Push>
static void build_structure(sfhe_mat* m, const double* vals, int64_t ld, Push push) {
  const int rows = m->rows, cols = m->cols;
  const sfhe_encoding enc = m->enc;
  auto nz = [&](int i, int j) { return vals[(int64_t)i * ld + j] != 0.0; };
  int64_t nnz = 0;
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < cols; ++j) nnz += nz(i, j);
  m->nnz = nnz;
  switch (enc) {
    case SFHE_ENC_DENSE:
    case SFHE_ENC_NAIVE_SPARSE:
      m->n_ct = (int64_t)rows * cols;
      for (int i = 0; i < rows; ++i)
        for (int j = 0; j < cols; ++j) push(i, j, (int64_t)i * cols + j);
      if (enc == SFHE_ENC_NAIVE_SPARSE) {
        m->zero_mask.assign((size_t)((int64_t)rows * cols + 31) / 32, 0u);
        for (int i = 0; i < rows; ++i)
          for (int j = 0; j < cols; ++j)
            if (!nz(i, j)) {
              const int64_t e = (int64_t)i * cols + j;
              m->zero_mask[e >> 5] |= 1u << (e & 31);
            }
      }
      break;
    case SFHE_ENC_CSR:
      m->row_ptr.assign(rows + 1, 0);
      for (int i = 0; i < rows; ++i) {
        m->row_ptr[i] = (int)m->col_idx.size();
        for (int j = 0; j < cols; ++j)
          if (nz(i, j)) { push(i, j, (int64_t)m->col_idx.size()); m->col_idx.push_back(j); }
      }
      m->row_ptr[rows] = (int)m->col_idx.size();
      m->n_ct = (int64_t)m->col_idx.size();
      break;
    case SFHE_ENC_ELL: {
      int w = 0;
      for (int i = 0; i < rows; ++i) {
        int n = 0;
        for (int j = 0; j < cols; ++j) n += nz(i, j);
        w = std::max(w, n);
      }
      m->ell_w = w;
      m->ell_col.assign((size_t)rows * w, -1);
      for (int i = 0; i < rows; ++i) {
        int n = 0;
        for (int j = 0; j < cols; ++j)
          if (nz(i, j)) { m->ell_col[(size_t)i * w + n] = j; push(i, j, (int64_t)i * w + n); ++n; }
      }
      m->n_ct = (int64_t)rows * w;
      break;
    }
  }
}

// stored slot of every element of a sparse-encoded matrix as a value to
// multiply, -1 for a zero: [rows][cols] (the right operand's side of the
// both-sparse product)
static void value_slots(const sfhe_mat* m, std::vector<int>& out) {
  out.assign((size_t)m->rows * m->cols, -1);
  switch (m->enc) {
    case SFHE_ENC_DENSE:
      for (int64_t e = 0; e < (int64_t)m->rows * m->cols; ++e) out[e] = (int)e;
      break;
    case SFHE_ENC_NAIVE_SPARSE:
      for (int64_t e = 0; e < (int64_t)m->rows * m->cols; ++e)
        if (!((m->zero_mask[e >> 5] >> (e & 31)) & 1u)) out[e] = (int)e;
      break;
    case SFHE_ENC_CSR:
      for (int r = 0; r < m->rows; ++r)
        for (int p = m->row_ptr[r]; p < m->row_ptr[r + 1]; ++p) out[(size_t)r * m->cols + m->col_idx[p]] = p;
      break;
    case SFHE_ENC_ELL:
      for (int r = 0; r < m->rows; ++r)
        for (int x = 0; x < m->ell_w; ++x) {
          const int col = m->ell_col[(size_t)r * m->ell_w + x];
          if (col >= 0) out[(size_t)r * m->cols + col] = r * m->ell_w + x;
        }
      break;
  }
}

}  // namespace sfhe

using namespace sfhe;

#define GUARD_BEGIN try {
#define GUARD_END                                                   \
  }                                                                 \
  catch (const std::bad_alloc&) {                                   \
    set_error("host allocation failed");                            \
    return SFHE_E_NOMEM;                                            \
  }                                                                 \
  catch (...) {                                                     \
    set_error("unexpected internal error");                         \
    return SFHE_E_INVALID_ARG;                                      \
  }

extern "C" {

const char* sfhe_last_error(void) { return g_err.c_str(); }

int sfhe_ctx_create(const sfhe_params* p, const sfhe_device_hooks* hooks, sfhe_ctx** out) {
  GUARD_BEGIN
  if (!out) { set_error("out is NULL"); return SFHE_E_INVALID_ARG; }
  *out = nullptr;
  if (!p || !p->q_bits || !p->p_bits) { set_error("params or bit lists are NULL"); return SFHE_E_INVALID_ARG; }
  if (p->log_n < 10 || p->log_n > 15) { set_error("log_n must be in [10, 15]"); return SFHE_E_PARAMS; }
  if (p->n_q < 2 || p->n_p < 1 || p->n_q + p->n_p > (uint32_t)kMaxBasis || p->n_p > (uint32_t)kMaxDigit) {
    set_error("need 2 <= n_q, 1 <= n_p <= 8, n_q + n_p <= 16");
    return SFHE_E_PARAMS;
  }
  if (p->dnum != (p->n_q + p->n_p - 1) / p->n_p) { set_error("dnum must equal ceil(n_q / n_p)"); return SFHE_E_PARAMS; }
  if (!(p->log2_scale >= 1 && p->log2_scale <= 60 && p->log2_scale == floor(p->log2_scale))) {
    set_error("log2_scale must be an integer in [1, 60]");
    return SFHE_E_PARAMS;
  }
  if (!(p->sigma > 0 && p->sigma < 100)) { set_error("sigma out of range"); return SFHE_E_PARAMS; }
  std::vector<uint32_t> bits;
  for (uint32_t i = 0; i < p->n_q; ++i) bits.push_back(p->q_bits[i]);
  for (uint32_t i = 0; i < p->n_p; ++i) bits.push_back(p->p_bits[i]);
  for (uint32_t b : bits)
    if (b < p->log_n + 2 || b > 61) { set_error("prime bit sizes must be in [log_n + 2, 61]"); return SFHE_E_PARAMS; }

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) { set_error("no HIP device"); return SFHE_E_DEVICE; }
  int dev = 0;
  SFHE_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  SFHE_HIP(hipGetDeviceProperties(&prop, dev));
  if (std::string(prop.gcnArchName).find("gfx950") == std::string::npos) {
    set_error(std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
    return SFHE_E_DEVICE;
  }

  sfhe_ctx* c = new sfhe_ctx();
  c->device = dev;
  c->logN = (int)p->log_n;
  c->N = 1 << c->logN;
  c->L = (int)p->n_q;
  c->alpha = (int)p->n_p;
  c->dnum = (int)p->dnum;
  c->nb = c->L + c->alpha;
  c->log2_scale = p->log2_scale;
  c->sigma = p->sigma;
  if (hooks) {
    if (!hooks->alloc || !hooks->free) { delete c; set_error("hooks need alloc and free"); return SFHE_E_INVALID_ARG; }
    c->alloc.hooks = *hooks;
    c->alloc.has_hooks = true;
  } else {
    // a stream-ordered pool that keeps freed blocks for reuse (no release
    // back to the driver at synchronisation points)
    hipMemPoolProps pp;
    std::memset(&pp, 0, sizeof(pp));
    pp.allocType = hipMemAllocationTypePinned;
    pp.handleTypes = hipMemHandleTypeNone;
    pp.location.type = hipMemLocationTypeDevice;
    pp.location.id = dev;
    hipError_t e = hipMemPoolCreate(&c->alloc.pool, &pp);
    if (e == hipSuccess) {
      uint64_t keep = UINT64_MAX;
      e = hipMemPoolSetAttribute(c->alloc.pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    // a block whose free has completed may be taken by any stream (streams
    // come and go: a server's, a caller's side streams); blocks freed by work
    // still in flight are reused only in that work's order
    const hipMemPoolAttr reuse[3] = {hipMemPoolReuseFollowEventDependencies, hipMemPoolReuseAllowOpportunistic,
                                     hipMemPoolReuseAllowInternalDependencies};
    for (int x = 0; x < 3 && e == hipSuccess; ++x) {
      int on = 1;
      e = hipMemPoolSetAttribute(c->alloc.pool, reuse[x], &on);
    }
    if (e != hipSuccess) {
      set_error(std::string("device memory pool: ") + hipGetErrorString(e));
      if (c->alloc.pool) (void)hipMemPoolDestroy(c->alloc.pool);
      delete c;
      return SFHE_E_DEVICE;
    }
  }
  int rc = gen_primes(c, bits);
  if (rc) { delete c; set_error("not enough NTT primes of the requested sizes"); return rc; }
  c->dp.N = c->N;
  c->dp.logN = c->logN;
  c->dp.L = c->L;
  c->dp.alpha = c->alpha;
  c->dp.dnum = c->dnum;
  c->dp.nb = c->nb;
  rc = build_tables(c);
  if (rc) {
    if (rc == SFHE_E_NOMEM) set_error("device allocation failed while building tables");
    delete c;
    return rc;
  }
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
    delete c;
    set_error("hipEventCreate failed");
    return SFHE_E_DEVICE;
  }
  rc = tune_ntt(c);
  if (!rc) rc = noalloc_setup(c);
  if (rc) {
    delete c;
    return rc;
  }
  *out = c;
  return SFHE_OK;
  GUARD_END
}

int sfhe_ntt_tuning(const sfhe_ctx* c, int32_t inverse, int32_t* variant, double* us_per_row, int32_t cap) {
  if (!c || !variant) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  const int d = inverse ? 1 : 0;
  *variant = c->ntt_var[d];
  if (us_per_row)
    for (int v = 0; v < 4 && v < cap; ++v) us_per_row[v] = c->ntt_us[d][v];
  return SFHE_OK;
}

int sfhe_set_ntt_variant(sfhe_ctx* c, int32_t inverse, int32_t variant) {
  if (!c) { set_error("NULL context"); return SFHE_E_INVALID_ARG; }
  const int d = inverse ? 1 : 0;
  if (variant == -1) { c->ntt_var[d] = c->ntt_tuned[d]; return SFHE_OK; }
  if (!ntt_variant_applies(c, variant)) { set_error("this NTT design does not apply to the ring"); return SFHE_E_UNSUPPORTED; }
  c->ntt_var[d] = variant;
  return SFHE_OK;
}

int sfhe_ks_tuning(const sfhe_ctx* c, int32_t* slice, int32_t* streams, int32_t* sizes, double* us_per_output,
                   int32_t cap, int32_t* sizes2, double* us_per_output2) {
  if (!c || !slice) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  *slice = c->ks_slice;
  if (streams) *streams = c->ks_streams;
  for (int x = 0; x < 2; ++x) {
    if (sizes2) sizes2[x] = (int32_t)c->ks_s2[x];
    if (us_per_output2) us_per_output2[x] = c->ks_us2[x];
  }
  for (int x = 0; x < kKsNumCandidates && x < cap; ++x) {
    if (sizes) sizes[x] = (int32_t)kKsCandidates[x];
    if (us_per_output) us_per_output[x] = c->ks_us[x];
  }
  return SFHE_OK;
}

int sfhe_set_ks_slice(sfhe_ctx* c, int32_t slice, int32_t streams) {
  if (!c) { set_error("NULL context"); return SFHE_E_INVALID_ARG; }
  if (slice == -1) {
    c->ks_slice = c->ks_tuned_slice;
    c->ks_streams = c->ks_tuned_streams;
    return SFHE_OK;
  }
  if (slice != 0 && (slice < 64 || slice > 4096 || (slice & (slice - 1)))) {
    set_error("slice must be a power of two in [64, 4096], 0 (tune again) or -1 (the tuned choice)");
    return SFHE_E_INVALID_ARG;
  }
  if (streams != 1 && streams != 2) { set_error("streams must be 1 or 2"); return SFHE_E_INVALID_ARG; }
  c->ks_slice = slice;
  c->ks_streams = streams;
  return SFHE_OK;
}

int sfhe_set_profiling(sfhe_ctx* c, int32_t on) {
  if (!c) { set_error("NULL context"); return SFHE_E_INVALID_ARG; }
  c->profiling = on != 0;
  return SFHE_OK;
}

void sfhe_ctx_destroy(sfhe_ctx* c) {
  if (!c) return;
  // work of any stream may still read the context's tables and keys
  (void)hipDeviceSynchronize();
  for (hipEvent_t e : c->prof_pool) (void)hipEventDestroy(e);
  for (int k = 0; k < 2; ++k) {
    if (c->ks_side[k]) (void)hipStreamDestroy(c->ks_side[k]);
    if (c->ks_join[k]) (void)hipEventDestroy(c->ks_join[k]);
  }
  if (c->ks_fork) (void)hipEventDestroy(c->ks_fork);
  if (c->tune_ev0) (void)hipEventDestroy(c->tune_ev0);
  if (c->tune_ev1) (void)hipEventDestroy(c->tune_ev1);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  hipMemPool_t pool = c->alloc.pool;
  delete c;   // gives the tables and keys back (stream-ordered)
  if (pool) {
    (void)hipDeviceSynchronize();
    (void)hipMemPoolDestroy(pool);
  }
}

int sfhe_ctx_n(const sfhe_ctx* c, int32_t* n) {
  if (!c || !n) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  *n = c->N;
  return SFHE_OK;
}

int sfhe_ctx_primes(const sfhe_ctx* c, uint64_t* out, size_t cap) {
  if (!c || !out) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  if (cap < (size_t)c->nb) { set_error("capacity below the basis size"); return SFHE_E_INVALID_ARG; }
  for (int r = 0; r < c->nb; ++r) out[r] = c->primes[r];
  return SFHE_OK;
}

int sfhe_keygen(sfhe_ctx* c, uint64_t seed) {
  GUARD_BEGIN
  if (!c) { set_error("NULL context"); return SFHE_E_INVALID_ARG; }
  c->has_keys = false;
  int rc = keygen_device(c, seed, nullptr);
  if (rc) return rc;
  c->has_keys = true;
  return SFHE_OK;
  GUARD_END
}

int sfhe_encrypt_matrix(sfhe_ctx* c, const double* vals, int32_t rows, int32_t cols, int64_t ld, sfhe_encoding enc,
                        uint64_t seed, uint32_t operand_id, void* stream, sfhe_mat** out) {
  GUARD_BEGIN
  if (!out) { set_error("out is NULL"); return SFHE_E_INVALID_ARG; }
  *out = nullptr;
  if (!c || !vals) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  if (!c->has_keys) { set_error("keygen first"); return SFHE_E_STATE; }
  if (rows < 1 || cols < 1 || ld < cols) { set_error("bad shape or leading dimension"); return SFHE_E_SHAPE; }
  if ((int)enc < 0 || (int)enc > 3) { set_error("bad encoding"); return SFHE_E_INVALID_ARG; }
  hipStream_t s = (hipStream_t)stream;
  StreamScope scope_(c->alloc, s);
  const double lim = ldexp(1.0, 62 - ((int)c->log2_scale + 1 - c->logN));
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < cols; ++j) {
      const double v = vals[(int64_t)i * ld + j];
      if (!(fabs(v) < lim)) { set_error("value not finite or too large to encode"); return SFHE_E_INVALID_ARG; }
    }
  sfhe_mat* m = new sfhe_mat();
  m->ctx = c;
  m->rows = rows;
  m->cols = cols;
  m->level = c->L - 1;
  m->scale = ldexp(1.0, (int)c->log2_scale);
  m->enc = enc;
  std::vector<int> ei, ej;
  std::vector<double> z;
  std::vector<int64_t> slot;
  build_structure(m, vals, ld, [&](int i, int j, int64_t sl) {
    ei.push_back(i);
    ej.push_back(j);
    z.push_back(vals[(int64_t)i * ld + j]);
    slot.push_back(sl);
  });
  const int N = c->N, L = c->L;
  int rc = SFHE_OK;
  const size_t words = (size_t)m->n_ct * 2 * L * N;
  if (!m->data.alloc(&c->alloc, words)) { delete m; set_error("device allocation failed for the ciphertexts"); return SFHE_E_NOMEM; }
  if (enc == SFHE_ENC_ELL) rc = launch_zero(m->data.ptr, (int64_t)words, s);   // padding: trivial zeros
  DevBuf<int> d_ei, d_ej;
  DevBuf<double> d_z;
  DevBuf<int64_t> d_slot;
  DevBuf<u64> tmp;
  const int64_t count = (int64_t)ei.size();
  const int64_t chunk = std::min<int64_t>(std::max<int64_t>(count, 1), 1024);
  if (!rc && (!upload(c, d_ei, ei, s) || !upload(c, d_ej, ej, s) || !upload(c, d_z, z, s) || !upload(c, d_slot, slot, s) ||
              !tmp.alloc(&c->alloc, (size_t)chunk * 2 * L * N))) {
    rc = SFHE_E_NOMEM;
    set_error("device allocation failed");
  }
  // per chunk of elements: sample, NTT, c0 -= c1 s, then store in the chunked layout
  for (int64_t x0 = 0; x0 < count && !rc; x0 += chunk) {
    const int64_t n = std::min(chunk, count - x0);
    rc = encrypt_elements(c, tmp.ptr, n, d_ei.ptr + x0, d_ej.ptr + x0, d_z.ptr + x0, seed, operand_id, s);
    if (!rc) rc = encrypt_finish(c, tmp.ptr, n, s);
    if (!rc) rc = launch_to_chunked(c, tmp.ptr, (int64_t)2 * L * N, L, n, m->data.ptr, m->n_ct, d_slot.ptr + x0, 0, s);
  }
  if (!rc && (!upload(c, m->d_row_ptr, m->row_ptr, s) || !upload(c, m->d_col_idx, m->col_idx, s) ||
              !upload(c, m->d_ell_col, m->ell_col, s) || !upload(c, m->d_mask, m->zero_mask, s))) {
    rc = SFHE_E_NOMEM;
    set_error("device allocation failed");
  }
  if (!rc && hipStreamSynchronize(s) != hipSuccess) { rc = SFHE_E_DEVICE; set_error("stream synchronize failed"); }
  if (rc) { delete m; return rc; }
  m->n_vals = m->n_ct;
  *out = m;
  return SFHE_OK;
  GUARD_END
}

int sfhe_matrix_info(const sfhe_mat* m, sfhe_mat_info* out) {
  if (!m || !out) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  out->rows = m->rows;
  out->cols = m->cols;
  out->level = m->level;
  out->scale = m->scale;
  out->enc = m->enc;
  out->n_ciphertexts = m->n_ct;
  out->nnz = m->nnz;
  out->ell_width = m->ell_w;
  out->device_bytes = m->plain ? (uint64_t)(m->d_tstart.count + m->d_ek.count + m->d_emask.count) * sizeof(int) +
                                     (uint64_t)(m->d_ew.count + m->d_ews.count) * sizeof(u64)
                                : (uint64_t)m->n_ct * 2 * (m->level + 1) * m->ctx->N * sizeof(u64);
  out->slots = m->slots;
  return SFHE_OK;
}

void sfhe_mat_destroy(sfhe_mat* m) { delete m; }

}  // extern "C"

// Key switching of a run of outputs in slices: slice i goes to stream s
// (nstr = 1) or alternately to the context's two side streams (nstr = 2),
// forked from s after the work already on it and joined back into it, so
// that one slice's memory-bound base conversions overlap the other's
// transforms.  scratch holds nstr slices' working rows.
static int ks_slices(sfhe_ctx* c, int lev, const u64* D, int64_t dw, OutLayout ol, int64_t n, int64_t S, int nstr,
                     u64* scratch, hipStream_t s) {
  const int64_t words = keyswitch_rescale_n14_scratch_words(c, lev, S);
  if (nstr == 2) {
    if (!c->ks_side[0]) {
      for (int k = 0; k < 2; ++k) {
        SFHE_HIP(hipStreamCreateWithFlags(&c->ks_side[k], hipStreamNonBlocking));
        SFHE_HIP(hipEventCreateWithFlags(&c->ks_join[k], hipEventDisableTiming));
      }
      SFHE_HIP(hipEventCreateWithFlags(&c->ks_fork, hipEventDisableTiming));
    }
    SFHE_HIP(hipEventRecord(c->ks_fork, s));
    for (int k = 0; k < 2; ++k) SFHE_HIP(hipStreamWaitEvent(c->ks_side[k], c->ks_fork, 0));
  }
  int rc = SFHE_OK;
  int64_t i = 0;
  for (int64_t o0 = 0; o0 < n && !rc; o0 += S, ++i) {
    OutLayout o = ol;
    o.elem_base += o0;
    const int k = nstr == 2 ? (int)(i & 1) : 0;
    rc = keyswitch_rescale_n14(c, lev, D + o0 * dw, dw, o, std::min(S, n - o0), nstr == 2 ? c->ks_side[k] : s,
                               scratch + k * words);
  }
  if (nstr == 2) {
    // joined even after an error: s must not run ahead of the side streams
    for (int k = 0; k < 2; ++k) {
      SFHE_HIP(hipEventRecord(c->ks_join[k], c->ks_side[k]));
      SFHE_HIP(hipStreamWaitEvent(s, c->ks_join[k], 0));
    }
  }
  return rc;
}

// Key-switch tuning (N = 2^14, fused kernels): the key switch and rescale of
// the first n outputs of a LAZY product's sums D are run for each candidate
// slice size on one stream, then for the best slice and half of it on two
// streams, each timed with an event pair on s; the fastest setting is kept
// in c->ks_slice / c->ks_streams, and c->ks_us / c->ks_us2 record the
// microseconds per output measured.  Every run writes the same ciphertexts,
// so *done = n outputs are finished.
static int tune_ks_slice(sfhe_ctx* c, int lev, const u64* D, int64_t dw, OutLayout ol, int64_t n, hipStream_t s,
                         int64_t* done) {
  *done = 0;
  if (!c->tune_ev0) {
    SFHE_HIP(hipEventCreate(&c->tune_ev0));
    SFHE_HIP(hipEventCreate(&c->tune_ev1));
  }
  const int64_t smax = std::min<int64_t>(n, kKsCandidates[kKsNumCandidates - 1]);
  DevBuf<u64> scr;
  if (!scr.alloc(&c->alloc, (size_t)keyswitch_rescale_n14_scratch_words(c, lev, smax))) {
    set_error("device allocation failed for the key-switch tuning scratch");
    return SFHE_E_NOMEM;
  }
  // microseconds per output of n outputs in slices of S on nstr streams
  auto measure = [&](int64_t S, int nstr, double* us) -> int {
    for (int rep = 0; rep < 2; ++rep) {   // the first run warms the caches and the code objects
      SFHE_HIP(hipEventRecord(c->tune_ev0, s));
      const int rc = ks_slices(c, lev, D, dw, ol, n, S, nstr, scr.ptr, s);
      if (rc) return rc;
      SFHE_HIP(hipEventRecord(c->tune_ev1, s));
      SFHE_HIP(hipEventSynchronize(c->tune_ev1));
    }
    float ms = 0;
    SFHE_HIP(hipEventElapsedTime(&ms, c->tune_ev0, c->tune_ev1));
    *us = 1e3 * ms / (double)n;
    return SFHE_OK;
  };
  double best = 0;
  int best_s = 0, best_str = 1;
  for (int x = 0; x < kKsNumCandidates; ++x) {
    c->ks_us[x] = -1;
    const int64_t S = kKsCandidates[x];
    if (S > n) continue;
    const int rc = measure(S, 1, &c->ks_us[x]);
    if (rc) return rc;
    if (best_s == 0 || c->ks_us[x] < best) { best = c->ks_us[x]; best_s = (int)S; }
  }
  // two streams: two slices in flight share the one-stream scratch
  c->ks_us2[0] = c->ks_us2[1] = -1;
  c->ks_s2[0] = std::min<int64_t>(best_s, smax / 2);
  c->ks_s2[1] = c->ks_s2[0] / 2;
  for (int x = 0; x < 2; ++x) {
    const int64_t S = c->ks_s2[x];
    if (S < kKsCandidates[0] || 2 * S > n) continue;
    const int rc = measure(S, 2, &c->ks_us2[x]);
    if (rc) return rc;
    if (c->ks_us2[x] < best) { best = c->ks_us2[x]; best_s = (int)S; best_str = 2; }
  }
  c->ks_slice = best_s;
  c->ks_tuned_slice = best_s;
  c->ks_streams = c->ks_tuned_streams = best_str;
  *done = n;
  return SFHE_OK;
}

// ---------------------------------------------------------------- LAZY product
// Everything the LAZY product's launches read or write, prepared before
// them, so that the launches alone can also be captured into a graph: the
// result, the tile lists of every batch (one per tile height: kTileRows for
// the 128-bit integer kernel, kColTileRows for the fp64 and carry-save column
// kernels), the lazy sums D, the key-switch scratch, the B slot table and the
// outputs with no product.
struct LazyPrep {
  struct Batch { int r0, nr, t0, nt, q0, qnt; };
  sfhe_mat* out = nullptr;
  const sfhe_mat *A = nullptr, *B = nullptr;
  std::vector<Batch> batches;
  DevBuf<int> d_ts, d_ek, d_em, d_es, q_ts, q_ek, q_em, q_es, d_bs;
  DevBuf<u64> D, kss;
  int kss_streams = 0;   // key-switch streams the scratch kss is sized for
  int64_t kss_slice = 0; // and its slice size
  DevBuf<int64_t> d_empty;
  int64_t n_empty = 0, products = 0, keyswitches = 0, max_out = 0, ks_slice = 2048, dw = 0;
  int lev = 0, Nc = 0;
  bool bsp = false, fused = false;
  ~LazyPrep() { delete out; }
};

// host tables and uploads of a LAZY product (P.out holds the allocated result)
static int lazy_prepare(sfhe_ctx* c, const sfhe_mat* A, const sfhe_mat* B, hipStream_t s, LazyPrep& P) {
  const int N = c->N, lev = A->level, nl = lev + 1, M = A->rows, Nc = B->cols;
  P.A = A;
  P.B = B;
  P.lev = lev;
  P.Nc = Nc;
  std::vector<int64_t> visits(M);
  for (int i = 0; i < M; ++i) visits[i] = row_visits(A, i);
  // a sparse right operand: products whose B_kj is zero are skipped too
  P.bsp = B->enc != SFHE_ENC_DENSE;
  std::vector<int> bslot;
  if (P.bsp) value_slots(B, bslot);
  // outputs with no product are trivial zeros
  std::vector<int64_t> empty;
  for (int i = 0; i < M; ++i)
    if (visits[i] == 0)
      for (int j = 0; j < Nc; ++j) empty.push_back((int64_t)i * Nc + j);
  P.n_empty = (int64_t)empty.size();
  // batches: runs of consecutive non-empty rows whose degree-2 sums D fit a
  // 32 GiB budget (all 128 rows at N = 2^14, L = 5); one tensor launch per
  // batch, then key switching and rescaling in slices
  const int64_t dw = (int64_t)3 * nl * N;
  P.dw = dw;
  const int64_t d_budget = (int64_t)32 << 30;
  int rb = (int)std::max<int64_t>(kTileRows, d_budget / ((int64_t)std::max(Nc, 1) * dw * 8) / kTileRows * kTileRows);
  P.fused = keyswitch_rescale_n14_supported(c);
  // outputs per key-switch launch group: the fused N = 2^14 kernels take
  // the tuned slice, the others 2048
  P.ks_slice = P.fused && c->ks_slice > 0 ? c->ks_slice : 2048;
  // tile lists: for every tile of TR consecutive rows of a batch, the
  // ascending union of the rows' visited k, each with the mask of the rows
  // that visit it and their A slots
  struct Tiles {
    int TR;
    std::vector<int> tstart, ek, emask, eslot;
  };
  Tiles ti{kTileRows, {}, {}, {}, {}}, tq{kColTileRows, {}, {}, {}, {}};
  std::vector<std::pair<int, int64_t>> pairs;
  std::vector<int> kmask(A->cols);
  std::vector<int> kslot((size_t)A->cols * std::max(kTileRows, kColTileRows));
  // tiles of rows r0 .. r0 + nr - 1 into T; returns the tile count
  auto add_tiles = [&](Tiles& T, int r0, int nr) {
    const int TR = T.TR;
    int nt = 0;
    for (int g = 0; g * TR < nr; ++g) {
      std::fill(kmask.begin(), kmask.end(), 0);
      for (int r = 0; r < TR && g * TR + r < nr; ++r) {
        row_pairs(A, r0 + g * TR + r, pairs);
        for (auto& pr : pairs) {
          kmask[pr.first] |= 1 << r;
          kslot[(size_t)pr.first * TR + r] = (int)pr.second;
        }
      }
      T.tstart.push_back((int)T.ek.size());
      for (int k = 0; k < A->cols; ++k) {
        if (!kmask[k]) continue;
        T.ek.push_back(k);
        T.emask.push_back(kmask[k]);
        for (int r = 0; r < TR; ++r) T.eslot.push_back((kmask[k] >> r) & 1 ? kslot[(size_t)k * TR + r] : -1);
      }
      ++nt;
    }
    return nt;
  };
  for (int i = 0; i < M;) {
    if (visits[i] == 0) { ++i; continue; }
    int nr = 0;
    while (i + nr < M && nr < rb && visits[i + nr] > 0) ++nr;
    LazyPrep::Batch bt{i, nr, (int)ti.tstart.size(), 0, (int)tq.tstart.size(), 0};
    bt.nt = add_tiles(ti, i, nr);
    bt.qnt = add_tiles(tq, i, nr);
    P.batches.push_back(bt);
    for (int r = 0; r < nr; ++r) P.products += visits[i + r] * (int64_t)Nc;
    P.keyswitches += (int64_t)nr * Nc;
    i += nr;
  }
  ti.tstart.push_back((int)ti.ek.size());
  tq.tstart.push_back((int)tq.ek.size());
  if (P.bsp) {   // products: the visited k whose B_kj is stored
    P.products = 0;
    for (int i = 0; i < M; ++i) {
      if (visits[i] == 0) continue;
      row_pairs(A, i, pairs);
      for (auto& pr : pairs)
        for (int j = 0; j < Nc; ++j) P.products += bslot[(size_t)pr.first * Nc + j] >= 0;
    }
  }
  for (auto& bt : P.batches) P.max_out = std::max<int64_t>(P.max_out, (int64_t)bt.nr * Nc);
  if (!upload(c, P.d_ts, ti.tstart, s) || !upload(c, P.d_ek, ti.ek, s) || !upload(c, P.d_em, ti.emask, s) ||
      !upload(c, P.d_es, ti.eslot, s) || !upload(c, P.q_ts, tq.tstart, s) ||
      !upload(c, P.q_ek, tq.ek, s) || !upload(c, P.q_em, tq.emask, s) || !upload(c, P.q_es, tq.eslot, s) ||
      (P.bsp && !upload(c, P.d_bs, bslot, s)) || !upload(c, P.d_empty, empty, s) ||
      !P.D.alloc(&c->alloc, (size_t)std::max<int64_t>(P.max_out, 1) * dw)) {
    set_error("device allocation failed");
    return SFHE_E_NOMEM;
  }
  return SFHE_OK;
}

// the launches of a LAZY product: per batch the tensor step and the key
// switch and rescale in slices, then the trivial zeros.  With events the
// steps are bracketed for sfhe_last_stats (not under graph capture); with
// tune, a context whose slice is not tuned yet tunes it on the first batch.
static int lazy_launch(sfhe_ctx* c, LazyPrep& P, hipStream_t s, bool events, bool tune, int64_t* tensor_launches,
                       int64_t* tensor_fp_launches) {
  const int N = c->N, lev = P.lev, nl = lev + 1, Nc = P.Nc;
  const int64_t dw = P.dw;
  sfhe_mat* out = P.out;
  int rc = SFHE_OK;
  for (size_t bi = 0; bi < P.batches.size() && !rc; ++bi) {
    const LazyPrep::Batch& bt = P.batches[bi];
    TileList tl;
    tl.tstart = P.d_ts.ptr + bt.t0;
    tl.ek = P.d_ek.ptr;
    tl.emask = P.d_em.ptr;
    tl.eslot = P.d_es.ptr;
    tl.n_row_tiles = bt.nt;
    tl.n_col_tiles = 0;
    tl.rows = bt.nr;
    tl.Nc = Nc;
    tl.nA = P.A->n_ct;
    tl.nB = P.B->n_ct;
    tl.bslot = P.bsp ? P.d_bs.ptr : nullptr;
    tl.tile_rows = kTileRows;
    TileList tlq = tl;
    tlq.tstart = P.q_ts.ptr + bt.q0;
    tlq.ek = P.q_ek.ptr;
    tlq.emask = P.q_em.ptr;
    tlq.eslot = P.q_es.ptr;
    tlq.n_row_tiles = bt.qnt;
    tlq.tile_rows = kColTileRows;
    const int64_t cnt = (int64_t)bt.nr * Nc;
    if (events) {
      StepTimer tm(c, s, kCatTensor);
      // the fp64 tensor launch is always bracketed (two events per step):
      // its duration is the dominant kernel's time in every timed product
      hipEvent_t f0 = c->prof_event(), f1 = c->prof_event();
      if (f0 && f1) c->prof_cat.push_back(kCatTensorFp);
      else f0 = f1 = nullptr;
      rc = launch_tensor_tiles(c, tl, tlq, P.A->data.ptr, P.B->data.ptr, P.D.ptr, s, f0, f1);
      if (f0) ++*tensor_fp_launches;
    } else {
      rc = launch_tensor_tiles(c, tl, tlq, P.A->data.ptr, P.B->data.ptr, P.D.ptr, s);
    }
    ++*tensor_launches;
    int64_t o_start = 0;
    if (tune && P.fused && !rc && c->ks_slice == 0 && cnt >= kKsTuneMin) {
      // first LAZY product of the context: time the key switch of the first
      // outputs with each candidate slice and keep the fastest (the outputs
      // are written identically by every candidate)
      rc = tune_ks_slice(c, lev, P.D.ptr, dw, OutLayout{out->data.ptr, 0, true, out->n_ct, (int64_t)bt.r0 * Nc},
                         std::min<int64_t>(cnt, kKsCandidates[kKsNumCandidates - 1]), s, &o_start);
      if (c->ks_slice > 0) P.ks_slice = c->ks_slice;
    }
    // the key-switch (and rescale) scratch of one slice per key-switch
    // stream, allocated once (under graph capture: one stream)
    const int nstr = P.fused && events ? c->ks_streams : 1;
    const int64_t sl = std::min(P.ks_slice, P.max_out);
    if (P.kss.ptr && (nstr > P.kss_streams || sl > P.kss_slice)) P.kss.release();
    const int64_t ks_words = P.fused ? keyswitch_rescale_n14_scratch_words(c, lev, sl) : keyswitch_scratch_words(c, lev, sl);
    if (!rc && !P.kss.ptr) {
      P.kss_streams = nstr;
      P.kss_slice = sl;
      StreamScope scope_(c->alloc, s);
      // rescale_batch's scratch: the last prime's rows and the lifted rows
      const int64_t rs_words = P.fused ? 0 : sl * 2 * N * (1 + lev);
      if (!P.kss.alloc(&c->alloc, (size_t)(nstr * ks_words + rs_words))) {
        rc = SFHE_E_NOMEM;
        set_error("device allocation failed for the key-switch scratch");
      }
    }
    if (P.fused && !rc && o_start < cnt) {   // fused transforms (key switch and rescale together)
      const OutLayout ol{out->data.ptr, 0, true, out->n_ct, (int64_t)bt.r0 * Nc + o_start};
      StepTimer tm(c, s, events ? kCatKeyswitch : -1);
      rc = ks_slices(c, lev, P.D.ptr + o_start * dw, dw, ol, cnt - o_start, P.ks_slice, nstr, P.kss.ptr, s);
    }
    for (int64_t o0 = o_start; o0 < cnt && !rc && !P.fused; o0 += P.ks_slice) {
      const int64_t n = std::min(P.ks_slice, cnt - o0);
      u64* Ds = P.D.ptr + o0 * dw;
      const OutLayout ol{out->data.ptr, 0, true, out->n_ct, (int64_t)bt.r0 * Nc + o0};
      {
        StepTimer tm(c, s, events ? kCatKeyswitch : -1);
        rc = keyswitch_batch(c, lev, Ds + (int64_t)2 * nl * N, dw, Ds, dw, true, n, s, nullptr, P.kss.ptr);
      }
      if (!rc) {
        StepTimer tm(c, s, events ? kCatRescale : -1);
        rc = rescale_batch(c, lev, Ds, dw, ol, n, s, P.kss.ptr + ks_words);
      }
    }
  }
  if (!rc && P.n_empty) rc = launch_zero_outputs(c, out->data.ptr, out->n_ct, lev, P.d_empty.ptr, P.n_empty, s);
  return rc;
}

// The one-value-per-ciphertext product (chunk size 1).  With timed, the
// call's device time is bracketed by the context's event pair.
// operand checks of a one-value-per-ciphertext product
static int matmul_check(const sfhe_ctx* c, const sfhe_mat* A, const sfhe_mat* B, sfhe_schedule sched) {
  if (!c || !A || !B) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  if (A->ctx != c || B->ctx != c) { set_error("matrices belong to another context"); return SFHE_E_INVALID_ARG; }
  if (A->plain || B->plain) { set_error("plaintext weights: use sfhe_matmul_plain"); return SFHE_E_UNSUPPORTED; }
  if (sched != SFHE_SCHED_PER_PRODUCT && sched != SFHE_SCHED_LAZY) { set_error("bad schedule"); return SFHE_E_INVALID_ARG; }
  if (!c->has_keys) { set_error("keygen first"); return SFHE_E_STATE; }
  if (A->cols != B->rows) { set_error("A.cols != B.rows"); return SFHE_E_SHAPE; }
  if ((int64_t)B->rows * B->cols > 0x7FFFFFFF) { set_error("B too large"); return SFHE_E_INVALID_ARG; }
  if (A->level != B->level) { set_error("operand levels differ"); return SFHE_E_LEVEL; }
  if (A->level != c->L - 1) { set_error("operands must be at the top level"); return SFHE_E_LEVEL; }
  if (A->level < 1) { set_error("no prime left to rescale"); return SFHE_E_LEVEL; }
  if (A->scale != B->scale) { set_error("operand scales differ"); return SFHE_E_SCALE; }
  return SFHE_OK;
}

// the (uninitialised) DENSE result of A B: one level lower, scale^2 / q_level
static sfhe_mat* new_product(sfhe_ctx* c, const sfhe_mat* A, const sfhe_mat* B) {
  const int lev = A->level;
  sfhe_mat* out = new sfhe_mat();
  out->ctx = c;
  out->rows = A->rows;
  out->cols = B->cols;
  out->level = lev - 1;
  out->scale = A->scale * B->scale / (double)c->primes[lev];
  out->enc = SFHE_ENC_DENSE;
  out->n_ct = (int64_t)A->rows * B->cols;
  out->nnz = out->n_ct;
  out->n_vals = out->n_ct;
  if (!out->data.alloc(&c->alloc, (size_t)out->n_ct * 2 * lev * c->N)) {
    delete out;
    set_error("device allocation failed for the result");
    return nullptr;
  }
  return out;
}

static int matmul_c1(sfhe_ctx* c, const sfhe_mat* A, const sfhe_mat* B, sfhe_schedule sched, hipStream_t s,
                     sfhe_mat** C, bool timed) {
  if (!C) { set_error("C is NULL"); return SFHE_E_INVALID_ARG; }
  *C = nullptr;
  int rc = matmul_check(c, A, B, sched);
  if (rc) return rc;
  const int N = c->N, lev = A->level, nl = lev + 1, M = A->rows, Nc = B->cols;
  if (timed) SFHE_HIP(hipEventRecord(c->ev0, s));
  sfhe_mat* out = new_product(c, A, B);
  if (!out) return SFHE_E_NOMEM;
  const int64_t ctw = (int64_t)2 * lev * N;   // words per output ciphertext
  std::vector<int64_t> visits(M);
  for (int i = 0; i < M; ++i) visits[i] = row_visits(A, i);
  // a sparse right operand: products whose B_kj is zero are skipped too
  const bool bsp = B->enc != SFHE_ENC_DENSE;
  std::vector<int> bslot;
  if (bsp) value_slots(B, bslot);
  auto b_slot = [&](int k, int j) -> int64_t { return bsp ? bslot[(size_t)k * Nc + j] : (int64_t)k * Nc + j; };
  int64_t products = 0, keyswitches = 0, tensor_launches = 0, tensor_fp_launches = 0;
  c->prof_used = 0;
  c->prof_cat.clear();
  // outputs with no product are trivial zeros
  std::vector<int64_t> empty;
  for (int i = 0; i < M; ++i)
    if (visits[i] == 0)
      for (int j = 0; j < Nc; ++j) empty.push_back((int64_t)i * Nc + j);
  if (sched == SFHE_SCHED_LAZY) {
    LazyPrep P;
    P.out = out;   // P owns the result until it is handed over
    out = nullptr;
    rc = lazy_prepare(c, A, B, s, P);
    if (!rc) rc = lazy_launch(c, P, s, true, true, &tensor_launches, &tensor_fp_launches);
    products = P.products;
    keyswitches = P.keyswitches;
    empty.clear();   // the trivial zeros are part of the LAZY launches
    out = P.out;
    P.out = nullptr;
  } else {
    // Algorithm 1 order: every product is relinearised and rescaled, then summed
    if (!rc) rc = launch_zero(out->data.ptr, out->n_ct * ctw, s);
    const int64_t tile_max = 512;
    std::vector<int> aidx, bidx, seg;
    std::vector<int64_t> oidx;
    std::vector<std::pair<int, int64_t>> pairs;
    DevBuf<u64> D, T;
    DevBuf<int> d_a, d_b, d_seg;
    DevBuf<int64_t> d_o;
    if (!D.alloc(&c->alloc, (size_t)tile_max * 3 * nl * N) || !T.alloc(&c->alloc, (size_t)tile_max * ctw)) {
      rc = SFHE_E_NOMEM;
      set_error("device allocation failed");
    }
    auto flush = [&]() -> int {
      if (aidx.empty()) return SFHE_OK;
      seg.push_back((int)aidx.size());
      const int64_t cnt = (int64_t)aidx.size();
      if (!upload(c, d_a, aidx, s) || !upload(c, d_b, bidx, s) || !upload(c, d_seg, seg, s) || !upload(c, d_o, oidx, s)) {
        set_error("device allocation failed");
        return SFHE_E_NOMEM;
      }
      int r;
      {
        StepTimer tm(c, s, kCatTensor);
        r = launch_tensor_gather(c, lev, A->data.ptr, A->n_ct, B->data.ptr, B->n_ct, d_a.ptr, d_b.ptr, D.ptr, cnt, s);
      }
      ++tensor_launches;
      const int64_t dw = (int64_t)3 * nl * N;
      const OutLayout ol{T.ptr, ctw, false, 0, 0};
      if (!r && keyswitch_rescale_n14_supported(c)) {   // fused transforms (key switch and rescale together)
        StepTimer tm(c, s, kCatKeyswitch);
        r = keyswitch_rescale_n14(c, lev, D.ptr, dw, ol, cnt, s);
      } else if (!r) {
        {
          StepTimer tm(c, s, kCatKeyswitch);
          r = keyswitch_batch(c, lev, D.ptr + (int64_t)2 * nl * N, dw, D.ptr, dw, true, cnt, s);
        }
        if (!r) {
          StepTimer tm(c, s, kCatRescale);
          r = rescale_batch(c, lev, D.ptr, dw, ol, cnt, s);
        }
      }
      if (!r) {
        StepTimer tm(c, s, kCatRescale);
        r = launch_segment_sum(c, lev, T.ptr, out->data.ptr, out->n_ct, d_seg.ptr, d_o.ptr, (int64_t)oidx.size(), s);
      }
      products += cnt;
      keyswitches += cnt;
      aidx.clear();
      bidx.clear();
      seg.clear();
      oidx.clear();
      return r;
    };
    for (int i = 0; i < M && !rc; ++i) {
      if (visits[i] == 0) continue;
      row_pairs(A, i, pairs);
      for (int j = 0; j < Nc && !rc; ++j) {
        bool opened = false;
        for (auto& pr : pairs) {
          const int64_t bs = b_slot(pr.first, j);
          if (bs < 0) continue;   // B_kj is zero
          if ((int64_t)aidx.size() >= tile_max) {
            rc = flush();
            if (rc) break;
            opened = false;
          }
          if (!opened) {
            seg.push_back((int)aidx.size());
            oidx.push_back((int64_t)i * Nc + j);
            opened = true;
          }
          aidx.push_back((int)pr.second);
          bidx.push_back((int)bs);
        }
      }
    }
    if (!rc) rc = flush();
  }
  if (!rc && !empty.empty()) {
    DevBuf<int64_t> d_e;
    if (!upload(c, d_e, empty, s)) { rc = SFHE_E_NOMEM; set_error("device allocation failed"); }
    if (!rc) rc = launch_zero_outputs(c, out->data.ptr, out->n_ct, lev, d_e.ptr, (int64_t)empty.size(), s);
  }
  if (!rc && timed) {
    hipError_t e = hipEventRecord(c->ev1, s);
    if (e != hipSuccess) { rc = SFHE_E_DEVICE; set_error(hipGetErrorString(e)); }
  }
  if (rc) {
    (void)hipStreamSynchronize(s);
    delete out;
    return rc;
  }
  out->n_vals = out->n_ct;
  c->stats = sfhe_stats{};
  c->stats.products = products;
  c->stats.keyswitches = keyswitches;
  c->stats.outputs = out->n_ct;
  c->stats.tensor_launches = tensor_launches;
  c->stats.tensor_fp_launches = tensor_fp_launches;
  c->stats.tensor_fp_primes = tensor_fp_prime_count(c);
  c->stats_pending = timed;
  *C = out;
  return SFHE_OK;
}

extern "C" {

int sfhe_matmul(sfhe_ctx* c, const sfhe_mat* A, const sfhe_mat* B, sfhe_schedule sched, void* stream, sfhe_mat** C) {
  GUARD_BEGIN
  if (A && B && (A->slots > 1 || B->slots > 1)) {
    if (C) *C = nullptr;
    set_error("several values per ciphertext: use sfhe_matmul_slots");
    return SFHE_E_UNSUPPORTED;
  }
  StreamScope scope_(c->alloc, (hipStream_t)stream);
  return matmul_c1(c, A, B, sched, (hipStream_t)stream, C, true);
  GUARD_END
}

}  // extern "C"

// The tile tables of plaintext weights W, built once when W is encoded and
// kept on the device beside it: W's rows in tiles of 16, each tile's entries
// (k, mask of the tile rows that visit k) in ascending k, and per entry and
// data prime the 16 rows' weights (0 where the row does not visit k): the
// residue's fp64 bits below 2^42, else the residue with its Shoup companion.
static int plain_tables(sfhe_ctx* c, sfhe_mat* W) {
  const int M = W->rows, K = W->cols, L = c->L;
  const int ntile = (M + 15) / 16;
  std::vector<int> tstart, ek, emask, kmask(K);
  std::vector<u64> ew, ews;
  std::vector<int64_t> kslot((size_t)K * 16);
  std::vector<std::pair<int, int64_t>> pairs;
  W->w_pairs = 0;
  for (int g = 0; g < ntile; ++g) {
    std::fill(kmask.begin(), kmask.end(), 0);
    for (int r = 0; r < 16 && g * 16 + r < M; ++r) {
      row_pairs(W, g * 16 + r, pairs);
      W->w_pairs += (int64_t)pairs.size();
      for (auto& pr : pairs) {
        kmask[pr.first] |= 1 << r;
        kslot[(size_t)pr.first * 16 + r] = pr.second;
      }
    }
    tstart.push_back((int)ek.size());
    for (int k = 0; k < K; ++k) {
      if (!kmask[k]) continue;
      ek.push_back(k);
      emask.push_back(kmask[k]);
      for (int l = 0; l < L; ++l) {
        const u64 q = c->primes[l];
        for (int r = 0; r < 16; ++r) {
          const u64 w = (kmask[k] >> r) & 1 ? W->w_res[(size_t)kslot[(size_t)k * 16 + r] * L + l] : 0;
          if (q < (1ull << 42)) {
            const double wd = (double)w;
            u64 bits;
            memcpy(&bits, &wd, sizeof(bits));
            ew.push_back(bits);
            ews.push_back(0);
          } else {
            ew.push_back(w);
            ews.push_back(hostmath::shoup(w, q));
          }
        }
      }
    }
  }
  tstart.push_back((int)ek.size());
  if (ek.size() > (size_t)0x7FFFFFFF / 16) { set_error("plaintext weights: too many tile entries"); return SFHE_E_INVALID_ARG; }
  // synchronous copies: the tables are complete when the call returns
  auto put = [&](auto& buf, const auto& v) -> bool {
    if (!buf.alloc(&c->alloc, v.size())) return false;
    return v.empty() || hipMemcpy(buf.ptr, v.data(), v.size() * sizeof(v[0]), hipMemcpyHostToDevice) == hipSuccess;
  };
  if (!put(W->d_tstart, tstart) || !put(W->d_ek, ek) || !put(W->d_emask, emask) || !put(W->d_ew, ew) ||
      !put(W->d_ews, ews)) {
    set_error("device allocation or copy failed for the weight tables");
    return SFHE_E_NOMEM;
  }
  return SFHE_OK;
}

extern "C" {

int sfhe_encode_matrix(sfhe_ctx* c, const double* vals, int32_t rows, int32_t cols, int64_t ld, sfhe_encoding enc,
                       int32_t log2_scale_w, sfhe_mat** out) {
  GUARD_BEGIN
  if (!out) { set_error("out is NULL"); return SFHE_E_INVALID_ARG; }
  *out = nullptr;
  if (!c || !vals) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  if (rows < 1 || cols < 1 || ld < cols) { set_error("bad shape or leading dimension"); return SFHE_E_SHAPE; }
  if ((int)enc < 0 || (int)enc > 3) { set_error("bad encoding"); return SFHE_E_INVALID_ARG; }
  if (log2_scale_w < 0 || log2_scale_w > 62) { set_error("log2_scale_w outside [0, 62]"); return SFHE_E_INVALID_ARG; }
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < cols; ++j) {
      const double x = ldexp(vals[(int64_t)i * ld + j], log2_scale_w);
      if (!(fabs(x) < 4.0e18)) { set_error("weight not finite or too large to encode"); return SFHE_E_INVALID_ARG; }
    }
  sfhe_mat* m = new sfhe_mat();
  m->ctx = c;
  m->rows = rows;
  m->cols = cols;
  m->level = c->L - 1;
  m->scale = ldexp(1.0, log2_scale_w);
  m->enc = enc;
  m->plain = true;
  const int L = c->L;
  std::vector<std::pair<int64_t, double>> stored;   // (slot, weight)
  build_structure(m, vals, ld, [&](int i, int j, int64_t sl) { stored.push_back({sl, vals[(int64_t)i * ld + j]}); });
  // the constant polynomial nearbyint(w 2^sw), reduced per data prime; ELL
  // padding slots stay 0 (never visited)
  m->w_res.assign((size_t)std::max<int64_t>(m->n_ct, 1) * L, 0);
  for (auto& st : stored) {
    const int64_t mi = (int64_t)nearbyint(ldexp(st.second, log2_scale_w));
    for (int l = 0; l < L; ++l) {
      const u64 q = c->primes[l];
      const u64 r = mi >= 0 ? (u64)mi % q : (q - 1) - (u64)(-(mi + 1)) % q;
      m->w_res[(size_t)st.first * L + l] = r;
    }
  }
  std::unique_ptr<sfhe_mat> keep(m);
  const int rc = plain_tables(c, m);
  if (rc) return rc;
  *out = keep.release();
  return SFHE_OK;
  GUARD_END
}

// checks of one plaintext-weight product W B
static int plain_check(const sfhe_ctx* c, const sfhe_mat* W, const sfhe_mat* B) {
  if (!W || !B) { set_error("NULL matrix"); return SFHE_E_INVALID_ARG; }
  if (W->ctx != c || B->ctx != c) { set_error("matrices belong to another context"); return SFHE_E_INVALID_ARG; }
  if (!W->plain) { set_error("the left operand must be plaintext weights (sfhe_encode_matrix)"); return SFHE_E_INVALID_ARG; }
  if (B->plain) { set_error("the right operand must be encrypted"); return SFHE_E_INVALID_ARG; }
  if (B->enc != SFHE_ENC_DENSE) { set_error("the right operand must be DENSE"); return SFHE_E_UNSUPPORTED; }
  if (B->slots > 1) { set_error("the encrypted operand must hold one value per ciphertext"); return SFHE_E_UNSUPPORTED; }
  if (W->cols != B->rows) { set_error("W.cols != B.rows"); return SFHE_E_SHAPE; }
  if (B->level != c->L - 1) { set_error("the encrypted operand must be at the top level"); return SFHE_E_LEVEL; }
  if (B->level < 1) { set_error("no prime left to rescale"); return SFHE_E_LEVEL; }
  return SFHE_OK;
}

constexpr int64_t kRescaleSlice = 2048;   // outputs per rescale launch set

// rescale scratch of a batch: one slice of its largest matrix
static int64_t plain_scratch_words(const sfhe_ctx* c, int64_t max_outputs) {
  return rescale_scratch_words(c, c->L - 1, std::max<int64_t>(1, std::min(kRescaleSlice, max_outputs)));
}

// device bytes a plaintext-weight product holds until it completes: its
// outputs' sums (2 (lev + 1) N words each) and results (2 lev N words each),
// a rescale scratch for one slice of its outputs, and its block descriptors
// (one per tile and group of 4 columns) and job record; W's tile tables are
// W's own, held from its encoding on
static uint64_t plain_bytes(const sfhe_ctx* c, const sfhe_mat* W, const sfhe_mat* B) {
  const int lev = c->L - 1, nl = lev + 1;
  const uint64_t outs = (uint64_t)W->rows * B->cols;
  const uint64_t tiles = (uint64_t)(W->rows + 15) / 16;
  const uint64_t tables = tiles * (uint64_t)((B->cols + 3) / 4) * sizeof(int4) + sizeof(PlainJob);
  return outs * (uint64_t)(2 * nl + 2 * lev) * c->N * sizeof(u64) +
         (uint64_t)plain_scratch_words(c, (int64_t)outs) * sizeof(u64) + tables;
}

// Everything the plaintext-weight launches read or write, allocated and
// uploaded before them, so that the launches alone can also be captured into
// a graph: results, sums, tile tables, per-product weights, rescale scratch.
struct PlainPrep {
  int count = 0;
  sfhe_plain_launch launch = SFHE_PLAIN_FUSED;
  std::vector<sfhe_mat*> C;
  std::vector<const sfhe_mat*> B;
  std::vector<PlainJob> jobs;
  DevBuf<u64> D, pw, pws, scratch;
  DevBuf<int4> desc;
  DevBuf<PlainJob> d_jobs;
  int n_desc = 0;
  std::vector<int64_t> pb_slot, pd;   // one launch per product: B slot, output
  std::vector<int> pjob;
  int64_t products = 0, launches = 0, outs = 0;
  ~PlainPrep() { for (auto* m : C) delete m; }
  // the results, handed over: the caller owns them from here on
  void release(sfhe_mat** out) {
    for (size_t n = 0; n < C.size(); ++n) out[n] = C[n];
    C.clear();
  }
};

// checks, tile tables, results, scratch and uploads (on stream s)
static int plain_prepare(sfhe_ctx* c, int32_t count, const sfhe_mat* const* Wm, const sfhe_mat* const* Bm,
                         sfhe_plain_launch launch, hipStream_t s, PlainPrep& P) {
  if (launch != SFHE_PLAIN_FUSED && launch != SFHE_PLAIN_LAUNCH_PER_PRODUCT) { set_error("bad launch mode"); return SFHE_E_INVALID_ARG; }
  for (int n = 0; n < count; ++n) {
    const int rc = plain_check(c, Wm[n], Bm[n]);
    if (rc) return rc;
  }
  P.count = count;
  P.launch = launch;
  P.B.assign(Bm, Bm + count);
  const int N = c->N, lev = c->L - 1, nl = lev + 1;
  const int64_t dw = (int64_t)2 * nl * N;   // words per output sum
  // per job: its outputs' place in D and W's tile tables; per block group:
  // (job, tile, column group)
  P.jobs.resize(count);
  std::vector<int4> desc;
  std::vector<std::pair<int, int64_t>> pairs;
  int64_t outs = 0, products = 0;
  for (int n = 0; n < count; ++n) {
    const sfhe_mat *W = Wm[n], *B = Bm[n];
    const int M = W->rows, Nc = B->cols;
    P.jobs[n] = PlainJob{B->data.ptr, B->n_ct, Nc, M, W->d_tstart.ptr, W->d_ek.ptr, W->d_emask.ptr,
                         W->d_ew.ptr, W->d_ews.ptr, outs};
    const int ntile = (M + 15) / 16, ncg = (Nc + 3) / 4;
    for (int g = 0; g < ntile; ++g)
      for (int h = 0; h < ncg; ++h) desc.push_back(make_int4(n, g, h, 0));
    products += W->w_pairs * Nc;
    outs += (int64_t)M * Nc;
  }
  P.n_desc = (int)desc.size();
  P.products = products;
  P.outs = outs;
  int64_t max_outs = 1;
  for (int n = 0; n < count; ++n) max_outs = std::max<int64_t>(max_outs, (int64_t)Wm[n]->rows * Bm[n]->cols);
  P.C.assign(count, nullptr);
  for (int n = 0; n < count; ++n) {
    sfhe_mat* o = new sfhe_mat();
    P.C[n] = o;
    o->ctx = c;
    o->rows = Wm[n]->rows;
    o->cols = Bm[n]->cols;
    o->level = lev - 1;
    o->scale = Wm[n]->scale * Bm[n]->scale / (double)c->primes[lev];
    o->enc = SFHE_ENC_DENSE;
    o->n_ct = (int64_t)o->rows * o->cols;
    o->nnz = o->n_ct;
    if (!o->data.alloc(&c->alloc, (size_t)o->n_ct * 2 * lev * N)) { set_error("device allocation failed for a result"); return SFHE_E_NOMEM; }
  }
  if (!P.D.alloc(&c->alloc, (size_t)std::max<int64_t>(outs, 1) * dw) || !upload(c, P.desc, desc, s) ||
      !upload(c, P.d_jobs, P.jobs, s) ||
      !P.scratch.alloc(&c->alloc, (size_t)plain_scratch_words(c, max_outs))) {
    set_error("device allocation failed (the sums of every output are held at once)");
    return SFHE_E_NOMEM;
  }
  if (launch == SFHE_PLAIN_FUSED) {
    P.launches = 1 + (tensor_fp_prime_count(c) > 0 && tensor_fp_prime_count(c) < nl);
  } else {
    // one launch per product: the weights of every product uploaded once
    std::vector<u64> pw, pws;
    for (int n = 0; n < count; ++n) {
      const sfhe_mat *W = Wm[n], *B = Bm[n];
      for (int i = 0; i < W->rows; ++i) {
        row_pairs(W, i, pairs);
        for (int j = 0; j < B->cols; ++j)
          for (auto& pr : pairs) {
            for (int l = 0; l < nl; ++l) {
              const u64 w = W->w_res[(size_t)pr.second * c->L + l];
              pw.push_back(w);
              pws.push_back(hostmath::shoup(w, c->primes[l]));
            }
            P.pb_slot.push_back((int64_t)pr.first * B->cols + j);
            P.pd.push_back(P.jobs[n].d0 + (int64_t)i * B->cols + j);
            P.pjob.push_back(n);
          }
      }
    }
    if (!upload(c, P.pw, pw, s) || !upload(c, P.pws, pws, s)) { set_error("device allocation failed"); return SFHE_E_NOMEM; }
    P.launches = (int64_t)P.pb_slot.size();
  }
  return SFHE_OK;
}

// the launches alone (nothing allocated, nothing copied): products, then one
// rescale per output in slices of kRescaleSlice outputs
static int plain_launch(sfhe_ctx* c, const PlainPrep& P, hipStream_t s) {
  const int N = c->N, lev = c->L - 1, nl = lev + 1;
  const int64_t dw = (int64_t)2 * nl * N;
  int rc = SFHE_OK;
  if (P.launch == SFHE_PLAIN_FUSED) {
    PlainBatch pb{P.d_jobs.ptr, P.desc.ptr, P.n_desc, nl, P.D.ptr};
    rc = launch_plain_batch(c, pb, s);
  } else {
    rc = launch_zero(P.D.ptr, std::max<int64_t>(P.outs, 1) * dw, s);
    for (size_t x = 0; x < P.pb_slot.size() && !rc; ++x) {
      const sfhe_mat* B = P.B[P.pjob[x]];
      rc = launch_plain_product(c, B->data.ptr, B->n_ct, P.pb_slot[x], P.pw.ptr + x * nl, P.pws.ptr + x * nl,
                                P.D.ptr + P.pd[x] * dw, nl, s);
    }
  }
  for (int n = 0; n < P.count && !rc; ++n) {
    const int64_t cnt = (int64_t)P.C[n]->n_ct;
    for (int64_t o0 = 0; o0 < cnt && !rc; o0 += kRescaleSlice) {
      const OutLayout ol{P.C[n]->data.ptr, 0, true, P.C[n]->n_ct, o0};
      const int64_t m = std::min<int64_t>(kRescaleSlice, cnt - o0);
      const u64* Ds = P.D.ptr + (P.jobs[n].d0 + o0) * dw;
      rc = c->logN == 14 ? rescale_n14(c, lev, Ds, dw, ol, m, s, P.scratch.ptr)
                         : rescale_batch(c, lev, Ds, dw, ol, m, s, P.scratch.ptr);
    }
  }
  return rc;
}

// Enqueue the plaintext-weight products of count (W, B) pairs on stream s.
// ev_start (nullable) is recorded after the set-up, before the first product
// launch.  On failure every C[n] is NULL.
static int plain_enqueue(sfhe_ctx* c, int32_t count, const sfhe_mat* const* Wm, const sfhe_mat* const* Bm,
                         sfhe_plain_launch launch, hipStream_t s, sfhe_mat** C, hipEvent_t ev_start,
                         int64_t* n_products, int64_t* n_launches, int64_t* n_outputs) {
  for (int n = 0; n < count; ++n) C[n] = nullptr;
  PlainPrep P;
  int rc = plain_prepare(c, count, Wm, Bm, launch, s, P);
  if (!rc && ev_start) {
    hipError_t e = hipEventRecord(ev_start, s);
    if (e != hipSuccess) { rc = SFHE_E_DEVICE; set_error(hipGetErrorString(e)); }
  }
  if (!rc) rc = plain_launch(c, P, s);
  if (rc) {
    (void)hipStreamSynchronize(s);
    return rc;   // P frees the partial results
  }
  *n_products = P.products;
  *n_launches = P.launches;
  *n_outputs = P.outs;
  P.release(C);
  return SFHE_OK;
}

// the synchronous-API form: timed by the context's event pair, stats recorded
static int plain_batch(sfhe_ctx* c, int32_t count, const sfhe_mat* const* Wm, const sfhe_mat* const* Bm,
                       sfhe_plain_launch launch, hipStream_t s, sfhe_mat** C) {
  int64_t products = 0, launches = 0, outs = 0;
  c->prof_used = 0;
  c->prof_cat.clear();
  int rc = plain_enqueue(c, count, Wm, Bm, launch, s, C, c->ev0, &products, &launches, &outs);
  if (rc) return rc;
  hipError_t e = hipEventRecord(c->ev1, s);
  if (e != hipSuccess) {
    set_error(hipGetErrorString(e));
    (void)hipStreamSynchronize(s);
    for (int n = 0; n < count; ++n) { delete C[n]; C[n] = nullptr; }
    return SFHE_E_DEVICE;
  }
  c->stats = sfhe_stats{};
  c->stats.products = products;
  c->stats.outputs = outs;
  c->stats.tensor_launches = launches;
  c->stats_pending = true;
  return SFHE_OK;
}

int sfhe_matmul_plain(sfhe_ctx* c, const sfhe_mat* W, const sfhe_mat* B, void* stream, sfhe_mat** C) {
  GUARD_BEGIN
  if (!C) { set_error("C is NULL"); return SFHE_E_INVALID_ARG; }
  *C = nullptr;
  if (!c || !W || !B) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  StreamScope scope_(c->alloc, (hipStream_t)stream);
  return plain_batch(c, 1, &W, &B, SFHE_PLAIN_FUSED, (hipStream_t)stream, C);
  GUARD_END
}

int sfhe_matmul_plain_batch(sfhe_ctx* c, int32_t count, const sfhe_mat* const* W, const sfhe_mat* const* B,
                            sfhe_plain_launch launch, void* stream, sfhe_mat** C) {
  GUARD_BEGIN
  if (!C) { set_error("C is NULL"); return SFHE_E_INVALID_ARG; }
  if (!c || !W || !B || count < 1) {
    if (count > 0) for (int n = 0; n < count; ++n) C[n] = nullptr;
    set_error("NULL argument or count < 1");
    return SFHE_E_INVALID_ARG;
  }
  StreamScope scope_(c->alloc, (hipStream_t)stream);
  return plain_batch(c, count, W, B, launch, (hipStream_t)stream, C);
  GUARD_END
}

// ---------------------------------------------------------------- graphs
}  // extern "C"

// a LAZY ct x ct product captured once into a HIP graph: its tile lists,
// lazy sums, key-switch scratch and result stay allocated, and every replay
// recomputes the result from the current contents of A and B
struct sfhe_matmul_graph {
  sfhe_ctx* c = nullptr;
  LazyPrep P;
  hipStream_t cs = nullptr;       // the capture stream (default priority)
  hipStream_t ls = nullptr;       // the stream of the last replay
  bool replayed = false;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  int64_t launches = 0;
  ~sfhe_matmul_graph() {
    // the buffers of P are given back after the last replay has ended
    if (replayed) (void)hipStreamSynchronize(ls);
    if (cs) (void)hipStreamSynchronize(cs);
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    if (cs) (void)hipStreamDestroy(cs);
  }
};

extern "C" {

int sfhe_matmul_graph_create(sfhe_ctx* c, const sfhe_mat* A, const sfhe_mat* B, void* stream,
                             sfhe_matmul_graph** out) {
  GUARD_BEGIN
  if (!out) { set_error("out is NULL"); return SFHE_E_INVALID_ARG; }
  *out = nullptr;
  int rc = matmul_check(c, A, B, SFHE_SCHED_LAZY);
  if (rc) return rc;
  if (A->slots > 1 || B->slots > 1) { set_error("several values per ciphertext: not a graph product"); return SFHE_E_UNSUPPORTED; }
  hipStream_t s = (hipStream_t)stream;
  StreamScope scope_(c->alloc, s);
  std::unique_ptr<sfhe_matmul_graph> G(new sfhe_matmul_graph());
  G->c = c;
  G->P.out = new_product(c, A, B);
  if (!G->P.out) return SFHE_E_NOMEM;
  rc = lazy_prepare(c, A, B, s, G->P);
  if (rc) return rc;
  SFHE_HIP(hipStreamSynchronize(s));
  SFHE_HIP(hipStreamCreate(&G->cs));
  // one run outside the capture: kernel attributes, the key-switch slice
  // (tuned here if the context has not tuned it yet) and its scratch
  int64_t tl = 0, fl = 0;
  rc = lazy_launch(c, G->P, G->cs, false, true, &tl, &fl);
  if (rc) return rc;
  SFHE_HIP(hipStreamSynchronize(G->cs));
  G->launches = tl;
  if (hipStreamBeginCapture(G->cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    set_error("stream capture failed");
    return SFHE_E_DEVICE;
  }
  rc = lazy_launch(c, G->P, G->cs, false, false, &tl, &fl);
  const hipError_t e = hipStreamEndCapture(G->cs, &G->g);
  if (rc) return rc;
  if (e != hipSuccess) { set_error(hipGetErrorString(e)); return SFHE_E_DEVICE; }
  if (hipGraphInstantiate(&G->ge, G->g, nullptr, nullptr, 0) != hipSuccess) {
    set_error("graph instantiation failed");
    return SFHE_E_DEVICE;
  }
  *out = G.release();
  return SFHE_OK;
  GUARD_END
}

int sfhe_matmul_graph_launch(sfhe_matmul_graph* G, void* stream) {
  GUARD_BEGIN
  if (!G) { set_error("NULL graph"); return SFHE_E_INVALID_ARG; }
  sfhe_ctx* c = G->c;
  hipStream_t s = (hipStream_t)stream;
  c->prof_used = 0;
  c->prof_cat.clear();
  SFHE_HIP(hipEventRecord(c->ev0, s));
  SFHE_HIP(hipGraphLaunch(G->ge, s));
  G->ls = s;
  G->replayed = true;
  SFHE_HIP(hipEventRecord(c->ev1, s));
  c->stats = sfhe_stats{};
  c->stats.products = G->P.products;
  c->stats.keyswitches = G->P.keyswitches;
  c->stats.outputs = G->P.out->n_ct;
  c->stats.tensor_launches = G->launches;
  c->stats.tensor_fp_primes = tensor_fp_prime_count(c);
  c->stats_pending = true;
  return SFHE_OK;
  GUARD_END
}

int sfhe_matmul_graph_result(const sfhe_matmul_graph* G, const sfhe_mat** out) {
  if (!G || !out) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  *out = G->P.out;
  return SFHE_OK;
}

void sfhe_matmul_graph_destroy(sfhe_matmul_graph* G) { delete G; }

}  // extern "C"

// a plaintext-weight batch captured once into a HIP graph: its tables, sums,
// scratch and results stay allocated, and every replay recomputes the results
// from the current contents of the B matrices
struct sfhe_plain_graph {
  sfhe_ctx* c = nullptr;
  PlainPrep P;
  hipStream_t cs = nullptr;       // the capture stream (default priority)
  hipStream_t ls = nullptr;       // the stream of the last replay
  bool replayed = false;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  ~sfhe_plain_graph() {
    // the buffers below are given back after the last replay has ended
    if (replayed) (void)hipStreamSynchronize(ls);
    if (cs) (void)hipStreamSynchronize(cs);
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    if (cs) (void)hipStreamDestroy(cs);
  }
};

extern "C" {

int sfhe_plain_graph_create(sfhe_ctx* c, int32_t count, const sfhe_mat* const* W, const sfhe_mat* const* B,
                            sfhe_plain_launch launch, void* stream, sfhe_plain_graph** out) {
  GUARD_BEGIN
  if (!out) { set_error("out is NULL"); return SFHE_E_INVALID_ARG; }
  *out = nullptr;
  if (!c || !W || !B || count < 1) { set_error("NULL argument or count < 1"); return SFHE_E_INVALID_ARG; }
  hipStream_t s = (hipStream_t)stream;
  StreamScope scope_(c->alloc, s);
  sfhe_plain_graph* G = new sfhe_plain_graph();
  G->c = c;
  int rc = plain_prepare(c, count, W, B, launch, s, G->P);
  if (!rc && hipStreamSynchronize(s) != hipSuccess) { set_error("stream synchronize failed"); rc = SFHE_E_DEVICE; }
  if (!rc && hipStreamCreate(&G->cs) != hipSuccess) { set_error("stream creation failed"); rc = SFHE_E_DEVICE; }
  // one run outside the capture (sets the kernels' attributes), then the capture
  if (!rc) rc = plain_launch(c, G->P, G->cs);
  if (!rc && hipStreamSynchronize(G->cs) != hipSuccess) { set_error("stream synchronize failed"); rc = SFHE_E_DEVICE; }
  if (!rc && hipStreamBeginCapture(G->cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    set_error("stream capture failed");
    rc = SFHE_E_DEVICE;
  }
  if (!rc) {
    const int lrc = plain_launch(c, G->P, G->cs);
    const hipError_t e = hipStreamEndCapture(G->cs, &G->g);
    if (lrc) rc = lrc;
    else if (e != hipSuccess) { set_error(hipGetErrorString(e)); rc = SFHE_E_DEVICE; }
  }
  if (!rc && hipGraphInstantiate(&G->ge, G->g, nullptr, nullptr, 0) != hipSuccess) {
    set_error("graph instantiation failed");
    rc = SFHE_E_DEVICE;
  }
  if (rc) { delete G; return rc; }
  *out = G;
  return SFHE_OK;
  GUARD_END
}

int sfhe_plain_graph_launch(sfhe_plain_graph* G, void* stream) {
  GUARD_BEGIN
  if (!G) { set_error("NULL graph"); return SFHE_E_INVALID_ARG; }
  sfhe_ctx* c = G->c;
  hipStream_t s = (hipStream_t)stream;
  StreamScope scope_(c->alloc, s);
  c->prof_used = 0;
  c->prof_cat.clear();
  SFHE_HIP(hipEventRecord(c->ev0, s));
  SFHE_HIP(hipGraphLaunch(G->ge, s));
  G->ls = s;
  G->replayed = true;
  SFHE_HIP(hipEventRecord(c->ev1, s));
  c->stats = sfhe_stats{};
  c->stats.products = G->P.products;
  c->stats.outputs = G->P.outs;
  c->stats.tensor_launches = G->P.launches;
  c->stats_pending = true;
  return SFHE_OK;
  GUARD_END
}

int sfhe_plain_graph_result(const sfhe_plain_graph* G, int32_t n, const sfhe_mat** out) {
  if (!G || !out) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  if (n < 0 || n >= G->P.count) { set_error("result index out of range"); return SFHE_E_INVALID_ARG; }
  *out = G->P.C[n];
  return SFHE_OK;
}

void sfhe_plain_graph_destroy(sfhe_plain_graph* G) { delete G; }

// ---------------------------------------------------------------- serving
}  // extern "C"

// A request loop over plaintext-weight products: requests queue in arrival
// order; each step first retires the batches whose end event has passed,
// then admits queued requests while the device bytes they hold until they
// complete (sums, results, rescale scratch, tables) fit the budget, and
// enqueues them as one fused batch on the server stream (at most
// kServerStreams, the hardware queues of a process) with the fewest running
// batches.  With one stream, batches run in admission order; with several,
// a batch admitted while others run starts at once on its own stream and
// overlaps them on the device.  With a slot limit, a stream holding that
// many running batches takes no more, and while every stream is full,
// arriving requests wait on the host and join the next batch.  A batch's
// launches first wait for the work the caller enqueued on the client stream
// before the step (the requests' encryptions).
constexpr int kServerStreams = 4;

struct sfhe_server {
  sfhe_ctx* c = nullptr;
  hipStream_t client = nullptr;           // the caller's stream (inputs are ready in its order)
  std::vector<hipStream_t> streams;       // the server's own, default priority
  std::vector<int> busy;                  // running batches per stream
  int slots = 0;                          // running batches a stream may hold (0: no limit)
  uint64_t batch_cap = 0;                 // bytes one batch may hold (0: no limit)
  hipEvent_t epoch = nullptr;             // device-time origin of the batch intervals
  uint64_t budget = 0, in_flight = 0;
  struct Req {
    int64_t ticket;
    const sfhe_mat *W, *X;
    uint64_t bytes;
  };
  struct Run {
    std::vector<int64_t> tickets;
    std::vector<sfhe_mat*> C;
    std::unique_ptr<PlainPrep> prep;      // the batch's sums, scratch and tables, freed at retirement
    hipEvent_t start = nullptr, end = nullptr;
    uint64_t bytes = 0;
    int64_t products = 0;
    int stream = 0;
  };
  struct Done {
    sfhe_mat* C;
    double ms;          // device time of the request's batch
    double t0, t1;      // its start and end, ms after the server's epoch
    int32_t batch_size;
  };
  std::deque<Req> queue;
  std::deque<Run> running;                // in launch order
  std::map<int64_t, Done> done;
  int64_t next_ticket = 0, batches = 0, products = 0, overlapped = 0;
  double last_end = -1.0;
  // move the batches whose end event has passed to `done` (any order); wait
  // for them all if `all`
  int retire(bool all) {
    for (auto it = running.begin(); it != running.end();) {
      Run& r = *it;
      hipError_t e = all ? hipEventSynchronize(r.end) : hipEventQuery(r.end);
      if (e == hipErrorNotReady) { ++it; continue; }
      if (e != hipSuccess) { set_error(hipGetErrorString(e)); return SFHE_E_DEVICE; }
      float ms = 0, t0 = 0, t1 = 0;
      (void)hipEventElapsedTime(&ms, r.start, r.end);
      (void)hipEventElapsedTime(&t0, epoch, r.start);
      (void)hipEventElapsedTime(&t1, epoch, r.end);
      for (size_t x = 0; x < r.tickets.size(); ++x)
        done[r.tickets[x]] = Done{r.C[x], ms, t0, t1, (int32_t)r.tickets.size()};
      in_flight -= r.bytes;
      products += r.products;
      --busy[r.stream];
      r.prep.reset();   // the batch has ended: its blocks go back in the client stream's order
      (void)hipEventDestroy(r.start);
      (void)hipEventDestroy(r.end);
      it = running.erase(it);
    }
    return SFHE_OK;
  }
  ~sfhe_server() {
    (void)retire(true);
    for (auto& d : done) delete d.second.C;
    for (hipStream_t st : streams) (void)hipStreamDestroy(st);
    if (epoch) (void)hipEventDestroy(epoch);
  }
};

extern "C" {

int sfhe_server_create(sfhe_ctx* c, uint64_t budget_bytes, int32_t n_streams, void* stream, sfhe_server** out) {
  GUARD_BEGIN
  if (!out) { set_error("out is NULL"); return SFHE_E_INVALID_ARG; }
  *out = nullptr;
  if (!c || budget_bytes == 0) { set_error("NULL context or zero budget"); return SFHE_E_INVALID_ARG; }
  if (n_streams < 1 || n_streams > kServerStreams) { set_error("n_streams must be in [1, 4]"); return SFHE_E_INVALID_ARG; }
  std::unique_ptr<sfhe_server> v(new sfhe_server());
  v->c = c;
  v->client = (hipStream_t)stream;
  v->budget = budget_bytes;
  for (int x = 0; x < n_streams; ++x) {
    hipStream_t st = nullptr;
    SFHE_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    v->streams.push_back(st);
    v->busy.push_back(0);
  }
  SFHE_HIP(hipEventCreate(&v->epoch));
  SFHE_HIP(hipEventRecord(v->epoch, v->streams[0]));
  SFHE_HIP(hipEventSynchronize(v->epoch));
  *out = v.release();
  return SFHE_OK;
  GUARD_END
}

int sfhe_server_request_bytes(const sfhe_ctx* c, const sfhe_mat* W, const sfhe_mat* X, uint64_t* bytes) {
  GUARD_BEGIN
  if (!c || !bytes) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  const int rc = plain_check(c, W, X);
  if (rc) return rc;
  *bytes = plain_bytes(c, W, X);
  return SFHE_OK;
  GUARD_END
}

int sfhe_server_submit(sfhe_server* v, const sfhe_mat* W, const sfhe_mat* X, int64_t* ticket) {
  GUARD_BEGIN
  if (!v || !ticket) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  const int rc = plain_check(v->c, W, X);
  if (rc) return rc;
  const uint64_t bytes = plain_bytes(v->c, W, X);
  if (bytes > v->budget) { set_error("request larger than the server's memory budget"); return SFHE_E_NOMEM; }
  *ticket = v->next_ticket++;
  v->queue.push_back(sfhe_server::Req{*ticket, W, X, bytes});
  return SFHE_OK;
  GUARD_END
}

int sfhe_server_step(sfhe_server* v, int32_t* admitted) {
  GUARD_BEGIN
  if (!v || !admitted) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  *admitted = 0;
  int rc = v->retire(false);
  if (rc) return rc;
  // the stream with the fewest running batches; at the slot limit the
  // requests wait and join the next batch
  int sx = 0;
  for (int x = 1; x < (int)v->streams.size(); ++x)
    if (v->busy[x] < v->busy[sx]) sx = x;
  if (v->slots > 0 && v->busy[sx] >= v->slots) return SFHE_OK;
  std::vector<const sfhe_mat*> Ws, Xs;
  sfhe_server::Run run;
  // requests join the batch in order while they fit the budget beside the
  // running batches and, with a cap, the batch's own limit (a request larger
  // than the cap forms a batch of its own)
  while (!v->queue.empty() && v->in_flight + run.bytes + v->queue.front().bytes <= v->budget &&
         (v->batch_cap == 0 || run.bytes == 0 || run.bytes + v->queue.front().bytes <= v->batch_cap)) {
    const sfhe_server::Req& q = v->queue.front();
    Ws.push_back(q.W);
    Xs.push_back(q.X);
    run.tickets.push_back(q.ticket);
    run.bytes += q.bytes;
    v->queue.pop_front();
  }
  if (Ws.empty()) return SFHE_OK;
  run.stream = sx;
  hipStream_t bs = v->streams[sx];
  run.C.assign(Ws.size(), nullptr);
  hipEvent_t ready = nullptr;
  if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess || hipEventCreate(&run.start) != hipSuccess ||
      hipEventCreate(&run.end) != hipSuccess) {
    set_error("event creation failed");
    rc = SFHE_E_DEVICE;
  }
  // Every block of the batch is taken in the client stream's order, and the
  // batch's own stream waits for the client stream after that, so blocks that
  // the client's earlier work used are safe to reuse.  The results pass to the
  // caller; the other blocks are given back at retirement, when the batch has
  // ended.  With several server streams all of them thus draw on one stream's
  // cached blocks.
  run.prep.reset(new PlainPrep());
  if (!rc) {
    StreamScope scope_(v->c->alloc, v->client);
    rc = plain_prepare(v->c, (int32_t)Ws.size(), Ws.data(), Xs.data(), SFHE_PLAIN_FUSED, v->client, *run.prep);
  }
  if (!rc && (hipEventRecord(ready, v->client) != hipSuccess || hipStreamWaitEvent(bs, ready, 0) != hipSuccess ||
              hipEventRecord(run.start, bs) != hipSuccess)) {
    set_error("stream ordering failed");
    rc = SFHE_E_DEVICE;
  }
  if (!rc) {
    StreamScope scope_(v->c->alloc, bs);
    rc = plain_launch(v->c, *run.prep, bs);
  }
  if (!rc && hipEventRecord(run.end, bs) != hipSuccess) { set_error("event record failed"); rc = SFHE_E_DEVICE; }
  if (ready) (void)hipEventDestroy(ready);
  if (!rc) {
    run.products = run.prep->products;
    run.prep->release(run.C.data());
  }
  if (rc) {
    (void)hipStreamSynchronize(bs);
    run.prep.reset();
    // the requests stay queued, in order, for a later step
    for (size_t x = Ws.size(); x-- > 0;) v->queue.push_front(sfhe_server::Req{run.tickets[x], Ws[x], Xs[x], plain_bytes(v->c, Ws[x], Xs[x])});
    for (auto* m : run.C) delete m;
    if (run.start) (void)hipEventDestroy(run.start);
    if (run.end) (void)hipEventDestroy(run.end);
    return rc;
  }
  v->in_flight += run.bytes;
  ++v->busy[sx];
  ++v->batches;
  *admitted = (int32_t)Ws.size();
  v->running.push_back(std::move(run));
  return SFHE_OK;
  GUARD_END
}

int sfhe_server_poll(sfhe_server* v, int64_t ticket, int32_t wait, int32_t* is_done, sfhe_mat** C, double* batch_ms,
                     int32_t* batch_size, double* start_ms, double* end_ms) {
  GUARD_BEGIN
  if (!v || !is_done || !C) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  *is_done = 0;
  *C = nullptr;
  if (ticket < 0 || ticket >= v->next_ticket) { set_error("unknown ticket"); return SFHE_E_INVALID_ARG; }
  int rc = v->retire(false);
  if (rc) return rc;
  auto it = v->done.find(ticket);
  if (it == v->done.end() && wait) {
    // wait for the batch that holds the ticket
    for (auto& r : v->running)
      if (std::find(r.tickets.begin(), r.tickets.end(), ticket) != r.tickets.end()) {
        SFHE_HIP(hipEventSynchronize(r.end));
        break;
      }
    rc = v->retire(false);
    if (rc) return rc;
    it = v->done.find(ticket);
  }
  if (it == v->done.end()) return SFHE_OK;
  *is_done = 1;
  // the result is the caller's from here on: its memory was taken, and goes
  // back when the caller frees it, in the client stream's order (the batch
  // has ended; the server's streams may be gone by then)
  *C = it->second.C;
  if (batch_ms) *batch_ms = it->second.ms;
  if (batch_size) *batch_size = it->second.batch_size;
  if (start_ms) *start_ms = it->second.t0;
  if (end_ms) *end_ms = it->second.t1;
  v->done.erase(it);
  return SFHE_OK;
  GUARD_END
}

int sfhe_server_set_slots(sfhe_server* v, int32_t per_stream) {
  GUARD_BEGIN
  if (!v || per_stream < 0) { set_error("NULL server or negative slot limit"); return SFHE_E_INVALID_ARG; }
  v->slots = per_stream;
  return SFHE_OK;
  GUARD_END
}

int sfhe_server_set_batch_bytes(sfhe_server* v, uint64_t max_bytes) {
  GUARD_BEGIN
  if (!v) { set_error("NULL server"); return SFHE_E_INVALID_ARG; }
  v->batch_cap = max_bytes;
  return SFHE_OK;
  GUARD_END
}

int sfhe_server_status(const sfhe_server* v, int64_t* queued, int64_t* running, uint64_t* bytes_in_flight,
                       int64_t* batches, int64_t* products) {
  if (!v) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  if (queued) *queued = (int64_t)v->queue.size();
  if (running) *running = (int64_t)v->running.size();
  if (bytes_in_flight) *bytes_in_flight = v->in_flight;
  if (batches) *batches = v->batches;
  if (products) *products = v->products;
  return SFHE_OK;
}

void sfhe_server_destroy(sfhe_server* v) { delete v; }

int sfhe_last_stats(const sfhe_ctx* cc, sfhe_stats* out) {
  if (!cc || !out) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  sfhe_ctx* c = const_cast<sfhe_ctx*>(cc);
  if (c->stats_pending) {
    SFHE_HIP(hipEventSynchronize(c->ev1));
    float ms = 0;
    SFHE_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->stats.ms = ms;
    double cat[4] = {0, 0, 0, 0};
    for (size_t x = 0; x < c->prof_cat.size(); ++x) {
      float e = 0;
      SFHE_HIP(hipEventElapsedTime(&e, c->prof_pool[2 * x], c->prof_pool[2 * x + 1]));
      cat[c->prof_cat[x]] += e;
    }
    c->stats.tensor_ms = cat[kCatTensor];
    c->stats.keyswitch_ms = cat[kCatKeyswitch];
    c->stats.rescale_ms = cat[kCatRescale];
    c->stats.tensor_fp_ms = cat[kCatTensorFp];
    c->stats_pending = false;
  }
  *out = c->stats;
  return SFHE_OK;
}

int sfhe_decrypt_matrix(sfhe_ctx* c, const sfhe_mat* m, double* out, int64_t ld, void* stream) {
  GUARD_BEGIN
  if (!c || !m || !out) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  if (m->ctx != c) { set_error("matrix belongs to another context"); return SFHE_E_INVALID_ARG; }
  if (m->plain) { set_error("plaintext weights hold no ciphertexts"); return SFHE_E_UNSUPPORTED; }
  if (!c->has_keys) { set_error("keygen first"); return SFHE_E_STATE; }
  if (ld < m->cols) { set_error("ld < cols"); return SFHE_E_SHAPE; }
  hipStream_t s = (hipStream_t)stream;
  StreamScope scope_(c->alloc, s);
  const int64_t nv = m->slots > 1 ? m->n_vals : m->n_ct;   // stored values
  std::vector<double> vals(nv > 0 ? nv : 1, 0.0);
  if (m->slots > 1) {
    int rc = slot_table(c);
    if (rc) return rc;
  }
  if (nv > 0) {
    DevBuf<double> d_v;
    DevBuf<int> d_flag;
    if (!d_v.alloc(&c->alloc, nv) || !d_flag.alloc(&c->alloc, 1)) { set_error("device allocation failed"); return SFHE_E_NOMEM; }
    SFHE_HIP(hipMemsetAsync(d_flag.ptr, 0, sizeof(int), s));
    int rc = decrypt_values(c, m->data.ptr, m->n_ct, m->level, m->scale, d_v.ptr, d_flag.ptr, s, m->slots, nv);
    if (rc) return rc;
    int flag = 0;
    SFHE_HIP(hipMemcpyAsync(vals.data(), d_v.ptr, nv * sizeof(double), hipMemcpyDeviceToHost, s));
    SFHE_HIP(hipMemcpyAsync(&flag, d_flag.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
    SFHE_HIP(hipStreamSynchronize(s));
    if (flag) { set_error("a decrypted coefficient is outside the decodable range"); return SFHE_E_DECRYPT; }
  }
  for (int i = 0; i < m->rows; ++i)
    for (int j = 0; j < m->cols; ++j) out[(int64_t)i * ld + j] = 0.0;
  switch (m->enc) {
    case SFHE_ENC_DENSE:
    case SFHE_ENC_NAIVE_SPARSE:
      for (int i = 0; i < m->rows; ++i)
        for (int j = 0; j < m->cols; ++j) out[(int64_t)i * ld + j] = vals[(int64_t)i * m->cols + j];
      break;
    case SFHE_ENC_CSR:
      for (int i = 0; i < m->rows; ++i)
        for (int p = m->row_ptr[i]; p < m->row_ptr[i + 1]; ++p) out[(int64_t)i * ld + m->col_idx[p]] = vals[p];
      break;
    case SFHE_ENC_ELL:
      for (int i = 0; i < m->rows; ++i)
        for (int sl = 0; sl < m->ell_w; ++sl) {
          const int k = m->ell_col[(size_t)i * m->ell_w + sl];
          if (k >= 0) out[(int64_t)i * ld + k] = vals[(int64_t)i * m->ell_w + sl];
        }
      break;
  }
  return SFHE_OK;
  GUARD_END
}

int sfhe_export_ct(sfhe_ctx* c, const sfhe_mat* m, int32_t i, int32_t j, uint64_t* out, size_t cap, void* stream) {
  GUARD_BEGIN
  if (!c || !m || !out) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  if (m->plain) { set_error("plaintext weights hold no ciphertexts"); return SFHE_E_UNSUPPORTED; }
  if (m->slots > 1) { set_error("several values per ciphertext: use sfhe_export_stored"); return SFHE_E_UNSUPPORTED; }
  if (i < 0 || i >= m->rows || j < 0 || j >= m->cols) { set_error("index out of range"); return SFHE_E_SHAPE; }
  const int N = c->N, nl = m->level + 1;
  const size_t words = (size_t)2 * nl * N;
  if (cap < words) { set_error("capacity below 2*(level+1)*N"); return SFHE_E_INVALID_ARG; }
  const int64_t sl = slot_of(m, i, j);
  if (sl < 0) { set_error("element not stored by this encoding"); return SFHE_E_SHAPE; }
  hipStream_t s = (hipStream_t)stream;
  StreamScope scope_(c->alloc, s);
  DevBuf<u64> tmp;
  if (!tmp.alloc(&c->alloc, words)) { set_error("device allocation failed"); return SFHE_E_NOMEM; }
  int rc = launch_from_chunked(c, m->data.ptr, m->n_ct, nl, 1, nullptr, sl, tmp.ptr, (int64_t)words, s);
  if (rc) return rc;
  int pos[2 * kMaxBasis], pr[2 * kMaxBasis];
  for (int r = 0; r < 2 * nl; ++r) { pos[r] = r; pr[r] = r % nl; }
  rc = launch_ntt(c, tmp.ptr, 1, 0, 2 * nl, pos, pr, true, s);
  if (rc) return rc;
  SFHE_HIP(hipMemcpyAsync(out, tmp.ptr, words * sizeof(u64), hipMemcpyDeviceToHost, s));
  SFHE_HIP(hipStreamSynchronize(s));
  return SFHE_OK;
  GUARD_END
}

// ---------------------------------------------------------------- primitives
int sfhe_ntt(sfhe_ctx* c, uint64_t* data, int32_t batch, int32_t n_limbs, int32_t first_prime, int32_t inverse,
             void* stream) {
  GUARD_BEGIN
  if (!c || !data) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  if (batch < 0 || n_limbs < 1 || first_prime < 0 || first_prime + n_limbs > c->nb) {
    set_error("limb range outside the basis");
    return SFHE_E_INVALID_ARG;
  }
  int pos[2 * kMaxBasis], pr[2 * kMaxBasis];
  for (int r = 0; r < n_limbs; ++r) { pos[r] = r; pr[r] = first_prime + r; }
  return launch_ntt(c, data, batch, (int64_t)n_limbs * c->N, n_limbs, pos, pr, inverse != 0, (hipStream_t)stream);
  GUARD_END
}

int sfhe_tensor(sfhe_ctx* c, int32_t level, const uint64_t* a, const uint64_t* b, uint64_t* d, int32_t batch,
                void* stream) {
  GUARD_BEGIN
  if (!c || !a || !b || !d) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  if (level < 0 || level >= c->L || batch < 0) { set_error("bad level or batch"); return SFHE_E_LEVEL; }
  const int64_t nl = level + 1, N = c->N;
  return launch_tensor_pointwise(c, level, a, 2 * nl * N, b, 2 * nl * N, d, 3 * nl * N, batch, (hipStream_t)stream);
  GUARD_END
}

int sfhe_keyswitch(sfhe_ctx* c, int32_t level, const uint64_t* d2, uint64_t* out, int32_t batch, void* stream) {
  GUARD_BEGIN
  if (!c || !d2 || !out) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  if (!c->has_keys) { set_error("keygen first"); return SFHE_E_STATE; }
  if (level < 0 || level >= c->L || batch < 0) { set_error("bad level or batch"); return SFHE_E_LEVEL; }
  const int64_t nl = level + 1, N = c->N;
  StreamScope scope_(c->alloc, (hipStream_t)stream);
  return keyswitch_batch(c, level, d2, nl * N, out, 2 * nl * N, false, batch, (hipStream_t)stream);
  GUARD_END
}

int sfhe_rescale(sfhe_ctx* c, int32_t level, const uint64_t* in, uint64_t* out, int32_t batch, void* stream) {
  GUARD_BEGIN
  if (!c || !in || !out) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  if (level < 1 || level >= c->L || batch < 0) { set_error("bad level or batch"); return SFHE_E_LEVEL; }
  const int64_t nl = level + 1, N = c->N;
  StreamScope scope_(c->alloc, (hipStream_t)stream);
  return rescale_batch(c, level, in, 2 * nl * N, OutLayout{out, 2 * level * N, false, 0, 0}, batch, (hipStream_t)stream);
  GUARD_END
}


// ---------------------------------------------------------------- several values per ciphertext
int sfhe_encrypt_matrix_slots(sfhe_ctx* c, const double* vals, int32_t rows, int32_t cols, int64_t ld,
                              sfhe_encoding enc, int32_t slots, uint64_t seed, uint32_t operand_id, void* stream,
                              sfhe_mat** out) {
  GUARD_BEGIN
  if (!out) { set_error("out is NULL"); return SFHE_E_INVALID_ARG; }
  *out = nullptr;
  if (!c || !vals) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  if (!c->has_keys) { set_error("keygen first"); return SFHE_E_STATE; }
  if (rows < 1 || cols < 1 || ld < cols) { set_error("bad shape or leading dimension"); return SFHE_E_SHAPE; }
  if ((int)enc < 0 || (int)enc > 3) { set_error("bad encoding"); return SFHE_E_INVALID_ARG; }
  if (slots < 1 || slots > 64 || slots > c->N / 2) { set_error("slots must be in [1, min(64, N/2)]"); return SFHE_E_INVALID_ARG; }
  hipStream_t s = (hipStream_t)stream;
  StreamScope scope_(c->alloc, s);
  sfhe_mat* m = new sfhe_mat();
  m->ctx = c;
  m->rows = rows;
  m->cols = cols;
  m->level = c->L - 1;
  m->scale = ldexp(1.0, (int)c->log2_scale);
  m->enc = enc;
  m->slots = slots;
  std::vector<std::pair<int64_t, double>> stored;
  build_structure(m, vals, ld, [&](int i, int j, int64_t sl) { stored.push_back({sl, vals[(int64_t)i * ld + j]}); });
  const int64_t nv = m->n_ct;   // stored values (ELL padding included, as zeros)
  std::vector<double> v((size_t)std::max<int64_t>(nv, 1), 0.0);
  for (auto& st : stored) v[st.first] = st.second;
  m->n_vals = nv;
  m->n_ct = (nv + slots - 1) / slots;
  // every scaled value of a chunk of cnt values must stay below 4e18 / cnt
  const double pow2 = ldexp(1.0, (int)c->log2_scale + 1 - c->logN);
  for (int64_t x = 0; x < nv; ++x) {
    const int64_t cnt = std::min<int64_t>(slots, nv - x / slots * slots);
    if (!(fabs(v[x] * pow2) < 4.0e18 / (double)cnt)) {
      delete m;
      set_error("value not finite or too large to encode");
      return SFHE_E_INVALID_ARG;
    }
  }
  const int N = c->N, L = c->L;
  int rc = SFHE_OK;
  const size_t words = (size_t)m->n_ct * 2 * L * N;
  if (!m->data.alloc(&c->alloc, words)) { delete m; set_error("device allocation failed for the ciphertexts"); return SFHE_E_NOMEM; }
  DevBuf<double> d_v;
  DevBuf<u64> tmp;
  const int64_t chunk = std::min<int64_t>(std::max<int64_t>(m->n_ct, 1), 1024);
  if (!upload(c, d_v, v, s) || !tmp.alloc(&c->alloc, (size_t)chunk * 2 * L * N)) {
    rc = SFHE_E_NOMEM;
    set_error("device allocation failed");
  }
  for (int64_t x0 = 0; x0 < m->n_ct && !rc; x0 += chunk) {
    const int64_t n = std::min(chunk, m->n_ct - x0);
    rc = encrypt_slots(c, tmp.ptr, n, x0, d_v.ptr, nv, slots, seed, operand_id, s);
    if (!rc) rc = launch_to_chunked(c, tmp.ptr, (int64_t)2 * L * N, L, n, m->data.ptr, m->n_ct, nullptr, x0, s);
  }
  if (!rc && hipStreamSynchronize(s) != hipSuccess) { rc = SFHE_E_DEVICE; set_error("stream synchronize failed"); }
  if (rc) { delete m; return rc; }
  *out = m;
  return SFHE_OK;
  GUARD_END
}

int sfhe_rotate(sfhe_ctx* c, int32_t level, const uint64_t* in, uint64_t* out, int32_t batch, int32_t r,
                void* stream) {
  GUARD_BEGIN
  if (!c || !in || !out) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  if (!c->has_keys) { set_error("keygen first"); return SFHE_E_STATE; }
  if (level < 0 || level >= c->L || batch < 0) { set_error("bad level or batch"); return SFHE_E_LEVEL; }
  if (in == out) { set_error("in and out must not overlap"); return SFHE_E_INVALID_ARG; }
  int rc = prepare_rotations(c, {(int64_t)r});
  if (rc) return rc;
  const int64_t w = (int64_t)2 * (level + 1) * c->N;
  StreamScope scope_(c->alloc, (hipStream_t)stream);
  return rotate_batch(c, level, in, w, r, out, w, batch, (hipStream_t)stream);
  GUARD_END
}

int sfhe_export_stored(sfhe_ctx* c, const sfhe_mat* m, int64_t n, uint64_t* out, size_t cap, void* stream) {
  GUARD_BEGIN
  if (!c || !m || !out) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  if (m->plain) { set_error("plaintext weights hold no ciphertexts"); return SFHE_E_UNSUPPORTED; }
  if (n < 0 || n >= m->n_ct) { set_error("ciphertext index out of range"); return SFHE_E_SHAPE; }
  const int N = c->N, nl = m->level + 1;
  const size_t words = (size_t)2 * nl * N;
  if (cap < words) { set_error("capacity below 2*(level+1)*N"); return SFHE_E_INVALID_ARG; }
  hipStream_t s = (hipStream_t)stream;
  StreamScope scope_(c->alloc, s);
  DevBuf<u64> tmp;
  if (!tmp.alloc(&c->alloc, words)) { set_error("device allocation failed"); return SFHE_E_NOMEM; }
  int rc = launch_from_chunked(c, m->data.ptr, m->n_ct, nl, 1, nullptr, n, tmp.ptr, (int64_t)words, s);
  if (rc) return rc;
  int pos[2 * kMaxBasis], pr[2 * kMaxBasis];
  for (int r = 0; r < 2 * nl; ++r) { pos[r] = r; pr[r] = r % nl; }
  rc = launch_ntt(c, tmp.ptr, 1, 0, 2 * nl, pos, pr, true, s);
  if (rc) return rc;
  SFHE_HIP(hipMemcpyAsync(out, tmp.ptr, words * sizeof(u64), hipMemcpyDeviceToHost, s));
  SFHE_HIP(hipStreamSynchronize(s));
  return SFHE_OK;
  GUARD_END
}

}  // extern "C"

// Stored values `list` of the chunked matrix src, each rotated from its slot
// v mod slots into slot 0, become the one-value ciphertexts dst[v] (top level).
static int unpack_values(sfhe_ctx* c, const sfhe_mat* src, const std::vector<int64_t>& list, sfhe_mat* dst,
                         hipStream_t s, int64_t& rotations) {
  const int N = c->N, lev = src->level, nl = lev + 1, cs = src->slots;
  const int64_t w = (int64_t)2 * nl * N, slice = 256;
  std::vector<std::vector<int64_t>> by_off(cs);
  for (int64_t v : list) by_off[v % cs].push_back(v);
  DevBuf<u64> a, b;
  DevBuf<int64_t> d_src, d_dst;
  const int64_t cap = std::min<int64_t>(slice, std::max<int64_t>((int64_t)list.size(), 1));
  if (!a.alloc(&c->alloc, (size_t)cap * w) || !b.alloc(&c->alloc, (size_t)cap * w)) {
    set_error("device allocation failed");
    return SFHE_E_NOMEM;
  }
  for (int o = 0; o < cs; ++o) {
    const std::vector<int64_t>& vs = by_off[o];
    for (size_t x0 = 0; x0 < vs.size(); x0 += slice) {
      const int64_t n = std::min<int64_t>(slice, (int64_t)(vs.size() - x0));
      std::vector<int64_t> es(vs.begin() + x0, vs.begin() + x0 + n), ed(es);
      for (auto& e : es) e /= cs;
      if (!upload(c, d_src, es, s) || !upload(c, d_dst, ed, s)) { set_error("device allocation failed"); return SFHE_E_NOMEM; }
      int rc = SFHE_OK;
      const u64* res = a.ptr;
      if (o && keyswitch_rescale_n14_supported(c)) {   // the rotation reads the chunks in place
        rc = rotate_chunked(c, lev, src->data.ptr, src->n_ct, d_src.ptr, o, b.ptr, w, n, s);
        res = b.ptr;
        rotations += n;
      } else {
        rc = launch_from_chunked(c, src->data.ptr, src->n_ct, nl, n, d_src.ptr, 0, a.ptr, w, s);
        if (!rc && o) {
          rc = rotate_batch(c, lev, a.ptr, w, o, b.ptr, w, n, s);
          res = b.ptr;
          rotations += n;
        }
      }
      if (!rc) rc = launch_to_chunked(c, res, w, nl, n, dst->data.ptr, dst->n_ct, d_dst.ptr, 0, s);
      if (rc) return rc;
    }
  }
  return SFHE_OK;
}

// The end of Algorithm 1 for n relinearised, rescaled products or sums x[b]
// (rows [2][lev+1][N], level lev, stride lev-wide ciphertexts), all bound for
// slot roff of their output chunk: multiply by the slot-zero mask, rescale,
// rotate from slot 0 to slot roff and add into the output chunks; segment o
// (items seg[o] .. seg[o+1]-1) goes to chunk oidx[o] of out.
static int finish_products(sfhe_ctx* c, int lev, u64* x, int64_t n, int roff, const std::vector<int>& seg,
                           const std::vector<int64_t>& oidx, sfhe_mat* out, hipStream_t s, int64_t& rotations) {
  const int N = c->N, nl = lev + 1;
  const int64_t wx = (int64_t)2 * nl * N, wy = (int64_t)2 * lev * N;
  int rc = mask_batch(c, lev, x, wx, n, s);
  DevBuf<u64> y, z;
  DevBuf<int> d_seg;
  DevBuf<int64_t> d_o;
  if (!rc && (!y.alloc(&c->alloc, (size_t)n * wy) || (roff && !z.alloc(&c->alloc, (size_t)n * wy)) ||
              !upload(c, d_seg, seg, s) || !upload(c, d_o, oidx, s))) {
    set_error("device allocation failed");
    rc = SFHE_E_NOMEM;
  }
  const OutLayout oy{y.ptr, wy, false, 0, 0};
  if (!rc) rc = c->logN == 14 ? rescale_n14(c, lev, x, wx, oy, n, s) : rescale_batch(c, lev, x, wx, oy, n, s);
  const u64* res = y.ptr;
  if (!rc && roff) {
    rc = rotate_batch(c, lev - 1, y.ptr, wy, -(int64_t)roff, z.ptr, wy, n, s);
    res = z.ptr;
    rotations += n;
  }
  if (!rc) rc = launch_segment_sum(c, lev, res, out->data.ptr, out->n_ct, d_seg.ptr, d_o.ptr, (int64_t)oidx.size(), s);
  return rc;
}

extern "C" {

int sfhe_matmul_slots(sfhe_ctx* c, const sfhe_mat* A, const sfhe_mat* B, sfhe_schedule sched, void* stream,
                      sfhe_mat** C) {
  GUARD_BEGIN
  if (!C) { set_error("C is NULL"); return SFHE_E_INVALID_ARG; }
  *C = nullptr;
  if (!c || !A || !B) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
  if (A->ctx != c || B->ctx != c) { set_error("matrices belong to another context"); return SFHE_E_INVALID_ARG; }
  if (A->plain || B->plain) { set_error("plaintext weights: use sfhe_matmul_plain"); return SFHE_E_UNSUPPORTED; }
  if (sched != SFHE_SCHED_PER_PRODUCT && sched != SFHE_SCHED_LAZY) { set_error("bad schedule"); return SFHE_E_INVALID_ARG; }
  if (!c->has_keys) { set_error("keygen first"); return SFHE_E_STATE; }
  if (A->slots != B->slots) { set_error("operands hold different numbers of values per ciphertext"); return SFHE_E_SHAPE; }
  if (B->enc != SFHE_ENC_DENSE) { set_error("the right operand must be DENSE"); return SFHE_E_UNSUPPORTED; }
  if (A->cols != B->rows) { set_error("A.cols != B.rows"); return SFHE_E_SHAPE; }
  if ((int64_t)B->rows * B->cols > 0x7FFFFFFF) { set_error("B too large"); return SFHE_E_INVALID_ARG; }
  if (A->level != c->L - 1 || B->level != c->L - 1) { set_error("operands must be at the top level"); return SFHE_E_LEVEL; }
  if (c->L < 4) { set_error("Algorithm 1 with the mask needs four data primes"); return SFHE_E_LEVEL; }
  if (A->scale != B->scale) { set_error("operand scales differ"); return SFHE_E_SCALE; }
  hipStream_t s = (hipStream_t)stream;
  StreamScope scope_(c->alloc, s);
  const int N = c->N, top = c->L - 1, M = A->rows, K = A->cols, Nc = B->cols, cs = A->slots;
  // rotation keys first: their generation synchronises the device
  std::vector<int64_t> offs;
  for (int o = 1; o < cs; ++o) { offs.push_back(o); offs.push_back(-o); }
  int rc = prepare_rotations(c, offs);
  if (rc) return rc;
  SFHE_HIP(hipEventRecord(c->ev0, s));
  int64_t rotations = 0, products = 0, keyswitches = 0;
  // 1. one-value operands: A's visited values and all of B rotated into slot 0
  auto one_value = [&](const sfhe_mat* X) {
    sfhe_mat* R = new sfhe_mat();
    R->ctx = c;
    R->rows = X->rows;
    R->cols = X->cols;
    R->level = X->level;
    R->scale = X->scale;
    R->enc = X->enc;
    R->nnz = X->nnz;
    R->row_ptr = X->row_ptr;
    R->col_idx = X->col_idx;
    R->ell_w = X->ell_w;
    R->ell_col = X->ell_col;
    R->zero_mask = X->zero_mask;
    R->n_ct = X->n_vals;
    R->n_vals = X->n_vals;
    return R;
  };
  std::unique_ptr<sfhe_mat> RA(one_value(A)), RB(one_value(B));
  const int64_t w_top = (int64_t)2 * (top + 1) * N;
  if (!RA->data.alloc(&c->alloc, (size_t)std::max<int64_t>(RA->n_ct, 1) * w_top) ||
      !RB->data.alloc(&c->alloc, (size_t)std::max<int64_t>(RB->n_ct, 1) * w_top)) {
    set_error("device allocation failed");
    return SFHE_E_NOMEM;
  }
  std::vector<int64_t> visits(M);
  std::vector<std::pair<int, int64_t>> pairs;
  std::vector<int64_t> used;
  {
    std::vector<char> seen((size_t)std::max<int64_t>(A->n_vals, 1), 0);
    for (int i = 0; i < M; ++i) {
      row_pairs(A, i, pairs);
      visits[i] = (int64_t)pairs.size();
      for (auto& pr : pairs) seen[pr.second] = 1;
    }
    for (int64_t v = 0; v < A->n_vals; ++v)
      if (seen[v]) used.push_back(v);
  }
  std::vector<int64_t> allb((size_t)K * Nc);
  for (int64_t v = 0; v < (int64_t)K * Nc; ++v) allb[v] = v;
  if (A->enc == SFHE_ENC_ELL || A->enc == SFHE_ENC_NAIVE_SPARSE)
    rc = launch_zero(RA->data.ptr, RA->n_ct * w_top, s);   // values no product visits stay trivial zeros
  if (!rc) rc = unpack_values(c, A, used, RA.get(), s, rotations);
  if (!rc) rc = unpack_values(c, B, allb, RB.get(), s, rotations);
  if (rc) return rc;
  // 2. the result: ceil(M Nc / cs) chunks at level top - 2, trivial zeros to start
  const int lo = top - 2;
  std::unique_ptr<sfhe_mat> out(new sfhe_mat());
  out->ctx = c;
  out->rows = M;
  out->cols = Nc;
  out->level = lo;
  out->scale = A->scale * B->scale / (double)c->primes[top] * ldexp(1.0, (int)c->log2_scale) / (double)c->primes[top - 1];
  out->enc = SFHE_ENC_DENSE;
  out->slots = cs;
  out->n_vals = (int64_t)M * Nc;
  out->n_ct = (out->n_vals + cs - 1) / cs;
  out->nnz = out->n_vals;
  if (!out->data.alloc(&c->alloc, (size_t)out->n_ct * 2 * (lo + 1) * N)) {
    set_error("device allocation failed for the result");
    return SFHE_E_NOMEM;
  }
  rc = launch_zero(out->data.ptr, out->n_ct * 2 * (lo + 1) * N, s);
  if (rc) return rc;
  const int l1 = top - 1;                            // level after the first rescale
  const int64_t w1 = (int64_t)2 * (l1 + 1) * N;
  const int64_t slice = 256;
  if (sched == SFHE_SCHED_LAZY) {
    // sums of the one-value products, relinearised and rescaled (level top - 1)
    sfhe_mat* C1 = nullptr;
    rc = matmul_c1(c, RA.get(), RB.get(), SFHE_SCHED_LAZY, s, &C1, false);
    if (rc) return rc;
    std::unique_ptr<sfhe_mat> C1p(C1);
    products = c->stats.products;
    keyswitches += c->stats.keyswitches;
    // outputs with a product, by their slot in the output chunk
    std::vector<std::vector<int64_t>> by_off(cs);
    for (int i = 0; i < M; ++i)
      if (visits[i])
        for (int j = 0; j < Nc; ++j) by_off[((int64_t)i * Nc + j) % cs].push_back((int64_t)i * Nc + j);
    DevBuf<u64> X;
    DevBuf<int64_t> d_e;
    if (!X.alloc(&c->alloc, (size_t)slice * w1)) { set_error("device allocation failed"); return SFHE_E_NOMEM; }
    for (int o = 0; o < cs && !rc; ++o)
      for (size_t x0 = 0; x0 < by_off[o].size() && !rc; x0 += slice) {
        const int64_t n = std::min<int64_t>(slice, (int64_t)(by_off[o].size() - x0));
        std::vector<int64_t> es(by_off[o].begin() + x0, by_off[o].begin() + x0 + n), oidx(es);
        std::vector<int> seg(n + 1);
        for (int64_t x = 0; x <= n; ++x) seg[x] = (int)x;
        for (auto& e : oidx) e /= cs;
        if (!upload(c, d_e, es, s)) { set_error("device allocation failed"); return SFHE_E_NOMEM; }
        rc = launch_from_chunked(c, C1->data.ptr, C1->n_ct, l1 + 1, n, d_e.ptr, 0, X.ptr, w1, s);
        if (!rc) rc = finish_products(c, l1, X.ptr, n, o, seg, oidx, out.get(), s, rotations);
      }
  } else {
    // Algorithm 1's order: every product relinearised, rescaled, masked,
    // rescaled and rotated on its own, then added into its output chunk
    struct Item { int64_t rs, sa, sb; };
    std::vector<std::vector<Item>> by_off(cs);
    for (int i = 0; i < M; ++i) {
      if (!visits[i]) continue;
      row_pairs(A, i, pairs);
      for (int j = 0; j < Nc; ++j) {
        const int64_t rs = (int64_t)i * Nc + j;
        for (auto& pr : pairs) by_off[rs % cs].push_back(Item{rs, pr.second, (int64_t)pr.first * Nc + j});
      }
    }
    const int64_t dw = (int64_t)3 * (top + 1) * N;
    DevBuf<u64> D, T;
    DevBuf<int> d_a, d_b;
    if (!D.alloc(&c->alloc, (size_t)slice * dw) || !T.alloc(&c->alloc, (size_t)slice * w1)) {
      set_error("device allocation failed");
      return SFHE_E_NOMEM;
    }
    for (int o = 0; o < cs && !rc; ++o)
      for (size_t x0 = 0; x0 < by_off[o].size() && !rc; x0 += slice) {
        const int64_t n = std::min<int64_t>(slice, (int64_t)(by_off[o].size() - x0));
        std::vector<int> ai(n), bi(n), seg;
        std::vector<int64_t> oidx;
        for (int64_t x = 0; x < n; ++x) {
          const Item& it = by_off[o][x0 + x];
          ai[x] = (int)it.sa;
          bi[x] = (int)it.sb;
          if (x == 0 || it.rs != by_off[o][x0 + x - 1].rs) { seg.push_back((int)x); oidx.push_back(it.rs / cs); }
        }
        seg.push_back((int)n);
        if (!upload(c, d_a, ai, s) || !upload(c, d_b, bi, s)) { set_error("device allocation failed"); return SFHE_E_NOMEM; }
        rc = launch_tensor_gather(c, top, RA->data.ptr, RA->n_ct, RB->data.ptr, RB->n_ct, d_a.ptr, d_b.ptr, D.ptr, n, s);
        const OutLayout ol{T.ptr, w1, false, 0, 0};
        if (!rc && keyswitch_rescale_n14_supported(c)) {
          rc = keyswitch_rescale_n14(c, top, D.ptr, dw, ol, n, s);
        } else if (!rc) {
          rc = keyswitch_batch(c, top, D.ptr + (int64_t)2 * (top + 1) * N, dw, D.ptr, dw, true, n, s);
          if (!rc) rc = rescale_batch(c, top, D.ptr, dw, ol, n, s);
        }
        if (!rc) rc = finish_products(c, l1, T.ptr, n, o, seg, oidx, out.get(), s, rotations);
        products += n;
        keyswitches += n;
      }
  }
  if (rc) return rc;
  SFHE_HIP(hipEventRecord(c->ev1, s));
  c->stats = sfhe_stats{};
  c->stats.products = products;
  c->stats.keyswitches = keyswitches + rotations;   // relinearisations and rotations
  c->stats.outputs = out->n_ct;
  c->stats.tensor_fp_primes = tensor_fp_prime_count(c);
  c->stats_pending = true;
  *C = out.release();
  return SFHE_OK;
  GUARD_END
}

}  // extern "C"
