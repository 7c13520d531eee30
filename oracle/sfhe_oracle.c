/*
 * sfhe_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-source CPU implementation of the encrypted matrix
 * product of Ferguson et al., "Exploiting Unstructured Sparsity in Fully
 * Homomorphic Encrypted DNNs" (EuroMLSys '25):
 *   - the naive dense product of Algorithm 1 at chunk size c = 1 (Sec. 3.2,
 *     Sec. 3.3.1): per (row, col, k) multiply, relinearise, rescale, accumulate;
 *   - the three sparse schemes of Sec. 3.3.2 (naive sparse with a plaintext
 *     zero mask, CSR, ELLPACK), which skip the products whose A element is 0;
 *   - the thread assignment of Sec. 3.4 (result value -> thread by its index
 *     modulo the pool size);
 *   - chunks of several values per ciphertext (Sec. 3.2) with Algorithm 1's
 *     rotations and slot-zero mask, and plaintext weights times encrypted
 *     values (Sec. 3.3.2);
 * over an RNS CKKS scheme (Sec. 3.1) with secret-key encryption, hybrid key
 * switching and exact rescaling.
 *
 * Every modular product is (unsigned __int128)a*b % q, every polynomial
 * product goes through a textbook radix-2 negacyclic NTT, and every
 * reduction is a plain %.  Nothing here is shared with the GPU library: the
 * two implementations meet only through their outputs.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load this file.
 *
 * Conventions fixed here because the paper is silent on them (each is a
 * documented reading):
 *   R1  one value per ciphertext, in slot 0 of the canonical embedding with
 *       zeta = exp(i*pi/N); m_t = nearbyint(z * 2*Delta/N * cos(pi*t/N)).
 *   R2  secret-key encryption c = (-a*s + e + m, a); a uniform per limb, e a
 *       discrete Gaussian (sigma = 3.2, |e| <= 19, cumulative-table sampler),
 *       s uniform ternary.
 *   R3  randomness from SplitMix64 used as a counter-based generator, one
 *       stream per (seed, tag, fields); see key_of() and word().
 *   R4  hybrid key switching with contiguous digits of alpha data primes,
 *       centered fast base conversions in ModUp and ModDown (the converted
 *       residues taken in (-q/2, q/2)): ModDown's division by P then carries
 *       no bias, and ModUp commutes with X -> X^g (it maps -x to -x), so a
 *       digit raised once serves every rotation of a ciphertext.
 *   R5  rescale by the last prime with the centered lift (exact rounding).
 *   R6  outputs with no product are trivial zero ciphertexts.
 *   R7  NTT-domain index k holds a(psi^(2*brv(k)+1)), psi the smallest
 *       primitive 2N-th root of unity mod q.
 *   R8  plaintext weights (the server-side weights of Sec. 3.3.2) are
 *       constant polynomials nearbyint(w * 2^sw); see orc_weight().
 *   R9  both operands sparse (the naive scheme's two masks, Sec. 3.3.2, and
 *       CSR/ELLPACK on the right operand): output (i, j) visits the k of row
 *       i whose B_kj the right operand's encoding stores; see out_ks().
 *   R10 several values per ciphertext: slot j at zeta^(5^j), rotations by
 *       X -> X^g with g = 5^r mod 2N and rotation keys; see the section on
 *       chunks below.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

typedef uint64_t u64;
typedef int64_t i64;
typedef unsigned __int128 u128;

#define ORC_MAXB 24          /* data + special primes */
#define ORC_CDT 20           /* |e| <= 19 */

enum { ORC_ENC_DENSE = 0, ORC_ENC_NAIVE = 1, ORC_ENC_CSR = 2, ORC_ENC_ELL = 3 };
enum { ORC_SCHED_PER_PRODUCT = 0, ORC_SCHED_LAZY = 1 };
enum { TAG_SK = 1, TAG_RLK_A = 2, TAG_RLK_E = 3, TAG_ENC_A = 4, TAG_ENC_E = 5, TAG_ROT_A = 6, TAG_ROT_E = 7 };

/* ------------------------------------------------------------------ */
/* modular arithmetic, plain                                           */
/* ------------------------------------------------------------------ */
static u64 addm(u64 a, u64 b, u64 q) { u64 s = a + b; return s >= q ? s - q : s; }
static u64 subm(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + (q - b); }
static u64 mulm(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }
static u64 powm(u64 a, u64 e, u64 q) {
  u64 r = 1 % q;
  a %= q;
  while (e) { if (e & 1) r = mulm(r, a, q); a = mulm(a, a, q); e >>= 1; }
  return r;
}
static u64 invm(u64 a, u64 q) { return powm(a, q - 2, q); } /* q prime */
/* signed integer -> residue */
static u64 redi(i64 v, u64 q) {
  if (v >= 0) return (u64)v % q;
  u64 r = (u64)(-(v + 1)) % q;  /* -(v+1) >= 0, avoids overflow at INT64_MIN */
  return (q - 1) - r;
}

/* ------------------------------------------------------------------ */
/* primes: deterministic Miller-Rabin (bases valid for all n < 2^64)    */
/* ------------------------------------------------------------------ */
static int is_prime(u64 n) {
  static const u64 bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; i++) { if (n == bases[i]) return 1; if (n % bases[i] == 0) return 0; }
  u64 d = n - 1; int r = 0;
  while ((d & 1) == 0) { d >>= 1; r++; }
  for (int i = 0; i < 12; i++) {
    u64 x = powm(bases[i], d, n);
    if (x == 1 || x == n - 1) continue;
    int comp = 1;
    for (int k = 1; k < r; k++) { x = mulm(x, x, n); if (x == n - 1) { comp = 0; break; } }
    if (comp) return 0;
  }
  return 1;
}

/* ------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea, Flood 2014) as a counter-based generator    */
/* ------------------------------------------------------------------ */
static const u64 GOLDEN = 0x9E3779B97F4A7C15ULL;
static u64 mix64(u64 z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
/* stream key: k = mix(seed + (tag+1)*G); then k = mix(k + (f+1)*G) per field */
static u64 key_of(u64 seed, u64 tag, int nf, const u64* f) {
  u64 k = mix64(seed + (tag + 1) * GOLDEN);
  for (int i = 0; i < nf; i++) k = mix64(k + (f[i] + 1) * GOLDEN);
  return k;
}
/* n-th word of a stream */
static u64 word(u64 key, u64 n) { return mix64(key + (n + 1) * GOLDEN); }
/* uniform residue for coefficient t: (w(2t) * 2^64 + w(2t+1)) mod q */
static u64 uniform_at(u64 key, u64 t, u64 q) {
  u128 x = ((u128)word(key, 2 * t) << 64) | word(key, 2 * t + 1);
  return (u64)(x % q);
}

/* ------------------------------------------------------------------ */
/* context                                                              */
/* ------------------------------------------------------------------ */
typedef struct {
  int logN, N, L, alpha, dnum, nb;   /* nb = L + alpha */
  u64 q[ORC_MAXB];                   /* data primes q_0..q_{L-1}, then p_0..p_{alpha-1} */
  u64 psi[ORC_MAXB];
  u64* fw[ORC_MAXB];                 /* psi^brv(m) */
  u64* iw[ORC_MAXB];                 /* psi^-brv(m) */
  u64 ninv[ORC_MAXB];
  double log2_scale, sigma;
  u64 cdt[ORC_CDT];
  double* cosv;                      /* cos(pi t / N) from the host libm */
  int has_keys;
  i64* s;                            /* ternary secret */
  u64* rlk;                          /* [dnum][2][nb][N] coefficient domain: (b_j, a_j) */
  u64* rlk_e;                        /* [dnum][N] the key errors, kept for the pins */
  u64* rlk_ntt;                      /* the same key in the NTT domain, for the products */
  u64 seed;
} orc_ctx;

static int brv(int x, int bits) {
  int r = 0;
  for (int i = 0; i < bits; i++) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
}

/* smallest primitive 2N-th root of unity: psi^N = -1 (mod q), minimal value */
static u64 min_root(u64 q, int N) {
  u64 g = 0;
  for (u64 x = 2; x < q; x++) {             /* a quadratic non-residue */
    if (powm(x, (q - 1) / 2, q) == q - 1) { g = x; break; }
  }
  u64 w = powm(g, (q - 1) / (2 * (u64)N), q);  /* order exactly 2N */
  u64 w2 = mulm(w, w, q), cur = w, best = w;
  for (int k = 1; k < N; k++) { cur = mulm(cur, w2, q); if (cur < best) best = cur; }
  return best;
}

static void cdt_build(double sigma, u64* T) {
  double rho[ORC_CDT];
  for (int x = 0; x < ORC_CDT; x++) rho[x] = exp(-(double)(x * x) / (2.0 * sigma * sigma));
  double Z = rho[0];
  for (int x = 1; x < ORC_CDT; x++) Z += 2.0 * rho[x];
  double cum = rho[0];
  for (int k = 0; k < ORC_CDT; k++) {
    if (k > 0) cum += 2.0 * rho[k];
    T[k] = (u64)((cum / Z) * 9223372036854775808.0);   /* 2^63 */
  }
}
static i64 cdt_sample(const u64* T, u64 w) {
  u64 u = w & 0x7FFFFFFFFFFFFFFFULL;
  int mag = ORC_CDT - 1;
  for (int k = 0; k < ORC_CDT; k++) if (u < T[k]) { mag = k; break; }
  return (w >> 63) ? -(i64)mag : (i64)mag;
}

/* ------------------------------------------------------------------ */
/* NTT: textbook negacyclic radix-2 (Cooley-Tukey forward with the psi  */
/* twist merged, Gentleman-Sande inverse), bit-reversed NTT order       */
/* ------------------------------------------------------------------ */
static void ntt_fwd(const orc_ctx* c, int r, u64* a) {
  int N = c->N; u64 q = c->q[r]; const u64* W = c->fw[r];
  int t = N;
  for (int m = 1; m < N; m <<= 1) {
    t >>= 1;
    for (int i = 0; i < m; i++) {
      int j1 = 2 * i * t; u64 S = W[m + i];
      for (int j = j1; j < j1 + t; j++) {
        u64 U = a[j], V = mulm(a[j + t], S, q);
        a[j] = addm(U, V, q); a[j + t] = subm(U, V, q);
      }
    }
  }
}
static void ntt_inv(const orc_ctx* c, int r, u64* a) {
  int N = c->N; u64 q = c->q[r]; const u64* W = c->iw[r];
  int t = 1;
  for (int m = N; m > 1; m >>= 1) {
    int h = m >> 1, j1 = 0;
    for (int i = 0; i < h; i++) {
      u64 S = W[h + i];
      for (int j = j1; j < j1 + t; j++) {
        u64 U = a[j], V = a[j + t];
        a[j] = addm(U, V, q); a[j + t] = mulm(subm(U, V, q), S, q);
      }
      j1 += 2 * t;
    }
    t <<= 1;
  }
  for (int j = 0; j < N; j++) a[j] = mulm(a[j], c->ninv[r], q);
}
/* out = a * b in Z_q[X]/(X^N + 1), coefficient domain in and out */
static void polymul(const orc_ctx* c, int r, const u64* a, const u64* b, u64* out) {
  int N = c->N;
  u64* A = malloc(sizeof(u64) * N); u64* B = malloc(sizeof(u64) * N);
  memcpy(A, a, sizeof(u64) * N); memcpy(B, b, sizeof(u64) * N);
  ntt_fwd(c, r, A); ntt_fwd(c, r, B);
  for (int j = 0; j < N; j++) A[j] = mulm(A[j], B[j], c->q[r]);
  ntt_inv(c, r, A);
  memcpy(out, A, sizeof(u64) * N);
  free(A); free(B);
}

/* ------------------------------------------------------------------ */
/* context creation                                                     */
/* ------------------------------------------------------------------ */
void orc_ctx_destroy(orc_ctx* c) {
  if (!c) return;
  for (int r = 0; r < c->nb; r++) { free(c->fw[r]); free(c->iw[r]); }
  free(c->cosv); free(c->s); free(c->rlk); free(c->rlk_e); free(c->rlk_ntt);
  free(c);
}

/* primes: for each requested size b (data first, then special), the largest
 * prime q < 2^b with q = 1 (mod 2N) not already taken. */
orc_ctx* orc_ctx_create(int logN, int L, const int* qbits, int alpha, const int* pbits,
                        int dnum, double log2_scale, double sigma) {
  if (logN < 2 || logN > 16 || L < 1 || alpha < 1 || L + alpha > ORC_MAXB) return NULL;
  if (dnum != (L + alpha - 1) / alpha) return NULL;
  orc_ctx* c = calloc(1, sizeof(orc_ctx));
  c->logN = logN; c->N = 1 << logN; c->L = L; c->alpha = alpha; c->dnum = dnum;
  c->nb = L + alpha; c->log2_scale = log2_scale; c->sigma = sigma;
  u64 twoN = 2 * (u64)c->N;
  for (int r = 0; r < c->nb; r++) {
    int b = r < L ? qbits[r] : pbits[r - L];
    if (b < logN + 2 || b > 61) { orc_ctx_destroy(c); return NULL; }
    u64 top = (u64)1 << b;
    u64 cand = ((top - 1) / twoN) * twoN + 1;
    if (cand >= top) cand -= twoN;
    for (;;) {
      int used = 0;
      for (int s = 0; s < r; s++) if (c->q[s] == cand) used = 1;
      if (!used && is_prime(cand)) break;
      if (cand <= twoN) { orc_ctx_destroy(c); return NULL; }
      cand -= twoN;
    }
    c->q[r] = cand;
  }
  for (int r = 0; r < c->nb; r++) {
    u64 q = c->q[r];
    c->psi[r] = min_root(q, c->N);
    u64 pinv = invm(c->psi[r], q);
    c->fw[r] = malloc(sizeof(u64) * c->N); c->iw[r] = malloc(sizeof(u64) * c->N);
    for (int m = 0; m < c->N; m++) {
      int e = brv(m, logN);
      c->fw[r][m] = powm(c->psi[r], (u64)e, q);
      c->iw[r][m] = powm(pinv, (u64)e, q);
    }
    c->ninv[r] = invm((u64)c->N % q, q);
  }
  cdt_build(sigma, c->cdt);
  c->cosv = malloc(sizeof(double) * c->N);
  for (int t = 0; t < c->N; t++) c->cosv[t] = cos(M_PI * (double)t / (double)c->N);
  return c;
}

int orc_n(const orc_ctx* c) { return c->N; }
int orc_nbasis(const orc_ctx* c) { return c->nb; }
void orc_primes(const orc_ctx* c, u64* out) { for (int r = 0; r < c->nb; r++) out[r] = c->q[r]; }
void orc_psi(const orc_ctx* c, u64* out) { for (int r = 0; r < c->nb; r++) out[r] = c->psi[r]; }
void orc_cdt_table(const orc_ctx* c, u64* out) { for (int k = 0; k < ORC_CDT; k++) out[k] = c->cdt[k]; }
void orc_ntt_forward(const orc_ctx* c, int r, u64* a) { ntt_fwd(c, r, a); }
void orc_ntt_inverse(const orc_ctx* c, int r, u64* a) { ntt_inv(c, r, a); }
void orc_polymul(const orc_ctx* c, int r, const u64* a, const u64* b, u64* out) { polymul(c, r, a, b, out); }
int orc_is_prime(u64 n) { return is_prime(n); }
u64 orc_stream_word(u64 seed, u64 tag, int nf, const u64* f, u64 n) { return word(key_of(seed, tag, nf, f), n); }

/* ------------------------------------------------------------------ */
/* encode (R1)                                                          */
/* ------------------------------------------------------------------ */
/* m_t for the value z in slot 0.  Returns -1 if the scaled value does not fit. */
int orc_encode(const orc_ctx* c, double z, i64* m) {
  double sz = ldexp(z, (int)c->log2_scale + 1 - c->logN);   /* z * 2*Delta/N, exact */
  if (!(fabs(sz) < 4.0e18)) return -1;
  for (int t = 0; t < c->N; t++) m[t] = (i64)nearbyint(sz * c->cosv[t]);
  return 0;
}

/* ------------------------------------------------------------------ */
/* keys (R2, R4)                                                        */
/* ------------------------------------------------------------------ */
/* digit j holds data primes j*alpha .. min((j+1)*alpha, L)-1 */
static int digit_lo(const orc_ctx* c, int j) { return j * c->alpha; }
static int digit_hi(const orc_ctx* c, int j) { int h = (j + 1) * c->alpha; return h < c->L ? h : c->L; }

void orc_keygen(orc_ctx* c, u64 seed) {
  int N = c->N, nb = c->nb;
  free(c->s); free(c->rlk); free(c->rlk_e); free(c->rlk_ntt);
  c->seed = seed;
  c->s = malloc(sizeof(i64) * N);
  u64 ks = key_of(seed, TAG_SK, 0, NULL);
  for (int t = 0; t < N; t++) c->s[t] = (i64)(word(ks, t) % 3) - 1;
  c->rlk = malloc(sizeof(u64) * (size_t)c->dnum * 2 * nb * N);
  c->rlk_e = malloc(sizeof(u64) * (size_t)c->dnum * N);
  u64* sr = malloc(sizeof(u64) * N);
  u64* s2 = malloc(sizeof(u64) * N);
  u64* as = malloc(sizeof(u64) * N);
  i64* e = malloc(sizeof(i64) * N);
  for (int j = 0; j < c->dnum; j++) {
    u64 fj = (u64)j;
    u64 ke = key_of(seed, TAG_RLK_E, 1, &fj);
    for (int t = 0; t < N; t++) { e[t] = cdt_sample(c->cdt, word(ke, t)); c->rlk_e[(size_t)j * N + t] = (u64)e[t]; }
    for (int r = 0; r < nb; r++) {
      u64 q = c->q[r];
      u64* b = c->rlk + (((size_t)j * 2 + 0) * nb + r) * N;
      u64* a = c->rlk + (((size_t)j * 2 + 1) * nb + r) * N;
      u64 f[2] = {(u64)j, (u64)r};
      u64 ka = key_of(seed, TAG_RLK_A, 2, f);
      for (int t = 0; t < N; t++) a[t] = uniform_at(ka, t, q);
      for (int t = 0; t < N; t++) sr[t] = redi(c->s[t], q);
      polymul(c, r, a, sr, as);
      polymul(c, r, sr, sr, s2);
      /* gadget: P * (Q/D_j) * [(Q/D_j)^-1]_{D_j} is P mod q_r on digit j, 0 elsewhere */
      u64 g = 0;
      if (r >= digit_lo(c, j) && r < digit_hi(c, j)) {
        g = 1;
        for (int k = c->L; k < nb; k++) g = mulm(g, c->q[k] % q, q);
      }
      for (int t = 0; t < N; t++) {
        u64 v = subm(redi(e[t], q), as[t], q);
        b[t] = addm(v, mulm(g, s2[t], q), q);
      }
    }
  }
  free(sr); free(s2); free(as); free(e);
  size_t kn = (size_t)c->dnum * 2 * nb * N;
  c->rlk_ntt = malloc(sizeof(u64) * kn);
  memcpy(c->rlk_ntt, c->rlk, sizeof(u64) * kn);
  for (int j = 0; j < c->dnum; j++)
    for (int p = 0; p < 2; p++)
      for (int r = 0; r < nb; r++) ntt_fwd(c, r, c->rlk_ntt + (((size_t)j * 2 + p) * nb + r) * N);
  c->has_keys = 1;
}
void orc_secret(const orc_ctx* c, i64* out) { memcpy(out, c->s, sizeof(i64) * c->N); }
void orc_rlk(const orc_ctx* c, int j, u64* out) {
  memcpy(out, c->rlk + (size_t)j * 2 * c->nb * c->N, sizeof(u64) * 2 * c->nb * c->N);
}
void orc_rlk_error(const orc_ctx* c, int j, i64* out) {
  for (int t = 0; t < c->N; t++) out[t] = (i64)c->rlk_e[(size_t)j * c->N + t];
}

/* ------------------------------------------------------------------ */
/* encrypt (R2): ct[2][L][N] coefficient domain at the top level         */
/* ------------------------------------------------------------------ */
void orc_enc_error(const orc_ctx* c, u64 seed, u64 operand, u64 i, u64 j, i64* e) {
  u64 f[3] = {operand, i, j};
  u64 k = key_of(seed, TAG_ENC_E, 3, f);
  for (int t = 0; t < c->N; t++) e[t] = cdt_sample(c->cdt, word(k, t));
}
int orc_encrypt(const orc_ctx* c, double z, u64 seed, u64 operand, u64 i, u64 j, u64* ct) {
  int N = c->N, L = c->L;
  i64* m = malloc(sizeof(i64) * N);
  i64* e = malloc(sizeof(i64) * N);
  u64* sr = malloc(sizeof(u64) * N);
  u64* as = malloc(sizeof(u64) * N);
  if (orc_encode(c, z, m) != 0) { free(m); free(e); free(sr); free(as); return -1; }
  orc_enc_error(c, seed, operand, i, j, e);
  for (int r = 0; r < L; r++) {
    u64 q = c->q[r];
    u64* c0 = ct + (size_t)r * N;
    u64* c1 = ct + (size_t)(L + r) * N;
    u64 f[4] = {operand, i, j, (u64)r};
    u64 ka = key_of(seed, TAG_ENC_A, 4, f);
    for (int t = 0; t < N; t++) c1[t] = uniform_at(ka, t, q);
    for (int t = 0; t < N; t++) sr[t] = redi(c->s[t], q);
    polymul(c, r, c1, sr, as);
    for (int t = 0; t < N; t++) c0[t] = subm(addm(redi(e[t], q), redi(m[t], q), q), as[t], q);
  }
  free(m); free(e); free(sr); free(as);
  return 0;
}

/* ------------------------------------------------------------------ */
/* tensor product of two degree-1 ciphertexts at level `lev`            */
/* (limbs 0..lev), coefficient domain: d0 = a0 b0, d1 = a0 b1 + a1 b0,  */
/* d2 = a1 b1.  Layout: ct[2][lev+1][N], d[3][lev+1][N].                 */
/* ------------------------------------------------------------------ */
void orc_tensor(const orc_ctx* c, int lev, const u64* a, const u64* b, u64* d) {
  int N = c->N, nl = lev + 1;
  u64* tmp = malloc(sizeof(u64) * N);
  for (int r = 0; r < nl; r++) {
    u64 q = c->q[r];
    const u64 *a0 = a + (size_t)r * N, *a1 = a + (size_t)(nl + r) * N;
    const u64 *b0 = b + (size_t)r * N, *b1 = b + (size_t)(nl + r) * N;
    u64 *d0 = d + (size_t)r * N, *d1 = d + (size_t)(nl + r) * N, *d2 = d + (size_t)(2 * nl + r) * N;
    polymul(c, r, a0, b0, d0);
    polymul(c, r, a0, b1, d1);
    polymul(c, r, a1, b0, tmp);
    for (int t = 0; t < N; t++) d1[t] = addm(d1[t], tmp[t], q);
    polymul(c, r, a1, b1, d2);
  }
  free(tmp);
}

/* ------------------------------------------------------------------ */
/* hybrid key switching (R4) of the degree-2 part d2 at level `lev`.    */
/* in: d2[lev+1][N] coefficient domain; out: ks[2][lev+1][N] with        */
/* ks0 + ks1*s = d2*s^2 + small (mod Q_lev).                            */
/* ------------------------------------------------------------------ */
/* basis index of the k-th special prime */
#define SP(c, k) ((c)->L + (k))

/* the extended basis at level lev: data primes 0..lev, then the special primes */
static int ext_basis(const orc_ctx* c, int lev, int* eb) {
  int nl = lev + 1;
  for (int r = 0; r < nl; r++) eb[r] = r;
  for (int k = 0; k < c->alpha; k++) eb[nl + k] = SP(c, k);
  return nl + c->alpha;
}

/* ModUp of digit j: the residues, over the extended basis, of the integer
 * x = sum_{i in D_j} [d2_i * (D_j/q_i)^-1]_{q_i} * (D_j/q_i) with each
 * [.]_{q_i} taken in (-q_i/2, q_i/2) (centered fast base conversion, R4),
 * which is congruent to d2 modulo every prime of the digit.
 * in: d2[lev+1][N] coefficient domain; out: x[lev+1+alpha][N] coefficient domain. */
void orc_modup(const orc_ctx* c, int lev, int j, const u64* d2, u64* x) {
  int N = c->N, nl = lev + 1, eb[ORC_MAXB];
  int ne = ext_basis(c, lev, eb);
  int lo = digit_lo(c, j), hi = digit_hi(c, j);
  if (hi > nl) hi = nl;
  u64* y = malloc(sizeof(u64) * (size_t)nl * N);
  for (int i = lo; i < hi; i++) {
    u64 qi = c->q[i], Dq = 1;
    for (int i2 = lo; i2 < hi; i2++) if (i2 != i) Dq = mulm(Dq, c->q[i2] % qi, qi);
    u64 inv = invm(Dq, qi);
    for (int t = 0; t < N; t++) y[(size_t)i * N + t] = mulm(d2[(size_t)i * N + t], inv, qi);
  }
  for (int e = 0; e < ne; e++) {
    int r = eb[e]; u64 qt = c->q[r];
    u64* xo = x + (size_t)e * N;
    if (r >= lo && r < hi) { memcpy(xo, d2 + (size_t)r * N, sizeof(u64) * N); continue; }
    memset(xo, 0, sizeof(u64) * N);
    for (int i = lo; i < hi; i++) {
      u64 qi = c->q[i], Dq = 1;                           /* [D_j/q_i]_t */
      for (int i2 = lo; i2 < hi; i2++) if (i2 != i) Dq = mulm(Dq, c->q[i2] % qt, qt);
      for (int t = 0; t < N; t++) {
        u64 yv = y[(size_t)i * N + t];
        i64 yc = yv > (qi - 1) / 2 ? -(i64)(qi - yv) : (i64)yv;   /* centered representative */
        xo[t] = addm(xo[t], mulm(redi(yc, qt), Dq, qt), qt);
      }
    }
  }
  free(y);
}

/* ModDown: divide by P = prod p_k.  out_i = (acc_i - F_i) * P^-1 mod q_i with
 * F = sum_k y_k (P/p_k), y_k = [acc_{p_k} (P/p_k)^-1]_{p_k} taken in
 * (-p_k/2, p_k/2): the centered fast base conversion of the special part, so
 * F = (acc mod P) + u P with u symmetric about zero (R4).  With y_k in
 * [0, p_k) instead, u would lie in [0, alpha) with mean near (alpha - 1)/2,
 * and the bias u s that the second component carries, a random walk over the
 * coefficients, would add a low-frequency error of order N^1.5 to every key
 * switch.  in: acc[lev+1+alpha][N], out: [lev+1][N], both coefficient domain. */
void orc_moddown(const orc_ctx* c, int lev, const u64* acc, u64* out) {
  int N = c->N, nl = lev + 1, al = c->alpha;
  u64* yk = malloc(sizeof(u64) * (size_t)al * N);
  for (int k = 0; k < al; k++) {
    u64 pk = c->q[SP(c, k)], Pq = 1;
    for (int k2 = 0; k2 < al; k2++) if (k2 != k) Pq = mulm(Pq, c->q[SP(c, k2)] % pk, pk);
    u64 inv = invm(Pq, pk);
    const u64* src = acc + (size_t)(nl + k) * N;
    for (int t = 0; t < N; t++) yk[(size_t)k * N + t] = mulm(src[t], inv, pk);
  }
  for (int i = 0; i < nl; i++) {
    u64 qi = c->q[i], Pinv = 1;
    for (int k = 0; k < al; k++) Pinv = mulm(Pinv, c->q[SP(c, k)] % qi, qi);
    Pinv = invm(Pinv, qi);
    const u64* ai = acc + (size_t)i * N;
    u64* o = out + (size_t)i * N;
    for (int t = 0; t < N; t++) {
      u64 z = 0;
      for (int k = 0; k < al; k++) {
        u64 pk = c->q[SP(c, k)], Pq = 1;                  /* [P/p_k]_{q_i} */
        for (int k2 = 0; k2 < al; k2++) if (k2 != k) Pq = mulm(Pq, c->q[SP(c, k2)] % qi, qi);
        u64 y = yk[(size_t)k * N + t];
        i64 yc = y > (pk - 1) / 2 ? -(i64)(pk - y) : (i64)y;   /* centered representative */
        z = addm(z, mulm(redi(yc, qi), Pq, qi), qi);
      }
      o[t] = mulm(subm(ai[t], z, qi), Pinv, qi);
    }
  }
  free(yk);
}

/* Hybrid key switching (R4) of the degree-2 part at level lev:
 * in d2[lev+1][N], out ks[2][lev+1][N], both coefficient domain, with
 * ks0 + ks1*s = d2*s^2 + small (mod Q_lev).  Per digit: ModUp, then the
 * products with the key (b_j, a_j) summed over the digits, then ModDown. */
static void ks_with(const orc_ctx* c, int lev, const u64* d2, const u64* key_ntt, u64* ks);
void orc_keyswitch(const orc_ctx* c, int lev, const u64* d2, u64* ks) { ks_with(c, lev, d2, c->rlk_ntt, ks); }
/* the same with any key [dnum][2][nb][N] (NTT domain) switching from its
 * target secret to s */
static void ks_with(const orc_ctx* c, int lev, const u64* d2, const u64* key_ntt, u64* ks) {
  int N = c->N, nl = lev + 1, eb[ORC_MAXB];
  int ne = ext_basis(c, lev, eb);
  u64* acc = calloc((size_t)2 * ne * N, sizeof(u64));   /* NTT domain */
  u64* x = malloc(sizeof(u64) * (size_t)ne * N);
  for (int j = 0; j < c->dnum; j++) {
    if (digit_lo(c, j) >= nl) continue;
    orc_modup(c, lev, j, d2, x);
    for (int e = 0; e < ne; e++) {
      int r = eb[e];
      u64* xe = x + (size_t)e * N;
      ntt_fwd(c, r, xe);
      for (int p = 0; p < 2; p++) {
        const u64* kp = key_ntt + (((size_t)j * 2 + p) * c->nb + r) * N;
        u64* A = acc + ((size_t)p * ne + e) * N;
        for (int t = 0; t < N; t++) A[t] = addm(A[t], mulm(xe[t], kp[t], c->q[r]), c->q[r]);
      }
    }
  }
  for (int p = 0; p < 2; p++) {
    for (int e = 0; e < ne; e++) ntt_inv(c, eb[e], acc + ((size_t)p * ne + e) * N);
    orc_moddown(c, lev, acc + (size_t)p * ne * N, ks + (size_t)p * nl * N);
  }
  free(acc); free(x);
}

/* ------------------------------------------------------------------ */
/* rescale (R5): ct[2][lev+1][N] -> out[2][lev][N], coefficient domain   */
/* ------------------------------------------------------------------ */
void orc_rescale(const orc_ctx* c, int lev, const u64* ct, u64* out) {
  int N = c->N, nl = lev + 1;
  u64 ql = c->q[lev];
  for (int p = 0; p < 2; p++) {
    const u64* last = ct + ((size_t)p * nl + lev) * N;
    for (int i = 0; i < lev; i++) {
      u64 qi = c->q[i], qinv = invm(ql % qi, qi);
      const u64* src = ct + ((size_t)p * nl + i) * N;
      u64* o = out + ((size_t)p * lev + i) * N;
      for (int t = 0; t < N; t++) {
        u64 v = last[t];
        i64 r = v > (ql - 1) / 2 ? -(i64)(ql - v) : (i64)v;   /* centered lift */
        o[t] = mulm(subm(src[t], redi(r, qi), qi), qinv, qi);
      }
    }
  }
}

/* ------------------------------------------------------------------ */
/* decrypt + decode (slot 0); exact CRT by Garner's mixed radix         */
/* ------------------------------------------------------------------ */
/* m[lev+1][N] = c0 + c1*s, coefficient domain */
void orc_decrypt_poly(const orc_ctx* c, int lev, const u64* ct, u64* m) {
  int N = c->N, nl = lev + 1;
  u64* sr = malloc(sizeof(u64) * N);
  u64* cs = malloc(sizeof(u64) * N);
  for (int r = 0; r < nl; r++) {
    u64 q = c->q[r];
    for (int t = 0; t < N; t++) sr[t] = redi(c->s[t], q);
    polymul(c, r, ct + (size_t)(nl + r) * N, sr, cs);
    for (int t = 0; t < N; t++) m[(size_t)r * N + t] = addm(ct[(size_t)r * N + t], cs[t], q);
  }
  free(sr); free(cs);
}
/* centered integer value of the residues v[0..nl-1] (stride N), as long double */
static long double crt_centered(const orc_ctx* c, int nl, const u64* v, size_t stride) {
  u64 dig[ORC_MAXB];
  for (int i = 0; i < nl; i++) {
    u64 qi = c->q[i];
    u64 x = v[(size_t)i * stride] % qi;
    /* subtract the value of the digits so far, then divide by q_0..q_{i-1} */
    u64 acc = 0, w = 1 % qi;
    for (int k = 0; k < i; k++) { acc = addm(acc, mulm(dig[k] % qi, w, qi), qi); w = mulm(w, c->q[k] % qi, qi); }
    dig[i] = mulm(subm(x, acc, qi), invm(w, qi), qi);
  }
  /* negative iff digits exceed those of (Q-1)/2 = sum ((q_i - 1)/2) W_i, compared from the top */
  int neg = 0;
  for (int i = nl - 1; i >= 0; i--) {
    u64 h = (c->q[i] - 1) / 2;
    if (dig[i] > h) { neg = 1; break; }
    if (dig[i] < h) break;
  }
  long double val = 0.0L, W = 1.0L;
  if (!neg) {
    for (int i = 0; i < nl; i++) { val += (long double)dig[i] * W; W *= (long double)c->q[i]; }
    return val;
  }
  /* Q - x = 1 + sum (q_i - 1 - d_i) W_i */
  val = 1.0L;
  for (int i = 0; i < nl; i++) { val += (long double)(c->q[i] - 1 - dig[i]) * W; W *= (long double)c->q[i]; }
  return -val;
}
double orc_decode(const orc_ctx* c, int lev, const u64* m, double scale) {
  long double s = 0.0L;
  for (int t = 0; t < c->N; t++) s += crt_centered(c, lev + 1, m + t, c->N) * (long double)c->cosv[t];
  return (double)(s / (long double)scale);
}
double orc_decrypt(const orc_ctx* c, int lev, const u64* ct, double scale) {
  u64* m = malloc(sizeof(u64) * (size_t)(lev + 1) * c->N);
  orc_decrypt_poly(c, lev, ct, m);
  double v = orc_decode(c, lev, m, scale);
  free(m);
  return v;
}
/* centered CRT of one coefficient, for the tests */
long double orc_crt_centered(const orc_ctx* c, int nl, const u64* v, size_t stride) { return crt_centered(c, nl, v, stride); }

/* ------------------------------------------------------------------ */
/* encrypted matmul (Algorithm 1 at c = 1 and the sparse schemes)       */
/* ------------------------------------------------------------------ */
/* The plaintext structures each sparse scheme exposes (Sec. 3.3.2). */
typedef struct {
  int enc, M, K;
  unsigned char* zero;   /* naive sparse: B_ik = [A_ik == 0] */
  int* row_ptr;          /* CSR */
  int* col_idx;
  int ell_w;             /* ELLPACK: width = max nonzeros per row */
  int* ell_col;          /* [M][w], -1 marks a padding slot */
} orc_struct;

static void struct_build(orc_struct* S, const double* A, int M, int K, int enc) {
  memset(S, 0, sizeof(*S));
  S->enc = enc; S->M = M; S->K = K;
  if (enc == ORC_ENC_NAIVE) {
    S->zero = malloc((size_t)M * K);
    for (int i = 0; i < M; i++) for (int k = 0; k < K; k++) S->zero[(size_t)i * K + k] = (A[(size_t)i * K + k] == 0.0);
  } else if (enc == ORC_ENC_CSR) {
    S->row_ptr = malloc(sizeof(int) * (M + 1));
    int nnz = 0;
    for (int i = 0; i < M; i++) for (int k = 0; k < K; k++) nnz += (A[(size_t)i * K + k] != 0.0);
    S->col_idx = malloc(sizeof(int) * (nnz ? nnz : 1));
    int p = 0;
    for (int i = 0; i < M; i++) {
      S->row_ptr[i] = p;
      for (int k = 0; k < K; k++) if (A[(size_t)i * K + k] != 0.0) S->col_idx[p++] = k;
    }
    S->row_ptr[M] = p;
  } else if (enc == ORC_ENC_ELL) {
    int w = 0;
    for (int i = 0; i < M; i++) {
      int n = 0;
      for (int k = 0; k < K; k++) n += (A[(size_t)i * K + k] != 0.0);
      if (n > w) w = n;
    }
    S->ell_w = w;
    S->ell_col = malloc(sizeof(int) * ((size_t)M * w + 1));
    for (int i = 0; i < M; i++) {
      int n = 0;
      for (int k = 0; k < K; k++) if (A[(size_t)i * K + k] != 0.0) S->ell_col[(size_t)i * w + n++] = k;
      for (; n < w; n++) S->ell_col[(size_t)i * w + n] = -1;
    }
  }
}
static void struct_free(orc_struct* S) { free(S->zero); free(S->row_ptr); free(S->col_idx); free(S->ell_col); }

/* the k that row i visits, ascending; returns the count */
static int row_ks(const orc_struct* S, int i, int* ks) {
  int n = 0;
  switch (S->enc) {
    case ORC_ENC_DENSE:
      for (int k = 0; k < S->K; k++) ks[n++] = k;
      break;
    case ORC_ENC_NAIVE:   /* skip when the LHS mask marks a zero (B is dense) */
      for (int k = 0; k < S->K; k++) if (!S->zero[(size_t)i * S->K + k]) ks[n++] = k;
      break;
    case ORC_ENC_CSR:
      for (int p = S->row_ptr[i]; p < S->row_ptr[i + 1]; p++) ks[n++] = S->col_idx[p];
      break;
    case ORC_ENC_ELL:
      for (int s = 0; s < S->ell_w; s++) { int k = S->ell_col[(size_t)i * S->ell_w + s]; if (k >= 0) ks[n++] = k; }
      break;
  }
  return n;
}

/* whether the encoding stores element (r, col) as a value to multiply: every
 * element for dense, the nonzeros for the three sparse schemes */
static int stores(const orc_struct* S, int r, int col) {
  switch (S->enc) {
    case ORC_ENC_DENSE: return 1;
    case ORC_ENC_NAIVE: return !S->zero[(size_t)r * S->K + col];
    case ORC_ENC_CSR:
      for (int p = S->row_ptr[r]; p < S->row_ptr[r + 1]; p++) if (S->col_idx[p] == col) return 1;
      return 0;
    case ORC_ENC_ELL:
      for (int s = 0; s < S->ell_w; s++) if (S->ell_col[(size_t)r * S->ell_w + s] == col) return 1;
      return 0;
  }
  return 0;
}

/* the k that output (i, j) visits: row i's visited k (ascending) whose B_kj
 * the right operand's encoding stores (R9) */
static int out_ks(const orc_struct* S, const orc_struct* SB, int i, int j, int* ks) {
  int n = row_ks(S, i, ks), m = 0;
  for (int x = 0; x < n; x++) if (stores(SB, ks[x], j)) ks[m++] = ks[x];
  return m;
}

int orc_row_ks(const double* A, int M, int K, int enc, int i, int* ks) {
  orc_struct S; struct_build(&S, A, M, K, enc);
  int n = row_ks(&S, i, ks);
  struct_free(&S);
  return n;
}

typedef struct {
  const orc_ctx* c;
  const orc_struct* S;
  const orc_struct* SB;   /* the right operand's structure */
  int M, K, Nc, sched, nthreads, tid;
  u64** encA;      /* [M*K] encrypted elements, NTT domain (NULL if unused) */
  u64** encB;      /* [K*Nc] */
  const int* orow; const int* ocol; int nout;
  u64* out;        /* [nout][2][L-1][N] */
} mm_job;

/* one output ciphertext (row i, col j) */
static void mm_output(const mm_job* J, int i, int j, u64* o) {
  const orc_ctx* c = J->c;
  int N = c->N, L = c->L, top = L - 1;
  size_t ct_top = (size_t)2 * L * N, ct_out = (size_t)2 * top * N;
  int* ks = malloc(sizeof(int) * (J->K + 1));
  int nk = out_ks(J->S, J->SB, i, j, ks);
  memset(o, 0, sizeof(u64) * ct_out);                       /* R6: trivial zero */
  if (nk == 0) { free(ks); return; }
  u64* d = malloc(sizeof(u64) * 3 * L * N);
  u64* ksw = malloc(sizeof(u64) * ct_top);
  u64* ct = malloc(sizeof(u64) * ct_top);
  u64* rs = malloc(sizeof(u64) * ct_out);
  if (J->sched == ORC_SCHED_LAZY) {
    /* sum the tensors over k (exactly, 128-bit, NTT domain), then one key
     * switch and one rescale */
    u128* acc = calloc((size_t)3 * L * N, sizeof(u128));
    for (int n = 0; n < nk; n++) {
      int k = ks[n];
      const u64* a = J->encA[(size_t)i * J->K + k];
      const u64* b = J->encB[(size_t)k * J->Nc + j];
      for (int r = 0; r < L; r++) {
        u64 q = c->q[r];
        const u64 *a0 = a + (size_t)r * N, *a1 = a + (size_t)(L + r) * N;
        const u64 *b0 = b + (size_t)r * N, *b1 = b + (size_t)(L + r) * N;
        u128* x0 = acc + (size_t)r * N; u128* x1 = acc + (size_t)(L + r) * N; u128* x2 = acc + (size_t)(2 * L + r) * N;
        for (int t = 0; t < N; t++) {
          x0[t] += (u128)a0[t] * b0[t];
          x1[t] += (u128)a0[t] * b1[t]; x1[t] += (u128)a1[t] * b0[t];
          x2[t] += (u128)a1[t] * b1[t];
          if ((n & 31) == 31) { x0[t] %= q; x1[t] %= q; x2[t] %= q; }   /* 64 terms < 2^122 stay below 2^128 */
        }
      }
    }
    for (int p = 0; p < 3; p++)
      for (int r = 0; r < L; r++) {
        u64* dd = d + ((size_t)p * L + r) * N;
        for (int t = 0; t < N; t++) dd[t] = (u64)(acc[((size_t)p * L + r) * N + t] % c->q[r]);
        ntt_inv(c, r, dd);
      }
    free(acc);
    orc_keyswitch(c, top, d + (size_t)2 * L * N, ksw);
    for (int p = 0; p < 2; p++) for (int r = 0; r < L; r++)
      for (int t = 0; t < N; t++) {
        size_t x = ((size_t)p * L + r) * N + t;
        ct[x] = addm(d[x], ksw[x], c->q[r]);
      }
    orc_rescale(c, top, ct, o);
  } else {
    /* Algorithm 1 order: multiply, relinearise, rescale, then accumulate */
    for (int n = 0; n < nk; n++) {
      int k = ks[n];
      const u64* a = J->encA[(size_t)i * J->K + k];
      const u64* b = J->encB[(size_t)k * J->Nc + j];
      for (int r = 0; r < L; r++) {
        u64 q = c->q[r];
        const u64 *a0 = a + (size_t)r * N, *a1 = a + (size_t)(L + r) * N;
        const u64 *b0 = b + (size_t)r * N, *b1 = b + (size_t)(L + r) * N;
        u64 *d0 = d + (size_t)r * N, *d1 = d + (size_t)(L + r) * N, *d2 = d + (size_t)(2 * L + r) * N;
        for (int t = 0; t < N; t++) {
          d0[t] = mulm(a0[t], b0[t], q);
          d1[t] = addm(mulm(a0[t], b1[t], q), mulm(a1[t], b0[t], q), q);
          d2[t] = mulm(a1[t], b1[t], q);
        }
        ntt_inv(c, r, d0); ntt_inv(c, r, d1); ntt_inv(c, r, d2);
      }
      orc_keyswitch(c, top, d + (size_t)2 * L * N, ksw);
      for (int p = 0; p < 2; p++) for (int r = 0; r < L; r++)
        for (int t = 0; t < N; t++) {
          size_t x = ((size_t)p * L + r) * N + t;
          ct[x] = addm(d[x], ksw[x], c->q[r]);
        }
      orc_rescale(c, top, ct, rs);
      for (int p = 0; p < 2; p++) for (int r = 0; r < top; r++)
        for (int t = 0; t < N; t++) {
          size_t x = ((size_t)p * top + r) * N + t;
          o[x] = addm(o[x], rs[x], c->q[r]);
        }
    }
  }
  free(ks); free(d); free(ksw); free(ct); free(rs);
}

static void* mm_worker(void* arg) {
  const mm_job* J = arg;
  size_t ct_out = (size_t)2 * (J->c->L - 1) * J->c->N;
  for (int n = 0; n < J->nout; n++) {
    long idx = (long)J->orow[n] * J->Nc + J->ocol[n];     /* Sec. 3.4 assignment, linear index (reading) */
    if (idx % J->nthreads != J->tid) continue;
    mm_output(J, J->orow[n], J->ocol[n], J->out + (size_t)n * ct_out);
  }
  return NULL;
}

typedef struct { const orc_ctx* c; const double* vals; int ld; u64 seed, op; u64** slots; int rows, cols; int nthreads, tid; } enc_job;
static void* enc_worker(void* arg) {
  enc_job* E = arg;
  size_t ct_top = (size_t)2 * E->c->L * E->c->N;
  long cnt = 0;
  for (int i = 0; i < E->rows; i++) for (int j = 0; j < E->cols; j++) {
    size_t x = (size_t)i * E->cols + j;
    if (!E->slots[x]) continue;
    if ((cnt++) % E->nthreads != E->tid) continue;
    orc_encrypt(E->c, E->vals[(size_t)i * E->ld + j], E->seed, E->op, (u64)i, (u64)j, E->slots[x]);
    /* stored in the NTT domain, as an evaluation-form ciphertext */
    int L = E->c->L, N = E->c->N;
    for (int p = 0; p < 2; p++) for (int r = 0; r < L; r++) ntt_fwd(E->c, r, E->slots[x] + ((size_t)p * L + r) * N);
    (void)ct_top;
  }
  return NULL;
}
static void encrypt_marked(const orc_ctx* c, const double* vals, int rows, int cols, u64 seed, u64 op, u64** slots, int nthreads) {
  pthread_t th[256]; enc_job jobs[256];
  if (nthreads > 256) nthreads = 256;
  for (int t = 0; t < nthreads; t++) {
    jobs[t] = (enc_job){c, vals, cols, seed, op, slots, rows, cols, nthreads, t};
    pthread_create(&th[t], NULL, enc_worker, &jobs[t]);
  }
  for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
}

static double now_s(void) { struct timespec ts; clock_gettime(CLOCK_MONOTONIC, &ts); return ts.tv_sec + 1e-9 * ts.tv_nsec; }

/* Compute the listed outputs of C = A B, A (M x K) with encoding `enc`,
 * B (K x Nc) dense, both row-major fp64.  A is encrypted with (seedA, opA),
 * B with (seedB, opB), element (i, j) keyed by its coordinates.  out receives
 * [nout][2][L-1][N] coefficient-domain residues; vals (nullable) the decrypted
 * values; seconds (nullable) the wall time of the multiply stage only
 * (encryption and decryption excluded, Sec. 4.1). */
int orc_matmul2(const orc_ctx* c, const double* A, int M, int K, const double* B, int Nc,
                int enc, int enc_b, int sched, u64 seedA, u64 opA, u64 seedB, u64 opB,
                const int* orow, const int* ocol, int nout, int nthreads,
                u64* out, double* vals, double* seconds) {
  if (!c->has_keys || c->L < 2 || nthreads < 1) return -1;
  for (int n = 0; n < nout; n++) if (orow[n] < 0 || orow[n] >= M || ocol[n] < 0 || ocol[n] >= Nc) return -2;
  orc_struct S; struct_build(&S, A, M, K, enc);
  orc_struct SB; struct_build(&SB, B, K, Nc, enc_b);
  size_t ct_top = (size_t)2 * c->L * c->N;
  u64** encA = calloc((size_t)M * K, sizeof(u64*));
  u64** encB = calloc((size_t)K * Nc, sizeof(u64*));
  int* ks = malloc(sizeof(int) * (K + 1));
  for (int n = 0; n < nout; n++) {
    int nk = out_ks(&S, &SB, orow[n], ocol[n], ks);
    for (int x = 0; x < nk; x++) {
      size_t ia = (size_t)orow[n] * K + ks[x], ib = (size_t)ks[x] * Nc + ocol[n];
      if (!encA[ia]) encA[ia] = malloc(sizeof(u64) * ct_top);
      if (!encB[ib]) encB[ib] = malloc(sizeof(u64) * ct_top);
    }
  }
  free(ks);
  encrypt_marked(c, A, M, K, seedA, opA, encA, nthreads);
  encrypt_marked(c, B, K, Nc, seedB, opB, encB, nthreads);

  pthread_t th[256]; mm_job jobs[256];
  int T = nthreads > 256 ? 256 : nthreads;
  double t0 = now_s();
  for (int t = 0; t < T; t++) {
    jobs[t] = (mm_job){c, &S, &SB, M, K, Nc, sched, T, t, encA, encB, orow, ocol, nout, out};
    pthread_create(&th[t], NULL, mm_worker, &jobs[t]);
  }
  for (int t = 0; t < T; t++) pthread_join(th[t], NULL);
  double t1 = now_s();
  if (seconds) *seconds = t1 - t0;

  if (vals) {
    int top = c->L - 1;
    double scale = ldexp(1.0, 2 * (int)c->log2_scale) / (double)c->q[top];
    size_t ct_out = (size_t)2 * top * c->N;
    for (int n = 0; n < nout; n++) vals[n] = orc_decrypt(c, top - 1, out + (size_t)n * ct_out, scale);
  }
  for (size_t x = 0; x < (size_t)M * K; x++) free(encA[x]);
  for (size_t x = 0; x < (size_t)K * Nc; x++) free(encB[x]);
  free(encA); free(encB);
  struct_free(&S);
  struct_free(&SB);
  return 0;
}

/* the right operand dense (the hot path's configuration) */
int orc_matmul(const orc_ctx* c, const double* A, int M, int K, const double* B, int Nc,
               int enc, int sched, u64 seedA, u64 opA, u64 seedB, u64 opB,
               const int* orow, const int* ocol, int nout, int nthreads,
               u64* out, double* vals, double* seconds) {
  return orc_matmul2(c, A, M, K, B, Nc, enc, ORC_ENC_DENSE, sched, seedA, opA, seedB, opB, orow, ocol, nout, nthreads,
                     out, vals, seconds);
}

/* ------------------------------------------------------------------ */
/* plaintext weights times encrypted values (Sec. 3.3.2: a server that   */
/* holds the model weights in plaintext multiplies them into the         */
/* client's encrypted input)                                              */
/* ------------------------------------------------------------------ */
/* R8  a weight w is the constant polynomial m = nearbyint(w * 2^sw): a
 *     constant takes the same value at every root of X^N + 1, so it scales
 *     every slot by m, and multiplying a ciphertext by it multiplies both
 *     polys coefficient-wise by m (in either domain).  Returns -1 if the
 *     scaled weight does not fit 62 bits. */
int orc_weight(double w, double sw, i64* m) {
  double x = ldexp(w, (int)sw);
  if (sw != floor(sw) || !(fabs(x) < 4.0e18)) return -1;
  *m = (i64)nearbyint(x);
  return 0;
}

typedef struct {
  const orc_ctx* c;
  const orc_struct* S;
  const double* W;
  double sw;
  int K, Nc, nthreads, tid;
  u64** encB;
  const int* orow; const int* ocol; int nout;
  u64* out;
} pm_job;

/* C_ij = Rescale(sum over the visited k, ascending, of m_ik B_kj) */
static void pm_output(const pm_job* J, int i, int j, u64* o) {
  const orc_ctx* c = J->c;
  int N = c->N, L = c->L, top = L - 1;
  size_t ct_top = (size_t)2 * L * N, ct_out = (size_t)2 * top * N;
  int* ks = malloc(sizeof(int) * (J->K + 1));
  int nk = row_ks(J->S, i, ks);
  memset(o, 0, sizeof(u64) * ct_out);                       /* R6: trivial zero */
  if (nk == 0) { free(ks); return; }
  u64* acc = calloc(ct_top, sizeof(u64));
  for (int n = 0; n < nk; n++) {
    int k = ks[n];
    i64 m;
    orc_weight(J->W[(size_t)i * J->K + k], J->sw, &m);
    const u64* b = J->encB[(size_t)k * J->Nc + j];
    for (int p = 0; p < 2; p++)
      for (int r = 0; r < L; r++) {
        u64 q = c->q[r], mq = redi(m, q);
        const u64* bb = b + ((size_t)p * L + r) * N;
        u64* aa = acc + ((size_t)p * L + r) * N;
        for (int t = 0; t < N; t++) aa[t] = addm(aa[t], mulm(mq, bb[t], q), q);
      }
  }
  for (int p = 0; p < 2; p++) for (int r = 0; r < L; r++) ntt_inv(c, r, acc + ((size_t)p * L + r) * N);
  orc_rescale(c, top, acc, o);
  free(ks); free(acc);
}

static void* pm_worker(void* arg) {
  const pm_job* J = arg;
  size_t ct_out = (size_t)2 * (J->c->L - 1) * J->c->N;
  for (int n = 0; n < J->nout; n++) {
    long idx = (long)J->orow[n] * J->Nc + J->ocol[n];
    if (idx % J->nthreads != J->tid) continue;
    pm_output(J, J->orow[n], J->ocol[n], J->out + (size_t)n * ct_out);
  }
  return NULL;
}

/* Listed outputs of C = W B with W (M x K) plaintext weights stored with
 * encoding `enc` and scaled by 2^sw (R8), B (K x Nc) dense and encrypted with
 * (seedB, opB).  out receives [nout][2][L-1][N] coefficient-domain residues,
 * vals (nullable) the values decrypted at scale 2^sw * Delta / q_{L-1},
 * seconds (nullable) the wall time of the multiply stage. */
int orc_matmul_plain(const orc_ctx* c, const double* W, int M, int K, const double* B, int Nc, int enc, double sw,
                     u64 seedB, u64 opB, const int* orow, const int* ocol, int nout, int nthreads,
                     u64* out, double* vals, double* seconds) {
  if (!c->has_keys || c->L < 2 || nthreads < 1) return -1;
  for (int n = 0; n < nout; n++) if (orow[n] < 0 || orow[n] >= M || ocol[n] < 0 || ocol[n] >= Nc) return -2;
  for (size_t x = 0; x < (size_t)M * K; x++) { i64 m; if (W[x] != 0.0 && orc_weight(W[x], sw, &m)) return -3; }
  orc_struct S; struct_build(&S, W, M, K, enc);
  size_t ct_top = (size_t)2 * c->L * c->N;
  u64** encB = calloc((size_t)K * Nc, sizeof(u64*));
  int* ks = malloc(sizeof(int) * (K + 1));
  for (int n = 0; n < nout; n++) {
    int nk = row_ks(&S, orow[n], ks);
    for (int x = 0; x < nk; x++) {
      size_t ib = (size_t)ks[x] * Nc + ocol[n];
      if (!encB[ib]) encB[ib] = malloc(sizeof(u64) * ct_top);
    }
  }
  free(ks);
  encrypt_marked(c, B, K, Nc, seedB, opB, encB, nthreads);

  pthread_t th[256]; pm_job jobs[256];
  int T = nthreads > 256 ? 256 : nthreads;
  double t0 = now_s();
  for (int t = 0; t < T; t++) {
    jobs[t] = (pm_job){c, &S, W, sw, K, Nc, T, t, encB, orow, ocol, nout, out};
    pthread_create(&th[t], NULL, pm_worker, &jobs[t]);
  }
  for (int t = 0; t < T; t++) pthread_join(th[t], NULL);
  double t1 = now_s();
  if (seconds) *seconds = t1 - t0;

  if (vals) {
    int top = c->L - 1;
    double scale = ldexp(1.0, (int)sw + (int)c->log2_scale) / (double)c->q[top];
    size_t ct_out = (size_t)2 * top * c->N;
    for (int n = 0; n < nout; n++) vals[n] = orc_decrypt(c, top - 1, out + (size_t)n * ct_out, scale);
  }
  for (size_t x = 0; x < (size_t)K * Nc; x++) free(encB[x]);
  free(encB);
  struct_free(&S);
  return 0;
}

/* ------------------------------------------------------------------ */
/* chunks of several values per ciphertext (Sec. 3.2) and Algorithm 1   */
/* with its rotations and slot-zero mask (Sec. 3.3.1)                   */
/* ------------------------------------------------------------------ */
/* R10 slot j of a ciphertext is its plaintext's value at zeta^(5^j),
 *     zeta = exp(i pi / N).  Real values z_0..z_{n-1} in slots 0..n-1 are the
 *     polynomial m_t = nearbyint(sum_j z_j 2 Delta / N cos(pi (5^j t mod 2N) / N)),
 *     summed in j order (n = 1 is R1's encoding).  A rotation by r (slot j
 *     receives slot j + r, indices mod N/2) applies X -> X^g, g = 5^r mod 2N,
 *     to both polys and switches c1(X^g) from s(X^g) back to s with a key
 *     built like the relinearisation key (target s(X^g) for s^2; randomness
 *     tags 6 and 7 with fields (g, j[, r])).  The slot-zero mask is the
 *     plaintext encoding 1.0 in slot 0 (R1) at scale Delta. */

/* 5^r mod 2N for any integer r (5 has order N/2 modulo 2N) */
u64 orc_galois(const orc_ctx* c, long r) {
  long h = c->N / 2;
  long e = ((r % h) + h) % h;
  u64 g = 1, m = 2 * (u64)c->N;
  for (long x = 0; x < e; x++) g = (g * 5) % m;
  return g;
}

/* cos(pi e / N) for 0 <= e < 2N from the host libm table (sign flip above N) */
static double cos2n(const orc_ctx* c, u64 e) { return e < (u64)c->N ? c->cosv[e] : -c->cosv[e - c->N]; }

int orc_encode_slots(const orc_ctx* c, const double* z, int n, i64* m) {
  double sz[64];
  u64 g[64], m2 = 2 * (u64)c->N;
  if (n < 1 || n > 64 || n > c->N / 2) return -1;
  for (int j = 0; j < n; j++) {
    sz[j] = ldexp(z[j], (int)c->log2_scale + 1 - c->logN);
    if (!(fabs(sz[j]) < 4.0e18 / n)) return -1;
    g[j] = orc_galois(c, j);
  }
  for (int t = 0; t < c->N; t++) {
    double acc = 0.0;
    for (int j = 0; j < n; j++) acc += sz[j] * cos2n(c, (g[j] * (u64)t) % m2);
    m[t] = (i64)nearbyint(acc);
  }
  return 0;
}

/* slot `slot` of the plaintext m[lev+1][N] (coefficient domain) at `scale` */
double orc_decode_slot(const orc_ctx* c, int lev, const u64* m, double scale, int slot) {
  u64 g = orc_galois(c, slot), m2 = 2 * (u64)c->N;
  long double s = 0.0L;
  for (int t = 0; t < c->N; t++) s += crt_centered(c, lev + 1, m + t, c->N) * (long double)cos2n(c, (g * (u64)t) % m2);
  return (double)(s / (long double)scale);
}
double orc_decrypt_slot(const orc_ctx* c, int lev, const u64* ct, double scale, int slot) {
  u64* m = malloc(sizeof(u64) * (size_t)(lev + 1) * c->N);
  orc_decrypt_poly(c, lev, ct, m);
  double v = orc_decode_slot(c, lev, m, scale, slot);
  free(m);
  return v;
}

/* X -> X^g on nl rows a[nl][N] (coefficient domain): X^(g t) = -X^(g t - N) above N */
void orc_automorphism(const orc_ctx* c, int nl, const u64* a, u64 g, u64* out) {
  int N = c->N;
  u64 m2 = 2 * (u64)N;
  for (int r = 0; r < nl; r++) {
    u64 q = c->q[r];
    const u64* ar = a + (size_t)r * N;
    u64* o = out + (size_t)r * N;
    for (int t = 0; t < N; t++) {
      u64 e = (g * (u64)t) % m2;
      if (e < (u64)N) o[e] = ar[t];
      else o[e - N] = ar[t] ? q - ar[t] : 0;
    }
  }
}

/* the rotation key for g: [dnum][2][nb][N] coefficient domain, digit j =
 * (-a_j s + e_j + gadget_j s(X^g), a_j) over Q u P; errors to e_out[dnum][N] */
void orc_rotkey(const orc_ctx* c, u64 g, u64* key, i64* e_out) {
  int N = c->N, nb = c->nb;
  u64* sr = malloc(sizeof(u64) * N);
  u64* sg = malloc(sizeof(u64) * N);
  u64* as = malloc(sizeof(u64) * N);
  i64* e = malloc(sizeof(i64) * N);
  for (int j = 0; j < c->dnum; j++) {
    u64 fe[2] = {g, (u64)j};
    u64 ke = key_of(c->seed, TAG_ROT_E, 2, fe);
    for (int t = 0; t < N; t++) { e[t] = cdt_sample(c->cdt, word(ke, t)); if (e_out) e_out[(size_t)j * N + t] = e[t]; }
    for (int r = 0; r < nb; r++) {
      u64 q = c->q[r];
      u64* b = key + (((size_t)j * 2 + 0) * nb + r) * N;
      u64* a = key + (((size_t)j * 2 + 1) * nb + r) * N;
      u64 fa[3] = {g, (u64)j, (u64)r};
      u64 ka = key_of(c->seed, TAG_ROT_A, 3, fa);
      for (int t = 0; t < N; t++) a[t] = uniform_at(ka, t, q);
      for (int t = 0; t < N; t++) sr[t] = redi(c->s[t], q);
      polymul(c, r, a, sr, as);
      /* s(X^g) on this prime */
      u64 m2 = 2 * (u64)N;
      for (int t = 0; t < N; t++) {
        u64 ex = (g * (u64)t) % m2;
        if (ex < (u64)N) sg[ex] = sr[t];
        else sg[ex - N] = sr[t] ? q - sr[t] : 0;
      }
      u64 gd = 0;
      if (r >= digit_lo(c, j) && r < digit_hi(c, j)) {
        gd = 1;
        for (int k = c->L; k < nb; k++) gd = mulm(gd, c->q[k] % q, q);
      }
      for (int t = 0; t < N; t++) b[t] = addm(subm(redi(e[t], q), as[t], q), mulm(gd, sg[t], q), q);
    }
  }
  free(sr); free(sg); free(as); free(e);
}

/* rotation by r of ct[2][lev+1][N] (coefficient domain) with key_ntt the
 * rotation key of g = 5^r (NTT domain) */
static void rotate_with(const orc_ctx* c, int lev, const u64* ct, u64 g, const u64* key_ntt, u64* out) {
  int N = c->N, nl = lev + 1;
  u64* t = malloc(sizeof(u64) * (size_t)2 * nl * N);
  u64* ks = malloc(sizeof(u64) * (size_t)2 * nl * N);
  orc_automorphism(c, nl, ct, g, t);
  orc_automorphism(c, nl, ct + (size_t)nl * N, g, t + (size_t)nl * N);
  ks_with(c, lev, t + (size_t)nl * N, key_ntt, ks);
  for (int p = 0; p < 2; p++)
    for (int r = 0; r < nl; r++)
      for (int x = 0; x < N; x++) {
        size_t i = ((size_t)p * nl + r) * N + x;
        out[i] = p == 0 ? addm(t[i], ks[i], c->q[r]) : ks[i];
      }
  free(t); free(ks);
}
static u64* rotkey_ntt(const orc_ctx* c, u64 g) {
  size_t kn = (size_t)c->dnum * 2 * c->nb * c->N;
  u64* k = malloc(sizeof(u64) * kn);
  orc_rotkey(c, g, k, NULL);
  for (int j = 0; j < c->dnum; j++)
    for (int p = 0; p < 2; p++)
      for (int r = 0; r < c->nb; r++) ntt_fwd(c, r, k + (((size_t)j * 2 + p) * c->nb + r) * c->N);
  return k;
}
int orc_rotate(const orc_ctx* c, int lev, const u64* ct, long r, u64* out) {
  if (!c->has_keys) return -1;
  u64 g = orc_galois(c, r);
  u64* k = rotkey_ntt(c, g);
  rotate_with(c, lev, ct, g, k, out);
  free(k);
  return 0;
}

/* encryption of the values z[0..n-1] in slots 0..n-1 (R2, R10), keyed by
 * (operand, chunk, 2^40 + n) */
int orc_encrypt_slots(const orc_ctx* c, const double* z, int n, u64 seed, u64 operand, u64 chunk, u64* ct) {
  int N = c->N, L = c->L;
  i64* m = malloc(sizeof(i64) * N);
  i64* e = malloc(sizeof(i64) * N);
  u64* sr = malloc(sizeof(u64) * N);
  u64* as = malloc(sizeof(u64) * N);
  if (orc_encode_slots(c, z, n, m) != 0) { free(m); free(e); free(sr); free(as); return -1; }
  u64 jf = ((u64)1 << 40) + (u64)n;
  orc_enc_error(c, seed, operand, chunk, jf, e);
  for (int r = 0; r < L; r++) {
    u64 q = c->q[r];
    u64* c0 = ct + (size_t)r * N;
    u64* c1 = ct + (size_t)(L + r) * N;
    u64 f[4] = {operand, chunk, jf, (u64)r};
    u64 ka = key_of(seed, TAG_ENC_A, 4, f);
    for (int t = 0; t < N; t++) c1[t] = uniform_at(ka, t, q);
    for (int t = 0; t < N; t++) sr[t] = redi(c->s[t], q);
    polymul(c, r, c1, sr, as);
    for (int t = 0; t < N; t++) c0[t] = subm(addm(redi(e[t], q), redi(m[t], q), q), as[t], q);
  }
  free(m); free(e); free(sr); free(as);
  return 0;
}

/* the stored value list of an encoding (R10: chunks of c consecutive stored
 * values): dense and naive sparse store all rows x cols, CSR the nonzeros in
 * row order, ELLPACK rows x width (pads hold 0); slot_of = index of (i, k) */
static long stored_slot(const orc_struct* S, int i, int k) {
  switch (S->enc) {
    case ORC_ENC_DENSE: case ORC_ENC_NAIVE: return (long)i * S->K + k;
    case ORC_ENC_CSR:
      for (int p = S->row_ptr[i]; p < S->row_ptr[i + 1]; p++) if (S->col_idx[p] == k) return p;
      return -1;
    case ORC_ENC_ELL:
      for (int s = 0; s < S->ell_w; s++) if (S->ell_col[(size_t)i * S->ell_w + s] == k) return (long)i * S->ell_w + s;
      return -1;
  }
  return -1;
}
static long stored_count(const orc_struct* S) {
  switch (S->enc) {
    case ORC_ENC_DENSE: case ORC_ENC_NAIVE: return (long)S->M * S->K;
    case ORC_ENC_CSR: return S->row_ptr[S->M];
    case ORC_ENC_ELL: return (long)S->M * S->ell_w;
  }
  return 0;
}
static void stored_values(const orc_struct* S, const double* A, double* v) {
  long n = stored_count(S);
  for (long x = 0; x < n; x++) v[x] = 0.0;
  for (int i = 0; i < S->M; i++)
    for (int k = 0; k < S->K; k++) {
      long sl = stored_slot(S, i, k);
      if (sl >= 0) v[sl] = A[(size_t)i * S->K + k];
    }
}

/* Algorithm 1 at chunk size cs (Sec. 3.2, 3.3) for the outputs listed: per
 * output (i, j), for every k that row i visits, the A and B values are
 * rotated into slot 0, multiplied, relinearised and rescaled; then (per
 * product for PER_PRODUCT, once on the sum for LAZY) multiplied by the
 * slot-zero mask, rescaled, rotated to the output's slot and added into its
 * output chunk.  out receives the result chunks touched, [nchunks][2][L-3][N]
 * coefficient domain (chunks of the outputs not listed stay trivial zeros);
 * vals (nullable) the listed outputs decrypted at Delta^3 / (q_{L-1} q_{L-2}). */
int orc_matmul_chunked(const orc_ctx* c, const double* A, int M, int K, const double* B, int Nc, int enc, int sched,
                       int cs, u64 seedA, u64 opA, u64 seedB, u64 opB, const int* orow, const int* ocol, int nout,
                       u64* out, double* vals) {
  int N = c->N, L = c->L, top = L - 1, lo = L - 3;
  if (!c->has_keys || L < 4 || cs < 1 || cs > 64 || cs > N / 2) return -1;
  orc_struct S; struct_build(&S, A, M, K, enc);
  orc_struct SB; struct_build(&SB, B, K, Nc, ORC_ENC_DENSE);
  long na = stored_count(&S), nbv = (long)K * Nc;
  double* av = malloc(sizeof(double) * (na + 1));
  double* bv = malloc(sizeof(double) * (nbv + 1));
  stored_values(&S, A, av);
  stored_values(&SB, B, bv);
  long nca = (na + cs - 1) / cs, ncb = (nbv + cs - 1) / cs, ncr = ((long)M * Nc + cs - 1) / cs;
  size_t ct_top = (size_t)2 * L * N, ct_lo = (size_t)2 * (lo + 1) * N;
  u64** ea = calloc(nca + 1, sizeof(u64*));
  u64** eb = calloc(ncb + 1, sizeof(u64*));
  memset(out, 0, sizeof(u64) * ncr * ct_lo);
  /* rotation keys for offsets -(cs-1) .. cs-1 */
  u64* keys[129] = {0};
  for (long r = -(cs - 1); r <= cs - 1; r++) if (r) keys[r + 64] = rotkey_ntt(c, orc_galois(c, r));
  /* the slot-zero mask */
  i64* mk = malloc(sizeof(i64) * N);
  orc_encode(c, 1.0, mk);
  u64* mask = malloc(sizeof(u64) * (size_t)L * N);
  for (int r = 0; r < L; r++) for (int t = 0; t < N; t++) mask[(size_t)r * N + t] = redi(mk[t], c->q[r]);
  u64* ra = malloc(sizeof(u64) * ct_top);
  u64* rb = malloc(sizeof(u64) * ct_top);
  u64* d = malloc(sizeof(u64) * 3 * L * N);
  u64* dsum = malloc(sizeof(u64) * 3 * L * N);
  u64* ks = malloc(sizeof(u64) * ct_top);
  u64* x1 = malloc(sizeof(u64) * ct_top);
  u64* x2 = malloc(sizeof(u64) * ct_top);
  u64* x3 = malloc(sizeof(u64) * ct_top);
  u64* tmp = malloc(sizeof(u64) * N);
  int* ks_k = malloc(sizeof(int) * (K + 1));
  int rc = 0;
  /* mask, rescale, rotate to the output slot and add: x holds a relinearised
   * product at level top - 1 */
  #define FINISH(x, rn, roff) do {                                                        \
    int l1 = top - 1;                                                                        \
    for (int p = 0; p < 2; p++) for (int r = 0; r <= l1; r++) {                              \
      polymul(c, r, (x) + ((size_t)p * (l1 + 1) + r) * N, mask + (size_t)r * N, tmp);       \
      memcpy((x) + ((size_t)p * (l1 + 1) + r) * N, tmp, sizeof(u64) * N);                   \
    }                                                                                        \
    orc_rescale(c, l1, (x), x3);                                                             \
    if (roff) rotate_with(c, lo, x3, orc_galois(c, -(long)(roff)), keys[64 - (roff)], x2);   \
    else memcpy(x2, x3, sizeof(u64) * ct_lo);                                                \
    u64* o = out + (size_t)(rn) * ct_lo;                                                     \
    for (int p = 0; p < 2; p++) for (int r = 0; r <= lo; r++) for (int t = 0; t < N; t++) {  \
      size_t ix = ((size_t)p * (lo + 1) + r) * N + t;                                        \
      o[ix] = addm(o[ix], x2[ix], c->q[r]);                                                  \
    }                                                                                        \
  } while (0)
  for (int n = 0; n < nout && !rc; n++) {
    int i = orow[n], j = ocol[n];
    long rs = (long)i * Nc + j, rn = rs / cs;
    int roff = (int)(rs % cs);
    int nk = row_ks(&S, i, ks_k);
    if (nk == 0) continue;                                 /* R6: nothing added */
    memset(dsum, 0, sizeof(u64) * 3 * L * N);
    for (int x = 0; x < nk; x++) {
      int k = ks_k[x];
      long sa = stored_slot(&S, i, k), sb = (long)k * Nc + j;
      long an = sa / cs, bn = sb / cs;
      int aoff = (int)(sa % cs), boff = (int)(sb % cs);
      if (!ea[an]) {
        ea[an] = malloc(sizeof(u64) * ct_top);
        int cnt = (int)((an + 1) * cs <= na ? cs : na - an * cs);
        orc_encrypt_slots(c, av + an * cs, cnt, seedA, opA, (u64)an, ea[an]);
      }
      if (!eb[bn]) {
        eb[bn] = malloc(sizeof(u64) * ct_top);
        int cnt = (int)((bn + 1) * cs <= nbv ? cs : nbv - bn * cs);
        orc_encrypt_slots(c, bv + bn * cs, cnt, seedB, opB, (u64)bn, eb[bn]);
      }
      if (aoff) rotate_with(c, top, ea[an], orc_galois(c, aoff), keys[64 + aoff], ra); else memcpy(ra, ea[an], sizeof(u64) * ct_top);
      if (boff) rotate_with(c, top, eb[bn], orc_galois(c, boff), keys[64 + boff], rb); else memcpy(rb, eb[bn], sizeof(u64) * ct_top);
      orc_tensor(c, top, ra, rb, d);
      if (sched == ORC_SCHED_LAZY) {
        for (size_t y = 0; y < (size_t)3 * L * N; y++) dsum[y] = addm(dsum[y], d[y], c->q[(y / N) % L]);
        continue;
      }
      /* PER_PRODUCT (Algorithm 1's order) */
      orc_keyswitch(c, top, d + (size_t)2 * L * N, ks);
      for (int p = 0; p < 2; p++) for (int r = 0; r < L; r++) for (int t = 0; t < N; t++) {
        size_t ix = ((size_t)p * L + r) * N + t;
        x1[ix] = addm(d[ix], ks[ix], c->q[r]);
      }
      orc_rescale(c, top, x1, x2);
      memcpy(x1, x2, sizeof(u64) * 2 * (size_t)top * N);
      FINISH(x1, rn, roff);
    }
    if (sched == ORC_SCHED_LAZY) {
      orc_keyswitch(c, top, dsum + (size_t)2 * L * N, ks);
      for (int p = 0; p < 2; p++) for (int r = 0; r < L; r++) for (int t = 0; t < N; t++) {
        size_t ix = ((size_t)p * L + r) * N + t;
        x1[ix] = addm(dsum[ix], ks[ix], c->q[r]);
      }
      orc_rescale(c, top, x1, x2);
      memcpy(x1, x2, sizeof(u64) * 2 * (size_t)top * N);
      FINISH(x1, rn, roff);
    }
  }
  #undef FINISH
  if (vals) {
    double scale = ldexp(1.0, 3 * (int)c->log2_scale) / (double)c->q[top] / (double)c->q[top - 1];
    for (int n = 0; n < nout; n++) {
      long rs = (long)orow[n] * Nc + ocol[n];
      vals[n] = orc_decrypt_slot(c, lo, out + (size_t)(rs / cs) * ct_lo, scale, (int)(rs % cs));
    }
  }
  for (long x = 0; x < nca; x++) free(ea[x]);
  for (long x = 0; x < ncb; x++) free(eb[x]);
  for (int x = 0; x < 129; x++) free(keys[x]);
  free(ea); free(eb); free(av); free(bv); free(mk); free(mask); free(ra); free(rb); free(d); free(dsum); free(ks);
  free(x1); free(x2); free(x3); free(tmp); free(ks_k);
  struct_free(&S); struct_free(&SB);
  return rc;
}
