// internal.hpp -- host-side runtime structures and kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "../../include/sfhe.h"
#include "device.hpp"

namespace sfhe {

constexpr int kMaxDigit = 8;   // primes per key-switching digit (alpha)

// NTT designs: the register transform of the 2^14 kernels (N >= 2^14), and
// the LDS transform with radix-16, radix-8 or radix-4 passes (N <= 2^14)
enum { kNttRegister = 0, kNttRadix16 = 1, kNttRadix8 = 2, kNttRadix4 = 3 };

// ---- constants of the base conversions, one block per (level, digit) ----
// ModUp of digit j at level lev: y_i = [x_i (D/q_i)^-1]_{q_i} for the digit's
// primes, taken in (-q_i/2, q_i/2), then target e of the extended basis (data
// 0..lev, then special) gets sum_i y_i [D/q_i]_{e}: the uncentered sum minus
// c [D]_e, c the count of y_i above (q_i - 1) / 2.
struct ModUpConst {
  int lo, hi;                          // digit primes lo..hi-1 (clipped to the level)
  int ne;                              // extended basis size = lev + 1 + alpha
  int basis[kMaxBasis];                // basis index of extended position e
  u64 inv[kMaxDigit], inv_s[kMaxDigit];
  u64 inv_n[kMaxDigit], inv_n_s[kMaxDigit];   // inv * N^-1 mod q_i (applied with an inverse NTT)
  u64 conv[kMaxDigit][kMaxBasis], conv_s[kMaxDigit][kMaxBasis];
  u64 dmod[kMaxBasis], dmod_s[kMaxBasis];     // [D]_e and its Shoup companion
};
// ModDown at level lev: y_k = [acc_{p_k} (P/p_k)^-1]_{p_k} taken in
// (-p_k/2, p_k/2) (the centered conversion: y_k above (p_k - 1)/2 stands for
// y_k - p_k); out_i = (acc_i - sum_k y_k [P/p_k]_{q_i}) [P^-1]_{q_i}, i.e. the
// uncentered sum minus c [P]_{q_i}, c the count of such y_k, before the
// product with P^-1 (or c added after it).
struct ModDownConst {
  u64 pinv[kMaxDigit], pinv_s[kMaxDigit];            // (P/p_k)^-1 mod p_k
  u64 pinv_n[kMaxDigit], pinv_n_s[kMaxDigit];        // (P/p_k)^-1 N^-1 mod p_k
  u64 conv[kMaxDigit][kMaxBasis], conv_s[kMaxDigit][kMaxBasis];   // [P/p_k]_{q_i}
  u64 convp[kMaxDigit][kMaxBasis], convp_s[kMaxDigit][kMaxBasis]; // [P/p_k]_{q_i} P^-1 mod q_i
  u64 Pinv[kMaxBasis], Pinv_s[kMaxBasis];            // P^-1 mod q_i
  u64 Pq[kMaxBasis];                                 // P mod q_i
};
// Rescale at level lev: q_lev^-1 mod q_i for i < lev.
struct RescaleConst {
  u64 qinv[kMaxBasis], qinv_s[kMaxBasis];
};

// ---- device allocation through the optional hooks ----
// Allocation is stream-ordered: a block is taken on the stream of the call in
// progress (`cur`, set by StreamScope at each entry point) and given back on
// the stream it was taken on, once the last launch that uses it has been
// enqueued there.  The allocator may hand a freed block to later work on that
// stream at once; stream order keeps that work behind the earlier launches.
// Without hooks the blocks come from a stream-ordered pool of the context
// (hipMallocFromPoolAsync / hipFreeAsync), so no free waits for the device.
struct Alloc {
  sfhe_device_hooks hooks{};
  bool has_hooks = false;
  hipMemPool_t pool = nullptr;
  hipStream_t cur = nullptr;
  void* get(size_t bytes);
  void put(void* p, size_t bytes, hipStream_t s);
};

// sets the stream that allocations of the enclosing call are ordered on
struct StreamScope {
  Alloc& a;
  hipStream_t prev;
  StreamScope(Alloc& al, hipStream_t s) : a(al), prev(al.cur) { a.cur = s; }
  ~StreamScope() { a.cur = prev; }
  StreamScope(const StreamScope&) = delete;
  StreamScope& operator=(const StreamScope&) = delete;
};

template <typename T>
struct DevBuf {
  Alloc* al = nullptr;
  T* ptr = nullptr;
  size_t count = 0;
  hipStream_t st = nullptr;   // the stream the block was taken on
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept { *this = std::move(o); }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      al = o.al; ptr = o.ptr; count = o.count; st = o.st;
      o.ptr = nullptr; o.count = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  bool alloc(Alloc* a, size_t n) {
    release();
    al = a;
    count = n;
    st = a->cur;
    ptr = n ? (T*)a->get(n * sizeof(T)) : nullptr;
    return n == 0 || ptr != nullptr;
  }
  void release() {
    if (ptr && al) al->put(ptr, count * sizeof(T), st);
    ptr = nullptr;
    count = 0;
  }
};

}  // namespace sfhe

struct sfhe_ctx {
  // parameters
  int logN = 0, N = 0, L = 0, alpha = 0, dnum = 0, nb = 0;
  double log2_scale = 0, sigma = 0;
  std::vector<sfhe::u64> primes;         // data then special
  sfhe::DevParams dp{};                  // per-prime constants + table pointers
  sfhe::Alloc alloc;
  int device = 0;
  // device tables
  sfhe::DevBuf<sfhe::u64> d_tables;      // [nb][4][N]: tw, tws, itw, itws
  sfhe::DevBuf<double> d_tables_d;       // [nb][2][N]: tw, itw as doubles
  // N = 2^15: the halves' twiddle tables (see build_tables)
  sfhe::DevBuf<sfhe::u64> d_sub, d_sub_s;
  sfhe::DevBuf<double> d_sub_d;
  sfhe::DevBuf<double> d_cos;            // cos(pi t / N)
  sfhe::DevBuf<sfhe::ModUpConst> d_modup;      // [L][dnum]
  sfhe::DevBuf<sfhe::ModDownConst> d_moddown;  // [L]
  sfhe::DevBuf<sfhe::RescaleConst> d_rescale;  // [L]
  sfhe::u64 cdt[sfhe::kCdtLen];
  // NTT design per direction (0 forward, 1 inverse): one of sfhe::kNtt*,
  // chosen by measurement when the context is made (tuned) and in use (var);
  // ntt_us: measured microseconds per row of each design, -1 where it does
  // not apply to the ring
  int ntt_var[2] = {0, 0}, ntt_tuned[2] = {0, 0};
  double ntt_us[2][4] = {{-1, -1, -1, -1}, {-1, -1, -1, -1}};
  // outputs per fused key-switch launch group (N = 2^14): in use (0 = tune
  // at the next LAZY product), as tuned, and the microseconds per output
  // measured for each candidate (-1: not measured)
  int ks_slice = 0, ks_tuned_slice = 0;
  double ks_us[6] = {-1, -1, -1, -1, -1, -1};
  hipEvent_t tune_ev0 = nullptr, tune_ev1 = nullptr;
  // key switching on one stream or on two side streams (forked from and
  // joined into the call's stream): in use, as tuned, the two-stream slices
  // measured and their microseconds per output
  int ks_streams = 1, ks_tuned_streams = 1;
  int64_t ks_s2[2] = {0, 0};
  double ks_us2[2] = {-1, -1};
  hipStream_t ks_side[2] = {nullptr, nullptr};
  hipEvent_t ks_fork = nullptr, ks_join[2] = {nullptr, nullptr};
  // keys
  bool has_keys = false;
  sfhe::DevBuf<sfhe::u64> d_s;           // secret, NTT domain [nb][N]
  sfhe::DevBuf<sfhe::u64> d_rlk;         // relinearisation key, NTT domain [dnum][2][nb][N]
  sfhe::DevBuf<sfhe::u64> d_rlk_s;       // its Shoup companions floor(k 2^64 / q), same layout
  // last matmul
  sfhe_stats stats{};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool stats_pending = false;
  // per-step timing: event pairs (start, stop) with a category each
  bool profiling = false;
  std::vector<hipEvent_t> prof_pool;
  size_t prof_used = 0;
  std::vector<int> prof_cat;
  hipEvent_t prof_event();
  // several values per ciphertext (rotate.hip): the key seed, then per Galois
  // element g its NTT-domain automorphism table and rotation key, built on
  // first use; 5^j mod 2N for j < 64; the slot-zero mask, NTT domain [L][N]
  sfhe::u64 key_seed = 0;
  std::map<sfhe::u64, sfhe::DevBuf<int>> auto_perm;
  std::map<sfhe::u64, sfhe::DevBuf<sfhe::u64>> rot_keys, rot_keys_s;   // keys and their Shoup companions
  sfhe::DevBuf<sfhe::u64> d_gal, d_mask0;
};

struct sfhe_mat {
  sfhe_ctx* ctx = nullptr;
  int rows = 0, cols = 0, level = 0;
  double scale = 0;
  sfhe_encoding enc = SFHE_ENC_DENSE;
  int64_t n_ct = 0, nnz = 0;
  sfhe::DevBuf<sfhe::u64> data;          // chunked layout (see chunk_index), NTT domain
  // plaintext structure (Sec. 3.3.2), host and device copies
  std::vector<int> row_ptr, col_idx;     // CSR
  int ell_w = 0;
  std::vector<int> ell_col;              // ELL [rows][ell_w], -1 = padding
  std::vector<uint32_t> zero_mask;       // naive sparse: bit (i*cols + k) set iff A_ik == 0
  sfhe::DevBuf<int> d_row_ptr, d_col_idx, d_ell_col;
  sfhe::DevBuf<uint32_t> d_mask;
  // plaintext weights (sfhe_encode_matrix): no ciphertexts; the residue of
  // each stored weight per data prime, host side, [n_ct][L]
  bool plain = false;
  std::vector<uint64_t> w_res;
  // and its tile tables on the device (the layout of PlainJob's)
  int64_t w_pairs = 0;                   // stored weights outside ELL padding
  sfhe::DevBuf<int> d_tstart, d_ek, d_emask;
  sfhe::DevBuf<sfhe::u64> d_ew, d_ews;
  // several values per ciphertext (Sec. 3.2): stored value v sits in slot
  // v mod slots of ciphertext v / slots; n_ct = ceil(n_vals / slots)
  int slots = 1;
  int64_t n_vals = 0;
};

namespace sfhe {

// candidate key-switch slices (outputs per launch group) and the smallest
// product whose first batch is large enough to tune on
constexpr int64_t kKsCandidates[6] = {128, 256, 512, 1024, 2048, 4096};
constexpr int kKsNumCandidates = 6;
constexpr int64_t kKsTuneMin = 1024;

// Storage layout of an encrypted matrix: residue t of poly p (0, 1) of prime
// i of stored ciphertext e sits at ((i * (N/64) + t/64) * 2 + p) * n_ct * 64
// + e * 64 + t % 64.  For one prime and one 64-coefficient chunk every
// ciphertext of the matrix is contiguous (n_ct * 1 KiB), so the tensor
// kernel's working set for a chunk is one contiguous region instead of one
// page per ciphertext; a 64-lane wavefront still reads 512 contiguous bytes.
__host__ __device__ __forceinline__ int64_t chunk_index(int64_t e, int p, int i, int t, int64_t n_ct, int nchunk) {
  return (((int64_t)i * nchunk + (t >> 6)) * 2 + p) * n_ct * 64 + e * 64 + (t & 63);
}

// ---- errors ----
void set_error(const std::string& msg);
#define SFHE_HIP(call)                                                               \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) {                                                          \
      ::sfhe::set_error(std::string(#call) + ": " + hipGetErrorString(e_));          \
      return SFHE_E_DEVICE;                                                          \
    }                                                                                \
  } while (0)

// ---- launchers (each returns SFHE_OK or an error code) ----
// NTT of `batch` groups of `nrow` rows: row r of group b starts at
// base + b*bstride + pos[r]*N and is reduced mod basis prime prime[r].
int launch_ntt(const sfhe_ctx* c, u64* base, int64_t batch, int64_t bstride, int nrow, const int* pos,
               const int* prime, bool inverse, hipStream_t s);

// fill n words with zero
int launch_zero(u64* p, int64_t n, hipStream_t s);

// coefficient-domain parts of `count` elements (coordinates ei, ej, values z):
// tmp[x][2][L][N] = (e + m, a)
int encrypt_elements(sfhe_ctx* c, u64* tmp, int64_t count, const int* d_ei, const int* d_ej,
                     const double* d_z, u64 seed, u64 operand, hipStream_t s);
// NTT of every row of tmp[count][2][L][N], then c0 <- c0 - c1 s
int encrypt_finish(sfhe_ctx* c, u64* tmp, int64_t count, hipStream_t s);
// layout conversions between limb-major rows src[x * sstride + (p * nl + i) * N + t]
// and the chunked matrix layout, element elem[x] (or elem_base + x when elem is NULL)
int launch_to_chunked(const sfhe_ctx* c, const u64* src, int64_t sstride, int nl, int64_t count, u64* dst,
                      int64_t n_ct, const int64_t* elem, int64_t elem_base, hipStream_t s);
int launch_from_chunked(const sfhe_ctx* c, const u64* src, int64_t n_ct, int nl, int64_t count, const int64_t* elem,
                        int64_t elem_base, u64* dst, int64_t dstride, hipStream_t s);
int keygen_device(sfhe_ctx* c, u64 seed, hipStream_t s);
// decrypt + decode: value v = e slots + j (slot j of ciphertext e, v < nvals)
// for every ciphertext of a chunked matrix at level lev
int decrypt_values(sfhe_ctx* c, const u64* data, int64_t n_ct, int lev, double scale, double* d_out, int* d_flag,
                   hipStream_t s, int slots = 1, int64_t nvals = -1);

// tensor products
int launch_tensor_pointwise(const sfhe_ctx* c, int lev, const u64* a, int64_t astride, const u64* b,
                            int64_t bstride, u64* d, int64_t dstride, int64_t batch, hipStream_t s);
// gathered product list: product p multiplies A ciphertext a_idx[p] by B
// ciphertext b_idx[p] (chunked matrices with nA, nB ciphertexts), d limb-major
int launch_tensor_gather(const sfhe_ctx* c, int lev, const u64* A, int64_t nA, const u64* B, int64_t nB,
                         const int* d_aidx, const int* d_bidx, u64* d, int64_t count, hipStream_t s);
// Row tiles of the lazy tensor: for tile g of kTileRows consecutive output
// rows of the batch, entries tstart[g] .. tstart[g+1]-1, each a visited k
// (ascending), a bit mask of the tile rows that visit it and, per tile row,
// the A ciphertext slot (or -1).
constexpr int kTileRows = 16;
// rows per tile of the column kernels (every wave owns all rows of its
// columns): the fp64 residues (3 sums per output, two columns per wave) and
// the carry-save sums of the primes 2^60 - c (9 sums per output, one column
// per wave) share one tile list
constexpr int kColTileRows = 4;
struct TileList {
  const int* tstart;
  const int* ek;
  const int* emask;
  const int* eslot;     // [entries][kTileRows]
  int n_row_tiles;
  int n_col_tiles;      // set per kernel from its TJ
  int rows;             // output rows in the batch
  int Nc;               // output columns (= B columns)
  int64_t nA, nB;       // ciphertexts stored by A and B (chunked layout)
  const int* bslot;     // [K][Nc] stored slot of B_kj, -1 if B_kj is zero; nullptr for a dense B
  int tile_rows;        // rows per tile (eslot stride)
};
// D[pos * Nc + j][3][L][N] = sum over the visited k of tensor(A[row pos, k], B[k, j]);
// the fp64 kernel's launch is bracketed by fp_start / fp_stop when non-null
// tl: tiles of kTileRows rows (the 128-bit integer kernel); tl_cols: tiles of
// kColTileRows rows (the column kernels: fp64 and carry-save)
int launch_tensor_tiles(const sfhe_ctx* c, const TileList& tl, const TileList& tl_cols, const u64* A, const u64* B,
                        u64* D, hipStream_t s, hipEvent_t fp_start = nullptr, hipEvent_t fp_stop = nullptr);
int tensor_fp_prime_count(const sfhe_ctx* c);

// ---- plaintext weights times encrypted values (ctpt.hip) ----
// one matmul W B of a batch: W's tile tables (held by W, built when it was
// encoded) and its outputs d0 .. d0 + rows * Nc - 1 of D (row-major)
struct PlainJob {
  const u64* B;          // encrypted K x Nc dense matrix, chunked layout, nB stored ciphertexts
  int64_t nB;
  int Nc, rows;
  const int* tstart;     // [tiles + 1] entry range of each 16-row tile of W
  const int* ek;         // k of each entry (ascending within a tile)
  const int* emask;      // bit r: tile row r visits k
  const u64* ew;         // [entry][L][16] weight of each tile row: the residue, as fp64 bits below 2^42
  const u64* ews;        // [entry][L][16] Shoup companions (primes of 2^42 and above)
  int64_t d0;
};
struct PlainBatch {
  const PlainJob* jobs;
  const int4* desc;      // per block group (job, tile within the job, column group of 4, 0)
  int n_desc;
  int nl;                // primes of B and of the weight tables (L: B at the top level)
  u64* D;                // [output][2][nl][N] sums, NTT domain
};
// every product of the batch, in one launch per arithmetic (fp64, integer)
int launch_plain_batch(const sfhe_ctx* c, const PlainBatch& pb, hipStream_t s);
// D[2][nl][N] += w B[slot] for one product (the one-launch-per-product form)
int launch_plain_product(const sfhe_ctx* c, const u64* B, int64_t nB, int64_t slot, const u64* w, const u64* ws,
                         u64* D, int nl, hipStream_t s);

// key switch of d2 rows (batch stride d2stride), result added into out
// (batch stride ostride, [2][nl][N]) if add_in, else written.
// key: [dnum][2][nb][N] NTT domain, the relinearisation key when null
// scratch (nullable): keyswitch_scratch_words(c, lev, batch) words the call
// uses instead of allocating
int keyswitch_batch(sfhe_ctx* c, int lev, const u64* d2, int64_t d2stride, u64* out, int64_t ostride,
                    bool add_in, int64_t batch, hipStream_t s, const u64* key = nullptr, u64* scratch = nullptr);
inline int64_t keyswitch_scratch_words(const sfhe_ctx* c, int lev, int64_t batch) {
  const int64_t nl = lev + 1, ne = nl + c->alpha;
  return batch * (nl + ne + 2 * ne + 2 * nl) * c->N;
}
// the allocation-free entry point's device scratch (noalloc.hip): its
// address on the context's device, looked up once per device at context
// creation; SFHE_OK or SFHE_E_DEVICE
int noalloc_setup(sfhe_ctx* c);
// where rescale writes: limb-major rows (stride words apart) or ciphertexts
// elem_base + b of a chunked matrix holding n_ct ciphertexts
struct OutLayout {
  u64* base;
  int64_t stride;
  bool chunked;
  int64_t n_ct, elem_base;
};
// scratch (nullable): rescale_scratch_words(c, lev, batch) words the call
// uses instead of allocating (for launches captured into a graph)
int rescale_batch(sfhe_ctx* c, int lev, const u64* in, int64_t istride, OutLayout out, int64_t batch, hipStream_t s,
                  u64* scratch = nullptr);
inline int64_t rescale_scratch_words(const sfhe_ctx* c, int lev, int64_t batch) {
  return c->logN == 14 ? batch * 2 * c->N : batch * 2 * c->N * (1 + lev);
}
// N = 2^14 only: Rescale((d0, d1) + KeySwitch(d2)) for n lazy sums D[b]
// (stride dw words; rows d0, d1, d2 of lev + 1 primes, NTT domain) in four
// fused transform kernels; the result goes to out (NTT domain, lev primes)
// scratch (nullable): keyswitch_rescale_n14_scratch_words(c, lev, n) words
// used instead of allocating (every word is written before it is read)
int keyswitch_rescale_n14(sfhe_ctx* c, int lev, const u64* D, int64_t dw, OutLayout out, int64_t n, hipStream_t s,
                          u64* scratch = nullptr);
int64_t keyswitch_rescale_n14_scratch_words(const sfhe_ctx* c, int lev, int64_t n);
// N = 2^14 only: Rescale((d0, d1)) for n sums D[b] (stride dw words, rows d0,
// d1 of lev + 1 primes, NTT domain) in two transform kernels
int rescale_n14(sfhe_ctx* c, int lev, const u64* D, int64_t dw, OutLayout out, int64_t n, hipStream_t s,
                u64* scratch = nullptr);
bool keyswitch_rescale_n14_supported(const sfhe_ctx* c);
// N = 2^14 only: (d0, d1) + KeySwitch(d2) with the given key (NTT domain
// [dnum][2][nb][N] and its Shoup companions) for n inputs D[b] (stride dw
// words; rows d0, d1, d2 of lev + 1 primes, NTT domain), written limb-major
// to out (lev + 1 primes per poly)
int keyswitch_n14(sfhe_ctx* c, int lev, const u64* D, int64_t dw, OutLayout out, int64_t n, const u64* key,
                  const u64* key_s, hipStream_t s);
// chunked out[oidx[o]] += sum of limb-major t[p] for p in seg[o] .. seg[o+1]-1 (rows [2][nl][N])
int launch_segment_sum(const sfhe_ctx* c, int nl, const u64* t, u64* out, int64_t n_ct, const int* d_seg,
                       const int64_t* d_oidx, int64_t nout, hipStream_t s);
// zero ciphertexts oidx[0..n) of a chunked matrix at nl primes
int launch_zero_outputs(const sfhe_ctx* c, u64* out, int64_t n_ct, int nl, const int64_t* d_oidx, int64_t n,
                        hipStream_t s);

// ---- several values per ciphertext and rotations (rotate.hip) ----
// 5^r mod 2N (slot j + r moves to slot j)
u64 galois_element(const sfhe_ctx* c, int64_t r);
// device table of X -> X^g on NTT-domain rows (out[p] = in[table[p]]), cached
const int* automorphism_table(sfhe_ctx* c, u64 g);
// rotation key of g, NTT domain [dnum][2][nb][N], generated on first use
const u64* rotation_key(sfhe_ctx* c, u64 g);
// the device table 5^j mod 2N, j < 64 (slot decoding), built once
int slot_table(sfhe_ctx* c);
// build the keys of the rotations by each of offsets (before enqueuing work)
int prepare_rotations(sfhe_ctx* c, const std::vector<int64_t>& offsets);
// rotate n ciphertexts in[x] ([2][lev+1][N] NTT domain, stride istride) by r
// slots into out (stride ostride); in and out must not overlap
int rotate_batch(sfhe_ctx* c, int lev, const u64* in, int64_t istride, int64_t r, u64* out, int64_t ostride,
                 int64_t n, hipStream_t s);
// N = 2^14: the same for n <= 1024 ciphertexts d_elem[x] of a chunked matrix
// (top level, n_ct ciphertexts), read in place
int rotate_chunked(sfhe_ctx* c, int lev, const u64* src, int64_t n_ct, const int64_t* d_elem, int64_t r, u64* out,
                   int64_t ostride, int64_t n, hipStream_t s);
// encrypt chunks x0 .. x0 + count - 1 of nvals stored values (slots per
// chunk) into tmp[count][2][L][N], NTT domain
int encrypt_slots(sfhe_ctx* c, u64* tmp, int64_t count, int64_t x0, const double* d_vals, int64_t nvals, int slots,
                  u64 seed, u64 operand, hipStream_t s);
// multiply n ciphertexts x[b] ([2][lev+1][N], stride words) by the slot-zero mask
int mask_batch(sfhe_ctx* c, int lev, u64* x, int64_t stride, int64_t n, hipStream_t s);

}  // namespace sfhe
