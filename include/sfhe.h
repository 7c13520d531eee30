/*
 * sfhe.h -- C ABI of the MI355X (gfx950) library for encrypted matrix
 * multiplication with unstructured sparsity.
 *
 * Method: Ferguson et al., "Exploiting Unstructured Sparsity in Fully
 * Homomorphic Encrypted DNNs" (EuroMLSys '25).  The operands are matrices of
 * CKKS ciphertexts, one value per ciphertext (chunk size c = 1, Sec. 3.2;
 * sfhe_matmul) or c values per ciphertext (sfhe_matmul_slots, with the
 * rotations and slot-zero mask of Algorithm 1); C = A*B is formed by
 * ciphertext products, relinearisation, rescaling and accumulation
 * (Algorithm 1), and the zeros of A are skipped through the plaintext
 * structure of one of the sparse schemes of Sec. 3.3.2 (naive sparse mask,
 * CSR, ELLPACK), or not at all (naive dense, Sec. 3.3.1).  Plaintext weights
 * times encrypted values (sfhe_matmul_plain*) and a request loop over them
 * (sfhe_server_*) are the server-side variant of Sec. 3.3.2.
 *
 * Every function returns an int status: SFHE_OK (0) or a negative SFHE_E_*
 * code; sfhe_last_error() then holds a message (thread-local).  No exception
 * or abort crosses this boundary; a failed call leaves its output handles NULL
 * and releases whatever it had allocated.
 *
 * Ownership: handles are opaque and owned by the library; the caller destroys
 * them.  Host arrays passed in are borrowed for the duration of the call only.
 * Device memory comes from the optional allocation hooks (a caching
 * allocator), otherwise from a stream-ordered memory pool of the context;
 * either way a block is taken and given back in the order of the stream of
 * the call that uses it (sfhe_device_hooks).  A `stream` argument is a
 * hipStream_t (NULL = the default stream); work is enqueued on it and calls
 * that return host data synchronise it.
 *
 * The library plays both parties for benchmarking: the secret key lives in
 * the context and never leaves it.
 *
 * Concurrency: a context and the handles made from it are used by one host
 * thread at a time (the context holds the last call's statistics, event
 * pool and key caches).  Work of one context may be enqueued on several
 * streams; results are not ordered across streams by the library.
 */
#ifndef SFHE_H
#define SFHE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SFHE_OK 0
#define SFHE_E_INVALID_ARG (-1)   /* NULL handle, bad enum, size out of range      */
#define SFHE_E_PARAMS (-2)        /* parameter set rejected                        */
#define SFHE_E_SHAPE (-3)         /* A.cols != B.rows, index out of range           */
#define SFHE_E_LEVEL (-4)         /* no prime left to rescale, level mismatch       */
#define SFHE_E_SCALE (-5)         /* operand scales differ                         */
#define SFHE_E_UNSUPPORTED (-6)   /* an operation the handle or ring does not support */
#define SFHE_E_NOMEM (-7)         /* device or host allocation failed               */
#define SFHE_E_DEVICE (-8)        /* a HIP call failed (its text is in last_error)  */
#define SFHE_E_STATE (-9)         /* keys not generated yet                        */
#define SFHE_E_DECRYPT (-10)      /* a decrypted coefficient left the decodable range */

typedef struct sfhe_ctx sfhe_ctx;   /* parameters, tables, keys (device resident) */
typedef struct sfhe_mat sfhe_mat;   /* an encrypted matrix and its plaintext structure */

/* Encodings of an operand (Sec. 3.3).  DENSE stores and visits every element
 * (naive dense, Algorithm 1).  NAIVE_SPARSE stores every element, zeros
 * included, and skips the products whose plaintext mask marks a zero.  CSR
 * stores the nonzeros only, with plaintext row pointers and column indices.
 * ELL stores max-nonzeros-per-row values per row, padded with trivial zero
 * ciphertexts whose plaintext column index is -1; padding is skipped. */
typedef enum {
  SFHE_ENC_DENSE = 0,
  SFHE_ENC_NAIVE_SPARSE = 1,
  SFHE_ENC_CSR = 2,
  SFHE_ENC_ELL = 3
} sfhe_encoding;

/* PER_PRODUCT follows Algorithm 1's order: every ciphertext product is
 * relinearised and rescaled, then added into its output.  LAZY sums the
 * degree-2 products of an output first and relinearises and rescales once per
 * output.  Both are exact up to the noise they add; their ciphertexts differ. */
typedef enum { SFHE_SCHED_PER_PRODUCT = 0, SFHE_SCHED_LAZY = 1 } sfhe_schedule;

/* An RNS CKKS parameter set (Sec. 3.1).  Primes are generated: for each bit
 * size in order (data primes q_0..q_{n_q-1}, then the special primes), the
 * largest prime below 2^bits that is 1 mod 2N and not already taken.  The
 * special primes form P for hybrid key switching with dnum digits of n_p data
 * primes each (dnum must equal ceil(n_q / n_p)).  log_n in [10, 15]; bits in
 * [log_n + 2, 61]; n_q >= 2; n_q + n_p <= 16. */
typedef struct {
  uint32_t log_n;
  uint32_t n_q, n_p, dnum;
  const uint32_t* q_bits;   /* n_q entries */
  const uint32_t* p_bits;   /* n_p entries */
  double log2_scale;        /* integer in [1, 60]: the encoding scale is 2^log2_scale */
  double sigma;             /* error standard deviation; the sampler clips at |e| <= 19 */
} sfhe_params;

/* Optional device allocator (a caching allocator such as PyTorch's).  alloc
 * returns device memory or NULL; free receives the pointer, the size it was
 * allocated with and the same stream.  Both are called from the thread that
 * called into the library.  `stream` (a hipStream_t, NULL = the default
 * stream) is the stream of the call that takes the block: allocation is
 * stream-ordered.  free is called once the last launch that reads or writes
 * the block has been enqueued on that stream, possibly before it has run, so
 * the allocator may hand the block only to work that follows on the same
 * stream (or to other streams once that stream has passed the point of the
 * free).  Temporaries of a call are taken and given back on the call's
 * stream; a matrix's ciphertexts on the stream of the call that made it,
 * given back by sfhe_mat_destroy, so that stream must still exist then (a
 * server takes every block of a batch on its client stream, and gives the
 * ones that are not results back there once the batch has ended).  A matrix read
 * by work on another stream must not be destroyed before that work has
 * ended.  Without hooks the library takes its blocks from a stream-ordered
 * memory pool of its own (hipMallocFromPoolAsync / hipFreeAsync on the same
 * streams); a block whose free has completed may go to any stream, and when
 * the pool cannot serve a request it waits for the device, gives its free
 * blocks back and tries once more. */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* ptr, size_t bytes, void* stream, void* user);
  void* user;
} sfhe_device_hooks;

typedef struct {
  int32_t rows, cols;
  int32_t level;            /* index of the last prime in use; limbs = level + 1 */
  double scale;
  sfhe_encoding enc;
  int64_t n_ciphertexts;    /* stored ciphertexts (ELL padding included) */
  int64_t nnz;              /* nonzero elements (the values that are encrypted) */
  int32_t ell_width;        /* ELL only, else 0 */
  uint64_t device_bytes;    /* ciphertext bytes held on the device: the memory of the
                               ciphertexts Sec. 4.1 records, compared across encodings
                               in Sec. 4.6 */
  int32_t slots;            /* values per ciphertext (the chunk size c of Sec. 3.2) */
} sfhe_mat_info;

typedef struct {
  double ms;                /* device time of the last sfhe_matmul (hipEvents) */
  int64_t products;         /* ct x ct tensor products executed */
  int64_t keyswitches;      /* relinearisations executed */
  int64_t outputs;          /* output ciphertexts written (trivial zeros included) */
  /* with profiling on (sfhe_set_profiling): device time per step, from
   * hipEvents recorded around each launch group on the call's stream */
  double tensor_ms;         /* tensor products and lazy sums, all primes        */
  double keyswitch_ms;      /* ModUp, key products, ModDown, their NTTs         */
  double rescale_ms;        /* rescale and per-product accumulation             */
  int64_t tensor_launches;  /* launch groups of the tensor step                 */
  /* always measured (one hipEvent pair per launch, profiling on or off):
   * device time of the tensor kernel for the primes below 2^42 */
  double tensor_fp_ms;
  int64_t tensor_fp_launches; /* launches of that kernel                        */
  int32_t tensor_fp_primes; /* primes it covers                                 */
  int32_t reserved;
} sfhe_stats;

/* Create a context for the RNS CKKS scheme of Sec. 3.1 (ring degree N, the
 * modulus chain of data primes, the special primes of key switching, the
 * encoding scale): generate the primes, twiddle and conversion tables and
 * upload them.  This is the context set-up Sec. 4.1 keeps outside the timed
 * region.  hooks may be NULL.  Fails with SFHE_E_PARAMS for an invalid set
 * and SFHE_E_DEVICE when no gfx950 device is usable. */
int sfhe_ctx_create(const sfhe_params* params, const sfhe_device_hooks* hooks, sfhe_ctx** out);
void sfhe_ctx_destroy(sfhe_ctx* ctx);

/* The ring degree N and the basis primes (data primes, then special primes);
 * cap is the capacity of out in entries. */
int sfhe_ctx_n(const sfhe_ctx* ctx, int32_t* n);
int sfhe_ctx_primes(const sfhe_ctx* ctx, uint64_t* out, size_t cap);

/* Generate the scheme's keys (Sec. 3.1): the ternary secret and the
 * relinearisation key every ciphertext product needs (Algorithm 1's
 * relinearise step), from seed; the keys stay on the device.  Part of the
 * set-up outside the timed region (Sec. 4.1).  Must precede any
 * encryption. */
int sfhe_keygen(sfhe_ctx* ctx, uint64_t seed);

/* Encrypt an operand matrix (Sec. 4.1: the operands are encrypted before the
 * timed product; Sec. 3.2: chunk size 1, one value per ciphertext; Sec.
 * 3.3.2: the encoding decides which elements are stored, the structure stays
 * plaintext).  A rows x cols row-major fp64 matrix (leading dimension ld >=
 * cols) with the given encoding: one secret-key ciphertext per stored element,
 * value in slot 0, at the top level with scale 2^log2_scale.  Element (i, j)
 * draws its randomness from (seed, operand_id, i, j) only, so an element has
 * the same ciphertext under every encoding.  An element is zero iff it
 * compares equal to 0.0.  |value| * 2^(log2_scale + 1 - log_n) must stay
 * below 2^62. */
int sfhe_encrypt_matrix(sfhe_ctx* ctx, const double* vals, int32_t rows, int32_t cols, int64_t ld,
                        sfhe_encoding enc, uint64_t seed, uint32_t operand_id, void* stream,
                        sfhe_mat** out);

/* C = A * B (Algorithm 1 at c = 1 with A's zeros skipped per its encoding).
 * A and B must be at the same level (>= 1) with equal scales.  B may be of
 * any encoding: with a sparse-encoded B (naive sparse, CSR, ELLPACK) a
 * product is skipped when A_ik or B_kj is zero (the naive scheme's two masks,
 * Sec. 3.3.2); a DENSE B multiplies every k of A's row.  The result is a DENSE
 * matrix one level lower with scale^2 / q_level.  Outputs with no product
 * are trivial zero ciphertexts.  The device time is reported by
 * sfhe_last_stats.  All work is ordered on `stream`: at N = 2^14 the LAZY
 * key switch may run its slices on two side streams of the context, forked
 * from `stream` after the tensor step and joined back into it before the
 * call's last launch (sfhe_ks_tuning); so calls of one context on several
 * streams do not overlap their key switches. */
int sfhe_matmul(sfhe_ctx* ctx, const sfhe_mat* A, const sfhe_mat* B, sfhe_schedule sched,
                void* stream, sfhe_mat** C);

/* Decrypt and decode every element to out (row-major, leading dimension ld),
 * the step after the product with which Sec. 4.5 compares the encrypted
 * result against the plaintext one.  Elements that an encoding does not
 * store decrypt to 0.0. */
int sfhe_decrypt_matrix(sfhe_ctx* ctx, const sfhe_mat* m, double* out, int64_t ld, void* stream);

/* Copy one stored ciphertext of element (i, j), in the coefficient domain
 * with residues in [0, q), to host memory: out[2][level+1][N] (for checking
 * a result word for word against another implementation of the same
 * scheme, beside the decrypted comparison of Sec. 4.5).  cap is the
 * capacity in entries.  An element the encoding does not store is an error
 * (SFHE_E_SHAPE); an ELL padding slot is not addressable. */
int sfhe_export_ct(sfhe_ctx* ctx, const sfhe_mat* m, int32_t i, int32_t j, uint64_t* out, size_t cap,
                   void* stream);

/* The launches of one LAZY sfhe_matmul (the batched form: every product of
 * the layer summed per output, one relinearisation and rescale per output,
 * Sec. 3.3 with Algorithm 1's steps) captured into a HIP graph for replay.
 * Creation prepares the tile lists, lazy sums, key-switch scratch and the
 * result once (on stream), runs the product once outside the capture (this
 * tunes the key-switch slice if the context has not yet), then captures its
 * launches on a stream of its own.  Each sfhe_matmul_graph_launch replays
 * them on stream, recomputing the result from the current contents of A and
 * B (which must outlive the graph); sfhe_last_stats reports the replay's
 * device time and counts.  The result belongs to the graph (read-only
 * handle from sfhe_matmul_graph_result, for export and decryption) and is
 * freed with it; destroying the graph waits for its last replay.  Replays
 * of one graph must not overlap.  Errors as sfhe_matmul; matrices with
 * several values per ciphertext are SFHE_E_UNSUPPORTED. */
typedef struct sfhe_matmul_graph sfhe_matmul_graph;
int sfhe_matmul_graph_create(sfhe_ctx* ctx, const sfhe_mat* A, const sfhe_mat* B, void* stream,
                             sfhe_matmul_graph** out);
int sfhe_matmul_graph_launch(sfhe_matmul_graph* graph, void* stream);
int sfhe_matmul_graph_result(const sfhe_matmul_graph* graph, const sfhe_mat** out);
void sfhe_matmul_graph_destroy(sfhe_matmul_graph* graph);

/* ---- Several values per ciphertext (Sec. 3.2, Algorithm 1) -------------
 * A matrix is a list of ciphertexts ("chunks") holding up to c = slots
 * values each.  The stored values of an encoding (all rows x cols entries
 * row-major for DENSE and NAIVE_SPARSE, the nonzeros in row order for CSR,
 * rows x width for ELLPACK with 0.0 in the padding) are cut into chunks of c
 * consecutive values: stored value v sits in slot v mod c of ciphertext
 * v / c.  Slot j of a ciphertext is its plaintext's value at zeta^(5^j),
 * zeta = exp(i pi / N): values z_0 .. z_{n-1} encode as
 * m_t = nearbyint(sum_j z_j 2 Delta / N cos(pi (5^j t mod 2N) / N)), summed
 * in slot order (n = 1 is the one-value encoding).  Secret-key encryption as
 * sfhe_encrypt_matrix, the randomness of chunk x keyed by (operand_id, x,
 * 2^40 + n).  sfhe_matmul, sfhe_matmul_plain and sfhe_export_ct reject
 * matrices with slots > 1 (SFHE_E_UNSUPPORTED); sfhe_decrypt_matrix decodes
 * every slot; sfhe_export_stored reads any ciphertext. */

/* Encrypt the stored values of vals (rows x cols, leading dimension ld) in
 * chunks of `slots` values, 1 <= slots <= min(64, N/2).  Every value of a
 * chunk of n values must satisfy |value| 2^(log2_scale + 1 - log_n) < 4e18 / n
 * (else SFHE_E_INVALID_ARG).  Needs keys. */
int sfhe_encrypt_matrix_slots(sfhe_ctx* ctx, const double* vals, int32_t rows, int32_t cols, int64_t ld,
                              sfhe_encoding enc, int32_t slots, uint64_t seed, uint32_t operand_id,
                              void* stream, sfhe_mat** out);

/* C = A * B by Algorithm 1 with chunks (Sec. 3.3.1): for output (i, j) and
 * every k that A's row i visits (its zeros skipped per its encoding), the
 * chunks holding A_ik and B_kj are rotated so that the two values sit in
 * slot 0, multiplied, relinearised and rescaled.  LAZY sums these products
 * of an output before the relinearisation; PER_PRODUCT does not.  Each
 * product (PER_PRODUCT) or sum (LAZY) is then multiplied by the slot-zero
 * mask (the plaintext of 1.0 in slot 0 at scale 2^log2_scale), rescaled,
 * rotated from slot 0 to slot (i Nc + j) mod c and added into result chunk
 * (i Nc + j) / c.  A and B hold the same number of values per ciphertext, B
 * is DENSE, both are at the top level, and the context has at least four
 * data primes.  C: DENSE, rows x cols of the product, c values per
 * ciphertext, level L - 3, scale scale_A scale_B 2^log2_scale / (q_{L-1}
 * q_{L-2}); chunks no product reaches stay trivial zeros.  Rotation keys
 * (for offsets -(c-1) .. c-1) are generated on first use and kept by the
 * context; generating them synchronises the device.  The call holds
 * temporary device memory for A's visited values and all of B as
 * one-value ciphertexts (top level) besides the lazy sums of the product.
 * sfhe_last_stats: products, relinearisations plus rotations (as
 * keyswitches), result ciphertexts and the device time of the whole call. */
int sfhe_matmul_slots(sfhe_ctx* ctx, const sfhe_mat* A, const sfhe_mat* B, sfhe_schedule sched,
                      void* stream, sfhe_mat** C);

/* Copy stored ciphertext n (0 <= n < n_ciphertexts) of any encrypted matrix,
 * in the coefficient domain, to host memory: out[2][level+1][N]. */
int sfhe_export_stored(sfhe_ctx* ctx, const sfhe_mat* m, int64_t n, uint64_t* out, size_t cap,
                       void* stream);

/* ---- Plaintext weights times encrypted values -------------------------
 * Sec. 3.3.2: a server that holds a layer's weights in plaintext multiplies
 * them into the client's encrypted input; the weights' zeros are skipped
 * through the same encodings.  A weight w is the constant polynomial
 * m = nearbyint(w * 2^log2_scale_w) (round half to even): a constant takes
 * the same value at every root of X^N + 1, so it scales every slot by m, and
 * its product with a ciphertext multiplies both polys coefficient-wise by
 * m mod q_i.  No relinearisation is needed. */

/* Encode a rows x cols row-major fp64 weight matrix (leading dimension ld >=
 * cols) with the given encoding (zeros: elements equal to 0.0), scale
 * 2^log2_scale_w, 0 <= log2_scale_w <= 62, and |w| * 2^log2_scale_w below
 * 2^62 (else SFHE_E_INVALID_ARG).  The weights' residues stay in host
 * memory owned by the handle, and their tile tables for the products (W's
 * rows in tiles of 16; per tile, the columns k some row visits with the mask
 * of those rows; per such entry and data prime, the 16 rows' weights) are
 * built once here and kept in device memory owned by the handle, copied
 * synchronously before the call returns.  No key is needed.  The handle is
 * a left operand of sfhe_matmul_plain only (sfhe_matmul,
 * sfhe_decrypt_matrix and sfhe_export_ct reject it with SFHE_E_UNSUPPORTED);
 * sfhe_matrix_info reports level L - 1, scale 2^log2_scale_w and the tables'
 * device bytes. */
int sfhe_encode_matrix(sfhe_ctx* ctx, const double* vals, int32_t rows, int32_t cols, int64_t ld,
                       sfhe_encoding enc, int32_t log2_scale_w, sfhe_mat** out);

/* C = W * B for plaintext weights W (from sfhe_encode_matrix) and an
 * encrypted DENSE B at the top level: per output, the products of the
 * visited k are summed in the NTT domain and the sum is rescaled once.  The
 * result is a DENSE encrypted matrix one level lower with scale
 * W.scale * B.scale / q_level; outputs with no visited k are trivial zeros.
 * Errors as sfhe_matmul (SFHE_E_SHAPE if W.cols != B.rows). */
int sfhe_matmul_plain(sfhe_ctx* ctx, const sfhe_mat* W, const sfhe_mat* B, void* stream, sfhe_mat** C);

typedef enum {
  SFHE_PLAIN_FUSED = 0,             /* every product of the batch in one launch per arithmetic */
  SFHE_PLAIN_LAUNCH_PER_PRODUCT = 1 /* one launch per (output, k) product: the unbatched form */
} sfhe_plain_launch;

/* count independent products C[n] = W[n] * B[n] (each as sfhe_matmul_plain,
 * shapes free per n) in one call.  SFHE_PLAIN_FUSED runs the products of all
 * of them in one kernel launch (two when the primes need both the fp64 and
 * the integer arithmetic), then one rescale per matrix;
 * SFHE_PLAIN_LAUNCH_PER_PRODUCT launches one kernel per product instead.
 * Both give the same bits.  The sums of all outputs are held on the device
 * at once (2 (L) N words per output): SFHE_E_NOMEM if they do not fit.  C
 * has count entries; on failure every entry is NULL.  sfhe_last_stats
 * reports the device time of the products and rescales (after the result,
 * scratch and table allocations and uploads), the products and the product
 * launches. */
int sfhe_matmul_plain_batch(sfhe_ctx* ctx, int32_t count, const sfhe_mat* const* W, const sfhe_mat* const* B,
                            sfhe_plain_launch launch, void* stream, sfhe_mat** C);

/* The launches of one sfhe_matmul_plain_batch (either form) captured into a
 * HIP graph for replay: creation prepares the tables, sums, scratch and
 * results once (on stream), runs the batch once, then captures its launches
 * on a stream of its own.  Each sfhe_plain_graph_launch replays them on
 * stream, recomputing the results from the current contents of the B
 * matrices (which must outlive the graph); sfhe_last_stats reports the
 * replay's device time.  The results belong to the graph
 * (sfhe_plain_graph_result gives read-only handles for export and decrypt)
 * and are freed with it.  Replays of one graph must not overlap. */
typedef struct sfhe_plain_graph sfhe_plain_graph;
int sfhe_plain_graph_create(sfhe_ctx* ctx, int32_t count, const sfhe_mat* const* W, const sfhe_mat* const* B,
                            sfhe_plain_launch launch, void* stream, sfhe_plain_graph** out);
int sfhe_plain_graph_launch(sfhe_plain_graph* graph, void* stream);
int sfhe_plain_graph_result(const sfhe_plain_graph* graph, int32_t n, const sfhe_mat** out);
void sfhe_plain_graph_destroy(sfhe_plain_graph* graph);

/* ---- Serving: a request loop over plaintext-weight products ------------
 * Continuous batching for the server side of Sec. 3.3.2 (plaintext weights,
 * encrypted activations).  Requests W X (plaintext weights from
 * sfhe_encode_matrix, encrypted DENSE activations X at the top level) queue
 * in arrival order.  Each sfhe_server_step first retires the batches whose
 * device work has ended, then admits queued requests, in order, while the
 * device bytes they hold until they complete fit budget_bytes beside the
 * batches still running (per request: 2 (L) N words of sums and 2 (L - 1) N
 * of results per output, a rescale scratch for up to 2048 of its outputs and
 * its block descriptors; W's tile tables are W's own), and enqueues them as one fused sfhe_matmul_plain_batch
 * on the stream, of the server's n_streams streams (1 to 4, created by the
 * server at the default priority), with the fewest running batches.  With
 * one stream the batches run in admission order; with several, a batch
 * admitted while others run starts at once and overlaps them on the
 * device.  With a slot limit (sfhe_server_set_slots), a stream that holds
 * that many running batches takes no more, and while every stream is full
 * requests stay queued and join the next batch.  A batch's launches first
 * wait for the work enqueued on `stream` (the client stream, e.g. the
 * requests' encryptions) before the step.  A request's result is the same,
 * bit for bit, alone or in any batch.  The caller keeps W and X alive until
 * its request is done; a finished result belongs to the caller from
 * sfhe_server_poll on.  Every block of a batch (results, sums, scratch,
 * descriptors) is taken in the client stream's order before the batch's
 * stream waits for that stream, so all server streams draw on one stream's
 * blocks; the blocks that are not results go back, in the same order, when
 * a step or poll finds the batch ended, and a result goes back there when
 * the caller frees it (so it may outlive the server).  Calls on one server
 * must not overlap. */
typedef struct sfhe_server sfhe_server;
int sfhe_server_create(sfhe_ctx* ctx, uint64_t budget_bytes, int32_t n_streams, void* stream, sfhe_server** out);
/* at most per_stream running batches per server stream (0, the default: no
 * limit); negative is SFHE_E_INVALID_ARG */
int sfhe_server_set_slots(sfhe_server* srv, int32_t per_stream);
/* at most max_bytes (as sfhe_server_request_bytes counts them) in one batch
 * (0, the default: no limit); a request larger than the limit runs as a
 * batch of its own.  With a limit of budget_bytes / n_streams every server
 * stream can hold a running batch at once, so batches overlap on the device
 * even when the requests alone would fill the budget. */
int sfhe_server_set_batch_bytes(sfhe_server* srv, uint64_t max_bytes);
/* the device bytes the server counts for request W X against its budget */
int sfhe_server_request_bytes(const sfhe_ctx* ctx, const sfhe_mat* W, const sfhe_mat* X, uint64_t* bytes);
/* queue W X; a request larger than the budget is SFHE_E_NOMEM */
int sfhe_server_submit(sfhe_server* srv, const sfhe_mat* W, const sfhe_mat* X, int64_t* ticket);
/* retire ended batches, admit and launch; *admitted = requests launched now */
int sfhe_server_step(sfhe_server* srv, int32_t* admitted);
/* whether ticket's request is done (with wait != 0, waiting for its batch if
 * it is running); if so *C receives its result, and (each nullable)
 * *batch_ms the device time of its batch, *batch_size the requests in it,
 * *start_ms and *end_ms the batch's device-time interval in ms after the
 * server's creation (intervals of different batches that intersect ran
 * concurrently) */
int sfhe_server_poll(sfhe_server* srv, int64_t ticket, int32_t wait, int32_t* done, sfhe_mat** C, double* batch_ms,
                     int32_t* batch_size, double* start_ms, double* end_ms);
int sfhe_server_status(const sfhe_server* srv, int64_t* queued, int64_t* running, uint64_t* bytes_in_flight,
                       int64_t* batches, int64_t* products);
/* waits for the running batches; results not yet polled are freed */
void sfhe_server_destroy(sfhe_server* srv);

/* Measurement support (not part of the method): the sustained issue rate,
 * in lane operations per second, of one VALU instruction class on the
 * current device, from a kernel of independent dependency chains timed with
 * hipEvents on the default stream: kind 0 = fp64 FMA, 1 = v_mad_u64_u32
 * (32 x 32 + 64 -> 64 bits), 2 = 32-bit integer add/xor.  Rooflines are
 * stated against these as well as against the published peaks.  Allocates
 * and frees a 2 KiB buffer; synchronises the device. */
int sfhe_probe_valu(int32_t kind, double* lane_ops_per_s);

int sfhe_matrix_info(const sfhe_mat* m, sfhe_mat_info* out);
/* Statistics of the last product call: its device time from hipEvents
 * around the multiplication alone (Sec. 4.1: execution time excluding
 * context set-up, encryption and decryption), products, relinearisations
 * and outputs; waits for the call's events. */
int sfhe_last_stats(const sfhe_ctx* ctx, sfhe_stats* out);

/* Per-step device timing of sfhe_matmul (off by default): with on != 0 the
 * library records a hipEvent pair around each launch group of the tensor,
 * key-switch and rescale steps; sfhe_last_stats sums them.  The events
 * serialise nothing beyond the stream order the launches already have. */
int sfhe_set_profiling(sfhe_ctx* ctx, int32_t on);
void sfhe_mat_destroy(sfhe_mat* m);
const char* sfhe_last_error(void);

/* ---- Primitive steps on caller-owned device buffers --------------------
 * The steps one ciphertext product goes through (Algorithm 1: multiply,
 * relinearise, rescale), exposed for testing and composition.  Polynomials
 * are rows of N uint64 residues in [0, q); "NTT domain" means the negacyclic
 * transform with index k holding a(psi^(2*brv(k)+1)), psi the smallest
 * primitive 2N-th root of unity mod q.  Storage order of an NTT-domain row:
 * index k at position k for N < 2^14; for N = 2^14 the transform kernels
 * keep each thread's registers contiguous, so position r * 512 + t holds
 * index ((r >> 4) << 13) | ((t & 63) << 4) | (t6 << 10) | (t8 << 11) |
 * (t7 << 12) | (r & 15), where 0 <= r < 32, 0 <= t < 512 and t6..t8 are
 * bits of t; for N = 2^15 each half of a row (positions h 2^14 ..
 * h 2^14 + 2^14 - 1) holds indices h 2^14 .. h 2^14 + 2^14 - 1 in that
 * N = 2^14 order.  Every NTT-domain buffer of the library (matrices, keys,
 * primitive inputs and outputs) uses that order; coefficient-domain rows are
 * always in natural order.  Buffers must not overlap unless stated. */

/* NTT designs (the transform radix and tile of every launch of
 * sfhe_ntt and of the library's unfused transforms: encryption, decryption,
 * the generic key switch and rescale, rotations): 0 = the register transform
 * (32 residues per thread, half-row LDS exchanges; N >= 2^14), 1, 2, 3 = the
 * LDS transform with radix-16, radix-8 or radix-4 passes (one thread per 16,
 * 8 or 4 residues; N <= 2^14).  All give the same bits in the storage order
 * above.  sfhe_ctx_create times every design that applies to the ring (a
 * scratch batch of about 2048 rows) and keeps the fastest per
 * direction; N = 2^15 has the register design only.  The fused N = 2^14
 * kernels (key switch, rescale) always use the register design. */
/* The design in use for direction `inverse` and, in us_per_row[0..cap), the
 * measured microseconds per row of each design (-1: does not apply). */
int sfhe_ntt_tuning(const sfhe_ctx* ctx, int32_t inverse, int32_t* variant, double* us_per_row, int32_t cap);
/* Use design `variant` for direction `inverse` (SFHE_E_UNSUPPORTED if it does
 * not apply to the ring); -1 returns to the measured choice. */
int sfhe_set_ntt_variant(sfhe_ctx* ctx, int32_t inverse, int32_t variant);

/* Key-switch tuning (the fused key switch and rescale at N = 2^14): the
 * outputs of a LAZY product are key-switched in slices, one launch of each
 * fused kernel per slice, on the call's stream or alternately on two side
 * streams forked from it and joined back (so one slice's memory-bound base
 * conversions overlap another's transforms).  The first LAZY product of a
 * context with at least 1024 outputs times every one-stream candidate (128
 * .. 4096 outputs per slice) on its first outputs, then the best slice and
 * half of it on two streams, and keeps the fastest.  *slice, *streams: the
 * setting in use (slice 0: not tuned yet); sizes[0..cap) /
 * us_per_output[0..cap): the one-stream candidates and their measured
 * microseconds per output (-1: not measured); sizes2[0..2) /
 * us_per_output2[0..2): the same for the two-stream candidates.  Pointers
 * other than slice may be NULL. */
int sfhe_ks_tuning(const sfhe_ctx* ctx, int32_t* slice, int32_t* streams, int32_t* sizes, double* us_per_output,
                   int32_t cap, int32_t* sizes2, double* us_per_output2);
/* Use `slice` outputs per launch group (a power of two in [64, 4096]) on
 * `streams` (1 or 2) key-switch streams; slice 0 tunes again at the next
 * LAZY product, -1 returns to the tuned setting. */
int sfhe_set_ks_slice(sfhe_ctx* ctx, int32_t slice, int32_t streams);

/* In-place negacyclic NTT (inverse = 0) or inverse NTT (inverse = 1) of
 * `batch` groups of n_limbs rows laid out [batch][n_limbs][N]; row l of a
 * group is taken modulo basis prime first_prime + l. */
int sfhe_ntt(sfhe_ctx* ctx, uint64_t* data, int32_t batch, int32_t n_limbs, int32_t first_prime,
             int32_t inverse, void* stream);

/* Tensor product of degree-1 ciphertexts at `level`, NTT domain:
 * a, b [batch][2][level+1][N] -> d [batch][3][level+1][N] with
 * d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1. */
int sfhe_tensor(sfhe_ctx* ctx, int32_t level, const uint64_t* a, const uint64_t* b, uint64_t* d,
                int32_t batch, void* stream);

/* Relinearisation key switch of degree-2 parts at `level`, NTT domain:
 * d2 [batch][level+1][N] -> out [batch][2][level+1][N] with
 * out0 + out1*s = d2*s^2 + small.  Needs keys. */
int sfhe_keyswitch(sfhe_ctx* ctx, int32_t level, const uint64_t* d2, uint64_t* out, int32_t batch,
                   void* stream);

/* sfhe_keyswitch for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same operation and bits, with every working row in one fixed device
 * array of 64 MiB per GPU that the library holds until the process ends
 * (its address is looked up when a context is created on the device).  The
 * call allocates nothing, host or device.  A batch needs
 * batch * (3 (level + 1) + 3 (level + 1 + n_p)) * N * 8 bytes of it (at
 * N = 2^14, five data and three special primes, level 4: up to 13
 * ciphertexts); a larger batch is SFHE_E_INVALID_ARG, to be split by the
 * caller.  All calls on one GPU share the array: calls whose work overlaps
 * on the device (other streams, other host threads or contexts) race and
 * must be ordered by the caller. */
int sfhe_keyswitch_noalloc(sfhe_ctx* ctx, int32_t level, const uint64_t* d2, uint64_t* out, int32_t batch,
                           void* stream);

/* Rescale by the last prime of `level` (level >= 1), NTT domain, with exact
 * rounding (centered lift): in [batch][2][level+1][N] -> out [batch][2][level][N]. */
int sfhe_rescale(sfhe_ctx* ctx, int32_t level, const uint64_t* in, uint64_t* out, int32_t batch,
                 void* stream);

/* Rotation by r slots (slot j receives slot j + r, indices mod N/2) of
 * ciphertexts at `level`, NTT domain: in [batch][2][level+1][N] -> out, same
 * shape (Sec. 3.3.1: the automorphism X -> X^g, g = 5^r mod 2N, of both
 * polys, then a key switch of c1(X^g) from s(X^g) back to s with the
 * rotation key of g: digit j = (-a s + e + [P]_{q} s(X^g) on digit j's
 * primes, a), built like the relinearisation key; randomness keyed by
 * (g, j[, prime])).  in and out must not overlap.  Needs keys. */
int sfhe_rotate(sfhe_ctx* ctx, int32_t level, const uint64_t* in, uint64_t* out, int32_t batch, int32_t r,
                void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SFHE_H */
