"""Python access to the CPU oracle (``sfhe_oracle.c``) -- TEST INFRASTRUCTURE ONLY.

The oracle is a plain, slow implementation of the encrypted matrix product of
Ferguson et al. (EuroMLSys '25): Algorithm 1 at chunk size c = 1, the three
sparse schemes of Sec. 3.3.2 and the thread assignment of Sec. 3.4, over an
RNS CKKS scheme (Sec. 3.1).  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the GPU library never
does, and the two share no code.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sfhe_oracle.c")
# SFHE_ORACLE_LIB names another build of the same source (the sanitizer
# build of the pin tests); the default is the in-tree library
LIB = os.environ.get("SFHE_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]

ENC = {"dense": 0, "naive": 1, "csr": 2, "ell": 3}
SCHED = {"per_product": 0, "lazy": 1}
CDT_LEN = 20

_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


def build(out=None, sanitize=False):
    """Compile the oracle with gcc (plain C11, no vectorisation tricks); with
    sanitize, an AddressSanitizer + UndefinedBehaviorSanitizer build that
    aborts on the first report (loaded with libasan preloaded)."""
    opt = SAN_FLAGS if sanitize else ["-O2"]
    cmd = ["gcc"] + opt + ["-std=gnu11", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", out or LIB, SRC, "-lm", "-lpthread"]
    subprocess.check_call(cmd)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.environ.get("SFHE_ORACLE_LIB") and (not os.path.exists(LIB) or
                                                       os.path.getmtime(LIB) < os.path.getmtime(SRC)):
            build()
        L = ctypes.CDLL(LIB)
        L.orc_ctx_create.restype = ctypes.c_void_p
        L.orc_ctx_create.argtypes = [ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int, _i32p,
                                     ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.orc_ctx_destroy.argtypes = [ctypes.c_void_p]
        for name in ("orc_n", "orc_nbasis"):
            getattr(L, name).argtypes = [ctypes.c_void_p]
            getattr(L, name).restype = ctypes.c_int
        for name in ("orc_primes", "orc_psi", "orc_cdt_table"):
            getattr(L, name).argtypes = [ctypes.c_void_p, _u64p]
        for name in ("orc_ntt_forward", "orc_ntt_inverse"):
            getattr(L, name).argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p]
        L.orc_polymul.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p, _u64p, _u64p]
        L.orc_is_prime.argtypes = [ctypes.c_uint64]
        L.orc_is_prime.restype = ctypes.c_int
        L.orc_stream_word.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, _u64p, ctypes.c_uint64]
        L.orc_stream_word.restype = ctypes.c_uint64
        L.orc_encode.argtypes = [ctypes.c_void_p, ctypes.c_double, _i64p]
        L.orc_encode.restype = ctypes.c_int
        L.orc_keygen.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        L.orc_secret.argtypes = [ctypes.c_void_p, _i64p]
        L.orc_rlk.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p]
        L.orc_rlk_error.argtypes = [ctypes.c_void_p, ctypes.c_int, _i64p]
        L.orc_enc_error.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.c_uint64, ctypes.c_uint64, _i64p]
        L.orc_encrypt.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                                  ctypes.c_uint64, ctypes.c_uint64, _u64p]
        L.orc_encrypt.restype = ctypes.c_int
        L.orc_tensor.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p, _u64p, _u64p]
        L.orc_keyswitch.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p, _u64p]
        L.orc_modup.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _u64p, _u64p]
        L.orc_moddown.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p, _u64p]
        L.orc_crt_centered.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p, ctypes.c_size_t]
        L.orc_crt_centered.restype = ctypes.c_longdouble
        L.orc_rescale.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p, _u64p]
        L.orc_decrypt_poly.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p, _u64p]
        L.orc_decode.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p, ctypes.c_double]
        L.orc_decode.restype = ctypes.c_double
        L.orc_decrypt.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p, ctypes.c_double]
        L.orc_decrypt.restype = ctypes.c_double
        L.orc_row_ks.argtypes = [_f64p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32p]
        L.orc_row_ks.restype = ctypes.c_int
        L.orc_matmul.argtypes = [ctypes.c_void_p, _f64p, ctypes.c_int, ctypes.c_int, _f64p, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                 ctypes.c_uint64, ctypes.c_uint64, _i32p, _i32p, ctypes.c_int,
                                 ctypes.c_int, _u64p, _f64p, _f64p]
        L.orc_matmul.restype = ctypes.c_int
        L.orc_matmul2.argtypes = [ctypes.c_void_p, _f64p, ctypes.c_int, ctypes.c_int, _f64p, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                  ctypes.c_uint64, ctypes.c_uint64, _i32p, _i32p, ctypes.c_int,
                                  ctypes.c_int, _u64p, _f64p, _f64p]
        L.orc_matmul2.restype = ctypes.c_int
        L.orc_galois.argtypes = [ctypes.c_void_p, ctypes.c_long]
        L.orc_galois.restype = ctypes.c_uint64
        L.orc_encode_slots.argtypes = [ctypes.c_void_p, _f64p, ctypes.c_int, _i64p]
        L.orc_encode_slots.restype = ctypes.c_int
        L.orc_decrypt_slot.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p, ctypes.c_double, ctypes.c_int]
        L.orc_decrypt_slot.restype = ctypes.c_double
        L.orc_automorphism.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p, ctypes.c_uint64, _u64p]
        L.orc_rotkey.argtypes = [ctypes.c_void_p, ctypes.c_uint64, _u64p, _i64p]
        L.orc_rotate.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p, ctypes.c_long, _u64p]
        L.orc_rotate.restype = ctypes.c_int
        L.orc_encrypt_slots.argtypes = [ctypes.c_void_p, _f64p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                        ctypes.c_uint64, _u64p]
        L.orc_encrypt_slots.restype = ctypes.c_int
        L.orc_matmul_chunked.argtypes = [ctypes.c_void_p, _f64p, ctypes.c_int, ctypes.c_int, _f64p, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_uint64, ctypes.c_uint64, _i32p, _i32p, ctypes.c_int, _u64p, _f64p]
        L.orc_matmul_chunked.restype = ctypes.c_int
        L.orc_weight.argtypes = [ctypes.c_double, ctypes.c_double, _i64p]
        L.orc_weight.restype = ctypes.c_int
        L.orc_matmul_plain.argtypes = [ctypes.c_void_p, _f64p, ctypes.c_int, ctypes.c_int, _f64p, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                                       _i32p, _i32p, ctypes.c_int, ctypes.c_int, _u64p, _f64p, _f64p]
        L.orc_matmul_plain.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _u64(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return a


class Oracle:
    """One parameter set plus (after keygen) its keys."""

    def __init__(self, log_n, q_bits, p_bits, dnum, log2_scale=40.0, sigma=3.2):
        self.log_n = int(log_n)
        self.n = 1 << self.log_n
        self.L = len(q_bits)
        self.alpha = len(p_bits)
        self.dnum = int(dnum)
        self.log2_scale = float(log2_scale)
        qb = np.asarray(q_bits, dtype=np.int32)
        pb = np.asarray(p_bits, dtype=np.int32)
        h = lib().orc_ctx_create(self.log_n, self.L, _p(qb, _i32p), self.alpha, _p(pb, _i32p),
                                 self.dnum, float(log2_scale), float(sigma))
        if not h:
            raise ValueError("oracle rejected the parameters")
        self._h = ctypes.c_void_p(h)
        nb = self.L + self.alpha
        self.primes = np.zeros(nb, dtype=np.uint64)
        lib().orc_primes(self._h, _p(self.primes, _u64p))
        self.psi = np.zeros(nb, dtype=np.uint64)
        lib().orc_psi(self._h, _p(self.psi, _u64p))
        self.q = [int(x) for x in self.primes[:self.L]]
        self.p = [int(x) for x in self.primes[self.L:]]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_ctx_destroy(h)
            self._h = None

    # ---- primitives -------------------------------------------------
    def cdt_table(self):
        out = np.zeros(CDT_LEN, dtype=np.uint64)
        lib().orc_cdt_table(self._h, _p(out, _u64p))
        return out

    def ntt(self, r, a):
        a = _u64(a).copy()
        lib().orc_ntt_forward(self._h, int(r), _p(a, _u64p))
        return a

    def intt(self, r, a):
        a = _u64(a).copy()
        lib().orc_ntt_inverse(self._h, int(r), _p(a, _u64p))
        return a

    def polymul(self, r, a, b):
        a = _u64(a); b = _u64(b)
        out = np.zeros(self.n, dtype=np.uint64)
        lib().orc_polymul(self._h, int(r), _p(a, _u64p), _p(b, _u64p), _p(out, _u64p))
        return out

    def encode(self, z):
        m = np.zeros(self.n, dtype=np.int64)
        if lib().orc_encode(self._h, float(z), _p(m, _i64p)) != 0:
            raise ValueError("value too large to encode")
        return m

    # ---- keys, encryption ---------------------------------------------
    def keygen(self, seed):
        lib().orc_keygen(self._h, ctypes.c_uint64(seed))

    def secret(self):
        s = np.zeros(self.n, dtype=np.int64)
        lib().orc_secret(self._h, _p(s, _i64p))
        return s

    def rlk(self, j):
        nb = self.L + self.alpha
        out = np.zeros((2, nb, self.n), dtype=np.uint64)
        lib().orc_rlk(self._h, int(j), _p(out, _u64p))
        return out

    def rlk_error(self, j):
        e = np.zeros(self.n, dtype=np.int64)
        lib().orc_rlk_error(self._h, int(j), _p(e, _i64p))
        return e

    def enc_error(self, seed, operand, i, j):
        e = np.zeros(self.n, dtype=np.int64)
        lib().orc_enc_error(self._h, ctypes.c_uint64(seed), ctypes.c_uint64(operand),
                            ctypes.c_uint64(i), ctypes.c_uint64(j), _p(e, _i64p))
        return e

    def encrypt(self, z, seed, operand, i, j):
        ct = np.zeros((2, self.L, self.n), dtype=np.uint64)
        rc = lib().orc_encrypt(self._h, float(z), ctypes.c_uint64(seed), ctypes.c_uint64(operand),
                               ctypes.c_uint64(i), ctypes.c_uint64(j), _p(ct, _u64p))
        if rc != 0:
            raise ValueError("encrypt failed")
        return ct

    # ---- homomorphic steps (coefficient domain) ------------------------
    def tensor(self, level, a, b):
        nl = level + 1
        a = _u64(a); b = _u64(b)
        d = np.zeros((3, nl, self.n), dtype=np.uint64)
        lib().orc_tensor(self._h, int(level), _p(a, _u64p), _p(b, _u64p), _p(d, _u64p))
        return d

    def keyswitch(self, level, d2):
        nl = level + 1
        d2 = _u64(d2)
        out = np.zeros((2, nl, self.n), dtype=np.uint64)
        lib().orc_keyswitch(self._h, int(level), _p(d2, _u64p), _p(out, _u64p))
        return out

    def modup(self, level, j, d2):
        d2 = _u64(d2)
        out = np.zeros((level + 1 + self.alpha, self.n), dtype=np.uint64)
        lib().orc_modup(self._h, int(level), int(j), _p(d2, _u64p), _p(out, _u64p))
        return out

    def moddown(self, level, acc):
        acc = _u64(acc)
        out = np.zeros((level + 1, self.n), dtype=np.uint64)
        lib().orc_moddown(self._h, int(level), _p(acc, _u64p), _p(out, _u64p))
        return out

    def crt_centered(self, residues):
        v = _u64(residues)
        return float(lib().orc_crt_centered(self._h, len(v), _p(v, _u64p), 1))

    def rescale(self, level, ct):
        ct = _u64(ct)
        out = np.zeros((2, level, self.n), dtype=np.uint64)
        lib().orc_rescale(self._h, int(level), _p(ct, _u64p), _p(out, _u64p))
        return out

    def decrypt_poly(self, level, ct):
        ct = _u64(ct)
        m = np.zeros((level + 1, self.n), dtype=np.uint64)
        lib().orc_decrypt_poly(self._h, int(level), _p(ct, _u64p), _p(m, _u64p))
        return m

    def decrypt(self, level, ct, scale):
        ct = _u64(ct)
        return lib().orc_decrypt(self._h, int(level), _p(ct, _u64p), float(scale))

    def out_scale(self):
        """Scale of a product after one rescale: Delta^2 / q_{L-1}."""
        return 2.0 ** (2 * self.log2_scale) / float(self.q[-1])

    # ---- matmul -------------------------------------------------------
    def row_ks(self, A, enc, i):
        A = np.ascontiguousarray(A, dtype=np.float64)
        M, K = A.shape
        ks = np.zeros(K + 1, dtype=np.int32)
        n = lib().orc_row_ks(_p(A, _f64p), M, K, ENC[enc], int(i), _p(ks, _i32p))
        return ks[:n].copy()

    def matmul(self, A, B, enc, sched, seedA, seedB, outputs=None, threads=1,
               opA=0, opB=1, decrypt=True, encB="dense"):
        """Selected outputs of the encrypted product.  Returns (cts, vals, seconds):
        cts[n] = [2][L-1][N] coefficient-domain residues of output `outputs[n]`.
        encB is the right operand's encoding: a sparse one skips its zeros too."""
        A = np.ascontiguousarray(A, dtype=np.float64)
        B = np.ascontiguousarray(B, dtype=np.float64)
        M, K = A.shape
        K2, Nc = B.shape
        assert K == K2
        if outputs is None:
            outputs = [(i, j) for i in range(M) for j in range(Nc)]
        rows = np.asarray([o[0] for o in outputs], dtype=np.int32)
        cols = np.asarray([o[1] for o in outputs], dtype=np.int32)
        nout = len(outputs)
        out = np.zeros((nout, 2, self.L - 1, self.n), dtype=np.uint64)
        vals = np.zeros(nout, dtype=np.float64)
        secs = np.zeros(1, dtype=np.float64)
        rc = lib().orc_matmul2(self._h, _p(A, _f64p), M, K, _p(B, _f64p), Nc, ENC[enc], ENC[encB], SCHED[sched],
                              ctypes.c_uint64(seedA), ctypes.c_uint64(opA), ctypes.c_uint64(seedB),
                              ctypes.c_uint64(opB), _p(rows, _i32p), _p(cols, _i32p), nout,
                              int(threads), _p(out, _u64p),
                              _p(vals, _f64p) if decrypt else None, _p(secs, _f64p))
        if rc != 0:
            raise ValueError("oracle matmul failed (%d)" % rc)
        return out, (vals if decrypt else None), float(secs[0])

    # ---- plaintext weights times encrypted values (Sec. 3.3.2) ----------
    def matmul_plain(self, W, B, enc, seedB, log2_scale_w=40, outputs=None, threads=1, opB=1, decrypt=True):
        """Selected outputs of W B for plaintext weights W (constant-polynomial
        encoding at scale 2^log2_scale_w) and B encrypted per element.  Returns
        (cts, vals, seconds) as matmul() does; the decryption scale is
        2^log2_scale_w * Delta / q_{L-1}."""
        W = np.ascontiguousarray(W, dtype=np.float64)
        B = np.ascontiguousarray(B, dtype=np.float64)
        M, K = W.shape
        K2, Nc = B.shape
        assert K == K2
        if outputs is None:
            outputs = [(i, j) for i in range(M) for j in range(Nc)]
        rows = np.asarray([o[0] for o in outputs], dtype=np.int32)
        cols = np.asarray([o[1] for o in outputs], dtype=np.int32)
        nout = len(outputs)
        out = np.zeros((nout, 2, self.L - 1, self.n), dtype=np.uint64)
        vals = np.zeros(nout, dtype=np.float64)
        secs = np.zeros(1, dtype=np.float64)
        rc = lib().orc_matmul_plain(self._h, _p(W, _f64p), M, K, _p(B, _f64p), Nc, ENC[enc], float(log2_scale_w),
                                    ctypes.c_uint64(seedB), ctypes.c_uint64(opB), _p(rows, _i32p), _p(cols, _i32p),
                                    nout, int(threads), _p(out, _u64p), _p(vals, _f64p) if decrypt else None,
                                    _p(secs, _f64p))
        if rc != 0:
            raise ValueError("oracle plaintext-weight matmul failed (%d)" % rc)
        return out, (vals if decrypt else None), float(secs[0])

    def plain_out_scale(self, log2_scale_w=40):
        """Scale of a plaintext-weight product after its rescale."""
        return 2.0 ** (log2_scale_w + self.log2_scale) / float(self.q[-1])

    # ---- chunks of several values per ciphertext (Sec. 3.2, R10) ----------
    def galois(self, r):
        return int(lib().orc_galois(self._h, int(r)))

    def encode_slots(self, z):
        z = np.ascontiguousarray(z, dtype=np.float64)
        m = np.zeros(self.n, dtype=np.int64)
        if lib().orc_encode_slots(self._h, _p(z, _f64p), len(z), _p(m, _i64p)) != 0:
            raise ValueError("values do not fit")
        return m

    def decrypt_slot(self, level, ct, scale, slot):
        ct = _u64(ct)
        return lib().orc_decrypt_slot(self._h, int(level), _p(ct, _u64p), float(scale), int(slot))

    def automorphism(self, a, g):
        a = _u64(a)
        out = np.zeros_like(a)
        lib().orc_automorphism(self._h, a.shape[0], _p(a, _u64p), ctypes.c_uint64(g), _p(out, _u64p))
        return out

    def rotkey(self, g):
        nb = self.L + self.alpha
        key = np.zeros((self.dnum, 2, nb, self.n), dtype=np.uint64)
        e = np.zeros((self.dnum, self.n), dtype=np.int64)
        lib().orc_rotkey(self._h, ctypes.c_uint64(g), _p(key, _u64p), _p(e, _i64p))
        return key, e

    def rotate(self, level, ct, r):
        ct = _u64(ct)
        out = np.zeros_like(ct)
        if lib().orc_rotate(self._h, int(level), _p(ct, _u64p), int(r), _p(out, _u64p)) != 0:
            raise ValueError("rotate failed")
        return out

    def encrypt_slots(self, z, seed, operand, chunk):
        z = np.ascontiguousarray(z, dtype=np.float64)
        ct = np.zeros((2, self.L, self.n), dtype=np.uint64)
        if lib().orc_encrypt_slots(self._h, _p(z, _f64p), len(z), ctypes.c_uint64(seed), ctypes.c_uint64(operand),
                                   ctypes.c_uint64(chunk), _p(ct, _u64p)) != 0:
            raise ValueError("encrypt failed")
        return ct

    def chunked_scale(self):
        """Scale of a chunked product's result: Delta^3 / (q_{L-1} q_{L-2})."""
        return 2.0 ** (3 * self.log2_scale) / float(self.q[-1]) / float(self.q[-2])

    def matmul_chunked(self, A, B, enc, sched, chunk, seedA, seedB, outputs=None, opA=0, opB=1, decrypt=True):
        """Algorithm 1 at chunk size `chunk`: (result chunks [n][2][L-3][N], values of
        the listed outputs or None)."""
        A = np.ascontiguousarray(A, dtype=np.float64)
        B = np.ascontiguousarray(B, dtype=np.float64)
        M, K = A.shape
        K2, Nc = B.shape
        assert K == K2
        if outputs is None:
            outputs = [(i, j) for i in range(M) for j in range(Nc)]
        rows = np.asarray([o[0] for o in outputs], dtype=np.int32)
        cols = np.asarray([o[1] for o in outputs], dtype=np.int32)
        nchunks = (M * Nc + chunk - 1) // chunk
        out = np.zeros((nchunks, 2, self.L - 2, self.n), dtype=np.uint64)
        vals = np.zeros(len(outputs), dtype=np.float64)
        rc = lib().orc_matmul_chunked(self._h, _p(A, _f64p), M, K, _p(B, _f64p), Nc, ENC[enc], SCHED[sched], int(chunk),
                                      ctypes.c_uint64(seedA), ctypes.c_uint64(opA), ctypes.c_uint64(seedB),
                                      ctypes.c_uint64(opB), _p(rows, _i32p), _p(cols, _i32p), len(outputs),
                                      _p(out, _u64p), _p(vals, _f64p) if decrypt else None)
        if rc != 0:
            raise ValueError("oracle chunked matmul failed (%d)" % rc)
        return out, (vals if decrypt else None)


def weight(w, log2_scale_w):
    """The constant-polynomial coefficient of weight w (None if it does not fit)."""
    m = np.zeros(1, dtype=np.int64)
    if lib().orc_weight(float(w), float(log2_scale_w), _p(m, _i64p)) != 0:
        return None
    return int(m[0])


def stream_word(seed, tag, fields, n):
    f = np.asarray(list(fields) + [0], dtype=np.uint64)
    return int(lib().orc_stream_word(ctypes.c_uint64(seed), ctypes.c_uint64(tag), len(fields),
                                     _p(f, _u64p), ctypes.c_uint64(n)))


def is_prime(n):
    return bool(lib().orc_is_prime(ctypes.c_uint64(n)))
