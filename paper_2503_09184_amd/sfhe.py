"""Python binding of the gfx950 library (ctypes over the C ABI in include/sfhe.h).

Argument marshalling only: every step of the encrypted product runs in the
library's HIP kernels.  PyTorch supplies device memory (its caching
allocator, through the library's allocation hooks) and the current stream.
Loading fails loudly when the built library is missing -- there is no
fallback path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsfhe.so")

ENC = {"dense": 0, "naive": 1, "csr": 2, "ell": 3}
SCHED = {"per_product": 0, "lazy": 1}

ERRORS = {
    -1: "SFHE_E_INVALID_ARG", -2: "SFHE_E_PARAMS", -3: "SFHE_E_SHAPE", -4: "SFHE_E_LEVEL",
    -5: "SFHE_E_SCALE", -6: "SFHE_E_UNSUPPORTED", -7: "SFHE_E_NOMEM", -8: "SFHE_E_DEVICE",
    -9: "SFHE_E_STATE", -10: "SFHE_E_DECRYPT",
}

EXPORTED = [
    "sfhe_ctx_create", "sfhe_ctx_destroy", "sfhe_ctx_n", "sfhe_ctx_primes", "sfhe_keygen",
    "sfhe_encrypt_matrix", "sfhe_matmul", "sfhe_decrypt_matrix", "sfhe_export_ct",
    "sfhe_matrix_info", "sfhe_last_stats", "sfhe_set_profiling", "sfhe_mat_destroy", "sfhe_last_error",
    "sfhe_ntt", "sfhe_tensor", "sfhe_keyswitch", "sfhe_rescale",
    "sfhe_encode_matrix", "sfhe_matmul_plain", "sfhe_matmul_plain_batch",
    "sfhe_server_create", "sfhe_server_submit", "sfhe_server_step", "sfhe_server_poll", "sfhe_server_status",
    "sfhe_server_destroy", "sfhe_plain_graph_create", "sfhe_plain_graph_launch", "sfhe_plain_graph_result",
    "sfhe_plain_graph_destroy", "sfhe_encrypt_matrix_slots", "sfhe_matmul_slots", "sfhe_export_stored",
    "sfhe_rotate", "sfhe_ntt_tuning", "sfhe_set_ntt_variant", "sfhe_keyswitch_noalloc",
    "sfhe_probe_valu", "sfhe_server_request_bytes", "sfhe_server_set_slots", "sfhe_server_set_batch_bytes",
    "sfhe_ks_tuning", "sfhe_set_ks_slice",
    "sfhe_matmul_graph_create", "sfhe_matmul_graph_launch", "sfhe_matmul_graph_result", "sfhe_matmul_graph_destroy",
]

PLAIN_LAUNCH = {"fused": 0, "per_product": 1}


PROBE_KINDS = {"fp64_fma": 0, "mad_u64_u32": 1, "int32_add": 2}


def probe_valu(kind):
    """Sustained lane operations per second of one VALU instruction class
    (sfhe_probe_valu): "fp64_fma", "mad_u64_u32" or "int32_add"."""
    out = ctypes.c_double()
    _check(lib().sfhe_probe_valu(PROBE_KINDS[kind], ctypes.byref(out)))
    return out.value


class SfheError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("n_q", ctypes.c_uint32), ("n_p", ctypes.c_uint32),
                ("dnum", ctypes.c_uint32), ("q_bits", ctypes.POINTER(ctypes.c_uint32)),
                ("p_bits", ctypes.POINTER(ctypes.c_uint32)), ("log2_scale", ctypes.c_double),
                ("sigma", ctypes.c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class Hooks(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


class MatInfo(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("cols", ctypes.c_int32), ("level", ctypes.c_int32),
                ("scale", ctypes.c_double), ("enc", ctypes.c_int), ("n_ciphertexts", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("ell_width", ctypes.c_int32), ("device_bytes", ctypes.c_uint64),
                ("slots", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("products", ctypes.c_int64), ("keyswitches", ctypes.c_int64),
                ("outputs", ctypes.c_int64), ("tensor_ms", ctypes.c_double), ("keyswitch_ms", ctypes.c_double),
                ("rescale_ms", ctypes.c_double), ("tensor_launches", ctypes.c_int64),
                ("tensor_fp_ms", ctypes.c_double), ("tensor_fp_launches", ctypes.c_int64),
                ("tensor_fp_primes", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsfhe.so is not built (run __graft_entry__.build()); no fallback exists")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        L.sfhe_ctx_create.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Hooks), ctypes.POINTER(vp)]
        L.sfhe_ctx_destroy.argtypes = [vp]
        L.sfhe_ctx_destroy.restype = None
        L.sfhe_ctx_n.argtypes = [vp, ctypes.POINTER(i32)]
        L.sfhe_ctx_primes.argtypes = [vp, ctypes.POINTER(u64), ctypes.c_size_t]
        L.sfhe_keygen.argtypes = [vp, u64]
        L.sfhe_encrypt_matrix.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32, i32, i64, ctypes.c_int, u64,
                                          ctypes.c_uint32, vp, ctypes.POINTER(vp)]
        L.sfhe_matmul.argtypes = [vp, vp, vp, ctypes.c_int, vp, ctypes.POINTER(vp)]
        L.sfhe_decrypt_matrix.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double), i64, vp]
        L.sfhe_export_ct.argtypes = [vp, vp, i32, i32, ctypes.POINTER(u64), ctypes.c_size_t, vp]
        L.sfhe_matrix_info.argtypes = [vp, ctypes.POINTER(MatInfo)]
        L.sfhe_last_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.sfhe_set_profiling.argtypes = [vp, i32]
        L.sfhe_mat_destroy.argtypes = [vp]
        L.sfhe_mat_destroy.restype = None
        L.sfhe_last_error.restype = ctypes.c_char_p
        L.sfhe_ntt.argtypes = [vp, vp, i32, i32, i32, i32, vp]
        L.sfhe_tensor.argtypes = [vp, i32, vp, vp, vp, i32, vp]
        L.sfhe_keyswitch.argtypes = [vp, i32, vp, vp, i32, vp]
        L.sfhe_keyswitch_noalloc.argtypes = [vp, i32, vp, vp, i32, vp]
        L.sfhe_probe_valu.argtypes = [i32, ctypes.POINTER(ctypes.c_double)]
        L.sfhe_rescale.argtypes = [vp, i32, vp, vp, i32, vp]
        L.sfhe_encode_matrix.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32, i32, i64, ctypes.c_int, i32,
                                         ctypes.POINTER(vp)]
        L.sfhe_matmul_plain.argtypes = [vp, vp, vp, vp, ctypes.POINTER(vp)]
        L.sfhe_matmul_plain_batch.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int, vp,
                                              ctypes.POINTER(vp)]
        L.sfhe_server_create.argtypes = [vp, u64, i32, vp, ctypes.POINTER(vp)]
        L.sfhe_server_set_slots.argtypes = [vp, i32]
        L.sfhe_server_set_batch_bytes.argtypes = [vp, ctypes.c_uint64]
        L.sfhe_server_submit.argtypes = [vp, vp, vp, ctypes.POINTER(i64)]
        L.sfhe_server_request_bytes.argtypes = [vp, vp, vp, ctypes.POINTER(u64)]
        L.sfhe_server_step.argtypes = [vp, ctypes.POINTER(i32)]
        L.sfhe_server_poll.argtypes = [vp, i64, i32, ctypes.POINTER(i32), ctypes.POINTER(vp),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.sfhe_server_status.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(u64),
                                         ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.sfhe_server_destroy.argtypes = [vp]
        L.sfhe_server_destroy.restype = None
        L.sfhe_plain_graph_create.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int, vp,
                                              ctypes.POINTER(vp)]
        L.sfhe_plain_graph_launch.argtypes = [vp, vp]
        L.sfhe_plain_graph_result.argtypes = [vp, i32, ctypes.POINTER(vp)]
        L.sfhe_plain_graph_destroy.argtypes = [vp]
        L.sfhe_plain_graph_destroy.restype = None
        L.sfhe_matmul_graph_create.argtypes = [vp, vp, vp, vp, ctypes.POINTER(vp)]
        L.sfhe_matmul_graph_launch.argtypes = [vp, vp]
        L.sfhe_matmul_graph_result.argtypes = [vp, ctypes.POINTER(vp)]
        L.sfhe_matmul_graph_destroy.argtypes = [vp]
        L.sfhe_matmul_graph_destroy.restype = None
        L.sfhe_encrypt_matrix_slots.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32, i32, i64, ctypes.c_int, i32,
                                                u64, ctypes.c_uint32, vp, ctypes.POINTER(vp)]
        L.sfhe_matmul_slots.argtypes = [vp, vp, vp, ctypes.c_int, vp, ctypes.POINTER(vp)]
        L.sfhe_export_stored.argtypes = [vp, vp, i64, ctypes.POINTER(u64), ctypes.c_size_t, vp]
        L.sfhe_rotate.argtypes = [vp, i32, vp, vp, i32, i32, vp]
        L.sfhe_ntt_tuning.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double), i32]
        L.sfhe_set_ntt_variant.argtypes = [vp, i32, i32]
        L.sfhe_ks_tuning.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                     ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(i32),
                                     ctypes.POINTER(ctypes.c_double)]
        L.sfhe_set_ks_slice.argtypes = [vp, i32, i32]
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise SfheError(rc, lib().sfhe_last_error().decode())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Matrix:
    """An encrypted matrix (library handle)."""

    def __init__(self, ctx, handle):
        self.ctx = ctx
        self._h = handle

    @property
    def handle(self):
        return self._h

    def info(self):
        out = MatInfo()
        _check(lib().sfhe_matrix_info(self._h, ctypes.byref(out)))
        return out

    def close(self):
        if self._h is not None and self._h.value:
            lib().sfhe_mat_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Borrowed(Matrix):
    """A matrix handle owned by another object (never destroyed here)."""

    def close(self):
        self._h = None


class PlainGraph:
    """A plaintext-weight batch captured into a HIP graph (library handle)."""

    def __init__(self, ctx, Ws, Bs, launch="fused", stream=None):
        self.ctx = ctx
        self._keep = (list(Ws), list(Bs))
        n = len(Ws)
        wh = (ctypes.c_void_p * n)(*[W.handle.value for W in Ws])
        bh = (ctypes.c_void_p * n)(*[B.handle.value for B in Bs])
        h = ctypes.c_void_p()
        _check(lib().sfhe_plain_graph_create(ctx._h, n, wh, bh, PLAIN_LAUNCH[launch], _stream_handle(stream),
                                             ctypes.byref(h)))
        self._h = h
        self.count = n

    def launch(self, stream=None):
        _check(lib().sfhe_plain_graph_launch(self._h, _stream_handle(stream)))

    def result(self, n):
        h = ctypes.c_void_p()
        _check(lib().sfhe_plain_graph_result(self._h, int(n), ctypes.byref(h)))
        return _Borrowed(self.ctx, h)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sfhe_plain_graph_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MatmulGraph:
    """A LAZY ct x ct product captured into a HIP graph (library handle)."""

    def __init__(self, ctx, A, B, stream=None):
        self.ctx = ctx
        self._keep = (A, B)
        h = ctypes.c_void_p()
        _check(lib().sfhe_matmul_graph_create(ctx._h, A.handle, B.handle, _stream_handle(stream), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(lib().sfhe_matmul_graph_launch(self._h, _stream_handle(stream)))

    def result(self):
        h = ctypes.c_void_p()
        _check(lib().sfhe_matmul_graph_result(self._h, ctypes.byref(h)))
        return _Borrowed(self.ctx, h)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sfhe_matmul_graph_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The library's request loop over plaintext-weight products (a handle)."""

    def __init__(self, ctx, budget_bytes, stream=None, n_streams=1, slots=0, batch_bytes=0):
        """n_streams: the server's streams (1: batches run in admission
        order); slots: running batches a stream may hold (0: no limit);
        batch_bytes: bytes one batch may hold (0: no limit)."""
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(lib().sfhe_server_create(ctx._h, ctypes.c_uint64(int(budget_bytes)), int(n_streams),
                                        _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        if slots:
            self.set_slots(slots)
        if batch_bytes:
            self.set_batch_bytes(batch_bytes)
        self.intervals = {}   # ticket -> (start_ms, end_ms) of its batch on the device

    def set_slots(self, per_stream):
        """at most per_stream running batches per server stream (0: no limit)"""
        _check(lib().sfhe_server_set_slots(self._h, int(per_stream)))

    def set_batch_bytes(self, max_bytes):
        """at most max_bytes in one batch (0: no limit)"""
        _check(lib().sfhe_server_set_batch_bytes(self._h, ctypes.c_uint64(int(max_bytes))))

    def request_bytes(self, W, X):
        """Device bytes counted for request W X against the budget."""
        out = ctypes.c_uint64()
        _check(lib().sfhe_server_request_bytes(self.ctx._h, W.handle, X.handle, ctypes.byref(out)))
        return out.value

    def submit(self, W, X):
        t = ctypes.c_int64()
        _check(lib().sfhe_server_submit(self._h, W.handle, X.handle, ctypes.byref(t)))
        return t.value

    def step(self):
        n = ctypes.c_int32()
        _check(lib().sfhe_server_step(self._h, ctypes.byref(n)))
        return n.value

    def poll(self, ticket, wait=False):
        """(done, result Matrix or None, batch device ms, batch size); the
        batch's device-time interval is kept in self.intervals[ticket]."""
        d = ctypes.c_int32()
        h = ctypes.c_void_p()
        ms = ctypes.c_double()
        bs = ctypes.c_int32()
        t0, t1 = ctypes.c_double(), ctypes.c_double()
        _check(lib().sfhe_server_poll(self._h, int(ticket), 1 if wait else 0, ctypes.byref(d), ctypes.byref(h),
                                      ctypes.byref(ms), ctypes.byref(bs), ctypes.byref(t0), ctypes.byref(t1)))
        if not d.value:
            return False, None, 0.0, 0
        self.intervals[int(ticket)] = (t0.value, t1.value)
        return True, Matrix(self.ctx, h), ms.value, bs.value

    def status(self):
        q, r, b, n, p = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_uint64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().sfhe_server_status(self._h, ctypes.byref(q), ctypes.byref(r), ctypes.byref(b), ctypes.byref(n),
                                        ctypes.byref(p)))
        return {"queued": q.value, "running": r.value, "bytes_in_flight": b.value, "batches": n.value,
                "products": p.value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sfhe_server_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """Parameters, tables and keys on the current device."""

    def __init__(self, log_n, q_bits, p_bits, dnum, log2_scale=40.0, sigma=3.2, torch_allocator=True, hooks=None):
        """torch_allocator: take device memory from torch's caching allocator
        (stream-ordered: a block is taken and given back on the stream of the
        library call that uses it); False: the library's own stream-ordered
        pool.  hooks: optional (alloc(nbytes, stream) -> ptr or 0,
        free(ptr, nbytes, stream)) replacing torch's allocator; stream is the
        raw hipStream_t as an int (0 = the default stream)."""
        import torch
        self._torch = torch
        self.device = torch.cuda.current_device()
        qb = (ctypes.c_uint32 * len(q_bits))(*q_bits)
        pb = (ctypes.c_uint32 * len(p_bits))(*p_bits)
        self._params = Params(int(log_n), len(q_bits), len(p_bits), int(dnum), qb, pb, float(log2_scale), float(sigma))
        self._keep = [qb, pb]
        hooks_p = None
        if hooks is not None or torch_allocator:
            dev = self.device
            if hooks is None:
                # bound now: at interpreter exit the torch module's attributes
                # may be gone before the context is destroyed
                t_alloc = torch.cuda.caching_allocator_alloc
                t_free = torch._C._cuda_cudaCachingAllocator_raw_delete

                def user_alloc(nbytes, stream):
                    return t_alloc(int(nbytes), dev, int(stream))

                def user_free(ptr, nbytes, stream):
                    t_free(ptr)
            else:
                user_alloc, user_free = hooks

            def _alloc(nbytes, stream, user):
                try:
                    return user_alloc(int(nbytes), int(stream or 0)) or None
                except Exception:
                    return None

            def _free(ptr, nbytes, stream, user):
                user_free(ptr, int(nbytes), int(stream or 0))

            self._alloc_cb = ALLOC_FN(_alloc)
            self._free_cb = FREE_FN(_free)
            self._hooks = Hooks(self._alloc_cb, self._free_cb, None)
            hooks_p = ctypes.byref(self._hooks)
        h = ctypes.c_void_p()
        _check(lib().sfhe_ctx_create(ctypes.byref(self._params), hooks_p, ctypes.byref(h)))
        self._h = h
        n = ctypes.c_int32()
        _check(lib().sfhe_ctx_n(self._h, ctypes.byref(n)))
        self.n = n.value
        self.L = len(q_bits)
        self.alpha = len(p_bits)
        buf = (ctypes.c_uint64 * (self.L + self.alpha))()
        _check(lib().sfhe_ctx_primes(self._h, buf, self.L + self.alpha))
        self.primes = [int(x) for x in buf]
        self.log2_scale = float(log2_scale)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sfhe_ctx_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- keys, matrices --------------------------------------------------
    def keygen(self, seed):
        _check(lib().sfhe_keygen(self._h, ctypes.c_uint64(seed)))

    def encrypt(self, vals, enc, seed, operand, stream=None):
        v = np.ascontiguousarray(vals, dtype=np.float64)
        rows, cols = v.shape
        h = ctypes.c_void_p()
        _check(lib().sfhe_encrypt_matrix(self._h, v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), rows, cols,
                                         cols, ENC[enc], ctypes.c_uint64(seed), int(operand),
                                         _stream_handle(stream), ctypes.byref(h)))
        return Matrix(self, h)

    def matmul(self, A, B, sched, stream=None):
        h = ctypes.c_void_p()
        _check(lib().sfhe_matmul(self._h, A.handle, B.handle, SCHED[sched], _stream_handle(stream),
                                 ctypes.byref(h)))
        return Matrix(self, h)

    # ---- several values per ciphertext (chunks) --------------------------
    def encrypt_slots(self, vals, enc, slots, seed, operand, stream=None):
        """The stored values of `enc` in chunks of `slots` values per ciphertext."""
        v = np.ascontiguousarray(vals, dtype=np.float64)
        rows, cols = v.shape
        h = ctypes.c_void_p()
        _check(lib().sfhe_encrypt_matrix_slots(self._h, v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), rows,
                                               cols, cols, ENC[enc], int(slots), ctypes.c_uint64(seed),
                                               int(operand), _stream_handle(stream), ctypes.byref(h)))
        return Matrix(self, h)

    def matmul_slots(self, A, B, sched, stream=None):
        """Algorithm 1 with rotations and the slot-zero mask."""
        h = ctypes.c_void_p()
        _check(lib().sfhe_matmul_slots(self._h, A.handle, B.handle, SCHED[sched], _stream_handle(stream),
                                       ctypes.byref(h)))
        return Matrix(self, h)

    def export_stored(self, M, n, stream=None):
        info = M.info()
        out = np.zeros((2, info.level + 1, self.n), dtype=np.uint64)
        _check(lib().sfhe_export_stored(self._h, M.handle, int(n), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                        out.size, _stream_handle(stream)))
        return out

    def rotate(self, level, ct, r, stream=None):
        """Rotation by r slots of a device tensor [batch, 2, level+1, N] (NTT domain)."""
        nl = level + 1
        assert ct.is_contiguous()
        batch = ct.numel() // (2 * nl * self.n)
        out = self._torch.empty(batch * 2 * nl * self.n, dtype=self._torch.int64, device="cuda")
        _check(lib().sfhe_rotate(self._h, level, ctypes.c_void_p(ct.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                 batch, int(r), _stream_handle(stream)))
        return out.view(batch, 2, nl, self.n)

    # ---- plaintext weights times encrypted values -----------------------
    def encode_weights(self, vals, enc, log2_scale_w=40):
        """Plaintext weight matrix (constant-polynomial weights at scale 2^log2_scale_w)."""
        v = np.ascontiguousarray(vals, dtype=np.float64)
        rows, cols = v.shape
        h = ctypes.c_void_p()
        _check(lib().sfhe_encode_matrix(self._h, v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), rows, cols,
                                        cols, ENC[enc], int(log2_scale_w), ctypes.byref(h)))
        return Matrix(self, h)

    def matmul_plain(self, W, B, stream=None):
        h = ctypes.c_void_p()
        _check(lib().sfhe_matmul_plain(self._h, W.handle, B.handle, _stream_handle(stream), ctypes.byref(h)))
        return Matrix(self, h)

    def matmul_plain_batch(self, Ws, Bs, launch="fused", stream=None):
        n = len(Ws)
        assert len(Bs) == n
        wh = (ctypes.c_void_p * n)(*[W.handle.value for W in Ws])
        bh = (ctypes.c_void_p * n)(*[B.handle.value for B in Bs])
        out = (ctypes.c_void_p * n)()
        _check(lib().sfhe_matmul_plain_batch(self._h, n, wh, bh, PLAIN_LAUNCH[launch], _stream_handle(stream), out))
        return [Matrix(self, ctypes.c_void_p(out[x])) for x in range(n)]

    def set_profiling(self, on):
        _check(lib().sfhe_set_profiling(self._h, 1 if on else 0))

    def last_stats(self):
        s = Stats()
        _check(lib().sfhe_last_stats(self._h, ctypes.byref(s)))
        return s

    def decrypt(self, M, stream=None):
        info = M.info()
        out = np.zeros((info.rows, info.cols), dtype=np.float64)
        _check(lib().sfhe_decrypt_matrix(self._h, M.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         info.cols, _stream_handle(stream)))
        return out

    def export_ct(self, M, i, j, stream=None):
        info = M.info()
        nl = info.level + 1
        out = np.zeros((2, nl, self.n), dtype=np.uint64)
        _check(lib().sfhe_export_ct(self._h, M.handle, int(i), int(j),
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), out.size,
                                    _stream_handle(stream)))
        return out

    # ---- NTT designs ---------------------------------------------------------
    NTT_DESIGNS = ("register", "radix16", "radix8", "radix4")

    def ntt_tuning(self, inverse=False):
        """(design in use, {design: measured us per row}) for one direction."""
        v = ctypes.c_int32()
        us = (ctypes.c_double * 4)()
        _check(lib().sfhe_ntt_tuning(self._h, 1 if inverse else 0, ctypes.byref(v), us, 4))
        return self.NTT_DESIGNS[v.value], {n: us[i] for i, n in enumerate(self.NTT_DESIGNS) if us[i] >= 0}

    def ks_tuning(self):
        """(slice in use, streams in use, {one-stream slice: us per output},
        {two-stream slice: us per output})."""
        sl, st = ctypes.c_int32(), ctypes.c_int32()
        sizes, sizes2 = (ctypes.c_int32 * 6)(), (ctypes.c_int32 * 2)()
        us, us2 = (ctypes.c_double * 6)(), (ctypes.c_double * 2)()
        _check(lib().sfhe_ks_tuning(self._h, ctypes.byref(sl), ctypes.byref(st), sizes, us, 6, sizes2, us2))
        return (sl.value, st.value, {int(sizes[x]): float(us[x]) for x in range(6)},
                {int(sizes2[x]): float(us2[x]) for x in range(2)})

    def set_ks_slice(self, slice_, streams=1):
        """slice_ -1: back to the tuned setting; 0: tune again."""
        _check(lib().sfhe_set_ks_slice(self._h, int(slice_), int(streams)))

    def set_ntt_design(self, inverse, design):
        """Force a design by name, or None for the measured choice."""
        v = -1 if design is None else self.NTT_DESIGNS.index(design)
        _check(lib().sfhe_set_ntt_variant(self._h, 1 if inverse else 0, v))

    # ---- primitives on device buffers --------------------------------------
    def to_device(self, arr):
        a = np.ascontiguousarray(arr, dtype=np.uint64)
        return self._torch.from_numpy(a.view(np.int64)).to("cuda")

    @staticmethod
    def to_host(t):
        return t.cpu().numpy().view(np.uint64)

    def ntt(self, t, n_limbs, first_prime=0, inverse=False, stream=None):
        """In place on a device tensor of shape [batch, n_limbs, N] (int64 view of uint64)."""
        assert t.is_cuda and t.is_contiguous() and t.numel() % (n_limbs * self.n) == 0
        batch = t.numel() // (n_limbs * self.n)
        _check(lib().sfhe_ntt(self._h, ctypes.c_void_p(t.data_ptr()), batch, n_limbs, first_prime,
                              1 if inverse else 0, _stream_handle(stream)))
        return t

    def tensor(self, level, a, b, stream=None):
        nl = level + 1
        assert a.is_contiguous() and b.is_contiguous() and a.numel() == b.numel()
        batch = a.numel() // (2 * nl * self.n)
        d = self._torch.empty(batch * 3 * nl * self.n, dtype=self._torch.int64, device="cuda")
        _check(lib().sfhe_tensor(self._h, level, ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                 ctypes.c_void_p(d.data_ptr()), batch, _stream_handle(stream)))
        return d.view(batch, 3, nl, self.n)

    def keyswitch(self, level, d2, stream=None):
        nl = level + 1
        assert d2.is_contiguous()
        batch = d2.numel() // (nl * self.n)
        out = self._torch.empty(batch * 2 * nl * self.n, dtype=self._torch.int64, device="cuda")
        _check(lib().sfhe_keyswitch(self._h, level, ctypes.c_void_p(d2.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                    batch, _stream_handle(stream)))
        return out.view(batch, 2, nl, self.n)

    def keyswitch_noalloc(self, level, d2, out, stream=None):
        """sfhe_keyswitch_noalloc: d2 [batch, level+1, N] into the caller's
        out [batch, 2, level+1, N] (int64 device tensors); nothing is
        allocated, the library's fixed device scratch is used."""
        nl = level + 1
        assert d2.is_contiguous() and out.is_contiguous()
        batch = d2.numel() // (nl * self.n)
        assert out.numel() == batch * 2 * nl * self.n
        _check(lib().sfhe_keyswitch_noalloc(self._h, level, ctypes.c_void_p(d2.data_ptr()),
                                            ctypes.c_void_p(out.data_ptr()), batch, _stream_handle(stream)))
        return out

    def rescale(self, level, ct, stream=None):
        nl = level + 1
        assert ct.is_contiguous()
        batch = ct.numel() // (2 * nl * self.n)
        out = self._torch.empty(batch * 2 * level * self.n, dtype=self._torch.int64, device="cuda")
        _check(lib().sfhe_rescale(self._h, level, ctypes.c_void_p(ct.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  batch, _stream_handle(stream)))
        return out.view(batch, 2, level, self.n)
