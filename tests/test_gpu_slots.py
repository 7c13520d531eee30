"""GPU parity of several values per ciphertext (Sec. 3.2) and Algorithm 1
with its rotations and slot-zero mask (Sec. 3.3.1): chunk encryption,
rotations and the whole product, against the CPU oracle on the same seeded
inputs, bit for bit in the coefficient domain; decrypted values against the
fp64 product.  Every call goes through the C ABI."""
import numpy as np
import pytest

from paper_2503_09184_amd import workloads as W
from tests.test_gpu_parity import HYB_SMALL, note, pair, torch_cuda  # noqa: F401

pytestmark = pytest.mark.gpu


def _stored_values(M, enc):
    """Stored value list of an encoding: row-major for dense and naive sparse,
    the nonzeros in row order for CSR, rows x width for ELLPACK (pads 0)."""
    if enc in ("dense", "naive"):
        return M.ravel().copy()
    if enc == "csr":
        return M[M != 0.0].copy()
    w = max(int(np.count_nonzero(r)) for r in M)
    out = np.zeros((M.shape[0], w))
    for i, r in enumerate(M):
        nz = r[r != 0.0]
        out[i, :len(nz)] = nz
    return out.ravel()


@pytest.mark.parametrize("enc,cs", [("csr", 4), ("ell", 3), ("dense", 64), ("naive", 1)])
def test_encrypt_slots_chunks_match_oracle(torch_cuda, enc, cs):
    """Every chunk of the stored values, bit for bit; the last chunk ragged."""
    ctx, orc = pair(HYB_SMALL, 21)
    A, _ = W.operands(7, 9, 2, 0.5, 31)
    note("encrypt slots %s cs=%d" % (enc, cs))
    EA = ctx.encrypt_slots(A, enc, cs, 41, 0)
    v = _stored_values(A, enc)
    info = EA.info()
    assert info.slots == cs and info.n_ciphertexts == (len(v) + cs - 1) // cs
    for x in range(info.n_ciphertexts):
        want = orc.encrypt_slots(v[x * cs:(x + 1) * cs], 41, 0, x)
        assert np.array_equal(ctx.export_stored(EA, x), want), x
    assert np.max(np.abs(ctx.decrypt(EA) - A)) < 1e-6


@pytest.mark.parametrize("name,r", [("hyb_small", 1), ("hyb_small", -3), ("hyb_small", 512),
                                    ("realistic_n16384", 5), ("serving_n32768", -2)])
def test_rotate_matches_oracle(torch_cuda, name, r):
    """A rotation of a chunk through the C ABI (NTT domain in the library's
    storage order) equals the oracle's, bit for bit; r = N/2 is the identity."""
    P = HYB_SMALL if name == "hyb_small" else W.PARAMS[name]
    ctx, orc = pair(P, 22)
    L = len(ctx.primes) - ctx.alpha
    z = W.uniform_matrix(1, 6, 5)[0]
    note("rotate %s r=%d" % (name, r))
    E = ctx.encrypt_slots(z[None, :], "dense", 8, 77, 0)
    ct = ctx.export_stored(E, 0)
    assert np.array_equal(ct, orc.encrypt_slots(z, 77, 0, 0))
    t = ctx.to_device(ct)
    ctx.ntt(t, L, 0)                                  # both polys: rows mod q_0 .. q_{L-1}
    rot = ctx.rotate(L - 1, t, r)
    ctx.ntt(rot, L, 0, inverse=True)
    got = ctx.to_host(rot).reshape(2, L, ctx.n)
    if r == ctx.n // 2:
        assert np.array_equal(got, ct)
    else:
        assert np.array_equal(got, orc.rotate(L - 1, ct, r))


def _check_product(ctx, orc, A, B, enc, sched, cs, sa, sb, outputs=None):
    M, K = A.shape
    Nc = B.shape[1]
    EA = ctx.encrypt_slots(A, enc, cs, sa, 0)
    EB = ctx.encrypt_slots(B, "dense", cs, sb, 1)
    C = ctx.matmul_slots(EA, EB, sched)
    info = C.info()
    st = ctx.last_stats()
    assert info.level == len(ctx.primes) - ctx.alpha - 3 and info.slots == cs
    assert info.n_ciphertexts == (M * Nc + cs - 1) // cs
    products = sum(int(np.count_nonzero(A[i])) if enc != "dense" else K for i in range(M)) * Nc
    assert st.products == products
    out, vals = orc.matmul_chunked(A, B, enc, sched, cs, sa, sb, outputs=outputs)
    if outputs is None:
        chunks = range(info.n_ciphertexts)
    else:
        chunks = sorted({(i * Nc + j) // cs for i, j in outputs})
    for x in chunks:
        assert np.array_equal(ctx.export_stored(C, x), out[x]), x
    dec = ctx.decrypt(C)
    assert abs(info.scale - orc.chunked_scale()) == 0.0
    assert np.max(np.abs(dec - A @ B)) < 1e-6
    if outputs is None:
        assert np.max(np.abs(dec.ravel() - vals)) < 1e-9
    return C


@pytest.mark.parametrize("sched", ["lazy", "per_product"])
@pytest.mark.parametrize("enc,cs", [("csr", 4), ("ell", 3), ("naive", 4), ("dense", 5), ("csr", 1)])
def test_matmul_slots_matches_oracle(torch_cuda, enc, cs, sched):
    """5 x 6 x 3 with an empty row: every result chunk bit for bit (the last
    one ragged), decrypted values against the fp64 product."""
    ctx, orc = pair(HYB_SMALL, 21)
    A, B = W.operands(5, 6, 3, 0.5, 61)
    A[2, :] = 0.0
    note("matmul slots %s cs=%d %s" % (enc, cs, sched))
    _check_product(ctx, orc, A, B, enc, sched, cs, 71, 72)


@pytest.mark.parametrize("sched", ["lazy", "per_product"])
def test_matmul_slots_realistic_sampled_chunks(torch_cuda, sched):
    """N = 2^14 with the benchmarked primes, 8 values per ciphertext: two
    result chunks (all of their outputs) bit for bit against the oracle."""
    ctx, orc = pair(W.PARAMS["realistic_n16384"], W.key_seed(3))
    A, B = W.operands(8, 8, 4, 0.5, 62)
    outs = [(i, j) for i in range(8) for j in range(4) if (i * 4 + j) // 8 in (1, 3)]
    note("matmul slots realistic %s" % sched)
    _check_product(ctx, orc, A, B, "csr", sched, 8, 73, 74, outputs=outs)


def test_matmul_slots_errors(torch_cuda):
    from paper_2503_09184_amd import sfhe
    ctx, _ = pair(HYB_SMALL, 21)
    A, B = W.operands(3, 4, 2, 0.5, 63)
    EA = ctx.encrypt_slots(A, "csr", 4, 1, 0)
    EB = ctx.encrypt_slots(B, "dense", 4, 2, 1)
    for call, code in [(lambda: ctx.matmul_slots(EA, ctx.encrypt_slots(B, "dense", 2, 2, 1), "lazy"), -3),
                       (lambda: ctx.matmul_slots(EA, ctx.encrypt_slots(B, "csr", 4, 2, 1), "lazy"), -6),
                       (lambda: ctx.matmul(EA, EB, "lazy"), -6),
                       (lambda: ctx.export_ct(EA, 0, 0), -6),
                       (lambda: ctx.export_stored(EA, 99), -3),
                       (lambda: ctx.encrypt_slots(A, "csr", 65, 1, 0), -1)]:
        with pytest.raises(sfhe.SfheError) as e:
            call()
        assert e.value.code == code
    small, _ = pair(dict(log_n=10, q_bits=[60, 40, 40], p_bits=[60], dnum=3), 5)
    with pytest.raises(sfhe.SfheError) as e:
        small.matmul_slots(small.encrypt_slots(A, "csr", 2, 1, 0), small.encrypt_slots(B, "dense", 2, 2, 1), "lazy")
    assert e.value.code == -4


def test_matmul_slots_benchmarked_size(torch_cuda):
    """The benchmarked product with 8 values per ciphertext (128 x 128 x 128,
    N = 2^14, CSR at 50%, LAZY, the same calls as the bench leg): every one
    of the 16384 outputs decrypts within 1e-6 of the fp64 product, the counts
    of products, rotations and result ciphertexts are the method's, and the
    result ciphertexts of a repeated call are identical."""
    ctx, _ = pair(W.PARAMS["realistic_n16384"], W.key_seed(3))
    A, B = W.operands(128, 128, 128, 0.5, W.workload_seed(3))
    sa, sb = W.enc_seed(3, 0), W.enc_seed(3, 1)
    note("matmul slots 128^3 c=8")
    EA = ctx.encrypt_slots(A, "csr", 8, sa, 0)
    EB = ctx.encrypt_slots(B, "dense", 8, sb, 1)
    C = ctx.matmul_slots(EA, EB, "lazy")
    st = ctx.last_stats()
    nnz = int(np.count_nonzero(A))
    assert st.products == nnz * 128
    # rotations: stored values off slot 0 (A's nonzeros, all of B), then one per output off slot 0
    rot = (nnz - (nnz + 7) // 8) + (128 * 128 - 128 * 128 // 8) + (128 * 128 - 128 * 128 // 8)
    assert st.keyswitches == 128 * 128 + rot
    assert C.info().n_ciphertexts == 2048
    assert np.max(np.abs(ctx.decrypt(C) - A @ B)) < 1e-6
    C2 = ctx.matmul_slots(EA, EB, "lazy")
    for x in (0, 777, 2047):
        assert np.array_equal(ctx.export_stored(C, x), ctx.export_stored(C2, x))


@pytest.mark.parametrize("sched", ["lazy", "per_product"])
def test_matmul_slots_degenerate(torch_cuda, sched):
    """An all-zero A in CSR (no stored value, no product: the result chunks
    stay trivial zeros) and a 1 x 1 x 1 product with 4 slots per ciphertext
    (one value in a chunk of four), against the oracle."""
    ctx, orc = pair(HYB_SMALL, 21)
    A = np.zeros((3, 4))
    _, B = W.operands(3, 4, 2, 0.5, 65)
    note("matmul slots all-zero A %s" % sched)
    EA = ctx.encrypt_slots(A, "csr", 4, 1, 0)
    assert EA.info().n_ciphertexts == 0
    C = ctx.matmul_slots(EA, ctx.encrypt_slots(B, "dense", 4, 2, 1), sched)
    assert ctx.last_stats().products == 0
    for x in range(C.info().n_ciphertexts):
        assert not np.any(ctx.export_stored(C, x))
    assert np.all(ctx.decrypt(C) == 0.0)
    note("matmul slots 1x1x1 %s" % sched)
    A1, B1 = np.array([[0.625]]), np.array([[-0.5]])
    _check_product(ctx, orc, A1, B1, "csr", sched, 4, 81, 82)
