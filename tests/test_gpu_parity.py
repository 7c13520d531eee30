"""GPU parity: the HIP library against the CPU oracle on the same seeded inputs.

Ciphertext residues are compared bit for bit in the coefficient domain
(integer work: exact); decrypted values against the fp64 product within the
bound the noise analysis gives.  Every call goes through the C ABI.
"""
import math
import sys

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2503_09184_amd import workloads as W

pytestmark = pytest.mark.gpu

HYB_SMALL = dict(log_n=10, q_bits=[60, 40, 40, 40, 40], p_bits=[60, 60, 60], dnum=2)
SINGLE_SMALL = dict(log_n=11, q_bits=[60, 40, 40], p_bits=[60], dnum=3)


def note(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


_ctx_cache = {}
_orc_cache = {}


def pair(params, seed):
    """(library context, oracle) with keys from the same seed."""
    from paper_2503_09184_amd import sfhe
    key = (tuple(sorted((k, tuple(v) if isinstance(v, list) else v) for k, v in params.items())), seed)
    if key not in _ctx_cache:
        note("ctx %s seed %d" % (params, seed))
        ctx = sfhe.Context(**params)
        ctx.keygen(seed)
        orc = Oracle(**params)
        orc.keygen(seed)
        _ctx_cache[key] = ctx
        _orc_cache[key] = orc
    return _ctx_cache[key], _orc_cache[key]


# ---------------------------------------------------------------- primitives
@pytest.mark.parametrize("name", list(W.PARAMS))
def test_primes_match_oracle(torch_cuda, name):
    ctx, orc = pair(W.PARAMS[name], 1)
    assert ctx.primes == [int(x) for x in orc.primes]


def ntt_storage_order(n):
    """NTT index stored at each position of a row (include/sfhe.h): the
    bit-reversed transform order itself below N = 2^14; at N = 2^14 position
    r * 512 + t holds index ((r >> 4) << 13) | ((t & 63) << 4) | (t6 << 10)
    | (t8 << 11) | (t7 << 12) | (r & 15), t6..t8 the bits of t; at N = 2^15
    each half (2^14 positions) holds its half of the indices in the N = 2^14
    order."""
    if n == 1 << 15:
        o = ntt_storage_order(1 << 14)
        return np.concatenate([o, o + (1 << 14)])
    if n != 1 << 14:
        return np.arange(n)
    order = np.zeros(n, dtype=np.int64)
    for t in range(512):
        b = lambda i: (t >> i) & 1
        c = ((t & 63) << 4) | (b(6) << 10) | (b(8) << 11) | (b(7) << 12)
        for r in range(32):
            order[r * 512 + t] = ((r >> 4) << 13) | c | (r & 15)
    assert sorted(order) == list(range(n))
    return order


@pytest.mark.parametrize("name", list(W.PARAMS))
def test_ntt_matches_oracle(torch_cuda, name):
    ctx, orc = pair(W.PARAMS[name], 1)
    rng = np.random.default_rng(11)
    nb = len(ctx.primes)
    x = np.stack([rng.integers(0, q, size=ctx.n, dtype=np.uint64) for q in ctx.primes])[None]
    note("ntt forward %s" % name)
    t = ctx.to_device(x)
    ctx.ntt(t, nb, 0, inverse=False)
    got = ctx.to_host(t).reshape(nb, ctx.n)
    order = ntt_storage_order(ctx.n)
    for r in range(nb):
        assert np.array_equal(got[r], orc.ntt(r, x[0, r])[order]), r
    note("ntt inverse %s" % name)
    ctx.ntt(t, nb, 0, inverse=True)
    assert np.array_equal(ctx.to_host(t).reshape(nb, ctx.n), x[0])


def _rand_ct(rng, qs, n, polys=2):
    return np.stack([np.stack([rng.integers(0, q, size=n, dtype=np.uint64) for q in qs]) for _ in range(polys)])


def _to_ntt(ctx, arr, nl):
    """coefficient [batch][polys][nl][N] -> device NTT domain"""
    t = ctx.to_device(arr)
    ctx.ntt(t, nl, 0, inverse=False)
    return t


def _from_ntt(ctx, t, nl):
    t = t.contiguous()
    ctx.ntt(t, nl, 0, inverse=True)
    return ctx.to_host(t)


@pytest.mark.parametrize("params", [HYB_SMALL, SINGLE_SMALL, W.PARAMS["realistic_n16384"], W.PARAMS["serving_n32768"]])
def test_tensor_keyswitch_rescale_match_oracle(torch_cuda, params):
    ctx, orc = pair(params, 5)
    rng = np.random.default_rng(12)
    n, L = ctx.n, ctx.L
    lev = L - 1
    qs = ctx.primes[:L]
    a = _rand_ct(rng, qs, n)
    b = _rand_ct(rng, qs, n)
    note("tensor %s" % params)
    d = ctx.tensor(lev, _to_ntt(ctx, a[None], L), _to_ntt(ctx, b[None], L))
    d_host = _from_ntt(ctx, d, L).reshape(3, L, n)
    assert np.array_equal(d_host, orc.tensor(lev, a, b))
    note("keyswitch %s" % params)
    d2 = np.stack([rng.integers(0, q, size=n, dtype=np.uint64) for q in qs])
    ks = ctx.keyswitch(lev, _to_ntt(ctx, d2[None], L))
    assert np.array_equal(_from_ntt(ctx, ks, L).reshape(2, L, n), orc.keyswitch(lev, d2))
    note("rescale %s" % params)
    for lv in range(1, L):
        ct = _rand_ct(rng, qs[:lv + 1], n)
        out = ctx.rescale(lv, _to_ntt(ctx, ct[None], lv + 1))
        assert np.array_equal(_from_ntt(ctx, out, lv).reshape(2, lv, n), orc.rescale(lv, ct))


def test_keyswitch_lower_levels_match_oracle(torch_cuda):
    ctx, orc = pair(HYB_SMALL, 6)
    rng = np.random.default_rng(13)
    for lev in (0, 1, 2, 3):
        qs = ctx.primes[:lev + 1]
        d2 = np.stack([rng.integers(0, q, size=ctx.n, dtype=np.uint64) for q in qs])
        note("keyswitch level %d" % lev)
        ks = ctx.keyswitch(lev, _to_ntt(ctx, d2[None], lev + 1))
        assert np.array_equal(_from_ntt(ctx, ks, lev + 1).reshape(2, lev + 1, ctx.n), orc.keyswitch(lev, d2))


def test_batched_primitives_match_single(torch_cuda):
    """A batch of 5 gives the same rows as 5 single calls."""
    ctx, orc = pair(HYB_SMALL, 6)
    rng = np.random.default_rng(14)
    L, n = ctx.L, ctx.n
    qs = ctx.primes[:L]
    d2 = np.stack([np.stack([rng.integers(0, q, size=n, dtype=np.uint64) for q in qs]) for _ in range(5)])
    note("keyswitch batch 5")
    ks = _from_ntt(ctx, ctx.keyswitch(L - 1, _to_ntt(ctx, d2, L)), L).reshape(5, 2, L, n)
    for x in range(5):
        assert np.array_equal(ks[x], orc.keyswitch(L - 1, d2[x]))


# ---------------------------------------------------------------- encryption
@pytest.mark.parametrize("enc", ["dense", "csr", "ell", "naive"])
def test_encryption_matches_oracle(torch_cuda, enc):
    ctx, orc = pair(HYB_SMALL, 7)
    A = W.sparse_matrix(5, 6, 0.4, 3)
    note("encrypt %s" % enc)
    M = ctx.encrypt(A, enc, seed=99, operand=0)
    for i in range(5):
        for j in range(6):
            if enc in ("csr", "ell") and A[i, j] == 0.0:
                continue
            got = ctx.export_ct(M, i, j)
            want = orc.encrypt(A[i, j], 99, 0, i, j)
            assert np.array_equal(got, want), (i, j)
    info = M.info()
    assert info.nnz == np.count_nonzero(A)


def test_decrypt_roundtrip(torch_cuda):
    ctx, orc = pair(SINGLE_SMALL, 7)
    A = W.sparse_matrix(7, 9, 0.3, 4)
    note("decrypt roundtrip")
    M = ctx.encrypt(A, "ell", seed=5, operand=0)
    back = ctx.decrypt(M)
    assert np.max(np.abs(back - A)) < 1e-9
    assert np.all(back[A == 0.0] == 0.0)


# ---------------------------------------------------------------- matmul, all outputs
def _all_outputs_equal(ctx, C, cts, M, Nc, tag):
    for i in range(M):
        for j in range(Nc):
            got = ctx.export_ct(C, i, j)
            assert np.array_equal(got, cts[i * Nc + j]), (tag, i, j)


@pytest.mark.parametrize("sched", ["lazy", "per_product"])
@pytest.mark.parametrize("enc", ["csr", "dense", "naive", "ell"])
def test_matmul_toy_all_outputs(torch_cuda, enc, sched):
    """8x8x8 at N = 2^10, Bernoulli(0.5) zeros in A: every output bit-exact."""
    P = W.PARAMS["toy_n1024"]
    ctx, orc = pair(P, W.key_seed(1))
    A, B = W.operands(8, 8, 8, 0.5, W.workload_seed(1))
    sa, sb = W.enc_seed(1, 0), W.enc_seed(1, 1)
    note("toy matmul %s %s" % (enc, sched))
    EA = ctx.encrypt(A, enc, sa, 0)
    EB = ctx.encrypt(B, "dense", sb, 1)
    C = ctx.matmul(EA, EB, sched)
    cts, vals, _ = orc.matmul(A, B, enc, sched, sa, sb, threads=4)
    _all_outputs_equal(ctx, C, cts, 8, 8, enc + sched)
    dec = ctx.decrypt(C)
    assert np.max(np.abs(dec.ravel() - vals)) < 1e-9
    assert np.max(np.abs(dec - A @ B)) < 1e-3


@pytest.mark.parametrize("sched", ["lazy", "per_product"])
@pytest.mark.parametrize("enc", ["csr", "ell", "naive", "dense"])
def test_matmul_ragged_hybrid_all_outputs(torch_cuda, enc, sched):
    """9x13x7 with an empty row and a full row, hybrid key switching (dnum = 2)."""
    ctx, orc = pair(HYB_SMALL, 21)
    A, B = W.operands(9, 13, 7, 0.6, 31)
    A[3, :] = 0.0
    A[5, :] = W.uniform_matrix(1, 13, 2)[0]
    note("ragged matmul %s %s" % (enc, sched))
    EA = ctx.encrypt(A, enc, 1234, 0)
    EB = ctx.encrypt(B, "dense", 4321, 1)
    C = ctx.matmul(EA, EB, sched)
    cts, _, _ = orc.matmul(A, B, enc, sched, 1234, 4321, threads=4)
    _all_outputs_equal(ctx, C, cts, 9, 7, enc + sched)
    dec = ctx.decrypt(C)
    if enc != "dense":            # dense multiplies encryptions of zero: noise, not 0
        assert np.all(dec[3] == 0.0)
    assert np.max(np.abs(dec - A @ B)) < 1e-6


@pytest.mark.parametrize("shape", [(11, 17, 29), (6, 9, 16)])
def test_column_tiles_ragged_all_outputs(torch_cuda, shape):
    """The fp64 column kernel takes 4-row tiles and 16 columns per block (two
    per wave: w and w + 8): 11 x 17 x 29 leaves a last row tile of 3 rows and
    a last column tile of 13 columns, so some waves hold one valid column of
    their two; 6 x 9 x 16 is one full column tile over a ragged row tile.
    Every output of the lazy product matches the oracle bit for bit."""
    M, K, Nc = shape
    ctx, orc = pair(HYB_SMALL, 21)
    A, B = W.operands(M, K, Nc, 0.45, 7700 + M)
    note("column tiles %dx%dx%d" % shape)
    EA = ctx.encrypt(A, "csr", 1777, 0)
    EB = ctx.encrypt(B, "dense", 1778, 1)
    C = ctx.matmul(EA, EB, "lazy")
    cts, _, _ = orc.matmul(A, B, "csr", "lazy", 1777, 1778, threads=_threads())
    _all_outputs_equal(ctx, C, cts, M, Nc, "column tiles")
    assert np.max(np.abs(ctx.decrypt(C) - A @ B)) < 1e-6
    for m in (C, EA, EB):
        m.close()


@pytest.mark.parametrize("sched", ["lazy", "per_product"])
def test_matmul_mixed_prime_sizes_all_outputs(torch_cuda, sched):
    """61-, 50- and 41-bit data primes: the 61- and 50-bit primes take the
    128-bit integer tensor arithmetic (neither is within 2^20 below 2^60),
    the 41-bit prime the fp64 residues."""
    P = dict(log_n=10, q_bits=[61, 50, 41], p_bits=[61, 61], dnum=2)
    ctx, orc = pair(P, 17)
    A, B = W.operands(6, 21, 5, 0.3, 41)
    note("mixed primes %s" % sched)
    C = ctx.matmul(ctx.encrypt(A, "csr", 5, 0), ctx.encrypt(B, "dense", 6, 1), sched)
    cts, _, _ = orc.matmul(A, B, "csr", sched, 5, 6, threads=4)
    _all_outputs_equal(ctx, C, cts, 6, 5, sched)


@pytest.mark.parametrize("q_bits", [[40, 60, 60], [60, 40, 40]])
def test_fused_rescale_target_arithmetic_n14(torch_cuda, q_bits):
    """N = 2^14 (the fused key switch and rescale) with the lift's two cases
    for a 40-bit target prime: the centered last prime already below the
    target ([60, 40, 40]) and above it, reduced first ([40, 60, 60]: a 60-bit
    last prime); both schedules, every output bit-exact against the oracle."""
    P = dict(log_n=14, q_bits=q_bits, p_bits=[60, 60], dnum=2)
    ctx, orc = pair(P, 19)
    A, B = W.operands(3, 5, 2, 0.4, 43)
    for sched in ("lazy", "per_product"):
        note("fused rescale targets %s %s" % (q_bits, sched))
        C = ctx.matmul(ctx.encrypt(A, "csr", 9, 0), ctx.encrypt(B, "dense", 10, 1), sched)
        cts, _, _ = orc.matmul(A, B, "csr", sched, 9, 10, threads=8)
        _all_outputs_equal(ctx, C, cts, 3, 2, sched)


@pytest.mark.parametrize("q_bits", [[61, 59, 40], [60, 60, 40]])
def test_long_rows_fold_the_sums(torch_cuda, q_bits):
    """K = 600 dense: every lazy sum crosses the fold points of the tensor
    arithmetics many times (the 128-bit sums for the 61- and 59-bit primes,
    the carry-save sums for primes just below 2^60, the fp64 sums below
    2^42)."""
    P = dict(log_n=10, q_bits=q_bits, p_bits=[61, 61], dnum=2)
    ctx, orc = pair(P, 18)
    A, B = W.operands(3, 600, 2, 0.0, 42)
    note("K=600 lazy")
    C = ctx.matmul(ctx.encrypt(A, "dense", 7, 0), ctx.encrypt(B, "dense", 8, 1), "lazy")
    cts, _, _ = orc.matmul(A, B, "dense", "lazy", 7, 8, outputs=[(0, 0), (2, 1)], threads=2)
    assert np.array_equal(ctx.export_ct(C, 0, 0), cts[0])
    assert np.array_equal(ctx.export_ct(C, 2, 1), cts[1])


def test_all_zero_left_operand(torch_cuda):
    ctx, orc = pair(HYB_SMALL, 21)
    A = np.zeros((3, 4))
    B = W.uniform_matrix(4, 2, 9)
    for enc in ("csr", "ell", "naive"):
        note("zero A %s" % enc)
        C = ctx.matmul(ctx.encrypt(A, enc, 1, 0), ctx.encrypt(B, "dense", 2, 1), "lazy")
        assert np.all(ctx.decrypt(C) == 0.0)
        assert not ctx.export_ct(C, 2, 1).any()


def test_one_by_one(torch_cuda):
    ctx, orc = pair(SINGLE_SMALL, 3)
    A = np.array([[0.75]])
    B = np.array([[-0.5]])
    for sched in ("lazy", "per_product"):
        note("1x1x1 %s" % sched)
        C = ctx.matmul(ctx.encrypt(A, "csr", 1, 0), ctx.encrypt(B, "dense", 2, 1), sched)
        cts, _, _ = orc.matmul(A, B, "csr", sched, 1, 2)
        assert np.array_equal(ctx.export_ct(C, 0, 0), cts[0])


def test_key_switch_slices_and_streams_give_identical_products(torch_cuda):
    """N = 2^14, 40 x 24 x 26 (1040 outputs: the first LAZY product of a
    fresh context tunes the key-switch slices): the tuned setting and fixed
    slices of 128, 256 and 2048 outputs on one stream and on two give the
    same ciphertexts; the tuner's report is consistent; bad settings are
    refused."""
    from paper_2503_09184_amd import sfhe
    P = W.PARAMS["realistic_n16384"]
    ctx = sfhe.Context(**P)
    ctx.keygen(W.key_seed(3))
    A, B = W.operands(40, 24, 26, 0.5, 7300)
    EA, EB = ctx.encrypt(A, "csr", 7301, 0), ctx.encrypt(B, "dense", 7302, 1)
    sl, st, us1, us2 = ctx.ks_tuning()
    assert sl == 0                                           # not tuned yet
    note("ks tuned product")
    C = ctx.matmul(EA, EB, "lazy")
    ref = [ctx.export_ct(C, i, j) for i in range(40) for j in range(26)]
    C.close()
    sl, st, us1, us2 = ctx.ks_tuning()
    assert st in (1, 2) and sl >= 64
    assert all(v > 0 for k, v in us1.items() if k <= 1040) and all(v < 0 for k, v in us1.items() if k > 1040)
    assert (sl, st) in [(k, 1) for k, v in us1.items() if v > 0] + [(k, 2) for k, v in us2.items() if v > 0]
    for setting in ((128, 1), (256, 2), (2048, 1), (2048, 2), (-1, 1)):
        note("ks setting %s" % (setting,))
        ctx.set_ks_slice(*setting)
        C = ctx.matmul(EA, EB, "lazy")
        got = [ctx.export_ct(C, i, j) for i in range(40) for j in range(26)]
        C.close()
        assert all(np.array_equal(x, y) for x, y in zip(got, ref)), setting
    assert ctx.ks_tuning()[:2] == (sl, st)                  # -1: back to the tuned setting
    for bad in ((100, 1), (8192, 1), (32, 1), (256, 3), (256, 0)):
        with pytest.raises(sfhe.SfheError) as e:
            ctx.set_ks_slice(*bad)
        assert e.value.code == -1
    assert np.max(np.abs(ctx.decrypt(ctx.matmul(EA, EB, "lazy")) - A @ B)) < 1e-6
    for m in (EA, EB):
        m.close()
    ctx.close()


def test_errors_are_reported(torch_cuda):
    from paper_2503_09184_amd import sfhe
    ctx, _ = pair(SINGLE_SMALL, 3)
    A = ctx.encrypt(np.ones((2, 3)), "csr", 1, 0)
    B = ctx.encrypt(np.ones((2, 2)), "dense", 1, 1)
    with pytest.raises(sfhe.SfheError) as e:
        ctx.matmul(A, B, "lazy")
    assert e.value.code == -3
    Bs = ctx.encrypt(np.ones((3, 2)), "csr", 1, 1)     # a sparse-encoded right operand is accepted
    assert ctx.matmul(A, Bs, "lazy").info().rows == 2
    with pytest.raises(sfhe.SfheError) as e:
        ctx.encrypt(np.full((1, 1), np.inf), "csr", 1, 0)
    assert e.value.code == -1
    with pytest.raises(sfhe.SfheError) as e:
        sfhe.Context(log_n=16, q_bits=[60, 40], p_bits=[60], dnum=2)
    assert e.value.code == -2


# ---------------------------------------------------------------- sweep size (N = 2^13, 64 x 64)
@pytest.mark.parametrize("sparsity", [0.0, 0.5, 0.9])
def test_sweep_n8192_sampled_outputs_and_cross_encoding(torch_cuda, sparsity):
    P = W.PARAMS["sweep_n8192"]
    ctx, orc = pair(P, W.key_seed(2))
    A, B = W.operands(64, 64, 64, sparsity, W.workload_seed(2))
    sa, sb = W.enc_seed(2, 0), W.enc_seed(2, 1)
    EB = ctx.encrypt(B, "dense", sb, 1)
    outs = {}
    rng = np.random.default_rng(int(sparsity * 100))
    sample = sorted({(int(rng.integers(64)), int(rng.integers(64))) for _ in range(6)})
    for enc in ("csr", "ell", "naive", "dense"):
        note("sweep %.2f %s lazy" % (sparsity, enc))
        EA = ctx.encrypt(A, enc, sa, 0)
        C = ctx.matmul(EA, EB, "lazy")
        outs[enc] = [ctx.export_ct(C, i, j) for (i, j) in sample]
        dec = ctx.decrypt(C)
        assert np.max(np.abs(dec - A @ B)) < 1e-6, enc
    for enc in ("ell", "naive"):
        for x, y in zip(outs["csr"], outs[enc]):
            assert np.array_equal(x, y)
    if sparsity == 0.0:
        for x, y in zip(outs["csr"], outs["dense"]):
            assert np.array_equal(x, y)
    cts, _, _ = orc.matmul(A, B, "csr", "lazy", sa, sb, outputs=sample, threads=8)
    for n, o in enumerate(outs["csr"]):
        assert np.array_equal(o, cts[n]), sample[n]


@pytest.mark.parametrize("sched", ["lazy", "per_product"])
@pytest.mark.parametrize("sparsity", [0.0, 0.25, 0.5, 0.75, 0.9])
def test_sweep_n8192_every_encoding_and_schedule(torch_cuda, sparsity, sched):
    """The sparsity sweep (N = 2^13, 64 x 64 x 64): for each sparsity and
    schedule, A in all four encodings times a dense B, 64 sampled outputs
    (an 8 x 8 grid with the corner rows and columns) of each encoding bit for
    bit against the oracle's schedule of that encoding (the sparse encodings
    against its CSR iteration, whose bits its naive and ELLPACK iterations
    share), and every output within 1e-6 of the fp64 product."""
    P = W.PARAMS["sweep_n8192"]
    ctx, orc = pair(P, W.key_seed(2))
    A, B = W.operands(64, 64, 64, sparsity, W.workload_seed(2))
    sa, sb = W.enc_seed(2, 0), W.enc_seed(2, 1)
    sample = _grid(4000 + int(sparsity * 100), 8, 8, 64)
    EB = ctx.encrypt(B, "dense", sb, 1)
    got = {}
    for enc in ("csr", "ell", "naive", "dense"):
        note("sweep %.2f %s %s" % (sparsity, enc, sched))
        EA = ctx.encrypt(A, enc, sa, 0)
        C = ctx.matmul(EA, EB, sched)
        got[enc] = [ctx.export_ct(C, i, j) for (i, j) in sample]
        assert np.max(np.abs(ctx.decrypt(C) - A @ B)) < 1e-6, enc
        C.close()
        EA.close()
    EB.close()
    note("sweep oracle %.2f %s" % (sparsity, sched))
    want = {enc: orc.matmul(A, B, enc, sched, sa, sb, outputs=sample, threads=_threads(), decrypt=False)[0]
            for enc in ("csr", "dense")}
    for enc in ("csr", "ell", "naive", "dense"):
        ref = want["dense" if enc == "dense" else "csr"]
        for n, o in enumerate(got[enc]):
            assert np.array_equal(o, ref[n]), (enc, sample[n])


@pytest.mark.parametrize("sparsity,sched", [(0.25, "lazy"), (0.75, "lazy"), (0.5, "per_product")])
def test_sweep_n8192_all_outputs(torch_cuda, sparsity, sched):
    """N = 2^13, 64 x 64 x 64 (CSR): every output bit-exact against the oracle
    (LAZY: all 4096; PER_PRODUCT, whose oracle relinearises every product:
    the 1024 outputs of rows 0-15), and decrypted within 1e-6 of the fp64
    product."""
    P = W.PARAMS["sweep_n8192"]
    ctx, orc = pair(P, W.key_seed(2))
    A, B = W.operands(64, 64, 64, sparsity, W.workload_seed(2))
    sa, sb = W.enc_seed(2, 0), W.enc_seed(2, 1)
    note("sweep all outputs %.2f %s" % (sparsity, sched))
    C = ctx.matmul(ctx.encrypt(A, "csr", sa, 0), ctx.encrypt(B, "dense", sb, 1), sched)
    assert np.max(np.abs(ctx.decrypt(C) - A @ B)) < 1e-6
    rows = 64 if sched == "lazy" else 16
    outs = [(i, j) for i in range(rows) for j in range(64)]
    cts, _, _ = orc.matmul(A, B, "csr", sched, sa, sb, outputs=outs, threads=_threads(), decrypt=False)
    for n, (i, j) in enumerate(outs):
        assert np.array_equal(ctx.export_ct(C, i, j), cts[n]), (i, j)


# ---------------------------------------------------------------- full size
def _threads():
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _realistic(sparsity):
    P = W.PARAMS["realistic_n16384"]
    ctx, orc = pair(P, W.key_seed(3))
    A, B = W.operands(128, 128, 128, sparsity, W.workload_seed(3))
    return ctx, orc, A, B, W.enc_seed(3, 0), W.enc_seed(3, 1)


@pytest.mark.parametrize("sparsity", [0.5, 0.9])
def test_realistic_128_lazy_sampled_outputs(torch_cuda, sparsity):
    """The benchmarked product itself: 128 x 128 x 128 at N = 2^14 with five
    data primes, CSR left operand, lazy schedule, the same calls and launch
    configuration as the timed step.  Sampled outputs (including the corner
    ones) match the oracle bit for bit, every one of the 16384 outputs
    decrypts within 1e-6 of the fp64 product, and the ELLPACK and naive-sparse
    encodings give the same ciphertexts on the samples."""
    ctx, orc, A, B, sa, sb = _realistic(sparsity)
    note("realistic 128^3 sparsity %.2f encrypt" % sparsity)
    EB = ctx.encrypt(B, "dense", sb, 1)
    # 256 sampled outputs: a 16 x 16 grid of rows and columns (corners
    # included), so the oracle encrypts only the rows and columns it needs
    rng = np.random.default_rng(1000 + int(sparsity * 100))
    rows = sorted({0, 127} | set(int(x) for x in rng.choice(np.arange(1, 127), 14, replace=False)))
    cols = sorted({0, 127} | set(int(x) for x in rng.choice(np.arange(1, 127), 14, replace=False)))
    sample = [(i, j) for i in rows for j in cols]
    assert len(sample) == 256
    outs = {}
    for enc in ("csr", "ell", "naive"):
        note("realistic 128^3 sparsity %.2f %s lazy" % (sparsity, enc))
        EA = ctx.encrypt(A, enc, sa, 0)
        C = ctx.matmul(EA, EB, "lazy")
        outs[enc] = [ctx.export_ct(C, i, j) for (i, j) in sample]
        if enc == "csr":
            dec = ctx.decrypt(C)
            err = np.max(np.abs(dec - A @ B))
            note("realistic max |err| %.3e" % err)
            assert err < 1e-6
        C.close()
        EA.close()
    for enc in ("ell", "naive"):
        for x, y in zip(outs["csr"], outs[enc]):
            assert np.array_equal(x, y), enc
    note("realistic oracle on %d outputs" % len(sample))
    cts, _, _ = orc.matmul(A, B, "csr", "lazy", sa, sb, outputs=sample, threads=_threads())
    for n, o in enumerate(outs["csr"]):
        assert np.array_equal(o, cts[n]), sample[n]


def _grid(seed, n_rows, n_cols, size=128):
    """A sample of outputs: n_rows x n_cols rows and columns drawn without
    replacement, the first and last of each included."""
    rng = np.random.default_rng(seed)
    rows = sorted({0, size - 1} | set(int(x) for x in rng.choice(np.arange(1, size - 1), n_rows - 2, replace=False)))
    cols = sorted({0, size - 1} | set(int(x) for x in rng.choice(np.arange(1, size - 1), n_cols - 2, replace=False)))
    return [(i, j) for i in rows for j in cols]


@pytest.mark.parametrize("sparsity,n_rows,n_cols", [(0.9, 16, 16), (0.5, 8, 8)])
def test_realistic_128_per_product_sampled_outputs(torch_cuda, sparsity, n_rows, n_cols):
    """The per-product schedule (Algorithm 1's order: relinearise and rescale
    every product, then add) at the benchmarked size, with the calls the
    bench times: 256 sampled outputs at 90% sparsity and 64 at 50% (the
    oracle key-switches every product of them) match the oracle bit for bit,
    and every output decrypts within 1e-6."""
    ctx, orc, A, B, sa, sb = _realistic(sparsity)
    note("realistic 128^3 per_product sparsity %.2f" % sparsity)
    EB = ctx.encrypt(B, "dense", sb, 1)
    EA = ctx.encrypt(A, "csr", sa, 0)
    C = ctx.matmul(EA, EB, "per_product")
    sample = _grid(2000 + int(sparsity * 100), n_rows, n_cols)
    got = [ctx.export_ct(C, i, j) for (i, j) in sample]
    dec = ctx.decrypt(C)
    assert np.max(np.abs(dec - A @ B)) < 1e-6
    C.close()
    EA.close()
    EB.close()
    note("realistic per_product oracle on %d outputs" % len(sample))
    cts, _, _ = orc.matmul(A, B, "csr", "per_product", sa, sb, outputs=sample, threads=_threads(), decrypt=False)
    for n, o in enumerate(got):
        assert np.array_equal(o, cts[n]), sample[n]


@pytest.mark.parametrize("sparsity", [0.5, 0.9])
def test_realistic_128_dense_lazy_sampled_outputs(torch_cuda, sparsity):
    """The naive dense schedule (every k visited, encryptions of zero
    included) on the operands of the 50% and 90% legs, as the bench times it
    for the sparse-over-dense speed-ups: 256 sampled outputs bit-exact
    against the oracle's dense schedule, all outputs within 1e-6."""
    ctx, orc, A, B, sa, sb = _realistic(sparsity)
    note("realistic 128^3 dense lazy sparsity %.2f" % sparsity)
    EB = ctx.encrypt(B, "dense", sb, 1)
    EA = ctx.encrypt(A, "dense", sa, 0)
    C = ctx.matmul(EA, EB, "lazy")
    assert ctx.last_stats().products == 128 ** 3
    sample = _grid(3000 + int(sparsity * 100), 16, 16)
    got = [ctx.export_ct(C, i, j) for (i, j) in sample]
    assert np.max(np.abs(ctx.decrypt(C) - A @ B)) < 1e-6
    C.close()
    EA.close()
    EB.close()
    note("realistic dense oracle on %d outputs" % len(sample))
    cts, _, _ = orc.matmul(A, B, "dense", "lazy", sa, sb, outputs=sample, threads=_threads(), decrypt=False)
    for n, o in enumerate(got):
        assert np.array_equal(o, cts[n]), sample[n]
