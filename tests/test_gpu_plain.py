"""GPU parity of the plaintext-weight product (Sec. 3.3.2: weights held in
plaintext by the server, multiplied into encrypted values): the HIP library
against the CPU oracle on the same seeded inputs, bit for bit in the
coefficient domain, and decrypted values against the fp64 product.  Every
call goes through the C ABI."""
import math

import numpy as np
import pytest

from paper_2503_09184_amd import workloads as W
from tests.test_gpu_parity import HYB_SMALL, note, pair, torch_cuda, _threads  # noqa: F401

pytestmark = pytest.mark.gpu


def _all_equal(ctx, C, cts, M, Nc, tag):
    for i in range(M):
        for j in range(Nc):
            assert np.array_equal(ctx.export_ct(C, i, j), cts[i * Nc + j]), (tag, i, j)


def _bound(ctx_n, log2_scale, sw, q_top, w_row):
    """6-sigma bound of one output: weighted fresh noise plus one rescale."""
    n = ctx_n
    dp = 2.0 ** (sw + log2_scale) / q_top
    sf = 3.2 * math.sqrt(n / 2) / 2.0 ** log2_scale
    srs = math.sqrt((1 + 2 * n / 3) / 12 * n / 2) / dp
    return 6 * math.sqrt(srs ** 2 + float(np.sum(np.asarray(w_row) ** 2)) * sf ** 2 * 2) + 1e-12


@pytest.mark.parametrize("enc", ["csr", "dense", "naive", "ell"])
def test_plain_toy_all_outputs(torch_cuda, enc):
    """8x8x8 at N = 2^10 with two 60-bit data primes, half of W zero."""
    P = W.PARAMS["toy_n1024"]
    ctx, orc = pair(P, W.key_seed(1))
    Wt, B = W.operands(8, 8, 8, 0.5, W.workload_seed(11))
    sb = W.enc_seed(11, 1)
    note("plain toy %s" % enc)
    C = ctx.matmul_plain(ctx.encode_weights(Wt, enc, 40), ctx.encrypt(B, "dense", sb, 1))
    cts, vals, _ = orc.matmul_plain(Wt, B, enc, sb, 40, threads=4)
    _all_equal(ctx, C, cts, 8, 8, enc)
    dec = ctx.decrypt(C)
    assert np.max(np.abs(dec.ravel() - vals)) < 1e-12
    ref = Wt @ B
    for i in range(8):
        for j in range(8):
            assert abs(dec[i, j] - ref[i, j]) <= _bound(ctx.n, 40, 40, ctx.primes[1], Wt[i]), (i, j)


@pytest.mark.parametrize("enc", ["csr", "ell", "naive", "dense"])
def test_plain_ragged_all_outputs(torch_cuda, enc):
    """21 x 37 x 9 with five 60/40-bit primes: a ragged last row tile (5 rows)
    and column group (1 column), an empty row and a full row."""
    ctx, orc = pair(HYB_SMALL, 21)
    Wt, B = W.operands(21, 37, 9, 0.6, 51)
    Wt[3, :] = 0.0
    Wt[17, :] = W.uniform_matrix(1, 37, 3)[0]
    note("plain ragged %s" % enc)
    C = ctx.matmul_plain(ctx.encode_weights(Wt, enc, 40), ctx.encrypt(B, "dense", 77, 1))
    cts, _, _ = orc.matmul_plain(Wt, B, enc, 77, 40, threads=4)
    _all_equal(ctx, C, cts, 21, 9, enc)
    dec = ctx.decrypt(C)
    if enc != "dense":
        assert np.all(dec[3] == 0.0)
    assert np.max(np.abs(dec - Wt @ B)) < 1e-6


def test_plain_mixed_prime_sizes(torch_cuda):
    """61-, 50- and 41-bit data primes: the integer arithmetic for the first
    two, fp64 residues for the last; weights at scale 2^30."""
    P = dict(log_n=10, q_bits=[61, 50, 41], p_bits=[61, 61], dnum=2)
    ctx, orc = pair(P, 17)
    Wt, B = W.operands(18, 11, 6, 0.4, 52)
    note("plain mixed primes")
    C = ctx.matmul_plain(ctx.encode_weights(Wt, "csr", 30), ctx.encrypt(B, "dense", 5, 1))
    cts, _, _ = orc.matmul_plain(Wt, B, "csr", 5, 30, threads=4)
    _all_equal(ctx, C, cts, 18, 6, "mixed")


def test_plain_long_rows_fold(torch_cuda):
    """K = 1100 dense: each fp64 sum crosses the fold point (1024 products)."""
    P = dict(log_n=10, q_bits=[61, 40, 40], p_bits=[61], dnum=3)
    ctx, orc = pair(P, 19)
    Wt, B = W.operands(17, 1100, 5, 0.0, 53)
    note("plain K=1100")
    C = ctx.matmul_plain(ctx.encode_weights(Wt, "dense", 40), ctx.encrypt(B, "dense", 9, 1))
    sample = [(0, 0), (16, 4), (9, 2)]
    cts, _, _ = orc.matmul_plain(Wt, B, "dense", 9, 40, outputs=sample, threads=3)
    for n, (i, j) in enumerate(sample):
        assert np.array_equal(ctx.export_ct(C, i, j), cts[n]), (i, j)


def test_plain_batch_fused_and_per_product_launches_match_single(torch_cuda):
    """An uneven batch of three products in one fused call, and again with one
    launch per product: both equal the single calls, bit for bit."""
    ctx, orc = pair(HYB_SMALL, 21)
    shapes = [(5, 9, 3, 0.5), (33, 4, 6, 0.7), (16, 20, 1, 0.0)]
    Ws, Bs = [], []
    for n, (M, K, Nc, s) in enumerate(shapes):
        Wt, B = W.operands(M, K, Nc, s, 60 + n)
        Ws.append(ctx.encode_weights(Wt, ["csr", "ell", "dense"][n], 40))
        Bs.append(ctx.encrypt(B, "dense", 90 + n, 1))
    note("plain batch fused")
    fused = ctx.matmul_plain_batch(Ws, Bs, "fused")
    st = ctx.last_stats()
    assert st.tensor_launches <= 2
    note("plain batch per product")
    pp = ctx.matmul_plain_batch(Ws, Bs, "per_product")
    assert ctx.last_stats().tensor_launches == st.products
    for n, (M, K, Nc, s) in enumerate(shapes):
        single = ctx.matmul_plain(Ws[n], Bs[n])
        for i in range(M):
            for j in range(Nc):
                a = ctx.export_ct(single, i, j)
                assert np.array_equal(a, ctx.export_ct(fused[n], i, j)), (n, i, j)
                assert np.array_equal(a, ctx.export_ct(pp[n], i, j)), (n, i, j)


def test_plain_errors(torch_cuda):
    from paper_2503_09184_amd import sfhe
    ctx, _ = pair(HYB_SMALL, 21)
    Wt, B = W.operands(4, 5, 3, 0.5, 61)
    Wp = ctx.encode_weights(Wt, "csr", 40)
    EB = ctx.encrypt(B, "dense", 1, 1)
    EA = ctx.encrypt(Wt, "csr", 2, 0)
    with pytest.raises(sfhe.SfheError) as e:
        ctx.matmul(Wp, EB, "lazy")
    assert e.value.code == -6
    with pytest.raises(sfhe.SfheError) as e:
        ctx.matmul_plain(EA, EB)
    assert e.value.code == -1
    with pytest.raises(sfhe.SfheError) as e:
        ctx.matmul_plain(Wp, ctx.encrypt(W.uniform_matrix(4, 3, 1), "dense", 1, 1))
    assert e.value.code == -3
    with pytest.raises(sfhe.SfheError) as e:
        ctx.decrypt(Wp)
    assert e.value.code == -6
    with pytest.raises(sfhe.SfheError) as e:
        ctx.encode_weights(np.full((2, 2), 2.0 ** 30), "dense", 40)
    assert e.value.code == -1
    # the tile tables: per 16-row tile its entries' k and row mask, per entry
    # and data prime 16 weights and 16 Shoup companions (4 x 3 weights: one tile)
    Wd = W.sparse_matrix(4, 3, 0.5, 7)
    kk = int(np.count_nonzero(np.any(Wd != 0.0, axis=0)))
    assert ctx.encode_weights(Wd, "csr", 40).info().device_bytes == (2 + 2 * kk) * 4 + kk * ctx.L * 16 * 2 * 8


@pytest.mark.parametrize("sparsity", [0.5, 0.9])
def test_plain_realistic_sampled_outputs(torch_cuda, sparsity):
    """N = 2^14 with the five data primes of the benchmarked parameters:
    W 128 x 128 (CSR), B 128 x 32; sampled outputs bit-exact against the
    oracle and every output within 1e-6 of the fp64 product."""
    P = W.PARAMS["realistic_n16384"]
    ctx, orc = pair(P, W.key_seed(3))
    Wt, B = W.operands(128, 128, 32, sparsity, W.workload_seed(4))
    sb = W.enc_seed(4, 1)
    note("plain realistic sparsity %.2f" % sparsity)
    C = ctx.matmul_plain(ctx.encode_weights(Wt, "csr", 40), ctx.encrypt(B, "dense", sb, 1))
    dec = ctx.decrypt(C)
    err = np.max(np.abs(dec - Wt @ B))
    note("plain realistic max |err| %.3e" % err)
    assert err < 1e-6
    sample = [(0, 0), (127, 31), (64, 5), (15, 16), (16, 15), (100, 30)]
    cts, _, _ = orc.matmul_plain(Wt, B, "csr", sb, 40, outputs=sample, threads=_threads())
    for n, (i, j) in enumerate(sample):
        assert np.array_equal(ctx.export_ct(C, i, j), cts[n]), (i, j)


def test_plain_n14_large_last_prime(torch_cuda):
    """N = 2^14 with a 60-bit last prime above the 40-bit ones: the rescale's
    centered lift must reduce the last prime's residues modulo each smaller
    prime (the fused N = 2^14 rescale)."""
    P = dict(log_n=14, q_bits=[40, 41, 60], p_bits=[60], dnum=3)
    ctx, orc = pair(P, 23)
    Wt, B = W.operands(20, 9, 5, 0.5, 54)
    note("plain N=2^14 large last prime")
    C = ctx.matmul_plain(ctx.encode_weights(Wt, "ell", 40), ctx.encrypt(B, "dense", 13, 1))
    sample = [(0, 0), (19, 4), (7, 2), (16, 1)]
    cts, _, _ = orc.matmul_plain(Wt, B, "ell", 13, 40, outputs=sample, threads=_threads())
    for n, (i, j) in enumerate(sample):
        assert np.array_equal(ctx.export_ct(C, i, j), cts[n]), (i, j)


@pytest.mark.parametrize("launch", ["fused", "per_product"])
def test_plain_graph_replays_match_eager(torch_cuda, launch):
    """The batch captured into a HIP graph: three replays, with eager library
    work between them, each give the eager results bit for bit."""
    from paper_2503_09184_amd import sfhe
    ctx, _ = pair(HYB_SMALL, 21)
    shapes = [(5, 9, 3, 0.5), (33, 4, 6, 0.7), (16, 20, 1, 0.0)]
    Ws, Bs = [], []
    for n, (M, K, Nc, s) in enumerate(shapes):
        Wt, B = W.operands(M, K, Nc, s, 70 + n)
        Ws.append(ctx.encode_weights(Wt, "csr", 40))
        Bs.append(ctx.encrypt(B, "dense", 95 + n, 1))
    eager = ctx.matmul_plain_batch(Ws, Bs, "fused")
    want = [[ctx.export_ct(eager[n], i, j) for i in range(M) for j in range(Nc)]
            for n, (M, K, Nc, s) in enumerate(shapes)]
    note("plain graph %s" % launch)
    g = sfhe.PlainGraph(ctx, Ws, Bs, launch)
    for rep in range(3):
        g.launch()
        st = ctx.last_stats()
        assert st.products == sum(int(np.count_nonzero(W.operands(M, K, Nc, s, 70 + n)[0])) * Nc
                                  for n, (M, K, Nc, s) in enumerate(shapes))
        for n, (M, K, Nc, s) in enumerate(shapes):
            C = g.result(n)
            got = [ctx.export_ct(C, i, j) for i in range(M) for j in range(Nc)]
            for x, y in zip(got, want[n]):
                assert np.array_equal(x, y), (rep, n)
        ctx.matmul_plain(Ws[0], Bs[0]).close()          # eager work between replays
    g.close()
