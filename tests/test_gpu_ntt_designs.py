"""GPU tests of the NTT designs and their tuning: every design that applies
to a ring transforms bit for bit like the CPU oracle in the library's storage
order, the context keeps the fastest measured design per direction, and a
whole product gives the same ciphertexts under every design.  Every call goes
through the C ABI."""
import numpy as np
import pytest

from paper_2503_09184_amd import workloads as W
from tests.test_gpu_parity import note, ntt_storage_order, pair, torch_cuda  # noqa: F401

pytestmark = pytest.mark.gpu

RINGS = ["toy_n1024", "sweep_n8192", "realistic_n16384", "serving_n32768"]


@pytest.mark.parametrize("name", RINGS)
def test_every_design_matches_oracle(torch_cuda, name):
    ctx, orc = pair(W.PARAMS[name], 1)
    nb = len(ctx.primes)
    rng = np.random.default_rng(12)
    x = np.stack([rng.integers(0, q, size=ctx.n, dtype=np.uint64) for q in ctx.primes])[None]
    order = ntt_storage_order(ctx.n)
    want = np.stack([orc.ntt(r, x[0, r])[order] for r in range(nb)])
    designs = sorted(set(ctx.ntt_tuning(False)[1]) | set(ctx.ntt_tuning(True)[1]))
    if ctx.n == 1 << 15:
        assert designs == []          # one design, not timed
        designs = ["register"]
    try:
        for d in designs:
            note("ntt design %s %s" % (name, d))
            ctx.set_ntt_design(False, d)
            ctx.set_ntt_design(True, d)
            t = ctx.to_device(x)
            ctx.ntt(t, nb, 0, inverse=False)
            assert np.array_equal(ctx.to_host(t).reshape(nb, ctx.n), want), d
            ctx.ntt(t, nb, 0, inverse=True)
            assert np.array_equal(ctx.to_host(t).reshape(nb, ctx.n), x[0]), d
    finally:
        ctx.set_ntt_design(False, None)
        ctx.set_ntt_design(True, None)


@pytest.mark.parametrize("name", RINGS)
def test_tuning_keeps_the_fastest_design(torch_cuda, name):
    from paper_2503_09184_amd import sfhe
    ctx, _ = pair(W.PARAMS[name], 1)
    expect = {1 << 10: {"radix16", "radix8", "radix4"}, 1 << 13: {"radix16", "radix8", "radix4"},
              1 << 14: {"register", "radix16", "radix8", "radix4"}, 1 << 15: set()}[ctx.n]
    for inverse in (False, True):
        used, us = ctx.ntt_tuning(inverse)
        note("ntt tuning %s inverse=%s: %s %s" % (name, inverse, used, us))
        assert set(us) == expect
        if us:
            assert used == min(us, key=us.get) and all(v > 0 for v in us.values())
        else:
            assert used == "register"
    bad = "radix16" if ctx.n == 1 << 15 else ("register" if ctx.n < 1 << 14 else None)
    if bad:
        with pytest.raises(sfhe.SfheError) as e:
            ctx.set_ntt_design(False, bad)
        assert e.value.code == -6


def test_product_is_identical_under_every_design(torch_cuda):
    """N = 2^14: encryption, the product and export under the register
    design and under each LDS design give the same ciphertexts."""
    ctx, _ = pair(W.PARAMS["realistic_n16384"], W.key_seed(3))
    A, B = W.operands(5, 6, 3, 0.5, 64)
    got = {}
    try:
        for d in ("register", "radix16", "radix8", "radix4"):
            note("product under ntt design %s" % d)
            ctx.set_ntt_design(False, d)
            ctx.set_ntt_design(True, d)
            C = ctx.matmul(ctx.encrypt(A, "csr", 5, 0), ctx.encrypt(B, "dense", 6, 1), "lazy")
            got[d] = [ctx.export_ct(C, i, j) for i in range(5) for j in range(3)]
    finally:
        ctx.set_ntt_design(False, None)
        ctx.set_ntt_design(True, None)
    for d in ("radix16", "radix8", "radix4"):
        for x, y in zip(got[d], got["register"]):
            assert np.array_equal(x, y), d
