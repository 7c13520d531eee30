"""The allocation-free key switch (sfhe_keyswitch_noalloc) against the
allocating one (sfhe_keyswitch) and the oracle: bit for bit, on two calls in
a row (the second smaller, so it runs over what the first left in the fixed
scratch), with no allocation through the hooks during the calls, and a batch
beyond the fixed scratch refused.  Every call goes through the C ABI."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2503_09184_amd import workloads as W
from tests.test_gpu_alloc import _Counting
from tests.test_gpu_parity import _from_ntt, _to_ntt, note, torch_cuda  # noqa: F401

pytestmark = pytest.mark.gpu


def _d2(rng, qs, n, batch):
    return np.stack([np.stack([rng.integers(0, q, size=n, dtype=np.uint64) for q in qs]) for _ in range(batch)])


@pytest.mark.parametrize("name", ["realistic_n16384", "toy_n1024"])
def test_keyswitch_noalloc_matches_keyswitch(torch_cuda, name):
    torch = torch_cuda
    from paper_2503_09184_amd import sfhe
    P = W.PARAMS[name]
    hk = _Counting(torch, torch.cuda.current_device())
    ctx = sfhe.Context(**P, hooks=(hk.alloc, hk.free))
    ctx.keygen(51)
    orc = Oracle(**P)
    orc.keygen(51)
    rng = np.random.default_rng(52)
    n, L = ctx.n, ctx.L
    # two calls in a row: a batch at the top level, then a smaller one lower down
    for lev, batch in ((L - 1, 6), (L - 2, 2)):
        nl = lev + 1
        qs = ctx.primes[:nl]
        d2 = _d2(rng, qs, n, batch)
        dev = _to_ntt(ctx, d2, nl)
        ref = ctx.keyswitch(lev, dev)
        out = torch.full((batch, 2, nl, n), -1, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        note("%s noalloc level %d batch %d" % (name, lev, batch))
        hk.arm(None)
        ctx.keyswitch_noalloc(lev, dev, out)
        torch.cuda.synchronize()
        assert hk.allocs == 0, "the call allocated through the hooks"
        assert torch.equal(out, ref)
        got = _from_ntt(ctx, out, nl).reshape(batch, 2, nl, n)
        assert np.array_equal(got[0], orc.keyswitch(lev, d2[0]))
    # a batch beyond the fixed scratch is refused with a clear error
    nl = L
    words = (3 * nl + 3 * (nl + ctx.alpha)) * n
    big = (64 << 20) // (8 * words) + 1
    dev = torch.zeros((big, nl, n), dtype=torch.int64, device="cuda")
    out = torch.zeros((big, 2, nl, n), dtype=torch.int64, device="cuda")
    with pytest.raises(sfhe.SfheError) as e:
        ctx.keyswitch_noalloc(L - 1, dev, out)
    assert e.value.code == -1 and "scratch" in str(e.value)
    ctx.close()
