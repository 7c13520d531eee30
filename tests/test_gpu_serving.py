"""GPU tests of the request loop (sfhe_server_*): requests admitted by
memory and batched as they arrive give each result bit for bit as when the
request runs alone, and match the CPU oracle.  Every call goes through the C
ABI."""
import numpy as np
import pytest

from paper_2503_09184_amd import workloads as W
from tests.test_gpu_parity import HYB_SMALL, note, pair, torch_cuda  # noqa: F401

pytestmark = pytest.mark.gpu

# (M, K, b, weight sparsity) of the test requests
REQS = [(20, 37, 3, 0.5), (16, 9, 1, 0.75), (33, 20, 5, 0.9), (7, 37, 2, 0.5), (20, 37, 4, 0.75), (1, 5, 1, 0.0)]


def _requests(ctx):
    out = []
    for n, (M, K, b, s) in enumerate(REQS):
        Wt, X = W.operands(M, K, b, s, 300 + n)
        out.append((Wt, X, ctx.encode_weights(Wt, "csr", 40), ctx.encrypt(X, "dense", 400 + n, 1)))
    return out


def _bytes(ctx, M, b):
    L = len(ctx.primes) - ctx.alpha
    return M * b * (2 * L + 2 * (L - 1)) * ctx.n * 8


def _cts(ctx, C, M, b):
    return [ctx.export_ct(C, i, j) for i in range(M) for j in range(b)]


def test_serving_mix_equals_alone_and_oracle(torch_cuda):
    from paper_2503_09184_amd import sfhe
    ctx, orc = pair(HYB_SMALL, 21)
    reqs = _requests(ctx)
    # alone: one server per request, one step each
    alone = []
    for n, (Wt, X, Wp, EX) in enumerate(reqs):
        note("serving alone %d" % n)
        srv = sfhe.Server(ctx, 1 << 40)
        t = srv.submit(Wp, EX)
        assert srv.step() == 1
        done, C, ms, bs = srv.poll(t, wait=True)
        assert done and bs == 1
        alone.append(_cts(ctx, C, REQS[n][0], REQS[n][2]))
        srv.close()
    # the mix: a budget of about two requests, requests arriving while batches run
    budget = 2 * max(_bytes(ctx, M, b) for (M, K, b, s) in REQS)
    srv = sfhe.Server(ctx, budget)
    tickets = [srv.submit(reqs[0][2], reqs[0][3])]
    assert srv.step() == 1
    for n in range(1, len(reqs)):
        tickets.append(srv.submit(reqs[n][2], reqs[n][3]))
    note("serving mix")
    results, sizes = {}, []
    for _ in range(1000):
        srv.step()
        for n, t in enumerate(tickets):
            if n in results:
                continue
            done, C, ms, bs = srv.poll(t)
            if done:
                results[n] = C
                sizes.append(bs)
        if len(results) == len(tickets):
            break
    assert len(results) == len(tickets)
    st = srv.status()
    assert st["queued"] == 0 and st["running"] == 0 and st["bytes_in_flight"] == 0
    assert st["batches"] >= 2 and max(sizes) >= 2          # admitted by memory, batched
    for n, (M, K, b, s) in enumerate(REQS):
        got = _cts(ctx, results[n], M, b)
        for x, y in zip(got, alone[n]):
            assert np.array_equal(x, y), n
    # against the oracle
    Wt, X = reqs[2][0], reqs[2][1]
    cts, _, _ = orc.matmul_plain(Wt, X, "csr", 402, 40, threads=4)
    for x, y in zip(_cts(ctx, results[2], 33, 5), cts):
        assert np.array_equal(x, y)
    dec = ctx.decrypt(results[0])
    assert np.max(np.abs(dec - reqs[0][0] @ reqs[0][1])) < 1e-6
    srv.close()


def test_serving_rejects_oversized_requests(torch_cuda):
    from paper_2503_09184_amd import sfhe
    ctx, _ = pair(HYB_SMALL, 21)
    reqs = _requests(ctx)
    srv = sfhe.Server(ctx, _bytes(ctx, 20, 3))
    with pytest.raises(sfhe.SfheError) as e:
        srv.submit(reqs[2][2], reqs[2][3])                   # 33 x 5 outputs
    assert e.value.code == -7
    t = srv.submit(reqs[0][2], reqs[0][3])                   # exactly the budget
    assert srv.step() == 1
    assert srv.poll(t, wait=True)[0]
    srv.close()
