"""GPU tests of the request loop (sfhe_server_*): requests admitted by
memory and batched as they arrive give each result bit for bit as when the
request runs alone, and match the CPU oracle.  Every call goes through the C
ABI."""
import time

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
    """sums and results alone (a lower bound of what the server counts)"""
    L = len(ctx.primes) - ctx.alpha
    return M * b * (2 * L + 2 * (L - 1)) * ctx.n * 8


def _counted(srv, req):
    return srv.request_bytes(req[2], req[3])


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
    probe = sfhe.Server(ctx, 1 << 40)
    budget = 2 * max(_counted(probe, r) for r in reqs)
    probe.close()
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
    probe = sfhe.Server(ctx, 1 << 40)
    need = _counted(probe, reqs[0])
    probe.close()
    assert need > _bytes(ctx, 20, 3)                         # scratch and tables are counted too
    srv = sfhe.Server(ctx, need)
    with pytest.raises(sfhe.SfheError) as e:
        srv.set_slots(-1)
    assert e.value.code == -1
    with pytest.raises(sfhe.SfheError) as e:
        srv.submit(reqs[2][2], reqs[2][3])                   # 33 x 5 outputs
    assert e.value.code == -7
    t = srv.submit(reqs[0][2], reqs[0][3])                   # exactly the budget
    assert srv.step() == 1
    assert srv.poll(t, wait=True)[0]
    srv.close()


def test_serving_policies_fifo_and_slot_limit(torch_cuda):
    """One stream: batches run in admission order (their device-time
    intervals do not intersect and follow the tickets).  Two streams with one
    slot each: never more than two batches running, requests that find both
    streams busy wait and join a later batch.  Every result equals the
    request alone."""
    from paper_2503_09184_amd import sfhe
    ctx, _ = pair(HYB_SMALL, 21)
    reqs = _requests(ctx)
    alone = []
    for n, (Wt, X, Wp, EX) in enumerate(reqs):
        srv = sfhe.Server(ctx, 1 << 40)
        t = srv.submit(Wp, EX)
        srv.step()
        alone.append(_cts(ctx, srv.poll(t, wait=True)[1], REQS[n][0], REQS[n][2]))
        srv.close()
    for n_streams, slots in ((1, 0), (2, 1)):
        note("serving policy %d streams, %d slots" % (n_streams, slots))
        srv = sfhe.Server(ctx, 1 << 40, n_streams=n_streams, slots=slots)
        tickets = []
        for Wt, X, Wp, EX in reqs:
            tickets.append(srv.submit(Wp, EX))
            srv.step()                                           # one request per step while a slot is free
            assert srv.status()["running"] <= (n_streams * slots if slots else len(tickets))
        results = {}
        for _ in range(1000):
            srv.step()
            assert srv.status()["running"] <= (n_streams * slots if slots else len(tickets))
            for n, t in enumerate(tickets):
                if n not in results:
                    done, C, _, _ = srv.poll(t)
                    if done:
                        results[n] = C
            if len(results) == len(tickets):
                break
        assert len(results) == len(tickets)
        if n_streams == 1:
            iv = [srv.intervals[t] for t in tickets]
            assert all(iv[x][1] <= iv[x + 1][0] + 1e-3 or iv[x] == iv[x + 1] for x in range(len(iv) - 1)), iv
        for n, (M, K, b, s) in enumerate(REQS):
            for x, y in zip(_cts(ctx, results[n], M, b), alone[n]):
                assert np.array_equal(x, y), (n_streams, slots, n)
        srv.close()


def test_batch_byte_limit(torch_cuda):
    """With a batch limit of about two requests' bytes, every batch holds at
    most what fits the limit (a request larger than it runs alone), the
    requests still run in ticket order on one stream, and every result equals
    the request alone."""
    from paper_2503_09184_amd import sfhe
    ctx, _ = pair(HYB_SMALL, 21)
    reqs = _requests(ctx)
    probe = sfhe.Server(ctx, 1 << 40)
    sizes = [_counted(probe, r) for r in reqs]
    probe.close()
    cap = sorted(sizes)[len(sizes) // 2] * 2
    alone = []
    for n, (Wt, X, Wp, EX) in enumerate(reqs):
        srv = sfhe.Server(ctx, 1 << 40)
        t = srv.submit(Wp, EX)
        srv.step()
        alone.append(_cts(ctx, srv.poll(t, wait=True)[1], REQS[n][0], REQS[n][2]))
        srv.close()
    note("serving batch limit %d bytes" % cap)
    srv = sfhe.Server(ctx, 1 << 40, batch_bytes=cap)
    tickets = [srv.submit(Wp, EX) for Wt, X, Wp, EX in reqs]
    while srv.status()["queued"]:
        srv.step()
    results, batch_of = {}, {}
    for n, t in enumerate(tickets):
        done, C, _, bs = srv.poll(t, wait=True)
        assert done
        results[n] = C
        batch_of[n] = srv.intervals[t]
    groups = {}
    for n, iv in batch_of.items():
        groups.setdefault(iv, []).append(n)
    assert len(groups) > 1
    for members in groups.values():
        assert len(members) == 1 or sum(sizes[n] for n in members) <= cap, (members, cap)
        assert members == list(range(members[0], members[0] + len(members)))   # consecutive tickets
    for n, (M, K, b, s) in enumerate(REQS):
        for x, y in zip(_cts(ctx, results[n], M, b), alone[n]):
            assert np.array_equal(x, y), n
    assert sfhe.lib().sfhe_server_set_batch_bytes(None, 5) == -1           # SFHE_E_INVALID_ARG
    srv.close()


@pytest.mark.parametrize("torch_allocator", [True, False])
def test_results_outlive_the_server(torch_cuda, torch_allocator):
    """A result polled from a server stays valid after the server (and its
    streams) is destroyed, and is freed afterwards, with torch's allocator
    and with the library's own stream-ordered pool; servers created one after
    another reuse the memory of the results freed in between."""
    from paper_2503_09184_amd import sfhe
    ctx = sfhe.Context(**HYB_SMALL, torch_allocator=torch_allocator)
    ctx.keygen(21)
    reqs = _requests(ctx)
    keep = []
    for rep in range(3):
        note("result outlives server %s %d" % (torch_allocator, rep))
        srv = sfhe.Server(ctx, 1 << 40, n_streams=2)
        t = srv.submit(reqs[0][2], reqs[0][3])
        assert srv.step() == 1
        done, C, _, _ = srv.poll(t, wait=True)
        assert done
        srv.close()
        keep.append((C, _cts(ctx, C, REQS[0][0], REQS[0][2])))
    for C, cts in keep:
        assert all(np.array_equal(x, y) for x, y in zip(_cts(ctx, C, REQS[0][0], REQS[0][2]), keep[0][1]))
        C.close()
    torch_cuda.cuda.synchronize()


# (M, K, b, weight sparsity) of the requests at the serving ring
REQS15 = [(48, 14, 8, 0.5), (5, 7, 1, 0.75), (12, 14, 3, 0.9), (3, 14, 2, 0.0), (20, 7, 4, 0.5)]


def test_serving_ring_n32768_mix_equals_alone_and_oracle(torch_cuda):
    """The request loop at the serving ring (N = 2^15, nine data and three
    special primes) with small layers: requests submitted while a batch runs
    are admitted on the server's other streams and their batches overlap the
    running one on the device (intersecting device-time intervals); each
    request's result is the same, bit for bit, alone and in the mix; one
    request matches the oracle on every output, another decrypts within
    1e-6."""
    from paper_2503_09184_amd import sfhe
    ctx, orc = pair(W.PARAMS["serving_n32768"], 22)
    reqs = []
    for n, (M, K, b, s) in enumerate(REQS15):
        Wt, X = W.operands(M, K, b, s, 500 + n)
        reqs.append((Wt, X, ctx.encode_weights(Wt, "csr", 40), ctx.encrypt(X, "dense", 600 + n, 1)))
    alone = []
    for n, (Wt, X, Wp, EX) in enumerate(reqs):
        note("n15 serving alone %d" % n)
        srv = sfhe.Server(ctx, 1 << 40)
        t = srv.submit(Wp, EX)
        assert srv.step() == 1
        done, C, _, bs = srv.poll(t, wait=True)
        assert done and bs == 1
        alone.append(_cts(ctx, C, REQS15[n][0], REQS15[n][2]))
        C.close()
        srv.close()
    budget = 3 * max(_counted(srv, r) for r in reqs)
    srv = sfhe.Server(ctx, budget, n_streams=2)
    tickets = [srv.submit(reqs[0][2], reqs[0][3])]
    assert srv.step() == 1
    tickets += [srv.submit(Wp, EX) for (_, _, Wp, EX) in reqs[1:]]
    note("n15 serving mix")
    results = {}
    t_end = time.time() + 60.0
    while len(results) < len(tickets) and time.time() < t_end:
        srv.step()
        for n, t in enumerate(tickets):
            if n not in results:
                done, C, _, _ = srv.poll(t)
                if done:
                    results[n] = C
        time.sleep(0.001)
    assert len(results) == len(tickets)
    assert srv.status()["batches"] >= 2
    iv = sorted(set(srv.intervals[t] for t in tickets))
    note("n15 batch intervals %s" % iv)
    assert len(iv) >= 2
    assert any(iv[x][0] < iv[y][1] and iv[y][0] < iv[x][1] for x in range(len(iv)) for y in range(x + 1, len(iv))), \
        "no two batches overlapped on the device"
    for n, (M, K, b, s) in enumerate(REQS15):
        for x, y in zip(_cts(ctx, results[n], M, b), alone[n]):
            assert np.array_equal(x, y), n
    note("n15 serving oracle")
    cts, _, _ = orc.matmul_plain(reqs[2][0], reqs[2][1], "csr", 602, 40, threads=8)
    for x, y in zip(_cts(ctx, results[2], 12, 3), cts):
        assert np.array_equal(x, y)
    assert np.max(np.abs(ctx.decrypt(results[0]) - reqs[0][0] @ reqs[0][1])) < 1e-6
    for C in results.values():
        C.close()
    srv.close()
