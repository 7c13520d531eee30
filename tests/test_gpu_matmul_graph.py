"""The LAZY ct x ct product captured into a HIP graph (sfhe_matmul_graph_*):
every replay, with the program's own eager work and synchronisations between
replays, gives the eager product's ciphertexts bit for bit, on the fused
N = 2^14 path and on the unfused path of the smaller rings; one output is
checked against the oracle.  Every call goes through the C ABI."""
import numpy as np
import pytest

from paper_2503_09184_amd import workloads as W
from tests.test_gpu_parity import HYB_SMALL, note, pair, torch_cuda  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("params,shape,seed", [
    (W.PARAMS["realistic_n16384"], (40, 24, 26), 3),   # 1040 outputs: the fused kernels, slice tuning
    (HYB_SMALL, (9, 13, 7), 21),                      # unfused key switch and rescale
])
def test_graph_replays_equal_eager_product(torch_cuda, params, shape, seed):
    torch = torch_cuda
    from paper_2503_09184_amd import sfhe
    ctx, orc = pair(params, seed)
    M, K, Nc = shape
    A, B = W.operands(M, K, Nc, 0.5, 7000 + M)
    A[2, :] = 0.0                                      # a row with no product: trivial zeros
    EA, EB = ctx.encrypt(A, "csr", 7001, 0), ctx.encrypt(B, "dense", 7002, 1)
    note("graph %s eager" % (shape,))
    C = ctx.matmul(EA, EB, "lazy")
    eager = [ctx.export_ct(C, i, j) for i in range(M) for j in range(Nc)]
    eager_products = ctx.last_stats().products
    C.close()
    G = sfhe.MatmulGraph(ctx, EA, EB)
    A2, B2 = W.operands(5, 6, 3, 0.3, 7100)
    E2a, E2b = ctx.encrypt(A2, "ell", 7101, 0), ctx.encrypt(B2, "dense", 7102, 1)
    for rep in range(3):
        note("graph %s replay %d" % (shape, rep))
        G.launch()
        st = ctx.last_stats()
        assert st.products == eager_products
        assert st.keyswitches == int(np.count_nonzero(np.any(A != 0.0, axis=1))) * Nc
        R = G.result()
        got = [ctx.export_ct(R, i, j) for i in range(M) for j in range(Nc)]
        for n, (x, y) in enumerate(zip(got, eager)):
            assert np.array_equal(x, y), (rep, n)
        assert np.max(np.abs(ctx.decrypt(R) - A @ B)) < 1e-6
        # eager work of the program between replays
        X = ctx.matmul(E2a, E2b, "lazy")
        assert np.max(np.abs(ctx.decrypt(X) - A2 @ B2)) < 1e-6
        X.close()
        torch.cuda.synchronize()
    cts, _, _ = orc.matmul(A, B, "csr", "lazy", 7001, 7002, outputs=[(M - 1, Nc - 1)], threads=4, decrypt=False)
    assert np.array_equal(ctx.export_ct(G.result(), M - 1, Nc - 1), cts[0])
    G.close()
    for m in (EA, EB, E2a, E2b):
        m.close()
