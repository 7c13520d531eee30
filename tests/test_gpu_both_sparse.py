"""GPU parity with both operands sparse (the naive scheme's two masks of
Sec. 3.3.2, and CSR / ELLPACK on the right operand): a product is skipped
when A_ik or B_kj is zero.  The HIP library against the CPU oracle on the
same seeded inputs, bit for bit in the coefficient domain."""
import numpy as np
import pytest

from paper_2503_09184_amd import workloads as W
from tests.test_gpu_parity import HYB_SMALL, note, pair, torch_cuda, _threads  # noqa: F401

pytestmark = pytest.mark.gpu


def _relu_like(B, seed, frac):
    """Zero a fraction of B's entries (i.i.d.), as a ReLU does to activations."""
    u = np.random.default_rng(seed).random(B.shape)
    B = B.copy()
    B[u < frac] = 0.0
    return B


@pytest.mark.parametrize("sched", ["lazy", "per_product"])
@pytest.mark.parametrize("encs", [("csr", "csr"), ("naive", "naive"), ("ell", "ell"), ("dense", "csr"),
                                  ("csr", "naive"), ("ell", "csr")])
def test_both_sparse_ragged_all_outputs(torch_cuda, encs, sched):
    """19 x 23 x 10 with a ragged row tile and column group, an empty row of A
    and an all-zero column of B (trivial zeros), five 60/40-bit primes."""
    ea, eb = encs
    ctx, orc = pair(HYB_SMALL, 21)
    A, B = W.operands(19, 23, 10, 0.5, 81)
    B = _relu_like(B, 82, 0.5)
    A[4, :] = 0.0
    B[:, 6] = 0.0
    note("both sparse %s x %s %s" % (ea, eb, sched))
    C = ctx.matmul(ctx.encrypt(A, ea, 31, 0), ctx.encrypt(B, eb, 32, 1), sched)
    cts, _, _ = orc.matmul(A, B, ea, sched, 31, 32, threads=4, encB=eb)
    for i in range(19):
        for j in range(10):
            assert np.array_equal(ctx.export_ct(C, i, j), cts[i * 10 + j]), (i, j)
    dec = ctx.decrypt(C)
    assert np.all(dec[:, 6] == 0.0)
    assert np.max(np.abs(dec - A @ B)) < 1e-6
    st = ctx.last_stats()
    want = sum(1 for i in range(19) for j in range(10) for k in range(23)
               if (A[i, k] != 0.0 or ea == "dense") and B[k, j] != 0.0)
    assert st.products == want


@pytest.mark.parametrize("sparsity", [0.5, 0.9])
def test_both_sparse_realistic_sampled_outputs(torch_cuda, sparsity):
    """128 x 128 x 128 at N = 2^14 (the benchmarked parameters) with A at the
    given sparsity and B with half its entries zero, both CSR, lazy schedule:
    sampled outputs bit-exact against the oracle, the same under the naive
    encodings, every output within 1e-6 of the fp64 product."""
    P = W.PARAMS["realistic_n16384"]
    ctx, orc = pair(P, W.key_seed(3))
    A, B = W.operands(128, 128, 128, sparsity, W.workload_seed(3))
    B = _relu_like(B, 83, 0.5)
    sa, sb = W.enc_seed(3, 0), W.enc_seed(3, 1)
    sample = [(0, 0), (127, 127), (5, 90), (64, 64), (100, 3), (31, 32)]
    outs = {}
    for enc in ("csr", "naive"):
        note("both sparse realistic %.2f %s" % (sparsity, enc))
        C = ctx.matmul(ctx.encrypt(A, enc, sa, 0), ctx.encrypt(B, enc, sb, 1), "lazy")
        outs[enc] = [ctx.export_ct(C, i, j) for (i, j) in sample]
        if enc == "csr":
            err = np.max(np.abs(ctx.decrypt(C) - A @ B))
            note("both sparse realistic max |err| %.3e" % err)
            assert err < 1e-6
        C.close()
    for x, y in zip(outs["csr"], outs["naive"]):
        assert np.array_equal(x, y)
    cts, _, _ = orc.matmul(A, B, "csr", "lazy", sa, sb, outputs=sample, threads=_threads(), encB="csr")
    for n, o in enumerate(outs["csr"]):
        assert np.array_equal(o, cts[n]), sample[n]
