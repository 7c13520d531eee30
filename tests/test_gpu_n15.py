"""GPU parity at N = 2^15 (the serving parameters: a 60-bit and eight
40-bit data primes, three 60-bit special primes, dnum = 3), where a row is
transformed as a first stage across its two halves and two 2^14-point
halves.  Ciphertexts bit-exact against the CPU oracle through the C ABI."""
import numpy as np
import pytest

from paper_2503_09184_amd import workloads as W
from tests.test_gpu_parity import note, pair, torch_cuda, _threads  # noqa: F401

pytestmark = pytest.mark.gpu

P15 = W.PARAMS["serving_n32768"]


def test_n15_encryption_matches_oracle(torch_cuda):
    ctx, orc = pair(P15, 7)
    A = W.uniform_matrix(2, 3, 90)
    note("n15 encrypt")
    EA = ctx.encrypt(A, "dense", 55, 0)
    for (i, j) in [(0, 0), (1, 2)]:
        assert np.array_equal(ctx.export_ct(EA, i, j), orc.encrypt(A[i, j], 55, 0, i, j)), (i, j)
    assert np.max(np.abs(ctx.decrypt(EA) - A)) < 1e-6


@pytest.mark.parametrize("sched", ["lazy", "per_product"])
def test_n15_matmul_all_outputs(torch_cuda, sched):
    ctx, orc = pair(P15, 7)
    A, B = W.operands(5, 6, 3, 0.5, 91)
    note("n15 matmul %s" % sched)
    C = ctx.matmul(ctx.encrypt(A, "csr", 56, 0), ctx.encrypt(B, "dense", 57, 1), sched)
    cts, _, _ = orc.matmul(A, B, "csr", sched, 56, 57, threads=_threads())
    for i in range(5):
        for j in range(3):
            assert np.array_equal(ctx.export_ct(C, i, j), cts[i * 3 + j]), (i, j)
    assert np.max(np.abs(ctx.decrypt(C) - A @ B)) < 1e-6


def test_n15_plain_product_all_outputs(torch_cuda):
    ctx, orc = pair(P15, 7)
    Wt, X = W.operands(18, 9, 4, 0.5, 92)
    note("n15 plain product")
    C = ctx.matmul_plain(ctx.encode_weights(Wt, "csr", 40), ctx.encrypt(X, "dense", 58, 1))
    cts, _, _ = orc.matmul_plain(Wt, X, "csr", 58, 40, threads=_threads())
    for i in range(18):
        for j in range(4):
            assert np.array_equal(ctx.export_ct(C, i, j), cts[i * 4 + j]), (i, j)
    assert np.max(np.abs(ctx.decrypt(C) - Wt @ X)) < 1e-6
