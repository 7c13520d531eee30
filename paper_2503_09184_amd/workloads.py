"""Seeded synthetic operands shaped like the paper's sweeps.

This module holds input generation only -- none of the encrypted arithmetic.
Both the GPU library's tests/benchmark and the CPU oracle receive the plain
fp64 matrices it returns.

Operands follow the profiling procedure of Sec. 4.1 (random square matrices
with a set fraction of zeros), with these distributions:
values i.i.d. uniform on [-1, 1], zeros placed by an i.i.d. Bernoulli mask on
A only (B dense), so a row's nonzero count is Binomial(K, 1 - s).  Masks are
nested: element (i, k) is zero iff its mask draw u_ik < s, so for one seed the
zero set at a higher sparsity contains the one at a lower sparsity.
"""
import numpy as np

#: master seed of the synthetic operands for a workload index c
MASTER_SEED = 0x2503091840000000


def workload_seed(c):
    return MASTER_SEED + int(c)


def uniform_matrix(rows, cols, seed):
    """fp64 values uniform on [-1, 1], never exactly 0.0."""
    rng = np.random.default_rng(np.random.PCG64(int(seed)))
    v = rng.uniform(-1.0, 1.0, size=(rows, cols))
    v[v == 0.0] = 0.5
    return v


def sparse_matrix(rows, cols, sparsity, seed):
    """Uniform values with an i.i.d. Bernoulli(sparsity) zero mask."""
    rng = np.random.default_rng(np.random.PCG64(int(seed)))
    v = rng.uniform(-1.0, 1.0, size=(rows, cols))
    v[v == 0.0] = 0.5
    u = rng.random(size=(rows, cols))
    v[u < float(sparsity)] = 0.0
    return v


def operands(M, K, Nc, sparsity, seed):
    """(A, B): A is M x K with the zero mask, B is K x Nc dense."""
    A = sparse_matrix(M, K, sparsity, seed)
    B = uniform_matrix(K, Nc, seed ^ 0x5A5A5A5A)
    return A, B


# Parameter sets.  Bit sizes of the data primes (q) and the special primes (p);
# dnum digits of alpha = len(p) data primes each.
PARAMS = {
    # N = 2^10, toy and insecure: two 60-bit data primes, one 60-bit special prime
    "toy_n1024": dict(log_n=10, q_bits=[60, 60], p_bits=[60], dnum=2),
    # N = 2^13: 60/40/40-bit data primes, one 60-bit special prime
    "sweep_n8192": dict(log_n=13, q_bits=[60, 40, 40], p_bits=[60], dnum=3),
    # N = 2^14: 60 + 4 x 40-bit data primes, three 60-bit special primes, dnum = 2
    "realistic_n16384": dict(log_n=14, q_bits=[60, 40, 40, 40, 40], p_bits=[60, 60, 60], dnum=2),
    # N = 2^14 for plaintext weights times encrypted values: the same five data
    # primes and one 60-bit special prime (unused: no relinearisation)
    "plain_n16384": dict(log_n=14, q_bits=[60, 40, 40, 40, 40], p_bits=[60], dnum=5),
    # N = 2^15 for the serving loop: a 60-bit and eight 40-bit data primes,
    # three 60-bit special primes, dnum = 3
    "serving_n32768": dict(log_n=15, q_bits=[60] + [40] * 8, p_bits=[60, 60, 60], dnum=3),
}


def uneven_batch(seed, count=32, dims=(32, 64, 128, 256), sparsity=(0.5, 0.9)):
    """Shapes of a batch of independent products W B: (M, K, Nc, s) with each
    of M, K, Nc drawn uniformly from dims and the zero fraction s of W uniform
    on the sparsity interval."""
    rng = np.random.default_rng(np.random.PCG64(int(seed)))
    out = []
    for _ in range(count):
        M, K, Nc = (int(x) for x in rng.choice(np.asarray(dims), size=3))
        out.append((M, K, Nc, float(rng.uniform(*sparsity))))
    return out

# Seeds for keys and encryptions derived from a workload seed.
def key_seed(seed):
    return (int(seed) * 0x9E3779B97F4A7C15 + 0x11) & 0xFFFFFFFFFFFFFFFF


def enc_seed(seed, operand):
    return (int(seed) * 0xBF58476D1CE4E5B9 + 0x1234 + int(operand)) & 0xFFFFFFFFFFFFFFFF
