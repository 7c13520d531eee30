"""Brute-force references on tiny inputs, in Python integers.

These are the pins of the oracle: textbook definitions written out with
arbitrary-precision integers and no transforms, used only on small rings.
"""


def negacyclic(a, b, q):
    """a*b in Z_q[X]/(X^N + 1), schoolbook."""
    n = len(a)
    out = [0] * n
    for i in range(n):
        ai = int(a[i])
        if ai == 0:
            continue
        for j in range(n):
            k = i + j
            v = ai * int(b[j])
            if k < n:
                out[k] += v
            else:
                out[k - n] -= v
    return [x % q for x in out]


def poly_add(a, b, q):
    return [(int(x) + int(y)) % q for x, y in zip(a, b)]


def poly_sub(a, b, q):
    return [(int(x) - int(y)) % q for x, y in zip(a, b)]


def evaluate(a, x, q):
    """a(x) mod q by Horner."""
    acc = 0
    for c in reversed(list(a)):
        acc = (acc * x + int(c)) % q
    return acc


def bitrev(x, bits):
    r = 0
    for _ in range(bits):
        r = (r << 1) | (x & 1)
        x >>= 1
    return r


def crt(residues, moduli):
    """The integer in [0, prod moduli) with the given residues."""
    M = 1
    for m in moduli:
        M *= m
    x = 0
    for r, m in zip(residues, moduli):
        Mi = M // m
        x += int(r) * Mi * pow(Mi, -1, m)
    return x % M


def centered(x, M):
    x %= M
    return x - M if x > (M - 1) // 2 else x


def prod(xs):
    p = 1
    for x in xs:
        p *= int(x)
    return p
