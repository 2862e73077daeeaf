"""Pins of the oracle's ring arithmetic R_q = Z_q[X]/(X^N+1) (Sec. 3.1).

Each check is anchored outside the oracle's own formulas: exhaustive monomial
products (X^N = -1), numpy's integer convolution folded by X^N = -1, ring
axioms, the defining property psi^N = -1 of the NTT root, and a pure-Python
big-integer product over the full modulus.
"""

import numpy as np
import pytest

from oracle import oracle as orc
from oracle import tiny
from paper_2505_07329_amd import synth

P2048 = synth.PRIMES_2048
P4096 = synth.PRIMES_4096


def monomial(N, a, q):
    v = np.zeros(N, dtype=np.uint64)
    v[a] = 1
    return v


@pytest.mark.parametrize("N,q", [(8, 17), (16, 97)])
@pytest.mark.parametrize("which", ["schoolbook", "ntt"])
def test_monomial_products_exhaustive(N, q, which):
    mul = orc.poly_mul_schoolbook if which == "schoolbook" else orc.poly_mul_ntt
    for a in range(N):
        for b in range(N):
            got = mul(monomial(N, a, q), monomial(N, b, q), q)
            want = np.zeros(N, dtype=np.uint64)
            if a + b < N:
                want[a + b] = 1
            else:
                want[a + b - N] = q - 1  # X^N = -1
            assert np.array_equal(got, want), (a, b)


@pytest.mark.parametrize("N,q", [(2048, P2048[0]), (4096, P4096[0]), (4096, P4096[1]), (16, 97)])
def test_psi_is_primitive_2N_root(N, q):
    psi = orc.find_psi(N, q)
    assert psi != 0
    assert pow(psi, N, q) == q - 1
    assert pow(psi, 2 * N, q) == 1


@pytest.mark.parametrize("N", [8, 64, 256])
def test_schoolbook_matches_numpy_convolution(N):
    g = np.random.default_rng(N)
    q = P4096[1]
    a = g.integers(-100, 101, N)
    b = g.integers(-100, 101, N)
    full = np.convolve(a, b)  # exact in int64 for these magnitudes
    folded = full[:N].copy()
    folded[: N - 1] -= full[N:]
    want = np.array([int(v) % q for v in folded], dtype=np.uint64)
    got = orc.poly_mul_schoolbook(np.array([int(v) % q for v in a], dtype=np.uint64),
                                  np.array([int(v) % q for v in b], dtype=np.uint64), q)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("N,q", [(8, P2048[0]), (64, P4096[0]), (512, P4096[1]), (2048, P2048[0]),
                                 (4096, P4096[0])])
def test_ntt_matches_schoolbook(N, q):
    g = np.random.default_rng(N + q % 1000)
    a = g.integers(0, q, N, dtype=np.uint64)
    b = g.integers(0, q, N, dtype=np.uint64)
    assert np.array_equal(orc.poly_mul_ntt(a, b, q), orc.poly_mul_schoolbook(a, b, q))


def test_ring_axioms():
    N, q = 256, P4096[0]
    g = np.random.default_rng(7)
    a, b, c = (g.integers(0, q, N, dtype=np.uint64) for _ in range(3))
    mul = lambda x, y: orc.poly_mul_ntt(x, y, q)
    add = lambda x, y: np.array([(int(u) + int(v)) % q for u, v in zip(x, y)], dtype=np.uint64)
    assert np.array_equal(mul(a, b), mul(b, a))
    assert np.array_equal(mul(a, add(b, c)), add(mul(a, b), mul(a, c)))
    assert np.array_equal(mul(mul(a, b), c), mul(a, mul(b, c)))
    one = monomial(N, 0, q)
    assert np.array_equal(mul(a, one), a)


def test_tiny_bigint_product_matches_c():
    N, q = 16, 97 * 193  # composite modulus: tiny works over Z_q, C per prime
    g = np.random.default_rng(3)
    a = [int(v) for v in g.integers(0, q, N)]
    b = [int(v) for v in g.integers(0, q, N)]
    want = tiny.negacyclic_mul(a, b, q)
    for p in (97, 193):
        got = orc.poly_mul_schoolbook(np.array([v % p for v in a], dtype=np.uint64),
                                      np.array([v % p for v in b], dtype=np.uint64), p)
        assert [int(v) for v in got] == [v % p for v in want]
