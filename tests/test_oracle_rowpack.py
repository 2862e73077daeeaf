"""Pins of the oracle's multi-row packing (the coefficient packing of Sec. 4.3.1, as in
Cheetah): for d_in = K <= N, the n_o = floor(N / K) rows of a group share one weight
polynomial with row rho reversed in slot rho, and row rho's output is SampleExtract
(Sec. 3.2) at h = (rho + 1) K - 1.

Anchors: with K = N (one row per product) it is the standard product of Eq. (LWEdot);
the pure-Python big-integer version on tiny rings (single modulus, no RNS); and real
encryptions, where every output decrypts to W x and its phase equals
Delta (W x)_j + (E w_g)[h] exactly, the error term taken from numpy's integer
convolution folded by X^N = -1.
"""

import numpy as np
import pytest

from oracle import oracle as orc
from oracle import tiny
from paper_2505_07329_amd import synth
from tests.cases import make_case

P2048 = synth.PRIMES_2048
P4096 = synth.PRIMES_4096


@pytest.mark.parametrize("N,primes", [(2048, P2048), (4096, P4096)])
def test_one_row_per_product_is_the_standard_product(N, primes):
    g = np.random.default_rng(N)
    W = synth.int8_uniform(g, (5, N))
    ct = synth.uniform_mod_primes(g, primes, (2, 1, 2), N)
    assert orc.rows_per_product(N, N) == 1
    assert np.array_equal(orc.matmul_rowpacked(N, primes, W, ct), orc.matmul_clear(N, primes, W, ct))


@pytest.mark.parametrize("primes", [(97,), (97, 193)])
@pytest.mark.parametrize("K,d_out", [(3, 7), (4, 8), (5, 2), (8, 3), (16, 2)])
def test_matches_bigint_tiny_oracle(primes, K, d_out):
    N = 16
    g = np.random.default_rng(K * 10 + d_out)
    q = orc.modulus(primes)
    W = g.integers(-127, 128, size=(d_out, K)).astype(np.int8)
    A = [int(v) for v in g.integers(0, q, size=N)]
    B = [int(v) for v in g.integers(0, q, size=N)]
    ct = np.zeros((1, 1, 2, len(primes), N), dtype=np.uint64)
    for p, qp in enumerate(primes):
        ct[0, 0, 0, p] = [a % qp for a in A]
        ct[0, 0, 1, p] = [b % qp for b in B]
    got = orc.matmul_rowpacked(N, primes, W, ct)
    want = tiny.matmul_rowpacked(q, N, W.tolist(), (A, B))
    for j, (a, b) in enumerate(want):
        for p, qp in enumerate(primes):
            assert got[0, j, p, :N].tolist() == [v % qp for v in a]
            assert int(got[0, j, p, N]) == b % qp


def negacyclic_coeff(a, b, h):
    """Coefficient h of a * b mod X^N + 1 from numpy's integer convolution (int64 is exact
    here: |e| <= 19, |w| <= 127, N <= 4096 terms)."""
    N = len(a)
    full = np.convolve(np.asarray(a, dtype=np.int64), np.asarray(b, dtype=np.int64))
    return full[h] - (full[h + N] if h + N < len(full) else 0)


@pytest.mark.parametrize("N,primes,log2_t,K,d_out", [
    (2048, P2048, 24, 256, 20),    # 8 rows per product, the last group holds 4
    (4096, P4096, 26, 2048, 5),    # 2 rows per product
    (4096, P4096, 28, 1000, 9),    # 4 rows per product, 96 unused coefficients
])
def test_rowpacked_outputs_decrypt_with_exact_phase(N, primes, log2_t, K, d_out):
    case = make_case(N, primes, log2_t, d_out, K, 2, config=73, salt=K)
    out = orc.matmul_rowpacked(N, primes, case.W, case.ct)
    q = orc.modulus(primes)
    delta = q >> log2_t
    n_o = orc.rows_per_product(K, N)
    Wg = orc.rowpack_weights(case.W, N)
    v = case.x.astype(np.int64) @ case.W.T.astype(np.int64)
    ph = orc.lwe_phase(N, primes, case.S, out)
    for t in range(2):
        for j in range(d_out):
            g, rho = divmod(j, n_o)
            h = (rho + 1) * K - 1
            e_term = negacyclic_coeff(case.E[t, 0], Wg[g], h)
            assert ph[t * d_out + j] == delta * int(v[t, j]) + int(e_term)
            assert orc.decode(ph[t * d_out + j], delta) == v[t, j]
