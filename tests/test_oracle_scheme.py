"""Pins of the oracle's scheme: RLWE encryption (Sec. 3.1), SampleExtract (Sec. 3.2)
and the encrypted clear-weight product of Eq. (LWEdot) (Sec. 4.3).

The anchor is mathematical: every output LWE must decrypt to the exact integer
product, and its phase must equal Delta*(W x)_j + (W e)_j with e the encryption
error; special inputs (A = 1, A = X^m, S = E = 0, x = e_k, W = I) have closed
forms; a pure-Python big-integer implementation over the full modulus must agree.
"""

import numpy as np
import pytest

from oracle import oracle as orc
from oracle import tiny
from paper_2505_07329_amd import synth
from tests.cases import exact_phase_targets, make_case

P2048 = synth.PRIMES_2048
P4096 = synth.PRIMES_4096


def test_rlwe_phase_is_message_plus_error():
    N, primes, log2_t = 512, P4096, 26
    g = np.random.default_rng(1)
    S = synth.ternary(g, N)
    A = synth.uniform_mod_primes(g, primes, (3,), N)
    E = synth.rounded_gaussian(g, (3, N))
    msg = synth.int8_uniform(g, (3, N)).astype(np.int64)
    B = orc.encrypt(N, primes, log2_t, S, A, E, msg)
    ph = orc.rlwe_phase(N, primes, S, A, B)
    q, d = orc.modulus(primes), orc.delta(primes, log2_t)
    for c in range(3):
        for k in range(0, N, 37):
            val = orc.centered(orc.crt(primes, ph[c, :, k]), q)
            assert val == d * int(msg[c, k]) + int(E[c, k])


def test_encrypt_schoolbook_equals_ntt():
    N, primes = 256, P2048
    g = np.random.default_rng(2)
    S = synth.ternary(g, N)
    A = synth.uniform_mod_primes(g, primes, (2,), N)
    E = synth.rounded_gaussian(g, (2, N))
    msg = synth.int8_uniform(g, (2, N)).astype(np.int64)
    assert np.array_equal(orc.encrypt(N, primes, 24, S, A, E, msg, use_ntt=False),
                          orc.encrypt(N, primes, 24, S, A, E, msg, use_ntt=True))


def test_sample_extract_closed_forms():
    N, q = 8, 17
    A = np.arange(1, N + 1, dtype=np.uint64)
    B = np.arange(101, 101 + N, dtype=np.uint64) % q
    a, b = orc.sample_extract(A, B, q, N - 1)
    # h = N-1: a'_i = A_{N-1-i}, no negation
    assert [int(v) for v in a] == [int(A[N - 1 - i]) for i in range(N)]
    assert b == int(B[N - 1])
    a, b = orc.sample_extract(A, B, q, 0)
    # h = 0: a'_0 = A_0, a'_i = -A_{N-i}
    assert [int(v) for v in a] == [int(A[0])] + [(q - int(A[N - i])) % q for i in range(1, N)]
    assert b == int(B[0])


@pytest.mark.parametrize("h", [0, 1, 100, 255])
def test_sample_extract_decrypts_coefficient(h):
    N, primes, log2_t = 256, P2048, 24
    g = np.random.default_rng(h)
    S = synth.ternary(g, N)
    A = synth.uniform_mod_primes(g, primes, (), N)
    E = synth.rounded_gaussian(g, (N,))
    msg = synth.int8_uniform(g, (N,)).astype(np.int64)
    B = orc.encrypt(N, primes, log2_t, S, A, E, msg)
    q = primes[0]
    a, b = orc.sample_extract(A[0], B[0], q, h)
    lwe = np.concatenate([a, np.array([b], dtype=np.uint64)]).reshape(1, 1, N + 1)
    ph = orc.lwe_phase(N, primes, S, lwe)[0]
    assert ph == orc.delta(primes, log2_t) * int(msg[h]) + int(E[h])


def check_decrypts(case, out, pairs):
    targets = exact_phase_targets(case)
    phases = orc.lwe_phase(case.N, case.primes, case.S, out)
    v_true = case.x.astype(object) @ case.W.T.astype(object)
    for (t, j), ph in zip(pairs, phases):
        assert ph == targets[t, j], (t, j)
        assert orc.decode(ph, case.delta) == v_true[t, j]


def test_matmul_config1_decrypts_exactly():
    """256x256, 16 tokens, N=2048, one prime, t=2^24: every output, phase exact."""
    case = make_case(2048, P2048, 24, 256, 256, 16, config=1)
    out = orc.matmul_clear(case.N, case.primes, case.W, case.ct, mode=1)
    pairs = orc.all_pairs(16, 256)
    check_decrypts(case, out.reshape(-1, 1, case.N + 1), pairs)


def test_matmul_attention_shape_sampled():
    """2048x2048 at N=4096 with two primes, t=2^26, on sampled outputs."""
    case = make_case(4096, P4096, 26, 2048, 2048, 3, config=2)
    pairs = np.array([(0, 0), (0, 2047), (1, 1000), (2, 5), (2, 1999)], dtype=np.uint32)
    out = orc.matmul_clear(case.N, case.primes, case.W, case.ct, pairs=pairs)
    check_decrypts(case, out, pairs)


def test_matmul_two_blocks_sampled():
    """d_in = 8192 > N = 4096 (L = 2), t=2^28: the MLP down-projection shape."""
    case = make_case(4096, P4096, 28, 64, 8192, 2, config=3)
    pairs = np.array([(0, 0), (1, 63), (1, 17)], dtype=np.uint32)
    out = orc.matmul_clear(case.N, case.primes, case.W, case.ct, pairs=pairs)
    check_decrypts(case, out, pairs)


def test_matmul_schoolbook_equals_ntt():
    case = make_case(256, P4096, 26, 24, 300, 2, config=9)
    a = orc.matmul_clear(case.N, case.primes, case.W, case.ct, mode=0)
    b = orc.matmul_clear(case.N, case.primes, case.W, case.ct, mode=1)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("d_in", [63, 64, 65, 127, 128])
def test_block_boundaries_decrypt(d_in):
    N = 64
    case = make_case(N, P4096, 26, 9, d_in, 2, config=10, salt=d_in)
    out = orc.matmul_clear(case.N, case.primes, case.W, case.ct)
    check_decrypts(case, out.reshape(-1, 2, N + 1), orc.all_pairs(2, 9))


def test_block_additivity():
    """[W0 | W1] applied to [c0; c1] equals W0 c0 + W1 c1 (sum over blocks)."""
    N, primes = 64, P4096
    case = make_case(N, primes, 26, 5, 2 * N, 2, config=11)
    full = orc.matmul_clear(N, primes, case.W, case.ct)
    part0 = orc.matmul_clear(N, primes, case.W[:, :N], case.ct[:, :1])
    part1 = orc.matmul_clear(N, primes, case.W[:, N:], case.ct[:, 1:])
    for p, q in enumerate(primes):
        s = (part0[:, :, p].astype(object) + part1[:, :, p].astype(object)) % q
        assert np.array_equal(s.astype(np.uint64), full[:, :, p])


def test_linearity_in_weights():
    N, primes = 128, P4096
    g = np.random.default_rng(5)
    W1 = g.integers(-60, 61, (6, 200)).astype(np.int8)
    W2 = g.integers(-60, 61, (6, 200)).astype(np.int8)
    case = make_case(N, primes, 26, 6, 200, 2, config=12, W=W1)
    o1 = orc.matmul_clear(N, primes, W1, case.ct)
    o2 = orc.matmul_clear(N, primes, W2, case.ct)
    o12 = orc.matmul_clear(N, primes, (W1.astype(np.int16) + W2).astype(np.int8), case.ct)
    for p, q in enumerate(primes):
        s = (o1[:, :, p].astype(object) + o2[:, :, p].astype(object)) % q
        assert np.array_equal(s.astype(np.uint64), o12[:, :, p])


def unit_mask_ct(N, primes, T, m, B=None):
    """Ciphertext layout with A = X^m (and the given bodies) for a 1-block input."""
    ct = np.zeros((T, 1, 2, len(primes), N), dtype=np.uint64)
    ct[:, 0, 0, :, m] = 1
    if B is not None:
        ct[:, 0, 1] = B
    return ct


@pytest.mark.parametrize("m", [0, 1, 37, 63])
def test_mask_closed_form_monomial(m):
    """A = X^m: a'_n = w[n+m] for n+m < N, -w[n+m-N] otherwise (w zero past d_in)."""
    N, primes, d_in = 64, P4096, 50
    g = np.random.default_rng(m)
    W = synth.int8_uniform(g, (3, d_in))
    out = orc.matmul_clear(N, primes, W, unit_mask_ct(N, primes, 1, m))
    wpad = np.zeros((3, 2 * N), dtype=np.int64)
    wpad[:, :d_in] = W
    for j in range(3):
        for p, q in enumerate(primes):
            for n in range(N):
                want = wpad[j, n + m] if n + m < N else -wpad[j, n + m - N]
                assert int(out[0, j, p, n]) == want % q


def test_zero_secret_zero_error_body_is_scaled_product():
    N, primes, log2_t = 128, P4096, 26
    case = make_case(N, primes, log2_t, 7, 100, 3, config=13, zero_secret=True, zero_error=True)
    out = orc.matmul_clear(N, primes, case.W, case.ct)
    v = case.x.astype(object) @ case.W.T.astype(object)
    for p, q in enumerate(primes):
        for t in range(3):
            for j in range(7):
                assert int(out[t, j, p, N]) == (case.delta * v[t, j]) % q


def test_unit_vectors_and_identity():
    N, primes, log2_t = 64, P2048, 24
    d = 40
    x = np.zeros((d, d), dtype=np.int8)
    np.fill_diagonal(x, 1)
    g = np.random.default_rng(9)
    W = synth.int8_uniform(g, (5, d))
    case = make_case(N, primes, log2_t, 5, d, d, config=14, W=W, x=x)
    out = orc.matmul_clear(N, primes, W, case.ct)
    ph = orc.lwe_phase(N, primes, case.S, out)
    dec = np.array([orc.decode(p, case.delta) for p in ph]).reshape(d, 5)
    assert np.array_equal(dec, W.T.astype(np.int64))  # x = e_k -> column k of W
    xi = synth.int8_uniform(g, (3, d))
    case = make_case(N, primes, log2_t, d, d, 3, config=14, W=np.eye(d, dtype=np.int8), x=xi)
    out = orc.matmul_clear(N, primes, case.W, case.ct)
    ph = orc.lwe_phase(N, primes, case.S, out)
    dec = np.array([orc.decode(p, case.delta) for p in ph]).reshape(3, d)
    assert np.array_equal(dec, xi.astype(np.int64))  # W = I -> x


def test_tiny_bigint_matmul_matches_c():
    """Pure-Python big ints over q = 97*193 (no RNS) against the residue-wise C oracle."""
    N, primes = 16, (97, 193)
    q = 97 * 193
    g = np.random.default_rng(11)
    W = g.integers(-5, 6, (4, 40)).astype(np.int8)
    L = 3
    A = [[int(v) for v in g.integers(0, q, N)] for _ in range(L)]
    B = [[int(v) for v in g.integers(0, q, N)] for _ in range(L)]
    ref = tiny.matmul_clear(q, N, W.astype(int).tolist(), list(zip(A, B)))
    ct = np.zeros((1, L, 2, 2, N), dtype=np.uint64)
    for i in range(L):
        for p, pr in enumerate(primes):
            ct[0, i, 0, p] = [v % pr for v in A[i]]
            ct[0, i, 1, p] = [v % pr for v in B[i]]
    out = orc.matmul_clear(N, primes, W, ct)
    for j, (a, b) in enumerate(ref):
        for p, pr in enumerate(primes):
            assert [int(v) for v in out[0, j, p, :N]] == [v % pr for v in a]
            assert int(out[0, j, p, N]) == b % pr
