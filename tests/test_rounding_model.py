"""CPU model of the GPU's fixed-point gadget rounding (Decomp's first step, Sec. 3.2):
a~ = round(c 2^K / q) mod 2^K from the residues c_p of c, with 32 fraction bits.

The model repeats the kernel's integer steps (32-bit partial products, 64-bit sums,
carries) with explicit masks and checks, against exact big-integer arithmetic, the two
facts the kernel relies on: the estimate of c 2^K / q is never above the exact value and
at most 7 units of 2^-32 below it, so outside an 8-unit window below each rounding
boundary its rounding is the exact one. Inputs: uniform residues, residues of c next to
rounding ties, and residues at the edge of the window.
"""

import random

import pytest

M32, M64 = (1 << 32) - 1, (1 << 64) - 1
P2 = (18014398509309953, 18014398509293569)
P1 = (18014398509404161,)


def constants(primes, K):
    """Per prime: f = floor(inv 2^K / q_p) mod 2^64 and G = floor(g 2^96 / q_p), with
    inv 2^K = f q_p + g, inv = (q / q_p)^-1 mod q_p (1 for one prime)."""
    q = 1
    for p in primes:
        q *= p
    out = []
    for p in primes:
        inv = pow(q // p, -1, p) if len(primes) > 1 else 1
        f, g = divmod(inv << K, p)
        out.append((f & M64, (g << 96) // p))
    return q, out


def estimate(cs, consts):
    """The kernel's sum, as (integer part mod 2^64, fraction in units of 2^-32)."""
    at, fr = 0, 0
    for c, (f, G) in zip(cs, consts):
        x0, x1 = c & M32, c >> 32
        G0, G1, G2 = G & M32, (G >> 32) & M32, G >> 64
        t = ((x0 * G1) >> 32) + ((x1 * G0) >> 32)
        t = t + x0 * G2
        assert t <= M64
        u, v = x1 * G1, x1 * G2
        s = (t + u) & M64
        carry = 1 if s < t else 0
        ip = ((s >> 32) + v + (carry << 32)) & M64
        at = (at + ((c * f) & M64) + ip) & M64
        f2 = (fr + (s & M32)) & M32
        at = (at + (1 if f2 < fr else 0)) & M64
        fr = f2
    return at, fr


def model_round(cs, consts, K):
    at, fr = estimate(cs, consts)
    sr = (fr + (1 << 31)) & M32
    at = (at + (1 if sr < fr else 0)) & M64
    near = sr >= 0xFFFFFFF8
    return at & ((1 << K) - 1), near


def exact_units(c, q, K):
    """floor(c 2^(K+32) / q) mod 2^(K+32): the exact value in units of 2^-32."""
    return ((c << (K + 32)) // q) % (1 << (K + 32))


def exact_round(c, q, K):
    return ((2 * (c << K) + q) // (2 * q)) % (1 << K)


def samples(q, K, rng, n):
    """Uniform c, c next to a tie (k + 1/2) q / 2^K, and c at the near window's edge."""
    out = [rng.randrange(q) for _ in range(n)]
    window = max(1, (8 * q) >> (K + 32))  # 8 units of 2^-32 in steps of c
    for _ in range(n):
        k = rng.randrange(1 << K)
        tie = ((2 * k + 1) * q) >> (K + 1)
        out.append(min(q - 1, max(0, tie + rng.randrange(-1000, 1001))))
        d = window // 2 + rng.randrange(window + 1)
        out.append(min(q - 1, max(0, tie + (d if rng.random() < 0.5 else -d))))
    return out


@pytest.mark.parametrize("primes,beta,ell", [
    (P2, 54, 1), (P2, 27, 2), (P2, 16, 4), (P2, 32, 2),
    (P1, 12, 3), (P1, 54, 1), (P1, 20, 2),
])
def test_estimate_bound_and_rounding(primes, beta, ell):
    K = beta * ell
    q, consts = constants(primes, K)
    rng = random.Random(20250507 + K + len(primes))
    near_count = 0
    for c in samples(q, K, rng, 3000):
        cs = [c % p for p in primes]
        at, fr = estimate(cs, consts)
        est = ((at << 32) | fr) % (1 << (K + 32))
        deficit = (exact_units(c, q, K) - est) % (1 << (K + 32))
        assert 0 <= deficit < 7, (c, deficit)
        got, near = model_round(cs, consts, K)
        if near:
            near_count += 1
        else:
            assert got == exact_round(c, q, K), c
    if (8 * q) >> (K + 32):  # the window spans values of c: the near-tie samples reach it
        assert near_count > 0


def test_residues_need_not_be_reduced():
    """Adding q_p to a residue adds inv_p 2^K, a multiple of 2^K: same rounding."""
    K = 54
    q, consts = constants(P2, K)
    rng = random.Random(7)
    for _ in range(500):
        c = rng.randrange(q)
        cs = [c % p for p in P2]
        base, near = model_round(cs, consts, K)
        lifted, near2 = model_round([cs[0] + P2[0], cs[1] + 3 * P2[1]], consts, K)
        if not (near or near2):
            assert lifted == base == exact_round(c, q, K)


@pytest.mark.parametrize("primes,beta,ell", [(P2, 54, 1), (P2, 27, 2), (P1, 54, 1)])
def test_deficit_bound_for_residues_near_2_64(primes, beta, ell):
    """Residues lifted by multiples of q_p up to just below 2^64 (any unreduced input):
    the estimate stays at most 7 units below the exact value and rounds exactly outside
    the window."""
    K = beta * ell
    q, consts = constants(primes, K)
    rng = random.Random(64 + K + len(primes))
    for c in samples(q, K, rng, 1500):
        cs = []
        for p in primes:
            r = c % p
            top = (M64 - r) // p  # largest lift below 2^64
            cs.append(r + p * (top - rng.randrange(min(top, 4) + 1)))
        assert all(x <= M64 for x in cs)
        at, fr = estimate(cs, consts)
        est = ((at << 32) | fr) % (1 << (K + 32))
        deficit = (exact_units(c, q, K) - est) % (1 << (K + 32))
        assert 0 <= deficit <= 7, (c, deficit)
        got, near = model_round(cs, consts, K)
        if not near:
            assert got == exact_round(c, q, K), c
