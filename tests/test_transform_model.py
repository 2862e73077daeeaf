"""CPU models of the lazy arithmetic of the NTT product's inverse transform (Sec. 4.5:
the pointwise product in the evaluation domain, then the inverse transform), checked
against exact integer arithmetic:
  * the truncated-quotient Shoup product returns a value congruent to a w and below 4p
    for every 64-bit a (the quotient drops the partial products below bit 64);
  * the Barrett step returns a value congruent to v and below 3p for every 64-bit v;
  * the pass schedule of the inverse (three radix-2 Gentleman-Sande stages per pass,
    sums left unreduced, each difference biased by its pass's bound, a Barrett step on
    two elements of eight after every second pass) never lets a value reach 2^64 nor a
    biased difference go negative, at N = 4096 and 2048, with the last stage's
    differences multiplied or handed to the epilogue unmultiplied;
  * run on numbers, that schedule gives the exact transform mod p.
"""

import random

import pytest

M32, M64 = (1 << 32) - 1, (1 << 64) - 1
PRIMES = (18014398509309953, 18014398509293569, 18014398509404161)


def mul_shoup4(a, w, wp, p):
    """The kernel's product: q = a1 wp1 + hi(a0 wp1) + hi(a1 wp0) (64-bit wrap),
    r = a w - q p taken mod 2^64 (as a w + q (2^64 - p))."""
    a0, a1 = a & M32, a >> 32
    wp0, wp1 = wp & M32, wp >> 32
    q = (a1 * wp1 + ((a0 * wp1) >> 32) + ((a1 * wp0) >> 32)) & M64
    return (a * w + q * ((1 << 64) - p)) & M64


def reduce_barrett(v, p):
    """The kernel's Barrett step: q = hi(v_hi floor(2^64 / p)), r = v - q p mod 2^64."""
    bm = ((1 << 64) // p) & M32
    q = ((v >> 32) * bm) >> 32
    return (v + q * ((1 << 64) - p)) & M64


@pytest.mark.parametrize("p", PRIMES)
def test_shoup_product_bound(p):
    rng = random.Random(p & 0xffff)
    ws = [1, p - 1, rng.randrange(p), rng.randrange(p)]
    As = [0, 1, M64, M64 - 1, p, 4 * p - 1, 512 * p - 1] + [rng.randrange(1 << 64) for _ in range(3000)]
    for w in ws:
        wp = (w << 64) // p
        for a in As:
            r = mul_shoup4(a, w, wp, p)
            assert r < 4 * p and r % p == a * w % p, (a, w)


@pytest.mark.parametrize("p", PRIMES)
def test_barrett_bound(p):
    rng = random.Random(7 + (p & 0xff))
    for v in [0, 1, p - 1, p, M64, M64 - 1, 512 * p - 1] + [rng.randrange(1 << 64) for _ in range(5000)]:
        r = reduce_barrett(v, p)
        assert r < 3 * p and r % p == v % p, v


def passes(N):
    """(S, EIN, END) of the four passes: spans S, 2S, 4S; inputs below 8p 2^EIN; END:
    elements k = 0, 1 (k = (pos / S) mod 8) reduced at the end."""
    return [(1, 0, False), (8, 3, True), (64, 0, False), (N // 8, 3, False)]


def skipped(P, t):
    return P == 3 and t <= 256  # at N = 2048 the span-256 stage is the third pass's last


@pytest.mark.parametrize("N", [4096, 2048])
@pytest.mark.parametrize("lastmul", [True, False])
def test_inverse_schedule_bounds(N, lastmul):
    """Interval model: upper bounds per position, a product below 4p, a sum the sum of
    its inputs' bounds, a biased difference X + B - Y below X + B and never negative."""
    for p in PRIMES:
        bound = [8 * p] * N  # pointwise sums: two blocks of products below 4p
        worst = 0
        for P, (S, ein, end) in enumerate(passes(N)):
            assert max(bound) <= (8 * p) << ein, (P, max(bound))  # the pass's entry bound
            B = (8 * p) << (2 + ein)  # the bias of every difference of the pass
            for st in range(3):
                t = S << st
                if skipped(P, t):
                    continue
                last = P == 3 and st == 2
                for pos in range(N):
                    if pos & t:
                        continue
                    X, Y = bound[pos], bound[pos + t]
                    assert X <= B and Y <= B, (P, st)  # X + B - Y >= 0
                    bound[pos] = X + Y
                    bound[pos + t] = X + B if (last and not lastmul) else 4 * p
                    worst = max(worst, X + Y, X + B)
            if end:
                for pos in range(N):
                    if (pos // S) % 8 < 2:
                        bound[pos] = 3 * p
        assert worst < 1 << 63 and max(bound) <= 512 * p, (p, worst)


def reference_inverse(x, tw, p):
    """The same butterflies with every value reduced mod p."""
    x = list(x)
    N = len(x)
    t = 1
    while t < N:
        for pos in range(N):
            if pos & t:
                continue
            X, Y = x[pos], x[pos + t]
            x[pos] = (X + Y) % p
            x[pos + t] = (X - Y) * tw[(pos, t)] % p
        t <<= 1
    return x


@pytest.mark.parametrize("N", [4096, 2048])
def test_inverse_schedule_numbers(N):
    """The lazy schedule on numbers (inputs at the bound and random, arbitrary twiddles):
    every value stays below 2^64 and the outputs are congruent to the reduced ones."""
    p = PRIMES[0] if N == 4096 else PRIMES[2]
    rng = random.Random(N)
    tw = {}
    t = 1
    while t < N:
        for pos in range(N):
            if not pos & t:
                tw[(pos, t)] = rng.randrange(1, p)
        t <<= 1
    for inputs in ([8 * p - 1] * N, [rng.randrange(8 * p) for _ in range(N)]):
        x = list(inputs)
        for P, (S, ein, end) in enumerate(passes(N)):
            B = (8 * p) << (2 + ein)
            for st in range(3):
                t = S << st
                if skipped(P, t):
                    continue
                for pos in range(N):
                    if pos & t:
                        continue
                    X, Y = x[pos], x[pos + t]
                    d = X + B - Y
                    assert 0 <= d <= M64 and X + Y <= M64
                    w = tw[(pos, t)]
                    x[pos] = X + Y
                    x[pos + t] = mul_shoup4(d, w, (w << 64) // p, p)
            if end:
                for pos in range(N):
                    if (pos // S) % 8 < 2:
                        x[pos] = reduce_barrett(x[pos], p)
        ref = reference_inverse([v % p for v in inputs], tw, p)
        assert all(v % p == r for v, r in zip(x, ref))
        assert max(x) < 512 * p
