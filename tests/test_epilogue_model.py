"""CPU model of the switched epilogue of the NTT product kernel (ModulusSwitch, Sec. 3.2):
round(c 2^k / q) mod 2^k from unreduced residues c_p of a coefficient c.

The kernel forms X = sum_p c_p H_p mod 2^32 in 32.32 fixed point, H_p = ((q/q_p)^-1 mod
q_p) 2^32 / q_p held as h_p = floor(crt_p 2^128 / q_p) mod 2^128, taking only the
partial products of c_p h_p at and above bit 64 (a 64-bit word per prime; the kernel
sums the words of all primes in one accumulation, `fixed_sum`). The model repeats those
integer steps (32-bit halves, 64-bit wrapping sums) and checks, against exact
big-integer arithmetic, the facts the kernel relies on:
  * the estimate is never above floor(c 2^64 / q) mod 2^64 and at most 7 units of
    2^-32 below it, for any 64-bit lift of the residues (the inverse transform hands
    over values below 64 q_p, not reduced);
  * its rounding to 2^k (k = 1..32) is the exact rounding unless the fraction lies
    within 8 units below one half (then the kernel recomputes exactly; its flag, the
    low word of the estimate plus one half at least 2^32 - 8, covers that window);
  * values next to rounding ties reach that window.
Inputs: uniform c, random lifts of its residues, c next to ties of every k tested,
c at the window's edge; one prime (N = 2048 parameters) and two (N = 4096).
"""

import random

import pytest

M32, M64 = (1 << 32) - 1, (1 << 64) - 1
P2 = (18014398509309953, 18014398509293569)
P1 = (18014398509404161,)


def modulus(primes):
    q = 1
    for p in primes:
        q *= p
    return q


def epilogue_constants(primes):
    """h_p = floor(crt_p 2^128 / q_p) mod 2^128 as four 32-bit words (little-endian)."""
    q = modulus(primes)
    hs = []
    for p in primes:
        crt = pow(q // p, -1, p) if len(primes) > 1 else 1
        h = ((crt << 128) // p) & ((1 << 128) - 1)
        hs.append([(h >> (32 * w)) & M32 for w in range(4)])
    return hs


def fixed_part(c, h):
    """The kernel's word: bits 64..127 of c h mod 2^128 without the partial products
    that end below bit 64 (c0 h0 and the low halves of c0 h1, c1 h0)."""
    c0, c1 = c & M32, c >> 32
    a = ((c0 * h[1]) >> 32) + ((c1 * h[0]) >> 32)
    a = (a + c0 * h[2] + c1 * h[1]) & M64
    a = (a + ((((c0 * h[3]) + (c1 * h[2])) & M32) << 32)) & M64
    return a


def estimate(cs, hs):
    a = 0
    for c, h in zip(cs, hs):
        a = (a + fixed_part(c, h)) & M64
    return a


def round_qout(W, k):
    """The kernel's rounding of 32.32 fixed point W to 2^k: value, and the fraction
    minus one half in units of W."""
    sh = 64 - k
    frac = W & ((1 << sh) - 1)
    half = 1 << (sh - 1)
    val = ((W >> sh) + (1 if frac >= half else 0)) & ((1 << k) - 1)
    return val, frac - half


def fixed_sum(cs, hs, bias):
    """The kernel's accumulation of the same words for all primes at once: bias, then
    per prime the two full products and the two high products into a 64-bit sum, and
    the low halves of the top products into a separate 32-bit high word."""
    a, hi = bias, 0
    for c, h in zip(cs, hs):
        c0, c1 = c & M32, c >> 32
        a = (a + c0 * h[2] + c1 * h[1] + ((c0 * h[1]) >> 32) + ((c1 * h[0]) >> 32)) & M64
        hi = (hi + c0 * h[3] + c1 * h[2]) & M32
    hi = (hi + (a >> 32)) & M32
    return a & M32, hi


def round_qout_near(vlo, vhi, k):
    """The NTT kernel's form of the same rounding from the words of V = W + one half
    (mod 2^64): value vhi >> (32 - k) = V >> (64 - k), and the window flag: the low word
    of V at least 2^32 - 8."""
    return vhi >> (32 - k), vlo >= (1 << 32) - 8


def round_qout_low8(W, k):
    """round_qout_near of W + one half."""
    V = (W + (1 << (63 - k))) & M64
    return round_qout_near(V & M32, V >> 32, k)


def exact_units(c, q):
    return ((c << 64) // q) & M64


def exact_round(c, q, k):
    return ((2 * (c << k) + q) // (2 * q)) % (1 << k)


def lift(c, p, rng, bound):
    """A residue of c mod p lifted by a random multiple of p, below `bound`."""
    r = c % p
    return r + p * rng.randrange((bound - r) // p)


def near_tie_values(q, k, rng, n, span_units=8):
    """c whose exact c 2^k / q lies within span_units units of 2^-32 (of c 2^32 / q) of
    a rounding tie m + 1/2, on either side."""
    out = []
    step = max(1, q >> 64)  # one unit of 2^-32 of c 2^32 / q in steps of c (two primes)
    for _ in range(n):
        m = rng.randrange(1 << k)
        tie = ((2 * m + 1) * q) >> (k + 1)
        d = rng.randrange(-span_units * step, span_units * step + 1)
        out.append(min(q - 1, max(0, tie + d)))
    return out


@pytest.mark.parametrize("primes", [P2, P1])
@pytest.mark.parametrize("k", [32, 26, 20, 1])
def test_epilogue_estimate_and_rounding(primes, k):
    q = modulus(primes)
    hs = epilogue_constants(primes)
    rng = random.Random(20250507 + 17 * k + len(primes))
    values = [rng.randrange(q) for _ in range(2000)] + near_tie_values(q, k, rng, 2000)
    values += [0, 1, q - 1, (q - 1) // 2, (q + 1) // 2]
    window_hits = 0
    for c in values:
        for bound in (64 * max(primes), 1 << 64):  # the transform's bound, any 64-bit lift
            cs = [lift(c, p, rng, bound) for p in primes]
            A = estimate(cs, hs)
            deficit = (exact_units(c, q) - A) & M64
            assert 0 <= deficit <= 7, (c, cs, deficit)
            val, near = round_qout_low8(A, k)
            if near:
                window_hits += 1
            else:
                assert val == exact_round(c, q, k), (c, k)
    if len(primes) == 2:  # the window spans values of c: the near-tie draws reach it
        assert window_hits > 0


def test_window_needs_the_exact_route():
    """Some coefficients just above a tie are estimated below it (inside the window): a
    kernel that skipped the exact route there would round them down, one unit wrong."""
    q = modulus(P2)
    hs = epilogue_constants(P2)
    rng = random.Random(5)
    wrong_if_skipped = 0
    for c in near_tie_values(q, 32, rng, 4000, span_units=4):
        A = estimate([c % p for p in P2], hs)
        val, dist = round_qout(A, 32)
        if -8 <= dist < 0 and val != exact_round(c, q, 32):
            wrong_if_skipped += 1
    assert wrong_if_skipped > 0


@pytest.mark.parametrize("k", list(range(1, 33)))
def test_rounding_forms_agree(k):
    """round_qout_low8 (the NTT epilogue) gives round_qout's value and flags every
    fraction 1..8 units below one half (exactly those at k = 32; at k < 32 also those
    whose fraction is 1..8 units below any multiple of 2^32, which only take the exact
    route), for W next to every kind of boundary: the half, the integer steps, the
    window's edges, and the wrap past 2^64."""
    sh = 64 - k
    half = 1 << (sh - 1)
    rng = random.Random(1000 + k)
    Ws = [0, 1, M64, M64 - 7, M64 - 8, half, half - 1]
    for _ in range(300):
        m = rng.randrange(1 << k)
        base = m << sh
        for d in range(-12, 12):
            Ws.append((base + half + d) & M64)  # around the tie
            Ws.append((base + d) & M64)         # around the integer step
        Ws.append(rng.randrange(1 << 64))
    for W in Ws:
        v_ref, dist = round_qout(W, k)
        v, near = round_qout_low8(W, k)
        assert v == v_ref, (W, k)
        if -8 <= dist < 0:
            assert near, (W, k, dist)
        elif near:
            assert k < 32 and (dist + 8) % (1 << 32) < 8, (W, k, dist)
    # uniform fractions: the false alarms have probability 2^-29 each
    assert not any(round_qout_low8(rng.randrange(1 << 64), k)[1] for _ in range(20000))


def test_fixed_sum_equals_the_per_prime_words():
    """The kernel's single accumulation (fixed_sum) equals the sum of the per-prime
    words plus the bias, mod 2^64, for any 64-bit lifts."""
    rng = random.Random(11)
    for primes in (P2, P1):
        hs = epilogue_constants(primes)
        for _ in range(3000):
            cs = [rng.randrange(1 << 64) for _ in primes]
            bias = rng.randrange(1 << 64)
            lo, hi = fixed_sum(cs, hs, bias)
            assert (hi << 32 | lo) == (estimate(cs, hs) + bias) & M64


def last_stage_twiddle(p, N):
    """psi^-bitrev(1) mod p for the psi-twisted inverse transform of degree N: the one
    twiddle of its last stage (span N/2). bitrev(1) over log2 N bits is N/2, so this is
    psi^(-N/2), a primitive fourth root of unity."""
    for g in range(2, 100000):
        psi = pow(g, (p - 1) // (2 * N), p)
        if pow(psi, N, p) == p - 1:
            return pow(pow(psi, p - 2, p), N // 2, p)
    raise AssertionError("no 2N-th root")


@pytest.mark.parametrize("primes,N", [(P2, 4096), (P1, 2048)])
@pytest.mark.parametrize("k", [32, 26, 1])
def test_last_stage_twiddle_folded_into_constants(primes, N, k):
    """The switched epilogue of the NTT product takes the last inverse stage's
    differences d (coefficient = d w mod p, w that stage's twiddle) with constants
    built from crt w mod p: the estimate keeps the 0..7-unit deficit against the exact
    value of the coefficient, and rounds exactly outside the window."""
    q = modulus(primes)
    ws = [last_stage_twiddle(p, N) for p in primes]
    for p, w in zip(primes, ws):
        assert pow(w, 4, p) == 1 and pow(w, 2, p) == p - 1
    hl = []
    for p, w in zip(primes, ws):
        crt = pow(q // p, -1, p) if len(primes) > 1 else 1
        h = (((crt * w % p) << 128) // p) & ((1 << 128) - 1)
        hl.append([(h >> (32 * i)) & M32 for i in range(4)])
    rng = random.Random(77 + k + len(primes))
    values = [rng.randrange(q) for _ in range(1500)] + near_tie_values(q, k, rng, 1500)
    for c in values:
        # residues of c divided by w, lifted as the transform hands them over
        ds = [lift(c * pow(w, p - 2, p) % p, p, rng, 64 * p) for p, w in zip(primes, ws)]
        A = estimate(ds, hl)
        deficit = (exact_units(c, q) - A) & M64
        assert 0 <= deficit <= 7, (c, deficit)
        val, near = round_qout_low8(A, k)
        if not near:
            assert val == exact_round(c, q, k)


# ---------------------------------------------------------------------------------
# Switched epilogue of the matrix-core product: V = sum_l 255^l S_l (S_l the int32 digit
# sums of the balanced base-255 expansion), c 2^32 / q mod 2^32 formed per digit in 32.32
# fixed point from G_l = round(255^l 2^96 / q) mod 2^96 in balanced 32-bit words.

def digit_constants(q, D):
    """The (a, b, c) words of every digit: G_l = a + b 2^32 + c 2^64, a and b in
    [-2^31, 2^31) (the host's table)."""
    out = []
    for l in range(D):
        num = pow(255, l) % q
        G = ((num << 96) + q // 2) // q  # round to nearest (q odd)
        a = G & M32
        a = a - (1 << 32) if a >= 1 << 31 else a
        g1 = (G - a) >> 32
        b = g1 & M32
        b = b - (1 << 32) if b >= 1 << 31 else b
        c = ((g1 - b) >> 32) & M32
        assert G == a + (b << 32) + (c << 64)
        out.append((a, b, c))
    return out


def switch_plan(q, D, maxS):
    """The host's choice of kept digits and uncertainty band (units of 2^-32)."""
    l0 = 0
    for c in range(1, D):
        if maxS * ((255.0 ** c - 1) / 254.0) * 2.0 ** 32 / q <= 2.0 ** -16:
            l0 = c
    dk = D - l0
    if D == 7:
        dk = 7
    else:
        dk = max(dk, 8)
        if dk == 13:
            dk = 14
    l0 = D - dk
    skipped = maxS * ((255.0 ** l0 - 1) / 254.0) * 2.0 ** 32 / q
    import math
    band = math.ceil(2.0 * skipped * 2.0 ** 32) + 2 * dk + 4
    return l0, dk, band


def digit_word(S, abc):
    """The kernel's word of one digit: floor(S a / 2^32) + S b + (S c mod 2^32) 2^32."""
    a, b, c = abc
    return ((S * a) >> 32) + S * b + (((S * c) & M32) << 32)


@pytest.mark.parametrize("primes", [P2, P1])
@pytest.mark.parametrize("k", [32, 26, 1])
@pytest.mark.parametrize("K", [512, 2048, 8192])
def test_matrix_core_digit_epilogue(primes, k, K):
    """The per-digit fixed-point sum stays within the host's band of the exact value, and
    rounds exactly outside it, for digit sums up to the bound of K int8 products; digit
    sums are drawn at random, at the bound, and next to rounding ties of V."""
    q = modulus(primes)
    D = 14 if len(primes) == 2 else 7
    maxS = 127 * 127 * K
    l0, dk, band = switch_plan(q, D, maxS)
    G = digit_constants(q, D)
    rng = random.Random(K + 3 * k + len(primes))
    sh = 64 - k
    checked = window = 0
    for trial in range(1500):
        S = [rng.randrange(-maxS, maxS + 1) for _ in range(D)]
        if trial % 7 == 0:
            S = [maxS if rng.random() < 0.5 else -maxS for _ in range(D)]
        if trial % 3 == 1:
            # move V next to a rounding tie of c 2^k / q: add the balanced base-255 digits
            # of the difference (at most 127 each) to digit sums drawn below maxS - 127
            S = [rng.randrange(-maxS + 127, maxS - 126) for _ in range(D)]
            V = sum(pow(255, l) * s for l, s in enumerate(S))
            m = rng.randrange(1 << k)
            tie = ((2 * m + 1) * q) >> (k + 1)
            delta = (tie - V % q + rng.randrange(-2, 3) * pow(255, l0)) % q
            delta = delta - q if delta > q // 2 else delta
            for l in range(D):
                dl = ((delta + 127) % 255) - 127
                S[l] += dl
                delta = (delta - dl) // 255
            assert delta == 0
        V = sum(pow(255, l) * s for l, s in enumerate(S))
        c = V % q
        W = sum(digit_word(S[l], G[l]) for l in range(l0, D)) & M64
        exact = exact_units(c, q)  # floor(c 2^64 / q) mod 2^64
        err = ((W - exact + (1 << 63)) & M64) - (1 << 63)
        assert abs(err) <= band, (err, band)
        V_ = (W + (1 << (sh - 1))) & M64
        amb = (((V_ + band) << k) & M64) < ((2 * band) << k)
        if not amb:
            assert V_ >> sh == exact_round(c, q, k), (k, c)
            checked += 1
        else:
            window += 1
    assert checked >= 1000
    if len(primes) == 2:  # the near-tie draws reach the exact route (one prime: a window of
        assert window > 0  # 2 dk + 4 units, narrower than one step of c)
