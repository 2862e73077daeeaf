"""Pins of the oracle's KeySwitch packing (Sec. 3.2 KeySwitching and Rotate, Sec. 4.3
Eq. (pack_rotate)); Decomp is the gadget decomposition of TFHE.

What fixes the oracle here, besides itself:
  * the big-integer version in ``oracle.tiny`` (full modulus q, no RNS, no NTT);
  * properties of the decomposition that follow from its definition: digit ranges,
    reconstruction within the rounding bound, exact values at chosen points;
  * closed forms: zero masks, a key-switching key without mask or error, rotation;
  * decryption of packed real encryptions to the clear integer products W x, inside a
    deterministic noise bound.
"""

from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as orc
from oracle import tiny
from paper_2505_07329_amd import synth
from tests.cases import make_case

P2 = synth.PRIMES_4096  # = 1 mod 8192: NTT-friendly for every N <= 4096
P1 = synth.PRIMES_2048


def crt_int(primes, res):
    q = orc.modulus(primes)
    c = 0
    for p, r in zip(primes, res):
        Mp = q // p
        c += int(r) * Mp * pow(Mp % p, -1, p)
    return c % q


def to_res(primes, c):
    return [c % p for p in primes]


def centered(v, q):
    v %= q
    return v - q if v > q // 2 else v


def rand_res(g, primes, shape):
    out = np.empty(tuple(shape) + (len(primes),), dtype=np.uint64)
    for p, q in enumerate(primes):
        out[..., p] = g.integers(0, q, size=shape, dtype=np.uint64)
    return out


GADGETS = [(P2, 54, 1), (P2, 27, 2), (P2, 16, 4), (P2, 1, 1), (P2, 7, 9 - 1),
           (P1, 12, 3), (P1, 14, 3), (P1, 32, 2), (P1, 53, 1)]


@pytest.mark.parametrize("primes,beta,ell", GADGETS)
def test_decomp_matches_big_integers(primes, beta, ell):
    g = synth.rng(0, synth.P_MISC, 11)
    res = rand_res(g, primes, (300,))
    got = orc.decomp(primes, res, beta, ell)
    q = orc.modulus(primes)
    for r, d in zip(res, got):
        assert list(d) == tiny.decomp(crt_int(primes, r), q, beta, ell)


@pytest.mark.parametrize("primes,beta,ell", GADGETS)
def test_decomp_digits_and_reconstruction(primes, beta, ell):
    """Digits lie in [-2^(beta-1), 2^(beta-1)) and sum_m d_m g_m is c mod q up to the
    rounding of c / q to K = beta ell bits and of every g_m to an integer."""
    g = synth.rng(0, synth.P_MISC, 12)
    res = rand_res(g, primes, (400,))
    q = orc.modulus(primes)
    K = beta * ell
    gad = [crt_int(primes, r) for r in orc.gadget(primes, beta, ell)]
    assert gad == tiny.gadget(q, beta, ell)
    for m, gm in enumerate(gad):  # g_m is q / 2^(beta (m+1)) rounded
        assert abs(2 * gm * (1 << (beta * (m + 1))) - 2 * q) <= 1 << (beta * (m + 1))
    d = orc.decomp(primes, res, beta, ell)
    half = 1 << (beta - 1)
    assert d.min() >= -half and d.max() < half
    bound_x2 = -(-q // (1 << K)) + ell * half  # 2 * (q / 2^(K+1) + ell 2^(beta-2))
    worst = 0
    for r, dig in zip(res, d):
        c = crt_int(primes, r)
        err = centered(sum(int(x) * gm for x, gm in zip(dig, gad)) - c, q)
        worst = max(worst, abs(err))
        assert 2 * abs(err) <= bound_x2 + 2
    # where the rounding of c / q dominates, the bound is not loose by orders of magnitude
    if q >> K >= ell * half:
        assert 2 * worst >= bound_x2 // 64


@pytest.mark.parametrize("primes,beta,ell", [(P2, 54, 1), (P2, 20, 3), (P1, 12, 3)])
def test_decomp_special_points(primes, beta, ell):
    q = orc.modulus(primes)
    K = beta * ell
    pts = [0, 1, q - 1, q // 2, q // 2 + 1]
    g = synth.rng(0, synth.P_MISC, 13)
    targets = [int(v) for v in g.integers(0, 1 << min(K, 62), size=40, dtype=np.uint64)]
    # c = floor(v q / 2^K) has c 2^K / q in (v - 2^K / q, v]: with q > 2^(K+1) it
    # rounds to exactly v
    assert q > 1 << (K + 1)
    chosen = [((v * q) >> K, v) for v in targets]
    res = np.array([to_res(primes, c) for c in pts] + [to_res(primes, c) for c, _ in chosen],
                   dtype=np.uint64)
    d = orc.decomp(primes, res, beta, ell)
    assert (d[0] == 0).all()                  # c = 0
    assert (d[2] == 0).all()                  # c = q - 1 rounds to 2^K = 0 mod 2^K
    # c = 1 rounds to 0 (q > 2^(K+1) here) or to 1 (q < 2^(K+1))
    assert list(d[1]) == tiny.decomp(1, q, beta, ell)
    for (c, at), dig in zip(chosen, d[len(pts):]):
        val = sum(int(x) << (beta * (ell - 1 - m)) for m, x in enumerate(dig))
        assert val % (1 << K) == at


def ksk_inputs(N, primes, beta, ell, salt, zero_mask=False, zero_error=False):
    g_a = synth.rng(0, synth.P_MASK, 50 + salt)
    g_s = synth.rng(0, synth.P_SECRET, 50 + salt)
    g_e = synth.rng(0, synth.P_ERROR, 50 + salt)
    A = synth.uniform_mod_primes(g_a, primes, (N, ell), N)
    E = synth.rounded_gaussian(g_e, (N, ell, N))
    S_src = synth.ternary(g_s, N)
    S_dst = synth.ternary(g_s, N)
    if zero_mask:
        A[:] = 0
    if zero_error:
        E[:] = 0
    return S_src, S_dst, A, E


@pytest.mark.parametrize("primes,beta,ell", [(P2, 54, 1), (P1, 12, 3)])
def test_ksk_phase(primes, beta, ell):
    """Phase of KSK_{i,m} under S_dst: E_{i,m} plus S_src[i] g_m in the constant coefficient."""
    N = 32
    S_src, S_dst, A, E = ksk_inputs(N, primes, beta, ell, 1)
    ksk = orc.ksk_gen(N, primes, beta, ell, S_src, S_dst, A, E)
    assert (ksk[:, :, 0] == A).all()
    ph = orc.rlwe_phase(N, primes, S_dst, ksk[:, :, 0], ksk[:, :, 1])  # (N, ell, P, N)
    q = orc.modulus(primes)
    gad = tiny.gadget(q, beta, ell)
    for i in range(N):
        for m in range(ell):
            v = [centered(crt_int(primes, ph[i, m, :, n]), q) for n in range(N)]
            want = [int(e) for e in E[i, m]]
            want[0] += int(S_src[i]) * gad[m]
            assert v == [centered(w, q) for w in want]


def big_lwes(primes, lwe):
    return [([crt_int(primes, lwe[j, :, n]) for n in range(lwe.shape[2] - 1)],
             crt_int(primes, lwe[j, :, -1])) for j in range(lwe.shape[0])]


def big_ksk(primes, ksk):
    N, ell = ksk.shape[:2]
    return [[tuple([crt_int(primes, ksk[i, m, c, :, n]) for n in range(ksk.shape[-1])]
                   for c in range(2)) for m in range(ell)] for i in range(N)]


@pytest.mark.parametrize("primes,beta,ell,n_pack,M", [
    (P2, 54, 1, 16, 20), (P2, 18, 3, 7, 15), (P1, 12, 3, 16, 16), (P1, 20, 2, 5, 9)])
def test_pack_matches_big_integers(primes, beta, ell, n_pack, M):
    N = 16
    S_src, S_dst, A, E = ksk_inputs(N, primes, beta, ell, 2)
    ksk = orc.ksk_gen(N, primes, beta, ell, S_src, S_dst, A, E)
    g = synth.rng(0, synth.P_MISC, 14)
    lwe = synth.uniform_mod_primes(g, primes, (M,), N + 1)
    q = orc.modulus(primes)
    kb = big_ksk(primes, ksk)
    lb = big_lwes(primes, lwe)
    out0 = orc.keyswitch_pack(N, primes, beta, ell, lwe, ksk, n_pack, mode=0)
    out1 = orc.keyswitch_pack(N, primes, beta, ell, lwe, ksk, n_pack, mode=1)
    assert out0.shape == (-(-M // n_pack), 2, len(primes), N)
    assert (out0 == out1).all()
    for gi in range(out0.shape[0]):
        Ab, Bb = tiny.keyswitch_pack(lb[gi * n_pack:(gi + 1) * n_pack], kb, q, beta, ell)
        got_A = [crt_int(primes, out0[gi, 0, :, n]) for n in range(N)]
        got_B = [crt_int(primes, out0[gi, 1, :, n]) for n in range(N)]
        assert got_A == Ab and got_B == Bb


@pytest.mark.parametrize("primes,beta,ell", [(P2, 54, 1), (P1, 12, 3)])
def test_pack_modes_agree_ragged(primes, beta, ell):
    N = 64
    S_src, S_dst, A, E = ksk_inputs(N, primes, beta, ell, 3)
    ksk = orc.ksk_gen(N, primes, beta, ell, S_src, S_dst, A, E)
    g = synth.rng(0, synth.P_MISC, 15)
    lwe = synth.uniform_mod_primes(g, primes, (2 * N + 5,), N + 1)
    for n_pack in (N, 50):
        a = orc.keyswitch_pack(N, primes, beta, ell, lwe, ksk, n_pack, mode=0)
        b = orc.keyswitch_pack(N, primes, beta, ell, lwe, ksk, n_pack, mode=1)
        assert (a == b).all()


def test_pack_closed_forms():
    N, primes, beta, ell = 32, P2, 27, 2
    q = orc.modulus(primes)
    P = len(primes)
    g = synth.rng(0, synth.P_MISC, 16)
    lwe = synth.uniform_mod_primes(g, primes, (N,), N + 1)
    S_src, S_dst, A, E = ksk_inputs(N, primes, beta, ell, 4)
    ksk = orc.ksk_gen(N, primes, beta, ell, S_src, S_dst, A, E)
    # zero masks: KeySwitching is the trivial (0, b), packed bodies in slot order
    z = lwe.copy()
    z[:, :, :N] = 0
    out = orc.keyswitch_pack(N, primes, beta, ell, z, ksk, N)
    assert (out[0, 0] == 0).all()
    assert (out[0, 1] == lwe[:, :, N].T).all()
    # a key without mask or error: A = 0 and B_s = b_s - sum_i sum_m d_m(a_si) s_i g_m
    _, _, A0, E0 = ksk_inputs(N, primes, beta, ell, 4, zero_mask=True, zero_error=True)
    k0 = orc.ksk_gen(N, primes, beta, ell, S_src, S_dst, A0, E0)
    out = orc.keyswitch_pack(N, primes, beta, ell, lwe, k0, N)
    assert (out[0, 0] == 0).all()
    gad = tiny.gadget(q, beta, ell)
    for s in range(N):
        b = crt_int(primes, lwe[s, :, N])
        acc = b
        for i in range(N):
            dig = tiny.decomp(crt_int(primes, lwe[s, :, i]), q, beta, ell)
            acc -= sum(d * gm for d, gm in zip(dig, gad)) * int(S_src[i])
        assert crt_int(primes, out[0, 1, :, s]) == acc % q
    # rotation: one LWE in slot s (earlier slots hold (0, 0)) is X^s times the slot-0 result
    one = lwe[:1]
    base = orc.keyswitch_pack(N, primes, beta, ell, one, ksk, N)
    for s in (1, 5, N - 1):
        pad = np.zeros((s + 1, P, N + 1), dtype=np.uint64)
        pad[s] = one[0]
        rot = orc.keyswitch_pack(N, primes, beta, ell, pad, ksk, N)
        for c in range(2):
            for p, qp in enumerate(primes):
                want = tiny.rotate([int(v) for v in base[0, c, p]], s, qp)
                assert [int(v) for v in rot[0, c, p]] == want


@pytest.mark.parametrize("primes,log2_t,beta,ell,same_key", [
    (P2, 26, 54, 1, False), (P2, 28, 54, 1, True), (P1, 24, 12, 3, False)])
def test_pack_of_real_products_decrypts(primes, log2_t, beta, ell, same_key):
    """Packed outputs of real products decrypt under S_dst to W x in their slots, zero in
    the empty slots; with two primes inside a deterministic noise bound, and after the
    switch of the packed ciphertexts to 2^32."""
    N, d_in, d_out, T = 256, 300, 200, 3
    case = make_case(N, primes, log2_t, d_out, d_in, T, salt=21)
    lwe = orc.matmul_clear(N, primes, case.W, case.ct)  # (T, d_out, P, N+1)
    S_src = case.S
    _, S_dst, A, E = ksk_inputs(N, primes, beta, ell, 5)
    if same_key:
        S_dst = S_src
    ksk = orc.ksk_gen(N, primes, beta, ell, S_src, S_dst, A, E)
    q, delta = case.q, case.delta
    y = case.x.astype(np.int64) @ case.W.astype(np.int64).T  # (T, d_out)
    M = T * d_out
    for n_pack in (N, d_out):
        out = orc.keyswitch_pack(N, primes, beta, ell, lwe.reshape(M, len(primes), N + 1), ksk,
                                 n_pack)
        ph = orc.rlwe_decrypt_slots(N, primes, S_dst, out)
        worst = 0
        for g in range(out.shape[0]):
            for s in range(N):
                m = g * n_pack + s
                want = int(y.reshape(-1)[m]) if s < n_pack and m < M else 0
                assert orc.decode(ph[g][s], delta) == want
                worst = max(worst, abs(ph[g][s] - delta * want))
        if len(primes) == 2:
            # product noise + KeySwitch noise (digit times key error) + Decomp rounding
            K = beta * ell
            bound = 19 * 127 * d_in + N * ell * n_pack * (1 << (beta - 1)) * 19 \
                + N * (q // (1 << (K + 1)) + ell * (1 << (beta - 1)))
            assert 2 * bound < delta
            assert worst <= bound
        if log2_t > 26:
            continue  # post-switch rounding noise is comparable to Delta' / 2 = 8
        sw = orc.rlwe_modswitch_bits(primes, out, 32)
        ph32 = orc.rlwe_phase_bits(S_dst, sw, 32)
        d32 = (1 << 32) >> log2_t
        for g in range(out.shape[0]):
            for s in range(N):
                m = g * n_pack + s
                want = int(y.reshape(-1)[m]) if s < n_pack and m < M else 0
                assert orc.decode(int(ph32[g, s]), d32) == want
