"""Pins of the oracle's switch to q_out = 2^k and of its bit-packing of switched outputs.

The switch (Sec. 3.2, ModulusSwitch) to 2^k is the oracle's binary long division;
it is pinned to Python big-integer rounding of the rational c 2^k / q and, at
k = 32, to the oracle's separate two-step division. The packing (Sec. 4.5: the
switched output is packed into a bit-vector) is pinned by a round trip, by
hand-computed words, and by the ciphertext sizes the paper derives for its
parameters (Sec. 4.4: N = 2048, 26-bit output modulus, 6656 bytes per component
and 13312 bytes per RLWE ciphertext).
"""

import numpy as np
import pytest

from oracle import oracle as orc
from oracle import tiny
from paper_2505_07329_amd import synth

P2048 = synth.PRIMES_2048
P4096 = synth.PRIMES_4096


def residues_of(cs, primes):
    return np.array([[c % p for p in primes] for c in cs], dtype=np.uint64)


@pytest.mark.parametrize("primes", [P2048, P4096])
@pytest.mark.parametrize("bits", [1, 8, 16, 26, 31, 32])
def test_switch_bits_matches_bigint_rounding(primes, bits):
    q = orc.modulus(primes)
    g = np.random.default_rng(bits * 7 + len(primes))
    cs = [int(g.integers(0, 2**62)) * int(g.integers(0, 2**62)) % q for _ in range(1500)]
    # points at and next to rounding ties of c 2^k / q: c = ceil((m + 1/2) q / 2^k) + d
    for m in (0, 1, 12345, (1 << bits) - 1):
        base = -(-((2 * m + 1) * q) // (2 << bits))
        cs += [(base + d) % q for d in (-1, 0, 1)]
    cs += [0, 1, q - 1, q // 2, q // 2 + 1]
    raw = residues_of(cs, primes)[:, :, None]
    got = orc.modswitch_bits(primes, raw, bits)[:, 0]
    assert [int(v) for v in got] == [tiny.modswitch(c, q, bits) for c in cs]


@pytest.mark.parametrize("primes", [P2048, P4096])
def test_switch_bits_32_equals_two_step_division(primes):
    g = np.random.default_rng(11)
    raw = np.stack([g.integers(0, p, size=(300, 9), dtype=np.uint64) for p in primes], axis=1)
    assert np.array_equal(orc.modswitch_bits(primes, raw, 32), orc.modswitch(primes, raw))


def test_switch_bits_values_fit():
    g = np.random.default_rng(3)
    raw = np.stack([g.integers(0, p, size=(200, 33), dtype=np.uint64) for p in P4096], axis=1)
    for bits in (5, 26):
        assert int(orc.modswitch_bits(P4096, raw, bits).max()) < (1 << bits)


@pytest.mark.parametrize("bits", [1, 7, 13, 26, 31, 32])
@pytest.mark.parametrize("length", [1, 5, 97])
def test_pack_round_trip(bits, length):
    g = np.random.default_rng(bits * 100 + length)
    v = g.integers(0, 1 << bits, size=(3, length), dtype=np.uint64).astype(np.uint32)
    w = orc.pack_bits(v, bits)
    assert w.shape == (3, (length * bits + 31) // 32)
    assert np.array_equal(orc.unpack_bits(w, bits, length), v)
    spare = 32 * w.shape[1] - length * bits  # unused high bits of the last word are zero
    if spare:
        assert int(w[:, -1].max()) >> (32 - spare) == 0


def test_pack_hand_computed_words():
    # 4-bit values 1..8 fill one word, least significant first
    assert orc.pack_bits(np.arange(1, 9, dtype=np.uint32), 4).tolist() == [0x87654321]
    # 26 ones then a one at stream bit 26; the second word is empty
    assert orc.pack_bits(np.array([(1 << 26) - 1, 1], dtype=np.uint32), 26).tolist() == [0x07FFFFFF, 0]
    # a 26-bit value straddling the word boundary: value 1 starts at stream bit 26
    w = orc.pack_bits(np.array([0, 0x2AAAAAA], dtype=np.uint32), 26)
    assert w.tolist() == [(0x2AAAAAA << 26) & 0xFFFFFFFF, 0x2AAAAAA >> 6]
    with pytest.raises(ValueError):
        orc.pack_bits(np.array([1 << 26], dtype=np.uint32), 26)


def test_paper_output_sizes():
    """Sec. 4.4 sizes at N = 2048 and a 26-bit output modulus: 6656 bytes per component
    (N coefficients) and 13312 bytes for the RLWE ciphertext (A', B')."""
    assert 4 * orc.packed_words(2048, 26) == 6656
    assert 4 * orc.packed_words(2 * 2048, 26) == 13312
    # and one LWE output of this build (N = 4096 mask coefficients and the body)
    assert 4 * orc.packed_words(4097, 26) == 13316


def test_switched_decryption_after_packing():
    """Real encryptions at N = 2048 (t = 2^12, so values in [-2, 2] keep |W x| < t/2):
    switched to 2^26, packed, unpacked, decrypted with Delta' = 2^26 / t = 2^14, far
    above the switch noise: every output equals W x."""
    from tests.cases import make_case
    g = np.random.default_rng(70)
    W = g.integers(-2, 3, size=(24, 64)).astype(np.int8)
    x = g.integers(-2, 3, size=(3, 64)).astype(np.int8)
    case = make_case(2048, P2048, 12, 24, 64, 3, config=70, W=W, x=x)
    raw = orc.matmul_clear(2048, P2048, case.W, case.ct)
    sw = orc.modswitch_bits(P2048, raw, 26)
    back = orc.unpack_bits(orc.pack_bits(sw, 26), 26, 2049)
    assert np.array_equal(back, sw)
    ph = orc.lwe_phase_bits(2048, case.S, back, 26)
    dprime = 1 << (26 - 12)
    dec = np.floor_divide(2 * ph + dprime, 2 * dprime)
    assert np.array_equal(dec, case.x.astype(np.int64) @ case.W.T.astype(np.int64))
