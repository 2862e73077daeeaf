"""Pins of the oracle's seeded masks (Sec. 3.1: the client sends a seed in place of the
uniform mask; Sec. 4.4: a seed and the body make up the input ciphertext).

Anchors: SplitMix64's published outputs for seeds 0 and 1234567; validity and
uniformity of the rejection-sampled residues (chi-square), also for a modulus where
half the draws are rejected; distinct masks for distinct seeds; the input size the
paper derives (8 + 2048 * 39 / 8 = 9992 bytes); and decryption of ciphertexts
rebuilt from the seeded layout.
"""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2505_07329_amd import synth

P2048 = synth.PRIMES_2048
P4096 = synth.PRIMES_4096


def test_splitmix64_published_outputs():
    assert [orc.splitmix64_at(0, c) for c in range(3)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert [orc.splitmix64_at(1234567, c) for c in range(2)] == [
        6457827717110365317, 3203168211198807973]


def chi2_uniform(values, modulus, buckets=64):
    counts = np.bincount((values.astype(object) * buckets // modulus).astype(np.int64), minlength=buckets)
    expect = len(values) / buckets
    return float(((counts - expect) ** 2 / expect).sum())


@pytest.mark.parametrize("primes", [P2048, P4096])
def test_expanded_masks_valid_and_uniform(primes):
    N = 2048 if len(primes) == 1 else 4096
    A = orc.expand_masks(np.arange(1, 9, dtype=np.uint64) * 0x1234567, N, primes)
    for p, q in enumerate(primes):
        v = A[:, p].reshape(-1)
        assert int(v.max()) < q
        # 63 degrees of freedom: mean 63, sd ~11; 130 is far in the tail
        assert chi2_uniform(v, q) < 130


def test_rejection_sampling_at_half_acceptance():
    q = (1 << 53) + 1  # about half of the 54-bit draws are rejected
    vals = np.array([orc.mask_coeff(99, 4096, 0, n, q) for n in range(20000)], dtype=np.uint64)
    assert int(vals.max()) < q
    assert chi2_uniform(vals, q) < 130
    plain = np.array([(orc.splitmix64_at(99, n << 4) >> 10) % q for n in range(20000)], dtype=np.uint64)
    assert np.count_nonzero(vals != plain) > 5000  # the second and later draws are in use


def test_masks_distinct_per_seed_and_deterministic():
    A1 = orc.expand_masks(np.array([5], dtype=np.uint64), 4096, P4096)
    A2 = orc.expand_masks(np.array([6], dtype=np.uint64), 4096, P4096)
    assert np.array_equal(A1, orc.expand_masks(np.array([5], dtype=np.uint64), 4096, P4096))
    assert np.count_nonzero(A1 != A2) > 8000
    assert len(set(A1.reshape(-1).tolist())) == A1.size  # no repeats among 8192 residues


def test_paper_input_size():
    """Sec. 4.4: the seed (8 bytes) and the body of N = 2048 coefficients at 39 bits."""
    assert 8 + 4 * orc.packed_words(2048, 39) == 9992


def test_seeded_layout_round_trip_decrypts():
    from tests.cases import make_case
    N, primes, T = 4096, P4096, 3
    seeds = np.array([[11], [12], [13]], dtype=np.uint64)  # (T, L)
    A = orc.expand_masks(seeds, N, primes)
    g = np.random.default_rng(4)
    x = synth.int8_uniform(g, (T, 1000))
    S = synth.ternary(g, N)
    E = synth.rounded_gaussian(g, (T, 1, N))
    ct = orc.encrypt_tokens(N, primes, 26, S, x, A, E)
    sl = orc.seeded_layout(ct, seeds)
    assert sl.shape == (T, 1, 2 * N + 2)
    assert 2 * sl.nbytes == ct.nbytes + 32 * T  # half the bytes, plus a 16-byte header per block
    rebuilt = np.stack([orc.expand_masks(sl[:, :, 0], N, primes),
                        sl[:, :, 2:].reshape(T, 1, len(primes), N)], axis=2)
    assert np.array_equal(rebuilt, ct)
    ph = orc.rlwe_phase(N, primes, S, rebuilt[:, :, 0], rebuilt[:, :, 1])
    q = orc.modulus(primes)
    delta = q >> 26
    for t in range(T):
        vals = [orc.decode(orc.centered(orc.crt(primes, ph[t, 0, :, n]), q), delta) for n in range(1000)]
        assert vals == x[t].tolist()
