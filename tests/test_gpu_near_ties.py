"""Coefficients next to ModulusSwitch rounding ties (Sec. 3.2), on the GPU.

With a weight row w_j = +-e_s the product of Eq. (LWEdot) copies the ciphertext:
a'_n = w_j[s] A[s - n] for n <= s, -w_j[s] A[N + s - n] otherwise, and b' = w_j[s] B[s].
So a mask A and body B whose coefficients c sit a few units of 2^-32 (of c 2^32 / q)
from a tie of round(c 2^k / q) make every output coefficient such a value (q - c is as
close to a tie as c, q being odd). Every kernel epilogue must still give the exact
rounding: the fast fixed-point route where it can decide, the exact route inside its
near-tie window, and the exact route for every coefficient when RLWE_OUT_FORCE_EXACT
is set. Both mask methods, switched to 2^32 and to 2^26, against the oracle.
"""

import random

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2505_07329_amd import synth
from tests.test_epilogue_model import epilogue_constants, estimate, near_tie_values, round_qout

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P4096 = synth.PRIMES_4096
N = 4096


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a.view(np.int64) if a.dtype == np.uint64 else a)).cuda()


def crafted(primes, k, T, M, K, seed):
    """Weights +-e_s per row and ciphertexts whose coefficients lie within 8 units of a
    tie of the rounding to 2^k."""
    rng = random.Random(seed)
    q = orc.modulus(primes)
    W = np.zeros((M, K), dtype=np.int8)
    for j in range(M):
        W[j, (j * 613 + 5) % K] = 1 if j % 3 else -1
    ct = np.empty((T, 1, 2, len(primes), N), dtype=np.uint64)
    vals = []
    for t in range(T):
        for part in range(2):
            cs = near_tie_values(q, k, rng, N)
            vals += cs
            for p, qp in enumerate(primes):
                ct[t, 0, part, p] = np.array([c % qp for c in cs], dtype=np.uint64)
    return W, ct, vals


@pytest.mark.parametrize("k", [32, 26])
def test_near_tie_coefficients_all_routes(k):
    print(f"case: near ties, q_out = 2^{k}", flush=True)
    from paper_2505_07329_amd import rlwe as r
    T, M, K = 2, 12, 2048
    W, ct, vals = crafted(P4096, k, T, M, K, seed=100 + k)
    # the draws do land in the fast route's window (CPU model of the epilogue)
    hs = epilogue_constants(P4096)
    in_window = sum(1 for c in vals[:4096]
                    if -8 <= round_qout(estimate([c % p for p in P4096], hs), k)[1] < 0)
    assert in_window > 100
    want = orc.modswitch_bits(P4096, orc.matmul_clear(N, P4096, W, ct), k)
    ctx = r.Context(N, P4096, 26, log2_q_out=k)
    ct_d = dev(ct)
    for method in (r.RLWE_W_NTT, r.RLWE_W_TOEPLITZ):
        w = r.Weights(ctx, dev(W), r.RLWE_W_FWD | method)
        fast = r.matmul(ctx, w, ct_d)
        forced = r.matmul(ctx, w, ct_d, force_exact=True)
        raw = r.matmul(ctx, w, ct_d, raw=True)
        sw = r.modswitch(ctx, raw)
        torch.cuda.synchronize()
        name = "ntt" if method == r.RLWE_W_NTT else "toeplitz"
        for label, got in (("fast", fast), ("forced", forced), ("ct_modswitch", sw)):
            got = got.cpu().numpy().view(np.uint32)
            bad = int((got != want).sum())
            assert bad == 0, f"{name} {label}: {bad} coefficients differ from the oracle"
        w.close()
    ctx.close()
