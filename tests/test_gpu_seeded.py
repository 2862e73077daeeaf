"""Seeded inputs (Sec. 3.1 / 4.4: a seed in place of the uniform mask), expanded on the
GPU, against the oracle's expansion and product.

The oracle expands every seed to its mask (SplitMix64, rejection sampling), encrypts
or takes uniform bodies, and computes the product from the full ciphertexts; the
GPU receives only [seed, 0, B] per block. Covered: both mask methods, one and two
primes, one and two input blocks, raw and switched outputs, a batch captured as a
graph, and end-to-end decryption.
"""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2505_07329_amd import synth
from tests.cases import make_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P4096 = synth.PRIMES_4096
P2048 = synth.PRIMES_2048


def rl():
    from paper_2505_07329_amd import rlwe
    return rlwe


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a.view(np.int64) if a.dtype == np.uint64 else a)).cuda()


def seeded_inputs(N, primes, T, L, salt):
    """Seeds, the oracle's full ciphertexts (expanded masks, uniform bodies), seeded layout."""
    g = np.random.default_rng(900 + salt)
    seeds = g.integers(0, 2**63, size=(T, L), dtype=np.uint64)
    A = orc.expand_masks(seeds, N, primes)
    B = synth.uniform_mod_primes(g, primes, (T, L), N)
    ct = np.stack([A, B], axis=2)
    return seeds, ct, orc.seeded_layout(ct, seeds)


@pytest.mark.parametrize("N,primes,method,d_out,d_in,T", [
    (4096, P4096, "ntt", 40, 2048, 2),
    (4096, P4096, "ntt", 24, 5000, 2),
    (4096, P4096, "toeplitz", 40, 3000, 2),
    (4096, P4096[:1], "ntt", 16, 1000, 3),
    (2048, P2048, "toeplitz", 32, 300, 3),
])
def test_seeded_product_matches_oracle(N, primes, method, d_out, d_in, T):
    print(f"case: seeded {method} N={N} P={len(primes)} {d_out}x{d_in} T={T}", flush=True)
    r = rl()
    L = (d_in + N - 1) // N
    _, ct, sl = seeded_inputs(N, primes, T, L, d_in)
    W = synth.int8_uniform(np.random.default_rng(d_out), (d_out, d_in))
    raw_want = orc.matmul_clear(N, primes, W, ct)
    ctx = r.Context(N, primes, 28 if N == 4096 else 24)
    flag = r.RLWE_W_NTT if method == "ntt" else r.RLWE_W_TOEPLITZ
    w = r.Weights(ctx, dev(W), r.RLWE_W_FWD | flag)
    x = dev(sl)
    raw = r.matmul(ctx, w, x, raw=True, seeded=True)
    sw = r.matmul(ctx, w, x, seeded=True)
    torch.cuda.synchronize()
    assert np.array_equal(raw.cpu().numpy().view(np.uint64), raw_want)
    assert np.array_equal(sw.cpu().numpy().view(np.uint32), orc.modswitch(primes, raw_want))
    w.close()
    ctx.close()


def test_seeded_batch_graph_replays():
    r = rl()
    N = 4096
    ctx = r.Context(N, P4096, 28)
    g = np.random.default_rng(8)
    W1 = synth.int8_uniform(g, (24, 6000))  # NTT, two blocks
    W2 = synth.int8_uniform(g, (32, 700))   # matrix cores
    w1 = r.Weights(ctx, dev(W1))
    w2 = r.Weights(ctx, dev(W2))
    items, wants = [], []
    for s, (w, W, T) in enumerate(((w1, W1, 2), (w2, W2, 3))):
        L = (W.shape[1] + N - 1) // N
        _, ct, sl = seeded_inputs(N, P4096, T, L, 50 + s)
        wants.append(orc.modswitch(P4096, orc.matmul_clear(N, P4096, W, ct)))
        out = torch.empty((T, W.shape[0], N + 1), dtype=torch.int32, device="cuda")
        items.append((w.handle, False, dev(sl), T, out))
    graph = r.rlwe_graph_capture_batch(ctx.handle, items, flags=r.RLWE_IN_SEEDED)
    for rep in range(3):
        for it in items:
            it[4].fill_(-1)
        torch.cuda.synchronize()
        r.rlwe_graph_launch(graph)
        torch.cuda.synchronize()
        for it, want in zip(items, wants):
            assert np.array_equal(it[4].cpu().numpy().view(np.uint32), want), f"replay {rep}"
    r.rlwe_graph_destroy(graph)
    w1.close()
    w2.close()
    ctx.close()


def test_seeded_end_to_end_decrypts():
    """Client: seeds, masks expanded by the oracle, encryption of x; server (GPU): the
    seeded layout only; client: switched outputs decrypt to W x (t = 2^24, Delta' = 2^8)."""
    r = rl()
    N, T, d_in, d_out = 2048, 3, 256, 40
    g = np.random.default_rng(12)
    seeds = g.integers(0, 2**63, size=(T, 1), dtype=np.uint64)
    A = orc.expand_masks(seeds, N, P2048)
    case = make_case(N, P2048, 24, d_out, d_in, T, config=72)
    E = synth.rounded_gaussian(g, (T, 1, N))
    ct = orc.encrypt_tokens(N, P2048, 24, case.S, case.x, A, E)
    ctx = r.Context(N, P2048, 24)
    w = r.Weights(ctx, dev(case.W))
    out = r.matmul(ctx, w, dev(orc.seeded_layout(ct, seeds)), seeded=True)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, orc.modswitch(P2048, orc.matmul_clear(N, P2048, case.W, ct)))
    ph = orc.lwe_phase_u32(N, case.S, got)
    dprime = 1 << (32 - 24)
    dec = np.floor_divide(2 * ph + dprime, 2 * dprime)
    assert np.array_equal(dec, case.x.astype(np.int64) @ case.W.T.astype(np.int64))
    w.close()
    ctx.close()
