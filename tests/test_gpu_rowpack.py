"""Multi-row packing (the coefficient packing of Sec. 4.3.1, as in Cheetah) on the GPU,
against the oracle.

With RLWE_W_ROWPACK and a contraction length K <= N/2, n_o = floor(N / K) rows share one
weight polynomial and row g n_o + rho is SampleExtract at h = (rho + 1) K - 1. Every
expected value comes from the oracle's ``matmul_rowpacked`` (its negacyclic NTT on the
packed weight polynomials) and its switch on the same seeded inputs. Covered: n_o = 2,
4, 8 and 1365, ragged last groups, K not a multiple of 4 (the body's byte path), one and
two primes, raw and switched outputs (2^32 and 2^26), the transposed orientation, seeded
inputs, a batch mixing packed and unpacked products captured as a graph, K > N/2 (no
packing: the standard product), flag validation, and end-to-end decryption.
"""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2505_07329_amd import synth
from tests.cases import make_case, uniform_ct

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 4096
P4096 = synth.PRIMES_4096


def rl():
    from paper_2505_07329_amd import rlwe
    return rlwe


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a.view(np.int64) if a.dtype == np.uint64 else a)).cuda()


@pytest.mark.parametrize("primes,d_out,K,T", [
    (P4096, 5, 2048, 2),        # n_o = 2, last group holds one row
    (P4096, 20, 512, 3),        # n_o = 8, last group holds four
    (P4096, 9, 1000, 2),        # n_o = 4, 96 coefficients unused
    (P4096, 7, 1001, 2),        # n_o = 4, K not a multiple of 4
    (P4096, 1400, 3, 1),        # n_o = 1365, second group of 35 rows
    (P4096[:1], 33, 640, 3),    # one prime, n_o = 6
])
def test_rowpacked_product_matches_oracle(primes, d_out, K, T):
    print(f"case: rowpack P={len(primes)} {d_out}x{K} T={T}", flush=True)
    r = rl()
    W = synth.int8_uniform(np.random.default_rng(K + d_out), (d_out, K))
    ct = uniform_ct(N, primes, T, 1, config=81, salt=K)
    raw_want = orc.matmul_rowpacked(N, primes, W, ct)
    ctx = r.Context(N, primes, 28)
    w = r.Weights(ctx, dev(W), r.RLWE_W_FWD | r.RLWE_W_ROWPACK)
    assert r.rlwe_weights_rows_per_product(w.handle) == orc.rows_per_product(K, N)
    assert r.rlwe_weights_method(w.handle) == r.RLWE_METHOD_NTT
    x = dev(ct)
    raw = r.matmul(ctx, w, x, raw=True)
    sw = r.matmul(ctx, w, x)
    torch.cuda.synchronize()
    assert np.array_equal(raw.cpu().numpy().view(np.uint64), raw_want)
    assert np.array_equal(sw.cpu().numpy().view(np.uint32), orc.modswitch(primes, raw_want))
    w.close()
    ctx.close()


def test_rowpacked_switch_to_26_bits_and_forced_exact_route():
    r = rl()
    W = synth.int8_uniform(np.random.default_rng(3), (24, 700))
    ct = uniform_ct(N, P4096, 2, 1, config=82)
    raw_want = orc.matmul_rowpacked(N, P4096, W, ct)
    ctx = r.Context(N, P4096, 28, log2_q_out=26)
    w = r.Weights(ctx, dev(W), r.RLWE_W_FWD | r.RLWE_W_ROWPACK)
    x = dev(ct)
    got = r.matmul(ctx, w, x)
    exact = r.matmul(ctx, w, x, force_exact=True)
    torch.cuda.synchronize()
    want = orc.modswitch_bits(P4096, raw_want, 26)
    assert np.array_equal(got.cpu().numpy().view(np.uint32), want)
    assert np.array_equal(exact.cpu().numpy().view(np.uint32), want)
    w.close()
    ctx.close()


def test_rowpacked_transposed_orientation():
    """Forward K = 4096 (no packing) and transposed K = 600 (n_o = 6) from one load."""
    r = rl()
    g = np.random.default_rng(6)
    W = synth.int8_uniform(g, (600, 4096))
    ct_f = uniform_ct(N, P4096, 2, 1, config=83, salt=1)
    ct_b = uniform_ct(N, P4096, 2, 1, config=83, salt=2)
    ctx = r.Context(N, P4096, 28)
    w = r.Weights(ctx, dev(W), r.RLWE_W_FWD | r.RLWE_W_TRANSPOSE | r.RLWE_W_ROWPACK)
    assert r.rlwe_weights_rows_per_product(w.handle, False) == 1
    assert r.rlwe_weights_rows_per_product(w.handle, True) == 6
    fwd = r.matmul(ctx, w, dev(ct_f), raw=True)
    bwd = r.matmul(ctx, w, dev(ct_b), transpose=True, raw=True)
    torch.cuda.synchronize()
    assert np.array_equal(fwd.cpu().numpy().view(np.uint64), orc.matmul_clear(N, P4096, W, ct_f))
    assert np.array_equal(bwd.cpu().numpy().view(np.uint64),
                          orc.matmul_rowpacked(N, P4096, np.ascontiguousarray(W.T), ct_b))
    w.close()
    ctx.close()


def test_rowpack_flag_above_half_ring_is_the_standard_product():
    r = rl()
    W = synth.int8_uniform(np.random.default_rng(7), (10, 2500))
    ct = uniform_ct(N, P4096, 2, 1, config=84)
    ctx = r.Context(N, P4096, 28)
    w = r.Weights(ctx, dev(W), r.RLWE_W_FWD | r.RLWE_W_ROWPACK)
    assert r.rlwe_weights_rows_per_product(w.handle) == 1
    got = r.matmul(ctx, w, dev(ct), raw=True)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().view(np.uint64), orc.matmul_clear(N, P4096, W, ct))
    w.close()
    ctx.close()


def test_rowpack_flag_validation():
    r = rl()
    W = dev(synth.int8_uniform(np.random.default_rng(8), (4, 64)))
    ctx = r.Context(N, P4096, 28)
    with pytest.raises(r.RlweError) as e:
        r.Weights(ctx, W, r.RLWE_W_FWD | r.RLWE_W_ROWPACK | r.RLWE_W_TOEPLITZ)
    assert e.value.code == r.RLWE_EINVAL
    ctx.close()
    ctx2 = r.Context(1024, synth.PRIMES_2048, 24)  # packed rows need the NTT method: N = 2048, 4096
    with pytest.raises(r.RlweError) as e:
        r.Weights(ctx2, W, r.RLWE_W_FWD | r.RLWE_W_ROWPACK)
    assert e.value.code == r.RLWE_EPARAM
    ctx2.close()


def test_rowpacked_seeded_inputs():
    r = rl()
    T, K, d_out = 3, 1024, 10
    g = np.random.default_rng(9)
    seeds = g.integers(0, 2**63, size=(T, 1), dtype=np.uint64)
    A = orc.expand_masks(seeds, N, P4096)
    B = synth.uniform_mod_primes(g, P4096, (T, 1), N)
    ct = np.stack([A, B], axis=2)
    W = synth.int8_uniform(g, (d_out, K))
    ctx = r.Context(N, P4096, 28)
    w = r.Weights(ctx, dev(W), r.RLWE_W_FWD | r.RLWE_W_ROWPACK)
    got = r.matmul(ctx, w, dev(orc.seeded_layout(ct, seeds)), seeded=True)
    torch.cuda.synchronize()
    want = orc.modswitch(P4096, orc.matmul_rowpacked(N, P4096, W, ct))
    assert np.array_equal(got.cpu().numpy().view(np.uint32), want)
    w.close()
    ctx.close()


def test_rowpacked_in_batch_graph_replays():
    """A packed product (n_o = 4), an unpacked NTT product and a matrix-core product in
    one captured batch, replayed three times with eager work between."""
    r = rl()
    ctx = r.Context(N, P4096, 28)
    g = np.random.default_rng(10)
    W1 = synth.int8_uniform(g, (30, 1024))
    W2 = synth.int8_uniform(g, (16, 6000))
    W3 = synth.int8_uniform(g, (32, 700))
    w1 = r.Weights(ctx, dev(W1), r.RLWE_W_FWD | r.RLWE_W_ROWPACK)
    w2 = r.Weights(ctx, dev(W2), r.RLWE_W_FWD | r.RLWE_W_NTT)
    w3 = r.Weights(ctx, dev(W3), r.RLWE_W_FWD | r.RLWE_W_TOEPLITZ)
    items, wants = [], []
    for s, (w, W, T, packed) in enumerate(((w1, W1, 3, True), (w2, W2, 2, False), (w3, W3, 2, False))):
        L = (W.shape[1] + N - 1) // N
        ct = uniform_ct(N, P4096, T, L, config=85, salt=s)
        raw = orc.matmul_rowpacked(N, P4096, W, ct) if packed else orc.matmul_clear(N, P4096, W, ct)
        wants.append(orc.modswitch(P4096, raw))
        out = torch.empty((T, W.shape[0], N + 1), dtype=torch.int32, device="cuda")
        items.append((w.handle, False, dev(ct), T, out))
    r.ct_matmul_batch(ctx.handle, items)
    torch.cuda.synchronize()
    for it, want in zip(items, wants):
        assert np.array_equal(it[4].cpu().numpy().view(np.uint32), want)
    graph = r.rlwe_graph_capture_batch(ctx.handle, items)
    for rep in range(3):
        for it in items:
            it[4].fill_(-1)
        torch.cuda.synchronize()
        r.rlwe_graph_launch(graph)
        torch.cuda.synchronize()
        for it, want in zip(items, wants):
            assert np.array_equal(it[4].cpu().numpy().view(np.uint32), want), f"replay {rep}"
    r.rlwe_graph_destroy(graph)
    for w in (w1, w2, w3):
        w.close()
    ctx.close()


def test_rowpacked_end_to_end_decrypts():
    """Encrypt x (t = 2^12), packed product on the GPU (n_o = 8), switch to 2^32: every
    output decrypts to W x, and the raw outputs carry the exact phase of the oracle's."""
    r = rl()
    T, K, d_out = 2, 512, 20
    g = np.random.default_rng(11)
    W = np.zeros((d_out, K), dtype=np.int8)
    for j in range(d_out):
        W[j, g.choice(K, size=12, replace=False)] = g.choice([-1, 1], size=12)
    x = g.integers(-2, 3, size=(T, K)).astype(np.int8)
    case = make_case(N, P4096, 12, d_out, K, T, config=86, W=W, x=x)
    ctx = r.Context(N, P4096, 12)
    w = r.Weights(ctx, dev(W), r.RLWE_W_FWD | r.RLWE_W_ROWPACK)
    xin = dev(case.ct)
    raw = r.matmul(ctx, w, xin, raw=True).cpu().numpy().view(np.uint64)
    sw = r.matmul(ctx, w, xin).cpu().numpy().view(np.uint32)
    torch.cuda.synchronize()
    want_raw = orc.matmul_rowpacked(N, P4096, W, case.ct)
    assert np.array_equal(raw, want_raw)
    Wx = x.astype(np.int64) @ W.T.astype(np.int64)
    ph = orc.lwe_phase(N, P4096, case.S, raw)
    assert [orc.decode(v, case.delta) for v in ph] == Wx.reshape(-1).tolist()
    ph32 = orc.lwe_phase_u32(N, case.S, sw)
    dprime = 1 << (32 - 12)
    assert np.array_equal(np.floor_divide(2 * ph32 + dprime, 2 * dprime), Wx)
    w.close()
    ctx.close()
