"""The NTT method of the mask product (N = 4096) on the GPU.

Both methods compute the same integers, so the NTT outputs must equal the
matrix-core outputs bit for bit (switched and raw), and sampled outputs must
equal the oracle's. Covered: one and two input blocks, a ragged last block,
forward and transposed weights, one and two primes, the default method choice,
mixed-method batches and graph replays.
"""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2505_07329_amd import synth
from tests.cases import make_case, uniform_ct

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P4096 = synth.PRIMES_4096
N = 4096


def rl():
    from paper_2505_07329_amd import rlwe
    return rlwe


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a.view(np.int64) if a.dtype == np.uint64 else a)).cuda()


def host_u32(t):
    return t.cpu().numpy().view(np.uint32)


def both_methods(ctx, W, flags_orient):
    r = rl()
    wn = r.Weights(ctx, dev(W), flags_orient | r.RLWE_W_NTT)
    wt = r.Weights(ctx, dev(W), flags_orient | r.RLWE_W_TOEPLITZ)
    return wn, wt


@pytest.mark.parametrize("primes,d_out,d_in,T,log_t", [
    (P4096, 64, 300, 3, 28),       # one block, ragged
    (P4096, 40, 5000, 2, 28),      # two blocks, ragged second block
    (P4096, 33, 8192, 2, 28),      # two full blocks
    (P4096[:1], 48, 4500, 2, 28),  # one prime
    (P4096[:1], 20, 12300, 2, 30),  # four blocks (one prime: two cap K near 8256 for exact
                                    # 128-bit sums): the pointwise sums are reduced per block
])
def test_ntt_equals_matrix_cores(primes, d_out, d_in, T, log_t):
    print(f"case: ntt vs toeplitz {len(primes)} primes {d_out}x{d_in} T={T}", flush=True)
    r = rl()
    # t = 2^28 keeps 127 * (row 1-norm) < t/2 up to K = 8192, 2^30 up to K = 33000
    ctx = r.Context(N, primes, log_t)
    g = np.random.default_rng(d_out * 7 + d_in)
    W = synth.int8_uniform(g, (d_out, d_in))
    wn, wt = both_methods(ctx, W, r.RLWE_W_FWD | r.RLWE_W_TRANSPOSE)
    assert r.rlwe_weights_method(wn.handle) == r.RLWE_METHOD_NTT
    assert r.rlwe_weights_method(wt.handle, True) == r.RLWE_METHOD_TOEPLITZ
    for tr in (False, True):
        K = d_out if tr else d_in
        L = (K + N - 1) // N
        ct = dev(uniform_ct(N, primes, T, L, config=60, salt=d_in + tr))
        for raw in (False, True):
            a = r.matmul(ctx, wn, ct, transpose=tr, raw=raw)
            b = r.matmul(ctx, wt, ct, transpose=tr, raw=raw)
            torch.cuda.synchronize()
            assert torch.equal(a, b), f"transpose={tr} raw={raw}"
    wn.close()
    wt.close()
    ctx.close()


def test_ntt_down_projection_against_oracle():
    """W 2048 x 8192 (the down projection, two blocks), t = 2^28, 4 tokens of real
    encryptions: sampled outputs equal the oracle's, raw outputs decrypt exactly."""
    print("case: ntt down 2048x8192 T=4 vs oracle", flush=True)
    r = rl()
    case = make_case(N, P4096, 28, 2048, 8192, 4, config=61)
    ctx = r.Context(N, P4096, 28)
    w = r.Weights(ctx, dev(case.W))  # default method: two blocks -> NTT
    assert r.rlwe_weights_method(w.handle) == r.RLWE_METHOD_NTT
    ct = dev(case.ct)
    out = r.matmul(ctx, w, ct)
    raw = r.matmul(ctx, w, ct, raw=True)
    torch.cuda.synchronize()
    pairs = np.array([(0, 0), (3, 2047), (1, 1000), (2, 17)], dtype=np.uint32)
    ref_raw = orc.matmul_clear(N, P4096, case.W, case.ct, pairs=pairs)
    ref = orc.modswitch(P4096, ref_raw)
    got = host_u32(out)
    got_raw = raw.cpu().numpy().view(np.uint64)
    for e, (t, j) in enumerate(pairs):
        assert np.array_equal(got[t, j], ref[e])
        assert np.array_equal(got_raw[t, j], ref_raw[e])
    ph = orc.lwe_phase(N, P4096, case.S, got_raw[pairs[:, 0], pairs[:, 1]])
    v = case.x.astype(object) @ case.W.T.astype(object)
    for (t, j), p in zip(pairs, ph):
        assert orc.decode(p, case.delta) == v[t, j]
    w.close()
    ctx.close()


def test_default_method_and_errors():
    r = rl()
    ctx = r.Context(N, P4096, 28)
    g = np.random.default_rng(3)
    # without a tuner the cost model decides; both methods give the same bits, so the
    # clear-cut cases are what matters: long contractions on the transforms, short ones
    # on the matrix cores
    W = synth.int8_uniform(g, (128, 2048))
    w = r.Weights(ctx, dev(W), r.RLWE_W_FWD | r.RLWE_W_TRANSPOSE)
    assert r.rlwe_weights_method(w.handle) == r.RLWE_METHOD_NTT  # K = 2048: transforms win
    assert r.rlwe_weights_method(w.handle, True) == r.RLWE_METHOD_TOEPLITZ  # K = 128
    w.close()
    W2 = synth.int8_uniform(g, (16, 4097))
    w2 = r.Weights(ctx, dev(W2))
    assert r.rlwe_weights_method(w2.handle) == r.RLWE_METHOD_NTT  # two blocks
    w2.close()
    with pytest.raises(r.RlweError):
        r.Weights(ctx, dev(W2), r.RLWE_W_FWD | r.RLWE_W_NTT | r.RLWE_W_TOEPLITZ)
    ctx.close()
    ctx2 = r.Context(1024, synth.PRIMES_2048, 28)
    with pytest.raises(r.RlweError) as ei:
        r.Weights(ctx2, dev(W2[:, :512]), r.RLWE_W_FWD | r.RLWE_W_NTT)
    assert ei.value.code == r.RLWE_EPARAM
    w3 = r.Weights(ctx2, dev(synth.int8_uniform(g, (8, 5000))))
    assert r.rlwe_weights_method(w3.handle) == r.RLWE_METHOD_TOEPLITZ  # NTT needs N = 2048, 4096
    w3.close()
    ctx2.close()


def test_mixed_batch_and_graph():
    """One batch with both methods: equals separate calls; graph replays equal eager."""
    r = rl()
    ctx = r.Context(N, P4096, 28)
    g = np.random.default_rng(5)
    W1 = synth.int8_uniform(g, (72, 6000))   # NTT (two blocks)
    W2 = synth.int8_uniform(g, (96, 1000))   # matrix cores
    W3 = synth.int8_uniform(g, (40, 3000))   # NTT (one block, forced)
    w1 = r.Weights(ctx, dev(W1), r.RLWE_W_FWD | r.RLWE_W_TRANSPOSE)
    w2 = r.Weights(ctx, dev(W2), r.RLWE_W_FWD | r.RLWE_W_TRANSPOSE)
    w3 = r.Weights(ctx, dev(W3), r.RLWE_W_FWD | r.RLWE_W_NTT)
    assert r.rlwe_weights_method(w1.handle) == r.RLWE_METHOD_NTT
    assert r.rlwe_weights_method(w1.handle, True) == r.RLWE_METHOD_TOEPLITZ
    # NTT products with one and with two input blocks go out as two launches
    specs = [(w1, False, 6000, 72, 3), (w2, True, 96, 1000, 2), (w1, True, 72, 6000, 2),
             (w2, False, 1000, 96, 9), (w3, False, 3000, 40, 5)]
    items = []
    for s, (w, tr, K, M, T) in enumerate(specs):
        L = (K + N - 1) // N
        ct = dev(uniform_ct(N, P4096, T, L, config=62, salt=s))
        out = torch.empty((T, M, N + 1), dtype=torch.int32, device="cuda")
        items.append((w, tr, ct, T, out))
    handles = [(w.handle, tr, ct, T, out) for (w, tr, ct, T, out) in items]
    r.ct_matmul_batch(ctx.handle, handles)
    torch.cuda.synchronize()
    eager = [o.clone() for (_, _, _, _, o) in items]
    for (w, tr, ct, T, out), e in zip(items, eager):
        sep = r.matmul(ctx, w, ct, transpose=tr)
        torch.cuda.synchronize()
        assert torch.equal(sep, e)
    graph = r.rlwe_graph_capture_batch(ctx.handle, handles)
    for rep in range(3):
        for (_, _, _, _, o) in items:
            o.fill_(-1)
        torch.cuda.synchronize()
        r.rlwe_graph_launch(graph)
        torch.cuda.synchronize()
        for (_, _, _, _, o), e in zip(items, eager):
            assert torch.equal(o, e), f"replay {rep}"
    r.rlwe_graph_destroy(graph)
    w1.close()
    w2.close()
    w3.close()
    ctx.close()
