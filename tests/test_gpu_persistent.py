"""The persistent batch launch (one kernel for every step of a batch of NTT-method
products, work taken from a queue) against the grouped launches, on the GPU.

Both launch shapes compute Eq. (LWEdot) and the ModulusSwitch of Sec. 3.2 with the same
arithmetic, so they must agree bit for bit; the grouped launches are tied to the oracle
by the parity tests, and sampled outputs here are compared with the oracle directly.
Covered: one and two input blocks, ragged token tiles, raw and switched outputs, seeded
inputs, packed rows (n_o > 1), one prime, a 14-product layer batch with uneven token
counts, several launches in a row (the queue resets itself) and graph replays.
"""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2505_07329_amd import synth
from tests.cases import uniform_ct

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 4096
P4096 = synth.PRIMES_4096


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a.view(np.int64) if a.dtype == np.uint64 else a)).cuda()


def run(r, ctx, w, ct, T, M, tr, flags, raw):
    shape = (T, M, ctx.P, N + 1) if raw else (T, M, N + 1)
    out = torch.full(shape, -1, dtype=torch.int64 if raw else torch.int32, device="cuda")
    r.ct_matmul_clear(ctx.handle, w.handle, ct, T, out, tr,
                      flags | (r.RLWE_OUT_RAW_Q if raw else 0))
    return out


@pytest.mark.parametrize("primes,d_out,d_in,T,wflags", [
    (P4096, 300, 2048, 13, 0),          # one block, ragged token tiles
    (P4096, 96, 8192, 9, 0),            # two blocks
    (P4096, 64, 5000, 3, 0),            # two blocks, ragged second block
    (P4096, 130, 512, 11, 16),          # packed rows: 8 per weight polynomial
    (P4096[:1], 80, 3000, 7, 0),        # one prime
])
def test_persistent_equals_grouped(primes, d_out, d_in, T, wflags):
    from paper_2505_07329_amd import rlwe as r
    print(f"case: persistent vs grouped P{len(primes)} {d_out}x{d_in} T={T} wflags={wflags}", flush=True)
    ctx = r.Context(N, primes, 28)
    W = synth.int8_uniform(np.random.default_rng(d_out + d_in), (d_out, d_in))
    w = r.Weights(ctx, dev(W), r.RLWE_W_FWD | r.RLWE_W_TRANSPOSE | r.RLWE_W_NTT | wflags)
    for tr in (False, True):
        K, M = (d_out, d_in) if tr else (d_in, d_out)
        L = (K + N - 1) // N
        ct_np = uniform_ct(N, primes, T, L, config=80, salt=d_in + tr)
        ct = dev(ct_np)
        switched = None
        for raw in (False, True):
            a = run(r, ctx, w, ct, T, M, tr, r.RLWE_LAUNCH_PERSISTENT, raw)
            b = run(r, ctx, w, ct, T, M, tr, r.RLWE_LAUNCH_GROUPED, raw)
            c = run(r, ctx, w, ct, T, M, tr, r.RLWE_LAUNCH_PERSISTENT, raw)  # queue reset
            torch.cuda.synchronize()
            assert torch.equal(a, b), f"transpose={tr} raw={raw}"
            assert torch.equal(a, c), f"second launch, transpose={tr} raw={raw}"
            if not raw:
                switched = a
        if wflags == 0:
            Wm = np.ascontiguousarray(W.T) if tr else W
            pairs = np.array([(0, 0), (T - 1, M - 1), (T // 2, M // 3)], dtype=np.uint32)
            want = orc.modswitch(primes, orc.matmul_clear(N, primes, Wm, ct_np, pairs=pairs))
            got = switched.cpu().numpy().view(np.uint32)
            for e, (t, j) in enumerate(pairs):
                assert np.array_equal(got[t, j], want[e])
    w.close()
    ctx.close()


def test_persistent_seeded_inputs():
    from paper_2505_07329_amd import rlwe as r
    print("case: persistent, seeded inputs", flush=True)
    ctx = r.Context(N, P4096, 26)
    g = np.random.default_rng(5)
    W = synth.int8_uniform(g, (200, 2048))
    w = r.Weights(ctx, dev(W), r.RLWE_W_FWD | r.RLWE_W_NTT)
    T = 10
    seeded = np.zeros((T, 1, len(P4096) * N + 2), dtype=np.uint64)
    seeded[:, :, 0] = g.integers(0, 2**63, size=(T, 1), dtype=np.uint64)
    seeded[:, :, 2:] = uniform_ct(N, P4096, T, 1, config=81)[:, :, 1].reshape(T, 1, -1)
    ct = dev(seeded)
    a = run(r, ctx, w, ct, T, 200, False, r.RLWE_LAUNCH_PERSISTENT | r.RLWE_IN_SEEDED, False)
    b = run(r, ctx, w, ct, T, 200, False, r.RLWE_LAUNCH_GROUPED | r.RLWE_IN_SEEDED, False)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    w.close()
    ctx.close()


def test_persistent_layer_batch_and_graph():
    """All 14 products of one layer on the NTT method (packed rows where K <= N/2), token
    counts 1..16: one persistent launch equals the grouped launches and the separate
    calls; three replays of the captured batch equal the eager result."""
    from paper_2505_07329_amd import rlwe as r
    print("case: persistent layer batch, 14 products", flush=True)
    ctx = r.Context(N, P4096, 28)
    g = np.random.default_rng(44)
    items, ws = [], []
    for pi, (name, (d_in, d_out)) in enumerate(synth.LLAMA_1B_PROJ.items()):
        W = synth.int8_uniform(synth.rng(4, synth.P_WEIGHTS, pi), (d_out, d_in))
        w = r.Weights(ctx, dev(W), r.RLWE_W_FWD | r.RLWE_W_TRANSPOSE | r.RLWE_W_NTT | r.RLWE_W_ROWPACK)
        ws.append(w)
        for tr in (False, True):
            K, M = (d_out, d_in) if tr else (d_in, d_out)
            T = int(g.integers(1, 17))
            ct = dev(uniform_ct(N, P4096, T, (K + N - 1) // N, config=82, salt=2 * pi + tr))
            out = torch.empty((T, M, N + 1), dtype=torch.int32, device="cuda")
            items.append((w, tr, ct, T, out, M))
    handles = [(w.handle, tr, ct, T, out) for (w, tr, ct, T, out, M) in items]
    r.rlwe_workspace_reserve(ctx.handle, r.rlwe_batch_workspace_bytes(ctx.handle, handles))
    r.ct_matmul_batch(ctx.handle, handles, r.RLWE_LAUNCH_PERSISTENT)
    torch.cuda.synchronize()
    eager = [o.clone() for (_, _, _, _, o, _) in items]
    r.ct_matmul_batch(ctx.handle, handles, r.RLWE_LAUNCH_GROUPED)
    torch.cuda.synchronize()
    for (w, tr, ct, T, out, M), e in zip(items, eager):
        assert torch.equal(out, e)
        sep = run(r, ctx, w, ct, T, M, tr, r.RLWE_LAUNCH_GROUPED, False)
        torch.cuda.synchronize()
        assert torch.equal(sep, e)
    graph = r.rlwe_graph_capture_batch(ctx.handle, handles, r.RLWE_LAUNCH_PERSISTENT)
    for rep in range(3):
        for (_, _, _, _, o, _) in items:
            o.fill_(-1)
        torch.cuda.synchronize()
        r.rlwe_graph_launch(graph)
        torch.cuda.synchronize()
        for (_, _, _, _, o, _), e in zip(items, eager):
            assert torch.equal(o, e), f"replay {rep}"
        w, tr, ct, T, _, M = items[0]  # eager work in between
        run(r, ctx, w, ct, T, M, tr, r.RLWE_LAUNCH_PERSISTENT, False)
        torch.cuda.synchronize()
    r.rlwe_graph_destroy(graph)
    for w in ws:
        w.close()
    ctx.close()


def test_persistent_refused_with_matrix_core_products():
    from paper_2505_07329_amd import rlwe as r
    ctx = r.Context(N, P4096, 28)
    w = r.Weights(ctx, dev(synth.int8_uniform(np.random.default_rng(1), (8, 512))),
                  r.RLWE_W_FWD | r.RLWE_W_TOEPLITZ)
    ct = torch.zeros((1, 1, 2, 2, N), dtype=torch.int64, device="cuda")
    out = torch.empty((1, 8, N + 1), dtype=torch.int32, device="cuda")
    with pytest.raises(r.RlweError) as ei:
        r.ct_matmul_clear(ctx.handle, w.handle, ct, 1, out, False, r.RLWE_LAUNCH_PERSISTENT)
    assert ei.value.code == r.RLWE_EINVAL
    w.close()
    ctx.close()
