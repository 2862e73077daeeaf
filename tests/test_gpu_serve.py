"""The request loop on the GPU: every served request's output (read back from the
ring arena, which wraps several times) equals a separate ct_matmul_clear of the
same product, and sampled output LWEs equal the oracle's."""

import math
import time

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2505_07329_amd import serve, synth
from tests.cases import uniform_ct

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P4096 = synth.PRIMES_4096
N = 1024
SHAPES = {"a": (300, 200), "b": (1500, 96), "c": (1024, 64)}   # (d_in, d_out) forward
LAYERS = 2
TMAX = 6


def _serve(rate, n, arena_bytes, max_batch, seed):
    from paper_2505_07329_amd import rlwe
    ctx = rlwe.Context(N, P4096, 26)
    dev = torch.device("cuda")
    Wnp, weights = {}, {}
    for layer in range(LAYERS):
        for pi, (name, (d_in, d_out)) in enumerate(SHAPES.items()):
            W = synth.int8_uniform(synth.rng(50, synth.P_WEIGHTS, layer * 8 + pi), (d_out, d_in))
            Wnp[(layer, name)] = W
            weights[(layer, name)] = rlwe.Weights(ctx, torch.from_numpy(W).to(dev),
                                                  rlwe.RLWE_W_FWD | rlwe.RLWE_W_TRANSPOSE)
    ct_np = {L: uniform_ct(N, P4096, TMAX, L, config=50, salt=L) for L in (1, 2)}
    pools = {L: torch.from_numpy(c.view(np.int64)).to(dev) for L, c in ct_np.items()}
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    backend = serve.GpuBackend(ctx, weights, pools, arena, stream, keep_outputs=True)
    reqs = serve.make_requests(SHAPES, LAYERS, 4, n, rate, np.random.default_rng(seed),
                               serve.switched_out_bytes(N), max_tokens=TMAX)
    sched = serve.Scheduler(serve.RingArena(arena_bytes), max_batch=max_batch)
    print(f"serve: rate={rate} n={n} arena={arena_bytes} max_batch={max_batch}", flush=True)
    res = serve.run_loop(reqs, sched, backend, time.perf_counter, lambda dt: time.sleep(min(dt, 0.01)))
    torch.cuda.synchronize()
    return ctx, weights, Wnp, ct_np, pools, backend, reqs, res


def _check(ctx, weights, Wnp, ct_np, pools, backend, reqs):
    from paper_2505_07329_amd import rlwe
    g = np.random.default_rng(9)
    for r in reqs:
        assert r.status == "done"
        got = backend.outputs[r.rid]
        L = (r.d_in + N - 1) // N
        w = weights[(r.layer, r.proj)]
        sep = rlwe.matmul(ctx, w, pools[L][: r.tokens], transpose=r.transpose)
        torch.cuda.synchronize()
        assert torch.equal(got, sep), f"request {r.rid} differs from a separate call"
        W = Wnp[(r.layer, r.proj)]
        Wm = np.ascontiguousarray(W.T) if r.transpose else W
        pairs = np.array([[int(g.integers(0, r.tokens)), int(g.integers(0, r.d_out))]], dtype=np.uint32)
        ref = orc.modswitch(P4096, orc.matmul_clear(N, P4096, Wm, ct_np[L][: r.tokens], pairs=pairs))
        t, j = pairs[0]
        assert np.array_equal(got[t, j].cpu().numpy().view(np.uint32), ref[0])
    for w in weights.values():
        w.close()
    ctx.close()


def test_serve_saturated_small_arena():
    # arena of ~3 of the largest outputs: admission blocks and the ring wraps
    biggest = serve.switched_out_bytes(N)(TMAX, max(max(s) for s in SHAPES.values()))
    state = _serve(math.inf, 40, 3 * biggest + 4096, 16, seed=1)
    res = state[-1]
    assert res["requests"] == 40 and res["rejected"] == 0
    _check(*state[:-1])


def test_serve_poisson_arrivals_batch_of_one():
    state = _serve(400.0, 30, 64 << 20, 1, seed=2)
    res = state[-1]
    assert res["requests"] == 30 and res["p50_s"] <= res["p99_s"]
    _check(*state[:-1])
