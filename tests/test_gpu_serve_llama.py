"""The request loop at the served model's real shapes: the seven projections of one
Llama-3.2-1B layer (q, k, v, o, gate, up, down), forward and transposed, N = 4096, two
54-bit primes, t = 2^28, 1..16 tokens per request (the paper's step runs 16 tokens per
call, Sec. 6.3), grouped launches of up to 16 requests into a ring arena that wraps.

Every served request's output equals, bit for bit, a separate ct_matmul_clear of the
same product, and sampled output LWEs equal the oracle's Eq. (LWEdot) + ModulusSwitch:
with plain weights, and with packed weight rows (the coefficient packing of Sec. 4.3.1,
n_o = floor(N / K) rows per weight polynomial where K <= N/2), whose sampled rows come
from the oracle's product on the one packed group that holds them; and with the
autotuner's committed cache for the device attached, as the serving benchmark runs."""

import os
import time

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2505_07329_amd import serve, synth
from tests.cases import uniform_ct

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P4096 = synth.PRIMES_4096
N = 4096
TMAX = 16
SAMPLES = 6


def _serve(extra_flags, n, seed, tuned=False):
    from paper_2505_07329_amd import rlwe, tune
    ctx = rlwe.Context(N, P4096, 28)
    tuner = None
    if tuned:
        path = tune.cache_path(0)
        if not os.path.exists(path):
            pytest.skip(f"no autotuner cache for this device ({path})")
        tuner = rlwe.Tuner(rlwe.rlwe_device_key(0))
        assert tuner.load(path) > 0
        rlwe.rlwe_ctx_set_tuner(ctx.handle, tuner.handle)
    dev = torch.device("cuda")
    Wnp, weights = {}, {}
    for pi, (name, (d_in, d_out)) in enumerate(synth.LLAMA_1B_PROJ.items()):
        W = synth.int8_uniform(synth.rng(55, synth.P_WEIGHTS, pi), (d_out, d_in))
        Wnp[(0, name)] = W
        weights[(0, name)] = rlwe.Weights(ctx, torch.from_numpy(W).to(dev),
                                          rlwe.RLWE_W_FWD | rlwe.RLWE_W_TRANSPOSE | extra_flags)
    ct_np = {L: uniform_ct(N, P4096, TMAX, L, config=55, salt=L) for L in (1, 2)}
    pools = {L: torch.from_numpy(c.view(np.int64)).to(dev) for L, c in ct_np.items()}
    out_bytes = serve.switched_out_bytes(N)
    biggest = out_bytes(TMAX, max(d for s in synth.LLAMA_1B_PROJ.values() for d in s))
    arena_bytes = 3 * biggest + 4096  # admission blocks and the ring wraps
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    backend = serve.GpuBackend(ctx, weights, pools, arena, stream, keep_outputs=True)
    reqs = serve.make_requests(synth.LLAMA_1B_PROJ, 1, 16, n, float("inf"),
                               np.random.default_rng(seed), out_bytes, max_tokens=TMAX)
    sched = serve.Scheduler(serve.RingArena(arena_bytes), max_batch=16)
    print(f"serve N=4096 P=2: flags={extra_flags:#x} tuned={tuned} n={n} arena={arena_bytes}",
          flush=True)
    res = serve.run_loop(reqs, sched, backend, time.perf_counter,
                         lambda dt: time.sleep(min(dt, 0.01)))
    torch.cuda.synchronize()
    assert res["requests"] == n and res["rejected"] == 0 and res["expired"] == 0
    methods = {rlwe.rlwe_weights_method(w.handle, tr) for w in weights.values() for tr in (0, 1)}
    print(f"methods in use: {sorted(methods)}", flush=True)
    return ctx, weights, Wnp, ct_np, pools, backend, reqs, tuner


def _check(ctx, weights, Wnp, ct_np, pools, backend, reqs, tuner, rowpack, seed):
    from paper_2505_07329_amd import rlwe
    g = np.random.default_rng(seed)
    wt = {}
    for r in reqs:
        assert r.status == "done"
        got = backend.outputs.pop(r.rid)
        L = (r.d_in + N - 1) // N
        w = weights[(r.layer, r.proj)]
        sep = rlwe.matmul(ctx, w, pools[L][: r.tokens], transpose=r.transpose)
        torch.cuda.synchronize()
        assert torch.equal(got, sep), f"request {r.rid} ({r.proj}, T={r.tokens}) differs from a separate call"
        del sep
        key = (r.layer, r.proj, r.transpose)
        if key not in wt:
            W = Wnp[(r.layer, r.proj)]
            wt[key] = np.ascontiguousarray(W.T) if r.transpose else W
        Wm = wt[key]
        ct = ct_np[L][: r.tokens]
        ts = g.integers(0, r.tokens, SAMPLES)
        js = g.integers(0, r.d_out, SAMPLES)
        if rowpack and r.d_in <= N // 2:
            n_o = orc.rows_per_product(r.d_in, N)
            for t, j in zip(ts, js):
                g0 = (j // n_o) * n_o
                raw = orc.matmul_rowpacked(N, P4096, Wm[g0: g0 + n_o], ct[t: t + 1])
                want = orc.modswitch(P4096, raw[0, j - g0])
                assert np.array_equal(got[t, j].cpu().numpy().view(np.uint32), want), \
                    f"request {r.rid} ({r.proj}, packed) output ({t}, {j})"
        else:
            pairs = np.stack([ts, js], 1).astype(np.uint32)
            want = orc.modswitch(P4096, orc.matmul_clear(N, P4096, Wm, ct, pairs=pairs))
            for (t, j), wv in zip(pairs, want):
                assert np.array_equal(got[t, j].cpu().numpy().view(np.uint32), wv), \
                    f"request {r.rid} ({r.proj}) output ({t}, {j})"
    for w in weights.values():
        w.close()
    ctx.close()
    if tuner is not None:
        tuner.close()


def test_serve_llama_layer_n4096():
    state = _serve(0, 64, seed=3)
    _check(*state, rowpack=False, seed=13)


def test_serve_llama_layer_n4096_packed_rows():
    from paper_2505_07329_amd import rlwe
    state = _serve(rlwe.RLWE_W_ROWPACK, 48, seed=4)
    _check(*state, rowpack=True, seed=14)


def test_serve_llama_layer_n4096_tuned():
    state = _serve(0, 48, seed=5, tuned=True)
    _check(*state, rowpack=False, seed=15)
