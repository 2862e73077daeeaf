"""The autotuner on the GPU: it times the candidate launch shapes of a product and keeps
the fastest; a context with the tuner attached uses the recorded choice (method at load,
token tile, order and launch per call) and its outputs are the same bits as without it
and equal the oracle's; the tuned call is not slower than the default one; a batch's
launch is tuned the same way."""

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


def time_ms(fn, reps=5):
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


@pytest.mark.parametrize("K,M,T", [(2048, 1024, 24), (512, 2048, 6)])
def test_tuned_product_is_exact_and_not_slower(K, M, T):
    from paper_2505_07329_amd import rlwe as r
    print(f"case: autotune {K}->{M} T={T}", flush=True)
    ctx = r.Context(N, P4096, 28)
    tuner = r.Tuner(r.rlwe_device_key(0))
    best = r.rlwe_autotune_product(ctx.handle, tuner.handle, K, M, T)
    assert best["method"] in (0, 1) and best["ms"] > 0
    assert r.rlwe_tuner_lookup(tuner.handle, N, 2, K, M, 1, False, T) == best
    W = synth.int8_uniform(np.random.default_rng(K + M), (M, K))
    ct_np = uniform_ct(N, P4096, T, 1, config=90, salt=K)
    ct = dev(ct_np)
    w_default = r.Weights(ctx, dev(W))
    out_default = r.matmul(ctx, w_default, ct)
    t_default = time_ms(lambda: r.matmul(ctx, w_default, ct, out=out_default))
    r.rlwe_ctx_set_tuner(ctx.handle, tuner.handle)
    w_tuned = r.Weights(ctx, dev(W))
    assert r.rlwe_weights_method(w_tuned.handle) == best["method"]
    out_tuned = r.matmul(ctx, w_tuned, ct)
    t_tuned = time_ms(lambda: r.matmul(ctx, w_tuned, ct, out=out_tuned))
    torch.cuda.synchronize()
    assert torch.equal(out_tuned, out_default)
    pairs = np.array([(0, 0), (T - 1, M - 1), (T // 2, M // 2)], dtype=np.uint32)
    want = orc.modswitch(P4096, orc.matmul_clear(N, P4096, W, ct_np, pairs=pairs))
    got = out_tuned.cpu().numpy().view(np.uint32)
    for e, (t, j) in enumerate(pairs):
        assert np.array_equal(got[t, j], want[e])
    # the tuned choice was the fastest measured candidate; the default is one of the
    # candidates, so the tuned call is not slower beyond timing noise
    print(f"tuned {best} {t_tuned:.3f} ms, default {t_default:.3f} ms", flush=True)
    assert t_tuned <= 1.15 * t_default + 0.05
    r.rlwe_ctx_set_tuner(ctx.handle, None)
    w_default.close()
    w_tuned.close()
    tuner.close()
    ctx.close()


def test_tuned_batch_launch_and_file(tmp_path):
    from paper_2505_07329_amd import rlwe as r
    print("case: autotune batch of 3 NTT products", flush=True)
    ctx = r.Context(N, P4096, 28)
    tuner = r.Tuner(r.rlwe_device_key(0))
    g = np.random.default_rng(7)
    items, ws = [], []
    for s, (K, M, T) in enumerate(((2048, 512, 5), (2048, 2048, 9), (8192, 256, 3))):
        w = r.Weights(ctx, dev(synth.int8_uniform(g, (M, K))), r.RLWE_W_FWD | r.RLWE_W_NTT)
        ws.append(w)
        ct = dev(uniform_ct(N, P4096, T, (K + N - 1) // N, config=91, salt=s))
        items.append((w.handle, False, ct, T, torch.empty((T, M, N + 1), dtype=torch.int32,
                                                          device="cuda")))
    r.rlwe_workspace_reserve(ctx.handle, r.rlwe_batch_workspace_bytes(ctx.handle, items))
    r.ct_matmul_batch(ctx.handle, items, r.RLWE_LAUNCH_GROUPED)
    torch.cuda.synchronize()
    ref = [it[4].clone() for it in items]
    best = r.rlwe_autotune_batch(ctx.handle, tuner.handle, items)
    assert best["launch"] in (0, 1) and best["method"] == 1
    r.rlwe_ctx_set_tuner(ctx.handle, tuner.handle)
    for it in items:
        it[4].fill_(-1)
    r.ct_matmul_batch(ctx.handle, items)  # the tuned launch
    torch.cuda.synchronize()
    for it, e in zip(items, ref):
        assert torch.equal(it[4], e)
    path = str(tmp_path / "tune.json")
    tuner.save(path)
    t2 = r.Tuner(r.rlwe_device_key(0))
    assert t2.load(path) == len(tuner) == 1
    r.rlwe_ctx_set_tuner(ctx.handle, None)
    t2.close()
    tuner.close()
    for w in ws:
        w.close()
    ctx.close()
