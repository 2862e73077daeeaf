"""Batched products (ct_matmul_batch) and their captured-graph replay, on the GPU.

A batch must give the same bits as separate ct_matmul_clear calls (which the
parity tests tie to the oracle); every replay of the captured graph must equal
the eager result, with eager work and synchronisation between replays.
"""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2505_07329_amd import synth
from tests.cases import make_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P4096 = synth.PRIMES_4096


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a.view(np.int64) if a.dtype == np.uint64 else a)).cuda()


def build_items(N=1024):
    """Mixed shapes: short and long contractions (different kept-digit counts),
    forward and transposed, one and two input blocks."""
    from paper_2505_07329_amd import rlwe
    ctx = rlwe.Context(N, P4096, 26)
    g = np.random.default_rng(77)
    W1 = synth.int8_uniform(g, (96, 64))     # short contraction
    W2 = synth.int8_uniform(g, (40, 1500))   # two blocks forward
    w1 = rlwe.Weights(ctx, dev(W1), rlwe.RLWE_W_FWD | rlwe.RLWE_W_TRANSPOSE)
    w2 = rlwe.Weights(ctx, dev(W2), rlwe.RLWE_W_FWD | rlwe.RLWE_W_TRANSPOSE)
    specs = [(w1, W1, False, 3), (w1, W1, True, 2), (w2, W2, False, 2), (w2, W2, True, 3),
             (w1, W1, False, 1)]
    items, cases = [], []
    for s, (w, W, tr, T) in enumerate(specs):
        Wm = np.ascontiguousarray(W.T) if tr else W
        case = make_case(N, P4096, 26, Wm.shape[0], Wm.shape[1], T, config=40, salt=s, W=Wm)
        ct = dev(case.ct)
        out = torch.empty((T, Wm.shape[0], N + 1), dtype=torch.int32, device="cuda")
        items.append((w, tr, ct, T, out))
        cases.append(case)
    return ctx, (w1, w2), items, cases


def test_batch_equals_separate_calls_and_oracle():
    from paper_2505_07329_amd import rlwe
    ctx, ws, items, cases = build_items()
    digits = {rlwe.rlwe_weights_digits(w.handle, tr)[0] for (w, tr, _, _, _) in items}
    assert len(digits) > 1  # several matrix-core launches inside the batch
    rlwe.ct_matmul_batch(ctx.handle, [(w.handle, tr, ct, T, out) for (w, tr, ct, T, out) in items])
    torch.cuda.synchronize()
    for (w, tr, ct, T, out), case in zip(items, cases):
        sep = rlwe.matmul(ctx, w, ct, transpose=tr)
        torch.cuda.synchronize()
        assert torch.equal(out, sep)
        pairs = np.array([(0, 0), (T - 1, case.W.shape[0] - 1)], dtype=np.uint32)
        ref = orc.modswitch(case.primes, orc.matmul_clear(case.N, case.primes, case.W, case.ct, pairs=pairs))
        got = out.cpu().numpy().view(np.uint32)
        for e, (t, j) in enumerate(pairs):
            assert np.array_equal(got[t, j], ref[e])
    for w in ws:
        w.close()
    ctx.close()


def test_graph_replays_match_eager():
    from paper_2505_07329_amd import rlwe
    ctx, ws, items, cases = build_items()
    handles = [(w.handle, tr, ct, T, out) for (w, tr, ct, T, out) in items]
    rlwe.ct_matmul_batch(ctx.handle, handles)
    torch.cuda.synchronize()
    eager = [out.clone() for (_, _, _, _, out) in items]
    graph = rlwe.rlwe_graph_capture_batch(ctx.handle, handles)
    for rep in range(3):
        for (_, _, _, _, out) in items:
            out.fill_(-1)  # eager work between replays
        torch.cuda.synchronize()
        rlwe.rlwe_graph_launch(graph)
        torch.cuda.synchronize()
        for (_, _, _, _, out), ref in zip(items, eager):
            assert torch.equal(out, ref), f"replay {rep}"
        # an eager product in between, on the same context
        w, tr, ct, T, _ = items[0]
        rlwe.matmul(ctx, w, ct, transpose=tr)
        torch.cuda.synchronize()
    rlwe.rlwe_graph_destroy(graph)
    for w in ws:
        w.close()
    ctx.close()
