"""The batched-layer workload on the GPU: all 7 projections of one Llama-3.2-1B layer
(q, k, v, o, gate, up, down), forward W.[x] and transposed W^T.[g], N = 4096, two
54-bit primes, t = 2^28, each product with its own small token count (1..16, the
paper's training step runs 16 tokens per call, Sec. 6.3), the default method choice.

The 14 products go out as one captured graph; every replay must equal, bit for bit,
the 14 separate ct_matmul_clear calls on every output, and 34 sampled outputs of every
product must equal the oracle's Eq. (LWEdot) + ModulusSwitch."""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2505_07329_amd import synth
from tests.cases import make_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 4096
P4096 = synth.PRIMES_4096


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a.view(np.int64) if a.dtype == np.uint64 else a)).cuda()


def host_u32(t):
    return t.cpu().numpy().view(np.uint32)


def layer_products(flags_extra=0, seed=44):
    """Weights of one layer and 14 encrypted inputs (real encryptions by the oracle)."""
    from paper_2505_07329_amd import rlwe as r
    ctx = r.Context(N, P4096, 28)
    g = np.random.default_rng(seed)
    weights, prods = [], []
    for pi, (name, (d_in, d_out)) in enumerate(synth.LLAMA_1B_PROJ.items()):
        W = synth.int8_uniform(synth.rng(4, synth.P_WEIGHTS, pi), (d_out, d_in))
        w = r.Weights(ctx, dev(W), r.RLWE_W_FWD | r.RLWE_W_TRANSPOSE | flags_extra)
        weights.append(w)
        for tr in (False, True):
            Wm = np.ascontiguousarray(W.T) if tr else W
            T = int(g.integers(1, 17))
            case = make_case(N, P4096, 28, Wm.shape[0], Wm.shape[1], T, config=4,
                             salt=2 * pi + tr, W=Wm)
            out = torch.empty((T, Wm.shape[0], N + 1), dtype=torch.int32, device="cuda")
            prods.append(dict(name=name + ("^T" if tr else ""), w=w, tr=tr, case=case,
                              ct=dev(case.ct), T=T, out=out))
    return ctx, weights, prods


def test_layer_graph_equals_separate_calls_and_oracle():
    from paper_2505_07329_amd import rlwe as r
    print("case: layer, 14 products, T in 1..16, one captured graph", flush=True)
    ctx, weights, prods = layer_products()
    sep = []
    for p in prods:
        o = r.matmul(ctx, p["w"], p["ct"], transpose=p["tr"])
        sep.append(o)
    torch.cuda.synchronize()
    handles = [(p["w"].handle, p["tr"], p["ct"], p["T"], p["out"]) for p in prods]
    r.rlwe_workspace_reserve(ctx.handle, r.rlwe_batch_workspace_bytes(ctx.handle, handles))
    graph = r.rlwe_graph_capture_batch(ctx.handle, handles)
    for rep in range(3):
        for p in prods:
            p["out"].fill_(-1)
        torch.cuda.synchronize()
        r.rlwe_graph_launch(graph)
        torch.cuda.synchronize()
        for p, s in zip(prods, sep):
            assert torch.equal(p["out"], s), f"replay {rep}: {p['name']}"
    r.rlwe_graph_destroy(graph)
    g = np.random.default_rng(4)
    for p in prods:
        case, T = p["case"], p["T"]
        M = case.W.shape[0]
        pairs = np.stack([g.integers(0, T, 32), g.integers(0, M, 32)], 1).astype(np.uint32)
        pairs = np.concatenate([pairs, np.array([[0, 0], [T - 1, M - 1]], dtype=np.uint32)])
        want = orc.modswitch(P4096, orc.matmul_clear(N, P4096, case.W, case.ct, pairs=pairs))
        got = host_u32(p["out"][torch.from_numpy(pairs[:, 0].astype(np.int64)).cuda(),
                                torch.from_numpy(pairs[:, 1].astype(np.int64)).cuda()])
        assert np.array_equal(got, want), p["name"]
    for w in weights:
        w.close()
    ctx.close()
