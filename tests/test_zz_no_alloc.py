"""ct_matmul_clear_noalloc: the product with its workspace in the library's fixed device
array. Its outputs must equal ct_matmul_clear's bit for bit (which the parity tests tie
to the oracle), on consecutive calls that reuse the array, the second one smaller, for
both mask methods and raw and switched outputs; a call that needs more workspace than
the array holds is refused before any GPU work."""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2505_07329_amd import synth
from tests.cases import uniform_ct

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P4096 = synth.PRIMES_4096
N = 4096


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a.view(np.int64) if a.dtype == np.uint64 else a)).cuda()


def test_noalloc_equals_ct_matmul_clear_on_two_calls():
    from paper_2505_07329_amd import rlwe as r
    print("case: noalloc 2048x2048 (NTT) T=96 then 512x2048^T (matrix cores) T=5", flush=True)
    ctx = r.Context(N, P4096, 26)
    g = np.random.default_rng(11)
    W1 = synth.int8_uniform(g, (2048, 2048))
    W2 = synth.int8_uniform(g, (512, 2048))
    w1 = r.Weights(ctx, dev(W1))  # K = 2048: NTT method
    w2 = r.Weights(ctx, dev(W2), r.RLWE_W_FWD | r.RLWE_W_TRANSPOSE | r.RLWE_W_TOEPLITZ)
    calls = [(w1, W1, False, 96), (w2, W2.T, True, 5)]
    for i, (w, Wm, tr, T) in enumerate(calls):
        K, M = Wm.shape[1], Wm.shape[0]
        ct_np = uniform_ct(N, P4096, T, 1, config=70, salt=i)
        ct = dev(ct_np)
        assert r.rlwe_workspace_bytes(ctx.handle, w.handle, tr, T) <= r.RLWE_NOALLOC_SCRATCH_BYTES
        for raw in (False, True):
            shape = (T, M, len(P4096), N + 1) if raw else (T, M, N + 1)
            dt = torch.int64 if raw else torch.int32
            a = torch.full(shape, -1, dtype=dt, device="cuda")
            b = torch.full(shape, -2, dtype=dt, device="cuda")
            flags = r.RLWE_OUT_RAW_Q if raw else r.RLWE_OUT_SWITCHED
            r.ct_matmul_clear_noalloc(ctx.handle, w.handle, ct, T, a, tr, flags)
            r.ct_matmul_clear(ctx.handle, w.handle, ct, T, b, tr, flags)
            torch.cuda.synchronize()
            assert torch.equal(a, b), f"call {i} raw={raw}"
        # a few outputs against the oracle as well
        pairs = np.array([(0, 0), (T - 1, M - 1)], dtype=np.uint32)
        want = orc.modswitch(P4096, orc.matmul_clear(N, P4096, np.ascontiguousarray(Wm), ct_np,
                                                     pairs=pairs))
        out = torch.empty((T, M, N + 1), dtype=torch.int32, device="cuda")
        r.ct_matmul_clear_noalloc(ctx.handle, w.handle, ct, T, out, tr)
        got = out.cpu().numpy().view(np.uint32)
        for e, (t, j) in enumerate(pairs):
            assert np.array_equal(got[t, j], want[e])
    w1.close()
    w2.close()
    ctx.close()


def test_noalloc_refuses_a_call_above_the_array():
    from paper_2505_07329_amd import rlwe as r
    ctx = r.Context(N, P4096, 26)
    W = synth.int8_uniform(np.random.default_rng(12), (64, 2048))
    w = r.Weights(ctx, dev(W))
    T = 1024
    assert r.rlwe_workspace_bytes(ctx.handle, w.handle, False, T) > r.RLWE_NOALLOC_SCRATCH_BYTES
    ct = torch.zeros((T, 1, 2, 2, N), dtype=torch.int64, device="cuda")
    out = torch.empty((T, 64, N + 1), dtype=torch.int32, device="cuda")
    with pytest.raises(r.RlweError) as ei:
        r.ct_matmul_clear_noalloc(ctx.handle, w.handle, ct, T, out)
    assert ei.value.code == r.RLWE_ESHAPE
    w.close()
    ctx.close()
