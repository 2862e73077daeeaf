"""The NTT method at ring degree N = 2048 (the paper's ring, Sec. 4.4 Table 1) on the GPU.

The inverse transforms run on 256 threads (the N = 4096 layouts with a two-stage last
pass), the forward transforms of masks and weights as plain radix-2 transforms. Both
methods compute the same integers, so NTT outputs must equal the matrix-core outputs bit
for bit, and the oracle's. Covered: config 1 (256 x 256, 16 tokens, one prime, t = 2^24)
in full with decryption, one, two and four input blocks (the Table 4 shapes reach
d_in = 8192), one and two primes, packed rows, transposed weights, raw and switched
outputs."""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2505_07329_amd import synth
from tests.cases import make_case, uniform_ct

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 2048
P1 = synth.PRIMES_2048
P2 = synth.PRIMES_4096  # both primes are 1 mod 8192, so 1 mod 2N here too


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a.view(np.int64) if a.dtype == np.uint64 else a)).cuda()


def test_config1_ntt_full_parity_and_decryption():
    from paper_2505_07329_amd import rlwe as r
    print("case: config1 on the NTT method, N = 2048", flush=True)
    case = make_case(N, P1, 24, 256, 256, 16, config=1)
    ctx = r.Context(N, P1, 24)
    w = r.Weights(ctx, dev(case.W), r.RLWE_W_FWD | r.RLWE_W_NTT)
    assert r.rlwe_weights_method(w.handle) == r.RLWE_METHOD_NTT
    ct = dev(case.ct)
    raw = r.matmul(ctx, w, ct, raw=True)
    sw = r.matmul(ctx, w, ct)
    ex = r.matmul(ctx, w, ct, force_exact=True)
    torch.cuda.synchronize()
    ref_raw = orc.matmul_clear(N, P1, case.W, case.ct)
    ref_sw = orc.modswitch(P1, ref_raw)
    assert np.array_equal(raw.cpu().numpy().view(np.uint64), ref_raw)
    got = sw.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, ref_sw)
    assert torch.equal(sw, ex)
    ph = orc.lwe_phase_u32(N, case.S, got)
    dprime = 1 << (32 - 24)
    dec = np.floor_divide(2 * ph + dprime, 2 * dprime)
    assert np.array_equal(dec, case.x.astype(np.int64) @ case.W.T.astype(np.int64))
    w.close()
    ctx.close()


@pytest.mark.parametrize("primes,d_out,d_in,T,log_t,wflags", [
    (P1, 96, 768, 3, 24, 0),        # one block (Table 4: 768 -> 768)
    (P1, 40, 3072, 2, 26, 0),       # two blocks (3072 -> 768)
    (P1, 24, 8192, 2, 28, 0),       # four blocks (8192 -> 2048)
    (P2, 64, 2048, 3, 26, 0),       # two primes, one block
    (P2, 33, 4000, 2, 28, 0),       # two primes, two blocks, ragged
    (P2, 20, 8192, 2, 28, 0),       # two primes, four blocks
    (P1, 130, 256, 5, 24, 16),      # packed rows: 8 per polynomial
])
def test_ntt2048_equals_matrix_cores_and_oracle(primes, d_out, d_in, T, log_t, wflags):
    from paper_2505_07329_amd import rlwe as r
    print(f"case: N2048 P{len(primes)} {d_out}x{d_in} T={T} wflags={wflags}", flush=True)
    ctx = r.Context(N, primes, log_t)
    W = synth.int8_uniform(np.random.default_rng(d_out + d_in + len(primes)), (d_out, d_in))
    wn = r.Weights(ctx, dev(W), r.RLWE_W_FWD | r.RLWE_W_TRANSPOSE | r.RLWE_W_NTT | wflags)
    wt = None if wflags else r.Weights(ctx, dev(W), r.RLWE_W_FWD | r.RLWE_W_TRANSPOSE | r.RLWE_W_TOEPLITZ)
    for tr in (False, True):
        K, M = (d_out, d_in) if tr else (d_in, d_out)
        L = (K + N - 1) // N
        ct_np = uniform_ct(N, primes, T, L, config=63, salt=d_in + tr)
        ct = dev(ct_np)
        for raw in (False, True):
            a = r.matmul(ctx, wn, ct, transpose=tr, raw=raw)
            if wt is not None:
                b = r.matmul(ctx, wt, ct, transpose=tr, raw=raw)
                torch.cuda.synchronize()
                assert torch.equal(a, b), f"transpose={tr} raw={raw}"
        Wm = np.ascontiguousarray(W.T) if tr else W
        sw = r.matmul(ctx, wn, ct, transpose=tr).cpu().numpy().view(np.uint32)
        if wflags:
            want = orc.modswitch(primes, orc.matmul_rowpacked(N, primes, Wm, ct_np)) if 2 * K <= N else \
                orc.modswitch(primes, orc.matmul_clear(N, primes, Wm, ct_np))
            assert np.array_equal(sw, want)
        else:
            pairs = np.array([(0, 0), (T - 1, M - 1), (T // 2, M // 2)], dtype=np.uint32)
            want = orc.modswitch(primes, orc.matmul_clear(N, primes, Wm, ct_np, pairs=pairs))
            for e, (t, j) in enumerate(pairs):
                assert np.array_equal(sw[t, j], want[e])
    wn.close()
    if wt is not None:
        wt.close()
    ctx.close()
