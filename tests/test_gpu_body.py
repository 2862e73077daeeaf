"""Full outputs at N = 4096 on ragged shapes, with an eye on the body b'_j = sum_k
w_j[k] B[k] (Eq. (LWEdot), SampleExtract's constant term): the matrix-core body kernel
(unpacked rows, K <= 2N) and the dot-product body kernel (K > 2N) against the oracle, with
rows not a multiple of 32, token counts not a multiple of the body kernel's token group,
contractions not a multiple of its four unrolled k-steps; both mask methods, switched and
raw outputs, one and two primes. Every output of every case is compared."""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2505_07329_amd import synth
from tests.cases import uniform_ct

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 4096
P4096 = synth.PRIMES_4096


def rl():
    from paper_2505_07329_amd import rlwe
    return rlwe


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a.view(np.int64) if a.dtype == np.uint64 else a)).cuda()


@pytest.mark.parametrize("primes,d_out,d_in,T", [
    (P4096, 40, 300, 5),        # one block, 300 = 9 k-steps of 32 plus a tail
    (P4096, 40, 4500, 3),       # two blocks, ragged second block
    (P4096[:1], 33, 9000, 2),   # three blocks (one prime: two cap K near 8256 for exact
                                # 128-bit sums): the dot-product body kernel
    (P4096[:1], 70, 2100, 5),   # one prime: 7 digits, four tokens per column tile
])
def test_full_outputs_ragged(primes, d_out, d_in, T):
    print(f"case: body P{len(primes)} {d_out}x{d_in} T{T}", flush=True)
    r = rl()
    ctx = r.Context(N, primes, 30)
    g = np.random.default_rng(d_out * 31 + d_in)
    W = synth.int8_uniform(g, (d_out, d_in))
    L = (d_in + N - 1) // N
    ct = uniform_ct(N, primes, T, L, config=70, salt=d_in + T)
    ref_raw = orc.matmul_clear(N, primes, W, ct)  # (T, d_out, P, N+1)
    ref_sw = orc.modswitch(primes, ref_raw)
    ctd = dev(ct)
    for method in (r.RLWE_W_NTT, r.RLWE_W_TOEPLITZ):
        w = r.Weights(ctx, dev(W), r.RLWE_W_FWD | method)
        raw = r.matmul(ctx, w, ctd, raw=True)
        sw = r.matmul(ctx, w, ctd)
        torch.cuda.synchronize()
        got_raw = raw.cpu().numpy().view(np.uint64).reshape(ref_raw.shape)
        got_sw = sw.cpu().numpy().view(np.uint32)
        assert np.array_equal(got_raw[..., N], ref_raw[..., N]), f"raw bodies, method {method}"
        assert np.array_equal(got_raw, ref_raw), f"raw outputs, method {method}"
        assert np.array_equal(got_sw, ref_sw), f"switched outputs, method {method}"
        w.close()
    ctx.close()
