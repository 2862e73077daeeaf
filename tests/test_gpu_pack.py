"""Outputs switched to q_out = 2^k and their bit-packing, on the GPU, against the oracle.

Every expected value comes from the oracle on the same seeded inputs: its product
(schoolbook/NTT), its switch by binary long division and its Python-integer
packing. Covered: both mask methods (one and two input blocks), the standalone
switch, the packing kernel at several widths and ragged lengths, and an end-to-end
decryption (encrypt, product, switch to 2^26, pack on the GPU, unpack, decrypt).
"""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2505_07329_amd import synth
from tests.cases import make_case, uniform_ct

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P4096 = synth.PRIMES_4096
P2048 = synth.PRIMES_2048


def rl():
    from paper_2505_07329_amd import rlwe
    return rlwe


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a.view(np.int64) if a.dtype == np.uint64 else a)).cuda()


def host_u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("bits", [26, 17])
@pytest.mark.parametrize("method", ["ntt", "toeplitz"])
@pytest.mark.parametrize("d_out,d_in,T", [(40, 2048, 2), (24, 5000, 2)])
def test_switch_to_qout_matches_oracle(bits, method, d_out, d_in, T):
    print(f"case: switch to 2^{bits} {method} {d_out}x{d_in} T={T}", flush=True)
    r = rl()
    N = 4096
    g = np.random.default_rng(bits * 1000 + d_in)
    W = synth.int8_uniform(g, (d_out, d_in))
    L = (d_in + N - 1) // N
    ct = uniform_ct(N, P4096, T, L, config=80, salt=bits + d_in)
    want = orc.modswitch_bits(P4096, orc.matmul_clear(N, P4096, W, ct), bits)
    ctx = r.Context(N, P4096, 28, log2_q_out=bits)
    flag = r.RLWE_W_NTT if method == "ntt" else r.RLWE_W_TOEPLITZ
    w = r.Weights(ctx, dev(W), r.RLWE_W_FWD | flag)
    out = r.matmul(ctx, w, dev(ct))
    torch.cuda.synchronize()
    got = host_u32(out)
    assert int(got.max()) < (1 << bits)
    assert np.array_equal(got, want)
    w.close()
    ctx.close()


@pytest.mark.parametrize("bits", [1, 26, 32])
def test_standalone_switch_to_qout(bits):
    r = rl()
    N = 4096
    g = np.random.default_rng(bits)
    raw = np.stack([g.integers(0, p, size=(37, N + 1), dtype=np.uint64) for p in P4096], axis=1)
    want = orc.modswitch_bits(P4096, raw, bits)
    ctx = r.Context(N, P4096, 26, log2_q_out=bits)
    got = host_u32(r.modswitch(ctx, dev(raw)))
    torch.cuda.synchronize()
    assert np.array_equal(got, want)
    ctx.close()


@pytest.mark.parametrize("bits", [1, 7, 17, 26, 31, 32])
@pytest.mark.parametrize("length", [5, 97, 4097])
def test_pack_kernel_matches_oracle(bits, length):
    r = rl()
    g = np.random.default_rng(bits * 10000 + length)
    count = 6
    v = g.integers(0, 1 << bits, size=(count, length), dtype=np.uint64).astype(np.uint32)
    want = orc.pack_bits(v, bits)
    ctx = r.Context(4096, P4096, 26, log2_q_out=bits)
    assert r.rlwe_packed_words(length, bits) == want.shape[1]
    got = host_u32(r.pack_bits(ctx, dev(v.view(np.int32))))
    torch.cuda.synchronize()
    assert np.array_equal(got, want)
    ctx.close()


def test_pack_ignores_bits_above_qout():
    r = rl()
    g = np.random.default_rng(5)
    v = g.integers(0, 1 << 32, size=(3, 97), dtype=np.uint64).astype(np.uint32)
    ctx = r.Context(4096, P4096, 26, log2_q_out=26)
    got = host_u32(r.pack_bits(ctx, dev(v.view(np.int32))))
    torch.cuda.synchronize()
    assert np.array_equal(got, orc.pack_bits(v & ((1 << 26) - 1), 26))
    ctx.close()


def test_end_to_end_decrypt_packed_26_bit():
    """N = 2048, one prime, t = 2^12: the GPU's switched (2^26) and packed outputs equal
    the oracle's bit for bit and decrypt to W x. Rows carry 12 entries of +-1 (the
    library refuses weights whose row 1-norm times 127 reaches t/2)."""
    r = rl()
    N = 2048
    g = np.random.default_rng(71)
    W = np.zeros((48, 300), dtype=np.int8)
    for j in range(48):
        W[j, g.choice(300, size=12, replace=False)] = g.choice([-1, 1], size=12)
    x = g.integers(-2, 3, size=(3, 300)).astype(np.int8)
    case = make_case(N, P2048, 12, 48, 300, 3, config=71, W=W, x=x)
    want = orc.pack_bits(orc.modswitch_bits(P2048, orc.matmul_clear(N, P2048, W, case.ct), 26), 26)
    ctx = r.Context(N, P2048, 12, log2_q_out=26)
    w = r.Weights(ctx, dev(W))
    packed = r.pack_bits(ctx, r.matmul(ctx, w, dev(case.ct)))
    torch.cuda.synchronize()
    got = host_u32(packed)
    assert np.array_equal(got, want)
    ph = orc.lwe_phase_bits(N, case.S, orc.unpack_bits(got, 26, N + 1), 26)
    dprime = 1 << (26 - 12)
    dec = np.floor_divide(2 * ph + dprime, 2 * dprime)
    assert np.array_equal(dec, x.astype(np.int64) @ W.T.astype(np.int64))
    w.close()
    ctx.close()
