"""GPU parity: the HIP library against the CPU oracle, bit for bit.

Every result of ct_matmul_clear / ct_modswitch is an integer function of its
inputs, so the bar is bit-exact equality (raw residues mod q_p and switched
uint32 coefficients), plus exact decryption where the parameters allow it.
Full-size workloads are checked on sampled outputs that the oracle computes one
by one, and on properties that hold at every size.
"""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2505_07329_amd import synth
from tests.cases import make_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P2048 = synth.PRIMES_2048
P4096 = synth.PRIMES_4096


def rl():
    from paper_2505_07329_amd import rlwe
    return rlwe


def dev(a: np.ndarray):
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    elif a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host_u64(t):
    return t.cpu().numpy().view(np.uint64)


def host_u32(t):
    return t.cpu().numpy().view(np.uint32)


class Setup:
    def __init__(self, case, flags=1):
        r = rl()
        self.case = case
        self.ctx = r.Context(case.N, case.primes, case.log2_t)
        self.Wd = dev(case.W)
        self.w = r.Weights(self.ctx, self.Wd, flags)
        self.ct = dev(case.ct)

    def run(self, raw=False, force_exact=False, transpose=False, ct=None):
        out = rl().matmul(self.ctx, self.w, self.ct if ct is None else ct, transpose=transpose,
                          raw=raw, force_exact=force_exact)
        torch.cuda.synchronize()
        return out

    def close(self):
        self.w.close()
        self.ctx.close()


def decrypt_switched(case, sw):
    ph = orc.lwe_phase_u32(case.N, case.S, sw)
    dprime = 1 << (32 - case.log2_t)
    return np.floor_divide(2 * ph + dprime, 2 * dprime), ph


def test_config1_full_parity_and_decryption():
    """256x256 weights, 16 tokens, N = 2048, one prime, t = 2^24: every output."""
    print("case: config1 256x256 T16 N2048", flush=True)
    case = make_case(2048, P2048, 24, 256, 256, 16, config=1)
    ref_raw = orc.matmul_clear(case.N, case.primes, case.W, case.ct)
    ref_sw = orc.modswitch(case.primes, ref_raw)
    s = Setup(case)
    raw = host_u64(s.run(raw=True))
    assert np.array_equal(raw, ref_raw)
    sw = host_u32(s.run())
    assert np.array_equal(sw, ref_sw)
    dec, _ = decrypt_switched(case, sw)
    assert np.array_equal(dec, case.x.astype(np.int64) @ case.W.T.astype(np.int64))
    again = host_u32(s.run())
    assert np.array_equal(again, sw)  # deterministic
    s.close()


SMALL = [
    # N, primes, d_out, d_in, T
    (64, P4096, 1, 1, 1),
    (64, P4096, 7, 63, 3),
    (64, P4096, 65, 64, 2),
    (64, P4096, 7, 65, 3),
    (64, P4096, 3, 127, 1),
    (64, P4096, 5, 128, 2),
    (128, P4096, 70, 300, 2),
    (64, P2048, 7, 65, 3),
    (64, P2048, 65, 128, 2),
    (256, P2048, 9, 1000, 2),
]


@pytest.mark.parametrize("N,primes,d_out,d_in,T", SMALL)
def test_small_shapes_full_parity(N, primes, d_out, d_in, T):
    print(f"case: small N{N} P{len(primes)} {d_out}x{d_in} T{T}", flush=True)
    log2_t = 26 if len(primes) == 2 else 24
    case = make_case(N, primes, log2_t, d_out, d_in, T, config=30, salt=N + d_out + d_in)
    ref_raw = orc.matmul_clear(N, primes, case.W, case.ct)
    ref_sw = orc.modswitch(primes, ref_raw)
    s = Setup(case)
    assert np.array_equal(host_u64(s.run(raw=True)), ref_raw)
    assert np.array_equal(host_u32(s.run()), ref_sw)
    assert np.array_equal(host_u32(s.run(force_exact=True)), ref_sw)
    s.close()


def test_attention_shape_all_paths_agree():
    """2048x2048, N = 4096, two primes, 4 tokens: switched fast path, forced exact
    path and ct_modswitch of the raw output agree on every coefficient; sampled
    outputs match the oracle."""
    print("case: attn 2048x2048 T4 all paths", flush=True)
    case = make_case(4096, P4096, 26, 2048, 2048, 4, config=2, salt=1)
    s = Setup(case)
    sw = s.run()
    ex = s.run(force_exact=True)
    assert torch.equal(sw, ex)
    raw = s.run(raw=True)
    ms = rl().modswitch(s.ctx, raw)
    torch.cuda.synchronize()
    assert torch.equal(ms, sw)
    pairs = np.array([(0, 0), (1, 2047), (2, 1024), (3, 77), (3, 1500)], dtype=np.uint32)
    ref = orc.matmul_clear(case.N, case.primes, case.W, case.ct, pairs=pairs)
    raw_h = host_u64(raw)
    sw_h = host_u32(sw)
    ref_sw = orc.modswitch(case.primes, ref)
    for e, (t, j) in enumerate(pairs):
        assert np.array_equal(raw_h[t, j], ref[e])
        assert np.array_equal(sw_h[t, j], ref_sw[e])
    s.close()


def test_config2_full_size_sampled():
    """The benchmark workload: 2048x2048, 128 tokens, N = 4096, t = 2^26, in the
    launch configuration the benchmark times. Every output of one full tile of 8
    tokens (tokens 8..15, all 2048 rows) and sampled outputs elsewhere against the
    oracle; a larger sample satisfies the deterministic switched-noise bound."""
    print("case: config2 2048x2048 T128 N4096", flush=True)
    case = make_case(4096, P4096, 26, 2048, 2048, 128, config=2)
    s = Setup(case)
    out = s.run()  # (128, 2048, 4097) int32 on the GPU
    tile = host_u32(out[8:16])
    want = orc.modswitch(case.primes, orc.matmul_clear(case.N, case.primes, case.W, case.ct[8:16]))
    assert np.array_equal(tile, want), f"{int((tile != want).sum())} coefficients of the tile differ"
    del tile, want
    g = np.random.default_rng(2)
    pairs = np.stack([g.integers(0, 128, 12), g.integers(0, 2048, 12)], 1).astype(np.uint32)
    pairs = np.concatenate([pairs, np.array([[0, 0], [127, 2047]], dtype=np.uint32)])
    ref = orc.modswitch(case.primes, orc.matmul_clear(case.N, case.primes, case.W, case.ct, pairs=pairs))
    got = host_u32(out[torch.from_numpy(pairs[:, 0].astype(np.int64)).cuda(),
                       torch.from_numpy(pairs[:, 1].astype(np.int64)).cuda()])
    assert np.array_equal(got, ref)
    # deterministic bound on 1024 random outputs (Sec. 3.2 modulus switch noise)
    ts = g.integers(0, 128, 1024)
    js = g.integers(0, 2048, 1024)
    rows = host_u32(out[torch.from_numpy(ts).cuda(), torch.from_numpy(js).cuda()])
    ph = orc.lwe_phase_u32(case.N, case.S, rows)
    q, t = case.q, 1 << case.log2_t
    dprime = (1 << 32) // t
    v = (case.x.astype(np.int64) @ case.W.T.astype(np.int64))[ts, js]
    e = (case.errors_flat().astype(np.int64) @ case.W.T.astype(np.int64))[ts, js]
    s1 = int(np.abs(case.S.astype(np.int64)).sum())
    bound = dprime * np.abs(v) * (q % t) / q + (2 ** 32) * np.abs(e) / q + (1 + s1) / 2 + 1e-6
    assert np.all(np.abs(ph - dprime * v) <= bound)
    s.close()


def test_two_blocks_and_transpose():
    """Gate-shaped W (8192 x 2048) loaded forward and transposed, N = 4096, t = 2^28:
    forward W x (L = 1, 8192 outputs) and backward W^T g (L = 2, 2048 outputs)."""
    print("case: gate 8192x2048 fwd+transposed", flush=True)
    N, primes, log2_t = 4096, P4096, 28
    fwd = make_case(N, primes, log2_t, 8192, 2048, 2, config=3)
    r = rl()
    ctx = r.Context(N, primes, log2_t)
    Wd = dev(fwd.W)
    w = r.Weights(ctx, Wd, r.RLWE_W_FWD | r.RLWE_W_TRANSPOSE)
    out_f = r.matmul(ctx, w, dev(fwd.ct))
    WT = np.ascontiguousarray(fwd.W.T)
    bwd = make_case(N, primes, log2_t, 2048, 8192, 2, config=3, salt=5, W=WT)
    out_b = r.matmul(ctx, w, dev(bwd.ct), transpose=True)
    raw_b = r.matmul(ctx, w, dev(bwd.ct), transpose=True, raw=True)
    torch.cuda.synchronize()
    pf = np.array([(0, 0), (1, 8191), (0, 4096), (1, 123)], dtype=np.uint32)
    ref_f = orc.modswitch(primes, orc.matmul_clear(N, primes, fwd.W, fwd.ct, pairs=pf))
    of = host_u32(out_f)
    for e, (t, j) in enumerate(pf):
        assert np.array_equal(of[t, j], ref_f[e])
    pb = np.array([(0, 0), (1, 2047), (1, 1000)], dtype=np.uint32)
    ref_raw_b = orc.matmul_clear(N, primes, WT, bwd.ct, pairs=pb)
    ref_b = orc.modswitch(primes, ref_raw_b)
    ob, rb = host_u32(out_b), host_u64(raw_b)
    for e, (t, j) in enumerate(pb):
        assert np.array_equal(ob[t, j], ref_b[e])
        assert np.array_equal(rb[t, j], ref_raw_b[e])
    # decryption of the backward outputs through the LWE phase (exact at q)
    ph = orc.lwe_phase(N, primes, bwd.S, rb[pb[:, 0], pb[:, 1]])
    v = bwd.x.astype(object) @ WT.T.astype(object)
    for (t, j), p in zip(pb, ph):
        assert orc.decode(p, bwd.delta) == v[t, j]
    w.close()
    ctx.close()


def _switched_bound_holds(case, W, out, g, n=512):
    """Deterministic modulus-switch noise bound (Sec. 3.2) on n random outputs."""
    T, M = out.shape[0], out.shape[1]
    ts = g.integers(0, T, n)
    js = g.integers(0, M, n)
    rows = host_u32(out[torch.from_numpy(ts).cuda(), torch.from_numpy(js).cuda()])
    ph = orc.lwe_phase_u32(case.N, case.S, rows)
    q, t = case.q, 1 << case.log2_t
    dprime = (1 << 32) // t
    Wr = W.astype(np.int64)[js]
    v = np.einsum("nk,nk->n", case.x.astype(np.int64)[ts], Wr)
    e = np.einsum("nk,nk->n", case.errors_flat().astype(np.int64)[ts], Wr)
    s1 = int(np.abs(case.S.astype(np.int64)).sum())
    bound = dprime * np.abs(v) * (q % t) / q + (2 ** 32) * np.abs(e) / q + (1 + s1) / 2 + 1e-6
    return bool(np.all(np.abs(ph - dprime * v) <= bound))


def _sampled_against_oracle(case, W, out, g, n=32):
    """n random outputs and the two corners of `out` (T, M, N+1) against the oracle."""
    T, M = out.shape[0], out.shape[1]
    pairs = np.stack([g.integers(0, T, n), g.integers(0, M, n)], 1).astype(np.uint32)
    pairs = np.concatenate([pairs, np.array([[0, 0], [T - 1, M - 1]], dtype=np.uint32)])
    ref = orc.modswitch(case.primes, orc.matmul_clear(case.N, case.primes, W, case.ct, pairs=pairs))
    got = host_u32(out[torch.from_numpy(pairs[:, 0].astype(np.int64)).cuda(),
                       torch.from_numpy(pairs[:, 1].astype(np.int64)).cuda()])
    return np.array_equal(got, ref)


MLP = [("gate", 2048, 8192), ("up", 2048, 8192), ("down", 8192, 2048)]


@pytest.mark.parametrize("name,d_in,d_out", MLP)
def test_config3_mlp_products_launch_config(name, d_in, d_out):
    """The MLP workload (t = 2^28) in the launch configuration the benchmark times:
    256-token calls of one projection forward (W x) and transposed (W^T g) with the
    default method. 34 sampled outputs of each product against the oracle, and the
    switched-noise bound on 512 random outputs."""
    print(f"case: mlp {name} {d_in}->{d_out} fwd+transposed, chunk 256", flush=True)
    N, primes, log2_t, C = 4096, P4096, 28, 256
    salt = {"gate": 21, "up": 23, "down": 11}[name]
    fwd = make_case(N, primes, log2_t, d_out, d_in, C, config=3, salt=salt)
    r = rl()
    ctx = r.Context(N, primes, log2_t)
    w = r.Weights(ctx, dev(fwd.W), r.RLWE_W_FWD | r.RLWE_W_TRANSPOSE)
    g = np.random.default_rng(3 + salt)
    out = r.matmul(ctx, w, dev(fwd.ct))
    torch.cuda.synchronize()
    assert _sampled_against_oracle(fwd, fwd.W, out, g)
    assert _switched_bound_holds(fwd, fwd.W, out, g)
    del out
    WT = np.ascontiguousarray(fwd.W.T)
    bwd = make_case(N, primes, log2_t, d_in, d_out, C, config=3, salt=salt + 1, W=WT)
    out = r.matmul(ctx, w, dev(bwd.ct), transpose=True)
    torch.cuda.synchronize()
    assert _sampled_against_oracle(bwd, WT, out, g)
    assert _switched_bound_holds(bwd, WT, out, g)
    del out
    w.close()
    ctx.close()


@pytest.mark.parametrize("primes,N", [(P2048, 2048), (P4096, 4096)])
def test_modswitch_standalone(primes, N):
    print(f"case: modswitch P{len(primes)}", flush=True)
    q = orc.modulus(primes)
    g = np.random.default_rng(len(primes))
    count = 300
    raw = synth.uniform_mod_primes(g, primes, (count,), N + 1)
    # edge values: 0, q - 1, (q - 1)/2, (q + 1)/2 in the first row
    for k, c in enumerate([0, q - 1, (q - 1) // 2, (q + 1) // 2, 1]):
        raw[0, :, k] = [c % p for p in primes]
    r = rl()
    ctx = r.Context(N, primes, 26)
    out = r.modswitch(ctx, dev(raw))
    torch.cuda.synchronize()
    assert np.array_equal(host_u32(out), orc.modswitch(primes, raw))
    ctx.close()


def test_overflow_and_flag_errors():
    r = rl()
    ctx = r.Context(1024, P2048, 16)
    W = torch.full((4, 300), 127, dtype=torch.int8, device="cuda")
    with pytest.raises(r.RlweError) as ei:
        r.Weights(ctx, W)  # 127 * 127 * 300 >= 2^15
    assert ei.value.code == -4
    w = r.Weights(ctx, torch.ones((4, 100), dtype=torch.int8, device="cuda"))  # 127*100 < 2^15
    ct = torch.zeros((1, 1, 2, 1, 1024), dtype=torch.int64, device="cuda")
    with pytest.raises(r.RlweError) as ei:
        r.matmul(ctx, w, ct, transpose=True)  # loaded without RLWE_W_TRANSPOSE
    assert ei.value.code == -1
    w.close()
    ctx.close()
