"""KeySwitch packing on the GPU (Sec. 3.2 KeySwitching and Rotate, Eq. (pack_rotate))
against the oracle, bit for bit, through the C ABI.

Covered: two primes with one gadget level (54-bit digits) and with 2 and 4 levels,
one prime with three 12-bit levels, raw and switched outputs (2^32 and 2^26), ragged
last groups and n_pack below N, two calls in a row with different shapes, the
full attention shape (262144 LWE ciphertexts of the 2048 x 2048, 128-token product
into 64 packed ciphertexts) on sampled groups, more than one pass of the kernels (66
packed ciphertexts), one slot per ciphertext, a single ciphertext, replays of a
captured graph, and end-to-end decryption of packed real products computed on the
GPU.
"""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2505_07329_amd import synth
from tests.cases import make_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 4096
P2 = synth.PRIMES_4096
P1 = synth.PRIMES_4096[:1]


def rl():
    from paper_2505_07329_amd import rlwe
    return rlwe


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a.view(np.int64) if a.dtype == np.uint64 else a)).cuda()


def host_u64(t):
    return t.cpu().numpy().view(np.uint64)


def uniform(primes, lead, n, salt):
    return synth.uniform_mod_primes(synth.rng(0, synth.P_MISC, 300 + salt), primes, lead, n)


def random_key(primes, ell, salt):
    """Uniform residues in the key layout [N][ell][2][P][N] (parity does not need a real key)."""
    return uniform(primes, (N, ell, 2), N, salt)


@pytest.mark.parametrize("primes,beta,ell,M,n_pack", [
    (P2, 54, 1, N + 300, N),
    (P2, 27, 2, 700, 500),
    (P2, 16, 4, 300, N),
    (P1, 12, 3, 1000, 700),
])
def test_pack_matches_oracle(primes, beta, ell, M, n_pack):
    print(f"case: keyswitch P={len(primes)} beta={beta} ell={ell} M={M} n_pack={n_pack}", flush=True)
    r = rl()
    lwe = uniform(primes, (M,), N + 1, M)
    ksk = random_key(primes, ell, beta)
    want = orc.keyswitch_pack(N, primes, beta, ell, lwe, ksk, n_pack)
    G = want.shape[0]
    with r.Context(N, primes, 26, log2_q_out=32) as ctx:
        k = r.KeySwitchKey(ctx, dev(ksk), beta, ell)
        got = r.keyswitch_pack(ctx, k, dev(lwe), n_pack, raw=True)
        sw = r.keyswitch_pack(ctx, k, dev(lwe), n_pack)
        torch.cuda.synchronize()
        assert got.shape == (G, 2, len(primes), N)
        g = host_u64(got)
        assert np.array_equal(g, want), f"{int((g != want).sum())} residues differ"
        s = sw.cpu().numpy().view(np.uint32)
        assert np.array_equal(s, orc.rlwe_modswitch_bits(primes, want, 32))
        k.close()
    with r.Context(N, primes, 26, log2_q_out=26) as ctx:
        k = r.KeySwitchKey(ctx, dev(ksk), beta, ell)
        sw = r.keyswitch_pack(ctx, k, dev(lwe), n_pack)
        torch.cuda.synchronize()
        assert np.array_equal(sw.cpu().numpy().view(np.uint32),
                              orc.rlwe_modswitch_bits(primes, want, 26))
        k.close()


def test_calls_in_a_row_and_edge_cases():
    """A larger call, then a smaller one, on one context and key; count = 0 is a no-op;
    invalid shapes and gadgets are refused."""
    print("case: keyswitch calls in a row, edge cases", flush=True)
    r = rl()
    ksk = random_key(P2, 1, 7)
    a = uniform(P2, (N + 5,), N + 1, 11)
    b = uniform(P2, (3,), N + 1, 12)
    with r.Context(N, P2, 26) as ctx:
        k = r.KeySwitchKey(ctx, dev(ksk), 54, 1)
        ga = r.keyswitch_pack(ctx, k, dev(a), raw=True)
        gb = r.keyswitch_pack(ctx, k, dev(b), raw=True)
        torch.cuda.synchronize()
        assert np.array_equal(host_u64(ga), orc.keyswitch_pack(N, P2, 54, 1, a, ksk))
        assert np.array_equal(host_u64(gb), orc.keyswitch_pack(N, P2, 54, 1, b, ksk))
        dummy = torch.zeros(1, dtype=torch.int64, device="cuda")
        r.ct_keyswitch_pack(ctx.handle, k.handle, dummy, 0, N, dummy)  # no-op
        for n_pack in (0, N + 1):
            with pytest.raises(r.RlweError) as ei:
                r.ct_keyswitch_pack(ctx.handle, k.handle, dummy, 1, n_pack, dummy)
            assert ei.value.code == r.RLWE_ESHAPE
        for beta, ell in ((55, 1), (20, 5), (33, 2), (0, 1)):
            with pytest.raises(r.RlweError) as ei:
                r.KeySwitchKey(ctx, dev(ksk), beta, ell)
            assert ei.value.code == r.RLWE_EPARAM
        k.close()
    with r.Context(8192, (18014398508400641,), 24) as ctx:  # prime, = 1 mod 16384: a valid ring
        with pytest.raises(r.RlweError) as ei:
            r.KeySwitchKey(ctx, dev(ksk[:1]), 12, 3)
        assert ei.value.code == r.RLWE_EPARAM  # packing is offered up to N = 4096


def test_attention_shape_sampled_groups():
    """The launch configuration of the benchmark: 128 tokens x 2048 outputs = 262144 LWE
    ciphertexts into 64 packed ciphertexts (n_pack = N); groups 0 and 63 against the
    oracle, and the switched output of every group against the raw one."""
    print("case: keyswitch attention shape, M=262144, sampled groups", flush=True)
    r = rl()
    T, d_out = 128, 2048
    M = T * d_out
    gen = torch.Generator(device="cuda")
    gen.manual_seed(synth.SEED_BASE + 2000 + 77)
    lwe = torch.empty((M, 2, N + 1), dtype=torch.int64, device="cuda")
    for p, q in enumerate(P2):
        lwe[:, p].random_(0, q, generator=gen)
    ksk = random_key(P2, 1, 13)
    with r.Context(N, P2, 26) as ctx:
        k = r.KeySwitchKey(ctx, dev(ksk), 54, 1)
        raw = r.keyswitch_pack(ctx, k, lwe, N, raw=True)
        sw = r.keyswitch_pack(ctx, k, lwe, N)
        torch.cuda.synchronize()
        assert raw.shape == (64, 2, 2, N)
        for g in (0, 63):
            part = host_u64(lwe[g * N:(g + 1) * N])
            want = orc.keyswitch_pack(N, P2, 54, 1, part, ksk)
            assert np.array_equal(host_u64(raw[g:g + 1]), want), f"group {g}"
        rr = host_u64(raw)
        assert np.array_equal(sw.cpu().numpy().view(np.uint32), orc.rlwe_modswitch_bits(P2, rr, 32))
        k.close()
    del lwe, raw, sw
    torch.cuda.empty_cache()


@pytest.mark.parametrize("method", ["ntt", "toeplitz", "rowpack"])
def test_packed_gpu_products_decrypt(method):
    """Product on the GPU (raw outputs; both mask methods, and packed rows), then packing on
    the GPU with a real key: every slot decrypts under the packing key to W x, the empty
    slots to 0, and the packed ciphertexts equal the oracle's packing of the same LWE
    ciphertexts."""
    print(f"case: keyswitch end to end, {method}", flush=True)
    r = rl()
    d_in, d_out, T, log2_t = 2048, 1500, 2, 26
    case = make_case(N, P2, log2_t, d_out, d_in, T, config=2, salt=31)
    g_a = synth.rng(2, synth.P_MASK, 40)
    g_s = synth.rng(2, synth.P_SECRET, 40)
    g_e = synth.rng(2, synth.P_ERROR, 40)
    A = synth.uniform_mod_primes(g_a, P2, (N, 1), N)
    E = synth.rounded_gaussian(g_e, (N, 1, N))
    S_dst = synth.ternary(g_s, N)
    ksk = orc.ksk_gen(N, P2, 54, 1, case.S, S_dst, A, E)
    flag = {"ntt": r.RLWE_W_NTT, "toeplitz": r.RLWE_W_TOEPLITZ,
            "rowpack": r.RLWE_W_NTT | r.RLWE_W_ROWPACK}[method]
    with r.Context(N, P2, log2_t) as ctx:
        w = r.Weights(ctx, dev(case.W), r.RLWE_W_FWD | flag)
        lwe = r.matmul(ctx, w, dev(case.ct), raw=True)  # (T, d_out, P, N+1)
        k = r.KeySwitchKey(ctx, dev(ksk), 54, 1)
        packed = r.keyswitch_pack(ctx, k, lwe, d_out, raw=True)  # one token per ciphertext
        torch.cuda.synchronize()
        lw = host_u64(lwe)
        pk = host_u64(packed)
        w.close()
        k.close()
    if method == "rowpack":  # two rows per weight polynomial (K = N/2)
        assert np.array_equal(lw, orc.matmul_rowpacked(N, P2, case.W, case.ct))
    else:
        assert np.array_equal(lw, orc.matmul_clear(N, P2, case.W, case.ct))
    assert np.array_equal(pk, orc.keyswitch_pack(N, P2, 54, 1, lw.reshape(-1, 2, N + 1), ksk, d_out))
    y = case.x.astype(np.int64) @ case.W.astype(np.int64).T
    ph = orc.rlwe_decrypt_slots(N, P2, S_dst, pk)
    for t in range(T):
        dec = [orc.decode(v, case.delta) for v in ph[t]]
        assert dec[:d_out] == [int(v) for v in y[t]]
        assert all(v == 0 for v in dec[d_out:])


def test_several_passes_and_graph_replay():
    """More than 64 packed ciphertexts (two passes of the kernels, the second starting at
    group 64) against the oracle on groups 0, 64 and 65; n_pack = 1 and a single LWE
    ciphertext; the call captured in a HIP graph after the workspace is reserved, replayed
    three times with eager work in between, each replay equal to the eager result."""
    print("case: keyswitch two passes, n_pack 1, graph replay", flush=True)
    r = rl()
    M = 65 * N + 100  # 66 packed ciphertexts
    gen = torch.Generator(device="cuda")
    gen.manual_seed(synth.SEED_BASE + 2000 + 78)
    lwe = torch.empty((M, 2, N + 1), dtype=torch.int64, device="cuda")
    for p, q in enumerate(P2):
        lwe[:, p].random_(0, q, generator=gen)
    ksk = random_key(P2, 1, 14)
    with r.Context(N, P2, 26) as ctx:
        k = r.KeySwitchKey(ctx, dev(ksk), 54, 1)
        raw = r.keyswitch_pack(ctx, k, lwe, N, raw=True)
        torch.cuda.synchronize()
        assert raw.shape == (66, 2, 2, N)
        for g in (0, 64, 65):
            part = host_u64(lwe[g * N:(g + 1) * N])
            want = orc.keyswitch_pack(N, P2, 54, 1, part, ksk)
            assert np.array_equal(host_u64(raw[g:g + 1]), want), f"group {g}"
        # one slot per ciphertext, and a single ciphertext
        few = lwe[:3]
        one = r.keyswitch_pack(ctx, k, few, 1, raw=True)
        single = r.keyswitch_pack(ctx, k, lwe[:1], N, raw=True)
        torch.cuda.synchronize()
        fh = host_u64(few)
        assert np.array_equal(host_u64(one), orc.keyswitch_pack(N, P2, 54, 1, fh, ksk, 1))
        assert np.array_equal(host_u64(single), orc.keyswitch_pack(N, P2, 54, 1, fh[:1], ksk, N))
        # graph capture and replay
        small = lwe[:2 * N + 10].clone()
        r.rlwe_workspace_reserve(ctx.handle, r.rlwe_keyswitch_workspace_bytes(
            ctx.handle, k.handle, small.shape[0], N))
        eager = r.keyswitch_pack(ctx, k, small, N)
        torch.cuda.synchronize()
        out = torch.zeros_like(eager)
        s = torch.cuda.Stream()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=s):
            r.keyswitch_pack(ctx, k, small, N, out=out, stream=s)
        for rep in range(3):
            out.zero_()
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, eager), f"replay {rep}"
            r.keyswitch_pack(ctx, k, lwe[:5], N)  # eager work between replays
            torch.cuda.synchronize()
        del graph
        k.close()
    del lwe, raw
    torch.cuda.empty_cache()


@pytest.mark.parametrize("primes,beta,ell", [(P2, 54, 1), (P2, 27, 2), (P1, 12, 3)])
def test_decomposition_near_rounding_ties(primes, beta, ell):
    """Mask coefficients whose scaled value c 2^K / q lies next to a rounding tie
    (x + 1/2), where the GPU's 32.32 fixed-point estimate (at most 7 units of 2^-32 low)
    falls inside its 8-unit window and hands over to exact integer arithmetic: the
    packed outputs equal the oracle's."""
    print(f"case: keyswitch near ties P={len(primes)} beta={beta} ell={ell}", flush=True)
    r = rl()
    q = orc.modulus(primes)
    K = beta * ell
    g = np.random.default_rng(4242 + K)
    vals = []
    for v in g.integers(0, 1 << min(K, 62), size=N, dtype=np.uint64).tolist():
        # c 2^K / q just below v + 1/2 (and the next integer just above it)
        c = ((2 * v + 1) * q) >> (K + 1)
        vals += [c % q, (c + 1) % q]
    # the two coefficients next to the tie of the fraction itself, c 2^K = (q -+ 1)/2 mod q
    inv2k = pow(pow(2, K, q), -1, q)
    vals += [((q - 1) // 2) * inv2k % q, ((q + 1) // 2) * inv2k % q]
    M = 3
    lwe = np.zeros((M, len(primes), N + 1), dtype=np.uint64)
    flat = vals[:M * N]
    for j in range(M):
        for i in range(N):
            c = flat[(j * N + i) % len(flat)]
            lwe[j, :, i] = [c % p for p in primes]
    lwe[:, :, N] = uniform(primes, (M,), 1, K)[:, :, 0]
    lwe[M - 1, :, :2] = np.array([[vals[-2] % p, vals[-1] % p] for p in primes], dtype=np.uint64)
    # these values really are near a tie (one prime: only the last two can be, as c 2^K / q
    # moves by 2^K / q = 2^-18 per unit of c)
    near = 0
    for c in flat[:64] + vals[-2:]:
        frac = (c * (1 << (K + 1))) % (2 * q)  # 2 q frac(c 2^K / q)
        near += abs(frac - q) * (1 << 40) < 2 * q
    assert near >= (2 if len(primes) == 1 else 32)
    ksk = random_key(primes, ell, 90 + K)
    want = orc.keyswitch_pack(N, primes, beta, ell, lwe, ksk, N)
    with r.Context(N, primes, 26) as ctx:
        k = r.KeySwitchKey(ctx, dev(ksk), beta, ell)
        got = r.keyswitch_pack(ctx, k, dev(lwe), N, raw=True)
        torch.cuda.synchronize()
        k.close()
    assert np.array_equal(host_u64(got), want)


@pytest.mark.parametrize("N_,primes,beta,ell,M,n_pack", [
    (2048, synth.PRIMES_2048, 12, 3, 2048 + 300, 2048),
    (2048, synth.PRIMES_2048, 18, 2, 700, 256),
    (256, P2, 54, 1, 600, 256),
    (64, P2, 27, 2, 100, 50),
])
def test_pack_smaller_rings_matches_oracle(N_, primes, beta, ell, M, n_pack):
    """The plain kernels for N below 4096 against the oracle: raw and switched outputs."""
    print(f"case: keyswitch N={N_} P={len(primes)} beta={beta} ell={ell} M={M}", flush=True)
    r = rl()
    g = synth.rng(0, synth.P_MISC, 500 + N_)
    lwe = synth.uniform_mod_primes(g, primes, (M,), N_ + 1)
    ksk = synth.uniform_mod_primes(g, primes, (N_, ell, 2), N_)
    want = orc.keyswitch_pack(N_, primes, beta, ell, lwe, ksk, n_pack)
    with r.Context(N_, primes, 24) as ctx:
        k = r.KeySwitchKey(ctx, dev(ksk), beta, ell)
        got = r.keyswitch_pack(ctx, k, dev(lwe), n_pack, raw=True)
        sw = r.keyswitch_pack(ctx, k, dev(lwe), n_pack)
        torch.cuda.synchronize()
        k.close()
    assert np.array_equal(host_u64(got), want)
    assert np.array_equal(sw.cpu().numpy().view(np.uint32), orc.rlwe_modswitch_bits(primes, want, 32))


def test_config1_products_packed_and_decrypted():
    """The 256 x 256 workload at N = 2048, one prime, t = 2^24, 16 tokens: product on the GPU
    (matrix cores, raw outputs), packing of each token's 256 outputs into one RLWE ciphertext
    with a real key, switch to 2^32: every slot decrypts to W x after the switch, and the
    packed ciphertexts equal the oracle's."""
    print("case: keyswitch config 1 end to end", flush=True)
    r = rl()
    N1, primes, log2_t, beta, ell = 2048, synth.PRIMES_2048, 24, 12, 3
    case = make_case(N1, primes, log2_t, 256, 256, 16, config=1, salt=32)
    g_a = synth.rng(1, synth.P_MASK, 41)
    g_s = synth.rng(1, synth.P_SECRET, 41)
    g_e = synth.rng(1, synth.P_ERROR, 41)
    A = synth.uniform_mod_primes(g_a, primes, (N1, ell), N1)
    E = synth.rounded_gaussian(g_e, (N1, ell, N1))
    S_dst = synth.ternary(g_s, N1)
    ksk = orc.ksk_gen(N1, primes, beta, ell, case.S, S_dst, A, E)
    with r.Context(N1, primes, log2_t) as ctx:
        w = r.Weights(ctx, dev(case.W))
        lwe = r.matmul(ctx, w, dev(case.ct), raw=True)  # (16, 256, 1, N+1)
        k = r.KeySwitchKey(ctx, dev(ksk), beta, ell)
        packed = r.keyswitch_pack(ctx, k, lwe, 256, raw=True)
        switched = r.keyswitch_pack(ctx, k, lwe, 256)
        torch.cuda.synchronize()
        lw = host_u64(lwe)
        pk = host_u64(packed)
        sw = switched.cpu().numpy().view(np.uint32)
        w.close()
        k.close()
    assert np.array_equal(lw, orc.matmul_clear(N1, primes, case.W, case.ct))
    want = orc.keyswitch_pack(N1, primes, beta, ell, lw.reshape(-1, 1, N1 + 1), ksk, 256)
    assert np.array_equal(pk, want)
    assert np.array_equal(sw, orc.rlwe_modswitch_bits(primes, want, 32))
    y = case.x.astype(np.int64) @ case.W.astype(np.int64).T  # (16, 256)
    ph = orc.rlwe_phase_bits(S_dst, sw, 32)
    dec = np.floor_divide(2 * ph + 256, 2 * 256)  # Delta' = 2^32 / 2^24
    assert np.array_equal(dec[:, :256], y)
    assert not dec[:, 256:].any()
