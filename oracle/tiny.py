"""Pure-Python big-integer version of the scheme for tiny rings (N <= 64).

TEST INFRASTRUCTURE ONLY. It works over Z_q with q the full modulus (no RNS
split, no CRT inside the products), so agreement with the C oracle on tiny
inputs checks the residue-wise C code against an independent route.

Passages: Sec. 3.1 (RLWE encryption), Sec. 3.2 (SampleExtract, ModulusSwitch),
Sec. 4.3 (block split, reversed weights, Eq. (LWEdot), Eq. (pack_rotate)); the
Decomp of KeySwitching is the gadget decomposition of TFHE.
"""

from __future__ import annotations


def negacyclic_mul(a, b, q):
    """a*b in Z_q[X]/(X^N+1), term by term."""
    N = len(a)
    out = [0] * N
    for i in range(N):
        for j in range(N):
            if i + j < N:
                out[i + j] += a[i] * b[j]
            else:
                out[i + j - N] -= a[i] * b[j]
    return [c % q for c in out]


def encrypt(q, t, S, A, E, msg):
    """B = A*S + E + floor(q/t)*msg in R_q."""
    delta = q // t
    AS = negacyclic_mul(A, S, q)
    return [(AS[k] + E[k] + delta * msg[k]) % q for k in range(len(A))]


def sample_extract(A, B, q, h):
    N = len(A)
    a = [A[h - i] % q if i <= h else (-A[N + h - i]) % q for i in range(N)]
    return a, B[h] % q


def matmul_clear(q, N, W, cts):
    """cts[i] = (A_i, B_i) for block i of one token; W rows w_j. Returns [(a, b)]."""
    d_in = len(W[0])
    L = len(cts)
    res = []
    for w in W:
        acc_a = [0] * N
        acc_b = 0
        for i in range(L):
            what = [w[i * N + N - 1 - k] if i * N + N - 1 - k < d_in else 0 for k in range(N)]
            A, B = cts[i]
            CA = negacyclic_mul(A, what, q)
            CB = negacyclic_mul(B, what, q)
            a, b = sample_extract(CA, CB, q, N - 1)
            acc_a = [(x + y) % q for x, y in zip(acc_a, a)]
            acc_b = (acc_b + b) % q
        res.append((acc_a, acc_b))
    return res


def matmul_rowpacked(q, N, W, ct):
    """Multi-row packing for one block (K = len(W[0]) <= N): rows g n_o + rho share the
    polynomial with row rho reversed in slot rho; row j's output is SampleExtract at
    (rho + 1) K - 1. ct = (A, B) of one token. Returns [(a, b)] per row."""
    K = len(W[0])
    n_o = N // K
    A, B = ct
    res = []
    for j, w in enumerate(W):
        g, rho = divmod(j, n_o)
        wg = [0] * N
        for r in range(n_o):
            if g * n_o + r < len(W):
                for k in range(K):
                    wg[r * K + K - 1 - k] = W[g * n_o + r][k]
        CA = negacyclic_mul(A, wg, q)
        CB = negacyclic_mul(B, wg, q)
        res.append(sample_extract(CA, CB, q, (rho + 1) * K - 1))
    return res


def modswitch(c, q, bits=32):
    """round(c 2^bits / q) mod 2^bits, half up."""
    return ((c * (1 << (bits + 1)) + q) // (2 * q)) % (1 << bits)


def lwe_phase(a, b, S, q):
    ph = (b - sum(x * s for x, s in zip(a, S))) % q
    return ph - q if ph > q // 2 else ph


def decomp(c, q, beta, ell):
    """TFHE gadget decomposition of c mod q: signed base-2^beta digits, most significant first,
    of round(c 2^(beta ell) / q) mod 2^(beta ell)."""
    K = beta * ell
    at = ((c % q) * (1 << (K + 1)) + q) // (2 * q) % (1 << K)
    d = []
    for k in range(ell):  # least significant first, balanced
        v = at % (1 << beta)
        at //= 1 << beta
        if v >= 1 << (beta - 1):
            v -= 1 << beta
            at += 1
        d.append(v)
    return d[::-1]


def gadget(q, beta, ell):
    return [(q + (1 << (beta * (m + 1) - 1))) >> (beta * (m + 1)) for m in range(ell)]


def keyswitch(a, b, ksk, q, beta, ell):
    """KeySwitching(a, b) = (0, b) - sum_i sum_m Decomp_m(a_i) KSK[i][m], KSK[i][m] = (A, B)."""
    N = len(a)
    A = [0] * N
    B = [b % q] + [0] * (N - 1)
    for i in range(N):
        for m, d in enumerate(decomp(a[i], q, beta, ell)):
            KA, KB = ksk[i][m]
            A = [(x - d * y) % q for x, y in zip(A, KA)]
            B = [(x - d * y) % q for x, y in zip(B, KB)]
    return A, B


def rotate(P, s, q):
    """P(X) X^s in Z_q[X]/(X^N + 1)."""
    N = len(P)
    X = [0] * N
    X[s] = 1
    return negacyclic_mul(P, X, q)


def keyswitch_pack(lwes, ksk, q, beta, ell):
    """Eq. (pack_rotate) before the switch: sum_s Rotate(KeySwitching(lwes[s]), s)."""
    N = len(lwes[0][0])
    A = [0] * N
    B = [0] * N
    for s, (a, b) in enumerate(lwes):
        KA, KB = keyswitch(a, b, ksk, q, beta, ell)
        A = [(x + y) % q for x, y in zip(A, rotate(KA, s, q))]
        B = [(x + y) % q for x, y in zip(B, rotate(KB, s, q))]
    return A, B
