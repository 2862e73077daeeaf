"""Python access to the CPU oracle (oracle/rlwe_oracle.c) and client-side helpers.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark. The product path never imports this module.

The client side of the protocol lives here too (Sec. 4.3): splitting an int8
activation vector into L = ceil(d_in / N) zero-padded blocks, encrypting every
block (Sec. 3.1) and decrypting returned LWE ciphertexts. Random draws (mask,
secret, error) are inputs produced by ``paper_2505_07329_amd.synth``.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Iterable, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rlwe_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i8p = ctypes.POINTER(ctypes.c_int8)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP); returns the library path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        L = _lib
        L.orc_mulmod.restype = ctypes.c_uint64
        L.orc_mulmod.argtypes = [ctypes.c_uint64] * 3
        L.orc_powmod.restype = ctypes.c_uint64
        L.orc_powmod.argtypes = [ctypes.c_uint64] * 3
        L.orc_find_psi.restype = ctypes.c_uint64
        L.orc_find_psi.argtypes = [ctypes.c_uint32, ctypes.c_uint64]
        L.orc_poly_mul_schoolbook.argtypes = [_u64p, _u64p, ctypes.c_uint32, ctypes.c_uint64, _u64p]
        L.orc_poly_mul_ntt.argtypes = [_u64p, _u64p, ctypes.c_uint32, ctypes.c_uint64,
                                       ctypes.c_uint64, _u64p]
        L.orc_delta.argtypes = [ctypes.c_uint32, _u64p, ctypes.c_uint32, _u64p, _u64p]
        L.orc_encrypt.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u64p, ctypes.c_uint32, _i8p,
                                  ctypes.c_size_t, _u64p, _i64p, _i64p, ctypes.c_int, _u64p]
        L.orc_rlwe_phase.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u64p, _i8p,
                                     ctypes.c_size_t, _u64p, _u64p, _u64p]
        L.orc_sample_extract.argtypes = [_u64p, _u64p, ctypes.c_uint32, ctypes.c_uint64,
                                         ctypes.c_uint32, _u64p, _u64p]
        L.orc_matmul_clear.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u64p, ctypes.c_uint32,
                                       ctypes.c_uint32, _i8p, ctypes.c_uint32, _u64p,
                                       ctypes.c_size_t, _u32p, ctypes.c_int, _u64p]
        L.orc_modswitch.argtypes = [ctypes.c_uint32, _u64p, ctypes.c_size_t, ctypes.c_uint32,
                                    _u64p, _u32p]
        L.orc_modswitch_bits.argtypes = [ctypes.c_uint32, _u64p, ctypes.c_size_t, ctypes.c_uint32,
                                         _u64p, ctypes.c_uint32, _u32p]
        L.orc_splitmix64_at.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_splitmix64_at.restype = ctypes.c_uint64
        L.orc_mask_coeff.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.c_uint32, ctypes.c_uint64]
        L.orc_mask_coeff.restype = ctypes.c_uint64
        L.orc_expand_mask.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, _u64p, _u64p]
        L.orc_crt.argtypes = [ctypes.c_uint32, _u64p, _u64p, _u64p, _u64p]
        L.orc_lwe_phase.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u64p, _i8p,
                                    ctypes.c_size_t, _u64p, _u64p]
        L.orc_lwe_phase_u32.argtypes = [ctypes.c_uint32, _i8p, ctypes.c_size_t, _u32p, _i64p]
        L.orc_decomp.argtypes = [ctypes.c_uint32, _u64p, ctypes.c_size_t, _u64p, ctypes.c_uint32,
                                 ctypes.c_uint32, _i64p]
        L.orc_gadget.argtypes = [ctypes.c_uint32, _u64p, ctypes.c_uint32, ctypes.c_uint32, _u64p]
        L.orc_ksk_gen.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u64p, ctypes.c_uint32,
                                  ctypes.c_uint32, _i8p, _i8p, _u64p, _i64p, _u64p]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_keyswitch_pack.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u64p, ctypes.c_uint32,
                                         ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _u64p,
                                         _u64p, ctypes.c_int, _u64p]
    return _lib


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (timing only)."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def _primes(primes: Sequence[int]) -> np.ndarray:
    return np.ascontiguousarray(np.array([int(p) for p in primes], dtype=np.uint64))


# ------------------------------------------------------------------ scalars

def modulus(primes: Sequence[int]) -> int:
    q = 1
    for p in primes:
        q *= int(p)
    return q


def delta(primes: Sequence[int], log2_t: int) -> int:
    """Delta = floor(q / t) (Sec. 3.1 writes q/p; q is odd so the floor is taken)."""
    pr = _primes(primes)
    hi = ctypes.c_uint64()
    lo = ctypes.c_uint64()
    lib().orc_delta(len(pr), _p(pr, _u64p), log2_t, ctypes.byref(hi), ctypes.byref(lo))
    return (hi.value << 64) | lo.value


def find_psi(N: int, q: int) -> int:
    return int(lib().orc_find_psi(N, int(q)))


def crt(primes: Sequence[int], residues: Sequence[int]) -> int:
    pr = _primes(primes)
    r = np.ascontiguousarray(np.array([int(x) for x in residues], dtype=np.uint64))
    hi = ctypes.c_uint64()
    lo = ctypes.c_uint64()
    lib().orc_crt(len(pr), _p(pr, _u64p), _p(r, _u64p), ctypes.byref(hi), ctypes.byref(lo))
    return (hi.value << 64) | lo.value


def centered(c: int, q: int) -> int:
    c %= q
    return c - q if c > q // 2 else c


# ------------------------------------------------------------------ ring

def poly_mul_schoolbook(a: np.ndarray, b: np.ndarray, q: int) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.empty_like(a)
    lib().orc_poly_mul_schoolbook(_p(a, _u64p), _p(b, _u64p), a.size, int(q), _p(out, _u64p))
    return out


def poly_mul_ntt(a: np.ndarray, b: np.ndarray, q: int, psi: int | None = None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    if psi is None:
        psi = find_psi(a.size, q)
    out = np.empty_like(a)
    lib().orc_poly_mul_ntt(_p(a, _u64p), _p(b, _u64p), a.size, int(q), int(psi), _p(out, _u64p))
    return out


def sample_extract(A: np.ndarray, B: np.ndarray, q: int, h: int):
    A = np.ascontiguousarray(A, dtype=np.uint64)
    B = np.ascontiguousarray(B, dtype=np.uint64)
    a = np.empty_like(A)
    b = ctypes.c_uint64()
    lib().orc_sample_extract(_p(A, _u64p), _p(B, _u64p), A.size, int(q), h, _p(a, _u64p),
                             ctypes.byref(b))
    return a, b.value


# ------------------------------------------------------------------ client side

def num_blocks(d_in: int, N: int) -> int:
    return (d_in + N - 1) // N


def split_blocks(x: np.ndarray, N: int) -> np.ndarray:
    """x: (T, d_in) int -> (T, L, N) int64, the last block zero-padded (Sec. 4.3)."""
    x = np.asarray(x)
    T, d_in = x.shape
    L = num_blocks(d_in, N)
    out = np.zeros((T, L * N), dtype=np.int64)
    out[:, :d_in] = x
    return out.reshape(T, L, N)


def encrypt(N: int, primes, log2_t: int, S: np.ndarray, A: np.ndarray, E: np.ndarray,
            msg: np.ndarray, use_ntt: bool = True) -> np.ndarray:
    """B for each (A, E, msg): A (..., P, N) u64, E (..., N), msg (..., N) -> B (..., P, N)."""
    pr = _primes(primes)
    P = len(pr)
    lead = A.shape[:-2]
    count = int(np.prod(lead)) if lead else 1
    A_ = np.ascontiguousarray(A.reshape(count, P, N), dtype=np.uint64)
    E_ = np.ascontiguousarray(E.reshape(count, N), dtype=np.int64)
    M_ = np.ascontiguousarray(msg.reshape(count, N), dtype=np.int64)
    S_ = np.ascontiguousarray(S, dtype=np.int8)
    B = np.empty_like(A_)
    lib().orc_encrypt(N, P, _p(pr, _u64p), log2_t, _p(S_, _i8p), count, _p(A_, _u64p),
                      _p(E_, _i64p), _p(M_, _i64p), int(use_ntt), _p(B, _u64p))
    return B.reshape(A.shape)


def encrypt_tokens(N: int, primes, log2_t: int, S: np.ndarray, x: np.ndarray, A: np.ndarray,
                   E: np.ndarray, use_ntt: bool = True) -> np.ndarray:
    """Encrypt T int8 vectors block by block.

    x (T, d_in), A (T, L, P, N) uniform residues, E (T, L, N) errors
    -> ct (T, L, 2, P, N) with ct[t, i, 0] = A, ct[t, i, 1] = B.
    """
    blocks = split_blocks(x, N)
    B = encrypt(N, primes, log2_t, S, A, E, blocks, use_ntt)
    T, L = blocks.shape[:2]
    ct = np.empty((T, L, 2, len(primes), N), dtype=np.uint64)
    ct[:, :, 0] = A
    ct[:, :, 1] = B
    return ct


def splitmix64_at(seed: int, ctr: int) -> int:
    return int(lib().orc_splitmix64_at(seed, ctr))


def mask_coeff(seed: int, N: int, p: int, n: int, q: int) -> int:
    return int(lib().orc_mask_coeff(seed, N, p, n, q))


def expand_masks(seeds: np.ndarray, N: int, primes) -> np.ndarray:
    """Masks of seeded ciphertexts (Sec. 3.1): seeds (...) u64 -> A (..., P, N) u64."""
    pr = _primes(primes)
    sd = np.asarray(seeds, dtype=np.uint64)
    out = np.empty(sd.shape + (len(pr), N), dtype=np.uint64)
    flat = out.reshape(-1, len(pr) * N)
    for c, s_ in enumerate(sd.reshape(-1).tolist()):
        row = np.empty(len(pr) * N, dtype=np.uint64)
        lib().orc_expand_mask(s_, N, len(pr), _p(pr, _u64p), _p(row, _u64p))
        flat[c] = row
    return out


def seeded_layout(ct: np.ndarray, seeds: np.ndarray) -> np.ndarray:
    """The seeded input layout of ciphertexts whose masks are expand_masks(seeds):
    ct (T, L, 2, P, N) -> (T, L, P N + 2) u64 = [seed, 0, B residues]; about half the
    bytes of the full layout (Sec. 4.4: a seed and the body are sent)."""
    T, L, _, P, N = ct.shape
    out = np.zeros((T, L, P * N + 2), dtype=np.uint64)
    out[:, :, 0] = np.asarray(seeds, dtype=np.uint64)
    out[:, :, 2:] = ct[:, :, 1].reshape(T, L, P * N)
    return out


def rlwe_phase(N: int, primes, S: np.ndarray, A: np.ndarray, B: np.ndarray) -> np.ndarray:
    pr = _primes(primes)
    P = len(pr)
    count = int(np.prod(A.shape[:-2])) if A.ndim > 2 else 1
    A_ = np.ascontiguousarray(A.reshape(count, P, N), dtype=np.uint64)
    B_ = np.ascontiguousarray(B.reshape(count, P, N), dtype=np.uint64)
    out = np.empty_like(A_)
    S_ = np.ascontiguousarray(S, dtype=np.int8)
    lib().orc_rlwe_phase(N, P, _p(pr, _u64p), _p(S_, _i8p), count, _p(A_, _u64p),
                         _p(B_, _u64p), _p(out, _u64p))
    return out.reshape(A.shape)


# ------------------------------------------------------------------ server product

def all_pairs(T: int, d_out: int) -> np.ndarray:
    t, j = np.meshgrid(np.arange(T), np.arange(d_out), indexing="ij")
    return np.stack([t.ravel(), j.ravel()], axis=1).astype(np.uint32)


def matmul_clear(N: int, primes, W: np.ndarray, ct: np.ndarray,
                 pairs: np.ndarray | None = None, mode: int = 1) -> np.ndarray:
    """LWE(x . w_j) for each (t, j) pair, Eq. (LWEdot): uint64 (npairs, P, N+1).

    W int8 (d_out, d_in); ct (T, L, 2, P, N); mode 0 schoolbook, 1 NTT.
    With pairs=None every (t, j) is computed and the result is (T, d_out, P, N+1).
    """
    pr = _primes(primes)
    P = len(pr)
    W_ = np.ascontiguousarray(W, dtype=np.int8)
    d_out, d_in = W_.shape
    T, L = ct.shape[:2]
    assert ct.shape == (T, L, 2, P, N) and L == num_blocks(d_in, N)
    full = pairs is None
    if full:
        pairs = all_pairs(T, d_out)
    pairs_ = np.ascontiguousarray(pairs, dtype=np.uint32)
    ct_ = np.ascontiguousarray(ct, dtype=np.uint64)
    out = np.empty((len(pairs_), P, N + 1), dtype=np.uint64)
    lib().orc_matmul_clear(N, P, _p(pr, _u64p), d_out, d_in, _p(W_, _i8p), T, _p(ct_, _u64p),
                           len(pairs_), _p(pairs_, _u32p), int(mode), _p(out, _u64p))
    if full:
        out = out.reshape(T, d_out, P, N + 1)
    return out


def rows_per_product(d_in: int, N: int) -> int:
    """Rows sharing one weight polynomial under multi-row packing: floor(N / d_in)."""
    if not 1 <= d_in <= N:
        raise ValueError("multi-row packing needs 1 <= d_in <= N")
    return N // d_in


def rowpack_weights(W: np.ndarray, N: int) -> np.ndarray:
    """Multi-row packing of the weights (the coefficient packing of Sec. 4.3.1, as in Cheetah):
    the n_o = floor(N / K) rows g n_o + rho (rho < n_o) of group g share one polynomial,
    w_g[rho K + K - 1 - k] = W[g n_o + rho, k] (each row reversed in its own slot of K
    coefficients; zero past the last row). W (d_out, K) -> (ceil(d_out / n_o), N) int64."""
    W = np.asarray(W, dtype=np.int64)
    d_out, K = W.shape
    n_o = rows_per_product(K, N)
    G = -(-d_out // n_o)
    out = np.zeros((G, N), dtype=np.int64)
    for j in range(d_out):
        g, rho = divmod(j, n_o)
        out[g, rho * K:(rho + 1) * K] = W[j, ::-1]
    return out


def matmul_rowpacked(N: int, primes, W: np.ndarray, ct: np.ndarray) -> np.ndarray:
    """LWE(x . w_j) under multi-row packing (d_in = K <= N, one input block): the output of row
    j = g n_o + rho is SampleExtract at h = (rho + 1) K - 1 of RLWE(x_hat) . w_g (Sec. 3.2),
    whose message coefficient h is sum_k x[k] w_j[k]. W int8 (d_out, K); ct (T, 1, 2, P, N)
    -> uint64 (T, d_out, P, N+1). Products by the oracle's negacyclic NTT."""
    pr = _primes(primes)
    P = len(pr)
    W = np.asarray(W)
    d_out, K = W.shape
    T = ct.shape[0]
    assert ct.shape == (T, 1, 2, P, N)
    n_o = rows_per_product(K, N)
    Wg = rowpack_weights(W, N)
    out = np.empty((T, d_out, P, N + 1), dtype=np.uint64)
    for p, q in enumerate(pr.tolist()):
        psi = find_psi(N, q)
        wq = [np.ascontiguousarray(w % q, dtype=np.uint64) for w in Wg]
        for t in range(T):
            A, B = ct[t, 0, 0, p], ct[t, 0, 1, p]
            for g, w in enumerate(wq):
                CA = poly_mul_ntt(A, w, q, psi)
                CB = poly_mul_ntt(B, w, q, psi)
                for rho in range(n_o):
                    j = g * n_o + rho
                    if j >= d_out:
                        break
                    a, b = sample_extract(CA, CB, q, (rho + 1) * K - 1)
                    out[t, j, p, :N] = a
                    out[t, j, p, N] = b
    return out


def modswitch(primes, raw: np.ndarray) -> np.ndarray:
    """round(c 2^32 / q) mod 2^32 of CRT(raw[..., p, n]): (..., P, len) -> (..., len) u32."""
    pr = _primes(primes)
    P = len(pr)
    ln = raw.shape[-1]
    lead = raw.shape[:-2]
    count = int(np.prod(lead)) if lead else 1
    r = np.ascontiguousarray(raw.reshape(count, P, ln), dtype=np.uint64)
    out = np.empty((count, ln), dtype=np.uint32)
    lib().orc_modswitch(P, _p(pr, _u64p), count, ln, _p(r, _u64p), _p(out, _u32p))
    return out.reshape(tuple(lead) + (ln,))


def modswitch_bits(primes, raw: np.ndarray, bits: int) -> np.ndarray:
    """round(c 2^bits / q) mod 2^bits of CRT(raw[..., p, n]), 1 <= bits <= 32, by binary long
    division (Sec. 3.2, ModulusSwitch to q_out = 2^bits): (..., P, len) -> (..., len) u32."""
    if not 1 <= bits <= 32:
        raise ValueError("bits must lie in [1, 32]")
    pr = _primes(primes)
    P = len(pr)
    ln = raw.shape[-1]
    lead = raw.shape[:-2]
    count = int(np.prod(lead)) if lead else 1
    r = np.ascontiguousarray(raw.reshape(count, P, ln), dtype=np.uint64)
    out = np.empty((count, ln), dtype=np.uint32)
    lib().orc_modswitch_bits(P, _p(pr, _u64p), count, ln, _p(r, _u64p), bits, _p(out, _u32p))
    return out.reshape(tuple(lead) + (ln,))


def packed_words(length: int, bits: int) -> int:
    """32-bit words of one ciphertext of `length` coefficients packed at `bits` bits each."""
    return (length * bits + 31) // 32


def pack_bits(values: np.ndarray, bits: int) -> np.ndarray:
    """Bit-pack the switched coefficients of each ciphertext (Sec. 4.5: the switched output
    is returned packed into a bit-vector): values (..., len) u32 below 2^bits -> (...,
    packed_words(len, bits)) u32. Coefficient i of a ciphertext occupies stream bits
    [i bits, (i + 1) bits), least significant first; stream bit b is bit b mod 32 of word
    b // 32; unused high bits of the last word are zero. Written with Python integers."""
    v = np.asarray(values, dtype=np.uint32)
    if v.size and int(v.max()) >> bits:
        raise ValueError("a coefficient does not fit in the given bits")
    ln = v.shape[-1]
    lead = v.shape[:-1]
    flat = v.reshape(-1, ln)
    nw = packed_words(ln, bits)
    out = np.empty((flat.shape[0], nw), dtype=np.uint32)
    for c in range(flat.shape[0]):
        acc = 0
        for i, x in enumerate(flat[c].tolist()):
            acc |= x << (i * bits)
        out[c] = [(acc >> (32 * w)) & 0xFFFFFFFF for w in range(nw)]
    return out.reshape(tuple(lead) + (nw,))


def unpack_bits(words: np.ndarray, bits: int, length: int) -> np.ndarray:
    """Inverse of pack_bits: (..., packed_words(length, bits)) u32 -> (..., length) u32."""
    w = np.asarray(words, dtype=np.uint32)
    lead = w.shape[:-1]
    flat = w.reshape(-1, w.shape[-1])
    out = np.empty((flat.shape[0], length), dtype=np.uint32)
    mask = (1 << bits) - 1
    for c in range(flat.shape[0]):
        acc = 0
        for i, x in enumerate(flat[c].tolist()):
            acc |= x << (32 * i)
        out[c] = [(acc >> (i * bits)) & mask for i in range(length)]
    return out.reshape(tuple(lead) + (length,))


def lwe_phase(N: int, primes, S: np.ndarray, lwe: np.ndarray) -> list[int]:
    """Centred phase b - <a, S> mod q of LWE ciphertexts (..., P, N+1), as Python ints."""
    pr = _primes(primes)
    P = len(pr)
    count = int(np.prod(lwe.shape[:-2])) if lwe.ndim > 2 else 1
    c = np.ascontiguousarray(lwe.reshape(count, P, N + 1), dtype=np.uint64)
    out = np.empty((count, P), dtype=np.uint64)
    S_ = np.ascontiguousarray(S, dtype=np.int8)
    lib().orc_lwe_phase(N, P, _p(pr, _u64p), _p(S_, _i8p), count, _p(c, _u64p), _p(out, _u64p))
    q = modulus(primes)
    return [centered(crt(primes, out[i]), q) for i in range(count)]


def lwe_phase_u32(N: int, S: np.ndarray, lwe: np.ndarray) -> np.ndarray:
    """Centred phase modulo 2^32 of switched LWE ciphertexts (..., N+1): int64 (...)."""
    count = int(np.prod(lwe.shape[:-1])) if lwe.ndim > 1 else 1
    c = np.ascontiguousarray(lwe.reshape(count, N + 1), dtype=np.uint32)
    out = np.empty(count, dtype=np.int64)
    S_ = np.ascontiguousarray(S, dtype=np.int8)
    lib().orc_lwe_phase_u32(N, _p(S_, _i8p), count, _p(c, _u32p), _p(out, _i64p))
    return out.reshape(lwe.shape[:-1])


def lwe_phase_bits(N: int, S: np.ndarray, lwe: np.ndarray, bits: int) -> np.ndarray:
    """Centred phase modulo 2^bits of LWE ciphertexts switched to 2^bits (..., N+1): int64."""
    ph = lwe_phase_u32(N, S, lwe).astype(np.int64) % (1 << bits)
    return np.where(ph >= (1 << (bits - 1)), ph - (1 << bits), ph)


def decode(phase: int, delta_: int) -> int:
    """Round a centred phase to the nearest multiple of Delta: the decrypted message."""
    return (2 * phase + delta_) // (2 * delta_)


# ------------------------------------------------------------------ KeySwitch packing

def check_gadget(primes, beta: int, ell: int) -> None:
    """Decomposition parameters the oracle accepts: K = beta ell <= 64 rounding bits, at most
    8 levels, and signed digits below every prime (2^(beta-1) < q_p)."""
    if not (1 <= beta <= 54 and 1 <= ell <= 8 and beta * ell <= 64):
        raise ValueError("need 1 <= beta <= 54, 1 <= ell <= 8, beta * ell <= 64")
    if any((1 << (beta - 1)) >= int(p) for p in primes):
        raise ValueError("digits must lie below every prime")


def decomp(primes, residues: np.ndarray, beta: int, ell: int) -> np.ndarray:
    """Gadget decomposition of TFHE (Decomp of KeySwitching, Sec. 3.2) of every coefficient
    given by its residues: (..., P) u64 -> (..., ell) int64 signed base-2^beta digits of
    round(c 2^K / q) mod 2^K, K = beta ell, most significant first."""
    check_gadget(primes, beta, ell)
    pr = _primes(primes)
    P = len(pr)
    r = np.ascontiguousarray(residues, dtype=np.uint64)
    assert r.shape[-1] == P
    lead = r.shape[:-1]
    count = int(np.prod(lead)) if lead else 1
    out = np.empty((count, ell), dtype=np.int64)
    lib().orc_decomp(P, _p(pr, _u64p), count, _p(r.reshape(count, P), _u64p), beta, ell,
                     _p(out, _i64p))
    return out.reshape(tuple(lead) + (ell,))


def gadget(primes, beta: int, ell: int) -> np.ndarray:
    """Residues of the gadget values g_m = round(q / 2^(beta (m + 1))): (ell, P) u64."""
    check_gadget(primes, beta, ell)
    pr = _primes(primes)
    out = np.empty((ell, len(pr)), dtype=np.uint64)
    lib().orc_gadget(len(pr), _p(pr, _u64p), beta, ell, _p(out, _u64p))
    return out


def ksk_gen(N: int, primes, beta: int, ell: int, S_src: np.ndarray, S_dst: np.ndarray,
            A: np.ndarray, E: np.ndarray) -> np.ndarray:
    """Key-switching key KSK_{i,m} = RLWE_{S_dst}(S_src[i] g_m) (message in the constant
    coefficient; Sec. 3.2). A (N, ell, P, N) uniform residues, E (N, ell, N) errors ->
    (N, ell, 2, P, N) u64: A, then B = A S_dst + E + S_src[i] g_m."""
    check_gadget(primes, beta, ell)
    pr = _primes(primes)
    P = len(pr)
    A_ = np.ascontiguousarray(A, dtype=np.uint64)
    E_ = np.ascontiguousarray(E, dtype=np.int64)
    assert A_.shape == (N, ell, P, N) and E_.shape == (N, ell, N)
    out = np.empty((N, ell, 2, P, N), dtype=np.uint64)
    Ss = np.ascontiguousarray(S_src, dtype=np.int8)
    Sd = np.ascontiguousarray(S_dst, dtype=np.int8)
    lib().orc_ksk_gen(N, P, _p(pr, _u64p), beta, ell, _p(Ss, _i8p), _p(Sd, _i8p), _p(A_, _u64p),
                      _p(E_, _i64p), _p(out, _u64p))
    return out


def packed_count(M: int, n_pack: int) -> int:
    """RLWE ciphertexts that M LWE ciphertexts fill at n_pack slots each."""
    return -(-M // n_pack)


def keyswitch_pack(N: int, primes, beta: int, ell: int, lwe: np.ndarray, ksk: np.ndarray,
                   n_pack: int | None = None, mode: int = 1) -> np.ndarray:
    """Eq. (pack_rotate) without the final switch: LWE ciphertexts (M, P, N+1) -> packed RLWE
    ciphertexts (ceil(M / n_pack), 2, P, N) u64, LWE g n_pack + s rotated into slot s of
    output g after KeySwitching. mode 0: the definition, one LWE at a time (tiny rings);
    mode 1: the same sums regrouped by input coefficient, products by NTT."""
    check_gadget(primes, beta, ell)
    pr = _primes(primes)
    P = len(pr)
    n_pack = N if n_pack is None else int(n_pack)
    if not 1 <= n_pack <= N:
        raise ValueError("n_pack must lie in [1, N]")
    lw = np.ascontiguousarray(lwe, dtype=np.uint64).reshape(-1, P, N + 1)
    M = lw.shape[0]
    k = np.ascontiguousarray(ksk, dtype=np.uint64)
    assert k.shape == (N, ell, 2, P, N)
    out = np.empty((packed_count(M, n_pack), 2, P, N), dtype=np.uint64)
    lib().orc_keyswitch_pack(N, P, _p(pr, _u64p), beta, ell, M, n_pack, _p(lw, _u64p),
                             _p(k, _u64p), int(mode), _p(out, _u64p))
    return out


def rlwe_modswitch_bits(primes, rlwe: np.ndarray, bits: int) -> np.ndarray:
    """ModulusSwitch of packed RLWE ciphertexts (G, 2, P, N) to 2^bits, coefficient by
    coefficient (Eq. (pack_rotate)): -> (G, 2, N) u32."""
    G, two, P, N = rlwe.shape
    return modswitch_bits(primes, np.ascontiguousarray(rlwe), bits).reshape(G, two, N)


def rlwe_decrypt_slots(N: int, primes, S: np.ndarray, rlwe: np.ndarray) -> list[list[int]]:
    """Centred phase B - A S mod q of packed RLWE ciphertexts (G, 2, P, N), per coefficient,
    as Python ints: [G][N]."""
    G = rlwe.shape[0]
    ph = rlwe_phase(N, primes, S, rlwe[:, 0], rlwe[:, 1])  # (G, P, N)
    q = modulus(primes)
    return [[centered(crt(primes, ph[g, :, n]), q) for n in range(N)] for g in range(G)]


def rlwe_phase_bits(S: np.ndarray, rlwe: np.ndarray, bits: int) -> np.ndarray:
    """Centred phase B - A S mod 2^bits of switched RLWE ciphertexts (G, 2, N) u32: (G, N)."""
    Sv = np.asarray(S, dtype=np.int64)
    G, _, N = rlwe.shape
    mod = 1 << bits
    out = np.empty((G, N), dtype=np.int64)
    for g in range(G):
        A = rlwe[g, 0].astype(np.int64)
        B = rlwe[g, 1].astype(np.int64)
        # negacyclic product A S modulo 2^bits (S ternary, |terms| < N 2^bits < 2^63)
        AS = np.zeros(N, dtype=np.int64)
        for k in np.nonzero(Sv)[0]:
            sh = np.roll(A, int(k))
            sh[:k] = -sh[:k]
            AS += sh * Sv[k]
        ph = (B - AS) % mod
        out[g] = np.where(ph >= mod // 2, ph - mod, ph)
    return out
