"""Seeded synthetic inputs shared by the CPU oracle tests, the GPU tests and the benchmark.

This module draws random numbers and nothing else: it holds none of the scheme's
arithmetic (no products, no encryption, no reduction beyond drawing a residue
uniformly below a modulus). Every random quantity the scheme consumes — the
weights, the activations, the RLWE mask, the secret key and the error — is drawn
here and handed to whichever side needs it as an explicit input.

Seeds follow ``base + 1000 * config + purpose`` so every workload is reproducible.

Distributions (Sec. 3.1 for the RLWE draws; Sec. 4.2 for the int8 symmetric
quantized operands):
  * weights / activations / gradients: int8 uniform in [-127, 127] (symmetric
    quantization keeps zero-points at 0, so -128 never occurs);
  * mask A: uniform in Z_q, drawn as independent uniform residues per RNS prime
    (the CRT map makes the two descriptions identical);
  * secret S: ternary, i.i.d. uniform over {-1, 0, 1};
  * error E: rounded Gaussian, sigma = 3.2, truncated to |e| <= 19 by resampling.
"""

from __future__ import annotations

import numpy as np

SEED_BASE = 20250507

# Purposes: offsets added to the per-config seed.
P_WEIGHTS = 1
P_ACTS = 2
P_MASK = 3
P_SECRET = 4
P_ERROR = 5
P_GRADS = 6
P_MISC = 7

SIGMA = 3.2
ERROR_BOUND = 19


def rng(config: int, purpose: int, salt: int = 0) -> np.random.Generator:
    """Generator seeded with base + 1000*config + purpose (+ 100000*salt)."""
    return np.random.default_rng(SEED_BASE + 1000 * config + purpose + 100000 * salt)


def int8_uniform(g: np.random.Generator, shape, lo: int = -127, hi: int = 127) -> np.ndarray:
    return g.integers(lo, hi + 1, size=shape, dtype=np.int64).astype(np.int8)


def int8_uniform_device(config: int, purpose: int, salt: int, shape, device):
    """int8 uniform in [-127, 127] drawn on a torch device (large resident weight sets)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(SEED_BASE + 1000 * config + purpose + 100000 * salt)
    return torch.randint(-127, 128, tuple(shape), generator=gen, device=device, dtype=torch.int8)


def uniform_mod_primes(g: np.random.Generator, primes, lead_shape, N: int) -> np.ndarray:
    """Uniform residues, shape ``lead_shape + (P, N)``, entry [..., p, k] in [0, primes[p])."""
    P = len(primes)
    out = np.empty(tuple(lead_shape) + (P, N), dtype=np.uint64)
    for p, q in enumerate(primes):
        out[..., p, :] = g.integers(0, int(q), size=tuple(lead_shape) + (N,), dtype=np.uint64)
    return out


def ternary(g: np.random.Generator, N: int) -> np.ndarray:
    return g.integers(-1, 2, size=N, dtype=np.int64).astype(np.int8)


def rounded_gaussian(g: np.random.Generator, shape, sigma: float = SIGMA,
                     bound: int = ERROR_BOUND) -> np.ndarray:
    """int64 rounded Gaussian draws with |e| <= bound (out-of-range draws are redrawn)."""
    e = np.rint(g.normal(0.0, sigma, size=shape)).astype(np.int64)
    bad = np.abs(e) > bound
    while bad.any():
        e[bad] = np.rint(g.normal(0.0, sigma, size=int(bad.sum()))).astype(np.int64)
        bad = np.abs(e) > bound
    return e


# ---------------------------------------------------------------- workloads
# RLWE parameters of the five workloads: ring degree, RNS primes (largest 54-bit
# primes with q = 1 mod 2N), log2 of the plaintext modulus t.
PRIMES_2048 = (18014398509404161,)
PRIMES_4096 = (18014398509309953, 18014398509293569)

LLAMA_1B_PROJ = {
    # name: (d_in, d_out) of the forward product W x (W is d_out x d_in)
    "q": (2048, 2048),
    "k": (2048, 512),
    "v": (2048, 512),
    "o": (2048, 2048),
    "gate": (2048, 8192),
    "up": (2048, 8192),
    "down": (8192, 2048),
}

WORKLOADS = {
    1: dict(name="plain-256x256-T16-N2048-P1", N=2048, primes=PRIMES_2048, log2_t=24,
            d_in=256, d_out=256, tokens=16),
    2: dict(name="llama1b-attn-2048x2048-T128-N4096-P2", N=4096, primes=PRIMES_4096, log2_t=26,
            d_in=2048, d_out=2048, tokens=128),
    3: dict(name="llama1b-mlp-T2048-N4096-P2", N=4096, primes=PRIMES_4096, log2_t=28,
            tokens=2048),
    4: dict(name="llama1b-layer-batched-N4096-P2", N=4096, primes=PRIMES_4096, log2_t=28),
    5: dict(name="llama1b-serving-N4096-P2", N=4096, primes=PRIMES_4096, log2_t=28),
}
