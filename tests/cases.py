"""Seeded encrypted test cases: synthetic draws from ``synth`` encrypted by the oracle."""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from oracle import oracle as orc
from paper_2505_07329_amd import synth


@dataclass
class Case:
    N: int
    primes: tuple
    log2_t: int
    W: np.ndarray      # int8 (d_out, d_in)
    x: np.ndarray      # int8 (T, d_in)
    S: np.ndarray      # int8 (N,)
    E: np.ndarray      # int64 (T, L, N)
    ct: np.ndarray     # uint64 (T, L, 2, P, N)

    @property
    def q(self) -> int:
        return orc.modulus(self.primes)

    @property
    def delta(self) -> int:
        return orc.delta(self.primes, self.log2_t)

    @property
    def L(self) -> int:
        return self.ct.shape[1]

    def errors_flat(self) -> np.ndarray:
        """(T, d_in) error coefficients aligned with x."""
        T = self.x.shape[0]
        return self.E.reshape(T, -1)[:, : self.x.shape[1]]


def make_case(N, primes, log2_t, d_out, d_in, T, config=0, salt=0, W=None, x=None,
              zero_secret=False, zero_error=False, use_ntt=True) -> Case:
    g_w = synth.rng(config, synth.P_WEIGHTS, salt)
    g_x = synth.rng(config, synth.P_ACTS, salt)
    g_a = synth.rng(config, synth.P_MASK, salt)
    g_s = synth.rng(config, synth.P_SECRET, salt)
    g_e = synth.rng(config, synth.P_ERROR, salt)
    if W is None:
        W = synth.int8_uniform(g_w, (d_out, d_in))
    if x is None:
        x = synth.int8_uniform(g_x, (T, d_in))
    L = orc.num_blocks(d_in, N)
    A = synth.uniform_mod_primes(g_a, primes, (T, L), N)
    S = synth.ternary(g_s, N)
    E = synth.rounded_gaussian(g_e, (T, L, N))
    if zero_secret:
        S = np.zeros_like(S)
    if zero_error:
        E = np.zeros_like(E)
    ct = orc.encrypt_tokens(N, primes, log2_t, S, x, A, E, use_ntt=use_ntt)
    return Case(N, tuple(primes), log2_t, np.asarray(W, np.int8), np.asarray(x, np.int8), S, E, ct)


def uniform_ct(N, primes, T, L, config=0, salt=0) -> np.ndarray:
    """Uniformly random residues in the ciphertext layout (T, L, 2, P, N)."""
    g = synth.rng(config, synth.P_MISC, salt)
    return synth.uniform_mod_primes(g, primes, (T, L, 2), N)


def exact_phase_targets(case: Case) -> np.ndarray:
    """Per (t, j): Delta*(W x)_j + (W e)_j as Python ints (the exact LWE phase)."""
    W = case.W.astype(object)
    x = case.x.astype(object)
    e = case.errors_flat().astype(object)
    return case.delta * (x @ W.T) + e @ W.T
