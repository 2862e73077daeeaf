// Gadget rounding of a coefficient given by its RNS residues: the first step of
// Decomp in KeySwitching (Sec. 3.2), a~ = round(c 2^K / q) mod 2^K, K <= 64. Used by
// the digit kernel of KeySwitch packing and by the product kernel's rounded output.
#pragma once
#include "rlwe_internal.hpp"

namespace rlwe {

typedef const __attribute__((address_space(4))) KsRound* KrPtr;  // in the kernarg segment

// a~ = round(c 2^K / q) mod 2^K for the coefficient with residues c0 (prime 0) and
// c1 (prime 1, NP = 2); residues need not be reduced (any c_p < 2^64 gives the
// same a~: adding q_p to c_p adds inv_p 2^K, a multiple of 2^K).
//
// With y_p = c_p inv_p mod q_p (inv_p = (q/q_p)^-1 mod q_p, 1 for one prime),
// c 2^K / q = sum_p y_p 2^K / q_p - kappa 2^K, and y_p 2^K / q_p is congruent mod 2^K
// to c_p inv_p 2^K / q_p = c_p f_p + c_p g_p / q_p with f_p = floor(inv_p 2^K / q_p)
// and g_p = inv_p 2^K mod q_p. So a~ is the rounding of sum_p (c_p f_p + c_p g_p / q_p)
// taken mod 2^K.

// Exact route: each prime contributes the integer c_p f_p + floor(c_p g_p / q_p) (one
// Shoup product) and the fraction rem_p / q_p, rem_p = c_p g_p mod q_p; the fractions'
// sum (in [0, P)) is compared with 1/2 and 3/2 in 128-bit integers (no tie for odd q).
template <int NP>
__device__ __noinline__ uint64_t round_exact(KrPtr a, uint64_t c0, uint64_t c1) {
  const uint64_t cs[2] = {c0, c1};
  uint64_t rem[NP];
  uint64_t at = 0;
#pragma unroll
  for (int r = 0; r < NP; ++r) {
    const uint64_t p = a->q[r];
    const uint64_t c = cs[r];
    const uint64_t qh = __umul64hi(c, a->g_shoup[r]);  // floor(c g / q_p) or 1 less
    uint64_t rr = c * a->g[r] - qh * p;                 // in [0, 2 q_p)
    uint64_t u = c * a->f[r] + qh;
    if (rr >= p) {
      rr -= p;
      ++u;
    }
    rem[r] = rr;
    at += u;
  }
  if (NP == 1) return at + (2 * rem[0] >= a->q[0] ? 1u : 0u);
  const u128 Q = make_u128(a->Q_hi, a->Q_lo);
  const u128 F = 2 * ((u128)rem[0] * a->q[NP - 1] + (u128)rem[NP - 1] * a->q[0]);
  return at + (F >= Q ? 1u : 0u) + (F >= 3 * Q ? 1u : 0u);
}

// Fixed-point route, 32 fraction bits: c_p g_p / q_p = c_p G_p / 2^96 with
// G_p = floor(g_p 2^96 / q_p) (96 bits), from the partial products of c_p G_p at and
// above bit 64 (c0 G0 and the low halves of c0 G1, c1 G0 dropped). Per prime the
// estimate is below the exact value by less than 3 units of 2^-32 from the dropped terms
// plus c_p / 2^64 < 1 unit from G_p's truncation, never above; the deficit of the sum is
// an integer number of units below 4 P, so at most 7 for any c_p < 2^64 (at most 6 for
// residues below 2^54, as callers pass them). Its rounding is therefore the exact one
// unless the estimate lies within 8 units below a rounding boundary: then `near` is set
// and the caller takes the exact route. Every sum below is exact mod 2^64 for any
// c_p < 2^64 (t stays below 2^64, the carry of s is kept, u and v are 64-bit products);
// the magnitudes noted are those of reduced residues.
template <int NP>
__device__ __forceinline__ uint64_t round_fast(KrPtr a, uint64_t c0, uint64_t c1, bool& near) {
  const uint64_t cs[2] = {c0, c1};
  uint64_t at = 0;
  uint32_t fr = 0;
#pragma unroll
  for (int r = 0; r < NP; ++r) {
    const uint64_t c = cs[r];
    const uint32_t x0 = (uint32_t)c, x1 = (uint32_t)(c >> 32);  // x1 < 2^22 when c < 2^54
    const uint64_t G = a->G_lo[r];
    const uint32_t G0 = (uint32_t)G, G1 = (uint32_t)(G >> 32), G2 = a->G_hi[r];
    // Z = t + u + v 2^32 ~ c G / 2^64 (< 2^86): integer part Z >> 32, fraction Z mod 2^32
    uint64_t t = (uint64_t)__umulhi(x0, G1) + __umulhi(x1, G0);
    t += (uint64_t)x0 * G2;  // below 2^64: x0 G2 <= 2^64 - 2^33 + 1
    const uint64_t u = (uint64_t)x1 * G1, v = (uint64_t)x1 * G2;  // below 2^54 when c < 2^54
    const uint64_t s = t + u;
    const uint64_t ip = (s >> 32) + v + (s < t ? 1ull << 32 : 0);
    at += c * a->f[r] + ip;
    const uint32_t f2 = fr + (uint32_t)s;
    at += f2 < fr ? 1 : 0;
    fr = f2;
  }
  const uint32_t sr = fr + 0x80000000u;  // carries out when the fraction is >= 1/2
  at += sr < fr ? 1 : 0;
  near = sr >= 0xFFFFFFF8u;
  return at;
}

}  // namespace rlwe
