// The product kernel's tile (Eq. (LWEdot) by number-theoretic transforms, N = 4096):
// pointwise products of the transformed masks and weights summed over input blocks,
// the inverse transform, SampleExtract and the output epilogue. Shared by the product
// kernel (one tile per workgroup) and the persistent batch kernel (tiles taken from a
// work queue).
#pragma once

#include "ks_round.hpp"
#include "ntt_device.hpp"

namespace rlwe {

// Weight polynomial j and token range [t0, t_end) of tile loc of an item. order 0:
// token tiles vary fastest, so workgroups running together share their weight
// polynomial, which then stays in L2 (4 % faster on the 2048 x 2048, 128-token
// projection than polynomials varying fastest; keeping all tiles of a polynomial on
// one XCD was slower, as every XCD then streams all tokens' masks); order 1: the
// polynomials vary fastest.
typedef const __attribute__((address_space(4))) Item* ItemPtr;
__device__ __forceinline__ void product_tile(ItemPtr it, uint32_t loc, uint32_t& j, uint32_t& t0,
                                             uint32_t& t_end) {
  const uint32_t T = it->T, lt = it->tt_log2;
  const uint32_t tiles = (T + (1u << lt) - 1) >> lt;
  if (it->order == 0) {
    j = loc / tiles;
    t0 = (loc % tiles) << lt;
  } else {
    const uint32_t groups = it->groups;
    j = loc % groups;
    t0 = (loc / groups) << lt;
  }
  t_end = min(T, t0 + (1u << lt));
}

// NTT of one mask: item ii, local index loc = (t L + i) P + p (token t, block i, prime
// p), on kThreads threads (tid < kThreads) with an LDS buffer of kLdsWords.
// ahat[(((t L + i) P + p) N + lane_major(pos)) * 2 + {0, 1}], bit-reversed position
// pos: residue in [0, p) and its Shoup companion (the mask side carries the
// companions, computed once per token, so the resident weights need only their
// residues). With valid = false the transform runs on zeros and stores nothing (the
// caller's threads still meet every barrier).
__device__ __forceinline__ void mask_forward(BatchPtr bt, uint32_t ii, uint32_t loc, uint64_t* lds,
                                             int tid, bool valid) {
  const uint32_t P = bt->rc.P;
  const uint32_t p_idx = loc % P, ti = loc / P;
  const uint64_t p = bt->rc.q[p_idx];
  const uint64_t* tw = bt->ntt.fwd[p_idx];
  const bool seeded = bt->seeded != 0;
  const uint64_t* blk_in = bt->it[ii].ct + ti * ct_block_words(P, kN, seeded);
  uint64_t x[16];
  if (!valid) {
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = 0;
  } else if (seeded) {
    const uint64_t seed = blk_in[0];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = seeded_mask(seed, kN, p_idx, tid + 256 * k, p);
  } else {
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = blk_in[(size_t)p_idx * kN + tid + 256 * k];
  }
  ntt_forward(x, lds, tw, p, tid);
  if (!valid) return;
  uint64_t* dst = bt->it[ii].ahat + 2 * (size_t)loc * kN;
  const uint64_t r1 = bt->ntt.rq[p_idx][0], r0 = bt->ntt.rq[p_idx][1];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const uint64_t v = reduce4(x[k], p);
    // Shoup companion floor(v 2^64 / p): v floor(2^128 / p) / 2^64 is at most 1 low
    uint64_t c = v * r1 + __umul64hi(v, r0);
    c += (0 - c * p) >= p ? 1 : 0;
    const uint32_t at = 2 * lane_major(16 * tid + k);
    dst[at] = v;
    dst[at + 1] = c;
  }
}

// NTT of one mask at a ring degree NN below kNttN: the plain radix-2 transform on
// nthreads threads (all threads of the block meet its barriers), lds of NN words;
// loc = (t L + i) P + p as above, stored lane-major for the NN / 8-thread product.
template <int NN>
__device__ __forceinline__ void mask_forward_small(BatchPtr bt, uint32_t ii, uint32_t loc,
                                                   uint64_t* lds, uint32_t nthreads) {
  const uint32_t P = bt->rc.P;
  const uint32_t p_idx = loc % P, ti = loc / P;
  const uint64_t p = bt->rc.q[p_idx];
  const bool seeded = bt->seeded != 0;
  const uint64_t* blk_in = bt->it[ii].ct + ti * ct_block_words(P, NN, seeded);
  const uint64_t seed = seeded ? blk_in[0] : 0;
  for (uint32_t n = threadIdx.x; n < (uint32_t)NN; n += nthreads)
    lds[n] = seeded ? seeded_mask(seed, NN, p_idx, n, p) : blk_in[(size_t)p_idx * NN + n];
  gen_forward(lds, NN, bt->ntt.fwd[p_idx], p, nthreads);
  uint64_t* dst = bt->it[ii].ahat + 2 * (size_t)loc * NN;
  const uint64_t r1 = bt->ntt.rq[p_idx][0], r0 = bt->ntt.rq[p_idx][1];
  for (uint32_t n = threadIdx.x; n < (uint32_t)NN; n += nthreads) {  // n: bit-reversed position
    const uint64_t v = reduce4(lds[n], p);
    uint64_t c = v * r1 + __umul64hi(v, r0);
    c += (0 - c * p) >= p ? 1 : 0;
    const uint32_t at = 2 * lane_major<NN>(n);
    dst[at] = v;
    dst[at + 1] = c;
  }
}

// One tile of the product: weight polynomial j (a row, or a group of n_o packed rows)
// of item ii and the tokens of one token tile, on kInvThreads threads; the NP = P
// primes of a token are transformed together. LC = 2: the item has exactly two input
// blocks; LC = 0: any number. OUT: 0 switched to 2^qbits (u32), 1 raw residues (u64
// per prime), 2 masks rounded to 2^K for the gadget decomposition (u64, bodies written
// by the body kernel). loc is the tile's index within the item (product_tile). NN: the
// ring degree (4096, or 2048 on 256 threads); lds holds NP * InvSize<NN>::kLds words.
template <int OUT, int NP, int LC, int NN = kNttN>
__device__ __forceinline__ void ntt_product(BatchPtr bt, uint32_t ii, uint32_t loc, uint64_t* lds) {
  static_assert(LC == 0 || LC == 2, "block classes: exactly two, or any");
  const uint32_t L = bt->it[ii].m.L, rows = bt->it[ii].m.rows;
  // rows sharing one weight polynomial (1 unless rows are packed) and their slot size
  const uint32_t n_o = bt->it[ii].m.n_o, slot = bt->it[ii].m.slot;
  uint32_t j, t0, t_end;
  product_tile(&bt->it[ii], loc, j, t0, t_end);
  const uint64_t* ahat = bt->it[ii].ahat;
  const uint64_t* what = bt->it[ii].what;  // [groups][L][P][N] residues
  void* out = bt->it[ii].out;
  // per-prime constants, indexed by compile-time prime numbers only (ring
  // constants are read in place: a local copy indexed at run time would live in
  // scratch)
  uint64_t p[NP];
  InvMod md[NP];
  const uint64_t* tw[NP];
#pragma unroll
  for (int r = 0; r < NP; ++r) {
    p[r] = bt->rc.q[r];
    md[r] = InvMod{0 - p[r], 8 * p[r], bt->ntt.bm[r]};
    tw[r] = bt->ntt.inv[r];
  }
  for (uint32_t t = t0; t < t_end; ++t) {
    // the thread index is opaque per token, so the many thread-dependent twiddle
    // and exchange addresses are formed where they are used instead of being
    // hoisted out of the token loop (and spilled)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    uint64_t x[NP][8];
    // pointwise products below 4p each: two blocks stay below 8p, more are reduced.
    // One block (LC = 0, L = 1) or two (LC = 2).
    if (LC == 2 || L == 1) {
      constexpr int NB = LC == 2 ? 2 : 1;
      // the token's transformed masks and the polynomial's transformed weights as buffers:
      // position 8 tid + k of (block i, prime r) at element k NN / 8 + tid (lane-major), the
      // mask elements as (residue, companion) pairs
      const Rsrc ra = buf_rsrc(ahat + (size_t)t * NB * NP * NN * 2, NB * NP * NN * 16);
      const Rsrc rw = buf_rsrc(what + (size_t)j * NB * NP * NN, NB * NP * NN * 8);
      // One block: the operands of every prime are loaded together (48 words per thread).
      // Two blocks: prime by prime, both blocks' operands of the prime together (48 words),
      // so that a token waits for two rounds of loads rather than three.
      constexpr int NG = NB == 1 ? 1 : NP;  // load groups
#pragma unroll
      for (int rg = 0; rg < NG; ++rg) {
        constexpr int GB = NB == 1 ? NP : 2;  // (block, prime) pairs of a group
        uint64_t wv[GB][8], av[GB][16];
#pragma unroll
        for (int u = 0; u < GB; ++u) {
          const int i = NB == 1 ? 0 : u, r = NB == 1 ? u : rg;
          const uint32_t e0 = (i * NP + r) * NN;  // element offset of (block, prime)
#pragma unroll
          for (int k = 0; k < 8; ++k) wv[u][k] = buf_ld64(rw, 8 * tid, 8 * (e0 + (NN / 8) * k));
#pragma unroll
          for (int k = 0; k < 8; ++k)
            buf_ld128(ra, 16 * tid, 16 * (e0 + (NN / 8) * k), av[u][2 * k], av[u][2 * k + 1]);
        }
#pragma unroll
        for (int u = 0; u < GB; ++u) {
          const int i = NB == 1 ? 0 : u, r = NB == 1 ? u : rg;
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const uint64_t v = mul_shoup4(wv[u][k], av[u][2 * k], av[u][2 * k + 1], md[r].pn);
            x[r][k] = i == 0 ? v : x[r][k] + v;
          }
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < NP; ++r) {
#pragma unroll
        for (int k = 0; k < 8; ++k) x[r][k] = 0;
        for (uint32_t i = 0; i < L; ++i) {  // positions 8 tid + k (layout Q1)
          const uint64_t* a = ahat + 2 * ((((size_t)t * L + i) * NP + r) * NN + tid);
          const uint64_t* w = what + (((size_t)j * L + i) * NP + r) * NN + tid;
          if (L <= 2) {
#pragma unroll
            for (int k = 0; k < 8; ++k)
              x[r][k] += mul_shoup4(w[(NN / 8) * k], a[(NN / 4) * k], a[(NN / 4) * k + 1], md[r].pn);
          } else {
#pragma unroll
            for (int k = 0; k < 8; ++k)
              x[r][k] = reduce_barrett(
                  x[r][k] + mul_shoup4(w[(NN / 8) * k], a[(NN / 4) * k], a[(NN / 4) * k + 1], md[r].pn), md[r]);
          }
        }
      }
    }
    // The inverse transform's loads stay below the pointwise stage: hoisted into it, they
    // pushed the two-block products past 128 VGPRs into spills (152 bytes per thread, the
    // kernel 27 % slower at K = 8192 than with this barrier and 20 bytes).
    __builtin_amdgcn_sched_barrier(0);
    // the switched epilogue takes the last stage's differences unmultiplied
    ntt_inverse<NP, NN, OUT != 0>(x, lds, tw, md, tid);
    // Coefficient m = tid + (NN / 8) k of C (layout Q4). Row rho of the group (row
    // j n_o + rho) is SampleExtract at h = (rho + 1) slot - 1 (Sec. 3.2): a'[n] =
    // C[h - n] for n <= h, -C[N + h - n] otherwise, so C[m] lands at n = h - m, or
    // negated at n = h - m + N. Unpacked rows: n_o = 1, slot = N, h = N - 1.
    if (OUT == 2) {
      // a~ = round(c 2^K / q) mod 2^K of every coefficient (Decomp's rounding, for
      // KeySwitch packing); the switch of -c is -(switch of c) (q is odd: no ties)
      uint64_t c[NP][8];
#pragma unroll
      for (int r = 0; r < NP; ++r)
#pragma unroll
        for (int k = 0; k < 8; ++k) c[r][k] = reduce4(reduce_barrett(x[r][k], md[r]), p[r]);
      uint64_t av[8];
      uint32_t nearm = bt->force_exact ? 0xffu : 0u;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        bool nr;
        av[k] = round_fast<NP>(&bt->kr, c[0][k], c[NP - 1][k], nr);
        nearm |= (nr ? 1u : 0u) << k;
      }
      while (nearm) {  // rare: exact rounding of the coefficient
        const int k = __builtin_ctz(nearm);
        nearm &= nearm - 1;
        uint64_t c0 = c[0][0], c1 = c[NP - 1][0];
#pragma unroll
        for (int kk = 1; kk < 8; ++kk) {
          c0 = k == kk ? c[0][kk] : c0;
          c1 = k == kk ? c[NP - 1][kk] : c1;
        }
        const uint64_t e = round_exact<NP>(&bt->kr, c0, NP == 2 ? c1 : 0);
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) av[kk] = k == kk ? e : av[kk];
      }
      const uint64_t km = bt->kmask;
      for (uint32_t rho = 0; rho < n_o && j * n_o + rho < rows; ++rho) {
        const uint32_t h = (rho + 1) * slot - 1;
        uint64_t* o = (uint64_t*)out + ((size_t)t * rows + j * n_o + rho) * (NN + NP);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t m = tid + (NN / 8) * k;
          if (m <= h)
            o[h - m] = av[k] & km;
          else
            o[h + NN - m] = (0 - av[k]) & km;
        }
      }
    } else if (OUT == 1) {
      uint64_t c[NP][8];
#pragma unroll
      for (int r = 0; r < NP; ++r)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          c[r][k] = reduce4(reduce_barrett(x[r][k], md[r]), p[r]);  // 1/N is in the weights
        }
      for (uint32_t rho = 0; rho < n_o && j * n_o + rho < rows; ++rho) {
        const uint32_t h = (rho + 1) * slot - 1;
#pragma unroll
        for (int r = 0; r < NP; ++r) {
          uint64_t* o = (uint64_t*)out + ((size_t)t * rows + j * n_o + rho) * NP * (NN + 1) +
                        r * (NN + 1);
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const uint32_t m = tid + (NN / 8) * k;
            if (m <= h)
              o[h - m] = c[r][k];
            else
              o[h + NN - m] = c[r][k] ? p[r] - c[r][k] : 0;
          }
        }
      }
    } else {
      uint32_t res[8];
      // coefficients within 8 units below a rounding tie (all of them when forced)
      uint32_t tie = bt->force_exact ? 0xffu : 0u;
      const uint32_t qbits = bt->rc.qbits;
      const uint64_t half = 1ull << (63 - qbits);
      uint32_t one[NP][2];
#pragma unroll
      for (int r = 0; r < NP; ++r)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          one[r][i] = 1;
          __asm__ volatile("" : "+s"(one[r][i]));  // volatile: four distinct registers
        }
      typedef const __attribute__((address_space(4))) uint32_t* HPtr;
      HPtr h0[NP], h1[NP];
#pragma unroll
      for (int r = 0; r < NP; ++r) {
        h0[r] = (HPtr)bt->ntt.h[r];
        h1[r] = (HPtr)bt->ntt.hl[r];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        // k >= 4: x holds C[m] / w (w the last stage's twiddle), and hl carries w.
        // V = W + one half, W = bits 64..127 of sum_p c_p H_p 2^96 (mod 2^128), at most 7
        // units low: c 2^32 / q mod 2^32 in 32.32 fixed point, rounded to q_out = 2^qbits
        uint64_t c[NP];
#pragma unroll
        for (int r = 0; r < NP; ++r) c[r] = x[r][k];
        uint32_t vlo, vhi;
        fixed_sum<NP>(c, k < 4 ? h0 : h1, half, one, vlo, vhi);
        bool near;
        res[k] = round_qout_near(vlo, vhi, qbits, near);
        tie |= (near ? 1u : 0u) << k;
      }
      while (tie) {  // rare: exact CRT and switch of the coefficient
        const int k = __builtin_ctz(tie);
        tie &= tie - 1;
        uint64_t c[NP];
#pragma unroll
        for (int r = 0; r < NP; ++r) {
          c[r] = x[r][0];
#pragma unroll
          for (int kk = 1; kk < 8; ++kk) c[r] = k == kk ? x[r][kk] : c[r];
        }
        const RingConst rc = kernarg_load(&bt->rc);
        uint64_t y[NP];
#pragma unroll
        for (int r = 0; r < NP; ++r) {
          y[r] = k < 4 ? mul_shoup(c[r], bt->ntt.crt[r], bt->ntt.crt_shoup[r], p[r])
                       : mul_shoup(c[r], bt->ntt.crtl[r], bt->ntt.crtl_shoup[r], p[r]);
          y[r] = y[r] >= p[r] ? y[r] - p[r] : y[r];
        }
        u128 v = y[0];
        if (NP == 2) {
          const u128 Q = make_u128(rc.Q_hi, rc.Q_lo);
          v = (u128)y[0] * p[NP - 1] + (u128)y[NP - 1] * p[0];
          v = v >= Q ? v - Q : v;
        }
        const uint32_t e = switch_exact((i128)v, rc);
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) res[kk] = k == kk ? e : res[kk];
      }
      // the switch of -c is -(switch of c) mod 2^qbits (q is odd: no ties)
      const uint32_t qmask = qout_mask(qbits);
      if (n_o == 1) {
        // one row per polynomial: h = NN - 1 >= m, coefficient m at word NN - 1 - m of the
        // row, i.e. at byte 4 (NN - 1 - tid - (NN/8) 7) + 4 (NN/8)(7 - k) >= 0
        const Rsrc ro = buf_rsrc((uint32_t*)out + ((size_t)t * rows + j) * (NN + 1), (NN + 1) * 4);
        const uint32_t vo = 4 * (NN - 1 - tid - (NN / 8) * 7);
#pragma unroll
        for (int k = 0; k < 8; ++k)
          __builtin_amdgcn_raw_buffer_store_b32(res[k], ro, (int)vo, (int)(4 * (NN / 8) * (7 - k)), 0);
        continue;
      }
      for (uint32_t rho = 0; rho < n_o && j * n_o + rho < rows; ++rho) {
        const uint32_t h = (rho + 1) * slot - 1;
        uint32_t* o = (uint32_t*)out + ((size_t)t * rows + j * n_o + rho) * (NN + 1);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t m = tid + (NN / 8) * k;
          if (m <= h)
            o[h - m] = res[k];
          else
            o[h + NN - m] = (0u - res[k]) & qmask;
        }
      }
    }
  }
}

}  // namespace rlwe
