// The mask part of Eq. (LWEdot) by number-theoretic transforms, for N = 4096
// (transform layouts and arithmetic: ntt_device.hpp).
#include "ks_round.hpp"
#include "ntt_device.hpp"

namespace rlwe {


// NTT of the masks of every NTT-method product: one workgroup per (token, block,
// prime). ahat[(((t L + i) P + p) N + lane_major(pos)) * 2 + {0, 1}], bit-reversed
// position pos: residue in [0, p) and its Shoup companion (the mask side carries
// the companions, computed once per token, so the resident weights need only their
// residues).
__global__ void __launch_bounds__(kThreads) ntt_mask_fwd_kernel(Batch) {
  __shared__ uint64_t lds[kLdsWords];
  const BatchPtr bt = kernarg_batch();
  const uint32_t blk = linear_block();
  const uint32_t nb = bt->n;
  if (blk >= bt->fwd_start[nb]) return;
  const uint32_t ii = find_item(bt->fwd_start, nb, blk);
  const uint32_t P = bt->rc.P;
  const uint32_t loc = blk - bt->fwd_start[ii];  // (t L + i) P + p
  const uint32_t p_idx = loc % P, ti = loc / P;
  const uint64_t p = bt->rc.q[p_idx];
  const uint64_t* tw = bt->ntt.fwd[p_idx];
  const bool seeded = bt->seeded != 0;
  const uint64_t* blk_in = bt->it[ii].ct + ti * ct_block_words(P, kN, seeded);
  const int tid = threadIdx.x;
  uint64_t x[16];
  if (seeded) {
    const uint64_t seed = blk_in[0];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = seeded_mask(seed, kN, p_idx, tid + 256 * k, p);
  } else {
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = blk_in[(size_t)p_idx * kN + tid + 256 * k];
  }
  ntt_forward(x, lds, tw, p, tid);
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

// Product kernel: one workgroup per (row j, tile of kTokTile tokens) of each item;
// the NP = P primes of a token are transformed together. LC = 2: every item has
// exactly two input blocks; LC = 0: any number (a launch holds one class).
// OUT: 0 switched to 2^qbits (u32), 1 raw residues (u64 per prime), 2 masks rounded
// to 2^K for the gadget decomposition (u64, bodies written by the body kernel).
template <int OUT, int NP, int LC>
__global__ void __launch_bounds__(kInvThreads, LC == 2 ? 4 : 1) ntt_mask_kernel(Batch) {
  static_assert(LC == 0 || LC == 2, "block classes: exactly two, or any");
  __shared__ uint64_t lds[NP * kInvLdsWords];
  const BatchPtr bt = kernarg_batch();
  const uint32_t blk = linear_block();
  const uint32_t nb = bt->n;
  if (blk >= bt->mask_start[nb]) return;
  const uint32_t ii = find_item(bt->mask_start, nb, blk);
  const uint32_t L = bt->it[ii].m.L, rows = bt->it[ii].m.rows, T = bt->it[ii].T;
  // rows sharing one weight polynomial (1 unless rows are packed) and their slot size
  const uint32_t n_o = bt->it[ii].m.n_o, slot = bt->it[ii].m.slot;
  const uint32_t groups = (rows + n_o - 1) / n_o;
  const uint32_t loc = blk - bt->mask_start[ii];
  // token tiles vary fastest: workgroups running together share their weight
  // polynomial, which then stays in L2 (4 % faster on the 2048 x 2048, 128-token
  // projection than polynomials varying fastest; keeping all tiles of a polynomial
  // on one XCD was slower, as every XCD then streams all tokens' masks)
  const uint32_t tiles = (T + kTokTile - 1) / kTokTile;
  const uint32_t j = loc / tiles, t0 = (loc % tiles) * kTokTile;  // j: the weight polynomial
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
  const uint32_t t_end = min(T, t0 + kTokTile);
  for (uint32_t t = t0; t < t_end; ++t) {
    // the thread index is opaque per token, so the many thread-dependent twiddle
    // and exchange addresses are formed where they are used instead of being
    // hoisted out of the token loop (and spilled)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    uint64_t x[NP][8];
    // pointwise products below 4p each: two blocks stay below 8p, more are reduced.
    // One block (LC = 0, L = 1) or two (LC = 2): the loads of every prime of a block
    // are issued together, before any use.
    if (LC == 2 || L == 1) {
      constexpr int NB = LC == 2 ? 2 : 1;
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        uint64_t wv[NP][8], av[NP][16];
#pragma unroll
        for (int r = 0; r < NP; ++r) {
          // lane-major operands: position 8 tid + k at k 512 + tid
          const uint64_t* a = ahat + 2 * ((((size_t)t * NB + i) * NP + r) * kN + tid);
          const uint64_t* w = what + (((size_t)j * NB + i) * NP + r) * kN + tid;
#pragma unroll
          for (int k = 0; k < 8; ++k) wv[r][k] = w[512 * k];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            av[r][2 * k] = a[1024 * k];
            av[r][2 * k + 1] = a[1024 * k + 1];
          }
        }
#pragma unroll
        for (int r = 0; r < NP; ++r)
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const uint64_t v = mul_shoup4(wv[r][k], av[r][2 * k], av[r][2 * k + 1], md[r].pn);
            x[r][k] = i == 0 ? v : x[r][k] + v;
          }
      }
    } else {
#pragma unroll
      for (int r = 0; r < NP; ++r) {
#pragma unroll
        for (int k = 0; k < 8; ++k) x[r][k] = 0;
        for (uint32_t i = 0; i < L; ++i) {  // positions 8 tid + k (layout Q1)
          const uint64_t* a = ahat + 2 * ((((size_t)t * L + i) * NP + r) * kN + tid);
          const uint64_t* w = what + (((size_t)j * L + i) * NP + r) * kN + tid;
          if (L <= 2) {
#pragma unroll
            for (int k = 0; k < 8; ++k)
              x[r][k] += mul_shoup4(w[512 * k], a[1024 * k], a[1024 * k + 1], md[r].pn);
          } else {
#pragma unroll
            for (int k = 0; k < 8; ++k)
              x[r][k] = reduce_barrett(
                  x[r][k] + mul_shoup4(w[512 * k], a[1024 * k], a[1024 * k + 1], md[r].pn), md[r]);
          }
        }
      }
    }
    ntt_inverse<NP>(x, lds, tw, md, tid);
    // Coefficient m = tid + 512 k of C (layout Q4). Row rho of the group (row
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
        uint64_t* o = (uint64_t*)out + ((size_t)t * rows + j * n_o + rho) * (kN + NP);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t m = tid + 512 * k;
          if (m <= h)
            o[h - m] = av[k] & km;
          else
            o[h + kN - m] = (0 - av[k]) & km;
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
          uint64_t* o = (uint64_t*)out + ((size_t)t * rows + j * n_o + rho) * NP * (kN + 1) +
                        r * (kN + 1);
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const uint32_t m = tid + 512 * k;
            if (m <= h)
              o[h - m] = c[r][k];
            else
              o[h + kN - m] = c[r][k] ? p[r] - c[r][k] : 0;
          }
        }
      }
    } else {
      uint32_t res[8];
      // coefficients within 8 units below a rounding tie (all of them when forced)
      uint32_t tie = bt->force_exact ? 0xffu : 0u;
      const uint32_t qbits = bt->rc.qbits;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        uint64_t A = fixed_part(x[0][k], bt->ntt.h[0]);
        if (NP == 2) A += fixed_part(x[NP - 1][k], bt->ntt.h[NP - 1]);
        // A = bits 64..127 of sum_p c_p H_p 2^96 (mod 2^128), at most 7 units low:
        // c 2^32 / q mod 2^32 in 32.32 fixed point, rounded to q_out = 2^qbits
        int64_t dist;
        res[k] = round_qout(A, qbits, dist);
        if (dist < 0 && dist >= -8) tie |= 1u << k;
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
          y[r] = mul_shoup(c[r], bt->ntt.crt[r], bt->ntt.crt_shoup[r], p[r]);
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
      for (uint32_t rho = 0; rho < n_o && j * n_o + rho < rows; ++rho) {
        const uint32_t h = (rho + 1) * slot - 1;
        uint32_t* o = (uint32_t*)out + ((size_t)t * rows + j * n_o + rho) * (kN + 1);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t m = tid + 512 * k;
          if (m <= h)
            o[h - m] = res[k];
          else
            o[h + kN - m] = (0u - res[k]) & qmask;
        }
      }
    }
  }
}

// NTT-domain weights: one workgroup per (weight polynomial j, block i, prime p).
// Unpacked (n_o = 1, slot = N), block i of row j is encoded reversed, w_hat[k] =
// w_j[iN + N - 1 - k] (zero past K), Sec. 4.3. Packed (one block, slot = K), row
// j n_o + rho of the group fills coefficients [rho K, rho K + K) reversed:
// w_hat[rho K + K - 1 - k] = w_{j n_o + rho}[k] (zero past the last row and N).
// what[((j L + i) P + p) N + lane_major(pos)], bit-reversed position pos, residues
// in [0, p), multiplied by N^-1 (the factor of the inverse transform).
__global__ void __launch_bounds__(kThreads) ntt_weights_kernel(MatArgs m, NttConst ntt,
                                                               RingConst rc, uint64_t* what) {
  __shared__ uint64_t lds[kLdsWords];
  const uint32_t P = rc.P;
  const uint32_t loc = blockIdx.x;  // (j L + i) P + p
  const uint32_t p_idx = loc % P, ji = loc / P, i = ji % m.L, j = ji / m.L;
  const uint64_t p = rc.q[p_idx];
  const int tid = threadIdx.x;
  uint64_t x[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const uint32_t pos = tid + 256 * k;
    const uint32_t rho = pos / m.slot, row = j * m.n_o + rho;
    const uint32_t col = i * kN + m.slot - 1 - (pos - rho * m.slot);
    const bool in = rho < m.n_o && row < m.rows && col < m.k;
    const int v = in ? (int)m.w[(size_t)row * m.kw + col] : 0;
    x[k] = v < 0 ? p - (uint64_t)(-v) : (uint64_t)v;
  }
  ntt_forward(x, lds, ntt.fwd[p_idx], p, tid);
  uint64_t* dst = what + (size_t)loc * kN;
  const uint64_t ninv = ntt.ninv[p_idx], ninv_shoup = ntt.ninv_shoup[p_idx];
#pragma unroll
  for (int k = 0; k < 16; ++k)  // the inverse transform's factor 1/N, applied once here
    dst[lane_major(16 * tid + k)] = mulmod_shoup(reduce4(x[k], p), ninv, ninv_shoup, p);
}

hipError_t launch_ntt_mask_fwd(const Batch& b, hipStream_t s) {
  const uint32_t blocks = b.fwd_start[b.n];
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(ntt_mask_fwd_kernel, grid_for(blocks), dim3(kThreads), 0, s, b);
  return hipGetLastError();
}

template <int OUT, int LC>
void launch_ntt_mask_out(const Batch& b, dim3 g, hipStream_t s) {
  if (b.rc.P == 2)
    hipLaunchKernelGGL((ntt_mask_kernel<OUT, 2, LC>), g, dim3(kInvThreads), 0, s, b);
  else
    hipLaunchKernelGGL((ntt_mask_kernel<OUT, 1, LC>), g, dim3(kInvThreads), 0, s, b);
}

template <int LC>
void launch_ntt_mask_lc(const Batch& b, dim3 g, hipStream_t s) {
  if (b.gadget)
    launch_ntt_mask_out<2, LC>(b, g, s);
  else if (b.raw)
    launch_ntt_mask_out<1, LC>(b, g, s);
  else
    launch_ntt_mask_out<0, LC>(b, g, s);
}

hipError_t launch_ntt_mask(const Batch& b, uint32_t lclass, hipStream_t s) {
  const uint32_t blocks = b.mask_start[b.n];
  if (blocks == 0) return hipSuccess;
  const dim3 g = grid_for(blocks);
  if (lclass == 2)
    launch_ntt_mask_lc<2>(b, g, s);
  else
    launch_ntt_mask_lc<0>(b, g, s);
  return hipGetLastError();
}

hipError_t launch_ntt_weights(const MatArgs& m, const NttConst& ntt, const RingConst& rc,
                              uint64_t* what, hipStream_t s) {
  const uint32_t blocks = (m.rows + m.n_o - 1) / m.n_o * m.L * rc.P;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(ntt_weights_kernel, dim3(blocks), dim3(kThreads), 0, s, m, ntt, rc, what);
  return hipGetLastError();
}

}  // namespace rlwe
