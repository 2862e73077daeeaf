// Device functions of the input preparation and the body product, shared by their
// own kernels and the persistent batch kernel.
//
// prep:  residues of every ciphertext coefficient -> centred integer c in
//        (-q/2, q/2) (CRT for two primes) -> balanced base-255 digits. Mask digits
//        are stored twice per plane, negated in front (plane index m in [0, N) holds
//        -d[m], m in [N, 2N) holds d[m - N]), so the Toeplitz operand of the
//        negacyclic product (Sec. 3.2, Eq. (LWEdot)) is the plain window
//        plane[N + k - n] for k, n in [0, N).
// body:  b'_j = sum_k w_j[k] B[k] (coefficient N-1 of the block products, the
//        SampleExtract body), exact per digit with packed int8 dot products.
#pragma once

#include "rlwe_internal.hpp"

namespace rlwe {

// Lift residues (P = 1 or 2) to the centred integer in (-q/2, q/2).
__device__ inline i128 lift_centered(const RingConst& rc, uint64_t r0, uint64_t r1) {
  u128 c;
  if (rc.P == 1) {
    c = r0;
  } else {
    const uint64_t y0 = mulmod_shoup(r0, rc.crt_inv[0], rc.crt_inv_shoup[0], rc.q[0]);
    const uint64_t y1 = mulmod_shoup(r1, rc.crt_inv[1], rc.crt_inv_shoup[1], rc.q[1]);
    c = (u128)y0 * rc.q[1] + (u128)y1 * rc.q[0];
    const u128 Q = make_u128(rc.Q_hi, rc.Q_lo);
    if (c >= Q) c -= Q;
  }
  const u128 half = make_u128(rc.half_hi, rc.half_lo);
  const u128 Q = make_u128(rc.Q_hi, rc.Q_lo);
  return c > half ? (i128)c - (i128)Q : (i128)c;
}

// Balanced base-255 digits of v (|v| < 2^108): v = sum_l d[l] 255^l, d in [-127, 127].
template <int D>
__device__ inline void digits255(i128 v, int8_t* d) {
  const bool neg = v < 0;
  u128 m = neg ? (u128)(-v) : (u128)v;
  uint32_t w[4] = {(uint32_t)m, (uint32_t)(m >> 32), (uint32_t)(m >> 64), (uint32_t)(m >> 96)};
#pragma unroll
  for (int l = 0; l < D; ++l) {
    uint64_t rem = 0;
#pragma unroll
    for (int i = 3; i >= 0; --i) {
      const uint64_t cur = (rem << 32) | w[i];
      w[i] = (uint32_t)(cur / 255u);
      rem = cur % 255u;
    }
    int r = (int)rem;
    if (r > 127) {  // carry into the next digit
      r -= 255;
      for (int i = 0; i < 4; ++i) {
        if (++w[i] != 0) break;
      }
    }
    d[l] = (int8_t)(neg ? -r : r);
  }
}

// Digit planes of coefficient k of input block ti = t L + i of item ii: the body
// digits always, the mask digits for the matrix-core method.
template <int D>
__device__ __forceinline__ void prep_coeff(BatchPtr bt, uint32_t ii, uint32_t ti, uint32_t k) {
  const RingConst rc = kernarg_load(&bt->rc);
  const Item a = kernarg_load(&bt->it[ii]);
  const uint32_t N = rc.N, P = rc.P, L = a.m.L;
  if (ti >= a.T * L || k >= N) return;
  const uint32_t i = ti % L;
  const uint32_t t = ti / L;
  const bool seeded = bt->seeded != 0;
  const uint64_t* blk_in = a.ct + ti * ct_block_words(P, N, seeded);
  const uint64_t* B = blk_in + (seeded ? 2 : (size_t)P * N);
  uint64_t a0 = 0, a1 = 0;
  if (a.method == 0) {  // the NTT method needs the body digits only
    if (seeded) {
      const uint64_t seed = blk_in[0];
      a0 = seeded_mask(seed, N, 0, k, rc.q[0]);
      if (P > 1) a1 = seeded_mask(seed, N, 1, k, rc.q[1]);
    } else {
      a0 = blk_in[k];
      if (P > 1) a1 = blk_in[N + k];
    }
  }
  int8_t da[D], db[D];
  if (a.method == 0) digits255<D>(lift_centered(rc, a0, a1), da);
  digits255<D>(lift_centered(rc, B[k], P > 1 ? B[N + k] : 0), db);
#pragma unroll
  for (int l = 0; l < D; ++l) {
    const size_t plane = ((size_t)t * D + l) * L + i;
    if (a.method == 0) {
      int8_t* em = a.emask + plane * 2 * N;
      em[N + k] = da[l];
      em[k] = (int8_t)(-da[l]);
    }
    a.ebody[plane * N + k] = db[l];
  }
}

// Sum of the 16 int8 products of two 16-byte vectors, added to acc.
__device__ inline int32_t dot16(int4 w, int4 e, int32_t acc) {
  acc = __builtin_amdgcn_sdot4(w.x, e.x, acc, false);
  acc = __builtin_amdgcn_sdot4(w.y, e.y, acc, false);
  acc = __builtin_amdgcn_sdot4(w.z, e.z, acc, false);
  return __builtin_amdgcn_sdot4(w.w, e.w, acc, false);
}

// Body of Eq. (LWEdot) (b'_j = sum_k w_j[k] B[k], the coefficient N - 1 of the block
// products) and its switch, for block loc of item ii: 256 threads (tid < 256), one per
// (token, row), rows in the packed slot-major order where rows are packed.
template <int D, bool RAW>
__device__ __forceinline__ void body_block(BatchPtr bt, uint32_t ii, uint32_t loc, uint32_t tid) {
  const RingConst rc = kernarg_load(&bt->rc);
  const Item a = kernarg_load(&bt->it[ii]);
  const MatArgs& m = a.m;
  // blocks of one token: body_blocks_per_token (rows, or the packed slot-major order)
  const uint32_t per = body_blocks_per_token(m);
  const uint32_t t = loc / per;
  const uint32_t v = (loc - t * per) * 256 + tid;
  if (t >= a.T) return;
  const uint32_t N = rc.N;
  uint32_t j = v;  // output row
  int32_t S[D];
#pragma unroll
  for (int l = 0; l < D; ++l) S[l] = 0;
  if (m.n_o > 1) {
    // Multi-row packing (one block): row j = g n_o + rho is the coefficient h = (rho
    // + 1) K - 1 of w_hat_g B, w_hat_g holding row g n_o + r reversed in [r K, r K +
    // K). Term r: sum_k w_{g n_o + r}[k] B[(rho - r) K + k], with B[-i] = -B[N - i]
    // (X^N = -1); every term lies on one side of the wrap. Threads run slot-major
    // (v = rho gpad + g, gpad a multiple of 64), so rho, and with it the offset into
    // B of every term, is the same across a wave: the digit loads stay uniform.
    const uint32_t K = m.k, gpad = body_group_pad(m);
    const uint32_t rho = __builtin_amdgcn_readfirstlane(v / gpad), g = v - rho * gpad;
    j = g * m.n_o + rho;
    if (rho >= m.n_o || j >= m.rows) return;
    const int8_t* eb = a.ebody + (size_t)t * D * N;
    for (uint32_t r = 0; r < m.n_o; ++r) {
      const uint32_t wr = g * m.n_o + r;
      const int8_t* wrow = m.w + (size_t)min(wr, m.rows - 1) * m.kw;
      const int wmask = wr < m.rows ? -1 : 0;  // rows past the last one are zero
      const bool neg = r > rho;
      const uint32_t base = neg ? N - (r - rho) * K : (rho - r) * K;
      int32_t U[D];
#pragma unroll
      for (int l = 0; l < D; ++l) U[l] = 0;
      if ((K & 15) == 0) {  // base is a multiple of 16: 16-byte loads stay aligned
        for (uint32_t k = 0; k < K; k += 16) {
          int4 w16 = *(const int4*)(wrow + k);
          w16.x &= wmask;
          w16.y &= wmask;
          w16.z &= wmask;
          w16.w &= wmask;
#pragma unroll
          for (int l = 0; l < D; ++l) U[l] = dot16(w16, *(const int4*)(eb + (size_t)l * N + base + k), U[l]);
        }
      } else if ((K & 3) == 0) {  // word loads stay aligned
        for (uint32_t k = 0; k < K; k += 4) {
          const int w4 = *(const int*)(wrow + k) & wmask;
#pragma unroll
          for (int l = 0; l < D; ++l)
            U[l] = __builtin_amdgcn_sdot4(w4, *(const int*)(eb + (size_t)l * N + base + k), U[l],
                                          false);
        }
      } else {
        for (uint32_t k = 0; k < K; ++k) {
          const int w1 = (int)wrow[k] & wmask;
#pragma unroll
          for (int l = 0; l < D; ++l) U[l] += w1 * (int)eb[(size_t)l * N + base + k];
        }
      }
#pragma unroll
      for (int l = 0; l < D; ++l) S[l] = neg ? S[l] - U[l] : S[l] + U[l];
    }
  } else if (j >= m.rows) {
    return;
  }
  for (uint32_t i = 0; i < m.L && m.n_o == 1; ++i) {
    const uint32_t kb = min(N, m.k - i * N);
    const uint32_t kp = (kb + 31u) & ~31u;
    const int8_t* wrow = m.w + (size_t)j * m.kw + (size_t)i * N;
    for (uint32_t k = 0; k < kp; k += 16) {
      const int4 w16 = *(const int4*)(wrow + k);
#pragma unroll
      for (int l = 0; l < D; ++l)
        S[l] = dot16(w16, *(const int4*)(a.ebody + (((size_t)t * D + l) * m.L + i) * N + k), S[l]);
    }
  }
  i128 V = 0;
#pragma unroll
  for (int l = D - 1; l >= 0; --l) V = V * 255 + S[l];
  const size_t row = (size_t)t * m.rows + j;
  if (RAW) {
    uint64_t* o = (uint64_t*)a.out;
    // raw [T][M][P][N+1], or after rounded masks (gadget output) [T][M][N+P]
    for (uint32_t p = 0; p < rc.P; ++p)
      o[bt->gadget ? row * (N + rc.P) + N + p : (row * rc.P + p) * (N + 1) + N] =
          mod_i128(V, bt->rc.q[p]);
  } else {
    ((uint32_t*)a.out)[row * (N + 1) + N] = switch_exact(V, rc);
  }
}

}  // namespace rlwe
