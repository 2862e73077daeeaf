// Input preparation, the body product and the standalone modulus switch.
//
// prep:      residues of every ciphertext coefficient -> centred integer c in
//            (-q/2, q/2) (CRT for two primes) -> balanced base-255 digits. Mask
//            digits are stored twice per plane, negated in front (plane index m in
//            [0, N) holds -d[m], m in [N, 2N) holds d[m - N]), so the Toeplitz
//            operand of the negacyclic product (Sec. 3.2, Eq. (LWEdot)) is the
//            plain window plane[N + k - n] for k, n in [0, N).
// body:      b'_j = sum_k w_j[k] B[k] (coefficient N-1 of the block products,
//            the SampleExtract body), exact per digit with packed int8 dot products.
// modswitch: round(c 2^32 / q) mod 2^32 of raw RNS outputs (Sec. 3.2).
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

template <int D>
__global__ void __launch_bounds__(256) prep_kernel(Batch) {
  const BatchPtr bt = kernarg_batch();
  const uint32_t blk = linear_block();
  const uint32_t nb = bt->n;
  if (blk >= bt->prep_start[nb]) return;
  const uint32_t ii = find_item(bt->prep_start, nb, blk);
  const RingConst rc = kernarg_load(&bt->rc);
  const Item a = kernarg_load(&bt->it[ii]);
  const uint32_t N = rc.N, P = rc.P, L = a.m.L;
  // blocks of one (token, input block) pair: N / 256 when N >= 256, else 1
  const uint32_t per = N >= 256 ? N >> 8 : 1;
  const uint32_t loc = blk - bt->prep_start[ii];
  const uint32_t ti = loc / per;  // t * L + i
  const uint32_t k = (loc - ti * per) * 256 + threadIdx.x;
  if (ti >= a.T * L || k >= N) return;
  const uint32_t i = ti % L;
  const uint32_t t = ti / L;
  const bool seeded = bt->seeded != 0;
  const uint64_t* blk_in = a.ct + ti * ct_block_words(P, N, seeded);
  const uint64_t* B = blk_in + (seeded ? 2 : (size_t)P * N);
  uint64_t a0, a1 = 0;
  if (seeded) {
    const uint64_t seed = blk_in[0];
    a0 = seeded_mask(seed, N, 0, k, rc.q[0]);
    if (P > 1) a1 = seeded_mask(seed, N, 1, k, rc.q[1]);
  } else {
    a0 = blk_in[k];
    if (P > 1) a1 = blk_in[N + k];
  }
  int8_t da[D], db[D];
  digits255<D>(lift_centered(rc, a0, a1), da);
  digits255<D>(lift_centered(rc, B[k], P > 1 ? B[N + k] : 0), db);
#pragma unroll
  for (int l = 0; l < D; ++l) {
    const size_t plane = ((size_t)t * D + l) * L + i;
    if (a.method == 0) {  // the NTT method needs the body digits only
      int8_t* em = a.emask + plane * 2 * N;
      em[N + k] = da[l];
      em[k] = (int8_t)(-da[l]);
    }
    a.ebody[plane * N + k] = db[l];
  }
}

hipError_t launch_prep(const Batch& b, hipStream_t s) {
  const uint32_t blocks = b.prep_start[b.n];
  if (blocks == 0) return hipSuccess;
  if (b.rc.D == 7)
    hipLaunchKernelGGL(prep_kernel<7>, grid_for(blocks), dim3(256), 0, s, b);
  else
    hipLaunchKernelGGL(prep_kernel<14>, grid_for(blocks), dim3(256), 0, s, b);
  return hipGetLastError();
}

// ---------------------------------------------------------------- body

// Sum of the 16 int8 products of two 16-byte vectors, added to acc.
__device__ inline int32_t dot16(int4 w, int4 e, int32_t acc) {
  acc = __builtin_amdgcn_sdot4(w.x, e.x, acc, false);
  acc = __builtin_amdgcn_sdot4(w.y, e.y, acc, false);
  acc = __builtin_amdgcn_sdot4(w.z, e.z, acc, false);
  return __builtin_amdgcn_sdot4(w.w, e.w, acc, false);
}

template <int D, bool RAW>
__global__ void __launch_bounds__(256) body_kernel(Batch) {
  const BatchPtr bt = kernarg_batch();
  const uint32_t blk = linear_block();
  const uint32_t nb = bt->n;
  if (blk >= bt->body_start[nb]) return;
  const uint32_t ii = find_item(bt->body_start, nb, blk);
  const RingConst rc = kernarg_load(&bt->rc);
  const Item a = kernarg_load(&bt->it[ii]);
  const MatArgs& m = a.m;
  // blocks of one token: body_blocks_per_token (rows, or the packed slot-major order)
  const uint32_t per = body_blocks_per_token(m);
  const uint32_t loc = blk - bt->body_start[ii];
  const uint32_t t = loc / per;
  const uint32_t v = (loc - t * per) * 256 + threadIdx.x;
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

hipError_t launch_body(const Batch& b, hipStream_t s) {
  const uint32_t blocks = b.body_start[b.n];
  if (blocks == 0) return hipSuccess;
  const dim3 grid = grid_for(blocks);
  if (b.rc.D == 7) {
    if (b.raw)
      hipLaunchKernelGGL((body_kernel<7, true>), grid, dim3(256), 0, s, b);
    else
      hipLaunchKernelGGL((body_kernel<7, false>), grid, dim3(256), 0, s, b);
  } else {
    if (b.raw)
      hipLaunchKernelGGL((body_kernel<14, true>), grid, dim3(256), 0, s, b);
    else
      hipLaunchKernelGGL((body_kernel<14, false>), grid, dim3(256), 0, s, b);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- modulus switch

__global__ void __launch_bounds__(256) modswitch_kernel(RingConst rc, const uint64_t* in,
                                                        size_t count, uint32_t* out) {
  const uint32_t len = rc.N + 1;
  const size_t idx = (size_t)linear_block() * blockDim.x + threadIdx.x;
  if (idx >= count * len) return;
  const size_t c = idx / len;
  const uint32_t n = (uint32_t)(idx % len);
  const uint64_t* r = in + c * rc.P * len + n;
  u128 v;
  if (rc.P == 1) {
    v = r[0];
  } else {
    const uint64_t y0 = mulmod_shoup(r[0], rc.crt_inv[0], rc.crt_inv_shoup[0], rc.q[0]);
    const uint64_t y1 = mulmod_shoup(r[len], rc.crt_inv[1], rc.crt_inv_shoup[1], rc.q[1]);
    v = (u128)y0 * rc.q[1] + (u128)y1 * rc.q[0];
    const u128 Q = make_u128(rc.Q_hi, rc.Q_lo);
    if (v >= Q) v -= Q;
  }
  out[idx] = switch_exact((i128)v, rc);
}

hipError_t launch_modswitch(const RingConst& rc, const uint64_t* in, size_t count, uint32_t* out,
                            hipStream_t s) {
  const size_t total = count * (rc.N + 1);
  if (total == 0) return hipSuccess;
  if ((total + 255) / 256 >= (1ull << 31)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(modswitch_kernel, grid_for((uint32_t)((total + 255) / 256)), dim3(256), 0, s,
                     rc, in, count, out);
  return hipGetLastError();
}

// Bit-packing of switched ciphertexts (Sec. 4.5: the switched output is returned
// packed into a bit-vector): in u32[count][len] with values below 2^k -> out
// u32[count][words], words = ceil(len k / 32). Coefficient i of a ciphertext
// occupies stream bits [i k, (i + 1) k), least significant first; unused high bits
// of the last word are zero. HBM-bound: a workgroup owns a tile of consecutive
// output words of one ciphertext, stages the coefficients they touch in LDS (sized
// for k at launch; every thread has several independent lane-consecutive loads in
// flight) and assembles up to eight words per thread, each store instruction
// lane-consecutive. The first coefficient of word w is floor(32 w / k) =
// umulhi(32 w, ceil(2^32 / k)), exact for 32 w < 2^21 and k >= 2.
// Words per workgroup tile: 2048 (eight per thread) for k >= 16, 1024 for k >= 8,
// else 256, so the staged coefficients stay below 33 KB of LDS.
__host__ __device__ inline uint32_t pack_tile_words(uint32_t k) {
  return k >= 16 ? 2048u : k >= 8 ? 1024u : 256u;
}
__host__ __device__ inline uint32_t pack_tile_coeffs(uint32_t k) {
  return (pack_tile_words(k) * 32 + k - 1) / k + 2;  // coefficients touching one tile, at most
}

__global__ void __launch_bounds__(256) pack_bits_kernel(const uint32_t* in, size_t count,
                                                        uint32_t len, uint32_t k, uint32_t kinv,
                                                        uint32_t words, uint32_t tiles,
                                                        uint32_t* out) {
  extern __shared__ uint32_t coeff[];
  const uint32_t tw = pack_tile_words(k);
  const uint32_t blk = linear_block();
  const uint32_t c = blk / tiles;
  if (c >= count) return;
  const uint32_t w0 = (blk - c * tiles) * tw;
  const uint32_t w1 = min(words, w0 + tw);
  const uint32_t i0 = k == 1 ? 32 * w0 : __umulhi(32 * w0, kinv);
  const uint32_t i1 = min(len, (32 * w1 + k - 1) / k);
  const uint32_t* src = in + (size_t)c * len;
  const uint32_t mask = qout_mask(k);
#pragma unroll 8
  for (uint32_t i = i0 + threadIdx.x; i < i1; i += 256) coeff[i - i0] = src[i] & mask;
  __syncthreads();
  uint32_t* dst = out + (size_t)c * words;
  for (uint32_t w = w0 + threadIdx.x; w < w1; w += 256) {
    const uint32_t b0 = 32 * w;  // first stream bit of this word
    const uint32_t first = k == 1 ? b0 : __umulhi(b0, kinv);
    uint64_t acc = 0;
    for (uint32_t i = first, sh0 = i * k; i < i1 && sh0 < b0 + 32; ++i, sh0 += k) {
      const uint64_t v = coeff[i - i0];
      acc |= sh0 >= b0 ? v << (sh0 - b0) : v >> (b0 - sh0);  // shifts below 64
    }
    dst[w] = (uint32_t)acc;
  }
}

hipError_t launch_pack_bits(const uint32_t* in, size_t count, uint32_t len, uint32_t k,
                            uint32_t* out, hipStream_t s) {
  const uint32_t words = (uint32_t)(((uint64_t)len * k + 31) / 32);
  if (count == 0 || words == 0) return hipSuccess;
  if (32ull * words >= (1ull << 21)) return hipErrorInvalidValue;  // len * k < 2^21 bits
  const uint32_t tiles = (words + pack_tile_words(k) - 1) / pack_tile_words(k);
  const uint64_t blocks = (uint64_t)count * tiles;
  if (blocks >= (1ull << 31)) return hipErrorInvalidValue;
  const uint32_t kinv = k == 1 ? 0u : (uint32_t)(((1ull << 32) + k - 1) / k);  // ceil(2^32 / k)
  const size_t lds = (size_t)pack_tile_coeffs(k) * 4;  // 33 KB at k = 1, 5 KB at k = 26
  hipLaunchKernelGGL(pack_bits_kernel, grid_for((uint32_t)blocks), dim3(256), lds, s, in, count,
                     len, k, kinv, words, tiles, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- weight set-up

__global__ void transpose_pad_kernel(const int8_t* src, uint32_t rows, uint32_t cols,
                                     int transpose, int8_t* dst, uint32_t dst_rows_pad,
                                     uint32_t dst_kw) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t r = blockIdx.y;
  if (k >= dst_kw || r >= dst_rows_pad) return;
  int8_t v = 0;
  if (transpose) {  // dst[r][k] = src[k][r], dst has cols rows and rows columns
    if (r < cols && k < rows) v = src[(size_t)k * cols + r];
  } else {
    if (r < rows && k < cols) v = src[(size_t)r * cols + k];
  }
  dst[(size_t)r * dst_kw + k] = v;
}

hipError_t launch_transpose_pad(const int8_t* src, uint32_t rows, uint32_t cols, bool transpose,
                                int8_t* dst, uint32_t dst_rows_pad, uint32_t dst_kw,
                                hipStream_t s) {
  hipLaunchKernelGGL(transpose_pad_kernel, dim3((dst_kw + 255) / 256, dst_rows_pad), dim3(256), 0,
                     s, src, rows, cols, (int)transpose, dst, dst_rows_pad, dst_kw);
  return hipGetLastError();
}

__global__ void row_l1_kernel(const int8_t* w, uint32_t rows, uint32_t kw, uint32_t* out) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  uint32_t s = 0;
  for (uint32_t k = 0; k < kw; ++k) {
    const int v = w[(size_t)r * kw + k];
    s += (uint32_t)(v < 0 ? -v : v);
  }
  out[r] = s;
}

hipError_t launch_row_l1(const int8_t* w, uint32_t rows, uint32_t kw, uint32_t* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(row_l1_kernel, dim3((rows + 255) / 256), dim3(256), 0, s, w, rows, kw, out);
  return hipGetLastError();
}

}  // namespace rlwe
