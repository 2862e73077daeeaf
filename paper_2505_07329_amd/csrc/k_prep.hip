// Kernels of the input preparation and the body product (device functions in
// prep_device.hpp), the standalone modulus switch (round(c 2^k / q) mod 2^k of raw
// RNS outputs, Sec. 3.2), bit-packing and the weight layout.
#include "prep_device.hpp"

namespace rlwe {

template <int D>
__global__ void __launch_bounds__(256) prep_kernel(Batch) {
  const BatchPtr bt = kernarg_batch();
  const uint32_t blk = linear_block();
  const uint32_t nb = bt->n;
  if (blk >= bt->prep_start[nb]) return;
  const uint32_t ii = find_item(bt->prep_start, nb, blk);
  // blocks of one (token, input block) pair: N / 256 when N >= 256, else 1
  const uint32_t N = bt->rc.N;
  const uint32_t per = N >= 256 ? N >> 8 : 1;
  const uint32_t loc = blk - bt->prep_start[ii];
  const uint32_t ti = loc / per;  // t * L + i
  prep_coeff<D>(bt, ii, ti, (loc - ti * per) * 256 + threadIdx.x);
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

template <int D, bool RAW>
__global__ void __launch_bounds__(256) body_kernel(Batch) {
  const BatchPtr bt = kernarg_batch();
  const uint32_t blk = linear_block();
  const uint32_t nb = bt->n;
  if (blk >= bt->body_start[nb]) return;
  const uint32_t ii = find_item(bt->body_start, nb, blk);
  body_block<D, RAW>(bt, ii, blk - bt->body_start[ii], threadIdx.x);
}

// The body of unpacked rows on the int8 matrix cores: S_l[j][t] = sum_k w_j[k] d_l[t][k]
// for every digit plane l of every token's body is an int8 matrix product (rows j against
// columns (token, digit)), exact in int32 (|S_l| <= 127^2 K < 2^31 for K <= 2 N). A wave
// owns 32 rows and NTW column tiles of 32 columns, each TPT tokens of SL digit slots (the
// slots past D are zero), so it reads each weight fragment once for NTW products; the
// four waves of a block take consecutive tokens of the same rows. The operands of four
// k-steps are requested before their products (the loop is bound by load latency
// otherwise). The digit sums of a (row, token) pair lie in one row of a tile; they meet
// through LDS, and V = sum_l 255^l S_l is switched exactly, as in body_block.
typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef int v16i_t __attribute__((ext_vector_type(16)));

template <int D>
struct BodyMma {
  static constexpr int SL = D == 14 ? 16 : 8;  // digit slots per token
  static constexpr int TPT = 32 / SL;          // tokens per column tile
  static constexpr int NTW = 2;                // column tiles per wave
  static constexpr int TPB = 4 * NTW * TPT;    // tokens per block
};

template <int D, bool RAW>
__global__ void __launch_bounds__(256) body_mma_kernel(Batch) {
  typedef BodyMma<D> G;
  __shared__ int32_t tr[4][32][33];  // per wave: one column tile, rows x columns
  const BatchPtr bt = kernarg_batch();
  const uint32_t blk = linear_block();
  const uint32_t nb = bt->n;
  if (blk >= bt->body_start[nb]) return;
  const uint32_t ii = find_item(bt->body_start, nb, blk);
  const RingConst rc = kernarg_load(&bt->rc);
  const Item a = kernarg_load(&bt->it[ii]);
  const MatArgs& m = a.m;
  const uint32_t N = rc.N;
  const uint32_t loc = blk - bt->body_start[ii];
  const uint32_t tgs = (a.T + G::TPB - 1) / G::TPB;  // token groups, fastest in the block order
  const uint32_t j0 = (loc / tgs) * 32, tb = (loc % tgs) * G::TPB;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = lane & 31, g = lane >> 5;
  // operands of this lane: row j0 + c of the weights; column c of each column tile,
  // token tw + f TPT + c / SL, digit c % SL (zero past D or past the last token)
  const uint32_t tw = tb + wave * G::NTW * G::TPT;
  const int l = c % G::SL;
  const int8_t* wrow = m.w + (size_t)(j0 + c) * m.kw + 16 * g;  // j0 + 32 <= rows_pad
  const int8_t* eb[G::NTW];
  bool live[G::NTW];
#pragma unroll
  for (int f = 0; f < G::NTW; ++f) {
    const uint32_t t = tw + f * G::TPT + c / G::SL;
    live[f] = l < D && t < a.T;
    const uint32_t tc = min(t, a.T - 1), lc = min(l, D - 1);
    eb[f] = a.ebody + (size_t)(tc * D + lc) * m.L * N + 16 * g;
  }
  v16i_t acc[G::NTW];
#pragma unroll
  for (int f = 0; f < G::NTW; ++f) acc[f] = v16i_t{0};
  for (uint32_t i = 0; i < m.L; ++i) {
    const uint32_t kb = min(N, m.k - i * N);
    const uint32_t kp = (kb + 31u) & ~31u;  // the weight rows are zero from K on
    for (uint32_t k = 0; k < kp; k += 128) {
      const uint32_t steps = min(4u, (kp - k) >> 5);  // uniform
      v4i_t wa[4], e[4][G::NTW];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if ((uint32_t)s >= steps) break;
        wa[s] = *(const v4i_t*)(wrow + (size_t)i * N + k + 32 * s);
#pragma unroll
        for (int f = 0; f < G::NTW; ++f) e[s][f] = *(const v4i_t*)(eb[f] + (size_t)i * N + k + 32 * s);
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if ((uint32_t)s >= steps) break;
#pragma unroll
        for (int f = 0; f < G::NTW; ++f)
          acc[f] = __builtin_amdgcn_mfma_i32_32x32x32_i8(wa[s], live[f] ? e[s][f] : v4i_t{0}, acc[f], 0,
                                                         0, 0);
      }
    }
  }
  // accumulator element e of a lane: row 8 (e / 4) + 4 g + e % 4, column c
#pragma unroll
  for (int f = 0; f < G::NTW; ++f) {
#pragma unroll
    for (int e = 0; e < 16; ++e) tr[wave][8 * (e >> 2) + 4 * g + (e & 3)][c] = acc[f][e];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int q = lane; q < 32 * G::TPT; q += 64) {
      const uint32_t r = q & 31, tt = q >> 5;
      const uint32_t j = j0 + r, t = tw + f * G::TPT + tt;
      i128 V = 0;
#pragma unroll
      for (int d = D - 1; d >= 0; --d) V = V * 255 + tr[wave][r][tt * G::SL + d];
      if (j < m.rows && t < a.T) {
        const size_t row = (size_t)t * m.rows + j;
        if (RAW) {
          uint64_t* o = (uint64_t*)a.out;
          for (uint32_t p = 0; p < rc.P; ++p)
            o[bt->gadget ? row * (N + rc.P) + N + p : (row * rc.P + p) * (N + 1) + N] =
                mod_i128(V, bt->rc.q[p]);
        } else {
          ((uint32_t*)a.out)[row * (N + 1) + N] = switch_exact(V, rc);
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();  // every lane has read the tile before the next is written
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

hipError_t launch_body(const Batch& b, hipStream_t s) {
  const uint32_t blocks = b.body_start[b.n];
  if (blocks == 0) return hipSuccess;
  // unpacked rows everywhere: the matrix-core body, blocks of 32 rows x TPB tokens
  bool mma = true;
  for (uint32_t x = 0; x < b.n; ++x)
    mma = mma && b.it[x].m.n_o == 1 && b.it[x].m.k <= 2 * b.rc.N && b.it[x].m.rows_pad % 32 == 0 &&
          (reinterpret_cast<uintptr_t>(b.it[x].ebody) & 15) == 0;
  if (mma) {
    Batch mb = b;
    const uint32_t tpb = b.rc.D == 7 ? BodyMma<7>::TPB : BodyMma<14>::TPB;
    for (uint32_t x = 0; x < b.n; ++x) {
      const Item& it = b.it[x];
      mb.body_start[x + 1] = mb.body_start[x] + (it.m.rows + 31) / 32 * ((it.T + tpb - 1) / tpb);
    }
    const dim3 grid = grid_for(mb.body_start[mb.n]);
    if (b.rc.D == 7) {
      if (b.raw)
        hipLaunchKernelGGL((body_mma_kernel<7, true>), grid, dim3(256), 0, s, mb);
      else
        hipLaunchKernelGGL((body_mma_kernel<7, false>), grid, dim3(256), 0, s, mb);
    } else {
      if (b.raw)
        hipLaunchKernelGGL((body_mma_kernel<14, true>), grid, dim3(256), 0, s, mb);
      else
        hipLaunchKernelGGL((body_mma_kernel<14, false>), grid, dim3(256), 0, s, mb);
    }
    return hipGetLastError();
  }
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

// ---------------------------------------------------------------- tuning inputs

// Random inputs for timing (the kernels are data-oblivious): uint64 words of the
// ciphertext layout [..][P][N], word w a residue mod q[(w / N) % P]; int8 values in
// [-s, s]. Counter-based (SplitMix64 finalizer of seed + w), reproducible.
__global__ void fill_residues_kernel(uint64_t* dst, size_t count, uint32_t N, uint32_t P,
                                     uint64_t q0, uint64_t q1, uint64_t seed) {
  const size_t w = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= count) return;
  const uint64_t q = ((w / N) % P) == 0 ? q0 : q1;
  dst[w] = splitmix64_at(seed, w) % q;
}
__global__ void fill_int8_kernel(int8_t* dst, size_t count, uint32_t s, uint64_t seed) {
  const size_t w = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= count) return;
  dst[w] = (int8_t)((int)(splitmix64_at(seed, w) % (2 * s + 1)) - (int)s);
}

hipError_t launch_fill_residues(uint64_t* dst, size_t count, const RingConst& rc, uint64_t seed,
                                hipStream_t s) {
  if (count == 0) return hipSuccess;
  const size_t blocks = (count + 255) / 256;
  if (blocks >= (1ull << 31)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fill_residues_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, dst, count,
                     rc.N, rc.P, rc.q[0], rc.P > 1 ? rc.q[1] : rc.q[0], seed);
  return hipGetLastError();
}
hipError_t launch_fill_int8(int8_t* dst, size_t count, uint32_t mag, uint64_t seed,
                            hipStream_t s) {
  if (count == 0) return hipSuccess;
  const size_t blocks = (count + 255) / 256;
  if (blocks >= (1ull << 31) || mag > 127) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fill_int8_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, dst, count, mag,
                     seed);
  return hipGetLastError();
}

}  // namespace rlwe
