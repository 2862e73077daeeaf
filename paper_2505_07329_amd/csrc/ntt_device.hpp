// Device helpers of the number-theoretic transforms (N = 4096, and N = 2048 for the
// inverse of the product): modular products, butterflies, register layouts and LDS
// exchanges of the forward and inverse transforms. Shared by the product kernels and
// the KeySwitch packing kernels.
//
// Transforms used by the mask part of Eq. (LWEdot), for N = 4096.
//
// Per prime q_p the negacyclic product in Z_p[X]/(X^N + 1) is computed as
// INTT(NTT(a) * NTT(b)) with the psi-twisted transform (psi a primitive 2N-th
// root of unity): a Cooley-Tukey forward transform from natural to bit-reversed
// order and a Gentleman-Sande inverse from bit-reversed to natural order, both
// with the twist folded into their twiddles psi^(+-bitrev(k)); the factor 1/N
// of the inverse is folded into the resident weights (product) or applied at the
// end (KeySwitch packing). For token t and output
// row j the polynomial C = sum_i A_{t,i} * w_hat_ij (Sec. 4.3, reversed weight
// encoding) gives the SampleExtract mask at N - 1 as a'[n] = C[N - 1 - n]
// (Sec. 3.2), so a'[n] is the inverse transform's coefficient N - 1 - n. The two
// residues are combined by CRT and switched to 2^32 exactly in the epilogue.
//
// The forward transforms (masks once per token, weights once per load) run on
// 256 threads holding 16 residues each, in three passes of four radix-2 stages
// in registers with two exchanges through LDS. Residue positions per thread:
//   L1: 16 tid + k          (spans 1..8)
//   L2: 256 b + r + 16 k    (spans 16..128, b = tid / 16, r = tid % 16)
//   L3: tid + 256 k         (spans 256..2048)
// The inverse transforms, one per output and prime, run on 512 threads holding
// 8 residues of each prime, in four passes of three stages:
//   Q1: 8 tid + k                      (spans 1..4)
//   Q2: 64 (tid / 8) + tid % 8 + 8 k    (spans 8..32)
//   Q3: 512 (tid / 64) + tid % 64 + 64 k (spans 64..256)
//   Q4: tid + 512 k                    (spans 512..2048)
// Q1 -> Q2 and Q2 -> Q3 move residues only among the 64 threads of one wave
// (positions 512 w .. 512 w + 511), so those exchanges need no workgroup
// barrier; Q3 -> Q4 crosses waves. The primes of a token are transformed
// together: two independent chains per butterfly position.
// Arithmetic is lazy (Harvey). The forward transforms keep values below 4p with
// exact Shoup products below 2p. The inverse trades exactness for instructions:
// its Shoup products take the quotient without the partial products that end
// below bit 64 (results below 4p for any 64-bit input), its sums are left
// unreduced inside a pass (each difference is biased by the stage's bound) and a
// Barrett step at the end of every second pass brings back the two elements that can
// exceed 8p. With q_p < 2^54 every intermediate stays below 512 q_p < 2^63.
#pragma once

#include "rlwe_internal.hpp"

namespace rlwe {
namespace {

constexpr int kN = kNttN;
constexpr int kThreads = 256;
constexpr int kLdsWords = kN + kN / 16;  // padded exchange buffer: position + position / 16
constexpr int kInvThreads = 512;
constexpr int kInvLdsWords = kN + kN / 8;  // inverse exchange buffer per prime (8 blocks of 576 words)

struct Tw {
  uint64_t w, wp;
};
__device__ __forceinline__ Tw ld_tw(const uint64_t* t, uint32_t k) {
  const uint4 v = *(const uint4*)(t + 2 * k);
  return Tw{((uint64_t)v.y << 32) | v.x, ((uint64_t)v.w << 32) | v.z};
}
// a * w mod p in [0, 2p) for any a < 2^64 (Shoup, wp = floor(w 2^64 / p))
__device__ __forceinline__ uint64_t mul_shoup(uint64_t a, uint64_t w, uint64_t wp, uint64_t p) {
  return a * w - __umul64hi(a, wp) * p;
}
// Buffer access (MUBUF): a resource of `bytes` bytes from a wave-uniform base, a per-lane
// byte offset in a VGPR and a uniform byte offset in an SGPR, so a thread's loads of one
// operand share one offset register and need no 64-bit address arithmetic. Accesses
// past `bytes` read zeros and write nothing.
typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ __forceinline__ Rsrc buf_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           0x00020000 /* 32-bit data format (gfx9) */);
}
__device__ __forceinline__ uint64_t buf_ld64(Rsrc r, uint32_t voff, uint32_t soff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
  return ((uint64_t)v[1] << 32) | v[0];
}
__device__ __forceinline__ void buf_ld128(Rsrc r, uint32_t voff, uint32_t soff, uint64_t& x,
                                          uint64_t& y) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
  x = ((uint64_t)v[1] << 32) | v[0];
  y = ((uint64_t)v[3] << 32) | v[2];
}

__device__ __forceinline__ uint64_t reduce4(uint64_t x, uint64_t p) {  // [0, 4p) -> [0, p)
  x = x >= 2 * p ? x - 2 * p : x;
  return x >= p ? x - p : x;
}
// bias + bits 64..127 of sum_r c_r h_r (mod 2^64) for any 64-bit c_r and 128-bit h_r
// (four words each, h_r a pointer in any address space), as its low and high words,
// dropping the partial products that end below bit 64 (the result is at most 3 NP
// units low); carries past bit 127 fall off, as the sum is wanted mod 2^128.
// one[r][i]: the value 1, in scalar registers the compiler cannot see through, so that
// each 32-bit high product is added as (u64) x one + a, one v_mad_u64_u32 (a
// zero-extending 64-bit add would need a register pair with a zero high word, a copy
// per term; one shared value would let the compiler sum the high products first, with
// the same copies). The high word is summed in 32-bit arithmetic behind an empty asm
// (as in mul_shoup4).
template <int NP, class HP>
__device__ __forceinline__ void fixed_sum(const uint64_t (&c)[NP], const HP (&h)[NP], uint64_t bias,
                                          const uint32_t (&one)[NP][2], uint32_t& lo, uint32_t& hi) {
  uint64_t a = bias;
  hi = 0;
#pragma unroll
  for (int r = 0; r < NP; ++r) {
    const uint32_t c0 = (uint32_t)c[r], c1 = (uint32_t)(c[r] >> 32);
    a = (uint64_t)c0 * h[r][2] + a;
    a = (uint64_t)c1 * h[r][1] + a;
    a = (uint64_t)__umulhi(c0, h[r][1]) * one[r][0] + a;
    a = (uint64_t)__umulhi(c1, h[r][0]) * one[r][1] + a;
    hi += c0 * h[r][3] + c1 * h[r][2];
  }
  hi += (uint32_t)(a >> 32);
  __asm__("" : "+v"(hi));
  lo = (uint32_t)a;
}

// a * w mod p in [0, 4p) for any a < 2^64, pn = 2^64 - p: Shoup's quotient
// floor(a wp / 2^64) less the partial products below bit 64 (at most 2 low), and
// the remainder a w + q pn taken mod 2^64.
// SPLIT (the kernels' form): the remainder's high word r_hi + a0 w1 + a1 w0 + q0 n1 +
// q1 n0 is formed from two 64-bit multiply-adds, a1 w0 + a0 w1 and q1 n0 + q0 n1 (kept
// whole behind an empty asm, so each is one v_mad_u64_u32 on a 32-bit product), and one
// three-way add, itself behind an empty asm: without them the compiler folds
// (h << 32) | lo(r) back into a 64-bit add of a zero-extended word (a register copy and
// a 64-bit add) and spends four multiplies and two three-way adds on the cross terms.
// 11 instructions against 13; measured 4.5 % + 1.3 % faster on the 2048 x 2048
// projection and 9 % at K = 8192. An isolated chain of products runs faster in the
// combined form, so the rate microbenchmarks time both. (Two other forms measured
// slower: the four cross products chained through 64-bit v_mad_u64_u32 with the high
// word added by inline asm, and the high-word add written as an instruction in inline
// asm, opaque to the scheduler's latency model.)
template <bool SPLIT = true>
__device__ __forceinline__ uint64_t mul_shoup4(uint64_t a, uint64_t w, uint64_t wp, uint64_t pn) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t wp0 = (uint32_t)wp, wp1 = (uint32_t)(wp >> 32);
  uint64_t q = (uint64_t)a1 * wp1 + __umulhi(a0, wp1);
  q += __umulhi(a1, wp0);
  const uint32_t q0 = (uint32_t)q, q1 = (uint32_t)(q >> 32);
  const uint32_t w0 = (uint32_t)w, w1 = (uint32_t)(w >> 32);
  const uint32_t n0 = (uint32_t)pn, n1 = (uint32_t)(pn >> 32);
  uint64_t r = (uint64_t)a0 * w0;
  r = (uint64_t)q0 * n0 + r;
  if (SPLIT) {
    uint64_t t1 = (uint64_t)a1 * w0 + (uint32_t)(a0 * w1);
    uint64_t t2 = (uint64_t)q1 * n0 + (uint32_t)(q0 * n1);
    __asm__("" : "+v"(t1), "+v"(t2));
    uint32_t h = (uint32_t)(r >> 32) + (uint32_t)t1 + (uint32_t)t2;
    __asm__("" : "+v"(h));
    return ((uint64_t)h << 32) | (uint32_t)r;
  }
  const uint32_t h = (uint32_t)(r >> 32) + a0 * w1 + a1 * w0 + q0 * n1 + q1 * n0;
  return ((uint64_t)h << 32) | (uint32_t)r;
}

// Constants of the inverse transform for one prime.
struct InvMod {
  uint64_t pn;  // 2^64 - p
  uint64_t p8;  // 8p, the bound of a pass's inputs
  uint32_t bm;  // floor(2^64 / p)
};
// v mod p in [0, 3p) for any v < 2^64: the quotient estimate from the high word
// is at most 2 low.
__device__ __forceinline__ uint64_t reduce_barrett(uint64_t v, const InvMod& md) {
  const uint32_t q = __umulhi((uint32_t)(v >> 32), md.bm);
  const uint64_t r = (uint64_t)q * (uint32_t)md.pn + v;
  // the high product behind an empty asm: a multiply and a 32-bit add, where the
  // combined form took a 64-bit multiply-add between two register copies
  uint32_t m = q * (uint32_t)(md.pn >> 32);
  __asm__("" : "+v"(m));
  return ((uint64_t)((uint32_t)(r >> 32) + m) << 32) | (uint32_t)r;
}

// forward butterfly: X, Y < 4p -> X + wY, X - wY (both < 4p)
__device__ __forceinline__ void ct_bfly(uint64_t& X, uint64_t& Y, const Tw& t, uint64_t p) {
  const uint64_t twop = 2 * p;
  const uint64_t x = X >= twop ? X - twop : X;
  const uint64_t v = mul_shoup(Y, t.w, t.wp, p);
  X = x + v;
  Y = x + twop - v;
}
// inverse butterfly: X, Y < B -> X + Y (< 2B), (X - Y) w (< 4p)
template <bool SPLIT = true>
__device__ __forceinline__ void gs_bfly(uint64_t& X, uint64_t& Y, const Tw& t, uint64_t B,
                                        uint64_t pn) {
  const uint64_t d = X + B - Y;
  X += Y;
  Y = mul_shoup4<SPLIT>(d, t.w, t.wp, pn);
}

// Storage index of bit-reversed position pos in the lane-major layout of operands
// read by the NN / 8-thread kernels (512 threads at N = 4096), whose thread t holds
// positions 8 t .. 8 t + 7 (layout Q1): position 8 t + k is stored at k NN / 8 + t,
// so each of a wave's loads of one k covers consecutive words.
template <int NN = kNttN>
__host__ __device__ __forceinline__ uint32_t lane_major(uint32_t pos) {
  return (pos % 8) * (NN / 8) + pos / 8;
}
__device__ __forceinline__ uint32_t pad(uint32_t pos) { return pos + pos / 16; }

// Four stages of one pass on x[16] at positions base + STRIDE * k. The twiddle
// of the pair at position pos, span t, is entry N / (2t) + pos / (2t) of the table.
// Forward: spans STRIDE * 8, * 4, * 2, * 1 (Cooley-Tukey).
template <int STRIDE>
__device__ __forceinline__ void fwd_pass(uint64_t* x, uint32_t base, const uint64_t* tw, uint64_t p) {
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int sp = 8 >> st;        // distance in k
    const uint32_t t = STRIDE * sp;  // span in positions
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      if (k & sp) continue;
      const uint32_t pos = base + STRIDE * k;
      ct_bfly(x[k], x[k + sp], ld_tw(tw, kN / (2 * t) + pos / (2 * t)), p);
    }
  }
}
__device__ __forceinline__ void store_l1(uint64_t* lds, const uint64_t* x, int tid) {
#pragma unroll
  for (int k = 0; k < 16; ++k) lds[pad(16 * tid + k)] = x[k];
}
__device__ __forceinline__ void load_l1(const uint64_t* lds, uint64_t* x, int tid) {
#pragma unroll
  for (int k = 0; k < 16; ++k) x[k] = lds[pad(16 * tid + k)];
}
__device__ __forceinline__ void store_l2(uint64_t* lds, const uint64_t* x, int tid) {
  const int b = tid >> 4, r = tid & 15;
#pragma unroll
  for (int k = 0; k < 16; ++k) lds[pad(256 * b + r + 16 * k)] = x[k];
}
__device__ __forceinline__ void load_l2(const uint64_t* lds, uint64_t* x, int tid) {
  const int b = tid >> 4, r = tid & 15;
#pragma unroll
  for (int k = 0; k < 16; ++k) x[k] = lds[pad(256 * b + r + 16 * k)];
}
__device__ __forceinline__ void store_l3(uint64_t* lds, const uint64_t* x, int tid) {
#pragma unroll
  for (int k = 0; k < 16; ++k) lds[pad(tid + 256 * k)] = x[k];
}
__device__ __forceinline__ void load_l3(const uint64_t* lds, uint64_t* x, int tid) {
#pragma unroll
  for (int k = 0; k < 16; ++k) x[k] = lds[pad(tid + 256 * k)];
}

// Forward transform: x in layout L3, natural order -> x in layout L1, bit-reversed order.
__device__ __forceinline__ void ntt_forward(uint64_t* x, uint64_t* lds, const uint64_t* tw,
                                            uint64_t p, int tid) {
  fwd_pass<256>(x, 0, tw, p);  // spans 2048..256: twiddles do not depend on tid
  store_l3(lds, x, tid);
  __syncthreads();
  load_l2(lds, x, tid);
  fwd_pass<16>(x, 256 * (tid >> 4), tw, p);  // spans 128..16: r never reaches a block edge
  __syncthreads();
  store_l2(lds, x, tid);
  __syncthreads();
  load_l1(lds, x, tid);
  fwd_pass<1>(x, 16 * tid, tw, p);
  __syncthreads();
}

// Inverse pass PASS (layout Q1..Q4) on NP transforms at once: three
// Gentleman-Sande stages, spans S, 2S, 4S, on inputs below B = 8p 2^EIN. Stage s
// sees inputs below B 2^s; element k keeps its sum through the stages after the
// last one in which it took a product (k's highest set bit), so at the end element
// 0 is below 8B, element 1 below 16p and the rest below 8p. END brings elements 0, 1
// below 3p. Passes alternate: one from below 8p (EIN = 0) leaves everything below
// 64p, the next starts there (EIN = 3) and ends below 512p < 2^63 (p < 2^54), where
// END reduces; half the passes need no reduction. Every difference of a pass is
// biased by the bound of its last stage, 4B (one constant per pass and prime, where
// one per stage ran out of scalar registers); the differences stay below 8B.
template <int PASS, int NN = kNttN>
struct InvLayout {
  static constexpr int S = PASS == 0 ? 1 : PASS == 1 ? 8 : PASS == 2 ? 64 : NN / 8;  // stride in k
  __device__ static uint32_t base(int tid) {
    return PASS == 0   ? 8 * tid
           : PASS == 1 ? 64 * (tid >> 3) + (tid & 7)
           : PASS == 2 ? 512 * (tid >> 6) + (tid & 63)
                       : tid;
  }
};
// Sizes of the inverse transforms of ring degree NN: NN / 8 threads, and the words of
// one prime's exchange buffer (blocks of 576 words per 512 positions).
template <int NN>
struct InvSize {
  static constexpr int kThreads = NN / 8;
  static constexpr int kLds = NN + NN / 8;
};
// Exchange buffer addresses (8-byte words) of position pos in exchange EX (1:
// Q1 -> Q2, 2: Q2 -> Q3, 3: Q3 -> Q4). 64-bit LDS accesses are served 32 lanes at
// a time over 32 banks of 8 bytes (measured on gfx950): Q1 and Q2 need the
// padding of exchange 1, Q3 and Q4 are conflict-free unpadded, and exchange 2
// swizzles bits 3-4 of the position within a wave's block. Exchanges 1 and 2
// keep each wave inside its own block of 576 words (no barrier around them);
// exchange 3 lies between workgroup barriers.
template <int EX>
__device__ __forceinline__ uint32_t xaddr(uint32_t pos) {
  if (EX == 1) return pos + pos / 8;
  if (EX == 2) {
    const uint32_t l = pos & 511;
    return 576 * (pos >> 9) + (l ^ (((l >> 6) & 3) << 3));
  }
  return pos;
}

// Twiddle of the butterfly with lower element k of a thread in 512-thread layout
// PASS (InvLayout), span t: entry N / (2t) + pos / (2t). In layouts Q4 and Q3 it is
// the same on every lane of a wave: positions tid + 512 k give pos / (2t) = 512 k /
// (2t) for t >= 512 (tid < 512), and positions 512 w + l + 64 k (wave w, lane l < 64)
// give (512 w + 64 k) / (2t) for t >= 64, since l never carries; those are read with
// scalar loads, the others per lane.
typedef const __attribute__((address_space(4))) uint64_t* TwScalarPtr;
template <int PASS, int NN = kNttN>
__device__ __forceinline__ Tw tw512(const uint64_t* tw, uint32_t t, int k, int tid) {
  if (PASS >= 2) {
    // positions tid + (NN / 8) k in Q4 with t >= NN / 8 (tid < NN / 8 never carries)
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane(tid) >> 6;
    const uint32_t upos = PASS == 3 ? (uint32_t)(NN / 8) * k : 512u * wave + 64u * k;
    const uint32_t idx = NN / (2 * t) + upos / (2 * t);
    return Tw{((TwScalarPtr)tw)[2 * idx], ((TwScalarPtr)tw)[2 * idx + 1]};
  }
  // per lane: one 16-byte buffer load at byte 16 idx of the table (N entries)
  const uint32_t idx =
      NN / (2 * t) + (InvLayout<PASS, NN>::base(tid) + InvLayout<PASS, NN>::S * k) / (2 * t);
  uint64_t w, wp;
  buf_ld128(buf_rsrc(tw, NN * 16), 16 * idx, 0, w, wp);
  return Tw{w, wp};
}

// At N = 2048 (S = 256 in Q4) the last pass has only the spans 512 and 1024: its
// stage of span 256 was Q3's last, and is skipped (the bound of a skipped stage's
// successor is then larger than needed, which only widens the biased differences).
// LASTMUL = false (last pass only): the last stage (span N/2, one twiddle) leaves its
// differences X + B - Y unmultiplied, for an epilogue that folds the twiddle into its
// own constants.
template <int NP, int PASS, bool END, int NN = kNttN, bool LASTMUL = true, int EIN = 0>
__device__ __forceinline__ void inv_pass(uint64_t (&x)[NP][8], int tid,
                                         const uint64_t* const (&tw)[NP], const InvMod (&md)[NP]) {
  constexpr int S = InvLayout<PASS, NN>::S;
  static_assert(LASTMUL || PASS == 3, "only the last pass can leave its last stage open");
#pragma unroll
  for (int st = 0; st < 3; ++st) {
    const int sp = 1 << st;
    const uint32_t t = S * sp;
    if (PASS == 3 && t <= 256) continue;  // done in Q3 (N = 2048)
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (k & sp) continue;
#pragma unroll
      for (int r = 0; r < NP; ++r) {
        if (!LASTMUL && st == 2) {
          const uint64_t d = x[r][k] + (md[r].p8 << (2 + EIN)) - x[r][k + sp];
          x[r][k] += x[r][k + sp];
          x[r][k + sp] = d;
        } else {
          gs_bfly(x[r][k], x[r][k + sp], tw512<PASS, NN>(tw[r], t, k, tid), md[r].p8 << (2 + EIN),
                  md[r].pn);
        }
      }
    }
  }
  if (END) {
#pragma unroll
    for (int r = 0; r < NP; ++r)
#pragma unroll
      for (int k = 0; k < 2; ++k) x[r][k] = reduce_barrett(x[r][k], md[r]);
  }
}
template <int NP, int PASS, int EX, int NN = kNttN>
__device__ __forceinline__ void inv_store(uint64_t* lds, const uint64_t (&x)[NP][8], int tid) {
  const uint32_t base = InvLayout<PASS, NN>::base(tid);
#pragma unroll
  for (int r = 0; r < NP; ++r)
#pragma unroll
    for (int k = 0; k < 8; ++k)
      lds[r * InvSize<NN>::kLds + xaddr<EX>(base + InvLayout<PASS, NN>::S * k)] = x[r][k];
}
template <int NP, int PASS, int EX, int NN = kNttN>
__device__ __forceinline__ void inv_load(const uint64_t* lds, uint64_t (&x)[NP][8], int tid) {
  const uint32_t base = InvLayout<PASS, NN>::base(tid);
#pragma unroll
  for (int r = 0; r < NP; ++r)
#pragma unroll
    for (int k = 0; k < 8; ++k)
      x[r][k] = lds[r * InvSize<NN>::kLds + xaddr<EX>(base + InvLayout<PASS, NN>::S * k)];
}
// Orders a wave's LDS stores before its following loads (the exchange partners
// are lanes of the same wave; the LDS serves one wave's operations in order).
__device__ __forceinline__ void wave_exchange_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inverse transforms of NP primes without the 1/N factor: x[r] in layout Q1,
// bit-reversed order, below 8p_r -> layout Q4, natural order, congruent to the
// result mod p_r (below 512p_r, not reduced). lds holds NP exchange buffers. With
// LASTMUL = false, x[r][4..7] are congruent to the result divided by the last
// stage's twiddle (psi^-bitrev(1)).
template <int NP, int NN = kNttN, bool LASTMUL = true>
__device__ __forceinline__ void ntt_inverse(uint64_t (&x)[NP][8], uint64_t* lds,
                                            const uint64_t* const (&tw)[NP],
                                            const InvMod (&md)[NP], int tid) {
  inv_pass<NP, 0, false, NN>(x, tid, tw, md);
  __syncthreads();  // no wave still reads the previous transform's Q4 positions
  inv_store<NP, 0, 1, NN>(lds, x, tid);
  wave_exchange_fence();
  inv_load<NP, 1, 1, NN>(lds, x, tid);
  inv_pass<NP, 1, true, NN, true, 3>(x, tid, tw, md);
  wave_exchange_fence();  // every lane of the wave has read its Q2 positions
  inv_store<NP, 1, 2, NN>(lds, x, tid);
  wave_exchange_fence();
  inv_load<NP, 2, 2, NN>(lds, x, tid);
  inv_pass<NP, 2, false, NN>(x, tid, tw, md);
  __syncthreads();  // every wave is done with its own block
  inv_store<NP, 2, 3, NN>(lds, x, tid);
  __syncthreads();
  inv_load<NP, 3, 3, NN>(lds, x, tid);
  inv_pass<NP, 3, false, NN, LASTMUL, 3>(x, tid, tw, md);
}

// Plain radix-2 transforms in LDS for any ring degree N <= kNttN (one stage per
// barrier, exact Shoup products): the forward transforms of small rings. nthreads
// threads (threadIdx.x < nthreads) take part; all threads of the block meet the
// barriers.
// Cooley-Tukey, natural -> bit-reversed order, in place in LDS; inputs and outputs
// below 4p. Ends with a barrier.
__device__ inline void gen_forward(uint64_t* x, uint32_t N, const uint64_t* tw, uint64_t p,
                                   uint32_t nthreads) {
  for (uint32_t t = N / 2; t >= 1; t >>= 1) {
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < N / 2; j += nthreads) {
      const uint32_t pos = (j / t) * 2 * t + (j % t);
      uint64_t X = x[pos], Y = x[pos + t];
      ct_bfly(X, Y, ld_tw(tw, N / (2 * t) + pos / (2 * t)), p);
      x[pos] = X;
      x[pos + t] = Y;
    }
  }
  __syncthreads();
}

}  // namespace
}  // namespace rlwe
