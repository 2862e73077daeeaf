// KeySwitch packing of LWE outputs into RLWE ciphertexts (Sec. 3.2 KeySwitching and
// Rotate, Sec. 4.3 Eq. (pack_rotate)): tuned kernels for N = 4096, plain ones for
// other ring degrees up to 4096.
//
// LWE ciphertext g n_pack + s (mask a, body b) goes to slot s of packed output g:
//   out_g = sum_s X^s ((0, b_s) - sum_i sum_m Decomp_m(a_s[i]) KSK_{i,m}).
// Both KeySwitching and the rotation are linear in the digits, so the sums are
// regrouped by key coefficient i and level m: with the digit polynomials
// D_{i,m}(X) = sum_s Decomp_m(a_s[i]) X^s,
//   A_g = -sum_{i,m} D_{i,m} KSK_{i,m}.A,   B_g = sum_s b_s X^s - sum_{i,m} D_{i,m} KSK_{i,m}.B
// in Z_q[X]/(X^N + 1), per prime. The key is resident in the NTT domain, so each
// D_{i,m} costs one forward transform per prime and two pointwise products; a
// group needs N ell transforms per prime and two inverse transforms per prime.
//
// Decomp is the gadget decomposition of TFHE: the coefficient c (CRT of its
// residues) is rounded to K = beta ell bits, a~ = round(c 2^K / q) mod 2^K, and
// a~ is written in signed base 2^beta (digits in [-2^(beta-1), 2^(beta-1)), most
// significant first). The rounding is exact (round_fast and round_exact, below). The signed digits
// are those of a~ + H, H = sum_m 2^(beta-1) 2^(beta m), less 2^(beta-1).
//
// Kernels (one pass covers up to kKsGroups output groups):
//   ks_digits_kernel  raw LWE masks [M][P][N+1] (or masks already rounded to 2^K by
//                     the product kernel, [M][N+P]) -> digits [group][i][m][slot]
//                     (int64), a 64 x 64 tile transpose through LDS
//   ks_accum_kernel   per (group, chunk of 64 key coefficients, prime): forward
//                     transforms of the digit polynomials, pointwise products
//                     with the resident key (value, Shoup companion pairs), partial
//                     sums [group][chunk][p][2][N] (lane-major positions)
//   ks_finish_kernel  per group: sum of the partials, inverse transforms, the
//                     factor 1/N, negation, bodies, optional switch to 2^k
#include "ks_round.hpp"
#include "ntt_device.hpp"

namespace rlwe {

namespace {

constexpr uint32_t kKsChunk = 64;                 // key coefficients per accumulate workgroup
constexpr uint32_t kKsChunks = kNttN / kKsChunk;  // chunks per group
constexpr uint32_t kTile = 64;                    // digit transpose tile (coefficients x slots)

typedef const __attribute__((address_space(4))) KsArgs* KsPtr;
__device__ __forceinline__ KsPtr ks_args() { return (KsPtr)__builtin_amdgcn_kernarg_segment_ptr(); }

// Index of LWE ciphertext j's body residue for prime r in the input.
__device__ __forceinline__ size_t body_index(KsPtr a, uint64_t j, uint32_t r) {
  const size_t N = a->rc.N, P = a->rc.P;
  return a->pre ? j * (N + P) + N + r : (j * P + r) * (N + 1) + N;
}

// Signed digits of a~ (most significant first): those of a~ + H less 2^(beta-1).
template <int ELL>
__device__ __forceinline__ void digits_of(KsPtr a, uint64_t at, int64_t (&d)[ELL]) {
  const uint32_t beta = a->kc.beta;
  const uint64_t v = (at & a->kc.kmask) + a->kc.H;
  const uint64_t bmask = (1ull << beta) - 1, half = 1ull << (beta - 1);
#pragma unroll
  for (int m = 0; m < ELL; ++m) {
    const uint32_t sh = beta * (ELL - 1 - m);
    d[m] = (int64_t)((v >> sh) & bmask) - (int64_t)half;
  }
}

// Forward butterfly without reductions (Harvey's lazy form, one step further): the
// product w Y mod p is taken below 4p for any 64-bit Y (truncated-quotient Shoup),
// so X, Y < B give X + wY and X + 4p - wY, both below B + 4p. From canonical inputs
// the twelve stages end below 49p < 2^60.
__device__ __forceinline__ void ct_bfly_lazy(uint64_t& X, uint64_t& Y, const Tw& t, uint64_t p4,
                                             uint64_t pn) {
  const uint64_t v = mul_shoup4(Y, t.w, t.wp, pn);
  const uint64_t x = X;
  X = x + v;
  Y = x + p4 - v;
}

// Forward pass of the 512-thread transform in layout PASS (InvLayout) on NC
// transforms of one prime at once: three Cooley-Tukey stages, spans 4S, 2S, S
// (twiddles as in the inverse, tw512, shared by the NC chains).
template <int NC, int PASS>
__device__ __forceinline__ void fwd512_pass(uint64_t (&x)[NC][8], int tid, const uint64_t* tw,
                                            uint64_t p4, uint64_t pn) {
  constexpr int S = InvLayout<PASS>::S;
#pragma unroll
  for (int st = 0; st < 3; ++st) {
    const int sp = 4 >> st;
    const uint32_t t = S * sp;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (k & sp) continue;
      const Tw w = tw512<PASS>(tw, t, k, tid);
#pragma unroll
      for (int c = 0; c < NC; ++c) ct_bfly_lazy(x[c][k], x[c][k + sp], w, p4, pn);
    }
  }
}

// NC forward transforms of one prime on 512 threads: x[c] in layout Q4 (positions tid
// + 512 k), natural order, canonical -> layout Q1 (8 tid + k), bit-reversed order,
// below 49p. The mirror of the inverse: Q4 -> Q3 crosses waves (between barriers),
// Q3 -> Q2 and Q2 -> Q1 stay inside each wave's block; lds holds NC exchange buffers
// of kInvLdsWords words, and a third barrier separates the Q3 loads of every wave
// from the wave-local stores that reuse the buffer.
template <int NC>
__device__ __forceinline__ void ntt_forward512(uint64_t (&x)[NC][8], uint64_t* lds,
                                               const uint64_t* tw, uint64_t p, int tid) {
  const uint64_t p4 = 4 * p, pn = 0 - p;
  fwd512_pass<NC, 3>(x, tid, tw, p4, pn);
  __syncthreads();  // no wave still reads the previous transforms' Q1 positions
  inv_store<NC, 3, 3>(lds, x, tid);
  __syncthreads();
  inv_load<NC, 2, 3>(lds, x, tid);
  fwd512_pass<NC, 2>(x, tid, tw, p4, pn);
  __syncthreads();  // every wave has read its Q3 positions
  inv_store<NC, 2, 2>(lds, x, tid);
  wave_exchange_fence();
  inv_load<NC, 1, 2>(lds, x, tid);
  fwd512_pass<NC, 1>(x, tid, tw, p4, pn);
  wave_exchange_fence();
  inv_store<NC, 1, 1>(lds, x, tid);
  wave_exchange_fence();
  inv_load<NC, 0, 1>(lds, x, tid);
  fwd512_pass<NC, 0>(x, tid, tw, p4, pn);
}

}  // namespace

// Digits: one workgroup per (group of the pass, tile of 64 key coefficients i,
// tile of 64 slots s). Loads run along i (coalesced rows of an LWE mask), stores
// along s (coalesced rows of a digit polynomial).
template <int NP, int ELL, bool PRE>
__global__ void __launch_bounds__(256) ks_digits_kernel(KsArgs) {
  __shared__ int64_t tile[kTile][kTile + 1];
  const KsPtr a = ks_args();
  const uint32_t N = a->rc.N;  // any N that is a multiple of 64
  const uint32_t tiles = N / kTile;
  const uint32_t blk = linear_block();
  const uint32_t gb = blk / (tiles * tiles);
  if (gb >= a->GB) return;
  const uint32_t it = (blk / tiles) % tiles, st = blk % tiles;
  const uint32_t i0 = it * kTile, s0 = st * kTile;
  const uint32_t g = a->g0 + gb;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  constexpr uint32_t ell = ELL;
  // LWE ciphertext j: raw residues [P][N+1], or (PRE) the rounded mask a~ [N] and the
  // bodies. Every load is issued before any rounding: rows past the last LWE
  // ciphertext (or past n_pack) read LWE 0 and are zeroed afterwards.
  const size_t stride = PRE ? N + NP : NP * (N + 1);
  uint64_t c0[16], c1[16];
  uint32_t okm = 0;
#pragma unroll
  for (int rep = 0; rep < 16; ++rep) {
    const uint32_t s = s0 + ty + 4 * rep;
    const uint64_t j = (uint64_t)g * a->n_pack + s;
    const bool ok = s < a->n_pack && j < a->M;
    okm |= (ok ? 1u : 0u) << rep;
    const uint64_t* row = a->lwe + (ok ? j : 0) * stride + i0 + tx;
    c0[rep] = row[0];
    c1[rep] = NP == 2 && !PRE ? row[N + 1] : 0;
  }
  uint64_t at[16];
  if (PRE) {
#pragma unroll
    for (int rep = 0; rep < 16; ++rep) at[rep] = c0[rep];
  } else {
    uint32_t nearm = 0;
#pragma unroll
    for (int rep = 0; rep < 16; ++rep) {
      bool nr;
      at[rep] = round_fast<NP>(&a->kc.rd, c0[rep], c1[rep], nr);
      nearm |= (nr ? 1u : 0u) << rep;
    }
    nearm &= okm;
    while (nearm) {  // rare: the exact rounding, residues read again
      const int k = __builtin_ctz(nearm);
      nearm &= nearm - 1;
      const uint64_t j = (uint64_t)g * a->n_pack + s0 + ty + 4 * k;
      const uint64_t* row = a->lwe + j * stride + i0 + tx;
      const uint64_t e = round_exact<NP>(&a->kc.rd, row[0], NP == 2 ? row[N + 1] : 0);
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) at[kk] = k == kk ? e : at[kk];
    }
  }
  int64_t d[16][ELL];
#pragma unroll
  for (int rep = 0; rep < 16; ++rep) {
    digits_of<ELL>(a, at[rep], d[rep]);
#pragma unroll
    for (int m = 0; m < ELL; ++m) d[rep][m] = (okm >> rep) & 1 ? d[rep][m] : 0;
  }
  int64_t* dst = a->dig + (size_t)gb * N * ell * N;
#pragma unroll
  for (int m = 0; m < ELL; ++m) {
    if (m) __syncthreads();  // the previous level's tile has been written out
#pragma unroll
    for (int rep = 0; rep < 16; ++rep) tile[tx][ty + 4 * rep] = d[rep][m];  // [i][s]
    __syncthreads();
#pragma unroll
    for (int rep = 0; rep < 16; ++rep) {
      const uint32_t il = ty + 4 * rep;
      dst[((size_t)(i0 + il) * ell + m) * N + s0 + tx] = tile[il][tx];
    }
  }
}

// Accumulation: one workgroup per (group of the pass, chunk of kKsChunk key
// coefficients, prime). Block b runs on XCD b mod 8; the mapping keeps every chunk
// on one XCD with the primes, then the groups varying fastest, so the workgroups
// that run together on an XCD read the same key polynomials from its L2, and the
// two primes of a group read each digit polynomial from HBM once.
template <int ELL>
__global__ void __launch_bounds__(kInvThreads, 4) ks_accum_kernel(KsArgs) {
  constexpr int NC = 2;  // key coefficients i, i + 1 transformed together (two chains)
  __shared__ uint64_t lds[NC * kInvLdsWords];
  const KsPtr a = ks_args();
  constexpr uint32_t ell = ELL;
  const uint32_t P = a->rc.P, GB = a->GB;
  const uint32_t blk = linear_block();
  const uint32_t rest = blk >> 3, xcd = blk & 7;
  const uint32_t r = rest % P, gb = (rest / P) % GB, cq = rest / P / GB;
  if (cq >= kKsChunks / 8) return;
  const uint32_t chunk = cq * 8 + xcd;
  const uint64_t p = a->rc.q[r];
  const uint64_t pn = 0 - p;
  const InvMod md{pn, 8 * p, a->ntt.bm[r]};
  const uint64_t* tw = a->ntt.fwd[r];
  const int tid0 = threadIdx.x;
  uint64_t accA[8], accB[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) accA[k] = accB[k] = 0;
  const int64_t* dig = a->dig + (size_t)gb * kN * ell * kN;
  for (uint32_t il = 0; il < kKsChunk; il += NC) {
    const uint32_t i = chunk * kKsChunk + il;
    for (uint32_t m = 0; m < ell; ++m) {
      int tid = tid0;
      asm volatile("" : "+v"(tid));
      uint64_t x[NC][8];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int64_t* dsrc = dig + ((size_t)(i + c) * ell + m) * kN + tid;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int64_t v = dsrc[512 * k];
          x[c][k] = v < 0 ? (uint64_t)(v + (int64_t)p) : (uint64_t)v;
        }
      }
      ntt_forward512<NC>(x, lds, tw, p, tid);
      // key (value, Shoup companion) pairs of mask and body at positions 8 tid + k; the
      // transformed digits (below 49p) are the free operand of the Shoup products
#pragma unroll
      for (int h = 0; h < 4; ++h) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const uint64_t* kh = a->khat + (((size_t)(i + c) * ell + m) * P + r) * 4 * kN;
          Tw ka[2], kb[2];
#pragma unroll
          for (int k = 0; k < 2; ++k) {  // lane-major key layout (lane_major)
            ka[k] = ld_tw(kh, (2 * h + k) * 512 + tid);
            kb[k] = ld_tw(kh + 2 * kN, (2 * h + k) * 512 + tid);
          }
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            accA[2 * h + k] += mul_shoup4(x[c][2 * h + k], ka[k].w, ka[k].wp, pn);
            accB[2 * h + k] += mul_shoup4(x[c][2 * h + k], kb[k].w, kb[k].wp, pn);
          }
        }
      }
    }
    if ((il & 15) == 16 - NC) {  // at most 64 products below 4p since the last reduction
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        accA[k] = reduce_barrett(accA[k], md);
        accB[k] = reduce_barrett(accB[k], md);
      }
    }
  }
  uint64_t* dst = a->part + (((size_t)gb * kKsChunks + chunk) * P + r) * 2 * kN + tid0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {  // lane-major: position 8 tid + k at k 512 + tid
    dst[512 * k] = reduce4(reduce_barrett(accA[k], md), p);
    dst[kN + 512 * k] = reduce4(reduce_barrett(accB[k], md), p);
  }
}

// Finish: one workgroup per group of the pass; the primes are transformed together.
template <bool RAW, int NP>
__global__ void __launch_bounds__(kInvThreads) ks_finish_kernel(KsArgs) {
  __shared__ uint64_t lds[NP * kInvLdsWords];
  const KsPtr a = ks_args();
  const uint32_t gb = linear_block();
  if (gb >= a->GB) return;
  const uint32_t g = a->g0 + gb;
  uint64_t p[NP];
  InvMod md[NP];
  const uint64_t* tw[NP];
#pragma unroll
  for (int r = 0; r < NP; ++r) {
    p[r] = a->rc.q[r];
    md[r] = InvMod{0 - p[r], 8 * p[r], a->ntt.bm[r]};
    tw[r] = a->ntt.inv[r];
  }
  const int tid = threadIdx.x;
  const uint32_t N = kN;
  for (uint32_t c = 0; c < 2; ++c) {
    uint64_t x[NP][8];
#pragma unroll
    for (int r = 0; r < NP; ++r) {
#pragma unroll
      for (int k = 0; k < 8; ++k) x[r][k] = 0;
      for (uint32_t ch = 0; ch < kKsChunks; ++ch) {
        const uint64_t* src =
            a->part + ((((size_t)gb * kKsChunks + ch) * NP + r) * 2 + c) * kN + tid;
#pragma unroll
        for (int k = 0; k < 8; ++k) x[r][k] += src[512 * k];  // 64 terms below p
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) x[r][k] = reduce_barrett(x[r][k], md[r]);
    }
    if (c) __syncthreads();  // the first component's transforms are done with lds
    ntt_inverse<NP>(x, lds, tw, md, tid);
    // coefficient n = tid + 512 k, natural order
    uint64_t v[NP][8];
#pragma unroll
    for (int r = 0; r < NP; ++r)
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        uint64_t t = mul_shoup(x[r][k], a->ntt.ninv[r], a->ntt.ninv_shoup[r], p[r]);
        t = t >= p[r] ? t - p[r] : t;
        uint64_t b = 0;
        if (c == 1) {
          const uint32_t s = tid + 512 * k;
          const uint64_t j = (uint64_t)g * a->n_pack + s;
          if (s < a->n_pack && j < a->M) b = a->lwe[body_index(a, j, r)];
        }
        v[r][k] = b >= t ? b - t : b + p[r] - t;  // (b - sum) mod p; b = 0 for the mask
      }
    if (RAW) {
      uint64_t* o = (uint64_t*)a->out + (((size_t)g * 2 + c) * NP) * N;
#pragma unroll
      for (int r = 0; r < NP; ++r)
#pragma unroll
        for (int k = 0; k < 8; ++k) o[(size_t)r * N + tid + 512 * k] = v[r][k];
    } else {
      uint32_t* o = (uint32_t*)a->out + ((size_t)g * 2 + c) * N;
      const RingConst rc = kernarg_load(&a->rc);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        u128 V = v[0][k];
        if (NP == 2) {
          const uint64_t y0 = mulmod_shoup(v[0][k], rc.crt_inv[0], rc.crt_inv_shoup[0], p[0]);
          const uint64_t y1 = mulmod_shoup(v[NP - 1][k], rc.crt_inv[NP - 1], rc.crt_inv_shoup[NP - 1], p[NP - 1]);
          V = (u128)y0 * p[NP - 1] + (u128)y1 * p[0];
          const u128 Q = make_u128(rc.Q_hi, rc.Q_lo);
          if (V >= Q) V -= Q;
        }
        o[tid + 512 * k] = switch_exact((i128)V, rc);
      }
    }
  }
}

// Key in the NTT domain: one workgroup per polynomial (i, m, c, p) of the key
// [N][ell][2][P][N] -> khat[((i ell + m) P + p) 2 + c][lane_major(pos)][2] for
// bit-reversed position pos: residue in [0, p) and its Shoup companion
// floor(v 2^64 / p).
__global__ void __launch_bounds__(kThreads) ksk_fwd_kernel(KsArgs) {
  __shared__ uint64_t lds[kLdsWords];
  const KsPtr a = ks_args();
  const uint32_t P = a->rc.P;
  const uint32_t loc = linear_block();  // ((i ell + m) 2 + c) P + p
  if (loc >= kN * a->kc.ell * 2 * P) return;
  const uint32_t r = loc % P, c = (loc / P) % 2, im = loc / (2 * P);
  const uint64_t p = a->rc.q[r];
  const int tid = threadIdx.x;
  const uint64_t* src = a->ksk_in + (size_t)loc * kN;
  uint64_t x[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) x[k] = src[tid + 256 * k];
  ntt_forward(x, lds, a->ntt.fwd[r], p, tid);
  uint64_t* dst = a->khat_out + (((size_t)im * P + r) * 2 + c) * kN * 2;
  const uint64_t r1 = a->ntt.rq[r][0], r0 = a->ntt.rq[r][1];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const uint64_t v = reduce4(x[k], p);
    // v floor(2^128 / p) / 2^64 is at most 1 below floor(v 2^64 / p)
    uint64_t cp = v * r1 + __umul64hi(v, r0);
    cp += (0 - cp * p) >= p ? 1 : 0;
    const uint32_t at = 2 * lane_major(16 * tid + k);
    dst[at] = v;
    dst[at + 1] = cp;
  }
}

// ---------------------------------------------------------------- other ring degrees
// For N != 4096 (64 <= N <= 4096) the same computation runs on 256 threads with
// plain radix-2 transforms in LDS, one stage per barrier, exact Shoup products (values
// below 4p forward, below 2p inverse), the key in natural bit-reversed order. These
// serve small rings (N = 2048 for one 54-bit prime); speed is not their aim.
namespace {
constexpr int kGenThreads = 256;

// Gentleman-Sande, bit-reversed -> natural order, without the factor 1/N, in place
// in LDS; inputs and outputs below 2p. Ends with a barrier.
__device__ void gen_inverse(uint64_t* x, uint32_t N, const uint64_t* tw, uint64_t p) {
  const uint64_t p2 = 2 * p;
  for (uint32_t t = 1; t < N; t <<= 1) {
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < N / 2; j += kGenThreads) {
      const uint32_t pos = (j / t) * 2 * t + (j % t);
      const uint64_t X = x[pos], Y = x[pos + t];
      const Tw w = ld_tw(tw, N / (2 * t) + pos / (2 * t));
      const uint64_t sum = X + Y;
      x[pos] = sum >= p2 ? sum - p2 : sum;
      x[pos + t] = mul_shoup(X + p2 - Y, w.w, w.wp, p);
    }
  }
  __syncthreads();
}
}  // namespace

// Key in the NTT domain, any N: khat[((i ell + m) P + p) 2 + c][pos][2], natural
// bit-reversed position order, residue and Shoup companion.
__global__ void __launch_bounds__(kGenThreads) ksk_fwd_generic(KsArgs) {
  __shared__ uint64_t x[kN];
  const KsPtr a = ks_args();
  const uint32_t N = a->rc.N, P = a->rc.P;
  const uint32_t loc = linear_block();  // ((i ell + m) 2 + c) P + p
  if (loc >= N * a->kc.ell * 2 * P) return;
  const uint32_t r = loc % P, c = (loc / P) % 2, im = loc / (2 * P);
  const uint64_t p = a->rc.q[r];
  const uint64_t* src = a->ksk_in + (size_t)loc * N;
  for (uint32_t n = threadIdx.x; n < N; n += kGenThreads) x[n] = src[n];
  gen_forward(x, N, a->ntt.fwd[r], p, kGenThreads);
  uint64_t* dst = a->khat_out + (((size_t)im * P + r) * 2 + c) * N * 2;
  const uint64_t r1 = a->ntt.rq[r][0], r0 = a->ntt.rq[r][1];
  for (uint32_t n = threadIdx.x; n < N; n += kGenThreads) {
    const uint64_t v = reduce4(x[n], p);
    uint64_t cp = v * r1 + __umul64hi(v, r0);
    cp += (0 - cp * p) >= p ? 1 : 0;
    dst[2 * n] = v;
    dst[2 * n + 1] = cp;
  }
}

// Accumulation, any N: one workgroup per (group of the pass, chunk of 64 key
// coefficients, prime); thread t holds positions t + 256 e, e < N / 256.
__global__ void __launch_bounds__(kGenThreads) ks_accum_generic(KsArgs) {
  __shared__ uint64_t x[kN];
  const KsPtr a = ks_args();
  const uint32_t N = a->rc.N, P = a->rc.P, GB = a->GB, ell = a->kc.ell;
  const uint32_t chunks = N / kKsChunk;
  const uint32_t blk = linear_block();
  const uint32_t r = blk % P, chunk = (blk / P) % chunks, gb = blk / P / chunks;
  if (gb >= GB) return;
  const uint64_t p = a->rc.q[r], pn = 0 - p;
  const InvMod md{pn, 8 * p, a->ntt.bm[r]};
  const uint64_t* tw = a->ntt.fwd[r];
  const uint32_t per = (N + kGenThreads - 1) / kGenThreads;  // at most 16
  const uint32_t tid = threadIdx.x;
  uint64_t accA[16], accB[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) accA[e] = accB[e] = 0;
  const int64_t* dig = a->dig + (size_t)gb * N * ell * N;
  for (uint32_t il = 0; il < kKsChunk; ++il) {
    const uint32_t i = chunk * kKsChunk + il;
    for (uint32_t m = 0; m < ell; ++m) {
      __syncthreads();  // the previous transform's products have read x
      const int64_t* dsrc = dig + ((size_t)i * ell + m) * N;
      for (uint32_t n = tid; n < N; n += kGenThreads) {
        const int64_t v = dsrc[n];
        x[n] = v < 0 ? (uint64_t)(v + (int64_t)p) : (uint64_t)v;
      }
      gen_forward(x, N, tw, p, kGenThreads);
      const uint64_t* kh = a->khat + (((size_t)i * ell + m) * P + r) * 4 * N;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const uint32_t pos = tid + kGenThreads * e;
        if ((uint32_t)e < per && pos < N) {
          const Tw ka = ld_tw(kh, pos), kb = ld_tw(kh + 2 * N, pos);
          accA[e] += mul_shoup4(x[pos], ka.w, ka.wp, pn);
          accB[e] += mul_shoup4(x[pos], kb.w, kb.wp, pn);
        }
      }
    }
    if ((il & 15) == 15) {  // at most 64 products below 4p since the last reduction
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        accA[e] = reduce_barrett(accA[e], md);
        accB[e] = reduce_barrett(accB[e], md);
      }
    }
  }
  uint64_t* dst = a->part + (((size_t)gb * chunks + chunk) * P + r) * 2 * N;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const uint32_t pos = tid + kGenThreads * e;
    if ((uint32_t)e < per && pos < N) {
      dst[pos] = reduce4(reduce_barrett(accA[e], md), p);
      dst[N + pos] = reduce4(reduce_barrett(accB[e], md), p);
    }
  }
}

// Finish, any N: one workgroup per group of the pass.
template <bool RAW, int NP>
__global__ void __launch_bounds__(kGenThreads) ks_finish_generic(KsArgs) {
  __shared__ uint64_t x[NP][kN];
  const KsPtr a = ks_args();
  const uint32_t gb = linear_block();
  if (gb >= a->GB) return;
  const uint32_t g = a->g0 + gb, N = a->rc.N, chunks = N / kKsChunk;
  const uint32_t tid = threadIdx.x;
  for (uint32_t c = 0; c < 2; ++c) {
    __syncthreads();  // the previous component's outputs have been read
#pragma unroll
    for (int r = 0; r < NP; ++r) {
      const uint64_t p = a->rc.q[r];
      const InvMod md{0 - p, 8 * p, a->ntt.bm[r]};
      for (uint32_t n = tid; n < N; n += kGenThreads) {
        uint64_t v = 0;
        for (uint32_t ch = 0; ch < chunks; ++ch)  // at most 64 terms below p
          v += a->part[((((size_t)gb * chunks + ch) * NP + r) * 2 + c) * N + n];
        x[r][n] = reduce4(reduce_barrett(v, md), p);
      }
    }
#pragma unroll
    for (int r = 0; r < NP; ++r) gen_inverse(x[r], N, a->ntt.inv[r], a->rc.q[r]);
    for (uint32_t n = tid; n < N; n += kGenThreads) {
      uint64_t v[NP];
#pragma unroll
      for (int r = 0; r < NP; ++r) {
        const uint64_t p = a->rc.q[r];
        uint64_t t = mul_shoup(x[r][n], a->ntt.ninv[r], a->ntt.ninv_shoup[r], p);
        t = t >= p ? t - p : t;
        uint64_t b = 0;
        const uint64_t j = (uint64_t)g * a->n_pack + n;
        if (c == 1 && n < a->n_pack && j < a->M) b = a->lwe[body_index(a, j, r)];
        v[r] = b >= t ? b - t : b + p - t;  // (b - sum) mod p; b = 0 for the mask
      }
      if (RAW) {
        uint64_t* o = (uint64_t*)a->out + (((size_t)g * 2 + c) * NP) * N;
#pragma unroll
        for (int r = 0; r < NP; ++r) o[(size_t)r * N + n] = v[r];
      } else {
        const RingConst rc = kernarg_load(&a->rc);
        u128 V = v[0];
        if (NP == 2) {
          const uint64_t y0 = mulmod_shoup(v[0], rc.crt_inv[0], rc.crt_inv_shoup[0], rc.q[0]);
          const uint64_t y1 =
              mulmod_shoup(v[NP - 1], rc.crt_inv[NP - 1], rc.crt_inv_shoup[NP - 1], rc.q[NP - 1]);
          V = (u128)y0 * rc.q[NP - 1] + (u128)y1 * rc.q[0];
          const u128 Q = make_u128(rc.Q_hi, rc.Q_lo);
          if (V >= Q) V -= Q;
        }
        ((uint32_t*)a->out)[((size_t)g * 2 + c) * N + n] = switch_exact((i128)V, rc);
      }
    }
  }
}

hipError_t launch_ksk_fwd(const KsArgs& a, hipStream_t s) {
  const uint32_t blocks = a.rc.N * a.kc.ell * 2 * a.rc.P;
  if (a.rc.N == kN)
    hipLaunchKernelGGL(ksk_fwd_kernel, grid_for(blocks), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(ksk_fwd_generic, grid_for(blocks), dim3(kGenThreads), 0, s, a);
  return hipGetLastError();
}

template <bool PRE>
hipError_t launch_ks_digits_pre(const KsArgs& a, dim3 g, hipStream_t s) {
  switch (a.rc.P * 8 + a.kc.ell) {
    case 9: hipLaunchKernelGGL((ks_digits_kernel<1, 1, PRE>), g, dim3(256), 0, s, a); break;
    case 10: hipLaunchKernelGGL((ks_digits_kernel<1, 2, PRE>), g, dim3(256), 0, s, a); break;
    case 11: hipLaunchKernelGGL((ks_digits_kernel<1, 3, PRE>), g, dim3(256), 0, s, a); break;
    case 12: hipLaunchKernelGGL((ks_digits_kernel<1, 4, PRE>), g, dim3(256), 0, s, a); break;
    case 17: hipLaunchKernelGGL((ks_digits_kernel<2, 1, PRE>), g, dim3(256), 0, s, a); break;
    case 18: hipLaunchKernelGGL((ks_digits_kernel<2, 2, PRE>), g, dim3(256), 0, s, a); break;
    case 19: hipLaunchKernelGGL((ks_digits_kernel<2, 3, PRE>), g, dim3(256), 0, s, a); break;
    case 20: hipLaunchKernelGGL((ks_digits_kernel<2, 4, PRE>), g, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ks_digits(const KsArgs& a, hipStream_t s) {
  const uint32_t tiles = a.rc.N / kTile;
  const uint32_t blocks = a.GB * tiles * tiles;
  const dim3 g = grid_for(blocks);
  return a.pre ? launch_ks_digits_pre<true>(a, g, s) : launch_ks_digits_pre<false>(a, g, s);
}

hipError_t launch_ks_accum(const KsArgs& a, hipStream_t s) {
  if (a.rc.N != kN) {
    const uint32_t blocks = a.GB * (a.rc.N / kKsChunk) * a.rc.P;
    hipLaunchKernelGGL(ks_accum_generic, grid_for(blocks), dim3(kGenThreads), 0, s, a);
    return hipGetLastError();
  }
  const uint32_t blocks = a.GB * kKsChunks * a.rc.P;  // kKsChunks P is a multiple of 8
  const dim3 g = grid_for(blocks);
  switch (a.kc.ell) {
    case 1: hipLaunchKernelGGL(ks_accum_kernel<1>, g, dim3(kInvThreads), 0, s, a); break;
    case 2: hipLaunchKernelGGL(ks_accum_kernel<2>, g, dim3(kInvThreads), 0, s, a); break;
    case 3: hipLaunchKernelGGL(ks_accum_kernel<3>, g, dim3(kInvThreads), 0, s, a); break;
    case 4: hipLaunchKernelGGL(ks_accum_kernel<4>, g, dim3(kInvThreads), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ks_finish(const KsArgs& a, hipStream_t s) {
  const dim3 g = grid_for(a.GB);
  if (a.rc.N != kN) {
    if (a.rc.P == 2) {
      if (a.raw)
        hipLaunchKernelGGL((ks_finish_generic<true, 2>), g, dim3(kGenThreads), 0, s, a);
      else
        hipLaunchKernelGGL((ks_finish_generic<false, 2>), g, dim3(kGenThreads), 0, s, a);
    } else {
      if (a.raw)
        hipLaunchKernelGGL((ks_finish_generic<true, 1>), g, dim3(kGenThreads), 0, s, a);
      else
        hipLaunchKernelGGL((ks_finish_generic<false, 1>), g, dim3(kGenThreads), 0, s, a);
    }
    return hipGetLastError();
  }
  if (a.rc.P == 2) {
    if (a.raw)
      hipLaunchKernelGGL((ks_finish_kernel<true, 2>), g, dim3(kInvThreads), 0, s, a);
    else
      hipLaunchKernelGGL((ks_finish_kernel<false, 2>), g, dim3(kInvThreads), 0, s, a);
  } else {
    if (a.raw)
      hipLaunchKernelGGL((ks_finish_kernel<true, 1>), g, dim3(kInvThreads), 0, s, a);
    else
      hipLaunchKernelGGL((ks_finish_kernel<false, 1>), g, dim3(kInvThreads), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace rlwe
