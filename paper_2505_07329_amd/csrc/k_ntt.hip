// The mask part of Eq. (LWEdot) by number-theoretic transforms, for N = 4096.
//
// Per prime q_p the negacyclic product in Z_p[X]/(X^N + 1) is computed as
// INTT(NTT(a) * NTT(b)) with the psi-twisted transform (psi a primitive 2N-th
// root of unity): a Cooley-Tukey forward transform from natural to bit-reversed
// order and a Gentleman-Sande inverse from bit-reversed to natural order, both
// with the twist folded into their twiddles psi^(+-bitrev(k)); the factor 1/N
// of the inverse is folded into the output constants. For token t and output
// row j the polynomial C = sum_i A_{t,i} * w_hat_ij (Sec. 4.3, reversed weight
// encoding) gives the SampleExtract mask at N - 1 as a'[n] = C[N - 1 - n]
// (Sec. 3.2), so a'[n] is the inverse transform's coefficient N - 1 - n. The two
// residues are combined by CRT and switched to 2^32 exactly in the epilogue.
//
// A transform runs on 256 threads holding 16 residues each, in three passes of
// four radix-2 stages in registers with two exchanges through LDS. Residue
// positions per thread in the three layouts:
//   L1: 16 tid + k          (spans 1..8)
//   L2: 256 b + r + 16 k    (spans 16..128, b = tid / 16, r = tid % 16)
//   L3: tid + 256 k         (spans 256..2048)
// Arithmetic is lazy (Harvey): values stay below 4p, Shoup products below 2p.
#include "rlwe_internal.hpp"

namespace rlwe {
namespace {

constexpr int kN = kNttN;
constexpr int kThreads = 256;
constexpr int kLdsWords = kN + kN / 16;  // padded exchange buffer: position + position / 16

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
__device__ __forceinline__ uint64_t reduce4(uint64_t x, uint64_t p) {  // [0, 4p) -> [0, p)
  x = x >= 2 * p ? x - 2 * p : x;
  return x >= p ? x - p : x;
}
// forward butterfly: X, Y < 4p -> X + wY, X - wY (both < 4p)
__device__ __forceinline__ void ct_bfly(uint64_t& X, uint64_t& Y, const Tw& t, uint64_t p) {
  const uint64_t twop = 2 * p;
  const uint64_t x = X >= twop ? X - twop : X;
  const uint64_t v = mul_shoup(Y, t.w, t.wp, p);
  X = x + v;
  Y = x + twop - v;
}
// inverse butterfly: X, Y < 2p -> X + Y, (X - Y) w (both < 2p)
__device__ __forceinline__ void gs_bfly(uint64_t& X, uint64_t& Y, const Tw& t, uint64_t p) {
  const uint64_t twop = 2 * p;
  uint64_t s = X + Y;
  s = s >= twop ? s - twop : s;
  Y = mul_shoup(X + twop - Y, t.w, t.wp, p);
  X = s;
}

__device__ __forceinline__ uint32_t pad(uint32_t pos) { return pos + pos / 16; }

// Four stages of one pass on x[16] at positions base + STRIDE * k. FWD: spans
// STRIDE * 8, * 4, * 2, * 1 (Cooley-Tukey); otherwise spans STRIDE * 1 .. * 8
// (Gentleman-Sande). The twiddle of the pair at position pos, span t, is entry
// N / (2t) + pos / (2t) of the table.
template <bool FWD, int STRIDE>
__device__ __forceinline__ void pass4(uint64_t* x, uint32_t base, const uint64_t* tw, uint64_t p) {
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int sp = FWD ? (8 >> st) : (1 << st);  // distance in k
    const uint32_t t = STRIDE * sp;               // span in positions
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      if (k & sp) continue;
      const uint32_t pos = base + STRIDE * k;
      const Tw w = ld_tw(tw, kN / (2 * t) + pos / (2 * t));
      if (FWD)
        ct_bfly(x[k], x[k + sp], w, p);
      else
        gs_bfly(x[k], x[k + sp], w, p);
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
  pass4<true, 256>(x, 0, tw, p);  // spans 2048..256: twiddles do not depend on tid
  store_l3(lds, x, tid);
  __syncthreads();
  load_l2(lds, x, tid);
  pass4<true, 16>(x, 256 * (tid >> 4), tw, p);  // spans 128..16: r never reaches a block edge
  __syncthreads();
  store_l2(lds, x, tid);
  __syncthreads();
  load_l1(lds, x, tid);
  pass4<true, 1>(x, 16 * tid, tw, p);
  __syncthreads();
}

// Inverse transform without the 1/N factor: x in layout L1, bit-reversed order ->
// x in layout L3, natural order.
__device__ __forceinline__ void ntt_inverse(uint64_t* x, uint64_t* lds, const uint64_t* tw,
                                            uint64_t p, int tid) {
  pass4<false, 1>(x, 16 * tid, tw, p);
  store_l1(lds, x, tid);
  __syncthreads();
  load_l2(lds, x, tid);
  pass4<false, 16>(x, 256 * (tid >> 4), tw, p);
  __syncthreads();
  store_l2(lds, x, tid);
  __syncthreads();
  load_l3(lds, x, tid);
  pass4<false, 256>(x, 0, tw, p);
  __syncthreads();
}

}  // namespace

// NTT of the masks of every NTT-method product: one workgroup per (token, block,
// prime). ahat[((t L + i) P + p) N + pos], bit-reversed order, residues in [0, p).
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
  const uint64_t* A = bt->it[ii].ct + ((size_t)ti * 2 * P + p_idx) * kN;
  const int tid = threadIdx.x;
  uint64_t x[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) x[k] = A[tid + 256 * k];
  ntt_forward(x, lds, tw, p, tid);
  uint64_t* dst = bt->it[ii].ahat + (size_t)loc * kN + 16 * tid;
#pragma unroll
  for (int k = 0; k < 16; ++k) dst[k] = reduce4(x[k], p);
}

// Product kernel: one workgroup per (row j, tile of kTokTile tokens) of each item.
template <bool RAW>
__global__ void __launch_bounds__(kThreads) ntt_mask_kernel(Batch) {
  __shared__ uint64_t lds[kLdsWords];
  __shared__ uint64_t stash[kN];  // first prime's coefficients while the second is computed
  const BatchPtr bt = kernarg_batch();
  const uint32_t blk = linear_block();
  const uint32_t nb = bt->n;
  if (blk >= bt->mask_start[nb]) return;
  const uint32_t ii = find_item(bt->mask_start, nb, blk);
  const RingConst rc = kernarg_load(&bt->rc);
  const uint32_t P = rc.P, L = bt->it[ii].m.L, rows = bt->it[ii].m.rows, T = bt->it[ii].T;
  const uint32_t loc = blk - bt->mask_start[ii];
  const uint32_t j = loc % rows, t0 = (loc / rows) * kTokTile;
  const uint64_t* ahat = bt->it[ii].ahat;
  const uint64_t* what = bt->it[ii].what;  // [rows][L][P][N] (w, w') pairs
  void* out = bt->it[ii].out;
  const int tid = threadIdx.x;
  const uint32_t t_end = min(T, t0 + kTokTile);
  for (uint32_t t = t0; t < t_end; ++t) {
    for (uint32_t pi = 0; pi < P; ++pi) {
      const uint64_t p = rc.q[pi];
      uint64_t x[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = 0;
      for (uint32_t i = 0; i < L; ++i) {
        const uint64_t* a = ahat + (((size_t)t * L + i) * P + pi) * kN + 16 * tid;
        const uint64_t* w = what + 2 * ((((size_t)j * L + i) * P + pi) * kN + 16 * tid);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const uint64_t v = x[k] + mul_shoup(a[k], w[2 * k], w[2 * k + 1], p);
          x[k] = v >= 2 * p ? v - 2 * p : v;
        }
      }
      ntt_inverse(x, lds, bt->ntt.inv[pi], p, tid);
      // coefficient m = tid + 256 k of C; a'[N - 1 - m]
      if (RAW) {
        uint64_t* o = (uint64_t*)out + ((size_t)t * rows + j) * P * (kN + 1) + pi * (kN + 1);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const uint32_t m = tid + 256 * k;
          const uint64_t c = mul_shoup(x[k], bt->ntt.ninv[pi], bt->ntt.ninv_shoup[pi], p);
          o[kN - 1 - m] = c >= p ? c - p : c;
        }
      } else if (P == 2 && pi == 0) {
#pragma unroll
        for (int k = 0; k < 16; ++k) stash[tid + 256 * k] = x[k];
      } else {
        uint32_t* o = (uint32_t*)out + ((size_t)t * rows + j) * (kN + 1);
        const u128 Q = make_u128(rc.Q_hi, rc.Q_lo);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const uint32_t m = tid + 256 * k;
          u128 v;
          if (P == 1) {
            const uint64_t c = mul_shoup(x[k], bt->ntt.crt[0], bt->ntt.crt_shoup[0], p);
            v = c >= p ? c - p : c;
          } else {
            // y_p = c_p N^-1 (q / q_p)^-1 mod q_p; c = y_0 q_1 + y_1 q_0 mod q
            uint64_t y0 = mul_shoup(stash[m], bt->ntt.crt[0], bt->ntt.crt_shoup[0], rc.q[0]);
            y0 = y0 >= rc.q[0] ? y0 - rc.q[0] : y0;
            uint64_t y1 = mul_shoup(x[k], bt->ntt.crt[1], bt->ntt.crt_shoup[1], rc.q[1]);
            y1 = y1 >= rc.q[1] ? y1 - rc.q[1] : y1;
            v = (u128)y0 * rc.q[1] + (u128)y1 * rc.q[0];
            v = v >= Q ? v - Q : v;
          }
          o[kN - 1 - m] = switch_exact((i128)v, rc);
        }
      }
    }
  }
}

// NTT-domain weights: one workgroup per (row j, block i, prime p). Block i of row
// j is encoded reversed, w_hat[k] = w_j[iN + N - 1 - k] (zero past K), Sec. 4.3.
// what[(((j L + i) P + p) N + pos) * 2 + {0, 1}] = (value, Shoup companion).
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
    const uint32_t col = i * kN + kN - 1 - pos;
    const int v = col < m.k ? (int)m.w[(size_t)j * m.kw + col] : 0;
    x[k] = v < 0 ? p - (uint64_t)(-v) : (uint64_t)v;
  }
  ntt_forward(x, lds, ntt.fwd[p_idx], p, tid);
  uint64_t* dst = what + 2 * ((size_t)loc * kN + 16 * tid);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const uint64_t v = reduce4(x[k], p);
    dst[2 * k] = v;
    dst[2 * k + 1] = (uint64_t)(((u128)v << 64) / p);
  }
}

hipError_t launch_ntt_mask_fwd(const Batch& b, hipStream_t s) {
  const uint32_t blocks = b.fwd_start[b.n];
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(ntt_mask_fwd_kernel, grid_for(blocks), dim3(kThreads), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_ntt_mask(const Batch& b, hipStream_t s) {
  const uint32_t blocks = b.mask_start[b.n];
  if (blocks == 0) return hipSuccess;
  if (b.raw)
    hipLaunchKernelGGL(ntt_mask_kernel<true>, grid_for(blocks), dim3(kThreads), 0, s, b);
  else
    hipLaunchKernelGGL(ntt_mask_kernel<false>, grid_for(blocks), dim3(kThreads), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_ntt_weights(const MatArgs& m, const NttConst& ntt, const RingConst& rc,
                              uint64_t* what, hipStream_t s) {
  const uint32_t blocks = m.rows * m.L * rc.P;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(ntt_weights_kernel, dim3(blocks), dim3(kThreads), 0, s, m, ntt, rc, what);
  return hipGetLastError();
}

}  // namespace rlwe
