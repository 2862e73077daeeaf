// The mask part of Eq. (LWEdot) by number-theoretic transforms, for N = 4096 and
// N = 2048 (transform layouts and arithmetic: ntt_device.hpp).
#include "ntt_product.hpp"

namespace rlwe {

// NTT of the masks of every NTT-method product: one workgroup per (token, block,
// prime) (mask_forward).
__global__ void __launch_bounds__(kThreads) ntt_mask_fwd_kernel(Batch) {
  __shared__ uint64_t lds[kLdsWords];
  const BatchPtr bt = kernarg_batch();
  const uint32_t blk = linear_block();
  const uint32_t nb = bt->n;
  if (blk >= bt->fwd_start[nb]) return;
  const uint32_t ii = find_item(bt->fwd_start, nb, blk);
  mask_forward(bt, ii, blk - bt->fwd_start[ii], lds, threadIdx.x, true);
}

// NTT of the masks at N = 2048 (plain radix-2 transform, 256 threads).
template <int NN>
__global__ void __launch_bounds__(kThreads) ntt_mask_fwd_small_kernel(Batch) {
  __shared__ uint64_t lds[NN];
  const BatchPtr bt = kernarg_batch();
  const uint32_t blk = linear_block();
  const uint32_t nb = bt->n;
  if (blk >= bt->fwd_start[nb]) return;
  const uint32_t ii = find_item(bt->fwd_start, nb, blk);
  mask_forward_small<NN>(bt, ii, blk - bt->fwd_start[ii], lds, kThreads);
}

// Product kernel: one workgroup per tile (weight polynomial, token tile) of each
// item, NN / 8 threads. LC = 2: every item has exactly two input blocks; LC = 0: any
// number (a launch holds one class).
template <int OUT, int NP, int LC, int NN>
__global__ void __launch_bounds__(InvSize<NN>::kThreads, LC == 2 ? 4 : 1) ntt_mask_kernel(Batch) {
  __shared__ uint64_t lds[NP * InvSize<NN>::kLds];
  const BatchPtr bt = kernarg_batch();
  const uint32_t blk = linear_block();
  const uint32_t nb = bt->n;
  if (blk >= bt->mask_start[nb]) return;
  const uint32_t ii = find_item(bt->mask_start, nb, blk);
  ntt_product<OUT, NP, LC, NN>(bt, ii, blk - bt->mask_start[ii], lds);
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

// NTT-domain weights at N = 2048 (plain radix-2 transform, 256 threads): the encoding,
// layout and factor N^-1 of ntt_weights_kernel.
template <int NN>
__global__ void __launch_bounds__(kThreads) ntt_weights_small_kernel(MatArgs m, NttConst ntt,
                                                                     RingConst rc, uint64_t* what) {
  __shared__ uint64_t lds[NN];
  const uint32_t P = rc.P;
  const uint32_t loc = blockIdx.x;  // (j L + i) P + p
  const uint32_t p_idx = loc % P, ji = loc / P, i = ji % m.L, j = ji / m.L;
  const uint64_t p = rc.q[p_idx];
  for (uint32_t pos = threadIdx.x; pos < (uint32_t)NN; pos += kThreads) {
    const uint32_t rho = pos / m.slot, row = j * m.n_o + rho;
    const uint32_t col = i * NN + m.slot - 1 - (pos - rho * m.slot);
    const bool in = rho < m.n_o && row < m.rows && col < m.k;
    const int v = in ? (int)m.w[(size_t)row * m.kw + col] : 0;
    lds[pos] = v < 0 ? p - (uint64_t)(-v) : (uint64_t)v;
  }
  gen_forward(lds, NN, ntt.fwd[p_idx], p, kThreads);
  uint64_t* dst = what + (size_t)loc * NN;
  const uint64_t ninv = ntt.ninv[p_idx], ninv_shoup = ntt.ninv_shoup[p_idx];
  for (uint32_t pos = threadIdx.x; pos < (uint32_t)NN; pos += kThreads)
    dst[lane_major<NN>(pos)] = mulmod_shoup(reduce4(lds[pos], p), ninv, ninv_shoup, p);
}

hipError_t launch_ntt_mask_fwd(const Batch& b, hipStream_t s) {
  const uint32_t blocks = b.fwd_start[b.n];
  if (blocks == 0) return hipSuccess;
  if (b.rc.N == 2048)
    hipLaunchKernelGGL(ntt_mask_fwd_small_kernel<2048>, grid_for(blocks), dim3(kThreads), 0, s, b);
  else
    hipLaunchKernelGGL(ntt_mask_fwd_kernel, grid_for(blocks), dim3(kThreads), 0, s, b);
  return hipGetLastError();
}

template <int OUT, int LC, int NN>
void launch_ntt_mask_out(const Batch& b, dim3 g, hipStream_t s) {
  if (b.rc.P == 2)
    hipLaunchKernelGGL((ntt_mask_kernel<OUT, 2, LC, NN>), g, dim3(InvSize<NN>::kThreads), 0, s, b);
  else
    hipLaunchKernelGGL((ntt_mask_kernel<OUT, 1, LC, NN>), g, dim3(InvSize<NN>::kThreads), 0, s, b);
}

template <int LC, int NN>
void launch_ntt_mask_lc(const Batch& b, dim3 g, hipStream_t s) {
  if (b.gadget)
    launch_ntt_mask_out<2, LC, NN>(b, g, s);
  else if (b.raw)
    launch_ntt_mask_out<1, LC, NN>(b, g, s);
  else
    launch_ntt_mask_out<0, LC, NN>(b, g, s);
}

hipError_t launch_ntt_mask(const Batch& b, uint32_t lclass, hipStream_t s) {
  const uint32_t blocks = b.mask_start[b.n];
  if (blocks == 0) return hipSuccess;
  const dim3 g = grid_for(blocks);
  if (b.rc.N == 2048) {
    if (lclass == 2)
      launch_ntt_mask_lc<2, 2048>(b, g, s);
    else
      launch_ntt_mask_lc<0, 2048>(b, g, s);
  } else {
    if (lclass == 2)
      launch_ntt_mask_lc<2, kNttN>(b, g, s);
    else
      launch_ntt_mask_lc<0, kNttN>(b, g, s);
  }
  return hipGetLastError();
}

hipError_t launch_ntt_weights(const MatArgs& m, const NttConst& ntt, const RingConst& rc,
                              uint64_t* what, hipStream_t s) {
  const uint32_t blocks = (m.rows + m.n_o - 1) / m.n_o * m.L * rc.P;
  if (blocks == 0) return hipSuccess;
  if (rc.N == 2048)
    hipLaunchKernelGGL(ntt_weights_small_kernel<2048>, dim3(blocks), dim3(kThreads), 0, s, m, ntt,
                       rc, what);
  else
    hipLaunchKernelGGL(ntt_weights_kernel, dim3(blocks), dim3(kThreads), 0, s, m, ntt, rc, what);
  return hipGetLastError();
}

}  // namespace rlwe
