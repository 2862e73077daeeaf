// Persistent batch kernel: every step of a batch of products on the NTT method in one
// launch (Eq. (LWEdot) and ModulusSwitch for all products of, e.g., a transformer
// layer, forward and transposed, with uneven token counts).
//
// A grid of at most two workgroups per compute unit takes work from one queue,
// in order, through an atomic counter:
//   [0, U)          units (item x, token t, block i): the body digit planes of B_i
//                   (prep_coeff) and the transforms of A_i for every prime
//                   (mask_forward, one prime per half of the workgroup);
//   [U, U + R)      product tiles (weight polynomial, token tile) of every item
//                   (ntt_product);
//   [U + R, total)  body blocks, two per work item (body_block).
// A product tile or body block of item x first waits until the T_x L_x units of x
// are done. Units never wait, and every unit lies before every tile in the queue, so
// a waited-for unit was taken by a workgroup that is running and will finish it:
// the waits always end. They are bounded nonetheless (kSpinLimit polls, then an error
// flag is raised and the work goes on), so every wave reaches the end of the kernel.
// The last workgroup to leave resets the counters for the next launch (graph replays
// included): no memset is needed between launches.
#include "ntt_product.hpp"
#include "prep_device.hpp"

namespace rlwe {

namespace {

constexpr uint32_t kSpinLimit = 1u << 22;  // polls: a few seconds at most

// Makes every thread's stores of a finished unit visible on the device, then counts it.
__device__ __forceinline__ void signal_done(uint32_t* cnt) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until *cnt reaches need (bounded; not at all once *err is set), then orders the
// workgroup's later loads after the producers' stores.
__device__ __forceinline__ void wait_done(const uint32_t* cnt, uint32_t need, uint32_t* err) {
  if (threadIdx.x == 0) {
    uint32_t spins = 0;
    while (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
      // after one wait has given up, later ones do not wait (the launch still drains)
      if (++spins > kSpinLimit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

}  // namespace

template <int OUT, int NP>
__global__ void __launch_bounds__(kInvThreads, 4) batch_persist_kernel(Batch) {
  constexpr int D = NP == 1 ? 7 : 14;  // balanced base-255 digits of the body
  constexpr int kFwdWords = 2 * kLdsWords;  // two 256-thread forward transforms side by side
  constexpr int kWords = NP * kInvLdsWords > kFwdWords ? NP * kInvLdsWords : kFwdWords;
  __shared__ uint64_t lds[kWords];
  __shared__ uint32_t s_work;
  const BatchPtr bt0 = kernarg_batch();
  uint32_t* sy = bt0->sync;
  const uint32_t nb = bt0->n;
  const uint32_t U = bt0->unit_start[nb], R = bt0->mask_start[nb];
  const uint32_t total = U + R + (bt0->body_start[nb] + 1) / 2;
  const uint32_t N = bt0->rc.N;
  for (;;) {
    // the thread index is opaque per work item: thread-dependent addresses are formed
    // where they are used instead of being hoisted out of the queue loop (and spilled)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    BatchPtr bt = bt0;  // opaque too: kernarg constants are loaded where they are used
    asm volatile("" : "+s"(bt));
    if (tid == 0) s_work = __hip_atomic_fetch_add(&sy[kSyncHead], 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const uint32_t w = s_work;
    __syncthreads();  // s_work is read by all before thread 0 overwrites it
    if (w >= total) break;
    if (w < U) {
      const uint32_t x = find_item(bt->unit_start, nb, w);
      const uint32_t ti = w - bt->unit_start[x];  // t L + i
      for (uint32_t k = tid; k < N; k += kInvThreads) prep_coeff<D>(bt, x, ti, k);
      const uint32_t half = tid >> 8;
      mask_forward(bt, x, ti * NP + half, lds + half * kLdsWords, tid & 255, half < (uint32_t)NP);
      signal_done(&sy[kSyncDone + x]);
    } else if (w < U + R) {
      const uint32_t r = w - U;
      const uint32_t x = find_item(bt->mask_start, nb, r);
      wait_done(&sy[kSyncDone + x], bt->it[x].T * bt->it[x].m.L, &sy[kSyncErr]);
      if (bt->it[x].m.L == 2)
        ntt_product<OUT, NP, 2>(bt, x, r - bt->mask_start[x], lds);
      else
        ntt_product<OUT, NP, 0>(bt, x, r - bt->mask_start[x], lds);
    } else {
      const uint32_t v0 = 2 * (w - U - R);
      const uint32_t nbody = bt->body_start[nb];
      const uint32_t x0 = find_item(bt->body_start, nb, v0);
      wait_done(&sy[kSyncDone + x0], bt->it[x0].T * bt->it[x0].m.L, &sy[kSyncErr]);
      if (v0 + 1 < nbody) {
        const uint32_t x1 = find_item(bt->body_start, nb, v0 + 1);
        if (x1 != x0) wait_done(&sy[kSyncDone + x1], bt->it[x1].T * bt->it[x1].m.L, &sy[kSyncErr]);
      }
      const uint32_t v = v0 + (tid >> 8);
      if (v < nbody) {
        const uint32_t x = find_item(bt->body_start, nb, v);
        body_block<D, OUT == 1>(bt, x, v - bt->body_start[x], tid & 255);
      }
    }
  }
  // the last workgroup out resets the queue for the next launch
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t grid = gridDim.x * gridDim.y;
    const uint32_t done = __hip_atomic_fetch_add(&sy[kSyncExit], 1u, __ATOMIC_ACQ_REL,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    if (done == grid - 1) {
      for (uint32_t x = 0; x < nb; ++x)
        __hip_atomic_store(&sy[kSyncDone + x], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&sy[kSyncHead], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&sy[kSyncExit], 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <int OUT, int NP>
static void launch_persist_np(const Batch& b, uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL((batch_persist_kernel<OUT, NP>), dim3(grid), dim3(kInvThreads), 0, s, b);
}

hipError_t launch_persist(const Batch& b, uint32_t grid, hipStream_t s) {
  if (grid == 0) return hipSuccess;
  if (b.rc.P == 2) {
    if (b.raw)
      launch_persist_np<1, 2>(b, grid, s);
    else
      launch_persist_np<0, 2>(b, grid, s);
  } else {
    if (b.raw)
      launch_persist_np<1, 1>(b, grid, s);
    else
      launch_persist_np<0, 1>(b, grid, s);
  }
  return hipGetLastError();
}

}  // namespace rlwe
