// Persistent batch kernel: every step of a batch of products on the NTT method in one
// launch (Eq. (LWEdot) and ModulusSwitch for all products of, e.g., a transformer
// layer, forward and transposed, with uneven token counts).
//
// A grid of at most two workgroups per compute unit takes work from one queue,
// in order, through an atomic counter:
//   [0, F)              transform units (item x, token t, block i): the transforms of
//                       A_i for every prime (mask_forward, one prime per half of the
//                       workgroup);
//   [F, F + G)          digit units: two blocks of 256 body coefficients each, their
//                       balanced base-255 digit planes (prep_coeff);
//   [F + G, F + G + R)  product tiles (weight polynomial, token tile) of every item
//                       (ntt_product);
//   [F + G + R, total)  body blocks, two per work item (body_block).
// A product tile of item x first waits until the T_x L_x transform units of x are
// done, a body block until the digit units of its item are. Units never wait, and
// every unit lies before every tile and body in the queue, so a waited-for unit was
// taken by a workgroup that is running and will finish it: the waits always end. They
// are bounded nonetheless (kSpinLimit polls, then an error flag is raised and the work
// goes on), so every wave reaches the end of the kernel. The last workgroup to leave
// resets the counters for the next launch (graph replays included): no memset is
// needed between launches.
#include "ntt_product.hpp"
#include "prep_device.hpp"

namespace rlwe {

namespace {

constexpr uint32_t kSpinLimit = 1u << 22;  // polls: a few seconds at most

// Counts a finished unit once every thread's stores of it are visible on the device:
// the barrier waits for the workgroup's stores, the release of the count makes them
// visible device-wide (one write-back per counting thread, `counts` set in one thread
// per count).
__device__ __forceinline__ void signal_done(uint32_t* cnt, bool counts) {
  __syncthreads();
  if (counts) __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until the count of item x reaches need, then orders the workgroup's later loads
// after the producers' stores. The count is polled without ordering (an acquire per
// poll would invalidate the caches each time, and with them the weights the product
// tiles share in L2) and acquired once; `ready` remembers the items a workgroup has
// already acquired, which need neither wait nor fence again. The wait is bounded (and
// skipped once *err is set): every wave reaches the end of the kernel.
__device__ __forceinline__ void wait_done(const uint32_t* cnt, uint32_t need, uint32_t* err,
                                          uint32_t x, uint32_t& ready) {
  if (ready & (1u << x)) return;  // uniform: the same bit in every thread
  if (threadIdx.x == 0) {
    uint32_t spins = 0;
    while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
      if (++spins > kSpinLimit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  ready |= 1u << x;
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
  const uint32_t F = bt0->unit_start[nb], G = (bt0->prep_start[nb] + 1) / 2;
  const uint32_t R = bt0->mask_start[nb];
  const uint32_t total = F + G + R + (bt0->body_start[nb] + 1) / 2;
  uint32_t ready = 0;  // items whose transforms (bit x) and digits (bit 16 + x) are acquired
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
    if (w < F) {
      const uint32_t x = find_item(bt->unit_start, nb, w);
      const uint32_t ti = w - bt->unit_start[x];  // t L + i
      const uint32_t half = tid >> 8;
      mask_forward(bt, x, ti * NP + half, lds + half * kLdsWords, tid & 255, half < (uint32_t)NP);
      signal_done(&sy[kSyncDone + x], tid == 0);
    } else if (w < F + G) {
      // prep blocks 2 (w - F) and 2 (w - F) + 1: N / 256 per (token, block)
      const uint32_t v = 2 * (w - F) + (tid >> 8);
      const uint32_t per = bt->rc.N >> 8;
      const bool live = v < bt->prep_start[nb];
      const uint32_t x = find_item(bt->prep_start, nb, live ? v : 0);
      if (live) {
        const uint32_t loc = v - bt->prep_start[x];
        const uint32_t ti = loc / per;
        prep_coeff<D>(bt, x, ti, (loc - ti * per) * 256 + (tid & 255));
      }
      // one count per prep block: threads 0 and 256 count their halves' blocks
      signal_done(&sy[kSyncPrep + x], live && (tid & 255) == 0);
    } else if (w < F + G + R) {
      const uint32_t r = w - F - G;
      const uint32_t x = find_item(bt->mask_start, nb, r);
      wait_done(&sy[kSyncDone + x], bt->it[x].T * bt->it[x].m.L, &sy[kSyncErr], x, ready);
      if (bt->it[x].m.L == 2)
        ntt_product<OUT, NP, 2>(bt, x, r - bt->mask_start[x], lds);
      else
        ntt_product<OUT, NP, 0>(bt, x, r - bt->mask_start[x], lds);
    } else {
      const uint32_t v0 = 2 * (w - F - G - R);
      const uint32_t nbody = bt->body_start[nb];
      const uint32_t x0 = find_item(bt->body_start, nb, v0);
      wait_done(&sy[kSyncPrep + x0], bt->prep_start[x0 + 1] - bt->prep_start[x0], &sy[kSyncErr],
                16 + x0, ready);
      if (v0 + 1 < nbody) {
        const uint32_t x1 = find_item(bt->body_start, nb, v0 + 1);
        wait_done(&sy[kSyncPrep + x1], bt->prep_start[x1 + 1] - bt->prep_start[x1],
                  &sy[kSyncErr], 16 + x1, ready);
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
      for (uint32_t x = 0; x < nb; ++x) {
        __hip_atomic_store(&sy[kSyncDone + x], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&sy[kSyncPrep + x], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
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
