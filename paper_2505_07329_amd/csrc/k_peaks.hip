// Measured peak rates of the operations the kernels are built from, for roofline
// accounting: 32-bit multiply issue, the 54-bit Shoup modular product and the lazy
// Gentleman-Sande butterfly of the NTT product kernel, and int8 matrix-core products.
// Every kernel keeps its operands in registers (independent dependency chains, enough
// waves per SIMD to hide latency) and writes one word per thread so nothing is removed.
#include <algorithm>

#include "ntt_device.hpp"
#include "rlwe.h"

namespace rlwe {
namespace {

constexpr int kPeakThreads = 256;
constexpr uint32_t kPeakIters = 2048;

// 8 chains x 8 unrolled v_mul_lo_u32 per iteration: 64 VALU instructions.
__global__ void __launch_bounds__(kPeakThreads) peak_mul32_kernel(uint32_t* out, uint32_t iters) {
  uint32_t x[8];
  const uint32_t c = 0x9E3779B1u ^ threadIdx.x;
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = threadIdx.x * 8 + k + 1;
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int k = 0; k < 8; ++k) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(x[k]) : "v"(c));
  }
  uint32_t r = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) r ^= x[k];
  out[blockIdx.x * kPeakThreads + threadIdx.x] = r;
}

// 8 chains of the truncated-quotient Shoup product (mul_shoup4, the product kernel's),
// in either instruction form (SPLIT); the faster one is reported.
template <bool SPLIT>
__global__ void __launch_bounds__(kPeakThreads) peak_modmul_kernel(uint64_t* out, uint32_t iters,
                                                                   uint64_t p, uint64_t w,
                                                                   uint64_t wp) {
  uint64_t a[8];
  const uint64_t pn = 0 - p;
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = (threadIdx.x * 8 + k + 1) % p;
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      a[k] = mul_shoup4<SPLIT>(a[k], w, wp, pn);
      asm volatile("" : "+v"(a[k]));  // opaque: no cross-iteration value analysis
    }
  }
  uint64_t r = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) r ^= a[k];
  out[blockIdx.x * kPeakThreads + threadIdx.x] = r;
}

// 8 independent lazy Gentleman-Sande butterflies per iteration (gs_bfly, the inverse
// transform's: a biased difference, a sum and a truncated-quotient Shoup product).
// The sums wrap modulo 2^64 over many iterations; the instruction stream is the
// kernel's, in either form of the product (the faster is reported).
template <bool SPLIT>
__global__ void __launch_bounds__(kPeakThreads) peak_bfly_kernel(uint64_t* out, uint32_t iters,
                                                                 uint64_t p, uint64_t w,
                                                                 uint64_t wp) {
  uint64_t x[16];
  const uint64_t pn = 0 - p, B = 8 * p;
  const Tw tw{w, wp};
#pragma unroll
  for (int k = 0; k < 16; ++k) x[k] = (threadIdx.x * 16 + k + 1) % p;
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      gs_bfly<SPLIT>(x[k], x[k + 8], tw, B, pn);
      asm volatile("" : "+v"(x[k]), "+v"(x[k + 8]));  // opaque, as above
    }
  }
  uint64_t r = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) r ^= x[k];
  out[blockIdx.x * kPeakThreads + threadIdx.x] = r;
}

typedef int32_t v4i __attribute__((ext_vector_type(4)));
typedef int32_t v16i __attribute__((ext_vector_type(16)));

// 4 independent accumulators of v_mfma_i32_32x32x32_i8 (2 * 32^3 int8 operations each).
__global__ void __launch_bounds__(kPeakThreads) peak_mfma_kernel(int32_t* out, uint32_t iters) {
  v16i acc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] = v16i{0};
  const v4i a = {(int32_t)threadIdx.x, 3, 5, 7}, b = {11, (int32_t)threadIdx.x, 13, 17};
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[k], 0, 0, 0);
  }
  int32_t r = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int e = 0; e < 16; ++e) r ^= acc[k][e];
  out[blockIdx.x * kPeakThreads + threadIdx.x] = r;
}

}  // namespace
}  // namespace rlwe

namespace rlwe {

int measure_peaks(int hip_device, rlwe_peaks* out, const char** why) {
  *why = "";
  *out = rlwe_peaks{};
  hipDeviceProp_t prop;
  if (hipSetDevice(hip_device) != hipSuccess || hipGetDeviceProperties(&prop, hip_device) != hipSuccess) {
    *why = "hipSetDevice / hipGetDeviceProperties failed";
    return RLWE_EHIP;
  }
  const uint32_t blocks = (uint32_t)prop.multiProcessorCount * 16;  // 16 blocks of 4 waves per CU
  const size_t words = (size_t)blocks * kPeakThreads;
  void* buf = nullptr;
  if (hipMalloc(&buf, words * 8) != hipSuccess) {
    *why = "hipMalloc failed";
    return RLWE_ENOMEM;
  }
  hipEvent_t a = nullptr, b = nullptr;
  int rc = RLWE_OK;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) rc = RLWE_EHIP;
  const uint64_t p = 18014398509309953ull;  // a 54-bit prime; the timing does not depend on it
  const uint64_t w = 0x2F0F0F0F0F0F0ull % p, wp = (uint64_t)(((unsigned __int128)w << 64) / p);
  // best of three timed launches after one untimed launch; rate = work / time
  auto best_ms = [&](auto launch) {
    float best = -1.f;
    launch();
    for (int rep = 0; rep < 3 && rc == RLWE_OK; ++rep) {
      float ms = 0.f;
      if (hipEventRecord(a, 0) != hipSuccess) rc = RLWE_EHIP;
      launch();
      if (hipGetLastError() != hipSuccess || hipEventRecord(b, 0) != hipSuccess ||
          hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess)
        rc = RLWE_EHIP;
      if (rc == RLWE_OK && (best < 0.f || ms < best)) best = ms;
    }
    return best;
  };
  const double threads = (double)words;
  const uint32_t it = kPeakIters;
  if (rc == RLWE_OK) {
    const float ms = best_ms([&] {
      hipLaunchKernelGGL(peak_mul32_kernel, dim3(blocks), dim3(kPeakThreads), 0, 0, (uint32_t*)buf, it);
    });
    out->mul32_lane_ops = threads * it * 64 / (ms * 1e-3);
    // both instruction forms of the modular product; the faster time of each kernel
    const float ms2 = std::min(best_ms([&] {
      hipLaunchKernelGGL(peak_modmul_kernel<true>, dim3(blocks), dim3(kPeakThreads), 0, 0, (uint64_t*)buf, it, p, w, wp);
    }), best_ms([&] {
      hipLaunchKernelGGL(peak_modmul_kernel<false>, dim3(blocks), dim3(kPeakThreads), 0, 0, (uint64_t*)buf, it, p, w, wp);
    }));
    out->modmul = threads * it * 8 / (ms2 * 1e-3);
    const float ms3 = std::min(best_ms([&] {
      hipLaunchKernelGGL(peak_bfly_kernel<true>, dim3(blocks), dim3(kPeakThreads), 0, 0, (uint64_t*)buf, it, p, w, wp);
    }), best_ms([&] {
      hipLaunchKernelGGL(peak_bfly_kernel<false>, dim3(blocks), dim3(kPeakThreads), 0, 0, (uint64_t*)buf, it, p, w, wp);
    }));
    out->butterfly = threads * it * 8 / (ms3 * 1e-3);
    const uint32_t mit = 2 * it;
    const float ms4 = best_ms([&] {
      hipLaunchKernelGGL(peak_mfma_kernel, dim3(blocks), dim3(kPeakThreads), 0, 0, (int32_t*)buf, mit);
    });
    // one 32x32x32 product per wave and accumulator: 65536 operations
    out->mfma_int8_ops = (threads / 64) * mit * 4 * 65536.0 / (ms4 * 1e-3);
    out->clock_mhz = prop.clockRate / 1000.0;
    out->compute_units = (uint32_t)prop.multiProcessorCount;
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(buf);
  if (rc != RLWE_OK) *why = "a timing kernel or event failed";
  return rc;
}

}  // namespace rlwe
