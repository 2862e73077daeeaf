// Host runtime behind include/rlwe.h: parameter validation, CRT and switching
// constants, resident weights, workspace and kernel launches.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rlwe.h"
#include "rlwe_internal.hpp"
#include "tune_cache.hpp"

using namespace rlwe;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int ok() {
  g_err.clear();
  return RLWE_OK;
}

uint64_t mulmod_h(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)(((u128)a * b) % m); }

uint64_t powmod_h(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = mulmod_h(r, a, m);
    a = mulmod_h(a, a, m);
    e >>= 1;
  }
  return r;
}

// Deterministic Miller-Rabin for n < 2^64 (first 12 primes as bases).
bool is_prime_h(uint64_t n) {
  if (n < 2) return false;
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (uint64_t p : bases)
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) {
    d >>= 1;
    ++s;
  }
  for (uint64_t a : bases) {
    uint64_t x = powmod_h(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s; ++r) {
      x = mulmod_h(x, x, n);
      if (x == n - 1) {
        comp = false;
        break;
      }
    }
    if (comp) return false;
  }
  return true;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Workspace of ct_matmul_clear_noalloc: a fixed device array, one copy per GPU the
// library runs on, held until the process ends. In host code `scratch` names a
// host-side stand-in; its device address on each GPU comes from hipGetSymbolAddress
// (taken once per device by rlwe_params_init, with that device current).
constexpr size_t kScratchBytes = RLWE_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device `dev` (looked up once).
int scratch_lookup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return RLWE_OK;  // such devices get no scratch
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return RLWE_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    char buf[256];
    snprintf(buf, sizeof buf, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
             hipGetErrorString(e));
    g_err = buf;
    return RLWE_EHIP;
  }
  g_scratch_ptr[dev] = ptr;
  return RLWE_OK;
}

}  // namespace

namespace {
enum KernelKind {
  K_PREP = 0, K_MASK = 1, K_BODY = 2, K_MODSWITCH = 3, K_NTT = 4, K_PACK = 5,
  K_KSDIG = 6, K_KSACC = 7, K_KSFIN = 8, K_PERSIST = 9, K_KINDS = 10
};
constexpr int kMaxProfiled = 4096;
struct Profiler {
  bool on = false;
  int used = 0;
  uint32_t dropped = 0;
  hipEvent_t ev[kMaxProfiled][2] = {};
  int kind[kMaxProfiled] = {};
  int created = 0;
};
}  // namespace

struct rlwe_ctx {
  int device = 0;
  uint32_t log2_t = 0;
  RingConst rc{};
  void* ws = nullptr;
  size_t ws_bytes = 0;
  Profiler* prof = nullptr;
  bool ntt_ok = false;      // the NTT method is available (N = kNttN)
  bool tw_ok = false;       // twiddle tables built (N <= kNttN): KeySwitch packing available
  NttConst ntt{};
  uint64_t* ntt_tables = nullptr;
  uint32_t cus = 0;         // compute units of the device
  uint32_t* sync = nullptr; // counters of the persistent launch (zero between launches)
  rlwe_tuner* tuner = nullptr;            // measured launch choices (rlwe_ctx_set_tuner)
  const rlwe_schedule* forced = nullptr;  // while tuning: the candidate being timed
};

namespace {
// Runs `launch` on stream s; while profiling, brackets it with two events.
template <class F>
hipError_t timed(rlwe_ctx* ctx, int kind, hipStream_t s, F launch) {
  Profiler* p = ctx ? ctx->prof : nullptr;
  if (!p || !p->on) return launch();
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return launch();  // no events inside a captured graph
  if (p->used >= kMaxProfiled) {
    ++p->dropped;
    return launch();
  }
  const int i = p->used;
  if (i >= p->created) {
    hipError_t e = hipEventCreate(&p->ev[i][0]);
    if (e == hipSuccess) e = hipEventCreate(&p->ev[i][1]);
    if (e != hipSuccess) return e;
    p->created = i + 1;
  }
  hipError_t e = hipEventRecord(p->ev[i][0], s);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(p->ev[i][1], s);
  if (e != hipSuccess) return e;
  p->kind[i] = kind;
  p->used = i + 1;
  return hipSuccess;
}
}  // namespace

namespace {

struct Mat {
  bool present = false;
  int8_t* w = nullptr;
  MatArgs args{};
  SwitchConst sc{};
  uint32_t max_l1 = 0;
  bool ntt = false;         // mask product by NTT (otherwise digit planes on the matrix cores)
  uint64_t* what = nullptr; // NTT method: [rows][L][P][N] (value, Shoup companion)
};

}  // namespace

struct rlwe_ksk {
  rlwe_ctx* ctx = nullptr;
  uint64_t* khat = nullptr;  // [N][ell][P][2][N][2], NTT domain, bit-reversed, with companions
  KsConst kc{};
};

struct rlwe_weights {
  rlwe_ctx* ctx = nullptr;
  Mat fwd, tr;
};

namespace {

// 255^e as a 128-bit integer (e <= 15).
u128 pow255(uint32_t e) {
  u128 r = 1;
  for (uint32_t i = 0; i < e; ++i) r *= 255;
  return r;
}

double u128_to_double(u128 v) { return (double)(uint64_t)(v >> 64) * 18446744073709551616.0 + (double)(uint64_t)v; }

// num * 2^bits / den rounded to nearest, for num < den < 2^126 and bits <= 128.
u128 frac_bits(u128 num, u128 den, int bits) {
  u128 r = num, quo = 0;
  for (int b = 0; b < bits; ++b) {
    r <<= 1;
    quo <<= 1;
    if (r >= den) {
      r -= den;
      quo |= 1;
    }
  }
  if (2 * r >= den) ++quo;
  return quo;
}

// Switched-epilogue constants for a contraction whose digit sums are bounded
// by 127 * max_l1 (max_l1 = largest 1-norm of a weight row).
int make_switch_const(const RingConst& rc, uint32_t max_l1, SwitchConst* sc) {
  const u128 q = make_u128(rc.Q_hi, rc.Q_lo);
  const double qd = u128_to_double(q);
  const double maxS = 127.0 * (double)(max_l1 > 0 ? max_l1 : 1);
  // Largest l0 whose skipped digits move V 2^32/q by at most 2^-16.
  uint32_t l0 = 0;
  for (uint32_t c = 1; c < rc.D; ++c) {
    const double skipped = maxS * ((pow(255.0, (double)c) - 1.0) / 254.0) * 4294967296.0 / qd;
    if (skipped <= 1.0 / 65536.0) l0 = c;
  }
  uint32_t dk = rc.D - l0;
  if (rc.D == 7) {
    dk = 7;
  } else {
    if (dk < 8) dk = 8;
    if (dk == 13) dk = 14;
  }
  l0 = rc.D - dk;
  sc->l0 = l0;
  sc->dk = dk;
  // Uncertainty of the per-digit fixed-point sum (RingConst::dg), in units of 2^-32 of
  // V 2^32 / q: the skipped digits (factor 2 margin), one unit of floor per kept digit,
  // the rounding of each G_l (|S| 2^-33 units, below one unit for |S| < 2^32), and a
  // margin.
  const double skipped = maxS * ((pow(255.0, (double)l0) - 1.0) / 254.0) * 4294967296.0 / qd;
  const double band = ceil(2.0 * skipped * 4294967296.0) + 2.0 * dk + 4.0;
  if (band > 1073741824.0) return fail(RLWE_ESHAPE, "internal: rounding band too wide");
  sc->epsw = (uint32_t)band;
  return RLWE_OK;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(RLWE_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Workspace of one product: mask digit planes (matrix-core method) or transformed
// masks with their Shoup companions (NTT method), then body digit planes.
size_t ws_mask_bytes(const RingConst& rc, const MatArgs& m, uint32_t T, bool ntt) {
  return ntt ? align_up((size_t)T * m.L * rc.P * rc.N * 16, 256)
             : align_up((size_t)T * rc.D * m.L * 2 * rc.N, 256);
}
size_t ws_item(const RingConst& rc, const MatArgs& m, uint32_t T, bool ntt) {
  return ws_mask_bytes(rc, m, T, ntt) + align_up((size_t)T * rc.D * m.L * rc.N, 256);
}

uint32_t bitrev_h(uint32_t x, uint32_t bits) {
  uint32_t r = 0;
  for (uint32_t i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

// Twiddle tables of the NTT method: per prime psi^bitrev(k) and psi^-bitrev(k) with
// Shoup companions, psi a primitive 2N-th root of unity (psi^N = -1 mod q_p).
int build_ntt(rlwe_ctx* ctx) {
  const RingConst& rc = ctx->rc;
  const uint32_t N = rc.N;
  const size_t per = (size_t)2 * N;  // (value, companion) pairs
  std::vector<uint64_t> host(per * 2 * rc.P);
  for (uint32_t pi = 0; pi < rc.P; ++pi) {
    const uint64_t q = rc.q[pi];
    uint64_t psi = 0;
    for (uint64_t g = 2; g < 100000 && !psi; ++g) {
      const uint64_t c = powmod_h(g, (q - 1) / (2 * N), q);
      if (powmod_h(c, N, q) == q - 1) psi = c;
    }
    if (!psi) return fail(RLWE_EPARAM, "no primitive 2N-th root of unity found mod %llu", (unsigned long long)q);
    const uint64_t psi_inv = powmod_h(psi, q - 2, q);
    uint64_t* f = host.data() + (2 * pi) * per;
    uint64_t* v = host.data() + (2 * pi + 1) * per;
    for (uint32_t k = 0; k < N; ++k) {
      const uint32_t e = bitrev_h(k, rc.logN);
      f[2 * k] = powmod_h(psi, e, q);
      f[2 * k + 1] = (uint64_t)(((u128)f[2 * k] << 64) / q);
      v[2 * k] = powmod_h(psi_inv, e, q);
      v[2 * k + 1] = (uint64_t)(((u128)v[2 * k] << 64) / q);
    }
    const uint64_t ninv = powmod_h(N % q, q - 2, q);
    ctx->ntt.ninv[pi] = ninv;
    ctx->ntt.bm[pi] = (uint32_t)(~0ull / q);
    const u128 rq = ~(u128)0 / q;  // floor((2^128 - 1) / q) = floor(2^128 / q) for odd q
    ctx->ntt.rq[pi][0] = (uint64_t)(rq >> 64);
    ctx->ntt.rq[pi][1] = (uint64_t)rq;
    ctx->ntt.ninv_shoup[pi] = (uint64_t)(((u128)ninv << 64) / q);
    const uint64_t c = rc.crt_inv[pi];  // N^-1 is folded into the transformed weights
    ctx->ntt.crt[pi] = c;
    ctx->ntt.crt_shoup[pi] = (uint64_t)(((u128)c << 64) / q);
    // h = floor(c 2^128 / q) mod 2^128 = c floor(2^128 / q) + floor(c (2^128 mod q) / q)
    const u128 all = ~(u128)0;                      // 2^128 - 1
    u128 qd = all / q, rm = all % q + 1;            // 2^128 = qd q + rm
    if (rm == q) {
      ++qd;
      rm = 0;
    }
    const u128 h = (u128)c * qd + ((u128)c * rm) / q;  // first product wraps mod 2^128
    for (int w = 0; w < 4; ++w) ctx->ntt.h[pi][w] = (uint32_t)(h >> (32 * w));
    // the inverse transform's last stage multiplies by psi^-bitrev(1) (entry 1)
    const uint64_t cl = (uint64_t)((u128)c * v[2] % q);
    ctx->ntt.crtl[pi] = cl;
    ctx->ntt.crtl_shoup[pi] = (uint64_t)(((u128)cl << 64) / q);
    const u128 hl = (u128)cl * qd + ((u128)cl * rm) / q;
    for (int w = 0; w < 4; ++w) ctx->ntt.hl[pi][w] = (uint32_t)(hl >> (32 * w));
  }
  hipError_t e = hipMalloc(&ctx->ntt_tables, host.size() * 8);
  if (e != hipSuccess) return fail(RLWE_ENOMEM, "hipMalloc(NTT tables): %s", hipGetErrorString(e));
  e = hipMemcpy(ctx->ntt_tables, host.data(), host.size() * 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "NTT tables upload");
  for (uint32_t pi = 0; pi < rc.P; ++pi) {
    ctx->ntt.fwd[pi] = ctx->ntt_tables + (2 * pi) * per;
    ctx->ntt.inv[pi] = ctx->ntt_tables + (2 * pi + 1) * per;
  }
  // the product's inverse transforms are written for N = 4096 and N = 2048
  ctx->ntt_ok = N == kNttN || N == kNttN / 2;
  ctx->tw_ok = true;
  return RLWE_OK;
}

int ensure_ws(rlwe_ctx* ctx, size_t bytes, hipStream_t s) {
  if (bytes <= ctx->ws_bytes) return RLWE_OK;
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (ctx->ws) {
    e = hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    if (e != hipSuccess) return hip_fail(e, "hipFree(workspace)");
  }
  e = hipMalloc(&ctx->ws, bytes);
  if (e != hipSuccess) {
    ctx->ws = nullptr;
    return fail(RLWE_ENOMEM, "hipMalloc(workspace, %zu bytes): %s", bytes, hipGetErrorString(e));
  }
  ctx->ws_bytes = bytes;
  return RLWE_OK;
}

}  // namespace

extern "C" {

const char* rlwe_last_error(void) { return g_err.c_str(); }

int rlwe_params_init(const rlwe_params* p, int hip_device, rlwe_ctx** out) {
  if (!p || !out) return fail(RLWE_EINVAL, "rlwe_params_init: null argument");
  *out = nullptr;
  const uint32_t N = p->N;
  if (N < 64 || N > 32768 || (N & (N - 1)))
    return fail(RLWE_EPARAM, "N = %u must be a power of two in [64, 32768]", N);
  if (p->num_primes < 1 || p->num_primes > 2)
    return fail(RLWE_EPARAM, "num_primes = %u must be 1 or 2", p->num_primes);
  if (!p->primes) return fail(RLWE_EINVAL, "primes is null");
  if (p->log2_q_out < 1 || p->log2_q_out > 32)
    return fail(RLWE_EPARAM, "log2_q_out = %u outside [1, 32]", p->log2_q_out);
  if (p->log2_t < 1 || p->log2_t > 32) return fail(RLWE_EPARAM, "log2_t = %u outside [1, 32]", p->log2_t);
  RingConst rc{};
  rc.N = N;
  rc.logN = 0;
  while ((1u << rc.logN) < N) ++rc.logN;
  rc.P = p->num_primes;
  rc.D = rc.P == 1 ? 7 : 14;
  for (uint32_t i = 0; i < rc.P; ++i) {
    const uint64_t q = p->primes[i];
    if (q >= (1ull << 54) || q <= 2ull * N)
      return fail(RLWE_EPARAM, "prime %llu must satisfy 2N < q < 2^54", (unsigned long long)q);
    if (!is_prime_h(q)) return fail(RLWE_EPARAM, "%llu is not prime", (unsigned long long)q);
    if (q % (2ull * N) != 1)
      return fail(RLWE_EPARAM, "prime %llu is not 1 mod 2N", (unsigned long long)q);
    rc.q[i] = q;
  }
  if (rc.P == 2 && rc.q[0] == rc.q[1]) return fail(RLWE_EPARAM, "primes must be distinct");
  u128 Q = 1;
  for (uint32_t i = 0; i < rc.P; ++i) Q *= rc.q[i];
  if ((Q >> p->log2_t) == 0) return fail(RLWE_EPARAM, "t exceeds q");
  for (uint32_t i = 0; i < rc.P; ++i) {
    const uint64_t Mi = rc.P == 1 ? 1 : (uint64_t)((Q / rc.q[i]) % rc.q[i]);
    rc.crt_inv[i] = rc.P == 1 ? 1 : powmod_h(Mi, rc.q[i] - 2, rc.q[i]);
    rc.crt_inv_shoup[i] = (uint64_t)(((u128)rc.crt_inv[i] << 64) / rc.q[i]);
  }
  rc.Q_lo = (uint64_t)Q;
  rc.Q_hi = (uint64_t)(Q >> 64);
  const u128 half = (Q - 1) / 2;
  rc.half_lo = (uint64_t)half;
  rc.half_hi = (uint64_t)(half >> 64);
  rc.qbits = p->log2_q_out;
  rc.inv_qout = ldexp(1.0, (int)rc.qbits) / u128_to_double(Q);
  for (uint32_t l = 0; l < rc.D; ++l) {
    // G_l mod 2^96 (the integer part of 255^l / q only adds multiples of 2^96)
    const i128 G = (i128)frac_bits(pow255(l) % Q, Q, 96);
    const int32_t a = (int32_t)(uint32_t)(uint64_t)G;
    const i128 g1 = (G - a) >> 32;
    const int32_t b = (int32_t)(uint32_t)(uint64_t)g1;
    rc.dg[l][0] = a;
    rc.dg[l][1] = b;
    rc.dg[l][2] = (int32_t)(uint32_t)(uint64_t)((g1 - b) >> 32);
  }

  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (hip_device < 0 || hip_device >= ndev)
    return fail(RLWE_EINVAL, "hip_device %d outside [0, %d)", hip_device, ndev);
  e = hipSetDevice(hip_device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  rlwe_ctx* ctx = new (std::nothrow) rlwe_ctx;
  if (!ctx) return fail(RLWE_ENOMEM, "out of host memory");
  ctx->device = hip_device;
  ctx->log2_t = p->log2_t;
  ctx->rc = rc;
  if (scratch_lookup(hip_device) != RLWE_OK) {
    delete ctx;
    return RLWE_EHIP;
  }
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, hip_device);
  if (e == hipSuccess) e = hipMalloc(&ctx->sync, kSyncWords * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemset(ctx->sync, 0, kSyncWords * sizeof(uint32_t));
  if (e != hipSuccess) {
    if (ctx->sync) (void)hipFree(ctx->sync);
    delete ctx;
    return hip_fail(e, "device attributes / persistent-launch counters");
  }
  ctx->cus = (uint32_t)cus;
  if (N <= kNttN) {
    const int r = build_ntt(ctx);
    if (r != RLWE_OK) {
      if (ctx->ntt_tables) (void)hipFree(ctx->ntt_tables);
      (void)hipFree(ctx->sync);
      delete ctx;
      return r;
    }
  }
  *out = ctx;
  return ok();
}

int rlwe_profile_begin(rlwe_ctx* ctx) {
  if (!ctx) return fail(RLWE_EINVAL, "rlwe_profile_begin: null context");
  if (!ctx->prof) {
    ctx->prof = new (std::nothrow) Profiler;
    if (!ctx->prof) return fail(RLWE_ENOMEM, "out of host memory");
  }
  ctx->prof->on = true;
  ctx->prof->used = 0;
  ctx->prof->dropped = 0;
  return ok();
}

int rlwe_profile_end(rlwe_ctx* ctx, rlwe_kernel_times* out) {
  if (!ctx || !out) return fail(RLWE_EINVAL, "rlwe_profile_end: null argument");
  memset(out, 0, sizeof *out);
  Profiler* p = ctx->prof;
  if (!p || !p->on) return fail(RLWE_EINVAL, "rlwe_profile_end: no profiling window open");
  p->on = false;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  double* ms[K_KINDS] = {&out->prep_ms,  &out->mask_ms,  &out->body_ms,
                         &out->modswitch_ms, &out->ntt_ms, &out->pack_ms,
                         &out->ksdig_ms, &out->ksacc_ms, &out->ksfin_ms, &out->persist_ms};
  uint32_t* n[K_KINDS] = {&out->prep_n,  &out->mask_n,  &out->body_n,
                          &out->modswitch_n, &out->ntt_n, &out->pack_n,
                          &out->ksdig_n, &out->ksacc_n, &out->ksfin_n, &out->persist_n};
  for (int i = 0; i < p->used; ++i) {
    e = hipEventSynchronize(p->ev[i][1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float t = 0.f;
    e = hipEventElapsedTime(&t, p->ev[i][0], p->ev[i][1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    *ms[p->kind[i]] += t;
    ++*n[p->kind[i]];
  }
  out->dropped = p->dropped;
  p->used = 0;
  return ok();
}

int rlwe_params_destroy(rlwe_ctx* ctx) {
  if (!ctx) return ok();
  if (ctx->prof) {
    (void)hipSetDevice(ctx->device);
    for (int i = 0; i < ctx->prof->created; ++i) {
      (void)hipEventDestroy(ctx->prof->ev[i][0]);
      (void)hipEventDestroy(ctx->prof->ev[i][1]);
    }
    delete ctx->prof;
  }
  if (ctx->ntt_tables) {
    (void)hipSetDevice(ctx->device);
    (void)hipFree(ctx->ntt_tables);
  }
  if (ctx->sync) {
    (void)hipSetDevice(ctx->device);
    (void)hipFree(ctx->sync);
  }
  if (ctx->ws) {
    (void)hipSetDevice(ctx->device);
    hipError_t e = hipFree(ctx->ws);
    if (e != hipSuccess) {
      delete ctx;
      return hip_fail(e, "hipFree(workspace)");
    }
  }
  delete ctx;
  return ok();
}

static void free_mat(Mat& m) {
  if (m.w) (void)hipFree(m.w);
  if (m.what) (void)hipFree(m.what);
  m.w = nullptr;
  m.what = nullptr;
  m.present = false;
}

static int load_mat(rlwe_ctx* ctx, const int8_t* W_dev, uint32_t d_out, uint32_t d_in,
                    bool transpose, int method, bool rowpack, hipStream_t s, Mat& m) {
  const RingConst& rc = ctx->rc;
  MatArgs& a = m.args;
  a.rows = transpose ? d_in : d_out;
  a.k = transpose ? d_out : d_in;
  a.kw = (uint32_t)align_up(a.k, 64);
  a.rows_pad = (uint32_t)align_up(a.rows, 64);
  a.L = (a.k + rc.N - 1) / rc.N;
  // multi-row packing where two or more rows fit one polynomial (Sec. 4.3.1)
  a.n_o = rowpack && 2 * a.k <= rc.N ? rc.N / a.k : 1;
  a.slot = a.n_o > 1 ? a.k : rc.N;
  // exact 128-bit accumulation: 127 * K' * (q-1)/2 < 2^127, K' the weights one
  // output sums over (n_o K with packing)
  const u128 Q = make_u128(rc.Q_hi, rc.Q_lo);
  const u128 lim = ((u128)1 << 127) / ((u128)127 * a.k * a.n_o);
  if ((Q - 1) / 2 >= lim)
    return fail(RLWE_ESHAPE, "contraction length %u too long for exact 128-bit sums at this q", a.k);
  hipError_t e = hipMalloc(&m.w, (size_t)a.rows_pad * a.kw);
  if (e != hipSuccess) return fail(RLWE_ENOMEM, "hipMalloc(weights): %s", hipGetErrorString(e));
  a.w = m.w;
  e = launch_transpose_pad(W_dev, d_out, d_in, transpose, m.w, a.rows_pad, a.kw, s);
  if (e != hipSuccess) return hip_fail(e, "weight layout kernel");
  uint32_t* norms = nullptr;
  e = hipMalloc(&norms, sizeof(uint32_t) * a.rows);
  if (e != hipSuccess) return fail(RLWE_ENOMEM, "hipMalloc(norms): %s", hipGetErrorString(e));
  e = launch_row_l1(m.w, a.rows, a.kw, norms, s);
  std::string hn;
  uint32_t* host = new (std::nothrow) uint32_t[a.rows];
  if (e == hipSuccess && host) e = hipMemcpyAsync(host, norms, sizeof(uint32_t) * a.rows, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(norms);
  if (!host) return fail(RLWE_ENOMEM, "out of host memory");
  if (e != hipSuccess) {
    delete[] host;
    return hip_fail(e, "weight norms");
  }
  uint32_t mx = 0;
  for (uint32_t r = 0; r < a.rows; ++r) mx = host[r] > mx ? host[r] : mx;
  delete[] host;
  m.max_l1 = mx;
  // |W x| <= 127 * max_l1 must stay below t/2 (no wrap modulo t, Sec. 4.4)
  const uint64_t t_half = 1ull << (ctx->log2_t - 1);
  if ((uint64_t)127 * mx >= t_half)
    return fail(RLWE_EOVERFLOW, "127 * max row 1-norm = %llu reaches t/2 = %llu%s",
                (unsigned long long)127 * mx, (unsigned long long)t_half,
                transpose ? " (transposed)" : "");
  const int rc2 = make_switch_const(rc, mx, &m.sc);
  if (rc2 != RLWE_OK) return rc2;
  // method: as asked for, else the tuner's measured choice for this shape, else the one
  // with the smaller estimated time per output (token x output row). The matrix-core
  // cost grows with K times the digit planes kept, the transform cost with the blocks L
  // only; the constants are fitted to MI355X timings of both kernels at N = 4096 with
  // two primes (matrix cores, K = 512 .. 8192; transforms 34.7 ns per output at K =
  // 2048, 128 tokens), the transform cost taken per prime.
  m.ntt = method == 1 || a.n_o > 1;
  if (method == 0 && a.n_o == 1 && ctx->ntt_ok) {
    uint32_t tuned;
    if (ctx->tuner && tune::find_method(ctx->tuner->cache, rc.N, rc.P, a.k, a.rows, &tuned)) {
      m.ntt = tuned == RLWE_METHOD_NTT;
    } else {  // both costs scale about linearly with N
      const double scale = (double)rc.N / kNttN;
      const double mfma_ns = (8.0 + 0.0033 * (double)a.k * m.sc.dk) * scale;
      const double ntt_ns = (5.0 + 12.35 * a.L) * rc.P * scale;
      m.ntt = ntt_ns < mfma_ns;
    }
  }
  if (m.ntt) {
    if (!ctx->ntt_ok) return fail(RLWE_EPARAM, "the NTT method needs N = %u or %u", kNttN / 2, kNttN);
    const size_t groups = (a.rows + a.n_o - 1) / a.n_o;
    const size_t bytes = groups * a.L * rc.P * rc.N * 8;
    e = hipMalloc(&m.what, bytes);
    if (e != hipSuccess) return fail(RLWE_ENOMEM, "hipMalloc(NTT weights, %zu bytes): %s", bytes, hipGetErrorString(e));
    e = launch_ntt_weights(a, ctx->ntt, rc, m.what, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "NTT weights kernel");
  }
  m.present = true;
  return RLWE_OK;
}

int rlwe_weights_load(rlwe_ctx* ctx, const int8_t* W_dev, uint32_t d_out, uint32_t d_in,
                      uint32_t flags, rlwe_stream_t stream, rlwe_weights** out) {
  if (!ctx || !W_dev || !out) return fail(RLWE_EINVAL, "rlwe_weights_load: null argument");
  *out = nullptr;
  if ((flags & (RLWE_W_FWD | RLWE_W_TRANSPOSE)) == 0 ||
      (flags & ~(RLWE_W_FWD | RLWE_W_TRANSPOSE | RLWE_W_NTT | RLWE_W_TOEPLITZ | RLWE_W_ROWPACK)) ||
      ((flags & RLWE_W_NTT) && (flags & RLWE_W_TOEPLITZ)) ||
      ((flags & RLWE_W_ROWPACK) && (flags & RLWE_W_TOEPLITZ)))
    return fail(RLWE_EINVAL, "rlwe_weights_load: flags 0x%x invalid", flags);
  if ((flags & (RLWE_W_NTT | RLWE_W_ROWPACK)) && !ctx->ntt_ok)
    return fail(RLWE_EPARAM, "RLWE_W_NTT and RLWE_W_ROWPACK need N = %u or %u (N = %u)",
                kNttN / 2, kNttN, ctx->rc.N);
  const int method = (flags & RLWE_W_NTT) ? 1 : (flags & RLWE_W_TOEPLITZ) ? 2 : 0;
  if (d_out < 1 || d_in < 1 || d_out > 65536 || d_in > 65536)
    return fail(RLWE_ESHAPE, "d_out = %u, d_in = %u must lie in [1, 65536]", d_out, d_in);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  rlwe_weights* w = new (std::nothrow) rlwe_weights;
  if (!w) return fail(RLWE_ENOMEM, "out of host memory");
  w->ctx = ctx;
  hipStream_t s = (hipStream_t)stream;
  int r = RLWE_OK;
  const bool rowpack = flags & RLWE_W_ROWPACK;
  if (flags & RLWE_W_FWD) r = load_mat(ctx, W_dev, d_out, d_in, false, method, rowpack, s, w->fwd);
  if (r == RLWE_OK && (flags & RLWE_W_TRANSPOSE))
    r = load_mat(ctx, W_dev, d_out, d_in, true, method, rowpack, s, w->tr);
  if (r != RLWE_OK) {
    std::string msg = g_err;
    (void)hipStreamSynchronize(s);
    free_mat(w->fwd);
    free_mat(w->tr);
    delete w;
    g_err = msg;
    return r;
  }
  *out = w;
  return ok();
}

int rlwe_weights_free(rlwe_weights* w) {
  if (!w) return ok();
  (void)hipSetDevice(w->ctx->device);
  free_mat(w->fwd);
  free_mat(w->tr);
  delete w;
  return ok();
}

size_t rlwe_workspace_bytes(const rlwe_ctx* ctx, const rlwe_weights* w, uint32_t transpose,
                            uint32_t tokens) {
  if (!ctx || !w) return 0;
  const Mat& m = transpose ? w->tr : w->fwd;
  if (!m.present) return 0;
  return ws_item(ctx->rc, m.args, tokens, m.ntt);
}

int rlwe_weights_digits(const rlwe_weights* w, uint32_t transpose, uint32_t* kept,
                        uint32_t* total) {
  if (!w || !kept || !total) return fail(RLWE_EINVAL, "rlwe_weights_digits: null argument");
  const Mat& m = transpose ? w->tr : w->fwd;
  if (!m.present) return fail(RLWE_EINVAL, "rlwe_weights_digits: orientation not loaded");
  *kept = m.sc.dk;
  *total = w->ctx->rc.D;
  return ok();
}

int rlwe_weights_method(const rlwe_weights* w, uint32_t transpose, uint32_t* method) {
  if (!w || !method) return fail(RLWE_EINVAL, "rlwe_weights_method: null argument");
  const Mat& m = transpose ? w->tr : w->fwd;
  if (!m.present) return fail(RLWE_EINVAL, "rlwe_weights_method: orientation not loaded");
  *method = m.ntt ? RLWE_METHOD_NTT : RLWE_METHOD_TOEPLITZ;
  return ok();
}

int rlwe_weights_rows_per_product(const rlwe_weights* w, uint32_t transpose, uint32_t* n_o) {
  if (!w || !n_o) return fail(RLWE_EINVAL, "rlwe_weights_rows_per_product: null argument");
  const Mat& m = transpose ? w->tr : w->fwd;
  if (!m.present) return fail(RLWE_EINVAL, "rlwe_weights_rows_per_product: orientation not loaded");
  *n_o = m.args.n_o;
  return ok();
}

int rlwe_workspace_reserve(rlwe_ctx* ctx, size_t bytes) {
  if (!ctx) return fail(RLWE_EINVAL, "rlwe_workspace_reserve: null context");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  const int r = ensure_ws(ctx, bytes, nullptr);
  return r == RLWE_OK ? ok() : r;
}

static int validate_desc(const rlwe_ctx* ctx, const ct_matmul_desc& d, const Mat** out) {
  if (!d.w) return fail(RLWE_EINVAL, "ct_matmul: null weights");
  if (d.w->ctx != ctx) return fail(RLWE_EINVAL, "ct_matmul: weights belong to another context");
  if (d.transpose > 1) return fail(RLWE_EINVAL, "ct_matmul: transpose must be 0 or 1");
  const Mat& m = d.transpose ? d.w->tr : d.w->fwd;
  if (!m.present)
    return fail(RLWE_EINVAL, "ct_matmul: weights were loaded without %s",
                d.transpose ? "RLWE_W_TRANSPOSE" : "RLWE_W_FWD");
  if (d.tokens > 65535) return fail(RLWE_ESHAPE, "tokens = %u exceeds 65535 per product", d.tokens);
  if (d.tokens && (!d.ct_in || !d.out)) return fail(RLWE_EINVAL, "ct_matmul: null buffer");
  const RingConst& rc = ctx->rc;
  if ((uint64_t)d.tokens * (m.args.rows_pad / 32) * (rc.N / 64) >= (1ull << 31) ||
      (uint64_t)d.tokens * m.args.L * rc.N / 256 >= (1ull << 31))
    return fail(RLWE_ESHAPE, "ct_matmul: product too large for one launch; split the tokens");
  *out = &m;
  return RLWE_OK;
}

static size_t batch_ws(const rlwe_ctx* ctx, const ct_matmul_desc* d, uint32_t n) {
  size_t total = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const Mat& m = d[i].transpose ? d[i].w->tr : d[i].w->fwd;
    total += ws_item(ctx->rc, m.args, d[i].tokens, m.ntt);
  }
  return total;
}

// Enqueue a validated batch using workspace `ws` (at least batch_ws bytes). With a
// key `gk` (NTT method only), masks are rounded to 2^K for its gadget decomposition
// and the outputs are [T][M][N+P] (a~, then the body residues).
static int run_batch(rlwe_ctx* ctx, const ct_matmul_desc* d, uint32_t n, uint32_t flags,
                     hipStream_t s, unsigned char* ws, uint32_t* sync,
                     const rlwe_ksk* gk = nullptr, bool profile = true) {
  const RingConst& rc = ctx->rc;
  rlwe_ctx* pc = profile ? ctx : nullptr;  // kernel timing events, unless switched off
  const bool raw = (flags & RLWE_OUT_RAW_Q) || gk;
  // longest contraction first: its tiles are the most expensive (tail balance)
  uint32_t order[kMaxBatch];
  uint32_t cnt = 0;
  for (uint32_t i = 0; i < n; ++i)
    if (d[i].tokens) order[cnt++] = i;
  const Mat* mats[kMaxBatch];
  for (uint32_t i = 0; i < n; ++i) mats[i] = d[i].transpose ? &d[i].w->tr : &d[i].w->fwd;
  for (uint32_t a = 1; a < cnt; ++a)
    for (uint32_t b = a; b > 0 && mats[order[b]]->args.k > mats[order[b - 1]]->args.k; --b) {
      const uint32_t tmp = order[b];
      order[b] = order[b - 1];
      order[b - 1] = tmp;
    }
  if (cnt == 0) return RLWE_OK;
  Batch all{};
  all.rc = rc;
  all.ntt = ctx->ntt;
  all.raw = raw;
  all.force_exact = (flags & RLWE_OUT_FORCE_EXACT) ? 1 : 0;
  all.seeded = (flags & RLWE_IN_SEEDED) ? 1 : 0;
  if (gk) {
    all.gadget = 1;
    all.kmask = gk->kc.kmask;
    all.kr = gk->kc.rd;
  }
  size_t off = 0;
  for (uint32_t x = 0; x < cnt; ++x) {
    const ct_matmul_desc& dd = d[order[x]];
    const Mat& m = *mats[order[x]];
    Item& it = all.it[x];
    it.m = m.args;
    it.sc = m.sc;
    if (raw) {
      it.sc.l0 = 0;
      it.sc.dk = rc.D;
    }
    it.method = m.ntt ? 1 : 0;
    it.what = m.what;
    it.ct = dd.ct_in;
    const size_t mask_bytes = ws_mask_bytes(rc, m.args, dd.tokens, m.ntt);
    it.emask = m.ntt ? nullptr : (int8_t*)(ws + off);
    it.ahat = m.ntt ? (uint64_t*)(ws + off) : nullptr;
    it.ebody = (int8_t*)(ws + off + mask_bytes);
    off += ws_item(rc, m.args, dd.tokens, m.ntt);
    it.out = dd.out;
    it.T = dd.tokens;
    it.tt_log2 = kTokTileLog2;
    it.order = 0;
    it.groups = (m.args.rows + m.args.n_o - 1) / m.args.n_o;
    const uint32_t prep_per = rc.N >= 256 ? rc.N / 256 : 1;
    all.prep_start[x + 1] = all.prep_start[x] + dd.tokens * m.args.L * prep_per;
    all.fwd_start[x + 1] = all.fwd_start[x] + (m.ntt ? dd.tokens * m.args.L * rc.P : 0);
    all.body_start[x + 1] = all.body_start[x] + dd.tokens * body_blocks_per_token(m.args);
  }
  all.n = cnt;
  // Launch choices: the candidate being timed while tuning, else the tuner's entries
  // (token tile and order per NTT product; for the launch, the product's entry alone,
  // or the entry of batches of this many products), else the defaults. RLWE_LAUNCH_*
  // flags decide the launch.
  bool want_persist = false;
  {
    const tune::Cache* tc = ctx->tuner ? &ctx->tuner->cache : nullptr;
    uint32_t maxT = 0;
    for (uint32_t x = 0; x < cnt; ++x) {
      Item& it = all.it[x];
      maxT = std::max(maxT, it.T);
      rlwe_schedule sc{};
      const bool have = ctx->forced ? (sc = *ctx->forced, true)
                        : tc ? tune::find_product(*tc, rc.N, rc.P, it.m.k, it.m.rows, it.m.n_o,
                                                  raw, it.T, &sc)
                             : false;
      if (have && it.method == 1) {
        it.tt_log2 = std::min<uint32_t>(sc.tt_log2, 5);
        it.order = sc.order ? 1 : 0;
      }
      if (have && cnt == 1) want_persist = sc.launch == 1;
    }
    rlwe_schedule sb{};
    if (!ctx->forced && tc && cnt > 1 && tune::find_batch(*tc, rc.N, rc.P, cnt, raw, maxT, &sb))
      want_persist = sb.launch == 1;
    if (flags & RLWE_LAUNCH_PERSISTENT) want_persist = true;
    if (flags & RLWE_LAUNCH_GROUPED) want_persist = false;
  }
  // One persistent launch for a batch whose products all use the NTT method (not for
  // the rounded-mask output of ct_matmul_pack).
  bool all_ntt = true;
  for (uint32_t x = 0; x < cnt; ++x) all_ntt = all_ntt && all.it[x].method == 1;
  const bool persist = sync && all_ntt && !gk && want_persist && rc.N == kNttN;
  if (persist) {
    all.sync = sync;
    for (uint32_t x = 0; x < cnt; ++x) {
      const Item& it = all.it[x];
      all.unit_start[x + 1] = all.unit_start[x] + it.T * it.m.L;
      const uint32_t tiles = (it.T + (1u << it.tt_log2) - 1) >> it.tt_log2;
      all.mask_start[x + 1] = all.mask_start[x] + it.groups * tiles;
    }
    const uint64_t total = (uint64_t)all.unit_start[cnt] + all.mask_start[cnt] +
                           (all.body_start[cnt] + 1) / 2;
    const uint32_t grid = (uint32_t)std::min<uint64_t>(total, (uint64_t)ctx->cus * 2);
    hipError_t e = timed(pc, K_PERSIST, s, [&] { return launch_persist(all, grid, s); });
    if (e != hipSuccess) return hip_fail(e, "persistent batch kernel");
    return RLWE_OK;
  }
  if (flags & RLWE_LAUNCH_PERSISTENT)
    return fail(RLWE_EINVAL,
                "RLWE_LAUNCH_PERSISTENT needs every product on the NTT method and N = %u", kNttN);
  hipError_t e = timed(pc, K_PREP, s, [&] { return launch_prep(all, s); });
  if (e != hipSuccess) return hip_fail(e, "prep kernel");
  if (all.fwd_start[cnt]) {
    e = timed(pc, K_PREP, s, [&] { return launch_ntt_mask_fwd(all, s); });
    if (e != hipSuccess) return hip_fail(e, "mask NTT kernel");
  }
  // matrix-core method: one mask launch per distinct number of kept digits;
  // NTT method: one launch for the products with two input blocks, one for the rest
  auto lclass = [](const Item& it) { return it.m.L == 2 ? 2u : 0u; };
  bool done[kMaxBatch] = {};
  for (uint32_t x = 0; x < cnt; ++x) {
    if (done[x]) continue;
    const bool ntt = all.it[x].method == 1;
    const uint32_t dk = all.it[x].sc.dk, lc = lclass(all.it[x]);
    Batch mb{};
    mb.rc = rc;
    mb.ntt = all.ntt;
    mb.raw = all.raw;
    mb.force_exact = all.force_exact;
    mb.gadget = all.gadget;
    mb.kmask = all.kmask;
    mb.kr = all.kr;
    for (uint32_t y = x; y < cnt; ++y) {
      if (done[y] || (all.it[y].method == 1) != ntt || (!ntt && all.it[y].sc.dk != dk) ||
          (ntt && lclass(all.it[y]) != lc))
        continue;
      done[y] = true;
      const Item& it = all.it[y];
      mb.it[mb.n] = it;
      const uint32_t groups = (it.m.rows + it.m.n_o - 1) / it.m.n_o;
      const uint32_t blocks = ntt ? groups * ((it.T + (1u << it.tt_log2) - 1) >> it.tt_log2)
                                  : it.T * (it.m.rows_pad / 32) * (rc.N / 64);
      mb.mask_start[mb.n + 1] = mb.mask_start[mb.n] + blocks;
      ++mb.n;
    }
    e = timed(pc, ntt ? K_NTT : K_MASK, s,
              [&] { return ntt ? launch_ntt_mask(mb, lc, s) : launch_mask(mb, dk, s); });
    if (e != hipSuccess) return hip_fail(e, "mask kernel");
  }
  e = timed(pc, K_BODY, s, [&] { return launch_body(all, s); });
  if (e != hipSuccess) return hip_fail(e, "body kernel");
  return RLWE_OK;
}

int ct_matmul_batch(rlwe_ctx* ctx, const ct_matmul_desc* descs, uint32_t n, uint32_t flags,
                    rlwe_stream_t stream) {
  if (!ctx) return fail(RLWE_EINVAL, "ct_matmul_batch: null context");
  if (n == 0) return ok();
  if (!descs) return fail(RLWE_EINVAL, "ct_matmul_batch: null descriptors");
  if (flags & ~(RLWE_OUT_RAW_Q | RLWE_OUT_FORCE_EXACT | RLWE_IN_SEEDED | RLWE_LAUNCH_PERSISTENT |
                RLWE_LAUNCH_GROUPED) ||
      (flags & RLWE_LAUNCH_PERSISTENT && flags & RLWE_LAUNCH_GROUPED))
    return fail(RLWE_EINVAL, "ct_matmul_batch: unknown flags 0x%x", flags);
  for (uint32_t i = 0; i < n; ++i) {
    const Mat* m;
    const int r = validate_desc(ctx, descs[i], &m);
    if (r != RLWE_OK) return r;
  }
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  // workspace for the largest group of kMaxBatch products
  size_t need = 0;
  for (uint32_t i = 0; i < n; i += kMaxBatch)
    need = std::max(need, batch_ws(ctx, descs + i, std::min<uint32_t>(kMaxBatch, n - i)));
  if (need > ctx->ws_bytes) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
      return fail(RLWE_EINVAL, "workspace must be reserved (rlwe_workspace_reserve) before capture");
    const int r = ensure_ws(ctx, need, s);
    if (r != RLWE_OK) return r;
  }
  for (uint32_t i = 0; i < n; i += kMaxBatch) {
    const int r = run_batch(ctx, descs + i, std::min<uint32_t>(kMaxBatch, n - i), flags, s,
                            (unsigned char*)ctx->ws, ctx->sync);
    if (r != RLWE_OK) return r;
  }
  return ok();
}

int ct_matmul_clear(rlwe_ctx* ctx, const rlwe_weights* w, uint32_t transpose,
                    const uint64_t* ct_in, uint32_t tokens, void* out, uint32_t flags,
                    rlwe_stream_t stream) {
  if (!ctx || !w) return fail(RLWE_EINVAL, "ct_matmul_clear: null context or weights");
  ct_matmul_desc d{};
  d.w = w;
  d.transpose = transpose;
  d.ct_in = ct_in;
  d.tokens = tokens;
  d.out = out;
  return ct_matmul_batch(ctx, &d, 1, flags, stream);
}

int ct_matmul_clear_noalloc(rlwe_ctx* ctx, const rlwe_weights* w, uint32_t transpose,
                            const uint64_t* ct_in, uint32_t tokens, void* out, uint32_t flags,
                            rlwe_stream_t stream) {
  if (!ctx || !w) return fail(RLWE_EINVAL, "ct_matmul_clear_noalloc: null context or weights");
  if (flags & ~(RLWE_OUT_RAW_Q | RLWE_OUT_FORCE_EXACT | RLWE_IN_SEEDED | RLWE_LAUNCH_GROUPED))
    return fail(RLWE_EINVAL, "ct_matmul_clear_noalloc: unknown flags 0x%x", flags);
  ct_matmul_desc d{};
  d.w = w;
  d.transpose = transpose;
  d.ct_in = ct_in;
  d.tokens = tokens;
  d.out = out;
  const Mat* m;
  const int r = validate_desc(ctx, d, &m);
  if (r != RLWE_OK) return r;
  if (tokens == 0) return ok();
  const size_t need = ws_item(ctx->rc, m->args, tokens, m->ntt);
  if (need > kScratchBytes)
    return fail(RLWE_ESHAPE,
                "ct_matmul_clear_noalloc: %u tokens need %zu bytes of workspace, above the "
                "fixed %zu; split the tokens or use ct_matmul_clear",
                tokens, need, kScratchBytes);
  void* ws = ctx->device >= 0 && ctx->device < kMaxDevices ? g_scratch_ptr[ctx->device] : nullptr;
  if (!ws) return fail(RLWE_EINVAL, "ct_matmul_clear_noalloc: no scratch on device %d", ctx->device);
  const hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  // the kernels write every workspace word they read (digit planes, transformed
  // masks) before reading it: nothing in the array has to start at zero
  const int r2 = run_batch(ctx, &d, 1, flags | RLWE_LAUNCH_GROUPED, (hipStream_t)stream,
                           (unsigned char*)ws, nullptr, nullptr, /*profile=*/false);
  return r2 == RLWE_OK ? ok() : r2;
}

size_t rlwe_batch_workspace_bytes(const rlwe_ctx* ctx, const ct_matmul_desc* descs, uint32_t n) {
  if (!ctx || !descs) return 0;
  size_t need = 0;
  for (uint32_t i = 0; i < n; ++i)
    if (!descs[i].w || (descs[i].transpose ? !descs[i].w->tr.present : !descs[i].w->fwd.present))
      return 0;
  for (uint32_t i = 0; i < n; i += kMaxBatch)
    need = std::max(need, batch_ws(ctx, descs + i, std::min<uint32_t>(kMaxBatch, n - i)));
  return need;
}

struct rlwe_graph {
  rlwe_ctx* ctx = nullptr;
  void* ws = nullptr;
  uint32_t* sync = nullptr;  // counters of a captured persistent launch (zeroed here)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

int rlwe_graph_capture_batch(rlwe_ctx* ctx, const ct_matmul_desc* descs, uint32_t n,
                             uint32_t flags, rlwe_graph** out) {
  if (!ctx || !descs || !out || n == 0) return fail(RLWE_EINVAL, "rlwe_graph_capture_batch: bad argument");
  *out = nullptr;
  if (flags & ~(RLWE_OUT_RAW_Q | RLWE_OUT_FORCE_EXACT | RLWE_IN_SEEDED | RLWE_LAUNCH_PERSISTENT |
                RLWE_LAUNCH_GROUPED) ||
      (flags & RLWE_LAUNCH_PERSISTENT && flags & RLWE_LAUNCH_GROUPED))
    return fail(RLWE_EINVAL, "rlwe_graph_capture_batch: unknown flags 0x%x", flags);
  for (uint32_t i = 0; i < n; ++i) {
    const Mat* m;
    const int r = validate_desc(ctx, descs[i], &m);
    if (r != RLWE_OK) return r;
  }
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  rlwe_graph* g = new (std::nothrow) rlwe_graph;
  if (!g) return fail(RLWE_ENOMEM, "out of host memory");
  g->ctx = ctx;
  size_t need = 0;
  for (uint32_t i = 0; i < n; i += kMaxBatch)
    need = std::max(need, batch_ws(ctx, descs + i, std::min<uint32_t>(kMaxBatch, n - i)));
  if (need && hipMalloc(&g->ws, need) != hipSuccess) {
    delete g;
    return fail(RLWE_ENOMEM, "hipMalloc(graph workspace, %zu bytes)", need);
  }
  if (hipMalloc(&g->sync, kSyncWords * sizeof(uint32_t)) != hipSuccess ||
      hipMemset(g->sync, 0, kSyncWords * sizeof(uint32_t)) != hipSuccess) {
    if (g->sync) (void)hipFree(g->sync);
    if (g->ws) (void)hipFree(g->ws);
    delete g;
    return fail(RLWE_ENOMEM, "graph counters");
  }
  hipStream_t cs = nullptr;
  e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  int r = RLWE_OK;
  Profiler* prof = ctx->prof;
  const bool was_on = prof && prof->on;
  if (prof) prof->on = false;  // no events inside a captured graph
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    for (uint32_t i = 0; i < n && r == RLWE_OK; i += kMaxBatch)
      r = run_batch(ctx, descs + i, std::min<uint32_t>(kMaxBatch, n - i), flags, cs,
                    (unsigned char*)g->ws, g->sync);
    const hipError_t e2 = hipStreamEndCapture(cs, &g->graph);
    if (r == RLWE_OK && e2 != hipSuccess) e = e2;
  }
  if (prof) prof->on = was_on;
  if (r == RLWE_OK && e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (cs) (void)hipStreamDestroy(cs);
  if (r != RLWE_OK || e != hipSuccess) {
    const std::string msg = r != RLWE_OK ? g_err : std::string("graph capture: ") + hipGetErrorString(e);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->ws) (void)hipFree(g->ws);
    if (g->sync) (void)hipFree(g->sync);
    delete g;
    g_err = msg;
    return r != RLWE_OK ? r : RLWE_EHIP;
  }
  *out = g;
  return ok();
}

int rlwe_graph_launch(rlwe_graph* g, rlwe_stream_t stream) {
  if (!g) return fail(RLWE_EINVAL, "rlwe_graph_launch: null graph");
  hipError_t e = hipSetDevice(g->ctx->device);
  if (e == hipSuccess) e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return ok();
}

int rlwe_graph_destroy(rlwe_graph* g) {
  if (!g) return ok();
  (void)hipSetDevice(g->ctx->device);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->ws) (void)hipFree(g->ws);
  if (g->sync) (void)hipFree(g->sync);
  delete g;
  return ok();
}

int ct_modswitch(rlwe_ctx* ctx, const uint64_t* in, size_t count, uint32_t* out,
                 rlwe_stream_t stream) {
  if (!ctx) return fail(RLWE_EINVAL, "ct_modswitch: null context");
  if (count == 0) return ok();
  if (!in || !out) return fail(RLWE_EINVAL, "ct_modswitch: null buffer");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  e = timed(ctx, K_MODSWITCH, s, [&] { return launch_modswitch(ctx->rc, in, count, out, s); });
  if (e != hipSuccess) return hip_fail(e, "modswitch kernel");
  return ok();
}

size_t rlwe_packed_words(uint32_t len, uint32_t bits) {
  if (bits < 1 || bits > 32) return 0;
  return ((size_t)len * bits + 31) / 32;
}

int ct_pack_bits(rlwe_ctx* ctx, const uint32_t* in, size_t count, uint32_t len, uint32_t* out,
                 rlwe_stream_t stream) {
  if (!ctx) return fail(RLWE_EINVAL, "ct_pack_bits: null context");
  if (count == 0 || len == 0) return ok();
  if (!in || !out) return fail(RLWE_EINVAL, "ct_pack_bits: null buffer");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  e = timed(ctx, K_PACK, s, [&] { return launch_pack_bits(in, count, len, ctx->rc.qbits, out, s); });
  if (e == hipErrorInvalidValue) return fail(RLWE_ESHAPE, "ct_pack_bits: %zu ciphertexts too many", count);
  if (e != hipSuccess) return hip_fail(e, "pack kernel");
  return ok();
}

}  // extern "C"

// ------------------------------------------------------------------ KeySwitch packing

namespace {
KsArgs ks_args_base(const rlwe_ctx* ctx) {
  KsArgs a{};
  a.rc = ctx->rc;
  a.ntt = ctx->ntt;
  return a;
}
// Output groups per pass and the workspace of one pass.
// Constants of the gadget rounding to 2^K (K <= 64) for the primes of rc.
void make_ks_round(const RingConst& rc, uint32_t K, KsRound* kr) {
  *kr = KsRound{};
  for (uint32_t r = 0; r < rc.P; ++r) {
    // inv_p 2^K = f q_p + g (inv_p < 2^54, so the product fits in 118 bits)
    const u128 x = (u128)(rc.P == 1 ? 1 : rc.crt_inv[r]) << K, q = rc.q[r];
    kr->q[r] = rc.q[r];
    kr->f[r] = (uint64_t)(x / q);  // mod 2^64
    kr->g[r] = (uint64_t)(x % q);
    kr->g_shoup[r] = (uint64_t)(((u128)kr->g[r] << 64) / q);
    u128 rem = kr->g[r];  // G = floor(g 2^96 / q_p), one 32-bit word at a time
    uint32_t Gw[3];
    for (int w = 2; w >= 0; --w) {
      const u128 n = rem << 32;
      Gw[w] = (uint32_t)(n / q);
      rem = n % q;
    }
    kr->G_lo[r] = ((uint64_t)Gw[1] << 32) | Gw[0];
    kr->G_hi[r] = Gw[2];
  }
  kr->Q_hi = rc.Q_hi;
  kr->Q_lo = rc.Q_lo;
}

uint32_t ks_pass_groups(size_t M, uint32_t n_pack) {
  const size_t G = (M + n_pack - 1) / n_pack;
  return (uint32_t)std::min<size_t>(G, kKsGroups);
}
size_t ks_ws_bytes(const rlwe_ctx* ctx, const rlwe_ksk* k, size_t M, uint32_t n_pack) {
  const size_t N = ctx->rc.N, GB = ks_pass_groups(M, n_pack);
  const size_t dig = GB * N * k->kc.ell * N * 8;
  const size_t part = GB * (N / 64) * ctx->rc.P * 2 * N * 8;
  return align_up(dig, 256) + part;
}
// The KeySwitch passes over `count` LWE ciphertexts (raw, or with masks already
// rounded when `pre`), workspace `ws` of ks_ws_bytes.
int ks_run(rlwe_ctx* ctx, const rlwe_ksk* k, const uint64_t* lwe_in, size_t count,
           uint32_t n_pack, void* out, bool raw_out, bool pre, unsigned char* ws, hipStream_t s) {
  const size_t G = (count + n_pack - 1) / n_pack;
  hipError_t e;
  const uint32_t GBmax = ks_pass_groups(count, n_pack);
  KsArgs a = ks_args_base(ctx);
  a.kc = k->kc;
  a.lwe = lwe_in;
  a.M = count;
  a.n_pack = n_pack;
  a.raw = raw_out ? 1 : 0;
  a.pre = pre ? 1 : 0;
  a.khat = k->khat;
  a.dig = (int64_t*)ws;
  a.part = (uint64_t*)(ws +
                       align_up((size_t)GBmax * ctx->rc.N * k->kc.ell * ctx->rc.N * 8, 256));
  a.out = out;
  for (size_t g0 = 0; g0 < G; g0 += GBmax) {
    a.g0 = (uint32_t)g0;
    a.GB = (uint32_t)std::min<size_t>(GBmax, G - g0);
    e = timed(ctx, K_KSDIG, s, [&] { return launch_ks_digits(a, s); });
    if (e != hipSuccess) return hip_fail(e, "KeySwitch digits kernel");
    e = timed(ctx, K_KSACC, s, [&] { return launch_ks_accum(a, s); });
    if (e != hipSuccess) return hip_fail(e, "KeySwitch accumulate kernel");
    e = timed(ctx, K_KSFIN, s, [&] { return launch_ks_finish(a, s); });
    if (e != hipSuccess) return hip_fail(e, "KeySwitch finish kernel");
  }
  return RLWE_OK;
}

}  // namespace

extern "C" {

int rlwe_ksk_load(rlwe_ctx* ctx, const uint64_t* ksk_dev, uint32_t log2_base, uint32_t levels,
                  rlwe_stream_t stream, rlwe_ksk** out) {
  if (!ctx || !ksk_dev || !out) return fail(RLWE_EINVAL, "rlwe_ksk_load: null argument");
  *out = nullptr;
  const RingConst& rc = ctx->rc;
  if (!ctx->tw_ok) return fail(RLWE_EPARAM, "KeySwitch packing needs N <= %u", kNttN);
  if (levels < 1 || levels > kMaxLevels)
    return fail(RLWE_EPARAM, "levels = %u outside [1, %u]", levels, kMaxLevels);
  if (log2_base < 1 || log2_base * levels > 64)
    return fail(RLWE_EPARAM, "log2_base = %u: need 1 <= log2_base and log2_base * levels <= 64", log2_base);
  for (uint32_t r = 0; r < rc.P; ++r)
    if (log2_base > 54 || (1ull << (log2_base - 1)) >= rc.q[r])
      return fail(RLWE_EPARAM, "digits of %u bits do not lie below prime %llu", log2_base,
                  (unsigned long long)rc.q[r]);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  rlwe_ksk* k = new (std::nothrow) rlwe_ksk;
  if (!k) return fail(RLWE_ENOMEM, "out of host memory");
  k->ctx = ctx;
  KsConst& kc = k->kc;
  kc.beta = log2_base;
  kc.ell = levels;
  kc.K = log2_base * levels;
  kc.kmask = kc.K == 64 ? ~0ull : (1ull << kc.K) - 1;
  kc.H = 0;
  for (uint32_t m = 0; m < levels; ++m) kc.H += (1ull << (log2_base - 1)) << (log2_base * m);
  make_ks_round(rc, kc.K, &kc.rd);
  const size_t N = rc.N;
  const size_t bytes = N * levels * rc.P * 2 * N * 16;
  e = hipMalloc(&k->khat, bytes);
  if (e != hipSuccess) {
    delete k;
    return fail(RLWE_ENOMEM, "hipMalloc(key, %zu bytes): %s", bytes, hipGetErrorString(e));
  }
  KsArgs a = ks_args_base(ctx);
  a.kc = kc;
  a.ksk_in = ksk_dev;
  a.khat_out = k->khat;
  hipStream_t s = (hipStream_t)stream;
  e = launch_ksk_fwd(a, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipFree(k->khat);
    delete k;
    return hip_fail(e, "key transform");
  }
  *out = k;
  return ok();
}

int rlwe_ksk_free(rlwe_ksk* k) {
  if (!k) return ok();
  (void)hipSetDevice(k->ctx->device);
  if (k->khat) (void)hipFree(k->khat);
  delete k;
  return ok();
}

size_t rlwe_keyswitch_workspace_bytes(const rlwe_ctx* ctx, const rlwe_ksk* k, size_t count,
                                      uint32_t n_pack) {
  if (!ctx || !k || count == 0 || n_pack < 1 || n_pack > ctx->rc.N) return 0;
  return ks_ws_bytes(ctx, k, count, n_pack);
}

size_t rlwe_packed_count(size_t count, uint32_t n_pack) {
  return n_pack ? (count + n_pack - 1) / n_pack : 0;
}

int ct_keyswitch_pack(rlwe_ctx* ctx, const rlwe_ksk* k, const uint64_t* lwe_in, size_t count,
                      uint32_t n_pack, void* out, uint32_t flags, rlwe_stream_t stream) {
  if (!ctx || !k) return fail(RLWE_EINVAL, "ct_keyswitch_pack: null context or key");
  if (k->ctx != ctx) return fail(RLWE_EINVAL, "ct_keyswitch_pack: key of another context");
  if (flags & ~RLWE_OUT_RAW_Q) return fail(RLWE_EINVAL, "ct_keyswitch_pack: unknown flags 0x%x", flags);
  if (n_pack < 1 || n_pack > ctx->rc.N)
    return fail(RLWE_ESHAPE, "n_pack = %u outside [1, N]", n_pack);
  if (count == 0) return ok();
  if (!lwe_in || !out) return fail(RLWE_EINVAL, "ct_keyswitch_pack: null buffer");
  const size_t G = (count + n_pack - 1) / n_pack;
  if (G >= (1ull << 31)) return fail(RLWE_ESHAPE, "ct_keyswitch_pack: %zu ciphertexts too many", count);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  const size_t need = ks_ws_bytes(ctx, k, count, n_pack);
  if (need > ctx->ws_bytes) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
      return fail(RLWE_EINVAL, "workspace must be reserved (rlwe_workspace_reserve) before capture");
    const int r = ensure_ws(ctx, need, s);
    if (r != RLWE_OK) return r;
  }
  const int r = ks_run(ctx, k, lwe_in, count, n_pack, out, flags & RLWE_OUT_RAW_Q, false,
                       (unsigned char*)ctx->ws, s);
  if (r != RLWE_OK) return r;
  return ok();
}

// Workspace of ct_matmul_pack: the product's, the LWE outputs between the two steps
// (rounded masks and bodies [M][N+P] with the NTT method, raw [M][P][N+1] otherwise),
// and the KeySwitch passes'.
static size_t matmul_pack_ws(const rlwe_ctx* ctx, const Mat& m, uint32_t tokens,
                             const rlwe_ksk* k, uint32_t n_pack, size_t* off_inter,
                             size_t* off_ks) {
  const RingConst& rc = ctx->rc;
  const size_t M = (size_t)tokens * m.args.rows;
  const bool gadget = m.ntt && rc.N == kNttN;  // the product rounds the masks itself
  const size_t inter = M * (gadget ? rc.N + rc.P : (size_t)rc.P * (rc.N + 1)) * 8;
  *off_inter = align_up(ws_item(rc, m.args, tokens, m.ntt), 256);
  *off_ks = *off_inter + align_up(inter, 256);
  return *off_ks + ks_ws_bytes(ctx, k, M, n_pack);
}

size_t rlwe_matmul_pack_workspace_bytes(const rlwe_ctx* ctx, const rlwe_weights* w,
                                        uint32_t transpose, uint32_t tokens, const rlwe_ksk* k,
                                        uint32_t n_pack) {
  if (!ctx || !w || !k || transpose > 1 || tokens == 0 || n_pack < 1 || n_pack > ctx->rc.N)
    return 0;
  const Mat& m = transpose ? w->tr : w->fwd;
  if (!m.present) return 0;
  size_t a, b;
  return matmul_pack_ws(ctx, m, tokens, k, n_pack, &a, &b);
}

int ct_matmul_pack(rlwe_ctx* ctx, const rlwe_weights* w, uint32_t transpose, const uint64_t* ct_in,
                   uint32_t tokens, const rlwe_ksk* k, uint32_t n_pack, void* out, uint32_t flags,
                   rlwe_stream_t stream) {
  if (!ctx || !w || !k) return fail(RLWE_EINVAL, "ct_matmul_pack: null context, weights or key");
  if (k->ctx != ctx) return fail(RLWE_EINVAL, "ct_matmul_pack: key of another context");
  if (flags & ~(RLWE_OUT_RAW_Q | RLWE_OUT_FORCE_EXACT | RLWE_IN_SEEDED))
    return fail(RLWE_EINVAL, "ct_matmul_pack: unknown flags 0x%x", flags);
  if (n_pack < 1 || n_pack > ctx->rc.N)
    return fail(RLWE_ESHAPE, "n_pack = %u outside [1, N]", n_pack);
  ct_matmul_desc d{};
  d.w = w;
  d.transpose = transpose;
  d.ct_in = ct_in;
  d.tokens = tokens;
  d.out = out;
  const Mat* m;
  int r = validate_desc(ctx, d, &m);
  if (r != RLWE_OK) return r;
  if (tokens == 0) return ok();
  const size_t M = (size_t)tokens * m->args.rows;
  if ((M + n_pack - 1) / n_pack >= (1ull << 31))
    return fail(RLWE_ESHAPE, "ct_matmul_pack: %zu ciphertexts too many", M);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  size_t off_inter, off_ks;
  const size_t need = matmul_pack_ws(ctx, *m, tokens, k, n_pack, &off_inter, &off_ks);
  if (need > ctx->ws_bytes) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
      return fail(RLWE_EINVAL, "workspace must be reserved (rlwe_workspace_reserve) before capture");
    r = ensure_ws(ctx, need, s);
    if (r != RLWE_OK) return r;
  }
  unsigned char* ws = (unsigned char*)ctx->ws;
  d.out = ws + off_inter;
  // NTT method at N = 4096: the product rounds the masks for the key's decomposition;
  // otherwise it writes raw residues and the digit kernel rounds them
  const bool gadget = m->ntt && ctx->rc.N == kNttN;
  const uint32_t pflags = (flags & (RLWE_OUT_FORCE_EXACT | RLWE_IN_SEEDED)) | (gadget ? 0 : RLWE_OUT_RAW_Q);
  r = run_batch(ctx, &d, 1, pflags | RLWE_LAUNCH_GROUPED, s, ws, nullptr, gadget ? k : nullptr);
  if (r != RLWE_OK) return r;
  r = ks_run(ctx, k, (const uint64_t*)(ws + off_inter), M, n_pack, out, flags & RLWE_OUT_RAW_Q,
             gadget, ws + off_ks, s);
  if (r != RLWE_OK) return r;
  return ok();
}

}  // extern "C"

// ------------------------------------------------------------------ autotuning

namespace rlwe {
int measure_peaks(int hip_device, rlwe_peaks* out, const char** why);
}

extern "C" {

int rlwe_measure_peaks(int hip_device, rlwe_peaks* out) {
  if (!out) return fail(RLWE_EINVAL, "rlwe_measure_peaks: null argument");
  const char* why = "";
  const int r = measure_peaks(hip_device, out, &why);
  return r == RLWE_OK ? ok() : fail(r, "rlwe_measure_peaks: %s", why);
}

int rlwe_tuner_create(const char* device_key, rlwe_tuner** out) {
  if (!device_key || !out) return fail(RLWE_EINVAL, "rlwe_tuner_create: null argument");
  *out = new (std::nothrow) rlwe_tuner;
  if (!*out) return fail(RLWE_ENOMEM, "out of host memory");
  (*out)->cache.device = device_key;
  return ok();
}

int rlwe_tuner_destroy(rlwe_tuner* t) {
  delete t;
  return ok();
}

size_t rlwe_tuner_size(const rlwe_tuner* t) { return t ? t->cache.entries.size() : 0; }

int rlwe_tune_key(uint32_t N, uint32_t P, uint32_t K, uint32_t M, uint32_t n_o, uint32_t raw,
                  uint32_t tokens, char* buf, size_t len) {
  if (!buf || len == 0) return fail(RLWE_EINVAL, "rlwe_tune_key: null buffer");
  const std::string k = tune::product_key(N, P, K, M, n_o, raw, tokens);
  if (k.size() + 1 > len) return fail(RLWE_EINVAL, "rlwe_tune_key: buffer of %zu bytes too small", len);
  memcpy(buf, k.c_str(), k.size() + 1);
  return ok();
}

static bool schedule_valid(const rlwe_schedule& s) {
  return s.method <= 1 && s.tt_log2 <= 5 && s.order <= 1 && s.launch <= 1;
}

int rlwe_tuner_put(rlwe_tuner* t, const char* key, const rlwe_schedule* s) {
  if (!t || !key || !s) return fail(RLWE_EINVAL, "rlwe_tuner_put: null argument");
  if (tune::parse_key(key).kind < 0) return fail(RLWE_EINVAL, "rlwe_tuner_put: malformed key '%s'", key);
  if (!schedule_valid(*s)) return fail(RLWE_EINVAL, "rlwe_tuner_put: schedule out of range");
  t->cache.entries[key] = *s;
  return ok();
}

int rlwe_tuner_get(const rlwe_tuner* t, const char* key, rlwe_schedule* s) {
  if (!t || !key || !s) return fail(RLWE_EINVAL, "rlwe_tuner_get: null argument");
  const auto it = t->cache.entries.find(key);
  if (it == t->cache.entries.end()) return fail(RLWE_EINVAL, "rlwe_tuner_get: no entry '%s'", key);
  *s = it->second;
  return ok();
}

int rlwe_tuner_lookup(const rlwe_tuner* t, uint32_t N, uint32_t P, uint32_t K, uint32_t M,
                      uint32_t n_o, uint32_t raw, uint32_t tokens, rlwe_schedule* s) {
  if (!t || !s) return fail(RLWE_EINVAL, "rlwe_tuner_lookup: null argument");
  g_err.clear();
  return tune::find_product(t->cache, N, P, K, M, n_o, raw, tokens, s) ? 1 : 0;
}

int rlwe_tuner_save(const rlwe_tuner* t, const char* path) {
  if (!t || !path) return fail(RLWE_EINVAL, "rlwe_tuner_save: null argument");
  const std::string text = tune::to_json(t->cache);
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "wb");
  if (!f) return fail(RLWE_EINVAL, "rlwe_tuner_save: cannot open %s", tmp.c_str());
  const bool wrote = fwrite(text.data(), 1, text.size(), f) == text.size();
  if (fclose(f) != 0 || !wrote || rename(tmp.c_str(), path) != 0) {
    (void)remove(tmp.c_str());
    return fail(RLWE_EINVAL, "rlwe_tuner_save: cannot write %s", path);
  }
  return ok();
}

int rlwe_tuner_load(rlwe_tuner* t, const char* path, size_t* loaded) {
  if (!t || !path) return fail(RLWE_EINVAL, "rlwe_tuner_load: null argument");
  if (loaded) *loaded = 0;
  FILE* f = fopen(path, "rb");
  if (!f) return fail(RLWE_EINVAL, "rlwe_tuner_load: cannot open %s", path);
  std::string text;
  char buf[65536];
  size_t got;
  while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
  fclose(f);
  size_t n = 0;
  std::string err;
  if (!tune::from_json(text, &t->cache, &n, &err))
    return fail(RLWE_EINVAL, "rlwe_tuner_load: %s: %s", path, err.c_str());
  if (loaded) *loaded = n;
  return ok();
}

int rlwe_device_key(int hip_device, char* buf, size_t len) {
  if (!buf || len == 0) return fail(RLWE_EINVAL, "rlwe_device_key: null buffer");
  hipDeviceProp_t prop;
  const hipError_t e = hipGetDeviceProperties(&prop, hip_device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  const int n = snprintf(buf, len, "%s|%s|%d", prop.gcnArchName, prop.name, prop.multiProcessorCount);
  if (n < 0 || (size_t)n >= len) return fail(RLWE_EINVAL, "rlwe_device_key: buffer too small");
  return ok();
}

int rlwe_ctx_set_tuner(rlwe_ctx* ctx, rlwe_tuner* t) {
  if (!ctx) return fail(RLWE_EINVAL, "rlwe_ctx_set_tuner: null context");
  ctx->tuner = t;
  return ok();
}

}  // extern "C"

namespace {

// Device memory freed on scope exit.
struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

// Mean time of `reps` calls of fn on stream s after one untimed call (ms); <0 on error.
template <class F>
float time_calls(hipStream_t s, F fn, int reps) {
  hipEvent_t a = nullptr, b = nullptr;
  float ms = -1.f;
  if (fn() != RLWE_OK) return -1.f;
  if (hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess &&
      hipEventRecord(a, s) == hipSuccess) {
    bool good = true;
    for (int r = 0; r < reps && good; ++r) good = fn() == RLWE_OK;
    if (good && hipEventRecord(b, s) == hipSuccess && hipEventSynchronize(b) == hipSuccess &&
        hipEventElapsedTime(&ms, a, b) == hipSuccess)
      ms /= (float)reps;
    else
      ms = -1.f;
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  return ms;
}

}  // namespace

extern "C" {

int rlwe_autotune_product(rlwe_ctx* ctx, rlwe_tuner* t, uint32_t K, uint32_t M, uint32_t wflags,
                          uint32_t tokens, uint32_t oflags, rlwe_stream_t stream,
                          rlwe_schedule* best) {
  if (!ctx || !t) return fail(RLWE_EINVAL, "rlwe_autotune_product: null context or tuner");
  if (K < 1 || M < 1 || K > 65536 || M > 65536 || tokens < 1 || tokens > 65535)
    return fail(RLWE_ESHAPE, "rlwe_autotune_product: K = %u, M = %u, tokens = %u out of range", K,
                M, tokens);
  if ((wflags & ~RLWE_W_ROWPACK) || (oflags & ~RLWE_OUT_RAW_Q))
    return fail(RLWE_EINVAL, "rlwe_autotune_product: flags 0x%x / 0x%x invalid", wflags, oflags);
  const bool rowpack = wflags & RLWE_W_ROWPACK;
  if (rowpack && !ctx->ntt_ok) return fail(RLWE_EPARAM, "RLWE_W_ROWPACK needs N = %u", kNttN);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const RingConst& rc = ctx->rc;
  const bool raw = oflags & RLWE_OUT_RAW_Q;
  // weights of the largest magnitude that loads at this t (127 s K < t / 2): the
  // kernels' time does not depend on the values, only the matrix cores' kept digits
  // on the row norms
  const uint64_t t_half = 1ull << (ctx->log2_t - 1);
  const uint64_t mag = std::min<uint64_t>(127, (t_half - 1) / (127ull * K));
  if (mag == 0) return fail(RLWE_EOVERFLOW, "rlwe_autotune_product: K = %u cannot load at t = 2^%u", K, ctx->log2_t);
  DevBuf W, ct, out;
  const uint32_t L = (K + rc.N - 1) / rc.N;
  const size_t ct_words = (size_t)tokens * L * 2 * rc.P * rc.N;
  const size_t out_bytes = (size_t)tokens * M * (raw ? (size_t)rc.P * (rc.N + 1) * 8 : (size_t)(rc.N + 1) * 4);
  if ((e = hipMalloc(&W.p, (size_t)M * K)) != hipSuccess ||
      (e = hipMalloc(&ct.p, ct_words * 8)) != hipSuccess ||
      (e = hipMalloc(&out.p, out_bytes)) != hipSuccess)
    return fail(RLWE_ENOMEM, "rlwe_autotune_product: hipMalloc: %s", hipGetErrorString(e));
  e = launch_fill_int8((int8_t*)W.p, (size_t)M * K, (uint32_t)mag, 0x5eed0001ull, s);
  if (e == hipSuccess) e = launch_fill_residues((uint64_t*)ct.p, ct_words, rc, 0x5eed0002ull, s);
  if (e != hipSuccess) return hip_fail(e, "tuning inputs");
  // weights on each method to try (explicit method flags: the tuner is not consulted)
  rlwe_weights* wn = nullptr;
  rlwe_weights* wt = nullptr;
  int r = RLWE_OK;
  if (ctx->ntt_ok)
    r = rlwe_weights_load(ctx, (const int8_t*)W.p, M, K,
                          RLWE_W_FWD | RLWE_W_NTT | (rowpack ? RLWE_W_ROWPACK : 0), stream, &wn);
  if (r == RLWE_OK && !rowpack)
    r = rlwe_weights_load(ctx, (const int8_t*)W.p, M, K, RLWE_W_FWD | RLWE_W_TOEPLITZ, stream, &wt);
  size_t need = 0;
  if (wn) need = std::max(need, rlwe_workspace_bytes(ctx, wn, 0, tokens));
  if (wt) need = std::max(need, rlwe_workspace_bytes(ctx, wt, 0, tokens));
  if (r == RLWE_OK) r = ensure_ws(ctx, need, s);
  const uint32_t n_o = wn ? wn->fwd.args.n_o : 1;
  std::vector<rlwe_schedule> cands;
  if (wt) cands.push_back(rlwe_schedule{RLWE_METHOD_TOEPLITZ, kTokTileLog2, 0, 0, 0.f});
  if (wn)
    for (uint32_t tl = 0; tl <= 4; ++tl) {
      if (tl > 0 && (1u << tl) >= 2 * tokens) break;
      for (uint32_t order = 0; order < 2; ++order)
        for (uint32_t launch = 0; launch < (rc.N == kNttN ? 2u : 1u); ++launch)
          cands.push_back(rlwe_schedule{RLWE_METHOD_NTT, tl, order, launch, 0.f});
    }
  rlwe_schedule pick{};
  float pick_ms = -1.f;
  for (size_t c = 0; c < cands.size() && r == RLWE_OK; ++c) {
    rlwe_weights* w = cands[c].method == RLWE_METHOD_NTT ? wn : wt;
    ctx->forced = &cands[c];
    auto call = [&] { return ct_matmul_clear(ctx, w, 0, (const uint64_t*)ct.p, tokens, out.p, oflags, stream); };
    float ms = time_calls(s, call, 1);  // a first estimate decides the repetitions
    if (ms >= 0.f && ms < 100.f) ms = time_calls(s, call, ms < 5.f ? 5 : 2);
    ctx->forced = nullptr;
    if (ms < 0.f) {
      if (g_err.empty()) r = fail(RLWE_EHIP, "rlwe_autotune_product: timing failed");
      else r = RLWE_EHIP;
      break;
    }
    cands[c].ms = ms;
    if (pick_ms < 0.f || ms < pick_ms) {
      pick = cands[c];
      pick_ms = ms;
    }
  }
  ctx->forced = nullptr;
  const std::string msg = g_err;
  (void)hipStreamSynchronize(s);
  rlwe_weights_free(wn);
  rlwe_weights_free(wt);
  if (r != RLWE_OK) {
    g_err = msg;
    return r;
  }
  t->cache.entries[tune::product_key(rc.N, rc.P, K, M, n_o, raw, tokens)] = pick;
  if (best) *best = pick;
  return ok();
}

int rlwe_autotune_batch(rlwe_ctx* ctx, rlwe_tuner* t, const ct_matmul_desc* descs, uint32_t n,
                        uint32_t flags, rlwe_stream_t stream, rlwe_schedule* best) {
  if (!ctx || !t || !descs) return fail(RLWE_EINVAL, "rlwe_autotune_batch: null argument");
  if (n < 1 || n > kMaxBatch) return fail(RLWE_EINVAL, "rlwe_autotune_batch: 1 <= n <= %d", kMaxBatch);
  if (flags & ~(RLWE_OUT_RAW_Q | RLWE_IN_SEEDED))
    return fail(RLWE_EINVAL, "rlwe_autotune_batch: flags 0x%x invalid", flags);
  uint32_t cnt = 0, maxT = 0;
  bool all_ntt = true;
  for (uint32_t i = 0; i < n; ++i) {
    const Mat* m;
    const int r = validate_desc(ctx, descs[i], &m);
    if (r != RLWE_OK) return r;
    if (descs[i].tokens) {
      ++cnt;
      maxT = std::max(maxT, descs[i].tokens);
      all_ntt = all_ntt && m->ntt;
    }
  }
  if (cnt == 0) return fail(RLWE_EINVAL, "rlwe_autotune_batch: no tokens");
  hipStream_t s = (hipStream_t)stream;
  auto run = [&](uint32_t launch) { return ct_matmul_batch(ctx, descs, n, flags | launch, stream); };
  const float g = time_calls(s, [&] { return run(RLWE_LAUNCH_GROUPED); }, 3);
  all_ntt = all_ntt && ctx->rc.N == kNttN;  // the persistent launch is written for N = 4096
  const float p = all_ntt ? time_calls(s, [&] { return run(RLWE_LAUNCH_PERSISTENT); }, 3) : -1.f;
  if (g < 0.f || (all_ntt && p < 0.f))
    return g_err.empty() ? fail(RLWE_EHIP, "rlwe_autotune_batch: timing failed") : RLWE_EHIP;
  rlwe_schedule pick{all_ntt ? RLWE_METHOD_NTT : RLWE_METHOD_TOEPLITZ, kTokTileLog2, 0, 0, g};
  if (all_ntt && p < g) {
    pick.launch = 1;
    pick.ms = p;
  }
  t->cache.entries[tune::batch_key(ctx->rc.N, ctx->rc.P, cnt, flags & RLWE_OUT_RAW_Q, maxT)] = pick;
  if (best) *best = pick;
  return ok();
}

}  // extern "C"
