// Internal declarations of the gfx950 library: kernel argument blocks, exact
// integer helpers shared by the kernels, launcher prototypes.
//
// Representation used by the kernels (free choices behind the ABI; none of them
// changes a result bit):
//   * A ciphertext coefficient, given by its residues mod q_p, is lifted once to
//     its centred integer value c in (-q/2, q/2) and written in balanced base 255,
//     c = sum_{l<D} d_l 255^l with every digit d_l in [-127, 127]. D = 7 for one
//     54-bit prime, 14 for two.
//   * The mask part of Eq. (LWEdot) becomes, per digit l, an exact int32 matrix
//     product of the int8 weights with a Toeplitz matrix of int8 digits (the
//     negacyclic sign is absorbed by storing the negated digits in front of each
//     digit plane), executed on the int8 matrix cores; the digit sums are
//     recombined (sum_l 255^l S_l) and the modulus switch is applied to the exact
//     integer they represent.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rlwe {

typedef unsigned __int128 u128;
typedef __int128 i128;

constexpr int kMaxDigits = 14;   // balanced base-255 digits of a value below 2^108
constexpr int kMaxPrimes = 2;

// Constants of the cryptosystem shared by every kernel (passed by value).
struct RingConst {
  uint32_t N, logN, P, D;          // ring degree, log2 N, #primes, #digits
  uint64_t q[kMaxPrimes];          // RNS primes
  uint64_t crt_inv[kMaxPrimes];    // (q / q_p)^-1 mod q_p
  uint64_t crt_inv_shoup[kMaxPrimes];  // floor(crt_inv * 2^64 / q_p)
  uint64_t Q_lo, Q_hi;             // q = prod q_p as 128-bit
  uint64_t half_lo, half_hi;       // (q - 1) / 2
  uint32_t qbits;                  // switched outputs are modulo q_out = 2^qbits (1..32)
  double inv_qout;                 // 2^qbits / q (estimate only; results are corrected exactly)
  // Digit l of the balanced base-255 expansion carries G_l = round(255^l 2^96 / q) mod 2^96
  // (255^l 2^32 / q mod 2^32 in 32.64 fixed point), as words G_l = a + b 2^32 + c 2^64 with
  // a, b in [-2^31, 2^31): the matrix-core epilogue adds floor(S a / 2^32) + S b +
  // (S c mod 2^32) 2^32 for a digit sum S.
  int32_t dg[kMaxDigits][3];
};

// Constants of the number-theoretic-transform method (N = kNttN only).
constexpr uint32_t kNttN = 4096;
constexpr uint32_t kTokTileLog2 = 3;  // default: 8 tokens per workgroup of the NTT product kernel
struct NttConst {
  const uint64_t* fwd[kMaxPrimes];  // [N] (psi^bitrev(k), Shoup companion), device
  const uint64_t* inv[kMaxPrimes];  // [N] (psi^-bitrev(k), Shoup companion), device
  uint64_t crt[kMaxPrimes];         // (q / q_p)^-1 mod q_p (1 for one prime); the factor N^-1 of
                                    // the inverse transform is folded into the NTT weights
  uint64_t crt_shoup[kMaxPrimes];
  uint64_t ninv[kMaxPrimes];        // N^-1 mod q_p
  uint64_t ninv_shoup[kMaxPrimes];
  uint32_t bm[kMaxPrimes];          // floor(2^64 / q_p), the Barrett factor of the inverse
  uint64_t rq[kMaxPrimes][2];       // floor(2^128 / q_p): high word, low word
  // H_p = crt_p 2^32 / q_p mod 2^32 in 32.96 fixed point (little-endian words):
  // the switched coefficient is round(sum_p c_p H_p) mod 2^32 for any integers
  // c_p = C mod q_p (multiples of q_p change the sum by multiples of 2^32)
  uint32_t h[kMaxPrimes][4];
  // The same for the outputs of the inverse transform's last stage that its twiddle w
  // (one value for the whole stage) would multiply: the product kernel's switched
  // epilogue takes those differences unmultiplied, with w folded into the constants:
  // crtl = crt w mod q_p (and its Shoup companion), hl = H_p for crtl.
  uint64_t crtl[kMaxPrimes];
  uint64_t crtl_shoup[kMaxPrimes];
  uint32_t hl[kMaxPrimes][4];
};

// Per weight-matrix constants of the switched epilogue (matrix-core method).
struct SwitchConst {
  uint32_t l0;        // digits below l0 are left out of the matrix-core sums
  uint32_t dk;        // digits kept: D - l0
  uint32_t epsw;      // half-width of the uncertain band around a rounding tie of the
                      // per-digit fixed-point sum (RingConst::dg), in 2^-32 units
};

// ---------------------------------------------------------------- integer helpers

__host__ __device__ inline u128 make_u128(uint64_t hi, uint64_t lo) {
  return ((u128)hi << 64) | lo;
}

// Canonical residue of a signed 128-bit value (|v| < 2^127) modulo q < 2^63.
__device__ inline uint64_t mod_i128(i128 v, uint64_t q) {
  const bool neg = v < 0;
  u128 m = neg ? (u128)(-v) : (u128)v;
  uint64_t r = (uint64_t)(m % q);
  return (neg && r) ? q - r : r;
}

__device__ inline double i128_to_double(i128 v) {
  const int64_t hi = (int64_t)(v >> 64);
  const uint64_t lo = (uint64_t)v;
  return (double)hi * 18446744073709551616.0 + (double)lo;
}

// Seeded masks (Sec. 3.1: the client sends a seed in place of the uniform mask).
// SplitMix64 (Steele, Lea and Flood, 2014) as a counter-based generator: output
// ctr under seed is the finalizer applied to seed + (ctr + 1) * golden gamma.
__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t ctr) {
  uint64_t z = seed + (ctr + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// Mask coefficient n of prime p (q_p < 2^54): the top 54 bits of the first of the
// draws (p N + n) 16 + j, j < 16, that lies below q_p; if none does (probability
// below 2^-200), the first draw mod q_p.
__device__ inline uint64_t seeded_mask(uint64_t seed, uint32_t N, uint32_t p, uint32_t n,
                                       uint64_t q) {
  const uint64_t base = ((uint64_t)p * N + n) << 4;
  for (uint32_t j = 0; j < 16; ++j) {
    const uint64_t v = splitmix64_at(seed, base | j) >> 10;
    if (v < q) return v;
  }
  return (splitmix64_at(seed, base) >> 10) % q;
}
// Words of one input block: the full layout [A, B] (2 P N) or the seeded one
// [seed, 0, B] (P N + 2).
__host__ __device__ inline size_t ct_block_words(uint32_t P, uint32_t N, bool seeded) {
  return seeded ? (size_t)P * N + 2 : (size_t)2 * P * N;
}

__host__ __device__ inline uint32_t qout_mask(uint32_t k) {
  return k >= 32 ? 0xffffffffu : (1u << k) - 1u;
}

// round(V * 2^k / q) mod 2^k (k = rc.qbits) for an exact integer V with
// |V| < 2^127 and |V 2^k / q| < 2^53. A double estimate is corrected by exact
// remainder arithmetic modulo 2^128: Z = V 2^k - F q is computed with wrapping
// 128-bit operations, which is exact because the true Z lies in [0, 2^128).
__device__ inline uint32_t switch_exact(i128 V, const RingConst& rc) {
  const u128 q = make_u128(rc.Q_hi, rc.Q_lo);
  const double est = i128_to_double(V) * rc.inv_qout;
  int64_t f = (int64_t)floor(est) - 8;  // |est - V 2^k/q| < 4 for these magnitudes
  u128 z = ((u128)V << rc.qbits) - (u128)(i128)f * q;
  for (int it = 0; it < 24 && z >= q; ++it) {
    z -= q;
    ++f;
  }
  return (uint32_t)(f + (2 * z > q ? 1 : 0)) & qout_mask(rc.qbits);
}

// Rounding to q_out = 2^k of a value given in 32.32 fixed point: W = x 2^32 with
// x = c 2^32 / q mod 2^32, so c 2^k / q = W / 2^(64 - k). Returns the rounded value
// mod 2^k and, in dist, the fraction minus one half in units of W (negative below
// the tie). With k = 32 this is the integer part W >> 32 and its top fraction bit.
__device__ inline uint32_t round_qout(uint64_t W, uint32_t k, int64_t& dist) {
  const uint32_t sh = 64 - k;  // fraction bits, 32..63
  const uint64_t frac = W & ((1ull << sh) - 1);
  const uint64_t half = 1ull << (sh - 1);
  dist = (int64_t)(frac - half);
  return (uint32_t)((W >> sh) + (frac >= half ? 1 : 0)) & qout_mask(k);
}

// The same rounding for a W known to be at most 7 units low, from the words of
// V = W + 2^(sh-1) (mod 2^64; the caller adds the half), k = 1..32, sh = 64 - k >= 32:
// floor(V / 2^sh) mod 2^k = vhi >> (32 - k) (adding one half carries into the integer
// part exactly when the fraction reaches it, and a wrap past 2^64 is a multiple of
// 2^sh 2^k), and in near whether the fraction may lie within 8 units below one half,
// where the exact value may round the other way. Then the fraction of V is at least
// 2^sh - 8, so the low word of V is at least 2^32 - 8: that test flags every such W,
// and when k < 32 also some others (with probability 2^-29), which only take the exact
// route.
__device__ __forceinline__ uint32_t round_qout_near(uint32_t vlo, uint32_t vhi, uint32_t k,
                                                    bool& near) {
  __asm__("" : "+v"(vlo));  // one 32-bit compare (else a masked 64-bit one)
  near = vlo >= 0xFFFFFFF8u;
  return vhi >> (32 - k);
}

// Shoup multiplication a * w mod q, wp = floor(w 2^64 / q), a < 2^64, q < 2^63.
__device__ inline uint64_t mulmod_shoup(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
  const uint64_t qh = __umul64hi(a, wp);
  uint64_t r = a * w - qh * q;
  return r >= q ? r - q : r;
}

// ---------------------------------------------------------------- launchers

struct MatArgs {
  const int8_t* w;      // resident weights [rows_pad][kw], zero padded
  uint32_t rows;        // outputs M
  uint32_t rows_pad;    // multiple of 64
  uint32_t k;           // contraction length K
  uint32_t kw;          // row pitch: K rounded up to 64
  uint32_t L;           // input blocks
  // Rows per weight polynomial and the slot each occupies (NTT method): 1 and N for
  // the reversed encoding of Sec. 4.3; with multi-row packing (K <= N/2, one block)
  // floor(N / K) rows, row rho of a group reversed in coefficients [rho K, rho K + K)
  uint32_t n_o;
  uint32_t slot;
};

// Body launch geometry (256 threads per block). Unpacked rows: one thread per row.
// Packed rows: threads in slot-major order v = rho gpad + g over the groups g padded
// to a multiple of 64, so that every wave holds a single slot rho.
__host__ __device__ inline uint32_t body_group_pad(const MatArgs& m) {
  return ((m.rows + m.n_o - 1) / m.n_o + 63) / 64 * 64;
}
__host__ __device__ inline uint32_t body_blocks_per_token(const MatArgs& m) {
  return m.n_o > 1 ? (m.n_o * body_group_pad(m) + 255) / 256 : (m.rows + 255) / 256;
}

// Constants of the gadget rounding a~ = round(c 2^K / q) mod 2^K of a coefficient
// given by its residues (Decomp's first step). With inv_p = (q/q_p)^-1 mod q_p (1 for
// one prime): inv_p 2^K = f_p q_p + g_p.
struct KsRound {
  uint64_t q[kMaxPrimes];
  uint64_t Q_hi, Q_lo;               // q = prod q_p (two primes)
  uint64_t f[kMaxPrimes];            // floor(inv_p 2^K / q_p) mod 2^64
  uint64_t g[kMaxPrimes];            // inv_p 2^K mod q_p
  uint64_t g_shoup[kMaxPrimes];      // floor(g 2^64 / q_p)
  uint64_t G_lo[kMaxPrimes];         // G = floor(g 2^96 / q_p) < 2^96: bits 0..63
  uint32_t G_hi[kMaxPrimes];         //   and bits 64..95
};
// One product of a batch: weights, input ciphertexts, workspace planes, output.
struct Item {
  MatArgs m;
  SwitchConst sc;
  uint32_t method;     // 0: digit planes on the matrix cores, 1: NTT
  const uint64_t* what;  // NTT method: [rows][L][P][N] transformed weight blocks (lane-major)
  uint64_t* ahat;        // NTT method: [T][L][P][N] (mask, Shoup companion) pairs, lane-major (workspace)
  const uint64_t* ct;  // [T][L][2][P][N]
  int8_t* emask;       // [T][D][L][2N]: per digit plane, index m <-> Toeplitz offset m - N
  int8_t* ebody;       // [T][D][L][N]
  void* out;           // switched u32 [T][M][N+1], raw u64 [T][M][P][N+1], or rounded u64 [T][M][N+P]
  uint32_t T;
  uint32_t tt_log2;    // NTT method: log2 of the tokens per workgroup (token tile)
  uint32_t order;      // NTT method: 0 token tiles vary fastest in the block order, 1 weight
                       // polynomials do
  uint32_t groups;     // weight polynomials: ceil(rows / n_o)
};

constexpr int kMaxBatch = 16;

// A batch of products launched together; every kernel maps its linear block index
// onto (item, local block) through the prefix sums below. Passed by value.
struct Batch {
  RingConst rc;
  uint32_t n;
  uint32_t raw;
  uint32_t force_exact;
  uint32_t seeded;  // inputs in the seeded layout: per block [seed, 0, B residues]
  uint32_t gadget;  // (with raw) masks rounded to 2^K: outputs [T][M][N+P], a~ then bodies
  uint64_t kmask;   // 2^K - 1
  KsRound kr;
  NttConst ntt;
  uint32_t prep_start[kMaxBatch + 1];  // blocks of 256 threads over T*L*N coefficients
  uint32_t fwd_start[kMaxBatch + 1];   // NTT method: one transform per (token, block, prime)
  uint32_t mask_start[kMaxBatch + 1];  // workgroups over T * rows_pad/32 * N/64 tiles (NTT: rows * token tiles)
  uint32_t body_start[kMaxBatch + 1];  // blocks of 256 threads over T * rows
  uint32_t unit_start[kMaxBatch + 1];  // persistent launch: transform units (token, input block)
  uint32_t* sync;                      // persistent launch: queue counters (kSync* words)
  Item it[kMaxBatch];
};
// Words of the persistent launch's counter block (zero between launches).
constexpr uint32_t kSyncHead = 0;   // next work item
constexpr uint32_t kSyncExit = 1;   // workgroups finished
constexpr uint32_t kSyncErr = 2;    // set if a bounded wait gave up
constexpr uint32_t kSyncDone = 4;   // + item: transform units of the item done
constexpr uint32_t kSyncPrep = kSyncDone + kMaxBatch;  // + item: digit blocks of the item done
constexpr uint32_t kSyncWords = kSyncPrep + kMaxBatch;

// KeySwitch packing (Sec. 3.2 KeySwitching, Eq. (pack_rotate)); N = kNttN only.
constexpr uint32_t kMaxLevels = 4;   // gadget levels ell
constexpr uint32_t kKsGroups = 64;   // packed outputs per pass of the kernels
struct KsConst {
  uint32_t beta, ell, K;             // digit bits, levels, K = beta ell rounding bits (<= 64)
  uint64_t kmask;                    // 2^K - 1
  uint64_t H;                        // sum_m 2^(beta-1) 2^(beta m) mod 2^64
  KsRound rd;
};
// Arguments of the KeySwitch kernels (read in place through the kernarg segment).
struct KsArgs {
  RingConst rc;
  NttConst ntt;
  KsConst kc;
  const uint64_t* lwe;   // [M][P][N+1] LWE ciphertexts, residues
  uint64_t M;
  uint32_t n_pack;       // slots filled per packed output
  uint32_t g0, GB;       // first output group of this pass, groups in the pass
  uint32_t raw;          // outputs modulo q per prime (else switched to 2^qbits)
  uint32_t pre;          // lwe holds rounded masks: [M][N+P] (a~ mod 2^K, then the P body
                         // residues), else raw LWE ciphertexts [M][P][N+1]
  int64_t* dig;          // workspace: digits [GB][N][ell][N]
  const uint64_t* khat;  // key in the NTT domain [N][ell][P][2][N][2] (value, Shoup companion), lane-major
  uint64_t* part;        // workspace: partial sums [GB][N / 64][P][2][N]
  void* out;             // [G][2][P][N] u64 or [G][2][N] u32
  const uint64_t* ksk_in;  // key load: [N][ell][2][P][N] canonical residues
  uint64_t* khat_out;      // key load: destination of the transformed key
};

// Kernels take the Batch as their only argument and read it in place through the
// kernarg segment pointer (constant address space, uniform scalar loads); indexing
// the by-value parameter directly would make every thread copy it to scratch.
typedef const __attribute__((address_space(4))) Batch* BatchPtr;
__device__ inline BatchPtr kernarg_batch() {
  return (BatchPtr)__builtin_amdgcn_kernarg_segment_ptr();
}

// Copy of a kernarg-resident object into private storage (registers).
template <class T>
__device__ inline T kernarg_load(const __attribute__((address_space(4))) T* p) {
  T r;
  __builtin_memcpy(&r, (const void*)p, sizeof(T));
  return r;
}

// Item owning linear block b (uniform per workgroup); start is a prefix-sum table.
__device__ inline uint32_t find_item(const __attribute__((address_space(4))) uint32_t* start,
                                     uint32_t n, uint32_t b) {
  uint32_t i = 0;
  while (i + 1 < n && b >= start[i + 1]) ++i;
  return i;
}

// Linear block index of a 2D grid (grids are split over y to keep x * block < 2^32).
__device__ inline uint32_t linear_block() { return blockIdx.y * gridDim.x + blockIdx.x; }


// 2D grid covering `blocks` blocks of `threads` threads.
inline dim3 grid_for(uint32_t blocks) {
  const uint32_t x = blocks < 32768u ? blocks : 32768u;
  return dim3(x, (blocks + x - 1) / x);
}

hipError_t launch_prep(const Batch& b, hipStream_t s);
hipError_t launch_mask(const Batch& b, uint32_t dk, hipStream_t s);
hipError_t launch_body(const Batch& b, hipStream_t s);
hipError_t launch_ntt_mask_fwd(const Batch& b, hipStream_t s);
// lclass: every item of b has L = 2 (2), or any L (0)
hipError_t launch_ntt_mask(const Batch& b, uint32_t lclass, hipStream_t s);
// every item of b on the NTT method, sync set; grid workgroups of kInvThreads threads
hipError_t launch_persist(const Batch& b, uint32_t grid, hipStream_t s);
hipError_t launch_ntt_weights(const MatArgs& m, const NttConst& ntt, const RingConst& rc,
                              uint64_t* what, hipStream_t s);
hipError_t launch_pack_bits(const uint32_t* in, size_t count, uint32_t len, uint32_t k,
                            uint32_t* out, hipStream_t s);
hipError_t launch_modswitch(const RingConst& rc, const uint64_t* in, size_t count, uint32_t* out,
                            hipStream_t s);
hipError_t launch_transpose_pad(const int8_t* src, uint32_t rows, uint32_t cols, bool transpose,
                                int8_t* dst, uint32_t dst_rows_pad, uint32_t dst_kw,
                                hipStream_t s);
hipError_t launch_ksk_fwd(const KsArgs& a, hipStream_t s);
hipError_t launch_ks_digits(const KsArgs& a, hipStream_t s);
hipError_t launch_ks_accum(const KsArgs& a, hipStream_t s);
hipError_t launch_ks_finish(const KsArgs& a, hipStream_t s);
hipError_t launch_row_l1(const int8_t* w, uint32_t rows, uint32_t kw, uint32_t* out,
                         hipStream_t s);
hipError_t launch_fill_residues(uint64_t* dst, size_t count, const RingConst& rc, uint64_t seed,
                                hipStream_t s);
hipError_t launch_fill_int8(int8_t* dst, size_t count, uint32_t mag, uint64_t seed,
                            hipStream_t s);

}  // namespace rlwe
