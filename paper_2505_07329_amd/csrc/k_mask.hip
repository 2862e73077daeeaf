// The mask part of Eq. (LWEdot) (Sec. 4.3) on the int8 matrix cores of gfx950.
//
// For token t, output row j and mask index n, summed over input blocks i,
//   a'_j[n] = sum_k w_j[iN + k] * ( A_i[k - n]        if k >= n
//                                  -A_i[N + k - n]    if k <  n )   (mod q)
// which is SampleExtract at N-1 of the product RLWE(x_i) . w_ij with the
// reversed weight encoding. With A_i written in balanced base-255 digits
// (A_i = sum_l 255^l d_l), every digit contributes an exact int32 matrix
// product S_l[j][n] = sum_k W[j][k] T_l[k][n], T_l[k][n] = plane_l[N + k - n],
// where the digit plane stores -d_l in front of d_l (the negacyclic wrap).
// T_l is Toeplitz: the operand fragment of a 32-wide column block at k-step k0
// is a 16-byte window of one plane, read from LDS at a byte offset.
//
// Epilogue, switched output: the integer V = sum_l 255^l S_l satisfies
// V = a'_j[n] (mod q), and round(V 2^32 / q) mod 2^32 is the switched
// coefficient. Digits below l0 change V 2^32/q by less than the host-computed
// bound eps; they are skipped, and every kept digit adds S_l G_l in 32.32 fixed
// point mod 2^64, G_l = round(255^l 2^96 / q) mod 2^96. Where the sum lies
// within eps of a rounding tie, the element is recomputed exactly from all
// digits (rare: probability about 2 eps). Raw output: all digits, V mod q_p.
#include "rlwe_internal.hpp"

namespace rlwe {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kKC = 256;                 // k-chunk staged in LDS per pass (8 k-steps)
// LDS layout of one digit window: four copies of kCopyWords dwords at dword offsets
// 0, 80, 168, 248. Copy 0 holds the window as is; copy s = 1..3 holds it shifted
// by s - 4 bytes (word u = window bytes [4u + s - 4, 4u + s)). A lane's 16-byte
// fragment starts at window byte lb + 32 st (lb = 16 g - c + 64 in [33, 80]); it
// is the aligned quad at word ceil(lb / 4) + 8 st of copy lb & 3, so the words
// read span [1, 80) for every copy. A fragment is read as dword pairs, which LDS
// serves as dword accesses of 32 lanes over 32 banks: per half-wave each copy is
// read at eight consecutive words starting at the same index, and offsets in four
// distinct residue classes mod 32 in steps of 8 put the four copies on disjoint
// banks. The offsets are multiples of four dwords (aligned 16-byte staging stores).
constexpr int kCopyWords = 80;
static_assert((80 + 3) / 4 + 8 * (kKC / 32 - 1) + 3 < kCopyWords, "window covers every fragment");
__host__ __device__ constexpr int copy_base(int s) { return s == 0 ? 0 : s == 1 ? 80 : s == 2 ? 168 : 248; }
constexpr int kDigitWords = 248 + kCopyWords;  // 328
constexpr int kWRowWords = kKC / 4 + 4;    // LDS row pitch of the weight tile (dwords)

// Exact switched value of element (t, jj, nn), computed by the whole wave: every
// lane accumulates a strided share of the contraction for all D digits, the
// shares are summed across the wave, and the exact rounding is taken from the
// integer V = sum_l 255^l S_l. Used where the fast path lies near a tie.
// The constants are read from the kernarg segment here: handing the caller's
// copies over by reference would force every thread to keep them in scratch.
template <int D>
__device__ inline uint32_t exact_element_wave(BatchPtr bt, uint32_t ii,
                                                                 uint32_t t, uint32_t jj,
                                                                 uint32_t nn, int lane) {
  const RingConst rc = kernarg_load(&bt->rc);
  const MatArgs m = kernarg_load(&bt->it[ii].m);
  const int8_t* emask = bt->it[ii].emask;
  const uint32_t N = rc.N;
  int32_t S[D];
#pragma unroll
  for (int l = 0; l < D; ++l) S[l] = 0;
  for (uint32_t i = 0; i < m.L; ++i) {
    const uint32_t kb = min(N, m.k - i * N);
    const int8_t* wrow = m.w + (size_t)jj * m.kw + (size_t)i * N;
    for (uint32_t k = lane; k < kb; k += 64) {
      const int32_t wv = wrow[k];
#pragma unroll
      for (int l = 0; l < D; ++l)
        S[l] += wv * (int32_t)emask[(((size_t)t * D + l) * m.L + i) * 2 * N + N + k - nn];
    }
  }
#pragma unroll
  for (int l = 0; l < D; ++l) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) S[l] += __shfl_xor(S[l], off);
  }
  i128 V = 0;
#pragma unroll
  for (int l = D - 1; l >= 0; --l) V = V * 255 + S[l];
  return switch_exact(V, rc);
}

// 16-byte Toeplitz fragment: four consecutive dwords of a byte-shifted window copy.
__device__ inline v4i toeplitz_frag(const uint32_t* p) {
  v4i f;
  __builtin_memcpy(&f, p, 16);
  return f;
}
__device__ inline v4i toeplitz_frag(const __attribute__((address_space(3))) uint32_t* p) {
  return v4i{(int)p[0], (int)p[1], (int)p[2], (int)p[3]};
}

// Asynchronous 16-byte copy global -> LDS (LDS DMA): lane x of the wave writes its
// 16 bytes at LDS byte address lds_wave + 16 x (lds_wave uniform across the wave).
// Issued as assembly so that the compiler does not make every later LDS read wait
// for it; callers wait for completion themselves (wait_vmem) before the barrier
// that publishes the data.
__device__ inline void lds_dma16(const void* src, uint32_t lds_wave) {
  asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off"
               :
               : "v"(src), "s"(lds_wave)
               : "memory", "m0");
}

__device__ inline uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) unsigned char*)p;
}

// s_waitcnt vmcnt(0): every vector memory load of this thread (LDS DMA included) landed.
__device__ inline void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0f70); }

// Work split: a workgroup owns a 32-row x 64-column output tile of one token
// and all DK kept digits; its NW = ceil(DK/3) waves each take at most 3 digits
// (the role of a wave rotates with the tile so that heavier roles spread over
// the SIMDs). Each wave covers both 32-column blocks: along a diagonal the
// Toeplitz fragment of block 1 at k-step k0 equals that of block 0 at k0 - 32,
// so every k-step reads one new fragment per digit and feeds two MFMAs.
// Epilogue: per-wave partial sums over its digits (int64) meet in LDS; each
// wave finishes a share of the elements.
// FULL: every chunk of every item spans kKC contraction bytes (K a multiple of kKC,
// N >= kKC), so the k-loop is straight-line code with immediate LDS offsets.
template <int D, int DK, bool RAW, bool FULL>
__global__ void __launch_bounds__(64 * ((DK + 2) / 3)) __attribute__((amdgpu_waves_per_eu(3)))
mask_kernel(Batch) {
  static_assert(!RAW || DK == D, "raw output keeps every digit");
  constexpr int NW = (DK + 2) / 3;
  constexpr int DPW = 3;
  constexpr int NT = 64 * NW;
  // LDS: per kept digit four copies of the chunk's window, copy s shifted by s bytes
  // (every fragment becomes an aligned-dword read), then two weight-tile buffers
  // (rows of 17 16-byte slots, the last one padding) filled by LDS DMA;
  // after the k-loop the same memory holds the per-wave partial sums.
  constexpr int kWinLds = DK * kDigitWords * 4;
  constexpr int kWSlots = 32 * (kWRowWords / 4);           // 544 16-byte slots per tile
  constexpr int kWIters = (kWSlots + NT - 1) / NT;         // DMA passes per thread
  constexpr int kWBuf = kWIters * NT * 16;                 // bytes per weight buffer
  constexpr int kPartLds = NW * 16 * 64 * 8;
  constexpr int kLds = kWinLds + 2 * kWBuf > kPartLds ? kWinLds + 2 * kWBuf : kPartLds;
  static_assert(kWRowWords == 68, "weight rows of 16 data slots and one pad slot");
  __shared__ __attribute__((aligned(16))) unsigned char smem[kLds];
  uint32_t* win = reinterpret_cast<uint32_t*>(smem);
  int64_t* part = reinterpret_cast<int64_t*>(smem);

  const BatchPtr bt = kernarg_batch();
  const uint32_t blk = linear_block();
  const uint32_t nb = bt->n;
  if (blk >= bt->mask_start[nb]) return;
  const uint32_t ii = find_item(bt->mask_start, nb, blk);
  const RingConst rc = kernarg_load(&bt->rc);
  const MatArgs m = kernarg_load(&bt->it[ii].m);
  const SwitchConst sc = kernarg_load(&bt->it[ii].sc);
  const int8_t* __restrict__ emask = bt->it[ii].emask;
  void* out = bt->it[ii].out;
  const int force_exact = bt->force_exact;
  const uint32_t N = rc.N;
  // tile order: column tiles fastest, then row tiles, then tokens
  const uint32_t ntn = N / 64, ntj = m.rows_pad / 32;
  const uint32_t loc = blk - bt->mask_start[ii];
  const uint32_t tn = loc % ntn, tj = (loc / ntn) % ntj;
  const uint32_t t = loc / (ntn * ntj);
  const uint32_t n0 = tn * 64, jb = tj * 32;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = lane & 31, g = lane >> 5;
  const int role = (wave + tn + tj) % NW;
  const int cnt = (DK % NW == 0) ? DK / NW : DK / NW + (role < DK % NW ? 1 : 0);
  const int dlo = role * (DK / NW) + min(role, DK % NW);
  const uint32_t l0 = D - DK;
  // lane byte offset of block 0 at k-step 0 inside a window; block 1 sits 32 bytes
  // (8 dwords) lower and each k-step moves 32 bytes up, so the shift is fixed
  const int lb = 16 * g - c + 64;
  const int sh = lb & 3;

  v16i acc0[DPW], acc1[DPW];
#pragma unroll
  for (int d = 0; d < DPW; ++d) acc0[d] = acc1[d] = v16i{0};

  // Fragment addresses of this lane are the same for every chunk: block 0's
  // Toeplitz fragment of digit d at k-step st is 16 bytes at ep[d] + 8 st
  // (dwords), the weight fragment at wl + 8 st.
  // Each base is made opaque to the compiler: derived from one another they would be
  // folded into one register plus offsets beyond the 8-bit range of ds_read2_b32,
  // costing an address addition per fragment.
  typedef const __attribute__((address_space(3))) uint32_t* lds_u32;
  lds_u32 ep[DPW];
#pragma unroll
  for (int d = 0; d < DPW; ++d) {
    ep[d] = (lds_u32)(win + (dlo + d) * kDigitWords + copy_base(sh) + ((lb + 3) >> 2));
    asm volatile("" : "+v"(ep[d]));
  }
  // weight fragment of this lane in buffer b: row c, bytes 16 g + 32 st
  const uint32_t* wl0 = reinterpret_cast<const uint32_t*>(smem + kWinLds) + c * kWRowWords + 4 * g;
  const uint32_t* wl = wl0;
  v4i fprev[DPW];
  // Operands of one k-step: the weight fragment and a new Toeplitz fragment per digit.
  struct Frags {
    v4i w, a[DPW];
  };
  auto load = [&](uint32_t st) __attribute__((always_inline)) {
    Frags f;
    f.w = toeplitz_frag(wl + 8 * st);
#pragma unroll
    for (int d = 0; d < DPW; ++d)
      if (d < cnt) f.a[d] = toeplitz_frag(ep[d] + 8 * st);
    return f;
  };
  // One k-step: each new fragment feeds block 0 and, one step late, block 1.
  auto mma = [&](const Frags& f) __attribute__((always_inline)) {
#pragma unroll
    for (int d = 0; d < DPW; ++d) {
      if (d < cnt) {
        acc0[d] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.w, f.a[d], acc0[d], 0, 0, 0);
        acc1[d] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.w, fprev[d], acc1[d], 0, 0, 0);
        fprev[d] = f.a[d];
      }
    }
  };

  const uint32_t L = __builtin_amdgcn_readfirstlane(m.L);
  // Staging of chunk (i, kc): plane bytes [N + kc - n0 - 64, N + kc - n0 + kKC) hold
  // every Toeplitz entry of rows [kc, kc + kKC) and columns [n0, n0 + 64). A chunk
  // shorter than kKC reads window bytes past the plane from the workspace that
  // follows it; they are never used (its Toeplitz entries end at plane byte
  // N + kp - n0 - 1 < 2N).
  // Windows: loaded 16 plane bytes (+ the dword before them) per item into
  // registers, written as four copies. Weights: LDS DMA into one of two buffers.
  constexpr int kQuads = kCopyWords / 4;
  constexpr int kItems = DK * kQuads;
  constexpr int kWinRegs = (kItems + NT - 1) / NT;
  static_assert(kWinRegs == 1, "one window item per thread");
  struct WinRegs {
    uint4 q;
    uint32_t qp;
  };
  auto win_load = [&](uint32_t i, uint32_t kc, WinRegs& r) __attribute__((always_inline)) {
    const int8_t* planes = emask + (((size_t)t * D + l0) * L + i) * 2 * N + (N + kc - n0 - 64);
    const uint32_t x = threadIdx.x;
    if (x < (uint32_t)kItems) {
      const uint32_t d = x / kQuads, v = x % kQuads;
      const int8_t* src = planes + (size_t)d * L * 2 * N + 16 * v;
      r.q = *(const uint4*)src;
      // word -1 of the window only feeds word 0 of copies 1..3, which no fragment reads
      r.qp = *(const uint32_t*)(v ? src - 4 : src);
    }
  };
  auto win_store = [&](const WinRegs& r) __attribute__((always_inline)) {
    const uint32_t x = threadIdx.x;
    if (x < (uint32_t)kItems) {
      const uint32_t d = x / kQuads, v = x % kQuads;
      const uint4 q = r.q;
      uint32_t* wd = win + d * kDigitWords + 4 * v;
      *(uint4*)(wd + copy_base(0)) = q;
#pragma unroll
      for (int sft = 1; sft < 4; ++sft)
        *(uint4*)(wd + copy_base(sft)) = make_uint4(__builtin_amdgcn_alignbyte(q.x, r.qp, sft),
                                                    __builtin_amdgcn_alignbyte(q.y, q.x, sft),
                                                    __builtin_amdgcn_alignbyte(q.z, q.y, sft),
                                                    __builtin_amdgcn_alignbyte(q.w, q.z, sft));
    }
  };
  const uint32_t wave_lds = __builtin_amdgcn_readfirstlane(wave * 64 * 16);
  auto w_dma = [&](int b, uint32_t i, uint32_t kc) __attribute__((always_inline)) {
    const int8_t* wsrc = m.w + (size_t)jb * m.kw + (size_t)i * N + kc;
    const uint32_t wlim = m.kw - i * N - kc;  // row bytes left from kc
    const uint32_t base = lds_addr(smem + kWinLds + b * kWBuf);
#pragma unroll
    for (int it = 0; it < kWIters; ++it) {
      const uint32_t x = it * NT + threadIdx.x;   // slot: row x / 17, position x % 17
      const uint32_t r = x / 17, pos = x % 17;
      const bool data = r < 32 && pos < 16 && 16 * pos < wlim;
      const int8_t* src = wsrc + (r < 32 ? r * m.kw : 0) + (data ? 16 * pos : 0);
      lds_dma16(src, __builtin_amdgcn_readfirstlane(base + it * NT * 16) + wave_lds);
    }
  };
  auto compute = [&](int b, uint32_t klen) __attribute__((always_inline)) {
    wl = wl0 + b * (kWBuf / 4);
#pragma unroll
    for (int d = 0; d < DPW; ++d)
      if (d < cnt) fprev[d] = toeplitz_frag(ep[d] - 8);
    if constexpr (FULL) {
      // full chunk: straight-line code with immediate LDS offsets; the operands of
      // step st + 1 are requested before the matrix instructions of step st
      Frags cur = load(0);
#pragma unroll
      for (int st = 0; st < kKC / 32; ++st) {
        Frags nxt;
        if (st + 1 < kKC / 32) nxt = load(st + 1);
        mma(cur);
        cur = nxt;
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
      for (uint32_t st = 0; st < klen / 32; st += 2) {  // klen is a multiple of 64
        const Frags f0 = load(st), f1 = load(st + 1);
        mma(f0);
        mma(f1);
      }
    }
  };

  // Chunks in order (block i, offset kc). The next chunk's window loads and weight
  // DMA are issued before the matrix-core work on the current one.
  WinRegs wr;
  win_load(0, 0, wr);
  w_dma(0, 0, 0);
  win_store(wr);
  wait_vmem();
  __syncthreads();
  uint32_t ci = 0, ckc = 0;
  int buf = 0;
  for (;;) {
    const uint32_t kb = __builtin_amdgcn_readfirstlane(min(N, m.k - ci * N));
    const uint32_t kp = (kb + 63u) & ~63u;  // the weight rows are zero up to a multiple of 64
    const uint32_t klen = min((uint32_t)kKC, kp - ckc);
    uint32_t ni = ci, nkc = ckc + kKC;
    if (nkc >= kp) {
      ++ni;
      nkc = 0;
    }
    const bool more = ni < L;
    if (more) {
      win_load(ni, nkc, wr);
      w_dma(buf ^ 1, ni, nkc);
    }
    __builtin_amdgcn_sched_barrier(0);
    compute(buf, klen);
    if (!more) break;
    __syncthreads();  // the windows of this chunk are no longer read
    win_store(wr);
    wait_vmem();      // the weight DMA of the next chunk landed
    __syncthreads();
    ci = ni;
    ckc = nkc;
    buf ^= 1;
  }

  // accumulator element e of this lane: row jb + 8(e/4) + 4g + e%4, column n0 + 32b + c.
  // The partials of the waves meet in LDS in two rounds (one per column block), and
  // every wave finishes a share of the elements.
  if constexpr (RAW) {
    // each wave folds its digits into int64 partials, V = sum_l 255^l S_l is then
    // rebuilt exactly (128-bit) and reduced mod every prime
    int64_t P0[16], P1[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      P0[e] = 0;
      P1[e] = 0;
#pragma unroll
      for (int d = DPW - 1; d >= 0; --d) {
        if (d < cnt) {
          P0[e] = P0[e] * 255 + acc0[d][e];
          P1[e] = P1[e] * 255 + acc1[d][e];
        }
      }
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      __syncthreads();  // LDS windows (or the previous round's partials) are no longer read
#pragma unroll
      for (int e = 0; e < 16; ++e) part[(role * 16 + e) * 64 + lane] = b == 0 ? P0[e] : P1[e];
      __syncthreads();
      const uint32_t n = n0 + 32 * b + c;
      for (int e = wave; e < 16; e += NW) {
        const uint32_t j = jb + 8 * (e >> 2) + 4 * g + (e & 3);
        // U = sum over roles of 255^dlo_r P_r, Horner from the highest role
        i128 U = 0;
#pragma unroll
        for (int r = NW - 1; r >= 0; --r) {
          const int cr = DK / NW + (r < DK % NW ? 1 : 0);
          i128 scale = 1;
          for (int x = 0; x < cr; ++x) scale *= 255;
          U = U * scale + part[(r * 16 + e) * 64 + lane];
        }
        if (j < m.rows) {
          const size_t row = (size_t)t * m.rows + j;
          uint64_t* o = (uint64_t*)out;
          for (uint32_t p = 0; p < rc.P; ++p) o[(row * rc.P + p) * (N + 1) + n] = mod_i128(U, rc.q[p]);
        }
      }
    }
  } else {
    // Switched output: c 2^32 / q mod 2^32 = sum_l S_l 255^l 2^32 / q mod 2^32. Each
    // wave adds, for its digits l = l0 + dlo + d, S_l G_l (G_l = round(255^l 2^96 / q)
    // in the balanced words a, b, c of RingConst::dg) in 32.32 fixed point mod 2^64:
    // floor(S a / 2^32) + S b + (S c mod 2^32) 2^32, exact but for the floor (at most one
    // unit low per digit) and the rounding of G_l; the waves' words then simply add.
    // The digits below l0 are left out; sc.epsw bounds all of it.
    int32_t ga[DPW], gb[DPW];
    uint32_t gc[DPW];
#pragma unroll
    for (int d = 0; d < DPW; ++d) {
      const int l = (int)l0 + dlo + (d < cnt ? d : 0);
      ga[d] = bt->rc.dg[l][0];
      gb[d] = bt->rc.dg[l][1];
      gc[d] = (uint32_t)bt->rc.dg[l][2];
    }
    uint64_t W0[16], W1[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      uint32_t H0 = 0, H1 = 0;
      int64_t w0 = 0, w1 = 0;  // sums mod 2^64 (each term below 2^62 in magnitude)
#pragma unroll
      for (int d = 0; d < DPW; ++d) {
        if (d < cnt) {
          const int32_t s0 = acc0[d][e], s1 = acc1[d][e];
          w0 += (int64_t)s0 * gb[d] + __mulhi(s0, ga[d]);
          w1 += (int64_t)s1 * gb[d] + __mulhi(s1, ga[d]);
          H0 += (uint32_t)s0 * gc[d];
          H1 += (uint32_t)s1 * gc[d];
        }
      }
      W0[e] = (uint64_t)w0 + ((uint64_t)H0 << 32);
      W1[e] = (uint64_t)w1 + ((uint64_t)H1 << 32);
    }
    uint64_t* partw = reinterpret_cast<uint64_t*>(smem);
    const uint32_t k = rc.qbits, sh = 64 - k;
    const uint64_t half = 1ull << (sh - 1), E = sc.epsw;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      __syncthreads();  // LDS windows (or the previous round's partials) are no longer read
#pragma unroll
      for (int e = 0; e < 16; ++e) partw[(role * 16 + e) * 64 + lane] = b == 0 ? W0[e] : W1[e];
      __syncthreads();
      const uint32_t n = n0 + 32 * b + c;
      for (int e = wave; e < 16; e += NW) {
        const uint32_t j = jb + 8 * (e >> 2) + 4 * g + (e & 3);
        uint64_t Wt = 0;
#pragma unroll
        for (int r = 0; r < NW; ++r) Wt += partw[(r * 16 + e) * 64 + lane];
        // round(Wt / 2^sh) mod 2^k, ties up; uncertain when the fraction lies within E
        // units of one half: then V = Wt + half is within E of a multiple of 2^sh
        const uint64_t V = Wt + half;
        uint32_t res = (uint32_t)(V >> sh);
        const bool amb = ((V + E) << k) < ((2 * E) << k);
        const bool live = j < m.rows;
        uint64_t pending = __ballot(live && (amb || force_exact));
        while (pending) {
          const int src = __ffsll((unsigned long long)pending) - 1;
          pending &= pending - 1;
          const uint32_t jj = __shfl(j, src), nn = __shfl(n, src);
          const uint32_t r = exact_element_wave<D>(bt, ii, t, jj, nn, lane);
          if (lane == src) res = r;
        }
        if (live) ((uint32_t*)out)[((size_t)t * m.rows + j) * (N + 1) + n] = res;
      }
    }
  }
}

template <int D, int DK, bool RAW>
static void launch_one(const Batch& b, hipStream_t s) {
  bool full = b.rc.N >= (uint32_t)kKC;
  for (uint32_t x = 0; x < b.n; ++x) full = full && b.it[x].m.k % kKC == 0;
  if (full)
    hipLaunchKernelGGL((mask_kernel<D, DK, RAW, true>), grid_for(b.mask_start[b.n]),
                       dim3(64 * ((DK + 2) / 3)), 0, s, b);
  else
    hipLaunchKernelGGL((mask_kernel<D, DK, RAW, false>), grid_for(b.mask_start[b.n]),
                       dim3(64 * ((DK + 2) / 3)), 0, s, b);
}

hipError_t launch_mask(const Batch& b, uint32_t dk, hipStream_t s) {
  if (b.n == 0 || b.mask_start[b.n] == 0) return hipSuccess;
  if (b.rc.D == 7) {
    if (b.raw)
      launch_one<7, 7, true>(b, s);
    else if (dk == 7)
      launch_one<7, 7, false>(b, s);
    else
      return hipErrorInvalidValue;
  } else {
    if (b.raw) {
      launch_one<14, 14, true>(b, s);
    } else {
      switch (dk) {
        case 8: launch_one<14, 8, false>(b, s); break;
        case 9: launch_one<14, 9, false>(b, s); break;
        case 10: launch_one<14, 10, false>(b, s); break;
        case 11: launch_one<14, 11, false>(b, s); break;
        case 12: launch_one<14, 12, false>(b, s); break;
        case 14: launch_one<14, 14, false>(b, s); break;
        default: return hipErrorInvalidValue;
      }
    }
  }
  return hipGetLastError();
}

}  // namespace rlwe
