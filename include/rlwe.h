/*
 * rlwe.h — C ABI of the MI355X (gfx950) library for the server side of private
 * LoRA fine-tuning under homomorphic encryption: the product of a clear int8
 * weight matrix with RLWE-encrypted int8 vectors, W.[x]_HE (and W^T.[g]_HE for
 * the backward pass through the frozen base), ending in a modulus switch.
 *
 * Paper: Frery, Bredehoft, Klemsa, Meyre, Stoian, "Private LoRA Fine-tuning of
 * Open-Source LLMs with Homomorphic Encryption" (arXiv 2505.07329).
 *   Sec. 3.1  RLWE ciphertext (A, B), B = A*S + E + Delta*M in Z_q[X]/(X^N+1);
 *             LWE ciphertext (a, b), b = <a, s> + e + Delta*m.
 *   Sec. 3.2  SampleExtract, ModulusSwitch, product with a clear polynomial.
 *   Sec. 4.2  symmetric int8 quantization: the server computes only sum x_q w_q.
 *   Sec. 4.3  x split into L = ceil(d_in/N) blocks, weights encoded in reverse,
 *             Eq. (LWEdot): LWE(x.w_j) = sum_i SampleExtract(RLWE(x_i).w_ij, N-1),
 *             then ModulusSwitch of the output.
 *
 * Everything here is exact integer arithmetic. Results are unique functions of
 * the inputs: the same call gives the same bits on every run and every tiling.
 *
 * Conventions
 *   - Pointers documented "device" are HIP device pointers (e.g. torch tensors
 *     on the GPU); "host" pointers are CPU memory. The caller owns every buffer
 *     it passes in; the library owns the context and weight handles.
 *   - rlwe_stream_t is a hipStream_t (0 = the null stream). Compute calls only
 *     enqueue work on it and return; errors of a kernel surface at the next
 *     synchronisation.
 *   - Residues crossing the ABI are canonical, in [0, q_p).
 *   - Return value: RLWE_OK (0) or a negative RLWE_E* code; rlwe_last_error()
 *     then describes the failure (thread-local, valid until the next call on the
 *     same thread). No C++ exception crosses the ABI.
 *   - A context and its workspace are not thread-safe: calls that use one
 *     context must be issued from one thread at a time, and compute calls on a
 *     context must be ordered on one stream (they share the workspace).
 */
#ifndef RLWE_H
#define RLWE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RLWE_OK 0
#define RLWE_EINVAL (-1)    /* null pointer, unknown flag, bad argument */
#define RLWE_EPARAM (-2)    /* invalid cryptosystem parameters */
#define RLWE_ESHAPE (-3)    /* shapes outside what the exact kernels support */
#define RLWE_EOVERFLOW (-4) /* the integer product could wrap modulo t */
#define RLWE_ENOMEM (-5)    /* device allocation failed */
#define RLWE_EHIP (-6)      /* a HIP runtime call failed */

typedef void* rlwe_stream_t; /* a hipStream_t */

typedef struct rlwe_ctx rlwe_ctx;
typedef struct rlwe_weights rlwe_weights;

/* Cryptosystem parameters (Sec. 3.1, Sec. 4.4).
 *   N           ring degree, a power of two in [64, 32768]
 *   num_primes  P, 1 or 2: q = q_1 ... q_P in RNS form
 *   primes      host pointer to P distinct primes, each < 2^54 and q_p = 1 mod 2N
 *   log2_t      plaintext modulus t = 2^log2_t, 1 <= log2_t <= 32; Delta = floor(q/t)
 *   log2_q_out  switched outputs are modulo q_out = 2^log2_q_out, 1..32 (the paper
 *               uses 26 bits, Sec. 4.4); values are returned in uint32 words */
typedef struct rlwe_params {
  uint32_t N;
  uint32_t num_primes;
  const uint64_t* primes;
  uint32_t log2_t;
  uint32_t log2_q_out;
} rlwe_params;

/* Validate the parameters, select device `hip_device` and build the context
 * (CRT and switching constants). Errors: RLWE_EINVAL (null), RLWE_EPARAM, RLWE_EHIP. */
int rlwe_params_init(const rlwe_params* params, int hip_device, rlwe_ctx** out);

/* Release the context and its workspace (after all its work has completed).
 * Weight handles created from it must be freed first. NULL is accepted. */
int rlwe_params_destroy(rlwe_ctx* ctx);

/* Flags of rlwe_weights_load */
#define RLWE_W_FWD 1u       /* keep W for products W.[x] */
#define RLWE_W_TRANSPOSE 2u /* keep W^T for products W^T.[g] (backward pass) */
#define RLWE_W_NTT 4u       /* mask product by number-theoretic transforms (N = 2048, 4096) */
#define RLWE_W_TOEPLITZ 8u  /* mask product on the int8 matrix cores (digit planes) */
#define RLWE_W_ROWPACK 16u  /* several rows per weight polynomial where K <= N/2 (NTT) */

/* Mask-product methods (rlwe_weights_method). Both give the same bits. */
#define RLWE_METHOD_TOEPLITZ 0u
#define RLWE_METHOD_NTT 1u

/* Make the clear weights resident on the device (Sec. 4.3: block i of row j is
 * used in the reversed encoding w_hat_ij[k] = w_j[iN + N - 1 - k]).
 *   W_dev   device pointer, int8 row-major [d_out][d_in], values in [-127, 127]
 *           (symmetric quantization, Sec. 4.2); read during the call only
 *   flags   RLWE_W_FWD and/or RLWE_W_TRANSPOSE, plus at most one method flag:
 *           RLWE_W_NTT keeps the reversed blocks in the NTT domain per prime
 *           (rows * L * P * N * 8 bytes; RLWE_EPARAM unless N = 2048 or 4096),
 *           RLWE_W_TOEPLITZ keeps int8 only; without one, each orientation
 *           (N = 2048, 4096) takes the method a tuner attached to the context measured
 *           fastest for its shape (rlwe_ctx_set_tuner), else the one with the
 *           smaller estimated time per output: matrix cores 8 + 0.0033 K dk ns (K
 *           the contraction length, dk the digit planes kept, rlwe_weights_digits),
 *           transforms (5 + 12.35 L) P ns (L = ceil(K / N) blocks, P primes),
 *           both scaled by N / 4096, fitted to MI355X timings; at other N the
 *           matrix-core method.
 *           RLWE_W_ROWPACK (N = 2048, 4096; not with RLWE_W_TOEPLITZ): an orientation
 *           whose contraction length K is at most N/2 packs n_o = floor(N / K)
 *           rows into each weight polynomial, row g n_o + rho reversed in
 *           coefficients [rho K, rho K + K) (the coefficient packing of Sec.
 *           4.3.1, as in Cheetah), with the NTT method: one polynomial product
 *           per n_o outputs. Other orientations load as without the flag. The
 *           outputs decrypt to the same values; their ciphertexts differ (see
 *           ct_matmul_clear). NTT memory: ceil(rows / n_o) * P * N * 8 bytes
 * Validation: 1 <= d_out, d_in <= 65536; the exact 128-bit accumulation needs
 * 127 * d * q / 2 < 2^127 for the contraction length d (d_in forward, d_out
 * transposed; n_o d when rows are packed) -> RLWE_ESHAPE. Overflow: returns RLWE_EOVERFLOW if 127 times the
 * largest row 1-norm (column 1-norm for W^T) reaches t/2, since W.x could then
 * wrap modulo t (Sec. 4.4). Synchronises `stream` (set-up call). */
int rlwe_weights_load(rlwe_ctx* ctx, const int8_t* W_dev, uint32_t d_out, uint32_t d_in,
                      uint32_t flags, rlwe_stream_t stream, rlwe_weights** out);

/* Release a weight handle (after all work that uses it has completed). NULL ok. */
int rlwe_weights_free(rlwe_weights* w);

/* Flags of ct_matmul_clear */
#define RLWE_OUT_SWITCHED 0u    /* outputs switched to q_out = 2^log2_q_out (uint32) */
#define RLWE_OUT_RAW_Q 1u       /* outputs modulo q, per prime (uint64) */
#define RLWE_OUT_FORCE_EXACT 2u /* switched outputs through the slow exact path
                                   for every coefficient (same bits; test hook) */
#define RLWE_IN_SEEDED 4u       /* inputs in the seeded layout (masks expanded on the GPU) */
/* Launch shape (same bits either way). By default a call or batch whose products all
 * use the NTT method runs as one persistent launch: a grid of at most two workgroups
 * per compute unit takes the steps of every product (mask transforms and body digit
 * planes per token and block, product tiles, bodies) from one work queue, each
 * product's tiles waiting on its own transforms; otherwise grouped launches (one per
 * step and kernel class) run. */
#define RLWE_LAUNCH_PERSISTENT 8u /* require the persistent launch (RLWE_EINVAL if a
                                     product uses the matrix cores, or N != 4096) */
#define RLWE_LAUNCH_GROUPED 16u   /* grouped launches even where all products use NTT */

/* The encrypted clear-weight product of Eq. (LWEdot) for `tokens` inputs.
 * With transpose = 0 it computes W.[x] (d_in -> d_out); with transpose = 1,
 * W^T.[g] (d_out -> d_in), which needs RLWE_W_TRANSPOSE at load time. Below,
 * K is the input length (d_in, or d_out when transposed), M the output count,
 * L = ceil(K / N).
 *   ct_in  device, uint64 [tokens][L][2][P][N]: for token t and block i,
 *          ct_in[t][i][0] = A and ct_in[t][i][1] = B of RLWE(x_hat_i), each
 *          per prime p in canonical residues; x_hat_i holds inputs iN .. iN+N-1
 *          (zero past K). With RLWE_IN_SEEDED, uint64 [tokens][L][P*N + 2]:
 *          [seed, 0, B residues [P][N]] per block (Sec. 3.1: the client sends a
 *          seed for the uniform mask; Sec. 4.4), about half the bytes; the GPU
 *          expands A[p][n] as the top 54 bits of the first of the SplitMix64
 *          outputs (p N + n) 16 + j, j < 16, under the seed that lies below q_p
 *          (the first output mod q_p if none does). SplitMix64 output c under
 *          seed s: z = s + (c + 1) 0x9E3779B97F4A7C15, z = (z ^ z >> 30)
 *          0xBF58476D1CE4E5B9, z = (z ^ z >> 27) 0x94D049BB133111EB, z ^ z >> 31.
 *   out    device; one LWE ciphertext per (token, output) under the key
 *          (S_0 .. S_{N-1}): mask a_0 .. a_{N-1} then body b, with
 *          a_n = sum_k w[k] * (A_i[k-n] if k >= n else -A_i[N+k-n]) summed over
 *          blocks (SampleExtract at N-1 of the block products), b = sum_k w[k] B_i[k]
 *            RLWE_OUT_SWITCHED: uint32 [tokens][M][N+1], each coefficient c
 *              replaced by round(c * 2^k / q) mod 2^k, k = log2_q_out
 *              (ModulusSwitch, Sec. 3.2)
 *            RLWE_OUT_RAW_Q:    uint64 [tokens][M][P][N+1], residues mod q_p
 *          With packed rows (RLWE_W_ROWPACK, n_o > 1; one block), output j = g n_o
 *          + rho is SampleExtract at h = (rho + 1) K - 1 of w_hat_g.(A, B), w_hat_g
 *          the polynomial of rows g n_o .. g n_o + n_o - 1: with c = w_hat_g A
 *          mod X^N + 1, a_n = c[h-n] for n <= h and -c[N+h-n] for n > h;
 *          b = sum_r sum_k w_{g n_o + r}[k] * B~[(rho - r) K + k], B~[-i] = -B[N-i]
 *          (the standard outputs are the case h = N - 1 of the same rule)
 * tokens = 0 is a no-op. Uses the context workspace (grown on demand with
 * hipMalloc unless rlwe_workspace_reserve made it large enough). Asynchronous
 * on `stream`. */
int ct_matmul_clear(rlwe_ctx* ctx, const rlwe_weights* w, uint32_t transpose,
                    const uint64_t* ct_in, uint32_t tokens, void* out, uint32_t flags,
                    rlwe_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): ct_matmul_clear with the
 * same arguments, flags and results, bit for bit, whose workspace is a fixed device
 * array of RLWE_NOALLOC_SCRATCH_BYTES in the library instead of the context
 * workspace. The array exists once per GPU, is held until the process ends and keeps
 * the last call's contents; calls never allocate or free memory and record no
 * profiling events. Calls that overlap on one GPU (any context, any stream) race on
 * the array: order them on one stream. RLWE_ESHAPE if the call needs more workspace
 * than the array holds (rlwe_workspace_bytes: e.g. at most 356 tokens of a 2048-input
 * product at N = 4096 with two primes on the NTT method); other errors as for
 * ct_matmul_clear. */
#define RLWE_NOALLOC_SCRATCH_BYTES (64u << 20)
int ct_matmul_clear_noalloc(rlwe_ctx* ctx, const rlwe_weights* w, uint32_t transpose,
                            const uint64_t* ct_in, uint32_t tokens, void* out, uint32_t flags,
                            rlwe_stream_t stream);

/* One product of a batch: W.[x] (transpose = 0) or W^T.[g] (transpose = 1) for
 * `tokens` inputs; ct_in and out are device buffers laid out as for
 * ct_matmul_clear. */
typedef struct ct_matmul_desc {
  const rlwe_weights* w;
  uint32_t transpose;
  const uint64_t* ct_in;
  uint32_t tokens;
  void* out;
} ct_matmul_desc;

/* Several products of Eq. (LWEdot) with different weights and token counts
 * (e.g. all projections of a transformer layer, forward and transposed) in
 * grouped launches: one preparation launch, one matrix-core launch per number of
 * kept digits, one body launch, for every 16 descriptors. `descs` is a host
 * array of n descriptors; flags as for ct_matmul_clear and applied to all. The
 * products with the longest contraction are scheduled first. Results are the
 * same bits as n separate ct_matmul_clear calls. Asynchronous; allocates only if
 * the context workspace is smaller than rlwe_batch_workspace_bytes (refused with
 * RLWE_EINVAL while the stream is being captured). */
int ct_matmul_batch(rlwe_ctx* ctx, const ct_matmul_desc* descs, uint32_t n, uint32_t flags,
                    rlwe_stream_t stream);

/* Workspace bytes ct_matmul_batch needs for these descriptors (0 on bad input). */
size_t rlwe_batch_workspace_bytes(const rlwe_ctx* ctx, const ct_matmul_desc* descs, uint32_t n);

/* A batch captured once into a HIP graph with its own workspace, for replay:
 * rlwe_graph_capture_batch records ct_matmul_batch(descs) (the descriptors'
 * buffers are baked into the graph and must stay valid); rlwe_graph_launch
 * replays it on `stream`; rlwe_graph_destroy frees it (after its work is done). */
typedef struct rlwe_graph rlwe_graph;
int rlwe_graph_capture_batch(rlwe_ctx* ctx, const ct_matmul_desc* descs, uint32_t n,
                             uint32_t flags, rlwe_graph** out);
int rlwe_graph_launch(rlwe_graph* g, rlwe_stream_t stream);
int rlwe_graph_destroy(rlwe_graph* g);

/* ModulusSwitch q -> 2^k, k = log2_q_out (Sec. 3.2), of `count` vectors of N+1
 * coefficients:
 *   in   device, uint64 [count][P][N+1] canonical residues
 *   out  device, uint32 [count][N+1], round(c * 2^k / q) mod 2^k with
 *        c = CRT(residues) in [0, q) (a tie cannot occur: q is odd)
 * count = 0 is a no-op. Asynchronous on `stream`; no workspace. */
int ct_modswitch(rlwe_ctx* ctx, const uint64_t* in, size_t count, uint32_t* out,
                 rlwe_stream_t stream);

/* Bit-packing of switched ciphertexts (Sec. 4.5: the switched output is packed
 * into a bit-vector before it is returned; sizes as in Sec. 4.4):
 *   in    device, uint32 [count][len], coefficients below 2^k (k = log2_q_out;
 *         higher bits are ignored), e.g. the switched outputs (len = N + 1)
 *   out   device, uint32 [count][rlwe_packed_words(len, k)]: coefficient i of a
 *         ciphertext occupies stream bits [i k, (i + 1) k), least significant
 *         first; stream bit b is bit b mod 32 of word b / 32; unused high bits of
 *         the last word are zero. Caller-owned; must not overlap `in`.
 * count = 0 or len = 0 is a no-op; RLWE_ESHAPE if count * words exceeds 2^39.
 * Asynchronous on `stream`; no workspace. HBM-bound (4 len bytes read, 4 words
 * written per ciphertext). */
int ct_pack_bits(rlwe_ctx* ctx, const uint32_t* in, size_t count, uint32_t len, uint32_t* out,
                 rlwe_stream_t stream);

/* 32-bit words of one ciphertext of `len` coefficients packed at `bits` bits:
 * ceil(len * bits / 32); 0 unless 1 <= bits <= 32. */
size_t rlwe_packed_words(uint32_t len, uint32_t bits);

/* Bytes of workspace ct_matmul_clear needs for this call shape. */
size_t rlwe_workspace_bytes(const rlwe_ctx* ctx, const rlwe_weights* w, uint32_t transpose,
                            uint32_t tokens);

/* Grow the context workspace to at least `bytes` now (hipMalloc), so that later
 * calls within that size allocate nothing. */
int rlwe_workspace_reserve(rlwe_ctx* ctx, size_t bytes);

/* Per-kernel device timing (HIP events recorded on the launch stream around
 * every kernel the library enqueues while profiling is on), for roofline
 * accounting. rlwe_profile_begin starts a recording window (at most 4096
 * launches are recorded, later ones are counted in `dropped`);
 * rlwe_profile_end waits for the recorded events, fills `out` (host pointer)
 * and closes the window. Not for use inside hipGraph capture. */
typedef struct rlwe_kernel_times {
  /* summed durations: digit preparation and mask transforms (prep), matrix-core
   * mask products (mask), NTT mask products (ntt), body, standalone switch,
   * bit-packing (pack), KeySwitch packing: gadget digits (ksdig), transforms and
   * key products (ksacc), inverse transforms and outputs (ksfin) */
  double prep_ms, mask_ms, body_ms, modswitch_ms, ntt_ms, pack_ms;
  uint32_t prep_n, mask_n, body_n, modswitch_n, ntt_n, pack_n; /* launches recorded */
  uint32_t dropped;
  double ksdig_ms, ksacc_ms, ksfin_ms;
  uint32_t ksdig_n, ksacc_n, ksfin_n;
  double persist_ms; /* persistent batch launches (all steps of their products) */
  uint32_t persist_n;
} rlwe_kernel_times;

int rlwe_profile_begin(rlwe_ctx* ctx);
int rlwe_profile_end(rlwe_ctx* ctx, rlwe_kernel_times* out);

/* Digits of the balanced base-255 expansion of ciphertext coefficients that
 * the switched product feeds to the int8 matrix cores (`kept`) out of `total`
 * (7 for one prime, 14 for two). Host pointers; for work accounting. */
int rlwe_weights_digits(const rlwe_weights* w, uint32_t transpose, uint32_t* kept,
                        uint32_t* total);

/* Mask-product method of one loaded orientation: *method = RLWE_METHOD_TOEPLITZ
 * or RLWE_METHOD_NTT (host pointer). RLWE_EINVAL for null arguments or an
 * orientation that was not loaded. */
int rlwe_weights_method(const rlwe_weights* w, uint32_t transpose, uint32_t* method);

/* Outputs per weight polynomial of one loaded orientation (host pointer): n_o =
 * floor(N / K) when it was loaded with RLWE_W_ROWPACK and K <= N/2, else 1.
 * RLWE_EINVAL for null arguments or an orientation that was not loaded. */
int rlwe_weights_rows_per_product(const rlwe_weights* w, uint32_t transpose, uint32_t* n_o);

/* KeySwitch packing (Sec. 3.2 KeySwitching and Rotate; Sec. 4.3 Eq. (pack_rotate)):
 * the LWE outputs of ct_matmul_clear are key-switched to RLWE ciphertexts and
 * rotated into the slots of packed RLWE ciphertexts, which are then switched to
 * q_out; N <= 4096 (tuned kernels at N = 4096, plain ones below).
 *
 * Decomp (the gadget decomposition of TFHE, to which Sec. 3.2 refers): a mask
 * coefficient c in [0, q) is rounded to K = log2_base * levels bits, a~ =
 * round(c 2^K / q) mod 2^K, and a~ = sum_m d_m 2^(log2_base (levels - 1 - m))
 * mod 2^K with signed digits d_m in [-2^(log2_base-1), 2^(log2_base-1)), d_0 the
 * most significant; the gadget values are g_m = round(q / 2^(log2_base (m+1))).
 * The key-switching key (a client-side secret product: it is built with both
 * secret keys) is KSK_{i,m} = RLWE_{S'}(s_i g_m) for i < N, m < levels, the
 * message in the constant coefficient, s the LWE key of the outputs (the
 * coefficients of the input key S) and S' the key of the packed outputs.
 *
 * rlwe_ksk_load: make the key resident in the NTT domain (N levels P 2 N 16 bytes:
 * residues and their Shoup companions).
 *   ksk_dev    device, uint64 [N][levels][2][P][N] canonical residues: A, then B of
 *              KSK_{i,m}; read during the call only
 *   log2_base  digit bits, 1 <= log2_base <= 54, 2^(log2_base-1) below every prime
 *   levels     1 <= levels <= 4, log2_base * levels <= 64 (e.g. 54 and 1 for two
 *              54-bit primes; 12 and 3 for one)
 * Errors: RLWE_EINVAL (null), RLWE_EPARAM (N > 4096, bad gadget), RLWE_ENOMEM.
 * Synchronises `stream` (set-up call). */
typedef struct rlwe_ksk rlwe_ksk;
int rlwe_ksk_load(rlwe_ctx* ctx, const uint64_t* ksk_dev, uint32_t log2_base, uint32_t levels,
                  rlwe_stream_t stream, rlwe_ksk** out);

/* Release a key (after all work that uses it has completed). NULL ok. */
int rlwe_ksk_free(rlwe_ksk* k);

/* Packed ciphertexts for `count` LWE ciphertexts at n_pack slots each:
 * ceil(count / n_pack) (0 if n_pack = 0). */
size_t rlwe_packed_count(size_t count, uint32_t n_pack);

/* Workspace bytes of ct_keyswitch_pack for this shape (0 on bad input); calls
 * within rlwe_workspace_reserve(that many) allocate nothing. */
size_t rlwe_keyswitch_workspace_bytes(const rlwe_ctx* ctx, const rlwe_ksk* k, size_t count,
                                      uint32_t n_pack);

/* Eq. (pack_rotate): packed output g = sum over slots s < n_pack of
 * Rotate(KeySwitching(LWE_{g n_pack + s}), s) (while g n_pack + s < count), with
 * KeySwitching(a, b) = (0, b) - sum_i sum_m Decomp_m(a_i) KSK_{i,m} and Rotate by
 * s the product with X^s in Z_q[X]/(X^N + 1); then, unless RLWE_OUT_RAW_Q, the
 * ModulusSwitch of every coefficient to q_out = 2^log2_q_out. Coefficient s of
 * output g decrypts under S' to the message of LWE g n_pack + s (e.g. n_pack =
 * d_out packs one token's outputs of W.[x] per ciphertext when d_out <= N;
 * n_pack = N fills every slot).
 *   lwe_in  device, uint64 [count][P][N+1]: LWE ciphertexts modulo q (mask, then
 *           body), e.g. the RLWE_OUT_RAW_Q output of ct_matmul_clear
 *   out     device: RLWE_OUT_SWITCHED uint32 [G][2][N] (A, then B, switched);
 *           RLWE_OUT_RAW_Q uint64 [G][2][P][N] residues; G = rlwe_packed_count
 * count = 0 is a no-op; RLWE_ESHAPE unless 1 <= n_pack <= N. Uses the context
 * workspace (grown with hipMalloc unless reserved; refused while the stream is
 * captured). Asynchronous on `stream`. */
int ct_keyswitch_pack(rlwe_ctx* ctx, const rlwe_ksk* k, const uint64_t* lwe_in, size_t count,
                      uint32_t n_pack, void* out, uint32_t flags, rlwe_stream_t stream);

/* Workspace bytes of ct_matmul_pack for this shape (0 on bad input); calls within
 * rlwe_workspace_reserve(that many) allocate nothing. */
size_t rlwe_matmul_pack_workspace_bytes(const rlwe_ctx* ctx, const rlwe_weights* w,
                                        uint32_t transpose, uint32_t tokens, const rlwe_ksk* k,
                                        uint32_t n_pack);

/* The product of ct_matmul_clear followed by ct_keyswitch_pack of its LWE outputs
 * (Eq. (LWEdot), then Eq. (pack_rotate)): output g packs the LWE outputs g n_pack +
 * s, s < n_pack, in the order (token, row) of ct_matmul_clear. The result is the
 * same, bit for bit, as the two calls. With the NTT method the product kernel
 * rounds every mask coefficient to 2^K for Decomp itself (K = log2_base * levels of
 * the key), so that only a~ (8 bytes) instead of P residues passes between the two
 * steps; with the matrix-core method the raw residues do.
 *   ct_in, tokens, transpose, w   as for ct_matmul_clear (flag RLWE_IN_SEEDED)
 *   k, n_pack, out                as for ct_keyswitch_pack (flag RLWE_OUT_RAW_Q);
 *                                 count = tokens * (rows of the product)
 *   RLWE_OUT_FORCE_EXACT          every rounding through the slow exact path (same
 *                                 bits; test hook)
 * tokens = 0 is a no-op. Errors as for the two calls. Uses the context workspace
 * (rlwe_matmul_pack_workspace_bytes: the product's, the LWE outputs between the
 * steps, M (N + P) 8 bytes with the NTT method, and ct_keyswitch_pack's; grown with
 * hipMalloc unless reserved; refused while the stream is captured). Asynchronous
 * on `stream`. */
int ct_matmul_pack(rlwe_ctx* ctx, const rlwe_weights* w, uint32_t transpose, const uint64_t* ct_in,
                   uint32_t tokens, const rlwe_ksk* k, uint32_t n_pack, void* out, uint32_t flags,
                   rlwe_stream_t stream);

/* ------------------------------------------------------------------ autotuning
 * The paper times its products per shape (Sec. 6.3, Table 4) and gives no tuning. These
 * calls choose, by timing on the device, among launch shapes of the same arithmetic;
 * no choice changes a result bit:
 *   method   RLWE_METHOD_NTT or RLWE_METHOD_TOEPLITZ, for an orientation loaded without
 *            a method flag (rlwe_weights_load);
 *   tt_log2  NTT method: 1 << tt_log2 tokens per workgroup (0..5);
 *   order    NTT method: 0 token tiles vary fastest in the block order, 1 rows do;
 *   launch   0 grouped launches, 1 one persistent launch (RLWE_LAUNCH_*).
 * A tuner holds measured choices keyed by N, P, the product's shape (K inputs, M outputs,
 * n_o rows per weight polynomial), raw or switched output and the token count rounded
 * up to a power of two, for one device. Attached to a context it is consulted by
 * rlwe_weights_load and by every product call and batch of the context: the entry of
 * the shape at the nearest token bucket; for a batch of several products, the batch
 * entry of that many products at the nearest bucket of their largest token count.
 * Without an entry: the cost model of rlwe_weights_load, 8 tokens per workgroup,
 * order 0, grouped launches. RLWE_LAUNCH_* flags of a call override the launch. */
typedef struct rlwe_schedule {
  uint32_t method, tt_log2, order, launch;
  float ms; /* measured time of the tuned call with this choice, milliseconds */
} rlwe_schedule;
typedef struct rlwe_tuner rlwe_tuner;

/* A tuner for the device named by device_key (host string, e.g. rlwe_device_key);
 * host memory only, no device needed. */
int rlwe_tuner_create(const char* device_key, rlwe_tuner** out);
int rlwe_tuner_destroy(rlwe_tuner* t);
size_t rlwe_tuner_size(const rlwe_tuner* t); /* number of entries */
/* Key of a product choice (rlwe_tuner_put/get) written to buf (host, len bytes). */
int rlwe_tune_key(uint32_t N, uint32_t P, uint32_t K, uint32_t M, uint32_t n_o, uint32_t raw,
                  uint32_t tokens, char* buf, size_t len);
/* Record / read the entry of a key; get returns RLWE_EINVAL if the key has none. */
int rlwe_tuner_put(rlwe_tuner* t, const char* key, const rlwe_schedule* s);
int rlwe_tuner_get(const rlwe_tuner* t, const char* key, rlwe_schedule* s);
/* The entry a product call uses (nearest token bucket of its shape): 1 and *s if there
 * is one, 0 if not, RLWE_EINVAL for null arguments. */
int rlwe_tuner_lookup(const rlwe_tuner* t, uint32_t N, uint32_t P, uint32_t K, uint32_t M,
                      uint32_t n_o, uint32_t raw, uint32_t tokens, rlwe_schedule* s);
/* JSON file at a host path. Load adds the entries recorded for this tuner's device
 * (*loaded = their number; NULL ok) and skips the entries of a file written for another
 * device; RLWE_EINVAL for an unreadable or malformed file (the tuner is then unchanged). */
int rlwe_tuner_save(const rlwe_tuner* t, const char* path);
int rlwe_tuner_load(rlwe_tuner* t, const char* path, size_t* loaded);
/* "<gcnArchName>|<name>|<compute units>" of HIP device hip_device into buf. */
int rlwe_device_key(int hip_device, char* buf, size_t len);
/* Attach a tuner to a context (NULL detaches); it must outlive the attachment and must
 * not change while calls of the context are being issued. */
int rlwe_ctx_set_tuner(rlwe_ctx* ctx, rlwe_tuner* t);

/* Times the candidates for one product shape on the context's device and records the
 * fastest in t (and *best, NULL ok):
 *   K, M     inputs and outputs of the product (one orientation, K -> M)
 *   wflags   0, or RLWE_W_ROWPACK (packed rows where K <= N/2; NTT method)
 *   tokens   token count of the calls tuned for, 1..65535
 *   oflags   RLWE_OUT_SWITCHED or RLWE_OUT_RAW_Q
 * Candidates: the matrix-core method (not with packed rows), and on the NTT method
 * (N = 2048, 4096) every tt_log2 with 1 << tt_log2 <= 16 and below 2 tokens, both
 * orders, and both launches at N = 4096. Uses random weights and inputs in its own
 * device memory (allocated and freed here) and the context workspace; synchronises
 * `stream`. */
int rlwe_autotune_product(rlwe_ctx* ctx, rlwe_tuner* t, uint32_t K, uint32_t M, uint32_t wflags,
                          uint32_t tokens, uint32_t oflags, rlwe_stream_t stream,
                          rlwe_schedule* best);
/* Times a batch (as for ct_matmul_batch, with flags RLWE_OUT_* / RLWE_IN_SEEDED; the
 * tuner's per-product choices apply) with grouped launches and, where every product uses
 * the NTT method, with the persistent launch, and records the faster launch for batches
 * of n products at the bucket of their largest token count. Runs the batch (its outputs
 * are written) a few times; synchronises `stream`. */
int rlwe_autotune_batch(rlwe_ctx* ctx, rlwe_tuner* t, const ct_matmul_desc* descs, uint32_t n,
                        uint32_t flags, rlwe_stream_t stream, rlwe_schedule* best);

/* Peak rates measured on a device by register-only microbenchmarks (independent
 * dependency chains, four waves per SIMD), the denominators of the roofline fractions:
 *   mul32_lane_ops  32-bit multiplies (v_mul_lo_u32) per second, per lane
 *   modmul          54-bit modular products per second (the product kernel's
 *                   truncated-quotient Shoup product, below 4p for any 64-bit input;
 *                   the faster of its two instruction forms)
 *   butterfly       lazy Gentleman-Sande butterflies per second (the product kernel's
 *                   inverse-transform butterfly: one Shoup product, a sum, a biased
 *                   difference; the faster of the product's two forms)
 *   mfma_int8_ops   int8 matrix-core operations per second (v_mfma_i32_32x32x32_i8,
 *                   two per multiply-add)
 *   clock_mhz, compute_units  as the device reports them (maximum clock)
 * Takes some milliseconds; allocates a scratch buffer; synchronises the device. */
typedef struct rlwe_peaks {
  double mul32_lane_ops, modmul, butterfly, mfma_int8_ops, clock_mhz;
  uint32_t compute_units;
} rlwe_peaks;
int rlwe_measure_peaks(int hip_device, rlwe_peaks* out);

/* Description of the last error on this thread ("" if none). */
const char* rlwe_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
