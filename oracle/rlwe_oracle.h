/*
 * Plain CPU oracle for the encrypted clear-weight product W.[x]_HE.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The product path (the
 * HIP library under paper_2505_07329_amd/) never links, loads or calls it, and
 * shares no code, header, table or constant with it.
 *
 * Everything here is deliberately slow and obvious: residues are uint64_t,
 * products go through unsigned __int128 and are reduced with '%'. The random
 * quantities of the scheme (mask, secret, error) are inputs, never drawn here.
 *
 * Conventions
 *   N            ring degree, power of two; ring R_q = Z_q[X]/(X^N + 1)   (Sec. 3.1)
 *   P, primes    RNS primes q_1..q_P (P = 1 or 2), q = prod q_p
 *   polynomial   uint64_t[N], coefficient k of X^k, canonical residue in [0, q_p)
 *   RLWE ct      per block: A[P][N] then B[P][N]                          (Sec. 3.1)
 *   LWE ct       per prime: a[N] then b  -> uint64_t[P][N+1]             (Sec. 3.1)
 *   switched LWE uint32_t[N+1] modulo 2^32                                (Sec. 3.2)
 */
#ifndef RLWE_ORACLE_H
#define RLWE_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* a*b mod q (exact, 128-bit intermediate). */
uint64_t orc_mulmod(uint64_t a, uint64_t b, uint64_t q);
/* a^e mod q. */
uint64_t orc_powmod(uint64_t a, uint64_t e, uint64_t q);

/* Negacyclic product out = a*b in Z_q[X]/(X^N+1) by the schoolbook definition:
 * out[m] = sum_{i+j=m} a_i b_j - sum_{i+j=m+N} a_i b_j. */
void orc_poly_mul_schoolbook(const uint64_t* a, const uint64_t* b, uint32_t N,
                             uint64_t q, uint64_t* out);

/* A primitive 2N-th root of unity psi mod q (psi^N = -1); 0 if q != 1 mod 2N. */
uint64_t orc_find_psi(uint32_t N, uint64_t q);

/* Negacyclic product through a psi-twisted cyclic NTT (independent of the
 * schoolbook routine; the two are cross-checked by the tests). */
void orc_poly_mul_ntt(const uint64_t* a, const uint64_t* b, uint32_t N, uint64_t q,
                      uint64_t psi, uint64_t* out);

/* Delta = floor(q / t), t = 2^log2_t, returned as two 64-bit halves. */
void orc_delta(uint32_t P, const uint64_t* primes, uint32_t log2_t, uint64_t* hi,
               uint64_t* lo);

/* RLWE encryption of `count` messages under one ternary secret S (Sec. 3.1):
 *   B = A*S + E + Delta*msg   in R_q, residue-wise for every prime.
 * A: [count][P][N] uniform residues (input), E: [count][N] small signed error,
 * msg: [count][N] signed message coefficients, B: [count][P][N] output.
 * use_ntt selects the product routine (identical results). */
void orc_encrypt(uint32_t N, uint32_t P, const uint64_t* primes, uint32_t log2_t,
                 const int8_t* S, size_t count, const uint64_t* A, const int64_t* E,
                 const int64_t* msg, int use_ntt, uint64_t* B);

/* RLWE phase B - A*S per prime: out [count][P][N]. */
void orc_rlwe_phase(uint32_t N, uint32_t P, const uint64_t* primes, const int8_t* S,
                    size_t count, const uint64_t* A, const uint64_t* B, uint64_t* out);

/* SampleExtract(RLWE(A,B), h) for one prime (Sec. 3.2):
 *   a'_i = A_{h-i} (i <= h),  a'_i = -A_{N+h-i} (i > h),  b' = B_h. */
void orc_sample_extract(const uint64_t* A, const uint64_t* B, uint32_t N, uint64_t q,
                        uint32_t h, uint64_t* a_out, uint64_t* b_out);

/* The server product of Eq. (LWEdot) for a list of (token, row) pairs.
 *   W   int8 [d_out][d_in], row j is w_j
 *   ct  uint64 [T][L][2][P][N], L = ceil(d_in / N): block i of token t is
 *       RLWE(x_hat_i) with A = ct[t][i][0], B = ct[t][i][1]
 *   pairs uint32 [npairs][2] = (t, j)
 *   out uint64 [npairs][P][N+1] = LWE(x . w_j) before any modulus switch
 * For every block i the weights are encoded in reverse, w_hat_ij[k] =
 * w_j[iN+N-1-k] (0 beyond d_in), the ciphertext is multiplied by w_hat_ij in
 * R_q, SampleExtract at index N-1 isolates the partial dot product, and the
 * block results are added (Sec. 4.3, Eq. (LWEdot)).
 * mode 0: products by the schoolbook definition; mode 1: by the NTT. */
void orc_matmul_clear(uint32_t N, uint32_t P, const uint64_t* primes, uint32_t d_out,
                      uint32_t d_in, const int8_t* W, uint32_t T, const uint64_t* ct,
                      size_t npairs, const uint32_t* pairs, int mode, uint64_t* out);

/* ModulusSwitch q -> 2^32 of `count` vectors of `len` coefficients (Sec. 3.2):
 * in uint64 [count][P][len] residues, out uint32 [count][len] with
 *   out = round(c * 2^32 / q) mod 2^32,  c = CRT(residues) in [0, q),
 * rounding half up (a tie cannot occur for odd q). The rational is rounded by
 * exact long division in two 16-bit steps. */
void orc_modswitch(uint32_t P, const uint64_t* primes, size_t count, uint32_t len,
                   const uint64_t* in, uint32_t* out);
/* round(c * 2^k / q) mod 2^k of the CRT value c of every coefficient, 1 <= k <= 32
 * (binary long division): in u64[count][P][len] -> out u32[count][len]. */
void orc_modswitch_bits(uint32_t P, const uint64_t* primes, size_t count, uint32_t len,
                        const uint64_t* in, uint32_t k, uint32_t* out);

/* CRT value of one residue vector, c in [0, q), as two 64-bit halves. */
void orc_crt(uint32_t P, const uint64_t* primes, const uint64_t* residues, uint64_t* hi,
             uint64_t* lo);

/* LWE phase b - <a, S> per prime for ciphertexts [count][P][N+1]: out [count][P]. */
void orc_lwe_phase(uint32_t N, uint32_t P, const uint64_t* primes, const int8_t* S,
                   size_t count, const uint64_t* ct, uint64_t* out);

/* LWE phase modulo 2^32 of switched ciphertexts [count][N+1], centred to
 * [-2^31, 2^31): out [count]. */
void orc_lwe_phase_u32(uint32_t N, const int8_t* S, size_t count, const uint32_t* ct,
                       int64_t* out);

#ifdef __cplusplus
}
#endif

/* Seeded masks (Sec. 3.1: the mask is generated from a seed sent by the client):
 * SplitMix64 output `ctr` under `seed`; mask coefficient n of prime p (rejection
 * sampling onto [0, q) from 54-bit draws); the whole mask A[P][N] of a seed. */
uint64_t orc_splitmix64_at(uint64_t seed, uint64_t ctr);
uint64_t orc_mask_coeff(uint64_t seed, uint32_t N, uint32_t p, uint32_t n, uint64_t q);
void orc_expand_mask(uint64_t seed, uint32_t N, uint32_t P, const uint64_t* primes, uint64_t* A);


/* KeySwitch packing (Sec. 3.2 KeySwitching and Rotate; Sec. 4.3 Eq. (pack_rotate)).
 * Decomp is the gadget decomposition of TFHE: a~ = round(c 2^K / q) mod 2^K with K =
 * beta ell, then ell signed base-2^beta digits d_0 (most significant) .. d_{ell-1} in
 * [-2^(beta-1), 2^(beta-1)); gadget g_m = round(q / 2^(beta (m+1))).
 *   orc_decomp          in [count][P] residues -> out [count][ell] digits
 *   orc_gadget          out [ell][P] residues of g_m
 *   orc_ksk_gen         KSK_{i,m} = RLWE_{S_dst}(S_src[i] g_m): A [N][ell][P][N],
 *                       E [N][ell][N] -> ksk [N][ell][2][P][N]
 *   orc_keyswitch_pack  M LWEs [M][P][N+1] -> ceil(M / n_pack) RLWEs [G][2][P][N];
 *                       LWE g n_pack + s lands in slot s of output g. mode 0: the
 *                       definition one LWE at a time; 1: digit polynomials by NTT */
void orc_decomp(uint32_t P, const uint64_t* primes, size_t count, const uint64_t* in,
                uint32_t beta, uint32_t ell, int64_t* out);
void orc_gadget(uint32_t P, const uint64_t* primes, uint32_t beta, uint32_t ell, uint64_t* out);
void orc_ksk_gen(uint32_t N, uint32_t P, const uint64_t* primes, uint32_t beta, uint32_t ell,
                 const int8_t* S_src, const int8_t* S_dst, const uint64_t* A, const int64_t* E,
                 uint64_t* ksk);
void orc_keyswitch_pack(uint32_t N, uint32_t P, const uint64_t* primes, uint32_t beta,
                        uint32_t ell, uint32_t M, uint32_t n_pack, const uint64_t* lwe,
                        const uint64_t* ksk, int mode, uint64_t* out);
/* Threads of the parallel loops (timing only; results do not depend on it). */
void orc_set_threads(int n);
int orc_max_threads(void);

#endif
