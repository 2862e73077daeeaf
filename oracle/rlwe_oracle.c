/*
 * Plain CPU oracle for the encrypted clear-weight product (see rlwe_oracle.h).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline of the benchmark; never by the product path.
 *
 * Paper passages followed:
 *   Sec. 3.1  RLWE / LWE ciphertexts, B = A*S + E + Delta*M, Delta = q/t
 *   Sec. 3.2  SampleExtract, ModulusSwitch, multiplication by a clear polynomial
 *   Sec. 4.3  block split of x, reversed weight encoding, Eq. (LWEdot)
 */
#include "rlwe_oracle.h"

#include <omp.h>

#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
typedef __int128 i128;

uint64_t orc_mulmod(uint64_t a, uint64_t b, uint64_t q) {
  return (uint64_t)(((u128)a * b) % q);
}

uint64_t orc_powmod(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  a %= q;
  while (e) {
    if (e & 1) r = orc_mulmod(r, a, q);
    a = orc_mulmod(a, a, q);
    e >>= 1;
  }
  return r;
}

/* signed integer -> canonical residue */
static uint64_t mod_i64(int64_t x, uint64_t q) {
  i128 r = (i128)x % (i128)q;
  if (r < 0) r += q;
  return (uint64_t)r;
}

/* ------------------------------------------------------------ ring products */

void orc_poly_mul_schoolbook(const uint64_t* a, const uint64_t* b, uint32_t N,
                             uint64_t q, uint64_t* out) {
  /* X^N = -1: a term a_i b_j with i + j >= N lands on X^{i+j-N} with a minus sign.
   * Each product is below 2^108 and at most N <= 2^15 of them are summed, so the
   * positive and negative parts fit in 128 bits before the final reduction. */
  for (uint32_t m = 0; m < N; ++m) {
    u128 pos = 0, neg = 0;
    for (uint32_t i = 0; i <= m; ++i) pos += (u128)a[i] * b[m - i];
    for (uint32_t i = m + 1; i < N; ++i) neg += (u128)a[i] * b[N + m - i];
    uint64_t p = (uint64_t)(pos % q), n = (uint64_t)(neg % q);
    out[m] = p >= n ? p - n : p + (q - n);
  }
}

uint64_t orc_find_psi(uint32_t N, uint64_t q) {
  if ((q - 1) % (2ull * N) != 0) return 0;
  for (uint64_t x = 2; x < q; ++x) {
    uint64_t psi = orc_powmod(x, (q - 1) / (2ull * N), q);
    /* psi^(2N) = 1 always; psi^N = -1 makes its order exactly 2N (N a power of 2) */
    if (orc_powmod(psi, N, q) == q - 1) return psi;
  }
  return 0;
}

static uint32_t bit_reverse(uint32_t x, uint32_t logn) {
  uint32_t r = 0;
  for (uint32_t i = 0; i < logn; ++i) r |= ((x >> i) & 1u) << (logn - 1 - i);
  return r;
}

/* In-place cyclic NTT of length n with root w (order n): X_k = sum_i x_i w^{ik}. */
static void ntt_cyclic(uint64_t* x, uint32_t n, uint64_t w, uint64_t q) {
  uint32_t logn = 0;
  while ((1u << logn) < n) ++logn;
  for (uint32_t i = 0; i < n; ++i) {
    uint32_t r = bit_reverse(i, logn);
    if (r > i) {
      uint64_t t = x[i];
      x[i] = x[r];
      x[r] = t;
    }
  }
  for (uint32_t len = 2; len <= n; len <<= 1) {
    uint64_t wl = orc_powmod(w, n / len, q);
    for (uint32_t s = 0; s < n; s += len) {
      uint64_t wk = 1;
      for (uint32_t k = 0; k < len / 2; ++k) {
        uint64_t u = x[s + k], v = orc_mulmod(x[s + k + len / 2], wk, q);
        x[s + k] = (u + v) % q;
        x[s + k + len / 2] = (u + q - v) % q;
        wk = orc_mulmod(wk, wl, q);
      }
    }
  }
}

void orc_poly_mul_ntt(const uint64_t* a, const uint64_t* b, uint32_t N, uint64_t q,
                      uint64_t psi, uint64_t* out) {
  /* a(X) b(X) mod X^N + 1: substitute X = psi Y, which turns X^N + 1 into
   * -(Y^N - 1) scaled, i.e. a cyclic product of the twisted sequences a_i psi^i. */
  uint64_t* ta = (uint64_t*)malloc(sizeof(uint64_t) * N);
  uint64_t* tb = (uint64_t*)malloc(sizeof(uint64_t) * N);
  uint64_t pw = 1;
  for (uint32_t i = 0; i < N; ++i) {
    ta[i] = orc_mulmod(a[i] % q, pw, q);
    tb[i] = orc_mulmod(b[i] % q, pw, q);
    pw = orc_mulmod(pw, psi, q);
  }
  uint64_t w = orc_mulmod(psi, psi, q);
  ntt_cyclic(ta, N, w, q);
  ntt_cyclic(tb, N, w, q);
  for (uint32_t i = 0; i < N; ++i) ta[i] = orc_mulmod(ta[i], tb[i], q);
  uint64_t winv = orc_powmod(w, q - 2, q);
  ntt_cyclic(ta, N, winv, q);
  uint64_t ninv = orc_powmod(N, q - 2, q), psiinv = orc_powmod(psi, q - 2, q);
  pw = ninv;
  for (uint32_t i = 0; i < N; ++i) {
    out[i] = orc_mulmod(ta[i], pw, q);
    pw = orc_mulmod(pw, psiinv, q);
  }
  free(ta);
  free(tb);
}

/* ------------------------------------------------------------ encryption */

static u128 product_q(uint32_t P, const uint64_t* primes) {
  u128 q = 1;
  for (uint32_t p = 0; p < P; ++p) q *= primes[p];
  return q;
}

void orc_delta(uint32_t P, const uint64_t* primes, uint32_t log2_t, uint64_t* hi,
               uint64_t* lo) {
  u128 d = product_q(P, primes) >> log2_t; /* floor(q / 2^log2_t) */
  *hi = (uint64_t)(d >> 64);
  *lo = (uint64_t)d;
}

static void poly_mul(const uint64_t* a, const uint64_t* b, uint32_t N, uint64_t q,
                     int use_ntt, uint64_t* out) {
  if (use_ntt)
    orc_poly_mul_ntt(a, b, N, q, orc_find_psi(N, q), out);
  else
    orc_poly_mul_schoolbook(a, b, N, q, out);
}

void orc_encrypt(uint32_t N, uint32_t P, const uint64_t* primes, uint32_t log2_t,
                 const int8_t* S, size_t count, const uint64_t* A, const int64_t* E,
                 const int64_t* msg, int use_ntt, uint64_t* B) {
  u128 delta = product_q(P, primes) >> log2_t;
#pragma omp parallel for schedule(dynamic) collapse(2)
  for (size_t c = 0; c < count; ++c) {
    for (uint32_t p = 0; p < P; ++p) {
      uint64_t q = primes[p];
      uint64_t dq = (uint64_t)(delta % q);
      uint64_t* s = (uint64_t*)malloc(sizeof(uint64_t) * N);
      uint64_t* as = (uint64_t*)malloc(sizeof(uint64_t) * N);
      for (uint32_t k = 0; k < N; ++k) s[k] = mod_i64(S[k], q);
      const uint64_t* a = A + (c * P + p) * N;
      poly_mul(a, s, N, q, use_ntt, as);
      uint64_t* b = B + (c * P + p) * N;
      for (uint32_t k = 0; k < N; ++k) {
        uint64_t e = mod_i64(E[c * N + k], q);
        uint64_t m = orc_mulmod(dq, mod_i64(msg[c * N + k], q), q);
        b[k] = (uint64_t)(((u128)as[k] + e + m) % q);
      }
      free(s);
      free(as);
    }
  }
}

void orc_rlwe_phase(uint32_t N, uint32_t P, const uint64_t* primes, const int8_t* S,
                    size_t count, const uint64_t* A, const uint64_t* B, uint64_t* out) {
#pragma omp parallel for schedule(dynamic) collapse(2)
  for (size_t c = 0; c < count; ++c) {
    for (uint32_t p = 0; p < P; ++p) {
      uint64_t q = primes[p];
      uint64_t* s = (uint64_t*)malloc(sizeof(uint64_t) * N);
      uint64_t* as = (uint64_t*)malloc(sizeof(uint64_t) * N);
      for (uint32_t k = 0; k < N; ++k) s[k] = mod_i64(S[k], q);
      poly_mul(A + (c * P + p) * N, s, N, q, 1, as);
      const uint64_t* b = B + (c * P + p) * N;
      for (uint32_t k = 0; k < N; ++k) out[(c * P + p) * N + k] = (b[k] + q - as[k]) % q;
      free(s);
      free(as);
    }
  }
}

/* ------------------------------------------------------------ server product */

void orc_sample_extract(const uint64_t* A, const uint64_t* B, uint32_t N, uint64_t q,
                        uint32_t h, uint64_t* a_out, uint64_t* b_out) {
  for (uint32_t i = 0; i < N; ++i) {
    if (i <= h)
      a_out[i] = A[h - i];
    else
      a_out[i] = (q - A[N + h - i]) % q;
  }
  *b_out = B[h];
}

/* Coefficient m of the negacyclic product a*b (schoolbook definition). */
static uint64_t product_coeff(const uint64_t* a, const uint64_t* b, uint32_t N, uint64_t q,
                              uint32_t m) {
  u128 pos = 0, neg = 0;
  for (uint32_t i = 0; i <= m; ++i) pos += (u128)a[i] * b[m - i];
  for (uint32_t i = m + 1; i < N; ++i) neg += (u128)a[i] * b[N + m - i];
  uint64_t p = (uint64_t)(pos % q), n = (uint64_t)(neg % q);
  return p >= n ? p - n : p + (q - n);
}

/* Schoolbook product that skips the zero coefficients of the clear operand b
 * (the weight block has at most d_in non-zeros); same definition as above. */
static void product_sparse(const uint64_t* a, const uint64_t* b, uint32_t N, uint64_t q,
                           uint64_t* out) {
  u128* pos = (u128*)calloc(N, sizeof(u128));
  u128* neg = (u128*)calloc(N, sizeof(u128));
  for (uint32_t j = 0; j < N; ++j) {
    if (b[j] == 0) continue;
    for (uint32_t i = 0; i < N; ++i) {
      uint32_t m = i + j;
      if (m < N)
        pos[m] += (u128)a[i] * b[j];
      else
        neg[m - N] += (u128)a[i] * b[j];
    }
  }
  for (uint32_t m = 0; m < N; ++m) {
    uint64_t p = (uint64_t)(pos[m] % q), n = (uint64_t)(neg[m] % q);
    out[m] = p >= n ? p - n : p + (q - n);
  }
  free(pos);
  free(neg);
}

void orc_matmul_clear(uint32_t N, uint32_t P, const uint64_t* primes, uint32_t d_out,
                      uint32_t d_in, const int8_t* W, uint32_t T, const uint64_t* ct,
                      size_t npairs, const uint32_t* pairs, int mode, uint64_t* out) {
  const uint32_t L = (d_in + N - 1) / N; /* number of input blocks (Sec. 4.3) */
  (void)d_out;
  (void)T;
#pragma omp parallel for schedule(dynamic)
  for (size_t e = 0; e < npairs; ++e) {
    const uint32_t t = pairs[2 * e], j = pairs[2 * e + 1];
    uint64_t* what = (uint64_t*)malloc(sizeof(uint64_t) * N);
    uint64_t* ca = (uint64_t*)malloc(sizeof(uint64_t) * N);
    uint64_t* cb = (uint64_t*)malloc(sizeof(uint64_t) * N);
    uint64_t* ea = (uint64_t*)malloc(sizeof(uint64_t) * N);
    for (uint32_t p = 0; p < P; ++p) {
      const uint64_t q = primes[p];
      uint64_t psi = mode == 1 ? orc_find_psi(N, q) : 0;
      uint64_t* acc = out + (e * P + p) * (size_t)(N + 1);
      memset(acc, 0, sizeof(uint64_t) * (N + 1));
      for (uint32_t i = 0; i < L; ++i) {
        /* reversed encoding of block i of w_j */
        for (uint32_t k = 0; k < N; ++k) {
          uint64_t src = (uint64_t)i * N + N - 1 - k;
          what[k] = src < d_in ? mod_i64(W[(size_t)j * d_in + src], q) : 0;
        }
        const uint64_t* A = ct + ((((size_t)t * L + i) * 2 + 0) * P + p) * N;
        const uint64_t* B = ct + ((((size_t)t * L + i) * 2 + 1) * P + p) * N;
        /* RLWE(x_hat_i) . w_hat_ij = (A w_hat, B w_hat) */
        uint64_t eb;
        if (mode == 1) {
          orc_poly_mul_ntt(A, what, N, q, psi, ca);
          orc_poly_mul_ntt(B, what, N, q, psi, cb);
          orc_sample_extract(ca, cb, N, q, N - 1, ea, &eb);
        } else {
          product_sparse(A, what, N, q, ca);
          /* SampleExtract reads only coefficient N-1 of the body product */
          cb[N - 1] = product_coeff(B, what, N, q, N - 1);
          orc_sample_extract(ca, cb, N, q, N - 1, ea, &eb);
        }
        for (uint32_t k = 0; k < N; ++k) acc[k] = (acc[k] + ea[k]) % q;
        acc[N] = (acc[N] + eb) % q;
      }
    }
    free(what);
    free(ca);
    free(cb);
    free(ea);
  }
}

/* ------------------------------------------------------------ seeded masks */

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) used as a counter-based
 * generator: output `ctr` under `seed` is the (ctr + 1)-th output of the
 * sequential generator whose state starts at `seed` (state += golden gamma,
 * then the published 64-bit finalizer). */
static uint64_t splitmix64_at(uint64_t seed, uint64_t ctr) {
  uint64_t z = seed + (ctr + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t orc_splitmix64_at(uint64_t seed, uint64_t ctr) { return splitmix64_at(seed, ctr); }

/* Mask coefficient n of prime p (modulus q < 2^54) of the ciphertext with this
 * seed: the top 54 bits of draws (p N + n) 16 + j, j = 0..15, the first below q
 * (rejection sampling: uniform on [0, q)); if all 16 are rejected (probability
 * below 2^-200 for the primes used here), the first draw reduced mod q. */
uint64_t orc_mask_coeff(uint64_t seed, uint32_t N, uint32_t p, uint32_t n, uint64_t q) {
  const uint64_t base = ((uint64_t)p * N + n) << 4;
  for (uint32_t j = 0; j < 16; ++j) {
    const uint64_t v = splitmix64_at(seed, base | j) >> 10;
    if (v < q) return v;
  }
  return (splitmix64_at(seed, base) >> 10) % q;
}

/* The mask A of one ciphertext expanded from its seed: A[p][n], P primes. */
void orc_expand_mask(uint64_t seed, uint32_t N, uint32_t P, const uint64_t* primes, uint64_t* A) {
  for (uint32_t p = 0; p < P; ++p)
    for (uint32_t n = 0; n < N; ++n) A[(size_t)p * N + n] = orc_mask_coeff(seed, N, p, n, primes[p]);
}

/* ------------------------------------------------------------ modulus switch */

static u128 crt(uint32_t P, const uint64_t* primes, const uint64_t* r, size_t stride) {
  if (P == 1) return r[0] % primes[0];
  /* c = sum_p y_p (q / q_p) mod q with y_p = r_p (q/q_p)^{-1} mod q_p; P = 2 here */
  u128 q = product_q(P, primes);
  u128 c = 0;
  for (uint32_t p = 0; p < P; ++p) {
    uint64_t qp = primes[p];
    u128 Mp = q / qp;
    uint64_t inv = orc_powmod((uint64_t)(Mp % qp), qp - 2, qp);
    uint64_t y = orc_mulmod(r[p * stride] % qp, inv, qp);
    c += (u128)y * Mp; /* each term < q, P = 2 terms < 2q < 2^128 */
    if (c >= q) c -= q;
  }
  return c;
}

void orc_crt(uint32_t P, const uint64_t* primes, const uint64_t* residues, uint64_t* hi,
             uint64_t* lo) {
  u128 c = crt(P, primes, residues, 1);
  *hi = (uint64_t)(c >> 64);
  *lo = (uint64_t)c;
}

/* round(c * 2^32 / q) mod 2^32 for 0 <= c < q < 2^110, by long division of
 * c * 2^32 by q in two steps of 16 bits (each partial dividend < 2^126). */
static uint32_t switch_one(u128 c, u128 q) {
  u128 t1 = c << 16;
  u128 q1 = t1 / q, r1 = t1 % q;
  u128 t2 = r1 << 16;
  u128 q2 = t2 / q, r2 = t2 % q;
  u128 fl = (q1 << 16) + q2;          /* floor(c 2^32 / q) */
  u128 rounded = fl + (2 * r2 >= q);  /* remainder r2/q >= 1/2 rounds up */
  return (uint32_t)rounded;
}

/* round(c * 2^k / q) mod 2^k for 0 <= c < q, 1 <= k <= 32, by binary long
 * division of c * 2^k by q, one quotient bit per step (remainder < q < 2^110). */
static uint32_t switch_bits(u128 c, u128 q, uint32_t k) {
  u128 rem = c;
  uint64_t quo = 0;
  for (uint32_t i = 0; i < k; ++i) {
    rem <<= 1;
    quo <<= 1;
    if (rem >= q) {
      rem -= q;
      quo |= 1;
    }
  }
  quo += (2 * rem >= q); /* remainder rem/q >= 1/2 rounds up */
  return (uint32_t)(quo & ((k == 32) ? 0xffffffffull : ((1ull << k) - 1)));
}

void orc_modswitch_bits(uint32_t P, const uint64_t* primes, size_t count, uint32_t len,
                        const uint64_t* in, uint32_t k, uint32_t* out) {
  u128 q = product_q(P, primes);
#pragma omp parallel for schedule(static)
  for (size_t c = 0; c < count; ++c) {
    for (uint32_t n = 0; n < len; ++n) {
      const uint64_t* r = in + c * (size_t)P * len + n;
      out[c * len + n] = switch_bits(crt(P, primes, r, len), q, k);
    }
  }
}

void orc_modswitch(uint32_t P, const uint64_t* primes, size_t count, uint32_t len,
                   const uint64_t* in, uint32_t* out) {
  u128 q = product_q(P, primes);
#pragma omp parallel for schedule(static)
  for (size_t c = 0; c < count; ++c) {
    for (uint32_t n = 0; n < len; ++n) {
      const uint64_t* r = in + c * (size_t)P * len + n;
      out[c * len + n] = switch_one(crt(P, primes, r, len), q);
    }
  }
}

/* ------------------------------------------------------------ decryption */

void orc_lwe_phase(uint32_t N, uint32_t P, const uint64_t* primes, const int8_t* S,
                   size_t count, const uint64_t* ct, uint64_t* out) {
#pragma omp parallel for schedule(static)
  for (size_t c = 0; c < count; ++c) {
    for (uint32_t p = 0; p < P; ++p) {
      uint64_t q = primes[p];
      const uint64_t* lwe = ct + (c * P + p) * (size_t)(N + 1);
      i128 dot = 0; /* <a, S>, S ternary: |dot| < N q */
      for (uint32_t n = 0; n < N; ++n) dot += (i128)lwe[n] * S[n];
      i128 ph = ((i128)lwe[N] - dot) % (i128)q;
      if (ph < 0) ph += q;
      out[c * P + p] = (uint64_t)ph;
    }
  }
}

void orc_lwe_phase_u32(uint32_t N, const int8_t* S, size_t count, const uint32_t* ct,
                       int64_t* out) {
  for (size_t c = 0; c < count; ++c) {
    const uint32_t* lwe = ct + c * (size_t)(N + 1);
    uint32_t dot = 0; /* arithmetic modulo 2^32 */
    for (uint32_t n = 0; n < N; ++n) dot += lwe[n] * (uint32_t)(int32_t)S[n];
    out[c] = (int64_t)(int32_t)(lwe[N] - dot);
  }
}

/* ------------------------------------------------------------ KeySwitch packing */

/* round(c * 2^K / q) mod 2^K for 0 <= c < q < 2^110, 1 <= K <= 64, by binary long
 * division of c * 2^K by q, one quotient bit per step (remainder < q). */
static uint64_t round_to_2k(u128 c, u128 q, uint32_t K) {
  u128 rem = c;
  uint64_t quo = 0;
  for (uint32_t i = 0; i < K; ++i) {
    rem <<= 1;
    quo <<= 1;
    if (rem >= q) {
      rem -= q;
      quo |= 1;
    }
  }
  quo += (2 * rem >= q); /* rem / q >= 1/2 rounds up; no tie for odd q */
  return K == 64 ? quo : quo & ((1ull << K) - 1);
}

/* Gadget decomposition of TFHE (the Decomp of KeySwitching, Sec. 3.2) of the
 * coefficient whose residues are r[p * stride]: the torus value c / q is rounded
 * to K = beta * ell bits, a~ = round(c 2^K / q) mod 2^K, and a~ is written in
 * signed base 2^beta, a~ = sum_m d_m 2^(beta (ell - 1 - m)) mod 2^K with every
 * d_m in [-2^(beta-1), 2^(beta-1)); d_0 is the most significant digit. The carry
 * out of d_0 is dropped (a multiple of 2^K stands for a multiple of q). */
static void decomp_one(uint32_t P, const uint64_t* primes, const uint64_t* r, size_t stride,
                       uint32_t beta, uint32_t ell, int64_t* d) {
  const u128 q = product_q(P, primes);
  const uint64_t at = round_to_2k(crt(P, primes, r, stride), q, beta * ell);
  const uint64_t base = beta == 64 ? 0 : 1ull << beta; /* beta <= 54 in practice */
  const int64_t half = (int64_t)1 << (beta - 1);
  uint64_t carry = 0;
  for (uint32_t k = 0; k < ell; ++k) { /* least significant digit first */
    const uint32_t m = ell - 1 - k;
    uint64_t v = ((at >> (beta * k)) & (base - 1)) + carry;
    if ((int64_t)v >= half) {
      d[m] = (int64_t)v - (int64_t)base;
      carry = 1;
    } else {
      d[m] = (int64_t)v;
      carry = 0;
    }
  }
}

void orc_decomp(uint32_t P, const uint64_t* primes, size_t count, const uint64_t* in,
                uint32_t beta, uint32_t ell, int64_t* out) {
#pragma omp parallel for schedule(static)
  for (size_t c = 0; c < count; ++c) decomp_one(P, primes, in + c * P, 1, beta, ell, out + c * ell);
}

/* Gadget values g_m = round(q / 2^(beta (m + 1))) as residues mod every prime:
 * out[m][p]. Together with decomp_one, sum_m d_m g_m = c mod q up to
 * q / 2^(K+1) + ell 2^(beta-2) (the rounding of c / q and of the g_m). */
void orc_gadget(uint32_t P, const uint64_t* primes, uint32_t beta, uint32_t ell, uint64_t* out) {
  const u128 q = product_q(P, primes);
  for (uint32_t m = 0; m < ell; ++m) {
    const uint32_t sh = beta * (m + 1);
    const u128 g = sh >= 128 ? 0 : (q + ((u128)1 << (sh - 1))) >> sh;
    for (uint32_t p = 0; p < P; ++p) out[m * P + p] = (uint64_t)(g % primes[p]);
  }
}

/* Key-switching key (Sec. 3.2, KeySwitching): KSK_{i,m} = RLWE_{S_dst}(s_i g_m), the
 * message in the constant coefficient, for every LWE key coefficient i < N
 * (s = S_src, the key SampleExtract leaves) and gadget level m < ell.
 *   A   [N][ell][P][N] uniform residues, E [N][ell][N] errors
 *   ksk [N][ell][2][P][N] (out): A, then B = A S_dst + E + s_i g_m */
void orc_ksk_gen(uint32_t N, uint32_t P, const uint64_t* primes, uint32_t beta, uint32_t ell,
                 const int8_t* S_src, const int8_t* S_dst, const uint64_t* A, const int64_t* E,
                 uint64_t* ksk) {
  uint64_t g[8 * 2];
  orc_gadget(P, primes, beta, ell, g);
#pragma omp parallel for schedule(dynamic) collapse(3)
  for (uint32_t i = 0; i < N; ++i) {
    for (uint32_t m = 0; m < ell; ++m) {
      for (uint32_t p = 0; p < P; ++p) {
        const uint64_t q = primes[p];
        uint64_t* s = (uint64_t*)malloc(sizeof(uint64_t) * N);
        uint64_t* as = (uint64_t*)malloc(sizeof(uint64_t) * N);
        for (uint32_t k = 0; k < N; ++k) s[k] = mod_i64(S_dst[k], q);
        const uint64_t* a = A + (((size_t)i * ell + m) * P + p) * N;
        poly_mul(a, s, N, q, 1, as);
        uint64_t* ka = ksk + ((((size_t)i * ell + m) * 2 + 0) * P + p) * N;
        uint64_t* kb = ksk + ((((size_t)i * ell + m) * 2 + 1) * P + p) * N;
        const uint64_t msg = orc_mulmod(mod_i64(S_src[i], q), g[m * P + p], q);
        for (uint32_t k = 0; k < N; ++k) {
          u128 v = (u128)as[k] + mod_i64(E[((size_t)i * ell + m) * N + k], q);
          if (k == 0) v += msg;
          ka[k] = a[k];
          kb[k] = (uint64_t)(v % q);
        }
        free(s);
        free(as);
      }
    }
  }
}

/* Packing of M LWE ciphertexts into G = ceil(M / n_pack) RLWE ciphertexts,
 * Eq. (pack_rotate): output g = sum over slots s < n_pack (LWE g n_pack + s, while
 * below M) of Rotate(KeySwitching(LWE), s), where
 *   KeySwitching(a, b) = (0, b) - sum_i sum_m Decomp_m(a_i) KSK_{i,m}   (Sec. 3.2)
 * and Rotate by s multiplies both polynomials by X^s in Z_q[X]/(X^N + 1).
 *   lwe  [M][P][N+1] residues (mask, then body), ksk [N][ell][2][P][N]
 *   out  [G][2][P][N]: A, then B of every packed ciphertext
 * mode 0 follows that definition literally, one LWE at a time (N^2 ell 2 P
 * products per LWE: tiny rings only). mode 1 uses the linearity of both steps:
 *   A_g = -sum_i sum_m D_{i,m} KSK_{i,m}.A,  B_g = sum_s b_s X^s - sum_i sum_m D_{i,m} KSK_{i,m}.B
 * with the digit polynomials D_{i,m} = sum_s Decomp_m(a_{g n_pack + s, i}) X^s, each
 * product by the oracle's negacyclic NTT. */
void orc_keyswitch_pack(uint32_t N, uint32_t P, const uint64_t* primes, uint32_t beta,
                        uint32_t ell, uint32_t M, uint32_t n_pack, const uint64_t* lwe,
                        const uint64_t* ksk, int mode, uint64_t* out) {
  const uint32_t G = (M + n_pack - 1) / n_pack;
  const size_t lw = (size_t)P * (N + 1);
  memset(out, 0, sizeof(uint64_t) * (size_t)G * 2 * P * N);
  /* digits of every mask coefficient: dg[(j N + i) ell + m] */
  int64_t* dg = (int64_t*)malloc(sizeof(int64_t) * (size_t)M * N * ell);
#pragma omp parallel for schedule(static)
  for (size_t ji = 0; ji < (size_t)M * N; ++ji) {
    const size_t j = ji / N, i = ji % N;
    decomp_one(P, primes, lwe + j * lw + i, N + 1, beta, ell, dg + ji * ell);
  }
  if (mode == 0) {
#pragma omp parallel for schedule(dynamic)
    for (uint32_t g = 0; g < G; ++g) {
      uint64_t* ks = (uint64_t*)malloc(sizeof(uint64_t) * 2 * P * N);
      for (uint32_t s = 0; s < n_pack && (size_t)g * n_pack + s < M; ++s) {
        const size_t j = (size_t)g * n_pack + s;
        /* KeySwitching(LWE_j), starting from the trivial (0, b) */
        for (uint32_t r = 0; r < P; ++r)
          for (uint32_t n = 0; n < N; ++n) {
            ks[(0 * P + r) * N + n] = 0;
            ks[(1 * P + r) * N + n] = n == 0 ? lwe[j * lw + (size_t)r * (N + 1) + N] : 0;
          }
        for (uint32_t i = 0; i < N; ++i)
          for (uint32_t m = 0; m < ell; ++m) {
            const int64_t d = dg[(j * N + i) * ell + m];
            if (d == 0) continue;
            for (uint32_t c = 0; c < 2; ++c)
              for (uint32_t r = 0; r < P; ++r) {
                const uint64_t q = primes[r], dq = mod_i64(d, q);
                const uint64_t* k = ksk + ((((size_t)i * ell + m) * 2 + c) * P + r) * N;
                uint64_t* o = ks + ((size_t)c * P + r) * N;
                for (uint32_t n = 0; n < N; ++n)
                  o[n] = (uint64_t)(((u128)o[n] + q - orc_mulmod(dq, k[n], q)) % q);
              }
          }
        /* Rotate by s and add: X^s X^n = X^(n+s), or -X^(n+s-N) past the degree */
        for (uint32_t c = 0; c < 2; ++c)
          for (uint32_t r = 0; r < P; ++r) {
            const uint64_t q = primes[r];
            const uint64_t* src = ks + ((size_t)c * P + r) * N;
            uint64_t* dst = out + (((size_t)g * 2 + c) * P + r) * N;
            for (uint32_t n = 0; n < N; ++n) {
              const uint32_t e = n + s;
              if (e < N)
                dst[e] = (dst[e] + src[n]) % q;
              else
                dst[e - N] = (dst[e - N] + q - src[n]) % q;
            }
          }
      }
      free(ks);
    }
  } else {
    for (uint32_t g = 0; g < G; ++g) {
      for (uint32_t r = 0; r < P; ++r) {
        const uint64_t q = primes[r];
        const uint64_t psi = orc_find_psi(N, q);
        uint64_t* acc[2] = {out + (((size_t)g * 2 + 0) * P + r) * N,
                            out + (((size_t)g * 2 + 1) * P + r) * N};
        /* the terms (i, m) are summed in per-thread copies, then added up */
#pragma omp parallel
        {
          uint64_t* D = (uint64_t*)malloc(sizeof(uint64_t) * N);
          uint64_t* prod = (uint64_t*)malloc(sizeof(uint64_t) * N);
          uint64_t* part = (uint64_t*)calloc(2 * (size_t)N, sizeof(uint64_t));
#pragma omp for schedule(dynamic)
          for (uint32_t im = 0; im < N * ell; ++im) {
            const uint32_t i = im / ell, m = im % ell;
            for (uint32_t s = 0; s < N; ++s) {
              const size_t j = (size_t)g * n_pack + s;
              D[s] = (s < n_pack && j < M) ? mod_i64(dg[(j * N + i) * ell + m], q) : 0;
            }
            for (uint32_t c = 0; c < 2; ++c) {
              const uint64_t* k = ksk + ((((size_t)i * ell + m) * 2 + c) * P + r) * N;
              orc_poly_mul_ntt(D, k, N, q, psi, prod);
              for (uint32_t n = 0; n < N; ++n) part[c * N + n] = (part[c * N + n] + prod[n]) % q;
            }
          }
#pragma omp critical
          for (uint32_t c = 0; c < 2; ++c)
            for (uint32_t n = 0; n < N; ++n) acc[c][n] = (acc[c][n] + q - part[c * N + n]) % q;
          free(D);
          free(prod);
          free(part);
        }
        for (uint32_t s = 0; s < n_pack && s < N && (size_t)g * n_pack + s < M; ++s) {
          const size_t j = (size_t)g * n_pack + s;
          acc[1][s] = (acc[1][s] + lwe[j * lw + (size_t)r * (N + 1) + N]) % q;
        }
      }
    }
  }
  free(dg);
}

/* Threads the oracle's parallel loops use (timing on a chosen number of cores). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }
