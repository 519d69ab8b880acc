/*
 * CPU oracle for the negacyclic NTT library -- TEST INFRASTRUCTURE ONLY.
 * Loaded by the test suite, the smoke check and the benchmark's cpu_baseline
 * leg; never by the product path. Shares no code with the GPU library.
 *
 * Every operation reduces with a full 128-bit product and '%', so there are
 * no lazy ranges or precomputed quotients to get wrong. Definitions and the
 * readings of the paper's garbled listings are stated in ntt_oracle.h.
 */
#include "ntt_oracle.h"
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* Planted mistakes for the mutation test of the pins (tests/ builds the
 * oracle with -DORC_MUTANT=k and checks that the pins reject it); the
 * default build has ORC_MUTANT = 0 and compiles none of them. */
#ifndef ORC_MUTANT
#define ORC_MUTANT 0
#endif

/* modulo_add (Alg. 4): inputs in [0,q), the sum lies in [0,2q) and needs at
 * most one subtraction of q; the difference lies in (-q,q) and needs at most
 * one addition of q. Written with '%' here, which gives the same value.   */
uint64_t orc_addmod(uint64_t a, uint64_t b, uint64_t q) {
  return (uint64_t)(((u128)a + b) % q);
}
uint64_t orc_submod(uint64_t a, uint64_t b, uint64_t q) {
  return (uint64_t)(((u128)a + q - b) % q);
}
/* modulo_mult (Alg. 5) computes x*tw mod q; the oracle uses the exact
 * 128-bit product and a remainder instead of the precomputed-quotient trick. */
uint64_t orc_mulmod(uint64_t a, uint64_t b, uint64_t q) {
  return (uint64_t)(((u128)a * b) % q);
}
uint64_t orc_powmod(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q, b = a % q;
  while (e) {
    if (e & 1) r = orc_mulmod(r, b, q);
    b = orc_mulmod(b, b, q);
    e >>= 1;
  }
  return r;
}
uint64_t orc_invmod(uint64_t a, uint64_t q) { return orc_powmod(a, q - 2, q); }

/* The paper's twiddle factors are powers of an unnamed generator g (Eq. 1-3).
 * For the negacyclic transform a primitive 2N-th root psi is needed; it is
 * taken as c^((q-1)/(2N)) with c the smallest quadratic non-residue, which
 * satisfies psi^N = c^((q-1)/2) = -1 by Euler's criterion.                  */
uint64_t orc_smallest_qnr(uint64_t q) {
  for (uint64_t c = 2; c < 1000 && c < q; ++c)
    if (orc_powmod(c, (q - 1) / 2, q) == q - 1) return c;
  return 0;
}
uint64_t orc_psi(uint64_t q, uint32_t N) {
  if (N == 0 || (q - 1) % (2ull * N) != 0) return 0;
  uint64_t c = orc_smallest_qnr(q);
  if (!c) return 0;
  return orc_powmod(c, (q - 1) / (2ull * N), q);
}

/* bit_reverse(x): swap x[i] with x[rev(i)], rev reversing log2(N) bits. */
void orc_bit_reverse(uint64_t* x, uint32_t N) {
  uint32_t L = 0;
  while ((1u << L) < N) ++L;
  for (uint32_t i = 0; i < N; ++i) {
    uint32_t r = 0;
    for (uint32_t b = 0; b < L; ++b) r |= ((i >> b) & 1u) << (L - 1 - b);
    if (i < r) { uint64_t t = x[i]; x[i] = x[r]; x[r] = t; }
  }
}

/* Cyclic NTT by the paper's iterative decimation in time (Alg. 1, Eq. 4-5):
 * bit_reverse, then for s = 1..L with m = 2^s and k < m/2, the twiddle
 * W[(N/m) k] multiplies the odd half of each butterfly. W[i] = w^i where w
 * is the primitive N-th root in use. Output in natural order.              */
static void orc_dit_cyclic(uint64_t* x, uint32_t N, uint64_t q, const uint64_t* W) {
  uint32_t L = 0;
  while ((1u << L) < N) ++L;
#if ORC_MUTANT != 8
  orc_bit_reverse(x, N);
#endif
  for (uint32_t s = 1; s <= L - (ORC_MUTANT == 4 ? 1 : 0); ++s) {
    uint32_t m = 1u << s, h = m >> 1;
    for (uint32_t k = 0; k < h; ++k) {
      uint64_t tw = W[((size_t)(N / m) * k + (ORC_MUTANT == 3 ? 1 : 0)) % N];
      for (uint32_t j = 0; j < N; j += m) {
        uint64_t f1 = x[j + k];
        uint64_t f2 = orc_mulmod(tw, x[j + k + h], q);
        x[j + k] = ORC_MUTANT == 7 ? orc_submod(f1, f2, q) : orc_addmod(f1, f2, q);
        x[j + k + h] = ORC_MUTANT == 7 ? orc_addmod(f1, f2, q) : orc_submod(f1, f2, q);
      }
    }
  }
}

/* Cyclic NTT by the paper's decimation in frequency (Alg. 2, Eq. 6): for
 * s = L..1, the twiddle multiplies the difference of each butterfly; the
 * result is in bit-reversed order and bit_reverse puts it back in order.   */
static void orc_dif_cyclic(uint64_t* x, uint32_t N, uint64_t q, const uint64_t* W) {
  uint32_t L = 0;
  while ((1u << L) < N) ++L;
  for (uint32_t s = L; s >= 1; --s) {
    uint32_t m = 1u << s, h = m >> 1;
    for (uint32_t k = 0; k < h; ++k) {
      uint64_t tw = W[(size_t)(N / m) * k];
      for (uint32_t j = 0; j < N; j += m) {
        uint64_t f1 = x[j + k];
        uint64_t f2 = x[j + k + h];
        x[j + k] = orc_addmod(f1, f2, q);
        x[j + k + h] = orc_mulmod(tw, orc_submod(f1, f2, q), q);
      }
    }
  }
  orc_bit_reverse(x, N);
}

static uint64_t* orc_power_table(uint64_t base, uint32_t count, uint64_t q) {
  uint64_t* t = (uint64_t*)malloc(sizeof(uint64_t) * (count ? count : 1));
  uint64_t v = 1 % q;
  for (uint32_t i = 0; i < count; ++i) { t[i] = v; v = orc_mulmod(v, base, q); }
  return t;
}

/* Negacyclic forward transform: X_k = sum_j (x_j psi^j) omega^(jk), i.e. the
 * cyclic transform of the psi-twisted input, evaluated with DIT.           */
void orc_ntt_forward(uint64_t* x, uint32_t N, uint64_t q, uint64_t psi) {
  uint64_t* P = orc_power_table(psi, N, q);                      /* psi^j   */
  uint64_t* W = orc_power_table(orc_mulmod(psi, psi, q), N, q);  /* omega^i */
#if ORC_MUTANT != 1
  for (uint32_t j = 0; j < N; ++j) x[j] = orc_mulmod(x[j], P[ORC_MUTANT == 2 ? (N - j) % N : j], q);
#endif
  orc_dit_cyclic(x, N, q, W);
  free(P); free(W);
}

/* Negacyclic inverse: x_j = N^-1 psi^-j sum_k X_k omega^(-jk), the cyclic
 * transform with omega^-1 evaluated with DIF, then untwist and scale.      */
void orc_ntt_inverse(uint64_t* x, uint32_t N, uint64_t q, uint64_t psi) {
  uint64_t psi_inv = orc_invmod(psi, q);
  uint64_t n_inv = orc_invmod(N % q, q);
  uint64_t* P = orc_power_table(psi_inv, N, q);                          /* psi^-j   */
  uint64_t* W = orc_power_table(orc_mulmod(psi_inv, psi_inv, q), N, q);  /* omega^-i */
  orc_dif_cyclic(x, N, q, W);
  if (ORC_MUTANT == 5) n_inv = 1;
  for (uint32_t j = 0; j < N; ++j) x[j] = orc_mulmod(orc_mulmod(x[j], P[j], q), n_inv, q);
  free(P); free(W);
}

/* ---- cyclic transform (Eq. 3 as printed) ------------------------------ */
uint64_t orc_omega(uint64_t q, uint32_t N) {
  if (N == 0 || (q - 1) % N != 0) return 0;
  uint64_t c = orc_smallest_qnr(q);
  if (!c) return 0;
  return orc_powmod(c, (q - 1) / N, q);
}
void orc_ntt_cyclic_forward(uint64_t* x, uint32_t N, uint64_t q, uint64_t omega) {
  uint64_t* W = orc_power_table(omega, N, q);
  orc_dit_cyclic(x, N, q, W);
  free(W);
}
void orc_ntt_cyclic_inverse(uint64_t* x, uint32_t N, uint64_t q, uint64_t omega) {
  uint64_t* W = orc_power_table(orc_invmod(omega, q), N, q);
  uint64_t n_inv = orc_invmod(N % q, q);
  orc_dif_cyclic(x, N, q, W);
  for (uint32_t j = 0; j < N; ++j) x[j] = orc_mulmod(x[j], n_inv, q);
  free(W);
}
uint64_t orc_ntt_cyclic_direct_coeff(const uint64_t* x, uint32_t N, uint64_t q, uint64_t omega, uint32_t k) {
  uint64_t step = orc_powmod(omega, k, q), pw = 1 % q, acc = 0;
  for (uint32_t j = 0; j < N; ++j) {
    acc = orc_addmod(acc, orc_mulmod(x[j], pw, q), q);
    pw = orc_mulmod(pw, step, q);
  }
  return acc;
}

void orc_pease_cyclic_forward(uint64_t* x, uint32_t N, uint64_t q, uint64_t omega) {
  uint32_t L = 0;
  while ((1u << L) < N) ++L;
  uint64_t* W = orc_power_table(omega, N / 2 ? N / 2 : 1, q);
  uint64_t* y = (uint64_t*)malloc(sizeof(uint64_t) * N);
  orc_bit_reverse(x, N);
  for (uint32_t s = L; s >= 1; --s) {
    uint32_t base = (1u << (s - 1)) - 1;
    for (uint32_t r = 0; r < N / 2; ++r) {
      uint64_t f1 = x[2 * r];
      uint64_t f2 = orc_mulmod(W[r & ~base], x[2 * r + 1], q);
      y[r] = orc_addmod(f1, f2, q);
      y[r + N / 2] = orc_submod(f1, f2, q);
    }
    memcpy(x, y, sizeof(uint64_t) * N);
  }
  free(y);
  free(W);
}

void orc_stockham_cyclic_forward(uint64_t* x, uint32_t N, uint64_t q, uint64_t omega) {
  uint32_t L = 0;
  while ((1u << L) < N) ++L;
  uint64_t* W = orc_power_table(omega, N, q);
  uint64_t* y = (uint64_t*)malloc(sizeof(uint64_t) * N);
  for (uint32_t t = 1; t <= L; ++t) {
    uint32_t Lt = 1u << t, h = Lt / 2, r = N / Lt;
    for (uint32_t j = 0; j < h; ++j) {
      uint64_t om = W[(size_t)(N / Lt) * j];
      for (uint32_t k = 0; k < r; ++k) {
        uint64_t u = x[j + h * k];
        uint64_t v = orc_mulmod(om, x[j + h * (k + r)], q);
        y[j + Lt * k] = orc_addmod(u, v, q);
        y[j + h + Lt * k] = orc_submod(u, v, q);
      }
    }
    memcpy(x, y, sizeof(uint64_t) * N);
  }
  free(y);
  free(W);
}

/* Direct evaluation of the definition, X_k = sum_j x_j psi^((2k+1) j), with
 * the exponent reduced mod 2N (psi has order 2N).                          */
uint64_t orc_ntt_direct_coeff(const uint64_t* x, uint32_t N, uint64_t q, uint64_t psi, uint32_t k) {
  uint64_t step = orc_powmod(psi, 2ull * k + 1, q);  /* psi^(2k+1) */
  uint64_t pw = 1 % q, acc = 0;
  for (uint32_t j = 0; j < N; ++j) {
    acc = orc_addmod(acc, orc_mulmod(x[j], pw, q), q);
    pw = orc_mulmod(pw, step, q);
  }
  return acc;
}
void orc_ntt_direct(const uint64_t* x, uint64_t* X, uint32_t N, uint64_t q, uint64_t psi) {
  uint64_t* P = orc_power_table(psi, 2 * N, q);  /* psi^e, e < 2N */
  for (uint32_t k = 0; k < N; ++k) {
    uint64_t acc = 0;
    for (uint32_t j = 0; j < N; ++j) {
      uint64_t e = ((2ull * k + (ORC_MUTANT == 6 ? 2 * N - 1 : 1)) * j) % (2ull * N);
      acc = orc_addmod(acc, orc_mulmod(x[j], P[e], q), q);
    }
    X[k] = acc;
  }
  free(P);
}
/* x_j = N^-1 sum_k X_k psi^(-(2k+1) j), the same as the form in the header */
uint64_t orc_intt_direct_coeff(const uint64_t* X, uint32_t N, uint64_t q, uint64_t psi, uint32_t j) {
  uint64_t psi_inv = orc_invmod(psi, q);
  uint64_t step = orc_powmod(psi_inv, 2ull * j, q);   /* omega^-j */
  uint64_t pw = orc_powmod(psi_inv, j, q);            /* psi^-j: the k = 0 term */
  uint64_t acc = 0;
  for (uint32_t k = 0; k < N; ++k) {
    acc = orc_addmod(acc, orc_mulmod(X[k], pw, q), q);
    pw = orc_mulmod(pw, step, q);
  }
  return orc_mulmod(acc, orc_invmod(N % q, q), q);
}

void orc_pointwise(const uint64_t* a, const uint64_t* b, uint64_t* c, uint32_t N, uint64_t q) {
  for (uint32_t k = 0; k < N; ++k) c[k] = orc_mulmod(a[k], ORC_MUTANT == 10 ? a[k] : b[k], q);
}

/* (a*b)_k = sum_{i<=k} a_i b_{k-i} - sum_{i>k} a_i b_{N+k-i}   (x^N = -1) */
uint64_t orc_negacyclic_coeff(const uint64_t* a, const uint64_t* b, uint32_t N, uint64_t q, uint32_t k) {
  uint64_t pos = 0, neg = 0;
  for (uint32_t i = 0; i <= k; ++i) pos = orc_addmod(pos, orc_mulmod(a[i], b[k - i], q), q);
  for (uint32_t i = k + 1; i < N; ++i) neg = orc_addmod(neg, orc_mulmod(a[i], b[N + k - i], q), q);
  return ORC_MUTANT == 9 ? orc_addmod(pos, neg, q) : orc_submod(pos, neg, q);
}
void orc_negacyclic_mul(const uint64_t* a, const uint64_t* b, uint64_t* c, uint32_t N, uint64_t q) {
  for (uint32_t k = 0; k < N; ++k) c[k] = orc_negacyclic_coeff(a, b, N, q, k);
}

/* ---- batched drivers: independent (poly, limb) transforms, one per task -- */
static int orc_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) return nthreads;
  return omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

int orc_ntt_forward_batch(uint64_t* x, uint32_t B, uint32_t L, uint32_t N,
                          const uint64_t* q, const uint64_t* psi, int nthreads) {
  int nt = orc_threads(nthreads);
  long total = (long)B * L;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (long t = 0; t < total; ++t) {
    uint32_t l = (uint32_t)(t % L);
    orc_ntt_forward(x + (size_t)t * N, N, q[l], psi[l]);
  }
  return nt;
}
int orc_ntt_inverse_batch(uint64_t* x, uint32_t B, uint32_t L, uint32_t N,
                          const uint64_t* q, const uint64_t* psi, int nthreads) {
  int nt = orc_threads(nthreads);
  long total = (long)B * L;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (long t = 0; t < total; ++t) {
    uint32_t l = (uint32_t)(t % L);
    orc_ntt_inverse(x + (size_t)t * N, N, q[l], psi[l]);
  }
  return nt;
}
int orc_pointwise_batch(const uint64_t* a, const uint64_t* b, uint64_t* c, uint32_t B,
                        uint32_t L, uint32_t N, const uint64_t* q, int nthreads) {
  int nt = orc_threads(nthreads);
  long total = (long)B * L;
#pragma omp parallel for schedule(static) num_threads(nt)
  for (long t = 0; t < total; ++t) {
    uint32_t l = (uint32_t)(t % L);
    orc_pointwise(a + (size_t)t * N, b + (size_t)t * N, c + (size_t)t * N, N, q[l]);
  }
  return nt;
}

/* ---- HE steps (definitions in ntt_oracle.h) ----------------------------- */
void orc_tensor_product(const uint64_t* a0, const uint64_t* a1, const uint64_t* b0, const uint64_t* b1,
                        uint64_t* d0, uint64_t* d1, uint64_t* d2, uint32_t N, uint64_t q) {
  for (uint32_t k = 0; k < N; ++k) {
    d0[k] = orc_mulmod(a0[k], b0[k], q);
    d1[k] = orc_addmod(orc_mulmod(a0[k], b1[k], q), orc_mulmod(a1[k], ORC_MUTANT == 16 ? b1[k] : b0[k], q), q);
    d2[k] = orc_mulmod(a1[k], b1[k], q);
  }
}
int orc_tensor_batch(const uint64_t* a, const uint64_t* b, uint64_t* d, uint32_t B, uint32_t L, uint32_t N,
                     const uint64_t* q, int nthreads) {
  int nt = orc_threads(nthreads);
  const size_t per = (size_t)L * N;
  long total = (long)B * L;
#pragma omp parallel for schedule(static) num_threads(nt)
  for (long t = 0; t < total; ++t) {
    const size_t c = (size_t)(t / L), l = (size_t)(t % L);
    const uint64_t* ac = a + 2 * per * c + l * N;
    const uint64_t* bc = b + 2 * per * c + l * N;
    uint64_t* dc = d + 3 * per * c + l * N;
    orc_tensor_product(ac, ac + per, bc, bc + per, dc, dc + per, dc + 2 * per, N, q[l]);
  }
  return nt;
}

/* shat_i mod m = prod_{k != i} s_k mod m */
static uint64_t orc_shat_mod(const uint64_t* s, uint32_t L, uint32_t i, uint64_t m) {
  uint64_t r = 1 % m;
  for (uint32_t k = 0; k < L; ++k)
    if (k != i || ORC_MUTANT == 13) r = orc_mulmod(r, s[k] % m, m);
  return r;
}

void orc_base_conv(const uint64_t* x, uint64_t* out, uint32_t N, const uint64_t* s, uint32_t L,
                   const uint64_t* t, uint32_t K) {
  uint64_t* inv = malloc(sizeof(uint64_t) * (L ? L : 1));
  for (uint32_t i = 0; i < L; ++i) inv[i] = orc_invmod(orc_shat_mod(s, L, i, s[i]), s[i]);
  for (uint32_t j = 0; j < K; ++j) {
    for (uint32_t n = 0; n < N; ++n) {
      uint64_t acc = 0;
      for (uint32_t i = 0; i < L - (ORC_MUTANT == 12 ? 1 : 0); ++i) {
        uint64_t y = ORC_MUTANT == 11 ? x[(size_t)i * N + n]
                                      : orc_mulmod(x[(size_t)i * N + n], inv[i], s[i]);
        acc = orc_addmod(acc, orc_mulmod(y % t[j], orc_shat_mod(s, L, i, t[j]), t[j]), t[j]);
      }
      out[(size_t)j * N + n] = acc;
    }
  }
  free(inv);
}

void orc_mod_down(const uint64_t* x, const uint64_t* y, uint64_t* out, uint32_t N, const uint64_t* s,
                  uint32_t L, const uint64_t* t, uint32_t K) {
  orc_base_conv(x, out, N, s, L, t, K);
  for (uint32_t j = 0; j < K; ++j) {
    uint64_t S_inv = orc_invmod(orc_shat_mod(s, L, L, t[j]), t[j]);  /* k != L: the full product */
    if (ORC_MUTANT == 15) S_inv = 1;
    for (uint32_t n = 0; n < N; ++n) {
      const size_t e = (size_t)j * N + n;
      uint64_t diff = ORC_MUTANT == 14 ? orc_submod(out[e], y[e], t[j]) : orc_submod(y[e], out[e], t[j]);
      out[e] = orc_mulmod(diff, S_inv, t[j]);
    }
  }
}

int orc_base_conv_batch(const uint64_t* x, uint64_t* out, uint32_t B, uint32_t N, const uint64_t* s,
                        uint32_t L, const uint64_t* t, uint32_t K, int nthreads) {
  int nt = orc_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (long b = 0; b < (long)B; ++b)
    orc_base_conv(x + (size_t)b * L * N, out + (size_t)b * K * N, N, s, L, t, K);
  return nt;
}
int orc_mod_down_batch(const uint64_t* x, const uint64_t* y, uint64_t* out, uint32_t B, uint32_t N,
                       const uint64_t* s, uint32_t L, const uint64_t* t, uint32_t K, int nthreads) {
  int nt = orc_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (long b = 0; b < (long)B; ++b)
    orc_mod_down(x + (size_t)b * L * N, y + (size_t)b * K * N, out + (size_t)b * K * N, N, s, L, t, K);
  return nt;
}
