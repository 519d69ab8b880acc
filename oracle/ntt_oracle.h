/*
 * CPU oracle for the negacyclic NTT library -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct reference arithmetic. Only the test suite,
 * the smoke check and the benchmark's cpu_baseline leg may load it; the
 * product path never links, imports or calls it, and it shares no code with
 * the GPU path. All arithmetic is exact over Z_q with 128-bit products and a
 * '%' reduction per operation (no lazy ranges, no precomputed quotients).
 *
 * Notation follows the paper (NTTSuite, "Twiddle Factors" paragraph, Eq. 1-3):
 * N = 2^L points, q the prime (the paper's P), W_N^i the twiddle factors.
 * The negacyclic twist, the inverse transform and the pointwise product are
 * not in the paper; their definitions are the textbook ones:
 *   psi     = c^((q-1)/(2N)), c the smallest quadratic non-residue mod q
 *             (a primitive 2N-th root of unity: psi^N = -1), omega = psi^2
 *   NTT(x)_k  = sum_j x_j psi^((2k+1) j)                    k = 0..N-1
 *   INTT(X)_j = N^-1 psi^-j sum_k X_k omega^(-jk)           j = 0..N-1
 *   (a*b)_k   = sum_{i+j=k} a_i b_j - sum_{i+j=k+N} a_i b_j (mod x^N + 1)
 * Parity status of each function is listed beside it.
 */
#ifndef NTT_ORACLE_H
#define NTT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* --- scalar arithmetic mod q (modulo_add / modulo_mult semantics, Alg. 4-5,
 *     computed the slow way: a full product and '%') ------------------------ */
uint64_t orc_addmod(uint64_t a, uint64_t b, uint64_t q);
uint64_t orc_submod(uint64_t a, uint64_t b, uint64_t q);
uint64_t orc_mulmod(uint64_t a, uint64_t b, uint64_t q);
uint64_t orc_powmod(uint64_t a, uint64_t e, uint64_t q);
uint64_t orc_invmod(uint64_t a, uint64_t q);           /* a^(q-2), q prime */

/* --- parameters ------------------------------------------------------------ */
/* smallest c >= 2 with c^((q-1)/2) == q-1 (Euler's criterion); 0 if none < 1000 */
uint64_t orc_smallest_qnr(uint64_t q);
/* psi = c^((q-1)/(2N)); returns 0 if 2N does not divide q-1 */
uint64_t orc_psi(uint64_t q, uint32_t N);

/* --- transforms on one length-N vector, values canonical in [0,q) --------- */
/* bit_reverse(x): the index permutation used by DIT (before) and DIF (after) */
void orc_bit_reverse(uint64_t* x, uint32_t N);
/* forward negacyclic NTT, natural order in and out: twist by psi^j, then the
 * paper's iterative DIT (Alg. 1, loop bounds read as m = 2^s, k < m/2)       */
void orc_ntt_forward(uint64_t* x, uint32_t N, uint64_t q, uint64_t psi);
/* inverse: the paper's DIF (Alg. 2) with omega^-1 twiddles, bit_reverse,
 * then untwist by psi^-j and scale by N^-1                                   */
void orc_ntt_inverse(uint64_t* x, uint32_t N, uint64_t q, uint64_t psi);
/* O(N^2) direct evaluation of the definition (the pin for the two above)    */
void orc_ntt_direct(const uint64_t* x, uint64_t* X, uint32_t N, uint64_t q, uint64_t psi);
/* single outputs of the definitions, O(N) each: sampled parity at full size */
uint64_t orc_ntt_direct_coeff(const uint64_t* x, uint32_t N, uint64_t q, uint64_t psi, uint32_t k);
uint64_t orc_intt_direct_coeff(const uint64_t* X, uint32_t N, uint64_t q, uint64_t psi, uint32_t j);
/* pointwise product Z_k = X_k Y_k mod q                                     */
void orc_pointwise(const uint64_t* a, const uint64_t* b, uint64_t* c, uint32_t N, uint64_t q);
/* negacyclic schoolbook product mod (x^N + 1, q), O(N^2), and one output     */
void orc_negacyclic_mul(const uint64_t* a, const uint64_t* b, uint64_t* c, uint32_t N, uint64_t q);
uint64_t orc_negacyclic_coeff(const uint64_t* a, const uint64_t* b, uint32_t N, uint64_t q, uint32_t k);

/* --- the cyclic transform of Eq. 3, X_k = sum_j x_j W_N^(jk), W_N = omega --- */
/* omega = c^((q-1)/N), c the smallest quadratic non-residue; 0 if N does not divide q-1 */
uint64_t orc_omega(uint64_t q, uint32_t N);
/* the paper's DIT (Alg. 1) as printed (with the loop-bound reading of the
 * negacyclic version), natural order in and out                              */
void orc_ntt_cyclic_forward(uint64_t* x, uint32_t N, uint64_t q, uint64_t omega);
/* DIF (Alg. 2) with omega^-1, bit_reverse, scale by N^-1                     */
void orc_ntt_cyclic_inverse(uint64_t* x, uint32_t N, uint64_t q, uint64_t omega);
uint64_t orc_ntt_cyclic_direct_coeff(const uint64_t* x, uint32_t N, uint64_t q, uint64_t omega, uint32_t k);
/* Pease constant geometry (Alg. 3): bit_reverse, then for s = L..1 every
 * stage reads the adjacent pair (x[2r], x[2r+1]) and writes y[r], y[r+N/2];
 * the twiddle the listing omits is W[r & ~(2^(s-1) - 1)] (reading of Alg. 3) */
void orc_pease_cyclic_forward(uint64_t* x, uint32_t N, uint64_t q, uint64_t omega);
/* Stockham autosort (§2 "Stockham"): two arrays and no bit reversal; stage
 * t (1..L) with Lt = 2^t, half h = Lt/2, r = N/Lt maps x(j + h k) and
 * x(j + h (k + r)) to y(j + Lt k) and y(j + h + Lt k), twiddle W^((N/Lt) j) */
void orc_stockham_cyclic_forward(uint64_t* x, uint32_t N, uint64_t q, uint64_t omega);

/* --- batched drivers over a row-major [B][L][N] array (limb l uses q[l]) ---
 * nthreads <= 0 means all OpenMP threads; returns the thread count used.    */
int orc_ntt_forward_batch(uint64_t* x, uint32_t B, uint32_t L, uint32_t N,
                          const uint64_t* q, const uint64_t* psi, int nthreads);
int orc_ntt_inverse_batch(uint64_t* x, uint32_t B, uint32_t L, uint32_t N,
                          const uint64_t* q, const uint64_t* psi, int nthreads);
int orc_pointwise_batch(const uint64_t* a, const uint64_t* b, uint64_t* c, uint32_t B,
                        uint32_t L, uint32_t N, const uint64_t* q, int nthreads);

/* --- HE steps on either side of the transform. The paper lists further HE
 * primitives as future work (Conclusion) and motivates the NTT by HE (§1);
 * these follow the standard definitions of the RNS HE literature.
 *
 * Ciphertext tensor product in the evaluation domain (first step of a
 * ciphertext-ciphertext product, Fan-Vercauteren / BGV / CKKS): for
 * ciphertexts a = (a0, a1) and b = (b0, b1),
 *   d0 = a0 b0,  d1 = a0 b1 + a1 b0,  d2 = a1 b1        (mod q, elementwise)
 * so that (a0 + a1 s)(b0 + b1 s) = d0 + d1 s + d2 s^2 for any s.
 * Batched layout: a, b [B][2][L][N], d [B][3][L][N]; limb l uses q[l].
 * Parity: pinned by the s-identity above (Python integers).                  */
void orc_tensor_product(const uint64_t* a0, const uint64_t* a1, const uint64_t* b0, const uint64_t* b1,
                        uint64_t* d0, uint64_t* d1, uint64_t* d2, uint32_t N, uint64_t q);
int orc_tensor_batch(const uint64_t* a, const uint64_t* b, uint64_t* d, uint32_t B, uint32_t L, uint32_t N,
                     const uint64_t* q, int nthreads);

/* Fast RNS basis conversion (Bajard, Eynard, Hasan, Zucca, SAC 2016) from
 * the source basis s_0..s_{L-1} (product S) to the target basis t_0..t_{K-1}
 * (all primes, pairwise distinct): with shat_i = S / s_i,
 *   conv(x)_j = sum_i [x_i shat_i^-1 mod s_i] shat_i   mod t_j.
 * The sum is an integer equal to X + alpha S, X in [0,S) the value with
 * residues x_i and 0 <= alpha < L; conv gives its residues mod each t_j.
 * ModDown (the division by S that ends key switching, Cheon-Han-Kim-Kim-Song,
 * SAC 2018): for y over the target basis and x over the source basis,
 *   moddown(x, y)_j = (y_j - conv(x)_j) S^-1   mod t_j.
 * Layouts: x [B][L][N], y and out [B][K][N]; canonical residues.
 * Parity: pinned through the CRT with Python integers (conv(X) = X + alpha S
 * for one alpha < L; moddown(X S + E) = X - beta for one beta < L).          */
void orc_base_conv(const uint64_t* x, uint64_t* out, uint32_t N, const uint64_t* s, uint32_t L,
                   const uint64_t* t, uint32_t K);
void orc_mod_down(const uint64_t* x, const uint64_t* y, uint64_t* out, uint32_t N, const uint64_t* s,
                  uint32_t L, const uint64_t* t, uint32_t K);
int orc_base_conv_batch(const uint64_t* x, uint64_t* out, uint32_t B, uint32_t N, const uint64_t* s,
                        uint32_t L, const uint64_t* t, uint32_t K, int nthreads);
int orc_mod_down_batch(const uint64_t* x, const uint64_t* y, uint64_t* out, uint32_t B, uint32_t N,
                       const uint64_t* s, uint32_t L, const uint64_t* t, uint32_t K, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
