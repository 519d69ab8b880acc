// Host-side parameter generation for the GPU library: primality, the root
// psi, twiddle tables with Shoup companions, per-limb constants. Written
// independently of the CPU oracle (which the library never links).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace nttp {

uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q);
uint64_t powmod(uint64_t a, uint64_t e, uint64_t q);
bool is_prime(uint64_t n);
// smallest c >= 2 with c^((q-1)/2) == -1 mod q (0 if none below 1000)
uint64_t smallest_qnr(uint64_t q);
// psi = c^((q-1)/2N); 0 if 2N does not divide q-1
uint64_t default_psi(uint64_t q, uint32_t N);

// omega = c^((q-1)/N) for the cyclic transform; 0 if N does not divide q-1
uint64_t default_omega(uint64_t q, uint32_t N);

// Twiddle tables, N entries of (w, floor(w * 2^word / q)), word = 64 or 32.
// Negacyclic (root = psi, a primitive 2N-th root of unity):
//  forward: slot k >= 1 holds psi^brv(k), the factor of butterfly group k
//           (stage floor(log2 k)); slot 0 holds 1 (unused)
//  inverse: slot k >= 2 holds psi^-brv(k); slot 1 holds psi^(-N/2) * N^-1 and
//           slot 0 holds N^-1 (the last inverse stage scales both outputs)
// Cyclic (root = omega, a primitive N-th root): slot 2^s + i holds
//  omega^((N >> (s+1)) * brv_s(i)), the root splitting x^(2m) - z into
//  x^m -+ sqrt(z) for the group's z; the inverse holds the inverses with the
//  same N^-1 fold in slots 0 and 1.
void twiddles(uint64_t q, uint64_t root, uint32_t logN, int word, bool inverse, void* out, bool cyclic = false);
// Twist table of the twisted four-step row pass, N = N1 * N2 entries of
// (w, Shoup companion): entry r * N2 + j holds beta_r^j (inverse: beta_r^-j)
// with beta_r = root^(2 brv(r) + 1) for a negacyclic root of order 2N, or
// root^brv(r) for a cyclic root of order N, brv over log2(N1) bits. Row r of
// the matrix left by the first log2(N1) merged stages is the residue modulo
// x^N2 - beta_r^N2, and its outputs are the values at beta_r * w2^brv(c), w2 =
// root^(2 N1) (negacyclic) or root^N1 (cyclic), the root of row_root().
void twist(uint64_t q, uint64_t root, uint32_t logN, uint32_t logN1, int word, bool inverse, bool cyclic, void* out);
// the primitive N2-th root shared by every row of that factorisation
uint64_t row_root(uint64_t q, uint64_t root, uint32_t logN1, bool cyclic);
// per-limb constants in the layout of nttk::ModInfo64 / ModInfo32
void modinfo(uint64_t q, int word, void* out);
// The fused product's last inverse stage: slots 0 and 1 of an inverse table
// (N^-1, and the first stage's twiddle times N^-1) times 2^word mod q, as two
// table entries with their companions. The fused product's Montgomery
// products leave a factor 2^-word that these multiply back out.
void mont_scale(uint64_t q, int word, const void* inv_table, void* out);
size_t tw_entry_bytes(int word);
size_t modinfo_bytes(int word);

}  // namespace nttp
