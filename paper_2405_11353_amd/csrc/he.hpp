// HE steps on either side of the transform: ciphertext tensor product in
// the evaluation domain, fast RNS basis conversion and ModDown. Device table
// layouts and the launchers of k_he.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nttk {

// One source prime s_i of a conversion: multiply by shat_i^-1 mod s_i.
struct BcSrc {
  uint64_t q;    // s_i
  uint64_t nq;   // 2^64 - s_i
  uint64_t w;    // shat_i^-1 mod s_i, shat_i = S / s_i
  uint64_t wp;   // floor(w * 2^64 / s_i)
};

// One target prime t_j: constants of the final reduction and of the ModDown
// scaling.
struct BcDst {
  uint64_t q;     // t_j
  uint64_t nq;    // 2^64 - t_j
  uint64_t ninv;  // -t_j^-1 mod 2^64 (Montgomery reduction by 2^64)
  uint64_t onep;  // floor(2^64 / t_j), Shoup companion of 1
  uint64_t sinv;  // S^-1 mod t_j
  uint64_t sinvp; // floor(sinv * 2^64 / t_j)
  uint64_t pad0, pad1;
};

// Largest source basis: the 128-bit accumulator holds L products < 2^122.
constexpr int BCONV_MAX_L = 64;
// Terms per group of the kernel's column sums: 8 when every prime of both
// bases is below 2^60, else 4.
inline uint32_t bconv_group(uint64_t max_prime) { return max_prime < (1ull << 60) ? 8 : 4; }
// Row stride of the [K][Lp] matrix (zero padded to a whole group). Entry
// (j, i) holds m = (shat_i mod t_j) * 2^64 mod t_j, the factor 2^64 undoing
// the Montgomery reduction that ends each dot product, stored split at bit
// 30 as (m mod 2^30) | (m >> 30) << 32.
inline uint32_t bconv_row(uint32_t L, uint32_t G) { return (L + G - 1) / G * G; }

hipError_t launch_tensor(int word, const void* a, const void* b, void* d, const void* mods, uint32_t L,
                         uint32_t logN, uint32_t batch, hipStream_t s);
// out [batch][K][N] = conv(x [batch][L][N]); with y (ModDown) out = (y - conv) S^-1.
// G from bconv_group; hi_reduce when sum_i (s_i - 1) >= 2^64 (the dot
// product may then reach t_j 2^64 and its high word is reduced first).
hipError_t launch_bconv(const uint64_t* x, const uint64_t* y, uint64_t* out, const BcSrc* src,
                        const uint64_t* mat, const BcDst* dst, uint32_t L, uint32_t K, uint32_t N, uint32_t batch,
                        uint32_t G, uint32_t hi_reduce, hipStream_t s);

}  // namespace nttk
