// Fused row pass of the polynomial product (see k_polymul.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nttk {

// For each of `batch` pairs (a, b) of [L][N] polynomials that have been
// through the forward column pass (rows of 2^(logN - logN1) words, row r at
// offset r << (logN - logN1)): forward row transform of a's and b's rows,
// elementwise product, inverse row transform, written over sa in the lazy
// range the inverse column pass accepts.
hipError_t launch_row_polymul(int word, int logN, int logN1, void* sa, const void* sb, const void* tw_fwd,
                              const void* tw_inv, const void* mods, uint32_t L, uint32_t batch, hipStream_t s);

}  // namespace nttk
