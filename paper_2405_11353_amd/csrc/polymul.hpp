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

struct ItemDesc;
struct BatchLaunch;
// Indirect mode (64-bit words): the fused row kernel over `items` descriptors
// (data: a's column-pass output, overwritten with the product's first
// inverse pass; aux: b's column-pass output), all of length 2^logN with the
// split 2^logN1 x 2^(logN - logN1).
hipError_t launch_ind_row_polymul(const ItemDesc* desc, uint32_t items, int logN, int logN1, hipStream_t s);
// Indirect mode: one column pass (forward or inverse) over c.items
// descriptors, reading and writing as `io` says (IO_DATA_SCRATCH: data ->
// scratch; IO_SCRATCH_DATA: scratch -> data).
hipError_t launch_batch_col_u64(const BatchLaunch& c, bool forward, int io);

}  // namespace nttk
