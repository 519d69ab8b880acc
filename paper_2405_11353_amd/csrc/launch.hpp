// Internal launch interface between the C ABI (host C++) and the kernel
// translation units. Not part of the public header.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nttk {

enum Path { PATH_TINY = 0, PATH_LDS = 1, PATH_TWO = 2 };

// One work item of the batched executor: a single (polynomial, limb) transform
// with its own buffers, twiddle tables and modulus constants.
struct ItemDesc {
  void* data;            // N words: input and output of the transform
  void* scratch;         // N words: four-step intermediate (natural order)
  const void* tw_fwd;    // N twiddle pairs of the item's modulus and length
  const void* tw_inv;
  const void* mod;       // ModInfo64 / ModInfo32 of the item's modulus
  const void* aux;       // copy: source; pointwise: second operand
  uint64_t logN;         // copy / pointwise: log2 of the item's length
  uint64_t pad;
};
// io codes for the four-step kernels in indirect mode
enum { IO_DATA_DATA = 0, IO_DATA_SCRATCH = 1, IO_SCRATCH_DATA = 2 };


struct Launch {
  int word = 64;      // 32 or 64-bit coefficients
  int exact = 0;      // 64-bit: exact Shoup quotient (lazy bound 2q) instead of approx (4q)
  int wide = 0;       // 64-bit approx, every q < 2^60: forward values in [0, 16q)
  int path = PATH_LDS;
  int logN = 0;
  int logN1 = 0;      // PATH_TWO: column length 2^logN1, row length 2^(logN-logN1)
  int natural = 1;    // natural-order spectrum (else bit-reversed)
  void* data = nullptr;
  void* scratch = nullptr;  // PATH_TWO with natural order: items << logN words
  const void* tw = nullptr; // [L][N] twiddle pairs of the direction being run
  const void* mods = nullptr;
  uint32_t L = 0, items = 0, batch = 0;  // items = batch * L
  hipStream_t stream = nullptr;
  int stage_mask = 3;       // PATH_TWO: bit 0 runs the first kernel, bit 1 the second
  int lv_col = 0;           // PATH_TWO, 64-bit: values per thread (log2, 3 or 4) of the column passes; 0 = default
  int col_tile = 0;         // PATH_TWO, 64-bit: columns per column-pass tile (32), 0 = default (16)
  const void* mul_a = nullptr;  // PATH_TWO inverse: if set, transform mul_a * mul_b into data
  const void* mul_b = nullptr;
  // PATH_TWO inverse column pass: [L][2] twiddle pairs that replace table
  // slots 0 and 1 (N^-1 times 2^w, w the word size), set when the row pass's
  // input is a Montgomery product (the fused product paths); else null
  const void* mul_scale = nullptr;
  // PATH_TWO: if set, the row pass is the twisted one (k_row_tw) with these
  // tables of the direction being run: [L][N] twist, [L][N2] cyclic twiddles
  const void* twist = nullptr;
  const void* cyc = nullptr;
};

// Batched executor launch: items are described by a device table of ItemDesc
// (64-bit words, natural order); PATH_LDS or PATH_TWO.
struct BatchLaunch {
  int path = PATH_LDS;
  int logN = 0, logN1 = 0;
  int wide = 0;  // forward only: every item's q < 2^60 (values in [0, 16q))
  const ItemDesc* desc = nullptr;  // device pointer, items entries
  uint32_t items = 0;
  hipStream_t stream = nullptr;
};
hipError_t launch_batch_u64(const BatchLaunch& c, bool forward);
// item-wise copy (data <- aux) and product (data <- data * aux mod q) over
// items of any length up to 2^max_logn
hipError_t launch_ind_copy(const ItemDesc* desc, uint32_t items, uint32_t max_logn, hipStream_t s);
hipError_t launch_ind_pointwise(const ItemDesc* desc, uint32_t items, uint32_t max_logn, hipStream_t s);

// The paper's algorithm variants (cyclic transform, natural order): one
// launch per stage; tables W[l][N/2] of omega^(+-i) and N^-1 per limb.
enum PaperPath { PAPER_DIT = 0, PAPER_DIF = 1, PAPER_PEASE = 2, PAPER_PEASE_NC = 3, PAPER_STOCKHAM = 4 };
struct PaperLaunch {
  int word = 64;
  int path = PAPER_DIT;
  int logN = 0;
  void* data = nullptr;
  void* scratch = nullptr;  // PEASE, PEASE_NC, STOCKHAM: items << logN words
  const void* tw_fwd = nullptr;
  const void* tw_inv = nullptr;
  const void* ninv = nullptr;
  const void* mods = nullptr;
  uint32_t L = 0, items = 0;
  hipStream_t stream = nullptr;
};
hipError_t launch_paper(const PaperLaunch& c, bool forward);

// Each returns hipErrorNotSupported for a shape it has no kernel for.
hipError_t launch_u64(const Launch& c, bool forward);
hipError_t launch_u64w(const Launch& c, bool forward);
hipError_t launch_u64x(const Launch& c, bool forward);
hipError_t launch_u32(const Launch& c, bool forward);
// *flag (device) set to 1 if any of the items * 2^logN words is >= its limb's
// modulus (the caller clears it first)
hipError_t launch_check_range(int word, const void* x, const void* mods, uint32_t L, uint32_t logN,
                              uint32_t items, uint32_t* flag, hipStream_t s);
hipError_t launch_pointwise(int word, const void* a, const void* b, void* out, const void* mods,
                            uint32_t L, uint32_t logN, uint32_t items, hipStream_t s);

// The wide range changes only the forward kernels (both passes of a forward
// transform run in it, the column pass's output feeding the row pass); the
// inverse kernels are the same in either, and run from launch_u64.
inline hipError_t launch_ntt(const Launch& c, bool forward) {
  if (c.word == 32) return launch_u32(c, forward);
  if (c.exact) return launch_u64x(c, forward);
  return c.wide && forward ? launch_u64w(c, forward) : launch_u64(c, forward);
}

// shape support, kept next to the instantiation lists in the .hip files
constexpr int kTwoPassMinLog = 6, kTwoPassMaxLog = 9;
inline int lds_max_logn(int word) { return word == 32 ? 15 : 14; }
inline bool shape_supported(int word, int exact, int path, int logN, int logN1) {
  if (path == PATH_TINY) return !exact && logN >= 1 && logN <= 3;
  if (path == PATH_LDS) return !exact && logN >= 4 && logN <= lds_max_logn(word);
  if (path == PATH_TWO) {
    const int logN2 = logN - logN1;
    return logN1 >= kTwoPassMinLog && logN1 <= kTwoPassMaxLog && logN2 >= kTwoPassMinLog &&
           logN2 <= kTwoPassMaxLog;
  }
  return false;
}

}  // namespace nttk
