// Host-side internals shared by the C ABI, the batched executor, the
// autotuner and the server. Not part of the public header.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <mutex>
#include <vector>

#include "launch.hpp"
#include "ntt.h"

struct ScratchSlot {
  void* stream;
  void* ptr;
  size_t bytes;
};

struct ntt_plan {
  uint32_t N = 0, logN = 0, L = 0, flags = 0;
  int word = 64;
  int device = 0;
  std::vector<uint64_t> moduli, psi;
  void* d_tw_fwd = nullptr;
  void* d_tw_inv = nullptr;
  void* d_mod = nullptr;
  void* d_mscale = nullptr;  // inside d_mod's allocation: [L][2] scaled last-stage pairs
  bool auto_variant = true;  // choose per call from the tuning table / defaults
  int path = NTT_PATH_LDS;
  int logN1 = 0;
  int exact = 0;
  // every modulus below 2^60 (64-bit words): the forward kernels keep values in
  // [0, 16q) and skip about half of their reductions (approximate quotient)
  bool wide = false;
  // NTT_DEBUG_CHECK: every call first checks its inputs are canonical
  // (d_flag: one device word for the result)
  bool debug_check = false;
  uint32_t* d_flag = nullptr;
  std::mutex mu;  // guards scratch and the paper-variant tables
  std::vector<ScratchSlot> scratch;
  // tables of the paper's algorithm variants (cyclic plans), built on first use
  void* d_paper = nullptr;  // [L][N/2] forward, [L][N/2] inverse, [L] N^-1
  // tables of the twisted row pass per direction (0 forward, 1 inverse) and
  // split log2(N1): [L][N] twist, then [L][N2] cyclic twiddles. The plan's
  // default split is built at creation for the directions its mask selects,
  // other splits on first use.
  void* d_rowtw[2][10] = {};
  int row_twist = NTT_ROW_TWIST_DEFAULT;  // directions whose four-step row pass is twisted
  bool auto_twist = true;             // until set: the tuning table's row form, if it has one
  int tune_lv_col = 0;                // the autotuner's own override of the column passes' values per thread
  int tune_col_tile = 0;              // and of their columns per tile
};

namespace ntti {

int ilog2(uint32_t x);
// library default variant for (word, logN): path, logN1
void default_variant(int word, int logN, int* path, int* logN1);
// tuned variant for (word, logN, items) if the tuning table has one
// twist: the row-form mask (NTT_ROW_TWIST_*) tuned with it, -1 if none;
// lv_col: log2 of the values per thread of the column passes, 0 = default;
// col_tile: their columns per tile (32), 0 = default
bool tune_lookup(int word, int logN, uint32_t items, int* path, int* logN1, int* exact, int* twist = nullptr,
                 int* lv_col = nullptr, int* col_tile = nullptr);
void tune_store(int word, int logN, uint32_t items, int path, int logN1, int exact, float us, int twist = -1,
                int lv_col = 0, int col_tile = 0);
// load the table named by NTT_TUNE_CACHE once per process (no-op if unset)
void tune_autoload();

// validation shared by plans and batch jobs: 0 or an NTT_ERR_ code
int check_modulus(uint64_t q, uint32_t N, int word);

// With the plan's NTT_DEBUG_CHECK: NTT_ERR_RANGE if a word of the batch *
// L * N words at d is not below its limb's modulus, after synchronizing the
// stream; NTT_OK without the check
int debug_range(const ntt_plan* p, const void* d, uint32_t batch, void* stream);

// twiddle tables of one (word, q, N) on a device, created on first use and
// kept for the life of the process
struct PoolEntry {
  const void* tw_fwd;
  const void* tw_inv;
  const void* mod;
};
int pool_get(int word, uint64_t q, uint32_t logN, PoolEntry* out);
size_t pool_bytes();
// the host copy of those tables (forward [N] pairs, inverse [N] pairs, the
// modulus constants), built and validated on first use and kept for the life
// of the process; pool_table_bytes is its size
struct HostTables {
  const unsigned char* data;  // pinned when a device was present to pin it
  size_t bytes;
};
int pool_host(int word, uint64_t q, uint32_t logN, HostTables* out);
size_t pool_table_bytes(int word, uint32_t logN);

// a prime q < 2^bits with q = 1 mod 2N (the largest one), for tuning runs
uint64_t tuning_prime(uint32_t N, int word);

// ntt_forward with a caller-supplied scratch of scratch_bytes bytes in place
// of the plan's per-stream scratch; allocates nothing and returns
// NTT_ERR_SCRATCH if the call needs more, NTT_ERR_UNSUPPORTED if it would need
// tables the plan has not built
int forward_fixed_scratch(const ntt_plan* p, void* data, uint32_t batch, void* stream, void* scratch,
                          size_t scratch_bytes);

// f(l) for every l < L, spread over up to 16 host threads (table generation)
void for_limbs(uint32_t L, const std::function<void(uint32_t)>& f);

// Every device and pinned-host allocation of the library goes through these.
// For tests of the failure paths, the environment variable NTT_FAIL_ALLOC=k
// makes the k-th allocation after the variable last changed value fail (as
// hipErrorOutOfMemory, *p = nullptr); unset or 0, nothing is forced.
hipError_t dev_malloc(void** p, size_t bytes);
hipError_t host_malloc(void** p, size_t bytes);
template <class T>
hipError_t dev_malloc(T** p, size_t bytes) {
  return dev_malloc(reinterpret_cast<void**>(p), bytes);
}
template <class T>
hipError_t host_malloc(T** p, size_t bytes) {
  return host_malloc(reinterpret_cast<void**>(p), bytes);
}

}  // namespace ntti
