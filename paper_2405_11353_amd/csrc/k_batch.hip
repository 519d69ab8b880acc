// Indirect-mode (descriptor table) kernels for the batched executor:
// 64-bit words, approximate quotient, natural order, forward and inverse.
#include "launch.hpp"
#include "ntt_core.hpp"
#include "polymul.hpp"

namespace nttk {

// ============================================================ indirect helpers
// Gather copy and pointwise product over items of mixed length: item i is
// split into chunks of CHUNK words; grid.x = items * max_chunks.
constexpr uint32_t kIndChunk = 4096;
__global__ void __launch_bounds__(256)
k_ind_copy(const ItemDesc* __restrict__ desc, uint32_t items, uint32_t max_chunks) {
  const uint32_t item = blockIdx.x / max_chunks, chunk = blockIdx.x % max_chunks;
  if (item >= items) return;
  const ItemDesc d = desc[item];
  const uint32_t n = 1u << (uint32_t)d.logN;
  const uint32_t lo = chunk * kIndChunk;
  if (lo >= n) return;
  const uint32_t hi = lo + kIndChunk < n ? lo + kIndChunk : n;
  const uint64_t* src = (const uint64_t*)d.aux;
  uint64_t* dst = (uint64_t*)d.data;
  for (uint32_t e = lo + threadIdx.x; e < hi; e += blockDim.x) dst[e] = src[e];
}
__global__ void __launch_bounds__(256)
k_ind_pointwise(const ItemDesc* __restrict__ desc, uint32_t items, uint32_t max_chunks) {
  const uint32_t item = blockIdx.x / max_chunks, chunk = blockIdx.x % max_chunks;
  if (item >= items) return;
  const ItemDesc d = desc[item];
  const uint32_t n = 1u << (uint32_t)d.logN;
  const uint32_t lo = chunk * kIndChunk;
  if (lo >= n) return;
  const uint32_t hi = lo + kIndChunk < n ? lo + kIndChunk : n;
  const ModInfo64 m = *(const ModInfo64*)d.mod;
  const uint64_t* b = (const uint64_t*)d.aux;
  uint64_t* a = (uint64_t*)d.data;
  for (uint32_t e = lo + threadIdx.x; e < hi; e += blockDim.x) a[e] = mulmod_general(a[e], b[e], m);
}

namespace {

using W = uint64_t;
using M = ModInfo64;
using AN = Arith64<false>;        // narrow range: inverse, and forward items with some q >= 2^60
using AW = Arith64<false, true>;  // wide range: forward items whose moduli are all below 2^60

// values per thread as in the plan kernels (dispatch.inc): 8 in the column
// passes and the inverse row pass, 16 in the forward row pass
constexpr int lv_for(int want, int logn) { return (16 << (logn - want)) <= 1024 ? want : 4; }

template <class A, int LOGN>
hipError_t ind_lds(const BatchLaunch& c, bool fwd) {
  constexpr int T = (1 << LOGN) / 16;
  constexpr int P = T >= 256 ? 1 : 256 / T;
  const dim3 grid((c.items + P - 1) / P), block(P * T);
  if (fwd) hipLaunchKernelGGL((k_lds<A, LOGN, P, true, true, true>), grid, block, 0, c.stream, nullptr, nullptr, nullptr, 1u, c.items, c.desc);
  else hipLaunchKernelGGL((k_lds<A, LOGN, P, false, true, true>), grid, block, 0, c.stream, nullptr, nullptr, nullptr, 1u, c.items, c.desc);
  return hipGetLastError();
}

template <class A, int LOGN1>
hipError_t ind_col(const BatchLaunch& c, bool fwd, int io) {
  constexpr int LV = lv_for(3, LOGN1);
  const uint32_t tiles = (1u << (c.logN - LOGN1)) / 16;
  const dim3 grid(c.items * tiles), block(16 << (LOGN1 - LV));
  if (fwd) hipLaunchKernelGGL((k_col<A, LOGN1, 16, true, true, LV>), grid, block, 0, c.stream, nullptr, nullptr, nullptr, nullptr, 1u, (uint32_t)c.logN, c.items, c.desc, io);
  else hipLaunchKernelGGL((k_col<A, LOGN1, 16, false, true, LV>), grid, block, 0, c.stream, nullptr, nullptr, nullptr, nullptr, 1u, (uint32_t)c.logN, c.items, c.desc, io);
  return hipGetLastError();
}

template <class A, int LOGN2>
hipError_t ind_row(const BatchLaunch& c, bool fwd, int io) {
  const uint32_t tiles = (1u << c.logN1) / 16;
  const uint32_t lg = (uint32_t)c.logN;
  if (fwd) {
    constexpr int LV = 4;
    hipLaunchKernelGGL((k_row<A, LOGN2, true, true, false, true, LV>), dim3(c.items * tiles), dim3(16 << (LOGN2 - LV)), 0,
                       c.stream, nullptr, nullptr, nullptr, nullptr, 1u, lg, c.items, c.items, nullptr, c.desc, io);
  } else {
    constexpr int LV = lv_for(3, LOGN2);
    hipLaunchKernelGGL((k_row<A, LOGN2, false, true, false, true, LV>), dim3(c.items * tiles), dim3(16 << (LOGN2 - LV)), 0,
                       c.stream, nullptr, nullptr, nullptr, nullptr, 1u, lg, c.items, c.items, nullptr, c.desc, io);
  }
  return hipGetLastError();
}

template <class A>
hipError_t col_sw(int lg1, const BatchLaunch& c, bool fwd, int io) {
  switch (lg1) {
    case 6: return ind_col<A, 6>(c, fwd, io);
    case 7: return ind_col<A, 7>(c, fwd, io);
    case 8: return ind_col<A, 8>(c, fwd, io);
    case 9: return ind_col<A, 9>(c, fwd, io);
    default: return hipErrorNotSupported;
  }
}
template <class A>
hipError_t row_sw(int lg2, const BatchLaunch& c, bool fwd, int io) {
  switch (lg2) {
    case 6: return ind_row<A, 6>(c, fwd, io);
    case 7: return ind_row<A, 7>(c, fwd, io);
    case 8: return ind_row<A, 8>(c, fwd, io);
    case 9: return ind_row<A, 9>(c, fwd, io);
    default: return hipErrorNotSupported;
  }
}

template <class A>
hipError_t lds_sw(const BatchLaunch& c, bool fwd) {
  switch (c.logN) {
    case 4: return ind_lds<A, 4>(c, fwd);
    case 5: return ind_lds<A, 5>(c, fwd);
    case 6: return ind_lds<A, 6>(c, fwd);
    case 7: return ind_lds<A, 7>(c, fwd);
    case 8: return ind_lds<A, 8>(c, fwd);
    case 9: return ind_lds<A, 9>(c, fwd);
    case 10: return ind_lds<A, 10>(c, fwd);
    case 11: return ind_lds<A, 11>(c, fwd);
    case 12: return ind_lds<A, 12>(c, fwd);
    case 13: return ind_lds<A, 13>(c, fwd);
    case 14: return ind_lds<A, 14>(c, fwd);
    default: return hipErrorNotSupported;
  }
}

template <class A>
hipError_t run_batch(const BatchLaunch& c, bool fwd) {
  if (c.path == PATH_LDS) return lds_sw<A>(c, fwd);
  if (c.path == PATH_TWO) {
    if (!shape_supported(64, 0, PATH_TWO, c.logN, c.logN1)) return hipErrorNotSupported;
    const int lg2 = c.logN - c.logN1;
    hipError_t e;
    if (fwd) {
      if ((e = col_sw<A>(c.logN1, c, true, IO_DATA_SCRATCH)) != hipSuccess) return e;
      return row_sw<A>(lg2, c, true, IO_SCRATCH_DATA);
    }
    if ((e = row_sw<A>(lg2, c, false, IO_DATA_SCRATCH)) != hipSuccess) return e;
    return col_sw<A>(c.logN1, c, false, IO_SCRATCH_DATA);
  }
  return hipErrorNotSupported;
}

}  // namespace

hipError_t launch_batch_u64(const BatchLaunch& c, bool fwd) {
  if (c.items == 0) return hipSuccess;
  // the wide range changes the forward kernels only (see launch_ntt)
  return c.wide && fwd ? run_batch<AW>(c, true) : run_batch<AN>(c, fwd);
}

// a column pass alone (the server's products feed it to the fused row
// kernel, which takes the narrow range)
hipError_t launch_batch_col_u64(const BatchLaunch& c, bool fwd, int io) {
  if (c.items == 0) return hipSuccess;
  if (c.path != PATH_TWO || c.wide || !shape_supported(64, 0, PATH_TWO, c.logN, c.logN1)) return hipErrorNotSupported;
  return col_sw<AN>(c.logN1, c, fwd, io);
}

hipError_t launch_ind_copy(const ItemDesc* desc, uint32_t items, uint32_t max_logn, hipStream_t s) {
  if (items == 0) return hipSuccess;
  const uint32_t n = 1u << max_logn, chunks = (n + kIndChunk - 1) / kIndChunk;
  hipLaunchKernelGGL(k_ind_copy, dim3(items * chunks), dim3(256), 0, s, desc, items, chunks);
  return hipGetLastError();
}

hipError_t launch_ind_pointwise(const ItemDesc* desc, uint32_t items, uint32_t max_logn, hipStream_t s) {
  if (items == 0) return hipSuccess;
  const uint32_t n = 1u << max_logn, chunks = (n + kIndChunk - 1) / kIndChunk;
  hipLaunchKernelGGL(k_ind_pointwise, dim3(items * chunks), dim3(256), 0, s, desc, items, chunks);
  return hipGetLastError();
}

}  // namespace nttk
