// Indirect-mode (descriptor table) kernels for the batched executor:
// 64-bit words, approximate quotient, natural order, forward and inverse.
#include "launch.hpp"
#include "ntt_core.hpp"

namespace nttk {
namespace {

using A = Arith64<false>;
using W = A::word;
using TW = A::tw_t;
using M = ModInfo64;

template <int LOGN>
hipError_t ind_lds(const BatchLaunch& c, bool fwd) {
  constexpr int T = (1 << LOGN) / 16;
  constexpr int P = T >= 256 ? 1 : 256 / T;
  const dim3 grid((c.items + P - 1) / P), block(P * T);
  if (fwd) hipLaunchKernelGGL((k_lds<A, LOGN, P, true, true, true>), grid, block, 0, c.stream, nullptr, nullptr, nullptr, 1u, c.items, c.desc);
  else hipLaunchKernelGGL((k_lds<A, LOGN, P, false, true, true>), grid, block, 0, c.stream, nullptr, nullptr, nullptr, 1u, c.items, c.desc);
  return hipGetLastError();
}

template <int LOGN1>
hipError_t ind_col(const BatchLaunch& c, bool fwd, int io) {
  const uint32_t tiles = (1u << (c.logN - LOGN1)) / 16;
  const dim3 grid(c.items * tiles), block(16 << (LOGN1 - 4));
  if (fwd) hipLaunchKernelGGL((k_col<A, LOGN1, 16, true, true>), grid, block, 0, c.stream, nullptr, nullptr, nullptr, nullptr, 1u, (uint32_t)c.logN, c.items, c.desc, io);
  else hipLaunchKernelGGL((k_col<A, LOGN1, 16, false, true>), grid, block, 0, c.stream, nullptr, nullptr, nullptr, nullptr, 1u, (uint32_t)c.logN, c.items, c.desc, io);
  return hipGetLastError();
}

template <int LOGN2>
hipError_t ind_row(const BatchLaunch& c, bool fwd, int io) {
  const uint32_t tiles = (1u << c.logN1) / 16;
  const dim3 grid(c.items * tiles), block(16 << (LOGN2 - 4));
  const uint32_t lg = (uint32_t)c.logN;
  if (fwd) hipLaunchKernelGGL((k_row<A, LOGN2, true, true, false, true>), grid, block, 0, c.stream, nullptr, nullptr, nullptr, nullptr, 1u, lg, c.items, c.items, nullptr, c.desc, io);
  else hipLaunchKernelGGL((k_row<A, LOGN2, false, true, false, true>), grid, block, 0, c.stream, nullptr, nullptr, nullptr, nullptr, 1u, lg, c.items, c.items, nullptr, c.desc, io);
  return hipGetLastError();
}

hipError_t col_sw(int lg1, const BatchLaunch& c, bool fwd, int io) {
  switch (lg1) {
    case 6: return ind_col<6>(c, fwd, io);
    case 7: return ind_col<7>(c, fwd, io);
    case 8: return ind_col<8>(c, fwd, io);
    case 9: return ind_col<9>(c, fwd, io);
    default: return hipErrorNotSupported;
  }
}
hipError_t row_sw(int lg2, const BatchLaunch& c, bool fwd, int io) {
  switch (lg2) {
    case 6: return ind_row<6>(c, fwd, io);
    case 7: return ind_row<7>(c, fwd, io);
    case 8: return ind_row<8>(c, fwd, io);
    case 9: return ind_row<9>(c, fwd, io);
    default: return hipErrorNotSupported;
  }
}

}  // namespace

hipError_t launch_batch_u64(const BatchLaunch& c, bool fwd) {
  if (c.items == 0) return hipSuccess;
  if (c.path == PATH_LDS) {
    switch (c.logN) {
      case 4: return ind_lds<4>(c, fwd);
      case 5: return ind_lds<5>(c, fwd);
      case 6: return ind_lds<6>(c, fwd);
      case 7: return ind_lds<7>(c, fwd);
      case 8: return ind_lds<8>(c, fwd);
      case 9: return ind_lds<9>(c, fwd);
      case 10: return ind_lds<10>(c, fwd);
      case 11: return ind_lds<11>(c, fwd);
      case 12: return ind_lds<12>(c, fwd);
      case 13: return ind_lds<13>(c, fwd);
      case 14: return ind_lds<14>(c, fwd);
      default: return hipErrorNotSupported;
    }
  }
  if (c.path == PATH_TWO) {
    if (!shape_supported(64, 0, PATH_TWO, c.logN, c.logN1)) return hipErrorNotSupported;
    const int lg2 = c.logN - c.logN1;
    hipError_t e;
    if (fwd) {
      if ((e = col_sw(c.logN1, c, true, IO_DATA_SCRATCH)) != hipSuccess) return e;
      return row_sw(lg2, c, true, IO_SCRATCH_DATA);
    }
    if ((e = row_sw(lg2, c, false, IO_DATA_SCRATCH)) != hipSuccess) return e;
    return col_sw(c.logN1, c, false, IO_SCRATCH_DATA);
  }
  return hipErrorNotSupported;
}

}  // namespace nttk
