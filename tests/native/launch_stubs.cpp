// Stand-ins for the kernel launchers of the .hip translation units, so that
// the library's host code can be built alone for the CPU under the
// sanitizers. Each reports that it has no kernel.
#include "he.hpp"
#include "launch.hpp"
#include "polymul.hpp"

namespace nttk {
hipError_t launch_u64(const Launch&, bool) { return hipErrorNotSupported; }
hipError_t launch_u64w(const Launch&, bool) { return hipErrorNotSupported; }
hipError_t launch_u64x(const Launch&, bool) { return hipErrorNotSupported; }
hipError_t launch_u32(const Launch&, bool) { return hipErrorNotSupported; }
hipError_t launch_pointwise(int, const void*, const void*, void*, const void*, uint32_t, uint32_t, uint32_t,
                            hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_check_range(int, const void*, const void*, uint32_t, uint32_t, uint32_t, uint32_t*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_paper(const PaperLaunch&, bool) { return hipErrorNotSupported; }
hipError_t launch_batch_u64(const BatchLaunch&, bool) { return hipErrorNotSupported; }
hipError_t launch_batch_col_u64(const BatchLaunch&, bool, int) { return hipErrorNotSupported; }
hipError_t launch_ind_copy(const ItemDesc*, uint32_t, uint32_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_ind_pointwise(const ItemDesc*, uint32_t, uint32_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_row_polymul(int, int, int, void*, const void*, const void*, const void*, const void*, uint32_t,
                              uint32_t, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_ind_row_polymul(const ItemDesc*, uint32_t, int, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_tensor(int, const void*, const void*, void*, const void*, uint32_t, uint32_t, uint32_t,
                         hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_bconv(const uint64_t*, const uint64_t*, uint64_t*, const BcSrc*, const uint64_t*, const BcDst*,
                        uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, hipStream_t) {
  return hipErrorNotSupported;
}
}  // namespace nttk
