// Pointwise product kernels (64- and 32-bit words).
#include "launch.hpp"
#include "ntt_core.hpp"

namespace nttk {

hipError_t launch_pointwise(int word, const void* a, const void* b, void* out, const void* mods,
                            uint32_t L, uint32_t logN, uint32_t items, hipStream_t s) {
  const size_t n_pairs = ((size_t)items << logN) / 2;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const size_t want = (n_pairs + 255) / 256;
  const size_t cap = (size_t)cus * 16;
  const dim3 grid((unsigned)(want < cap ? (want ? want : 1) : cap)), block(256);
  if (word == 32)
    hipLaunchKernelGGL((k_pointwise<ModInfo32, uint32_t>), grid, block, 0, s, (const uint32_t*)a,
                       (const uint32_t*)b, (uint32_t*)out, (const ModInfo32*)mods, L, logN, n_pairs);
  else
    hipLaunchKernelGGL((k_pointwise<ModInfo64, uint64_t>), grid, block, 0, s, (const uint64_t*)a,
                       (const uint64_t*)b, (uint64_t*)out, (const ModInfo64*)mods, L, logN, n_pairs);
  return hipGetLastError();
}

}  // namespace nttk
