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

// Debug check of the canonical-input precondition: *flag becomes nonzero if
// any word of [items][N] is at least its limb's modulus.
template <class M, class W>
__global__ void __launch_bounds__(256)
k_check_range(const W* __restrict__ x, const M* __restrict__ mods, uint32_t L, uint32_t logN, size_t n,
              uint32_t* flag) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
    bad |= x[e] >= (W)mods[(e >> logN) % L].q;
  if (bad) *flag = 1u;
}

hipError_t launch_check_range(int word, const void* x, const void* mods, uint32_t L, uint32_t logN,
                              uint32_t items, uint32_t* flag, hipStream_t s) {
  const size_t n = (size_t)items << logN;
  const size_t want = (n + 255) / 256, cap = 4096;
  const dim3 grid((unsigned)(want < cap ? (want ? want : 1) : cap)), block(256);
  if (word == 32)
    hipLaunchKernelGGL((k_check_range<ModInfo32, uint32_t>), grid, block, 0, s, (const uint32_t*)x,
                       (const ModInfo32*)mods, L, logN, n, flag);
  else
    hipLaunchKernelGGL((k_check_range<ModInfo64, uint64_t>), grid, block, 0, s, (const uint64_t*)x,
                       (const ModInfo64*)mods, L, logN, n, flag);
  return hipGetLastError();
}

}  // namespace nttk
