// ntt_forward_noalloc: the forward transform for callers that cannot
// allocate device memory. Its four-step intermediate lives in the fixed array
// below, one copy per GPU, instead of the plan's per-stream scratch.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address on the current GPU comes from hipGetSymbolAddress, looked up
// once per device (with that device current) and kept in g_addr. Only that
// address is ever handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ntt.h"
#include "ntt_internal.hpp"
#include "trace.hpp"

static_assert(NTT_NOALLOC_SCRATCH_BYTES % 256 == 0, "whole 256-byte blocks");

static __device__ __align__(256) uint64_t scratch[NTT_NOALLOC_SCRATCH_BYTES / sizeof(uint64_t)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};  // device address of `scratch` on each device

// the array's address on the current device, looked up on the first call
int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return NTT_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) return NTT_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return NTT_ERR_HIP;
    g_addr[dev] = p;
  }
  *out = g_addr[dev];
  return NTT_OK;
}
}  // namespace

extern "C" int ntt_forward_noalloc(const ntt_plan* plan, void* d_data, uint32_t batch, void* stream) {
  ntti::Range r("ntt_forward_noalloc");
  if (!plan || !d_data || batch == 0) return NTT_ERR_ARG;
  void* s = nullptr;
  const int rc = scratch_address(&s);
  if (rc != NTT_OK) return rc;
  return ntti::forward_fixed_scratch(plan, d_data, batch, stream, s, NTT_NOALLOC_SCRATCH_BYTES);
}
