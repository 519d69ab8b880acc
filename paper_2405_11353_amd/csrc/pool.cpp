// Process-wide pool of twiddle tables keyed by (device, word, q, log2 N).
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "ntt_internal.hpp"
#include "params.hpp"

namespace ntti {
namespace {
struct Key {
  int device, word;
  uint64_t q;
  uint32_t logN;
  bool operator<(const Key& o) const {
    return std::tie(device, word, q, logN) < std::tie(o.device, o.word, o.q, o.logN);
  }
};
std::mutex g_mu;
std::map<Key, PoolEntry> g_pool;
size_t g_bytes = 0;
}  // namespace

int pool_get(int word, uint64_t q, uint32_t logN, PoolEntry* out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return NTT_ERR_HIP;
  const Key k{dev, word, q, logN};
  std::lock_guard<std::mutex> g(g_mu);
  auto it = g_pool.find(k);
  if (it != g_pool.end()) {
    *out = it->second;
    return NTT_OK;
  }
  const uint32_t N = 1u << logN;
  // validated once, when the tables are first built
  if (check_modulus(q, N, word) != NTT_OK) return NTT_ERR_MODULUS;
  const uint64_t psi = nttp::default_psi(q, N);
  if (!psi) return NTT_ERR_MODULUS;
  const size_t tb = (size_t)N * nttp::tw_entry_bytes(word), mb = nttp::modinfo_bytes(word);
  std::vector<unsigned char> host(2 * tb + mb);
  nttp::twiddles(q, psi, logN, word, false, host.data());
  nttp::twiddles(q, psi, logN, word, true, host.data() + tb);
  nttp::modinfo(q, word, host.data() + 2 * tb);
  void* d = nullptr;
  if (hipMalloc(&d, host.size()) != hipSuccess) return NTT_ERR_NOMEM;
  if (hipMemcpy(d, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return NTT_ERR_HIP;
  }
  PoolEntry e{d, (const unsigned char*)d + tb, (const unsigned char*)d + 2 * tb};
  g_pool[k] = e;
  g_bytes += host.size();
  *out = e;
  return NTT_OK;
}

size_t pool_bytes() {
  std::lock_guard<std::mutex> g(g_mu);
  return g_bytes;
}

}  // namespace ntti
