// Process-wide pool of twiddle tables keyed by (device, word, q, log2 N).
#include <string.h>

#include <map>
#include <new>
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
std::mutex g_host_mu;
std::map<Key, HostTables> g_host;  // device field unused (0); kept until exit
}  // namespace

size_t pool_table_bytes(int word, uint32_t logN) {
  return 2 * ((size_t)1 << logN) * nttp::tw_entry_bytes(word) + nttp::modinfo_bytes(word);
}

int pool_host(int word, uint64_t q, uint32_t logN, HostTables* out) {
  const Key k{0, word, q, logN};
  {
    std::lock_guard<std::mutex> g(g_host_mu);
    auto it = g_host.find(k);
    if (it != g_host.end()) {
      *out = it->second;
      return NTT_OK;
    }
  }
  const uint32_t N = 1u << logN;
  // validated once, when the tables are first built
  if (check_modulus(q, N, word) != NTT_OK) return NTT_ERR_MODULUS;
  const uint64_t psi = nttp::default_psi(q, N);
  if (!psi) return NTT_ERR_MODULUS;
  const size_t tb = (size_t)N * nttp::tw_entry_bytes(word);
  std::vector<unsigned char> host(pool_table_bytes(word, logN));
  nttp::twiddles(q, psi, logN, word, false, host.data());
  nttp::twiddles(q, psi, logN, word, true, host.data() + tb);
  nttp::modinfo(q, word, host.data() + 2 * tb);
  std::lock_guard<std::mutex> g(g_host_mu);
  auto it = g_host.find(k);  // a concurrent builder may have won: same contents
  if (it == g_host.end()) {
    // pinned when a device is there, so that uploads from it are asynchronous
    void* p = nullptr;
    if (ntti::host_malloc(&p, host.size()) != hipSuccess) {
      p = new (std::nothrow) unsigned char[host.size()];
      if (!p) return NTT_ERR_NOMEM;
    }
    memcpy(p, host.data(), host.size());
    it = g_host.emplace(k, HostTables{(const unsigned char*)p, host.size()}).first;
  }
  *out = it->second;
  return NTT_OK;
}

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
  HostTables host;
  const int rc = pool_host(word, q, logN, &host);
  if (rc != NTT_OK) return rc;
  const size_t tb = ((size_t)1 << logN) * nttp::tw_entry_bytes(word);
  void* d = nullptr;
  if (ntti::dev_malloc(&d, host.bytes) != hipSuccess) return NTT_ERR_NOMEM;
  if (hipMemcpy(d, host.data, host.bytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return NTT_ERR_HIP;
  }
  PoolEntry e{d, (const unsigned char*)d + tb, (const unsigned char*)d + 2 * tb};
  g_pool[k] = e;
  g_bytes += host.bytes;
  *out = e;
  return NTT_OK;
}

size_t pool_bytes() {
  std::lock_guard<std::mutex> g(g_mu);
  return g_bytes;
}

}  // namespace ntti
