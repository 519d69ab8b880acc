// C ABI of libntt.so: plans (parameters and resident twiddle tables),
// argument checking, variant dispatch and per-stream scratch.
#include <hip/hip_runtime.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "launch.hpp"
#include "ntt.h"
#include "ntt_internal.hpp"
#include "params.hpp"
#include "polymul.hpp"
#include "trace.hpp"

namespace {
thread_local int g_last_error = NTT_OK;

int fail(int code) {
  g_last_error = code;
  return code;
}
}  // namespace

using ntti::ilog2;

static bool is_paper_path(int path) { return path >= NTT_PATH_PAPER_DIT && path <= NTT_PATH_PAPER_STOCKHAM; }

static bool variant_ok(const ntt_plan* p, int path, int logN1, int exact) {
  using namespace nttk;
  const int lg = (int)p->logN;
  if (is_paper_path(path)) return !exact && (p->flags & NTT_CYCLIC) && !(p->flags & NTT_ORDER_BITREV);
  switch (path) {
    case NTT_PATH_TINY: return shape_supported(p->word, exact, PATH_TINY, lg, 0);
    case NTT_PATH_LDS: return shape_supported(p->word, exact, PATH_LDS, lg, 0);
    case NTT_PATH_FOURSTEP: return shape_supported(p->word, exact, PATH_TWO, lg, logN1);
    default: return false;
  }
}

static void default_variant(ntt_plan* p) {
  ntti::default_variant(p->word, (int)p->logN, &p->path, &p->logN1);
  p->exact = 0;
  p->auto_variant = true;
}

// the variant a call on `items` transforms runs with; twist (the row-form
// mask), lv_col (column passes' values per thread, 0 = default) and col_tile
// (their columns per tile, 0 = default) as tuned with it, or the plan's own
static void select_variant(const ntt_plan* p, uint32_t items, int* path, int* logN1, int* exact,
                           int* twist = nullptr, int* lv_col = nullptr, int* col_tile = nullptr) {
  *path = p->path;
  *logN1 = p->logN1;
  *exact = p->exact;
  int tw = -1, lv = 0, ct = 0;
  if (p->auto_variant) {
    int tp, tn1, tex;
    if (ntti::tune_lookup(p->word, (int)p->logN, items, &tp, &tn1, &tex, &tw, &lv, &ct) &&
        variant_ok(p, tp, tn1, tex)) {
      *path = tp;
      *logN1 = tn1;
      *exact = tex;
    } else {
      tw = -1;
      lv = 0;
      ct = 0;
    }
  }
  if (twist) *twist = (p->auto_twist && tw >= 0) ? tw : p->row_twist;
  if (lv_col) *lv_col = p->tune_lv_col ? p->tune_lv_col : (p->word == 64 ? lv : 0);
  if (col_tile) *col_tile = p->tune_col_tile ? p->tune_col_tile : (p->word == 64 ? ct : 0);
}

namespace ntti {
namespace {
std::mutex g_alloc_mu;
std::string g_alloc_env;  // NTT_FAIL_ALLOC as last seen
long g_alloc_count = 0;   // allocations since it changed
bool forced_failure() {
  const char* e = getenv("NTT_FAIL_ALLOC");
  std::lock_guard<std::mutex> g(g_alloc_mu);
  const std::string v = e ? e : "";
  if (v != g_alloc_env) {
    g_alloc_env = v;
    g_alloc_count = 0;
  }
  const long k = v.empty() ? 0 : atol(v.c_str());
  return k > 0 && ++g_alloc_count == k;
}
}  // namespace
hipError_t dev_malloc(void** p, size_t bytes) {
  if (forced_failure()) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}
hipError_t host_malloc(void** p, size_t bytes) {
  if (forced_failure()) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipHostMalloc(p, bytes, hipHostMallocDefault);
}

void for_limbs(uint32_t L, const std::function<void(uint32_t)>& f) {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const unsigned n = std::min<unsigned>(L, std::min(16u, hw));
  std::atomic<uint32_t> next{0};
  auto work = [&] {
    for (uint32_t l; (l = next.fetch_add(1)) < L;) f(l);
  };
  std::vector<std::thread> th;
  try {
    for (unsigned i = 1; i < n; ++i) th.emplace_back(work);
  } catch (...) {
    // no more threads: the ones started and this one share the rest
  }
  work();
  for (auto& t : th) t.join();
}

int debug_range(const ntt_plan* p, const void* d, uint32_t batch, void* stream) {
  if (!p->debug_check) return NTT_OK;
  const hipStream_t s = (hipStream_t)stream;
  uint32_t bad = 0;
  if (hipMemsetAsync(p->d_flag, 0, sizeof(uint32_t), s) != hipSuccess ||
      nttk::launch_check_range(p->word, d, p->d_mod, p->L, p->logN, batch * p->L, p->d_flag, s) != hipSuccess ||
      hipMemcpyAsync(&bad, p->d_flag, sizeof bad, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return NTT_ERR_HIP;
  return bad ? NTT_ERR_RANGE : NTT_OK;
}

int check_modulus(uint64_t q, uint32_t N, int word) {
  const uint64_t qmax = word == 32 ? (1ull << 30) : (1ull << 61);
  if (q < 3 || q >= qmax || (q - 1) % (2ull * N) || !nttp::is_prime(q)) return NTT_ERR_MODULUS;
  return NTT_OK;
}
}  // namespace ntti

static int row_tables(ntt_plan* p, int logN1, bool fwd, nttk::Launch* c);

// the twisted row-pass tables of the plan's own four-step split, for the
// directions its mask selects (calls that the autotuner sends to another
// split build that split's tables on first use)
static int prepare_row_tables(ntt_plan* p) {
  if (p->path != NTT_PATH_FOURSTEP) return NTT_OK;
  for (int dir = 0; dir < 2; ++dir) {
    if (!(p->row_twist & (dir == 0 ? NTT_ROW_TWIST_FWD : NTT_ROW_TWIST_INV))) continue;
    const int rc = row_tables(p, p->logN1, dir == 0, nullptr);
    if (rc != NTT_OK) return rc;
  }
  return NTT_OK;
}

static void release(ntt_plan* p) {
  if (!p) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(p->device);
  for (auto& s : p->scratch)
    if (s.ptr) (void)hipFree(s.ptr);
  if (p->d_tw_fwd) (void)hipFree(p->d_tw_fwd);
  if (p->d_tw_inv) (void)hipFree(p->d_tw_inv);
  if (p->d_mod) (void)hipFree(p->d_mod);
  if (p->d_paper) (void)hipFree(p->d_paper);
  if (p->d_flag) (void)hipFree(p->d_flag);
  for (auto& dir : p->d_rowtw)
    for (void* t : dir)
      if (t) (void)hipFree(t);
  (void)hipSetDevice(cur);
  delete p;
}

extern "C" {

int ntt_last_error(void) { return g_last_error; }
void ntt_set_last_error(int code) { g_last_error = code; }

const char* ntt_strerror(int code) {
  switch (code) {
    case NTT_OK: return "ok";
    case NTT_ERR_ARG: return "invalid argument";
    case NTT_ERR_N: return "N must be a power of two in [2, 2^17]";
    case NTT_ERR_MODULUS: return "modulus is not prime, 2N does not divide q-1, or q is too large for the word size";
    case NTT_ERR_NOMEM: return "out of memory";
    case NTT_ERR_HIP: return "HIP runtime or kernel launch error";
    case NTT_ERR_BUDGET: return "job larger than the memory budget";
    case NTT_ERR_UNSUPPORTED: return "no kernel for this shape or variant";
    case NTT_ERR_STATE: return "unknown ticket or object shut down";
    case NTT_ERR_TIMEOUT: return "timed out";
    case NTT_ERR_SCRATCH: return "workspace larger than the fixed scratch of the no-allocation entry point";
    case NTT_ERR_RANGE: return "input word not below its modulus (NTT_DEBUG_CHECK)";
    default: return "unknown error";
  }
}

ntt_plan* ntt_plan_create_ex(uint32_t N, const uint64_t* moduli, uint32_t L, uint32_t flags,
                             const uint64_t* psi) {
  g_last_error = NTT_OK;
  if (!moduli || L == 0 || (flags & ~(NTT_WORD32 | NTT_ORDER_BITREV | NTT_CYCLIC | NTT_DEBUG_CHECK))) {
    fail(NTT_ERR_ARG);
    return nullptr;
  }
  if (N < 2 || N > (1u << 17) || (N & (N - 1))) {
    fail(NTT_ERR_N);
    return nullptr;
  }
  const int word = (flags & NTT_WORD32) ? 32 : 64;
  const bool cyclic = (flags & NTT_CYCLIC) != 0;
  std::vector<uint64_t> roots(L);
  for (uint32_t l = 0; l < L; ++l) {
    const uint64_t q = moduli[l];
    // the cyclic transform needs N | q-1; the negacyclic one 2N | q-1
    if (ntti::check_modulus(q, cyclic ? N / 2 : N, word) != NTT_OK) {
      fail(NTT_ERR_MODULUS);
      return nullptr;
    }
    if (psi) {
      // a primitive 2N-th (negacyclic) or N-th (cyclic) root: r^(order/2) = -1
      const uint64_t r = psi[l];
      if (r == 0 || r >= q || nttp::powmod(r, cyclic ? N / 2 : N, q) != q - 1) {
        fail(NTT_ERR_ARG);
        return nullptr;
      }
      roots[l] = r;
    } else {
      roots[l] = cyclic ? nttp::default_omega(q, N) : nttp::default_psi(q, N);
      if (!roots[l]) {
        fail(NTT_ERR_MODULUS);
        return nullptr;
      }
    }
  }
  ntt_plan* p = new (std::nothrow) ntt_plan;
  if (!p) {
    fail(NTT_ERR_NOMEM);
    return nullptr;
  }
  p->N = N;
  p->logN = (uint32_t)ilog2(N);
  p->L = L;
  p->flags = flags;
  p->word = word;
  p->moduli.assign(moduli, moduli + L);
  p->psi = roots;
#ifndef NTT_WIDE_RANGE
#define NTT_WIDE_RANGE 1
#endif
  p->wide = NTT_WIDE_RANGE && word == 64 &&
            std::all_of(p->moduli.begin(), p->moduli.end(), [](uint64_t q) { return q < (1ull << 60); });
  if (hipGetDevice(&p->device) != hipSuccess) {
    release(p);
    fail(NTT_ERR_HIP);
    return nullptr;
  }
  ntti::tune_autoload();
  default_variant(p);

  const size_t tw_bytes = (size_t)N * nttp::tw_entry_bytes(word);
  const size_t mod_bytes = nttp::modinfo_bytes(word);
  // d_mod holds the limbs' constants, then their scaled last-stage pairs
  const size_t pair_bytes = 2 * nttp::tw_entry_bytes(word);
  std::vector<unsigned char> fwd(tw_bytes * L), inv(tw_bytes * L), mod((mod_bytes + pair_bytes) * L);
  ntti::for_limbs(L, [&](uint32_t l) {
    nttp::twiddles(moduli[l], roots[l], p->logN, word, false, fwd.data() + l * tw_bytes, cyclic);
    nttp::twiddles(moduli[l], roots[l], p->logN, word, true, inv.data() + l * tw_bytes, cyclic);
    nttp::modinfo(moduli[l], word, mod.data() + l * mod_bytes);
    nttp::mont_scale(moduli[l], word, inv.data() + l * tw_bytes, mod.data() + L * mod_bytes + l * pair_bytes);
  });
  if (ntti::dev_malloc(&p->d_tw_fwd, fwd.size()) != hipSuccess || ntti::dev_malloc(&p->d_tw_inv, inv.size()) != hipSuccess ||
      ntti::dev_malloc(&p->d_mod, mod.size()) != hipSuccess) {
    release(p);
    fail(NTT_ERR_NOMEM);
    return nullptr;
  }
  p->d_mscale = (unsigned char*)p->d_mod + L * mod_bytes;
  if (hipMemcpy(p->d_tw_fwd, fwd.data(), fwd.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->d_tw_inv, inv.data(), inv.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->d_mod, mod.data(), mod.size(), hipMemcpyHostToDevice) != hipSuccess) {
    release(p);
    fail(NTT_ERR_HIP);
    return nullptr;
  }
  const char* dbg = getenv("NTT_DEBUG_CHECK");
  p->debug_check = (flags & NTT_DEBUG_CHECK) || (dbg && *dbg && strcmp(dbg, "0") != 0);
  if (p->debug_check && ntti::dev_malloc(&p->d_flag, 256) != hipSuccess) {
    release(p);
    fail(NTT_ERR_NOMEM);
    return nullptr;
  }
  const int rc = prepare_row_tables(p);
  if (rc != NTT_OK) {
    release(p);
    fail(rc);
    return nullptr;
  }
  return p;
}

ntt_plan* ntt_plan_create(uint32_t N, const uint64_t* moduli, uint32_t L) {
  return ntt_plan_create_ex(N, moduli, L, 0, nullptr);
}

void ntt_plan_destroy(ntt_plan* plan) { release(plan); }

int ntt_plan_get_psi(const ntt_plan* p, uint64_t* out) {
  if (!p || !out) return NTT_ERR_ARG;
  memcpy(out, p->psi.data(), p->L * sizeof(uint64_t));
  return NTT_OK;
}

int ntt_plan_get_variant(const ntt_plan* p, int* path, int* log_n1) {
  if (!p) return NTT_ERR_ARG;
  if (path) *path = p->path;
  if (log_n1) *log_n1 = p->path == NTT_PATH_FOURSTEP ? p->logN1 : 0;
  return NTT_OK;
}

int ntt_plan_get_variant_for(const ntt_plan* p, uint32_t batch, int* path, int* log_n1, int* exact) {
  if (!p || batch == 0) return NTT_ERR_ARG;
  int pa, n1, ex;
  select_variant(p, batch * p->L, &pa, &n1, &ex);
  if (path) *path = pa;
  if (log_n1) *log_n1 = pa == NTT_PATH_FOURSTEP ? n1 : 0;
  if (exact) *exact = ex;
  return NTT_OK;
}

int ntt_plan_get_col_tile(const ntt_plan* p, uint32_t batch, int* columns) {
  if (!p || batch == 0 || !columns) return NTT_ERR_ARG;
  int pa, n1, ex, tw, lv, ct;
  select_variant(p, batch * p->L, &pa, &n1, &ex, &tw, &lv, &ct);
  *columns = pa != NTT_PATH_FOURSTEP ? 0 : p->word == 32 ? 32 : (ct == 32 ? 32 : 16);
  return NTT_OK;
}

int ntt_plan_get_row_form(const ntt_plan* p, uint32_t batch, int* row_twist, int* log_values) {
  if (!p || batch == 0) return NTT_ERR_ARG;
  int pa, n1, ex, tw, lv;
  select_variant(p, batch * p->L, &pa, &n1, &ex, &tw, &lv);
  if (row_twist) *row_twist = tw;
  if (log_values) *log_values = pa == NTT_PATH_FOURSTEP && p->word == 64 ? (lv ? lv : 3) : 0;
  return NTT_OK;
}

int ntt_plan_set_variant(ntt_plan* p, int path, int log_n1) {
  if (!p) return NTT_ERR_ARG;
  if (path == NTT_PATH_AUTO) {
    default_variant(p);
    return NTT_OK;
  }
  if (!variant_ok(p, path, log_n1, 0)) return NTT_ERR_UNSUPPORTED;
  if (is_paper_path(path) && !(p->N >= 2)) return NTT_ERR_UNSUPPORTED;
  p->path = path;
  p->logN1 = path == NTT_PATH_FOURSTEP ? log_n1 : 0;
  p->exact = 0;
  p->auto_variant = false;
  return prepare_row_tables(p);
}

int ntt_plan_set_quotient(ntt_plan* p, int exact) {
  if (!p || p->word != 64) return NTT_ERR_ARG;
  if (!variant_ok(p, p->path, p->logN1, exact ? 1 : 0)) return NTT_ERR_UNSUPPORTED;
  p->exact = exact ? 1 : 0;
  p->auto_variant = false;
  return NTT_OK;
}

int ntt_plan_set_row_twist(ntt_plan* p, int mask) {
  if (!p || (mask & ~(NTT_ROW_TWIST_FWD | NTT_ROW_TWIST_INV))) return NTT_ERR_ARG;
  p->row_twist = mask;
  p->auto_twist = false;
  return prepare_row_tables(p);
}

size_t ntt_workspace_bytes(const ntt_plan* p, uint32_t batch) {
  if (!p || batch == 0 || (p->flags & NTT_ORDER_BITREV)) return 0;
  int path, n1, ex;
  select_variant(p, batch * p->L, &path, &n1, &ex);
  const bool needs = path == NTT_PATH_FOURSTEP || path == NTT_PATH_PAPER_PEASE || path == NTT_PATH_PAPER_PEASE_NC ||
                     path == NTT_PATH_PAPER_STOCKHAM;
  if (!needs) return 0;
  return ((size_t)batch * p->L << p->logN) * (p->word / 8);
}

}  // extern "C"

// scratch for one stream, grown on demand (the stream is drained before an
// old buffer is released, since kernels queued on it may still use it)
static int get_scratch(ntt_plan* p, void* stream, size_t bytes, void** out) {
  std::lock_guard<std::mutex> g(p->mu);
  for (auto& s : p->scratch) {
    if (s.stream != stream) continue;
    if (s.bytes >= bytes) {
      *out = s.ptr;
      return NTT_OK;
    }
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return NTT_ERR_HIP;
    (void)hipFree(s.ptr);
    s.ptr = nullptr;
    s.bytes = 0;
    if (ntti::dev_malloc(&s.ptr, bytes) != hipSuccess) return NTT_ERR_NOMEM;
    s.bytes = bytes;
    *out = s.ptr;
    return NTT_OK;
  }
  void* ptr = nullptr;
  if (ntti::dev_malloc(&ptr, bytes) != hipSuccess) return NTT_ERR_NOMEM;
  p->scratch.push_back({stream, ptr, bytes});
  *out = ptr;
  return NTT_OK;
}

extern "C" int ntt_pointwise_mul(const ntt_plan* p, const void* a, const void* b, void* c, uint32_t batch,
                                 void* stream);

// tables for the paper's variants: omega^i and omega^-i for i < N/2 (with
// Shoup companions) and N^-1 per limb, built and uploaded on first use
static int paper_tables(ntt_plan* p) {
  std::lock_guard<std::mutex> g(p->mu);
  if (p->d_paper) return NTT_OK;
  const uint32_t half = p->N / 2;
  const size_t eb = nttp::tw_entry_bytes(p->word);
  std::vector<unsigned char> host((2 * (size_t)half + 1) * p->L * eb);
  auto put = [&](size_t slot, uint64_t w, uint64_t q) {
    if (p->word == 32) {
      uint32_t* o = (uint32_t*)(host.data() + slot * eb);
      o[0] = (uint32_t)w;
      o[1] = (uint32_t)(((uint64_t)w << 32) / q);
    } else {
      uint64_t* o = (uint64_t*)(host.data() + slot * eb);
      o[0] = w;
      o[1] = (uint64_t)(((unsigned __int128)w << 64) / q);
    }
  };
  for (uint32_t l = 0; l < p->L; ++l) {
    const uint64_t q = p->moduli[l], w = p->psi[l], wi = nttp::powmod(w, q - 2, q);
    uint64_t a = 1, b = 1;
    for (uint32_t i = 0; i < half; ++i) {
      put((size_t)l * half + i, a, q);
      put((size_t)(p->L + l) * half + i, b, q);
      a = nttp::mulmod(a, w, q);
      b = nttp::mulmod(b, wi, q);
    }
    put(2 * (size_t)p->L * half + l, nttp::powmod(p->N % q, q - 2, q), q);
  }
  void* d = nullptr;
  if (ntti::dev_malloc(&d, host.size()) != hipSuccess) return NTT_ERR_NOMEM;
  if (hipMemcpy(d, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);  // not kept: a later call builds the tables again
    return NTT_ERR_HIP;
  }
  p->d_paper = d;
  return NTT_OK;
}

static int get_scratch(ntt_plan* p, void* stream, size_t bytes, void** out);

// tables of the twisted row pass for one direction and the split N1 =
// 2^logN1, built and uploaded on first use: [L][N] twist, then [L][N2] cyclic
// twiddles. Sets the launch's pointers when c is given.
static int row_tables(ntt_plan* p, int logN1, bool fwd, nttk::Launch* c) {
  if (logN1 < 0 || logN1 >= (int)(sizeof p->d_rowtw[0] / sizeof p->d_rowtw[0][0])) return NTT_ERR_UNSUPPORTED;
  const uint32_t N = p->N, logN2 = p->logN - (uint32_t)logN1, N2 = 1u << logN2, L = p->L;
  const size_t eb = nttp::tw_entry_bytes(p->word);
  const size_t twist_bytes = (size_t)N * eb, cyc_bytes = (size_t)N2 * eb;
  void*& slot = p->d_rowtw[fwd ? 0 : 1][logN1];
  {
    std::lock_guard<std::mutex> g(p->mu);
    if (!slot) {
      const bool cyclic = (p->flags & NTT_CYCLIC) != 0;
      std::vector<unsigned char> host(L * (twist_bytes + cyc_bytes));
      unsigned char* tt = host.data();
      unsigned char* ct = tt + L * twist_bytes;
      ntti::for_limbs(L, [&](uint32_t l) {
        const uint64_t q = p->moduli[l], root = p->psi[l];
        nttp::twist(q, root, p->logN, (uint32_t)logN1, p->word, !fwd, cyclic, tt + l * twist_bytes);
        const uint64_t w2 = nttp::row_root(q, root, (uint32_t)logN1, cyclic);
        nttp::twiddles(q, w2, logN2, p->word, !fwd, ct + l * cyc_bytes, true);
      });
      void* d = nullptr;
      if (ntti::dev_malloc(&d, host.size()) != hipSuccess) return NTT_ERR_NOMEM;
      if (hipMemcpy(d, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return NTT_ERR_HIP;
      }
      slot = d;
    }
  }
  if (c) {
    c->twist = slot;
    c->cyc = (const unsigned char*)slot + L * twist_bytes;
  }
  return NTT_OK;
}

static int run_paper(ntt_plan* p, void* data, uint32_t batch, void* stream, bool fwd, int path) {
  int rc = paper_tables(p);
  if (rc != NTT_OK) return rc;
  nttk::PaperLaunch c;
  c.word = p->word;
  c.path = path - NTT_PATH_PAPER_DIT;
  c.logN = (int)p->logN;
  c.data = data;
  const size_t eb = nttp::tw_entry_bytes(p->word), half = p->N / 2;
  c.tw_fwd = p->d_paper;
  c.tw_inv = (const unsigned char*)p->d_paper + (size_t)p->L * half * eb;
  c.ninv = (const unsigned char*)p->d_paper + 2 * (size_t)p->L * half * eb;
  c.mods = p->d_mod;
  c.L = p->L;
  c.items = batch * p->L;
  c.stream = (hipStream_t)stream;
  if (path != NTT_PATH_PAPER_DIT && path != NTT_PATH_PAPER_DIF) {
    rc = get_scratch(p, stream, ((size_t)c.items << p->logN) * (p->word / 8), &c.scratch);
    if (rc != NTT_OK) return rc;
  }
  const hipError_t e = nttk::launch_paper(c, fwd);
  return e == hipSuccess ? NTT_OK : NTT_ERR_HIP;
}

static int check_common(const ntt_plan* p, uint32_t batch) {
  if (!p || batch == 0) return NTT_ERR_ARG;
  if ((uint64_t)batch * p->L > 0xFFFFFFFFull / 64) return NTT_ERR_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return NTT_ERR_HIP;
  if (dev != p->device) return NTT_ERR_ARG;
  return NTT_OK;
}

// fixed_scratch: the caller's scratch of fixed_bytes bytes instead of the
// plan's, and nothing allocated: a call that would need a device allocation
// (a larger scratch, row tables not built yet, the paper variants' tables)
// is refused instead
static int run_ntt(const ntt_plan* pc, void* data, uint32_t batch, void* stream, bool fwd, int stage_mask = 3,
                   void* fixed_scratch = nullptr, size_t fixed_bytes = 0) {
  int rc = check_common(pc, batch);
  if (rc != NTT_OK) return rc;
  if (!data) return NTT_ERR_ARG;
  // the input of a whole transform, or of its first kernel, is canonical
  if ((stage_mask & 1) && (rc = ntti::debug_range(pc, data, batch, stream)) != NTT_OK) return rc;
  ntt_plan* p = const_cast<ntt_plan*>(pc);
  int path, logN1, exact, twist_mask, lv_col, col_tile;
  select_variant(p, batch * p->L, &path, &logN1, &exact, &twist_mask, &lv_col, &col_tile);
  if (is_paper_path(path)) {
    if (stage_mask != 3 || fixed_scratch) return NTT_ERR_UNSUPPORTED;
    return run_paper(p, data, batch, stream, fwd, path);
  }
  nttk::Launch c;
  c.word = p->word;
  c.exact = exact;
  c.wide = p->wide && !exact;
  c.path = path == NTT_PATH_TINY ? nttk::PATH_TINY : path == NTT_PATH_LDS ? nttk::PATH_LDS : nttk::PATH_TWO;
  c.logN = (int)p->logN;
  c.logN1 = logN1;
  c.natural = (p->flags & NTT_ORDER_BITREV) ? 0 : 1;
  c.data = data;
  c.tw = fwd ? p->d_tw_fwd : p->d_tw_inv;
  c.mods = p->d_mod;
  c.L = p->L;
  c.batch = batch;
  c.items = batch * p->L;
  c.stream = (hipStream_t)stream;
  c.stage_mask = stage_mask;
  c.lv_col = lv_col;
  c.col_tile = col_tile;
  if (stage_mask != 3 && c.path != nttk::PATH_TWO) return NTT_ERR_UNSUPPORTED;
  bool twisted = c.path == nttk::PATH_TWO && (twist_mask & (fwd ? NTT_ROW_TWIST_FWD : NTT_ROW_TWIST_INV));
  if (fixed_scratch) {
    if (c.path == nttk::PATH_TWO && c.natural) {
      if (ntt_workspace_bytes(p, batch) > fixed_bytes) return NTT_ERR_SCRATCH;
      c.scratch = fixed_scratch;
    }
    if (twisted) {
      // without the split's twisted tables, the merged row pass (the same
      // transform) instead of building them
      std::lock_guard<std::mutex> g(p->mu);
      if (!p->d_rowtw[fwd ? 0 : 1][logN1]) twisted = false;
    }
  } else if (c.path == nttk::PATH_TWO && c.natural) {
    rc = get_scratch(p, stream, ntt_workspace_bytes(p, batch), &c.scratch);
    if (rc != NTT_OK) return rc;
  }
  // tables that exist are only looked up (row_tables allocates only when a
  // split's tables are missing, which the fixed-scratch form has ruled out)
  if (twisted && (rc = row_tables(p, logN1, fwd, &c)) != NTT_OK) return rc;
  const hipError_t e = nttk::launch_ntt(c, fwd);
  if (e == hipErrorNotSupported) return NTT_ERR_UNSUPPORTED;
  return e == hipSuccess ? NTT_OK : NTT_ERR_HIP;
}

extern "C" {

int ntt_forward(const ntt_plan* p, void* d, uint32_t batch, void* stream) {
  ntti::Range r("ntt_forward");
  return run_ntt(p, d, batch, stream, true);
}
int ntt_inverse(const ntt_plan* p, void* d, uint32_t batch, void* stream) {
  ntti::Range r("ntt_inverse");
  return run_ntt(p, d, batch, stream, false);
}

int ntt_forward_stage(const ntt_plan* p, void* d, uint32_t batch, int stage, void* stream) {
  ntti::Range r("ntt_forward_stage");
  if (stage != 0 && stage != 1) return NTT_ERR_ARG;
  return run_ntt(p, d, batch, stream, true, 1 << stage);
}
int ntt_inverse_stage(const ntt_plan* p, void* d, uint32_t batch, int stage, void* stream) {
  ntti::Range r("ntt_inverse_stage");
  if (stage != 0 && stage != 1) return NTT_ERR_ARG;
  return run_ntt(p, d, batch, stream, false, 1 << stage);
}

static int run_mul_inverse(const ntt_plan* pc, const void* a, const void* b, void* c, uint32_t batch,
                           void* stream, int stage_mask);

int ntt_pointwise_mul_inverse(const ntt_plan* pc, const void* a, const void* b, void* c, uint32_t batch,
                              void* stream) {
  ntti::Range r("ntt_pointwise_mul_inverse");
  return run_mul_inverse(pc, a, b, c, batch, stream, 3);
}

int ntt_pointwise_mul_inverse_stage(const ntt_plan* pc, const void* a, const void* b, void* c, uint32_t batch,
                                    int stage, void* stream) {
  ntti::Range r("ntt_pointwise_mul_inverse_stage");
  if (stage != 0 && stage != 1) return NTT_ERR_ARG;
  return run_mul_inverse(pc, a, b, c, batch, stream, 1 << stage);
}

}  // extern "C"

int ntti::forward_fixed_scratch(const ntt_plan* p, void* data, uint32_t batch, void* stream, void* scratch,
                                size_t scratch_bytes) {
  if (!scratch) return NTT_ERR_ARG;
  return run_ntt(p, data, batch, stream, true, 3, scratch, scratch_bytes);
}

static int run_mul_inverse(const ntt_plan* pc, const void* a, const void* b, void* c, uint32_t batch,
                           void* stream, int stage_mask) {
  int rc = check_common(pc, batch);
  if (rc != NTT_OK) return rc;
  if (!a || !b || !c) return NTT_ERR_ARG;
  if ((stage_mask & 1) && ((rc = ntti::debug_range(pc, a, batch, stream)) != NTT_OK ||
                           (rc = ntti::debug_range(pc, b, batch, stream)) != NTT_OK))
    return rc;
  ntt_plan* p = const_cast<ntt_plan*>(pc);
  int path, logN1, exact, twist_mask, lv_col, col_tile;
  select_variant(p, batch * p->L, &path, &logN1, &exact, &twist_mask, &lv_col, &col_tile);
  if (path != NTT_PATH_FOURSTEP) {
    if (stage_mask != 3) return NTT_ERR_UNSUPPORTED;
    // no fused kernel for this shape: the two steps, still on the device
    rc = ntt_pointwise_mul(p, a, b, c, batch, stream);
    return rc != NTT_OK ? rc : run_ntt(p, c, batch, stream, false);
  }
  nttk::Launch L;
  L.word = p->word;
  L.exact = exact;
  L.path = nttk::PATH_TWO;
  L.logN = (int)p->logN;
  L.logN1 = logN1;
  L.natural = (p->flags & NTT_ORDER_BITREV) ? 0 : 1;
  L.data = c;
  L.mul_a = a;
  L.mul_b = b;
  L.mul_scale = p->d_mscale;
  L.tw = p->d_tw_inv;
  L.mods = p->d_mod;
  L.L = p->L;
  L.batch = batch;
  L.items = batch * p->L;
  L.stream = (hipStream_t)stream;
  L.stage_mask = stage_mask;
  L.lv_col = lv_col;
  L.col_tile = col_tile;
  if (L.natural) {
    rc = get_scratch(p, stream, ntt_workspace_bytes(p, batch), &L.scratch);
    if (rc != NTT_OK) return rc;
  }
  if ((twist_mask & NTT_ROW_TWIST_INV) && (rc = row_tables(p, logN1, false, &L)) != NTT_OK) return rc;
  const hipError_t e = nttk::launch_ntt(L, false);
  if (e == hipErrorNotSupported) return NTT_ERR_UNSUPPORTED;
  return e == hipSuccess ? NTT_OK : NTT_ERR_HIP;
}

extern "C" {

int ntt_pointwise_mul(const ntt_plan* p, const void* a, const void* b, void* c, uint32_t batch, void* stream) {
  ntti::Range r("ntt_pointwise_mul");
  int rc = check_common(p, batch);
  if (rc != NTT_OK) return rc;
  if (!a || !b || !c) return NTT_ERR_ARG;
  if ((rc = ntti::debug_range(p, a, batch, stream)) != NTT_OK || (rc = ntti::debug_range(p, b, batch, stream)) != NTT_OK)
    return rc;
  const hipError_t e = nttk::launch_pointwise(p->word, a, b, c, p->d_mod, p->L, p->logN, batch * p->L,
                                              (hipStream_t)stream);
  return e == hipSuccess ? NTT_OK : NTT_ERR_HIP;
}

}  // extern "C"

static int run_polymul(const ntt_plan* pc, const void* a, const void* b, void* c, uint32_t batch, void* stream) {
  int rc = check_common(pc, batch);
  if (rc != NTT_OK) return rc;
  if (!a || !b || !c) return NTT_ERR_ARG;
  if ((rc = ntti::debug_range(pc, a, batch, stream)) != NTT_OK || (rc = ntti::debug_range(pc, b, batch, stream)) != NTT_OK)
    return rc;
  ntt_plan* p = const_cast<ntt_plan*>(pc);
  int path, logN1, exact;
  select_variant(p, 2 * batch * p->L, &path, &logN1, &exact);
  if (is_paper_path(path)) ntti::default_variant(p->word, (int)p->logN, &path, &logN1);
  const size_t bytes = (((size_t)batch * p->L) << p->logN) * (p->word / 8);
  void* ws = nullptr;
  rc = get_scratch(p, stream, 2 * bytes, &ws);
  if (rc != NTT_OK) return rc;
  void* sa = ws;
  void* sb = (unsigned char*)ws + bytes;
  const hipStream_t s = (hipStream_t)stream;
  nttk::Launch L;
  L.word = p->word;
  L.exact = 0;  // one quotient flavour for every pass, so the lazy ranges agree
  L.wide = 0;   // and the narrow range: the fused row kernel reads the column passes' output
  L.logN = (int)p->logN;
  L.logN1 = logN1;
  L.natural = 1;
  L.mods = p->d_mod;
  L.L = p->L;
  L.batch = batch;
  L.items = batch * p->L;
  L.stream = s;
  hipError_t e;
  if (path == NTT_PATH_FOURSTEP) {
    // column passes of a and b into the workspace, the fused row kernel, and
    // the inverse column pass into c
    L.path = nttk::PATH_TWO;
    L.tw = p->d_tw_fwd;
    L.stage_mask = 1;
    L.data = const_cast<void*>(a);
    L.scratch = sa;
    if ((const unsigned char*)b == (const unsigned char*)a + bytes) {
      // b follows a: one column-pass launch over both
      L.batch = 2 * batch;
      L.items = 2 * batch * p->L;
      e = nttk::launch_ntt(L, true);
      L.batch = batch;
      L.items = batch * p->L;
      if (e != hipSuccess) return e == hipErrorNotSupported ? NTT_ERR_UNSUPPORTED : NTT_ERR_HIP;
    } else {
      if ((e = nttk::launch_ntt(L, true)) != hipSuccess) return e == hipErrorNotSupported ? NTT_ERR_UNSUPPORTED : NTT_ERR_HIP;
      L.data = const_cast<void*>(b);
      L.scratch = sb;
      if ((e = nttk::launch_ntt(L, true)) != hipSuccess) return NTT_ERR_HIP;
    }
    if ((e = nttk::launch_row_polymul(p->word, (int)p->logN, logN1, sa, sb, p->d_tw_fwd, p->d_tw_inv, p->d_mod,
                                      p->L, batch, s)) != hipSuccess)
      return e == hipErrorNotSupported ? NTT_ERR_UNSUPPORTED : NTT_ERR_HIP;
    L.tw = p->d_tw_inv;
    L.mul_scale = p->d_mscale;  // the fused row kernel's products are Montgomery products
    L.stage_mask = 2;
    L.data = c;
    L.scratch = sa;
    return nttk::launch_ntt(L, false) == hipSuccess ? NTT_OK : NTT_ERR_HIP;
  }
  // LDS-resident shapes: the operands are copied into the workspace and
  // transformed in place; the product goes to c, which is transformed back
  if (hipMemcpyAsync(sa, a, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(sb, b, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return NTT_ERR_HIP;
  L.path = path == NTT_PATH_TINY ? nttk::PATH_TINY : nttk::PATH_LDS;
  L.stage_mask = 3;
  L.tw = p->d_tw_fwd;
  L.data = sa;
  if ((e = nttk::launch_ntt(L, true)) != hipSuccess) return e == hipErrorNotSupported ? NTT_ERR_UNSUPPORTED : NTT_ERR_HIP;
  L.data = sb;
  if (nttk::launch_ntt(L, true) != hipSuccess) return NTT_ERR_HIP;
  if (nttk::launch_pointwise(p->word, sa, sb, c, p->d_mod, p->L, p->logN, batch * p->L, s) != hipSuccess)
    return NTT_ERR_HIP;
  L.tw = p->d_tw_inv;
  L.data = c;
  return nttk::launch_ntt(L, false) == hipSuccess ? NTT_OK : NTT_ERR_HIP;
}

extern "C" int ntt_polymul(const ntt_plan* p, const void* a, const void* b, void* c, uint32_t batch, void* stream) {
  ntti::Range r("ntt_polymul");
  return run_polymul(p, a, b, c, batch, stream);
}
