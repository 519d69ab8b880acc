// Autotuner: times every kernel variant the library has for a (word, N,
// batch size) on the current GPU and keeps the fastest in a table that plans
// and batches consult; the table persists as JSON keyed by the GPU's arch.
#include <dlfcn.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "ntt_internal.hpp"
#include "params.hpp"
#include "trace.hpp"

namespace ntti {
namespace {
struct TKey {
  int word, logN, items_log2;
  bool operator<(const TKey& o) const {
    return std::tie(word, logN, items_log2) < std::tie(o.word, o.logN, o.items_log2);
  }
};
struct TVal {
  int path, logN1, exact;
  float us;
  int twist = -1;  // row-form mask tuned with the variant, -1: none
  int lv_col = 0;  // column passes' values per thread (log2), 0: default
  int col_tile = 0;  // column passes' columns per tile (32), 0: default
};
std::mutex g_mu;
std::map<TKey, TVal> g_table;
std::once_flag g_autoload;

int items_bucket(uint32_t items) {
  int b = 0;
  while ((2u << b) <= items && b < 24) ++b;
  return b;
}

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}
}  // namespace

int ilog2(uint32_t x) {
  int l = 0;
  while ((1u << l) < x) ++l;
  return l;
}

void default_variant(int word, int logN, int* path, int* logN1) {
  *logN1 = 0;
  if (logN <= 3) {
    *path = NTT_PATH_TINY;
  } else if (logN <= (word == 32 ? 14 : 13)) {
    *path = NTT_PATH_LDS;
  } else {
    *path = NTT_PATH_FOURSTEP;
    *logN1 = logN / 2;
  }
}

bool tune_lookup(int word, int logN, uint32_t items, int* path, int* logN1, int* exact, int* twist, int* lv_col,
                 int* col_tile) {
  std::lock_guard<std::mutex> g(g_mu);
  if (g_table.empty()) return false;
  const int b = items_bucket(items);
  // nearest tuned batch size for this (word, N)
  const TVal* best = nullptr;
  int best_d = 1 << 30;
  for (auto it = g_table.lower_bound(TKey{word, logN, 0}); it != g_table.end(); ++it) {
    if (it->first.word != word || it->first.logN != logN) break;
    const int d = abs(it->first.items_log2 - b);
    if (d < best_d) {
      best_d = d;
      best = &it->second;
    }
  }
  if (!best) return false;
  *path = best->path;
  *logN1 = best->logN1;
  *exact = best->exact;
  if (twist) *twist = best->twist;
  if (lv_col) *lv_col = best->lv_col;
  if (col_tile) *col_tile = best->col_tile;
  return true;
}

void tune_store(int word, int logN, uint32_t items, int path, int logN1, int exact, float us, int twist,
                int lv_col, int col_tile) {
  std::lock_guard<std::mutex> g(g_mu);
  g_table[TKey{word, logN, items_bucket(items)}] = TVal{path, logN1, exact, us, twist, lv_col, col_tile};
}

uint64_t tuning_prime(uint32_t N, int word) {
  const uint64_t step = 2ull * N;
  uint64_t q = (word == 32 ? (1ull << 30) : (1ull << 60)) - 1;
  q = q / step * step + 1;
  if (q >= (word == 32 ? (1ull << 30) : (1ull << 60))) q -= step;
  for (; q > step; q -= step)
    if (nttp::is_prime(q)) return q;
  return 0;
}

// directory of this shared library (for the tuning table shipped next to it)
static std::string library_dir() {
  Dl_info info;
  if (dladdr((void*)&library_dir, &info) && info.dli_fname) {
    std::string f = info.dli_fname;
    const size_t slash = f.rfind('/');
    if (slash != std::string::npos) return f.substr(0, slash);
  }
  return ".";
}

void tune_autoload() {
  std::call_once(g_autoload, [] {
    const char* p = getenv("NTT_TUNE_CACHE");
    if (p) {
      if (*p) (void)ntt_tune_load(p);  // an empty value disables loading
      return;
    }
    const std::string f = library_dir() + "/tune_" + arch_name() + ".json";
    (void)ntt_tune_load(f.c_str());
  });
}

}  // namespace ntti

using namespace ntti;

extern "C" {

int ntt_autotune(uint32_t N, uint32_t flags, uint32_t items, uint32_t reps, ntt_tune_choice* best_out) {
  ntti::Range r("ntt_autotune");
  if (N < 2 || N > (1u << 17) || (N & (N - 1))) return NTT_ERR_N;
  if (items == 0 || reps == 0 || (flags & ~NTT_WORD32)) return NTT_ERR_ARG;
  const int word = (flags & NTT_WORD32) ? 32 : 64;
  const uint64_t q = tuning_prime(N, word);
  if (!q) return NTT_ERR_MODULUS;
  std::vector<uint64_t> moduli(1, q);
  ntt_plan* plan = ntt_plan_create_ex(N, moduli.data(), 1, flags, nullptr);
  if (!plan) return ntt_last_error();
  // the calls rotate over enough copies of the batch that each reads its
  // data from memory, as a stream of real work does, not from the caches
  // (the Infinity Cache alone holds 256 MiB): 512 MiB in all, at most 64
  const size_t bytes = (size_t)items * N * (word / 8);
  const size_t nbuf = std::max<size_t>(1, std::min<size_t>(64, ((size_t)512 << 20) / bytes));
  void* buf = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = NTT_OK;
  if (ntti::dev_malloc(&buf, nbuf * bytes) != hipSuccess) rc = NTT_ERR_NOMEM;
  // zeros are valid canonical inputs; the kernels' timing does not depend on values
  if (rc == NTT_OK && (hipMemset(buf, 0, nbuf * bytes) != hipSuccess ||
                       hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
                       hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    rc = NTT_ERR_HIP;
  uint32_t next = 0;
  auto batch_buf = [&]() { return (void*)((unsigned char*)buf + (next++ % nbuf) * bytes); };
  // candidates: the LDS kernel, and every four-step split with either
  // quotient flavour (64-bit), and 8 or 16 values per thread and 16 or 32
  // columns per tile in the column passes (64-bit), all timed as forward
  // transforms with merged row passes; then, for a four-step winner, the row
  // form of each direction
  struct Cand {
    int path, logN1, exact, lv, tile;
  };
  std::vector<Cand> cands;
  const int lg = ilog2(N);
  if (lg <= 3) cands.push_back({NTT_PATH_TINY, 0, 0, 0, 0});
  if (lg >= 4 && lg <= nttk::lds_max_logn(word)) cands.push_back({NTT_PATH_LDS, 0, 0, 0, 0});
  for (int a = nttk::kTwoPassMinLog; a <= nttk::kTwoPassMaxLog; ++a)
    if (nttk::shape_supported(word, 0, nttk::PATH_TWO, lg, a)) {
      cands.push_back({NTT_PATH_FOURSTEP, a, 0, 0, 0});
      if (word == 64) {
        cands.push_back({NTT_PATH_FOURSTEP, a, 1, 0, 0});
        cands.push_back({NTT_PATH_FOURSTEP, a, 0, 4, 0});
        cands.push_back({NTT_PATH_FOURSTEP, a, 0, 0, 32});
        cands.push_back({NTT_PATH_FOURSTEP, a, 0, 4, 32});
      }
    }
  // one timed configuration: `reps` calls after two warm-up calls
  auto time_us = [&](bool fwd, float* us) {
    bool ok = true;
    for (uint32_t r = 0; r < 2 && ok; ++r) ok = (fwd ? ntt_forward : ntt_inverse)(plan, batch_buf(), items, s) == NTT_OK;
    if (!ok || hipStreamSynchronize(s) != hipSuccess) return false;
    (void)hipEventRecord(e0, s);
    for (uint32_t r = 0; r < reps && ok; ++r)
      ok = (fwd ? ntt_forward : ntt_inverse)(plan, batch_buf(), items, s) == NTT_OK;
    (void)hipEventRecord(e1, s);
    if (!ok || hipEventSynchronize(e1) != hipSuccess) return false;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *us = ms * 1000.f / reps;
    return true;
  };
  Cand best{-1, 0, 0, 0, 0};
  float best_us = 1e30f;
  for (const Cand& c : cands) {
    if (rc != NTT_OK) break;
    if (ntt_plan_set_variant(plan, c.path, c.logN1) != NTT_OK) continue;
    if (c.exact && ntt_plan_set_quotient(plan, 1) != NTT_OK) continue;
    if (ntt_plan_set_row_twist(plan, 0) != NTT_OK) continue;
    plan->tune_lv_col = c.lv;
    plan->tune_col_tile = c.tile;
    float us;
    if (time_us(true, &us) && us < best_us) {
      best_us = us;
      best = c;
    }
  }
  plan->tune_lv_col = 0;
  plan->tune_col_tile = 0;
  int twist = -1;
  if (rc == NTT_OK && best.path == NTT_PATH_FOURSTEP && ntt_plan_set_variant(plan, best.path, best.logN1) == NTT_OK &&
      (!best.exact || ntt_plan_set_quotient(plan, 1) == NTT_OK)) {
    // each direction's row form, at the winning split: merged or twisted.
    // The default form stays unless the other is more than 5% faster: the
    // twisted rows move less memory, which pays when kernels overlap (calls
    // on several streams) and which a call timed alone does not see.
    plan->tune_lv_col = best.lv;
    plan->tune_col_tile = best.tile;
    int mask = NTT_ROW_TWIST_DEFAULT;
    for (int bit : {NTT_ROW_TWIST_FWD, NTT_ROW_TWIST_INV}) {
      float merged, twisted;
      if (ntt_plan_set_row_twist(plan, 0) == NTT_OK && time_us(bit == NTT_ROW_TWIST_FWD, &merged) &&
          ntt_plan_set_row_twist(plan, bit) == NTT_OK && time_us(bit == NTT_ROW_TWIST_FWD, &twisted)) {
        const bool dflt_twisted = (NTT_ROW_TWIST_DEFAULT & bit) != 0;
        const float dflt = dflt_twisted ? twisted : merged, other = dflt_twisted ? merged : twisted;
        if (other < 0.95f * dflt) mask ^= bit;
      }
    }
    twist = mask == NTT_ROW_TWIST_DEFAULT ? -1 : mask;
    plan->tune_lv_col = 0;
    plan->tune_col_tile = 0;
  }
  if (rc == NTT_OK && best.path < 0) rc = NTT_ERR_UNSUPPORTED;
  if (rc == NTT_OK) {
    tune_store(word, lg, items, best.path, best.logN1, best.exact, best_us, twist, best.lv, best.tile);
    if (best_out) {
      best_out->path = best.path;
      best_out->log_n1 = best.logN1;
      best_out->exact = best.exact;
      best_out->us_per_call = best_us;
      best_out->row_twist = twist;
      best_out->lv_col = best.lv;
      best_out->col_tile = best.tile;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  if (buf) (void)hipFree(buf);
  ntt_plan_destroy(plan);
  return rc;
}

int ntt_tune_save(const char* path) {
  if (!path) return NTT_ERR_ARG;
  FILE* f = fopen(path, "w");
  if (!f) return NTT_ERR_ARG;
  std::lock_guard<std::mutex> g(g_mu);
  fprintf(f, "{\"arch\": \"%s\", \"entries\": [", arch_name().c_str());
  bool first = true;
  for (auto& kv : g_table) {
    fprintf(f,
            "%s\n  {\"word\": %d, \"log_n\": %d, \"items_log2\": %d, \"path\": %d, \"log_n1\": %d, "
            "\"exact\": %d, \"us\": %.3f, \"row_twist\": %d, \"lv_col\": %d, \"col_tile\": %d}",
            first ? "" : ",", kv.first.word, kv.first.logN, kv.first.items_log2, kv.second.path, kv.second.logN1,
            kv.second.exact, kv.second.us, kv.second.twist, kv.second.lv_col, kv.second.col_tile);
    first = false;
  }
  fprintf(f, "\n]}\n");
  fclose(f);
  return NTT_OK;
}

// Reads the format ntt_tune_save writes. Entries for another arch are skipped.
int ntt_tune_load(const char* path) {
  if (!path) return NTT_ERR_ARG;
  FILE* f = fopen(path, "r");
  if (!f) return NTT_ERR_ARG;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
  fclose(f);
  const size_t ap = text.find("\"arch\"");
  if (ap == std::string::npos) return NTT_ERR_ARG;
  const size_t colon = text.find(':', ap);
  if (colon == std::string::npos) return NTT_ERR_ARG;
  const size_t q1 = text.find('"', colon + 1);
  if (q1 == std::string::npos) return NTT_ERR_ARG;
  const size_t q2 = text.find('"', q1 + 1);
  if (q2 == std::string::npos) return NTT_ERR_ARG;
  if (text.substr(q1 + 1, q2 - q1 - 1) != arch_name()) return NTT_ERR_STATE;
  auto field = [&](size_t from, size_t to, const char* name, double* v) {
    const std::string key = std::string("\"") + name + "\"";
    const size_t k = text.find(key, from);
    if (k == std::string::npos || k > to) return false;
    const size_t c = text.find(':', k);
    if (c == std::string::npos || c > to) return false;
    char* end = nullptr;
    *v = strtod(text.c_str() + c + 1, &end);
    return end != text.c_str() + c + 1;
  };
  size_t pos = text.find('[', q2);
  int count = 0;
  while (pos != std::string::npos) {
    const size_t b = text.find('{', pos), e = text.find('}', b == std::string::npos ? pos : b);
    if (b == std::string::npos || e == std::string::npos) break;
    double w, lg, il, pa, n1, ex, us;
    // every field present and in range before any conversion to int (a
    // damaged file then loses entries instead of reaching undefined casts)
    auto in = [](double v, double lo, double hi) { return v >= lo && v <= hi; };
    if (field(b, e, "word", &w) && field(b, e, "log_n", &lg) && field(b, e, "items_log2", &il) &&
        field(b, e, "path", &pa) && field(b, e, "log_n1", &n1) && field(b, e, "exact", &ex) &&
        field(b, e, "us", &us) && (w == 32 || w == 64) && in(lg, 1, 17) && in(il, 0, 40) &&
        in(pa, NTT_PATH_TINY, NTT_PATH_FOURSTEP) && in(n1, 0, 9) && in(ex, 0, 1) && in(us, 0, 1e9)) {
      // optional fields of later tables: the row form and the column passes'
      // values per thread and columns per tile (an entry without them keeps
      // the plan's own)
      double tw = -1, lvc = 0, ct = 0;
      const bool has_tw = field(b, e, "row_twist", &tw), has_lv = field(b, e, "lv_col", &lvc),
                 has_ct = field(b, e, "col_tile", &ct);
      if ((has_tw && !in(tw, -1, 3)) || (has_lv && !(lvc == 0 || lvc == 3 || lvc == 4)) ||
          (has_ct && !(ct == 0 || ct == 16 || ct == 32))) {
        pos = e + 1;
        continue;
      }
      std::lock_guard<std::mutex> g(g_mu);
      g_table[TKey{(int)w, (int)lg, (int)il}] =
          TVal{(int)pa, (int)n1, (int)ex, (float)us, (int)tw, (int)lvc, ct == 32 ? 32 : 0};
      ++count;
    }
    pos = e + 1;
  }
  return count > 0 ? NTT_OK : NTT_ERR_ARG;
}

int ntt_tune_clear(void) {
  std::lock_guard<std::mutex> g(g_mu);
  g_table.clear();
  return NTT_OK;
}

}  // extern "C"
