// Serving loop: continuous batching of NTT, inverse-NTT and polynomial-product
// requests on device-resident polynomials.
//
// Requests enter a FIFO. A scheduler thread owns K stream slots; whenever a
// slot is free it admits jobs from the head of the queue while their working
// memory (temporary operand copy and four-step scratch) fits in the server's
// HBM arena, packs them into one batch -- a descriptor table uploaded with one
// copy, then one launch per (phase, N) bucket of the indirect-mode kernels --
// and records an event. Jobs that arrive while earlier batches run are
// admitted as soon as a slot and arena space free up, so their work overlaps
// on the device. Completion is detected by polling the slots' events; latency
// is measured from submit to detected completion.
//
// Twiddle tables live in the same arena and count against the same budget:
// each (q, N) a job needs is made resident when the job is admitted (uploaded
// from the process-wide host copy by the first batch that uses it) and stays
// resident after its jobs finish; when an admission needs space, resident
// tables that no queued or running job references are evicted, least
// recently used first. With NTT_SERVER_SIMULATE no device is touched and a
// batch completes after a modelled time (scheduler tests without a GPU); the
// arena accounting, tables included, is the same.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ntt_internal.hpp"
#include "params.hpp"
#include "polymul.hpp"
#include "trace.hpp"

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// one resident (q, N) table set in the arena: forward and inverse twiddles
// and the modulus constants (ntti::pool_table_bytes)
struct Table {
  uint64_t q = 0;
  uint32_t logN = 0;
  size_t off = 0, bytes = 0;
  uint32_t refs = 0;           // queued-and-admitted or running jobs using it
  uint64_t last_use = 0;
  bool resident = false;       // holds arena space
  bool uploaded = false;       // an upload has been enqueued since it became resident
  hipStream_t up_stream = nullptr;
  hipEvent_t ready = nullptr;  // recorded after the upload on up_stream
  ntti::HostTables host{};
};

struct Job {
  uint64_t ticket = 0;
  uint32_t op = 0, N = 0, logN = 0, L = 0;
  bool fourstep = false;
  std::vector<uint64_t> moduli;
  std::vector<Table*> tw;       // per limb (set at admission)
  std::vector<ntti::HostTables> host;  // per limb (real mode)
  size_t table_need = 0;        // bytes of the job's distinct tables
  const uint64_t* a = nullptr;
  const uint64_t* b = nullptr;
  uint64_t* out = nullptr;
  size_t ws_bytes = 0, arena_off = 0;
  double t_submit = 0;
  uint32_t items() const { return op == NTT_REQ_POLYMUL ? 2 * L : L; }
  uint32_t transforms() const { return op == NTT_REQ_POLYMUL ? 3 * L : L; }
};

// first-fit allocator over [0, cap) with coalescing (offsets only)
class Arena {
 public:
  void init(size_t cap) {
    cap_ = cap;
    free_.clear();
    free_[0] = cap;
    used_ = peak_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) {
      *off = 0;
      return true;
    }
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) return;
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t cap() const { return cap_; }

 private:
  std::map<size_t, size_t> free_;
  size_t cap_ = 0, used_ = 0, peak_ = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  nttk::ItemDesc* d_desc = nullptr;
  nttk::ItemDesc* h_desc = nullptr;  // pinned staging
  size_t cap = 0;
  std::vector<Job*> jobs;
  bool busy = false;
  int err = NTT_OK;
  double sim_done_at = 0;
};

// the path a server job of this size uses (fixed per N so that the scratch
// reserved at admission always matches what the kernels need)
bool server_fourstep(uint32_t logN) {
  int path, n1;
  ntti::default_variant(64, (int)logN, &path, &n1);
  return path == NTT_PATH_FOURSTEP;
}

constexpr uint32_t kMaxL = 256;

}  // namespace

struct ntt_server {
  ntt_server_config cfg{};
  bool simulate = false;
  int device = 0;
  void* base = nullptr;  // device arena
  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::deque<Job*> pending;
  std::unordered_map<uint64_t, int> state;  // 1 queued/running, 0 done, < 0 error
  std::vector<Slot> slots;
  std::thread th;
  bool stop = false;
  uint64_t next_ticket = 1;
  Arena arena;
  // resident twiddle tables, keyed by (q, logN); touched by the scheduler
  // thread only (admission, upload, completion)
  std::map<std::pair<uint64_t, uint32_t>, Table> tables;
  uint64_t use_clock = 0;
  size_t table_bytes = 0;
  // statistics since the last reset
  ntt_server_stats st{};
  std::vector<float> lat_us;
  double t0 = 0, busy_since = -1, busy_acc = 0;
  uint32_t inflight = 0;
};

static int launch_batch(ntt_server* s, Slot& slot) {
  ntti::Range r("ntt_server batch");
  if (s->simulate) {
    uint64_t items = 0;
    for (Job* j : slot.jobs) items += j->items();
    slot.sim_done_at = now_s() + std::max(5e-6, s->cfg.simulate_ns_per_item * 1e-9 * (double)items);
    return NTT_OK;
  }
  using nttk::ItemDesc;
  std::vector<ItemDesc> copy, pw;
  std::map<uint32_t, std::vector<ItemDesc>> fwd, inv;
  // four-step products: column passes of a and b into the workspace, the
  // fused row kernel (both forward row passes, the product, the first
  // inverse pass), the inverse column pass into the output
  std::map<uint32_t, std::vector<ItemDesc>> pm_col, pm_row, pm_inv;
  uint32_t max_logn = 0;
  for (Job* j : slot.jobs) {
    const size_t n = (size_t)j->N;
    uint64_t* ws = (uint64_t*)((char*)s->base + j->arena_off);
    uint64_t* btmp = j->op == NTT_REQ_POLYMUL ? ws : nullptr;
    uint64_t* scr = j->op == NTT_REQ_POLYMUL ? ws + j->L * n : ws;
    max_logn = std::max(max_logn, j->logN);
    for (uint32_t l = 0; l < j->L; ++l) {
      ItemDesc d{};
      d.logN = j->logN;
      const char* tb = (const char*)s->base + j->tw[l]->off;
      const size_t half = n * nttp::tw_entry_bytes(64);
      d.tw_fwd = tb;
      d.tw_inv = tb + half;
      d.mod = tb + 2 * half;
      uint64_t* out_l = j->out + l * n;
      if (j->op == NTT_REQ_POLYMUL && j->fourstep) {
        uint64_t* sa = ws + l * n;
        uint64_t* sb = ws + (j->L + l) * n;
        ItemDesc ca = d, cb = d, r = d, v = d;
        ca.data = const_cast<uint64_t*>(j->a + l * n);  // read only (data -> scratch)
        ca.scratch = sa;
        cb.data = const_cast<uint64_t*>(j->b + l * n);
        cb.scratch = sb;
        r.data = sa;
        r.aux = sb;
        v.data = out_l;
        v.scratch = sa;
        pm_col[j->logN].push_back(ca);
        pm_col[j->logN].push_back(cb);
        pm_row[j->logN].push_back(r);
        pm_inv[j->logN].push_back(v);
        continue;
      }
      if (j->a != j->out) {
        ItemDesc c = d;
        c.data = out_l;
        c.aux = j->a + l * n;
        copy.push_back(c);
      }
      ItemDesc t = d;
      t.data = out_l;
      t.scratch = j->fourstep ? scr + l * n : nullptr;
      if (j->op == NTT_REQ_NTT) {
        fwd[j->logN].push_back(t);
      } else if (j->op == NTT_REQ_INTT) {
        inv[j->logN].push_back(t);
      } else {
        ItemDesc c = d;
        c.data = btmp + l * n;
        c.aux = j->b + l * n;
        copy.push_back(c);
        fwd[j->logN].push_back(t);
        ItemDesc tb = d;
        tb.data = btmp + l * n;
        tb.scratch = j->fourstep ? scr + (j->L + l) * n : nullptr;
        fwd[j->logN].push_back(tb);
        ItemDesc p = d;
        p.data = out_l;
        p.aux = btmp + l * n;
        pw.push_back(p);
        inv[j->logN].push_back(t);
      }
    }
  }
  std::vector<ItemDesc> all;
  all.insert(all.end(), copy.begin(), copy.end());
  struct Run {
    bool fwd;
    uint32_t logN;
    size_t off, n;
  };
  auto append = [&all](std::map<uint32_t, std::vector<ItemDesc>>& m, std::vector<Run>& out, bool f) {
    for (auto& kv : m) {
      out.push_back({f, kv.first, all.size(), kv.second.size()});
      all.insert(all.end(), kv.second.begin(), kv.second.end());
    }
  };
  std::vector<Run> pm_col_runs, pm_row_runs, pm_inv_runs;
  append(pm_col, pm_col_runs, true);
  append(pm_row, pm_row_runs, true);
  std::vector<Run> runs;
  for (auto& kv : fwd) {
    runs.push_back({true, kv.first, all.size(), kv.second.size()});
    all.insert(all.end(), kv.second.begin(), kv.second.end());
  }
  const size_t pw_off = all.size();
  all.insert(all.end(), pw.begin(), pw.end());
  for (auto& kv : inv) {
    runs.push_back({false, kv.first, all.size(), kv.second.size()});
    all.insert(all.end(), kv.second.begin(), kv.second.end());
  }
  append(pm_inv, pm_inv_runs, false);
  if (all.size() > slot.cap) return NTT_ERR_ARG;
  hipError_t e = hipSuccess;
  // tables: the first batch that uses a newly resident table uploads it;
  // later batches on other streams wait for that upload
  for (Job* j : slot.jobs)
    for (Table* t : j->tw) {
      if (e != hipSuccess) break;
      if (!t->uploaded) {
        e = hipMemcpyAsync((char*)s->base + t->off, t->host.data, t->bytes, hipMemcpyHostToDevice, slot.stream);
        if (e == hipSuccess && !t->ready) e = hipEventCreateWithFlags(&t->ready, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(t->ready, slot.stream);
        t->uploaded = true;
        t->up_stream = slot.stream;
      } else if (t->up_stream != slot.stream) {
        e = hipStreamWaitEvent(slot.stream, t->ready, 0);
      }
    }
  std::copy(all.begin(), all.end(), slot.h_desc);
  if (e == hipSuccess)
    e = hipMemcpyAsync(slot.d_desc, slot.h_desc, all.size() * sizeof(ItemDesc), hipMemcpyHostToDevice, slot.stream);
  if (e == hipSuccess) e = nttk::launch_ind_copy(slot.d_desc, (uint32_t)copy.size(), max_logn, slot.stream);
  auto col_launch = [&](const Run& r, bool f, int io) {
    nttk::BatchLaunch c;
    int path, n1;
    ntti::default_variant(64, (int)r.logN, &path, &n1);
    c.path = nttk::PATH_TWO;
    c.logN = (int)r.logN;
    c.logN1 = n1;
    c.desc = slot.d_desc + r.off;
    c.items = (uint32_t)r.n;
    c.stream = slot.stream;
    return nttk::launch_batch_col_u64(c, f, io);
  };
  for (const Run& r : pm_col_runs)
    if (e == hipSuccess) e = col_launch(r, true, nttk::IO_DATA_SCRATCH);
  for (const Run& r : pm_row_runs) {
    int path, n1;
    ntti::default_variant(64, (int)r.logN, &path, &n1);
    if (e == hipSuccess) e = nttk::launch_ind_row_polymul(slot.d_desc + r.off, (uint32_t)r.n, (int)r.logN, n1, slot.stream);
  }
  bool pw_done = false;
  for (const Run& r : runs) {
    if (!r.fwd && !pw_done) {
      if (e == hipSuccess) e = nttk::launch_ind_pointwise(slot.d_desc + pw_off, (uint32_t)pw.size(), max_logn, slot.stream);
      pw_done = true;
    }
    nttk::BatchLaunch c;
    int path, n1;
    ntti::default_variant(64, (int)r.logN, &path, &n1);
    c.path = path == NTT_PATH_FOURSTEP ? nttk::PATH_TWO : nttk::PATH_LDS;
    c.logN = (int)r.logN;
    c.logN1 = n1;
    c.desc = slot.d_desc + r.off;
    c.items = (uint32_t)r.n;
    c.stream = slot.stream;
    if (e == hipSuccess) e = nttk::launch_batch_u64(c, r.fwd);
  }
  if (!pw_done && e == hipSuccess)
    e = nttk::launch_ind_pointwise(slot.d_desc + pw_off, (uint32_t)pw.size(), max_logn, slot.stream);
  for (const Run& r : pm_inv_runs)
    if (e == hipSuccess) e = col_launch(r, false, nttk::IO_SCRATCH_DATA);
  if (e == hipSuccess) e = hipEventRecord(slot.done, slot.stream);
  return e == hipSuccess ? NTT_OK : NTT_ERR_HIP;
}

static void finish_slot(ntt_server* s, Slot& slot, double t) {
  for (Job* j : slot.jobs) {
    s->state[j->ticket] = slot.err;
    if (slot.err == NTT_OK) {
      s->st.completed++;
      s->st.ntts += j->transforms();
      s->lat_us.push_back((float)((t - j->t_submit) * 1e6));
    } else {
      s->st.failed++;
    }
    s->arena.release(j->arena_off, j->ws_bytes);
    for (Table* t : j->tw) t->refs--;
    delete j;
  }
  slot.jobs.clear();
  slot.busy = false;
  slot.err = NTT_OK;
  s->inflight--;
  if (s->inflight == 0 && s->busy_since >= 0) {
    s->busy_acc += t - s->busy_since;
    s->busy_since = -1;
  }
}

// Reserves j's working memory, then makes its tables resident, evicting
// resident tables that no admitted job references (least recently used
// first) when the arena is full. The working memory goes first, as the
// largest block; a table of this job already placed is never evicted for the
// next one, so an admission ends. When nothing runs, every table is
// unreferenced and can go, so a job that fits the budget alone (checked at
// submit) is always admitted once the device drains. On failure the working
// memory is released; tables made resident on the way stay, evictable.
static bool admit(ntt_server* s, Job* j) {
  std::vector<Table*> mine(j->L);
  for (uint32_t l = 0; l < j->L; ++l) {
    Table& t = s->tables[{j->moduli[l], j->logN}];
    if (!t.bytes) {
      t.q = j->moduli[l];
      t.logN = j->logN;
      t.bytes = ntti::pool_table_bytes(64, j->logN);
      if (!s->simulate) t.host = j->host[l];
    }
    mine[l] = &t;
  }
  std::vector<Table*> placed;  // this job's tables resident so far
  auto alloc = [&](size_t bytes, size_t* off) {
    while (!s->arena.alloc(bytes, off)) {
      Table* lru = nullptr;
      for (auto& kv : s->tables) {
        Table& t = kv.second;
        if (t.resident && t.refs == 0 && std::find(placed.begin(), placed.end(), &t) == placed.end() &&
            (!lru || t.last_use < lru->last_use))
          lru = &t;
      }
      if (!lru) return false;
      s->arena.release(lru->off, lru->bytes);
      lru->resident = false;
      lru->uploaded = false;
      s->table_bytes -= lru->bytes;
      s->st.table_evictions++;
    }
    return true;
  };
  if (!alloc(j->ws_bytes, &j->arena_off)) return false;
  for (Table* t : mine) {
    if (!t->resident) {
      if (!alloc(t->bytes, &t->off)) {
        s->arena.release(j->arena_off, j->ws_bytes);
        return false;
      }
      t->resident = true;
      t->uploaded = s->simulate;
      s->table_bytes += t->bytes;
      s->st.table_uploads++;
    }
    placed.push_back(t);
  }
  for (Table* t : mine) {
    t->refs++;
    t->last_use = ++s->use_clock;
  }
  j->tw = std::move(mine);
  return true;
}

static void scheduler(ntt_server* s) {
  if (!s->simulate) (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // completions
    bool any_done = false;
    for (Slot& slot : s->slots) {
      if (!slot.busy) continue;
      bool done;
      if (s->simulate) {
        done = now_s() >= slot.sim_done_at;
      } else {
        const hipError_t q = hipEventQuery(slot.done);
        done = q != hipErrorNotReady;
        if (done && q != hipSuccess) slot.err = NTT_ERR_HIP;
      }
      if (done) {
        finish_slot(s, slot, now_s());
        any_done = true;
      }
    }
    if (any_done) s->cv_done.notify_all();
    if (s->stop && s->pending.empty() && s->inflight == 0) break;
    // admission: fill free slots from the head of the queue
    for (Slot& slot : s->slots) {
      if (slot.busy || s->pending.empty()) continue;
      uint64_t items = 0;
      while (!s->pending.empty()) {
        Job* j = s->pending.front();
        if (!slot.jobs.empty() && items + j->items() > s->cfg.max_batch_items) break;
        if (!admit(s, j)) {
          if (slot.jobs.empty()) s->st.admission_stalls++;
          break;
        }
        slot.jobs.push_back(j);
        s->pending.pop_front();
        items += j->items();
      }
      if (slot.jobs.empty()) break;
      slot.busy = true;
      s->inflight++;
      if (s->busy_since < 0) s->busy_since = now_s();
      s->st.batches++;
      s->st.items += items;
      s->st.max_inflight_batches = std::max<uint32_t>(s->st.max_inflight_batches, s->inflight);
      s->st.peak_bytes = std::max<uint64_t>(s->st.peak_bytes, s->arena.used());
      s->st.table_bytes = s->table_bytes;
      lk.unlock();
      const int rc = launch_batch(s, slot);
      lk.lock();
      if (rc != NTT_OK) {
        slot.err = rc;
        if (!s->simulate) (void)hipStreamSynchronize(slot.stream);
        finish_slot(s, slot, now_s());
        s->cv_done.notify_all();
      }
    }
    // while batches run, poll their events in a yield loop (the scheduler owns
    // a core; a timed wait would add tens of microseconds of timer slack to
    // every completion); otherwise sleep until work arrives
    if (s->inflight) {
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
    } else {
      s->cv_sched.wait_for(lk, std::chrono::milliseconds(2), [s] { return s->stop || !s->pending.empty(); });
    }
  }
}

static void server_free(ntt_server* s) {
  if (!s) return;
  if (!s->simulate) {
    for (Slot& sl : s->slots) {
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
      if (sl.done) (void)hipEventDestroy(sl.done);
      if (sl.d_desc) (void)hipFree(sl.d_desc);
      if (sl.h_desc) (void)hipHostFree(sl.h_desc);
    }
    for (auto& kv : s->tables)
      if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
    if (s->base) (void)hipFree(s->base);
  }
  delete s;
}

extern "C" {

ntt_server* ntt_server_create(const ntt_server_config* cfg) {
  if (!cfg || cfg->n_streams == 0 || cfg->n_streams > 64 || cfg->max_batch_items == 0 ||
      cfg->hbm_budget_bytes == 0 || (cfg->flags & ~NTT_SERVER_SIMULATE)) {
    ntt_set_last_error(NTT_ERR_ARG);
    return nullptr;
  }
  ntt_server* s = new (std::nothrow) ntt_server;
  if (!s) {
    ntt_set_last_error(NTT_ERR_NOMEM);
    return nullptr;
  }
  s->cfg = *cfg;
  s->simulate = (cfg->flags & NTT_SERVER_SIMULATE) != 0;
  s->arena.init(cfg->hbm_budget_bytes);
  s->slots.resize(cfg->n_streams);
  const size_t cap = 5 * (size_t)std::max<uint32_t>(cfg->max_batch_items, 2 * kMaxL);
  int rc = NTT_OK;
  if (!s->simulate) {
    ntti::tune_autoload();
    if (hipGetDevice(&s->device) != hipSuccess) rc = NTT_ERR_HIP;
    if (rc == NTT_OK && ntti::dev_malloc(&s->base, cfg->hbm_budget_bytes) != hipSuccess) rc = NTT_ERR_NOMEM;
    for (Slot& sl : s->slots) {
      if (rc != NTT_OK) break;
      sl.cap = cap;
      if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
        rc = NTT_ERR_HIP;
      else if (ntti::dev_malloc(&sl.d_desc, cap * sizeof(nttk::ItemDesc)) != hipSuccess ||
               ntti::host_malloc(&sl.h_desc, cap * sizeof(nttk::ItemDesc)) != hipSuccess)
        rc = NTT_ERR_NOMEM;
    }
  }
  if (rc != NTT_OK) {
    server_free(s);
    ntt_set_last_error(rc);
    return nullptr;
  }
  s->t0 = now_s();
  s->th = std::thread(scheduler, s);
  return s;
}

int ntt_server_submit(ntt_server* s, const ntt_request* r, uint64_t* ticket) {
  if (!s || !r || !ticket) return NTT_ERR_ARG;
  if (r->op > NTT_REQ_POLYMUL || r->L == 0 || r->L > kMaxL || !r->moduli || !r->d_a || !r->d_out ||
      (r->op == NTT_REQ_POLYMUL && !r->d_b))
    return NTT_ERR_ARG;
  if (r->N < 16 || r->N > (1u << 17) || (r->N & (r->N - 1))) return NTT_ERR_N;
  Job* j = new (std::nothrow) Job;
  if (!j) return NTT_ERR_NOMEM;
  j->op = r->op;
  j->N = r->N;
  j->logN = (uint32_t)ntti::ilog2(r->N);
  j->L = r->L;
  j->a = (const uint64_t*)r->d_a;
  j->b = (const uint64_t*)r->d_b;
  j->out = (uint64_t*)r->d_out;
  if (j->op == NTT_REQ_POLYMUL && j->out == j->b && j->out != j->a) std::swap(j->a, j->b);  // a*b = b*a
  j->fourstep = server_fourstep(j->logN);
  const size_t poly = (size_t)j->L * j->N * 8;
  // products: an operand copy (LDS sizes) or the two column-pass outputs
  // (four-step sizes); transforms: the four-step intermediate
  j->ws_bytes = j->op == NTT_REQ_POLYMUL ? poly * (j->fourstep ? 2 : 1) : (j->fourstep ? poly : 0);
  int rc = NTT_OK;
  j->moduli.assign(r->moduli, r->moduli + r->L);
  // simulate mode validates here; otherwise the host copy of the tables is
  // built (and the modulus validated) the first time the process sees (q, N)
  if (s->simulate) {
    for (uint32_t l = 0; l < j->L && rc == NTT_OK; ++l) rc = ntti::check_modulus(r->moduli[l], r->N, 64);
  } else {
    j->host.resize(j->L);
    for (uint32_t l = 0; l < j->L && rc == NTT_OK; ++l) rc = ntti::pool_host(64, r->moduli[l], j->logN, &j->host[l]);
  }
  // the job alone must fit: its working memory and its distinct tables
  std::vector<uint64_t> distinct(j->moduli);
  std::sort(distinct.begin(), distinct.end());
  distinct.erase(std::unique(distinct.begin(), distinct.end()), distinct.end());
  j->table_need = distinct.size() * ntti::pool_table_bytes(64, j->logN);
  const size_t pad = 256 * (distinct.size() + 1);  // the arena's 256-byte granules
  if (rc == NTT_OK && j->ws_bytes + j->table_need + pad > s->cfg.hbm_budget_bytes) rc = NTT_ERR_BUDGET;
  std::lock_guard<std::mutex> g(s->mu);
  if (rc == NTT_OK && s->stop) rc = NTT_ERR_STATE;
  if (rc != NTT_OK) {
    s->st.rejected++;
    delete j;
    return rc;
  }
  j->ticket = s->next_ticket++;
  j->t_submit = now_s();
  *ticket = j->ticket;
  s->state[j->ticket] = 1;
  s->pending.push_back(j);
  s->st.submitted++;
  s->cv_sched.notify_one();
  return NTT_OK;
}

int ntt_server_wait(ntt_server* s, uint64_t ticket, int64_t timeout_us) {
  if (!s) return NTT_ERR_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->state.find(ticket);
  if (it == s->state.end()) return NTT_ERR_STATE;
  auto ready = [&] { return s->state[ticket] != 1; };
  if (timeout_us < 0) s->cv_done.wait(lk, ready);
  else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) return NTT_ERR_TIMEOUT;
  const int rc = s->state[ticket];
  s->state.erase(ticket);
  return rc;
}

int ntt_server_get_stats(ntt_server* s, ntt_server_stats* out) {
  if (!s || !out) return NTT_ERR_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  *out = s->st;
  const double t = now_s();
  out->wall_s = t - s->t0;
  out->busy_s = s->busy_acc + (s->busy_since >= 0 ? t - s->busy_since : 0);
  out->queued = s->pending.size();
  out->table_bytes = s->table_bytes;
  if (!s->lat_us.empty()) {
    std::vector<float> v = s->lat_us;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) { return (double)v[std::min(v.size() - 1, (size_t)(p * (v.size() - 1) + 0.5))]; };
    double sum = 0;
    for (float x : v) sum += x;
    out->p50_us = pct(0.50);
    out->p99_us = pct(0.99);
    out->mean_us = sum / v.size();
    out->max_us = v.back();
  }
  return NTT_OK;
}

int ntt_server_reset_stats(ntt_server* s) {
  if (!s) return NTT_ERR_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  s->st = ntt_server_stats{};
  s->lat_us.clear();
  s->t0 = now_s();
  s->busy_acc = 0;
  s->busy_since = s->inflight ? s->t0 : -1;
  return NTT_OK;
}

void ntt_server_destroy(ntt_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_sched.notify_all();
  if (s->th.joinable()) s->th.join();
  server_free(s);
}

}  // extern "C"
