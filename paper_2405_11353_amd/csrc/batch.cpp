// Batched executor: many polynomials of uneven N and limb count in one
// hipGraph launch. Every (polynomial, limb) is an item with its own buffers,
// twiddle tables (from the process-wide pool) and modulus constants; items
// are bucketed by (N, direction), each bucket runs the variant the tuning
// table (or the default) picks for its size, and the buckets are captured as
// one graph: as parallel branches (the default), or one bucket after another
// (largest first).
#include <algorithm>
#include <map>
#include <new>
#include <vector>

#include "ntt_internal.hpp"
#include "trace.hpp"

namespace {
struct Bucket {
  int logN, op, path, logN1;
  bool wide = true;         // every item's modulus below 2^60 (forward: values in [0, 16q))
  std::vector<nttk::ItemDesc> items;
  size_t desc_off = 0;      // index of the first descriptor in the device table
  void* scratch = nullptr;  // four-step intermediate for all items of the bucket
  hipStream_t branch = nullptr;
  hipEvent_t done = nullptr;
};
}  // namespace

struct ntt_batch {
  int device = 0;
  uint32_t flags = 0;
  std::vector<Bucket> buckets;
  nttk::ItemDesc* d_desc = nullptr;
  uint32_t n_items = 0;
  size_t scratch_bytes = 0;
  hipStream_t capture = nullptr;
  hipEvent_t fork = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int kernels = 0;
};

static void batch_free(ntt_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto& k : b->buckets) {
    if (k.scratch) (void)hipFree(k.scratch);
    if (k.branch) (void)hipStreamDestroy(k.branch);
    if (k.done) (void)hipEventDestroy(k.done);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  if (b->d_desc) (void)hipFree(b->d_desc);
  delete b;
}

static hipError_t launch_bucket(const ntt_batch* b, const Bucket& k, hipStream_t s) {
  nttk::BatchLaunch c;
  c.path = k.path == NTT_PATH_LDS ? nttk::PATH_LDS : nttk::PATH_TWO;
  c.logN = k.logN;
  c.logN1 = k.logN1;
  c.wide = k.wide ? 1 : 0;
  c.desc = b->d_desc + k.desc_off;
  c.items = (uint32_t)k.items.size();
  c.stream = s;
  return nttk::launch_batch_u64(c, k.op == NTT_JOB_FORWARD);
}

static int fail_batch(ntt_batch* b, int code, int* err) {
  batch_free(b);
  *err = code;
  return code;
}

static int build(ntt_batch* b, const ntt_job_desc* jobs, uint32_t n_jobs) {
  int err = NTT_OK;
  std::map<std::pair<int, int>, Bucket> by;
  for (uint32_t j = 0; j < n_jobs; ++j) {
    const ntt_job_desc& J = jobs[j];
    if (!J.d_data || !J.moduli || J.L == 0 || (J.op != NTT_JOB_FORWARD && J.op != NTT_JOB_INVERSE)) return NTT_ERR_ARG;
    if (J.N < 16 || J.N > (1u << 17) || (J.N & (J.N - 1))) return NTT_ERR_N;
    const int lg = ntti::ilog2(J.N);
    Bucket& k = by[{lg, (int)J.op}];
    k.logN = lg;
    k.op = (int)J.op;
    for (uint32_t l = 0; l < J.L; ++l) {
      const uint64_t q = J.moduli[l];
      ntti::PoolEntry e;  // the pool validates (q, N) when it first builds its tables
      if ((err = ntti::pool_get(64, q, (uint32_t)lg, &e)) != NTT_OK) return err;
      k.wide = k.wide && q < (1ull << 60);
      nttk::ItemDesc d{};
      d.data = (uint64_t*)J.d_data + ((size_t)l << lg);
      d.tw_fwd = e.tw_fwd;
      d.tw_inv = e.tw_inv;
      d.mod = e.mod;
      k.items.push_back(d);
    }
  }
  // items sharing a modulus next to each other (row-pass twiddles are reused in L2)
  for (auto& kv : by) {
    auto& v = kv.second.items;
    std::stable_sort(v.begin(), v.end(), [](const nttk::ItemDesc& x, const nttk::ItemDesc& y) { return x.mod < y.mod; });
  }
  // largest buckets first (the graph then ends on the short ones)
  std::vector<Bucket> order;
  for (auto& kv : by) order.push_back(kv.second);
  std::stable_sort(order.begin(), order.end(), [](const Bucket& x, const Bucket& y) {
    return (x.items.size() << x.logN) > (y.items.size() << y.logN);
  });
  size_t off = 0;
  for (auto& ko : order) {
    Bucket k = std::move(ko);
    const uint32_t n = (uint32_t)k.items.size();
    int path, logN1, exact = 0;
    if (!ntti::tune_lookup(64, k.logN, n, &path, &logN1, &exact) || exact ||
        !(path == NTT_PATH_LDS ? nttk::shape_supported(64, 0, nttk::PATH_LDS, k.logN, 0)
                               : path == NTT_PATH_FOURSTEP && nttk::shape_supported(64, 0, nttk::PATH_TWO, k.logN, logN1)))
      ntti::default_variant(64, k.logN, &path, &logN1);
    k.path = path;
    k.logN1 = logN1;
    if (path == NTT_PATH_FOURSTEP) {
      const size_t bytes = ((size_t)n << k.logN) * 8;
      if (ntti::dev_malloc(&k.scratch, bytes) != hipSuccess) return NTT_ERR_NOMEM;
      b->scratch_bytes += bytes;
      for (uint32_t i = 0; i < n; ++i) k.items[i].scratch = (uint64_t*)k.scratch + ((size_t)i << k.logN);
      b->kernels += 2;
    } else {
      b->kernels += 1;
    }
    k.desc_off = off;
    off += n;
    b->buckets.push_back(std::move(k));
  }
  b->n_items = (uint32_t)off;
  std::vector<nttk::ItemDesc> all;
  all.reserve(off);
  for (auto& k : b->buckets) all.insert(all.end(), k.items.begin(), k.items.end());
  if (ntti::dev_malloc(&b->d_desc, all.size() * sizeof(nttk::ItemDesc)) != hipSuccess) return NTT_ERR_NOMEM;
  if (hipMemcpy(b->d_desc, all.data(), all.size() * sizeof(nttk::ItemDesc), hipMemcpyHostToDevice) != hipSuccess)
    return NTT_ERR_HIP;
  if (b->flags & NTT_BATCH_NO_GRAPH) return NTT_OK;

  // one graph: a fork from the capture stream to a branch per bucket, joined
  // back; or with NTT_BATCH_SERIAL every bucket in turn on the capture stream
  if (hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
    return NTT_ERR_HIP;
  if (b->flags & NTT_BATCH_SERIAL) {
    if (hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal) != hipSuccess) return NTT_ERR_HIP;
    hipError_t e = hipSuccess;
    for (auto& k : b->buckets)
      if (e == hipSuccess) e = launch_bucket(b, k, b->capture);
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(b->capture, &g);
    if (e != hipSuccess || ee != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return e == hipErrorNotSupported ? NTT_ERR_UNSUPPORTED : NTT_ERR_HIP;
    }
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) return NTT_ERR_HIP;
    return NTT_OK;
  }
  for (auto& k : b->buckets)
    if (hipStreamCreateWithFlags(&k.branch, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&k.done, hipEventDisableTiming) != hipSuccess)
      return NTT_ERR_HIP;
  if (hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal) != hipSuccess) return NTT_ERR_HIP;
  hipError_t e = hipEventRecord(b->fork, b->capture);
  for (auto& k : b->buckets) {
    if (e == hipSuccess) e = hipStreamWaitEvent(k.branch, b->fork, 0);
    if (e == hipSuccess) e = launch_bucket(b, k, k.branch);
    if (e == hipSuccess) e = hipEventRecord(k.done, k.branch);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->capture, k.done, 0);
  }
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(b->capture, &g);
  if (e != hipSuccess || ee != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return e == hipErrorNotSupported ? NTT_ERR_UNSUPPORTED : NTT_ERR_HIP;
  }
  b->graph = g;
  if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) return NTT_ERR_HIP;
  return NTT_OK;
}

extern "C" {

ntt_batch* ntt_batch_create(const ntt_job_desc* jobs, uint32_t n_jobs, uint32_t flags) {
  if (!jobs || n_jobs == 0 || (flags & ~(NTT_BATCH_NO_GRAPH | NTT_BATCH_BRANCHES | NTT_BATCH_SERIAL)) ||
      ((flags & NTT_BATCH_BRANCHES) && (flags & NTT_BATCH_SERIAL))) {
    ntt_set_last_error(NTT_ERR_ARG);
    return nullptr;
  }
  ntt_batch* b = new (std::nothrow) ntt_batch;
  if (!b) return nullptr;
  b->flags = flags;
  ntti::tune_autoload();
  if (hipGetDevice(&b->device) != hipSuccess) {
    batch_free(b);
    return nullptr;
  }
  const int rc = build(b, jobs, n_jobs);
  if (rc != NTT_OK) {
    int dummy;
    fail_batch(b, rc, &dummy);
    ntt_set_last_error(rc);
    return nullptr;
  }
  return b;
}

int ntt_batch_run(ntt_batch* b, void* stream) {
  ntti::Range r("ntt_batch_run");
  if (!b) return NTT_ERR_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return NTT_ERR_HIP;
  if (dev != b->device) return NTT_ERR_ARG;
  const hipStream_t s = (hipStream_t)stream;
  if (b->exec) return hipGraphLaunch(b->exec, s) == hipSuccess ? NTT_OK : NTT_ERR_HIP;
  for (auto& k : b->buckets)
    if (launch_bucket(b, k, s) != hipSuccess) return NTT_ERR_HIP;
  return NTT_OK;
}

int ntt_batch_get_info(const ntt_batch* b, ntt_batch_info* out) {
  if (!b || !out) return NTT_ERR_ARG;
  out->items = b->n_items;
  out->buckets = (uint32_t)b->buckets.size();
  out->kernels = (uint32_t)b->kernels;
  out->uses_graph = b->exec ? 1u : 0u;
  out->scratch_bytes = b->scratch_bytes;
  out->twiddle_pool_bytes = ntti::pool_bytes();
  return NTT_OK;
}

void ntt_batch_destroy(ntt_batch* b) { batch_free(b); }

}  // extern "C"
