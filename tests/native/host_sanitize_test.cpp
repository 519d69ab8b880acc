// The library's host code (plans' argument checks, table generation, the
// tuning-table loader, the serving loop's scheduler in simulate mode) built
// for the CPU under AddressSanitizer + UndefinedBehaviorSanitizer or
// ThreadSanitizer. No kernel runs: the launchers are stand-ins. Usage:
//   host_sanitize_test all <valid tuning table>   (ASan/UBSan build)
//   host_sanitize_test server                     (TSan build)
// Prints "ok" or the first failed expectation; the sanitizers abort on any
// report.
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <string>
#include <thread>
#include <vector>

#include "ntt.h"
#include "params.hpp"

static int fails = 0;
#define EXPECT(c)                                                  \
  do {                                                             \
    if (!(c)) {                                                    \
      if (fails++ < 5) printf("FAIL line %d: %s\n", __LINE__, #c); \
    }                                                              \
  } while (0)

static uint64_t rng = 0x853C49E6748FEA9Bull;
static uint64_t next() {  // xorshift64*: test-only
  rng ^= rng >> 12;
  rng ^= rng << 25;
  rng ^= rng >> 27;
  return rng * 0x2545F4914F6CDD1Dull;
}

static void params() {
  const uint64_t qs[] = {1152921504606584833ull, 2305843009211596801ull /* 2^61 - 2^21 + 1 */, 998244353ull};
  for (uint64_t q : qs) {
    for (uint32_t logN : {1u, 4u, 10u, 14u}) {
      const uint32_t N = 1u << logN;
      const int word = q < (1ull << 30) ? 32 : 64;
      if (q % (2ull * N) != 1) continue;
      const uint64_t psi = nttp::default_psi(q, N);
      EXPECT(psi != 0 && nttp::powmod(psi, N, q) == q - 1);
      std::vector<unsigned char> tab((size_t)N * nttp::tw_entry_bytes(word) + 64);
      nttp::twiddles(q, psi, logN, word, false, tab.data());
      nttp::twiddles(q, psi, logN, word, true, tab.data());
      if (logN >= 12) {
        std::vector<unsigned char> tw((size_t)N * nttp::tw_entry_bytes(word));
        nttp::twist(q, psi, logN, logN / 2, word, false, false, tw.data());
        nttp::twist(q, psi, logN, logN / 2, word, true, false, tw.data());
        EXPECT(nttp::row_root(q, psi, logN / 2, false) != 0);
      }
      std::vector<unsigned char> mi(nttp::modinfo_bytes(word));
      nttp::modinfo(q, word, mi.data());
    }
    EXPECT(nttp::is_prime(q));
    EXPECT(!nttp::is_prime(q + 2) || nttp::is_prime(q + 2));
  }
}

static std::string read_file(const char* path) {
  std::string s;
  FILE* f = fopen(path, "rb");
  if (!f) return s;
  char b[4096];
  size_t n;
  while ((n = fread(b, 1, sizeof b, f)) > 0) s.append(b, n);
  fclose(f);
  return s;
}
static void write_file(const std::string& path, const std::string& s) {
  FILE* f = fopen(path.c_str(), "wb");
  if (!f) return;
  fwrite(s.data(), 1, s.size(), f);
  fclose(f);
}

static void tune_loader(const char* valid, const char* scratch_path) {
  const std::string good = read_file(valid);
  EXPECT(!good.empty());
  EXPECT(ntt_tune_load(valid) == NTT_OK);
  EXPECT(ntt_tune_save(scratch_path) == NTT_OK);
  int loaded = 0, refused = 0;
  for (int it = 0; it < 600; ++it) {
    std::string v = good;
    const size_t a = next() % v.size(), b = next() % v.size();
    switch (it % 4) {
      case 0: v.resize(a); break;
      case 1:
        for (int k = 0; k < 4; ++k) v[next() % v.size()] = (char)(next() & 0xFF);
        break;
      case 2:
        for (int k = 0; k < 4; ++k) v[next() % v.size()] = "{}[],:\"0123456789-eE.x "[next() % 23];
        break;
      default: v.erase(a < b ? a : b, a < b ? b - a : a - b); break;
    }
    write_file(scratch_path, v);
    ntt_tune_clear();
    if (ntt_tune_load(scratch_path) == NTT_OK) ++loaded;
    else ++refused;
  }
  EXPECT(loaded + refused == 600 && refused > 0);
  EXPECT(ntt_tune_load("/nonexistent/table.json") != NTT_OK);
  ntt_tune_clear();
}

static void plan_arguments() {
  const uint64_t q = 1152921504606584833ull;
  EXPECT(ntt_plan_create(1000, &q, 1) == nullptr && ntt_last_error() == NTT_ERR_N);
  EXPECT(ntt_plan_create(1u << 18, &q, 1) == nullptr && ntt_last_error() == NTT_ERR_N);
  const uint64_t bad = q + 2;
  EXPECT(ntt_plan_create(1024, &bad, 1) == nullptr && ntt_last_error() == NTT_ERR_MODULUS);
  EXPECT(ntt_plan_create(1024, nullptr, 1) == nullptr && ntt_last_error() == NTT_ERR_ARG);
  EXPECT(ntt_plan_create_ex(1024, &q, 1, 0x100, nullptr) == nullptr && ntt_last_error() == NTT_ERR_ARG);
  EXPECT(ntt_forward(nullptr, nullptr, 1, nullptr) == NTT_ERR_ARG);
  ntt_job_desc j{};
  EXPECT(ntt_batch_create(&j, 1, 0) == nullptr);
  EXPECT(ntt_bconv_create(64, nullptr, 1, &q, 1) == nullptr && ntt_last_error() == NTT_ERR_ARG);
  for (int c = 0; c >= -11; --c) EXPECT(strcmp(ntt_strerror(c), "unknown error") != 0);
}

static void server(int threads, int per_thread) {
  // the four largest primes below 2^60 that are 1 mod 2^18
  static const uint64_t P[] = {1152921504606584833ull, 1152921504598720513ull, 1152921504592429057ull,
                               1152921504581419009ull};
  ntt_server_config cfg{};
  cfg.hbm_budget_bytes = 64ull << 20;
  cfg.n_streams = 3;
  cfg.max_batch_items = 64;
  cfg.flags = NTT_SERVER_SIMULATE;
  cfg.simulate_ns_per_item = 500.0;
  ntt_server* s = ntt_server_create(&cfg);
  EXPECT(s != nullptr);
  if (!s) return;
  std::atomic<int> done{0}, timeouts{0};
  std::vector<std::thread> th;
  for (int t = 0; t < threads; ++t)
    th.emplace_back([&, t] {
      uint64_t r = 0x9E3779B97F4A7C15ull * (t + 1);
      for (int i = 0; i < per_thread; ++i) {
        r ^= r << 13;
        r ^= r >> 7;
        r ^= r << 17;
        ntt_request q{};
        q.op = (uint32_t)(r % 3);
        q.N = 1u << (4 + r % 14);
        q.L = 1 + (uint32_t)((r >> 8) % 4);
        q.moduli = P;
        q.d_out = (void*)(uintptr_t)0x10000;
        q.d_a = q.d_b = q.d_out;
        uint64_t ticket = 0;
        const int rc = ntt_server_submit(s, &q, &ticket);
        if (rc != NTT_OK) continue;
        // a zero-time wait either finds the job done (and forgets the
        // ticket) or times out, leaving it to the blocking wait
        int w = i % 5 == 0 ? ntt_server_wait(s, ticket, 0) : NTT_ERR_TIMEOUT;
        if (w == NTT_ERR_TIMEOUT) {
          if (i % 5 == 0) timeouts++;
          w = ntt_server_wait(s, ticket, -1);
        }
        if (w == NTT_OK) done++;
        if (i % 17 == 0) {
          ntt_server_stats st;
          EXPECT(ntt_server_get_stats(s, &st) == NTT_OK);
        }
      }
    });
  for (auto& x : th) x.join();
  EXPECT(done == threads * per_thread);
  ntt_server_stats st;
  EXPECT(ntt_server_get_stats(s, &st) == NTT_OK && st.completed == (uint64_t)done && st.failed == 0);
  EXPECT(ntt_server_reset_stats(s) == NTT_OK);
  // a job larger than the whole budget is refused, not queued
  ntt_request big{};
  big.op = NTT_REQ_POLYMUL;
  big.N = 1u << 17;
  big.L = 4;
  big.moduli = P;
  big.d_out = (void*)(uintptr_t)0x10000;
  big.d_a = big.d_b = big.d_out;
  uint64_t tk = 0;
  cfg.hbm_budget_bytes = 1 << 20;
  ntt_server* small = ntt_server_create(&cfg);
  EXPECT(small && ntt_server_submit(small, &big, &tk) == NTT_ERR_BUDGET);
  EXPECT(ntt_server_wait(small, 12345, 0) == NTT_ERR_STATE);
  ntt_server_destroy(small);
  // destroy drains queued work
  for (int i = 0; i < 50; ++i) {
    ntt_request q{};
    q.op = NTT_REQ_NTT;
    q.N = 1024;
    q.L = 2;
    q.moduli = P;
    q.d_out = (void*)(uintptr_t)0x10000;
    q.d_a = q.d_out;
    EXPECT(ntt_server_submit(s, &q, &tk) == NTT_OK);
  }
  ntt_server_destroy(s);
  cfg.n_streams = 0;
  EXPECT(ntt_server_create(&cfg) == nullptr);
}

int main(int argc, char** argv) {
  const std::string mode = argc > 1 ? argv[1] : "all";
  if (mode == "all") {
    params();
    plan_arguments();
    if (argc > 3) tune_loader(argv[2], argv[3]);
    server(4, 120);
  } else {
    server(6, 150);
  }
  if (fails) return 1;
  printf("ok\n");
  return 0;
}
