// Host check of the library's table generators (params.cpp) against their
// definitions with plain 128-bit arithmetic: every sampled entry's value is
// the stated power of the root (powmod from scratch) and its companion is
// floor(w * 2^word / q) by division. Prints "ok" and the time of the largest
// tables, or the first mismatch.
#include <chrono>
#include <stdint.h>
#include <stdio.h>
#include <vector>

#include "params.hpp"

using u128 = unsigned __int128;

static uint32_t brv(uint32_t x, uint32_t bits) {
  uint32_t r = 0;
  for (uint32_t b = 0; b < bits; ++b) r |= ((x >> b) & 1u) << (bits - 1 - b);
  return r;
}
static uint64_t inv(uint64_t a, uint64_t q) { return nttp::powmod(a, q - 2, q); }

static int fails = 0;
static void expect(bool ok, const char* what, uint64_t q, size_t k) {
  if (!ok && fails++ < 5) printf("mismatch %s q=%llu k=%zu\n", what, (unsigned long long)q, k);
}
static void check_entry(const void* tab, int word, size_t k, uint64_t want, uint64_t q, const char* what) {
  if (word == 32) {
    const uint32_t* o = (const uint32_t*)tab + 2 * k;
    expect(o[0] == want && o[1] == (uint32_t)(((uint64_t)want << 32) / q), what, q, k);
  } else {
    const uint64_t* o = (const uint64_t*)tab + 2 * k;
    expect(o[0] == want && o[1] == (uint64_t)(((u128)want << 64) / q), what, q, k);
  }
}

int main() {
  struct P { uint64_t q; int word; };
  // 60-bit and 61-bit NTT primes (1 mod 2^18) and 30-bit ones (1 mod 2^25)
  const P primes[] = {{1152921504606584833ull, 64}, {1152921504598720513ull, 64},
                      {2305843009211596801ull, 64}, {998244353ull, 32}, {469762049ull, 32}};
  uint64_t seed = 0x9E3779B97F4A7C15ull;
  auto rnd = [&]() { seed ^= seed << 13; seed ^= seed >> 7; seed ^= seed << 17; return seed; };
  for (const P& pr : primes) {
    const uint64_t q = pr.q;
    if (pr.word == 64) {
      // per-limb constants: q, -8q, -q, q^-1, 2^64 mod q and its companion, -2q, -4q (all mod
      // 2^64), and the canonicalisation's reciprocal word
      uint64_t m[9];
      expect(nttp::modinfo_bytes(64) == sizeof m, "modinfo size", q, 0);
      nttp::modinfo(q, 64, m);
      const uint64_t r1 = (uint64_t)(((u128)1 << 64) % q);
      expect(m[0] == q && m[2] + q == 0 && m[3] * q == 1 && m[4] == r1, "modinfo", q, 0);
      expect(m[1] + 8 * q == 0, "modinfo -8q", q, 1);
      expect(m[5] == (uint64_t)(((u128)r1 << 64) / q), "modinfo r1 companion", q, 5);
      expect(m[6] + 2 * q == 0 && m[7] + 4 * q == 0, "modinfo -2q, -4q", q, 6);
      // c q <= 2^(s+32+e) < (c+1) q with c < 2^32; bit length b of q: s = b - 28, e = 26
      const uint64_t c = m[8] & 0xffffffffu, sh = (m[8] >> 32) & 0xff, e = (m[8] >> 40) & 0xff;
      int b = 0;
      while (q >> b) ++b;
      const u128 p2 = (u128)1 << (sh + 32 + e);
      expect((int)sh == b - 28 && e == 26 && (m[8] >> 48) == 0, "modinfo canon shifts", q, 8);
      expect((u128)c * q <= p2 && p2 < (u128)(c + 1) * q, "modinfo canon reciprocal", q, 8);
    }
    for (uint32_t logN = 12; logN <= 16; logN += 2) {
      const uint32_t N = 1u << logN;
      if ((q - 1) % (2ull * N)) continue;
      const size_t eb = nttp::tw_entry_bytes(pr.word);
      for (int cyclic = 0; cyclic < 2; ++cyclic) {
        const uint64_t root = cyclic ? nttp::default_omega(q, N) : nttp::default_psi(q, N);
        const uint64_t order = cyclic ? N : 2ull * N;
        std::vector<unsigned char> f(N * eb), iv(N * eb);
        nttp::twiddles(q, root, logN, pr.word, false, f.data(), cyclic);
        nttp::twiddles(q, root, logN, pr.word, true, iv.data(), cyclic);
        const uint64_t ninv = inv(N, q);
        for (int s = 0; s < 300; ++s) {
          const uint32_t k = 2 + (uint32_t)(rnd() % (N - 2));
          uint32_t st = 0;
          while ((2u << st) <= k) ++st;
          const uint64_t e = cyclic ? (uint64_t)(N >> (st + 1)) * brv(k - (1u << st), st) : brv(k, logN);
          const uint64_t w = nttp::powmod(root, e, q);
          check_entry(f.data(), pr.word, k, w, q, "twiddle");
          check_entry(iv.data(), pr.word, k, inv(w, q), q, "inverse twiddle");
        }
        check_entry(iv.data(), pr.word, 0, ninv, q, "N^-1 slot 0");
        const uint64_t e1 = cyclic ? 0 : brv(1, logN);
        check_entry(iv.data(), pr.word, 1, nttp::mulmod(inv(nttp::powmod(root, e1, q), q), ninv, q), q, "slot 1");
        // the fused product's pair: slots 0 and 1 times 2^word mod q
        std::vector<unsigned char> ms(2 * eb);
        nttp::mont_scale(q, pr.word, iv.data(), ms.data());
        const uint64_t rw = (uint64_t)(((u128)1 << pr.word) % q);
        check_entry(ms.data(), pr.word, 0, nttp::mulmod(ninv, rw, q), q, "scaled slot 0");
        check_entry(ms.data(), pr.word, 1,
                    nttp::mulmod(nttp::mulmod(inv(nttp::powmod(root, e1, q), q), ninv, q), rw, q), q,
                    "scaled slot 1");
        for (uint32_t logN1 = 6; logN1 + 6 <= logN && logN1 <= 9; ++logN1) {
          const uint32_t N1 = 1u << logN1, N2 = N >> logN1;
          std::vector<unsigned char> tf(N * eb), ti(N * eb);
          nttp::twist(q, root, logN, logN1, pr.word, false, cyclic, tf.data());
          nttp::twist(q, root, logN, logN1, pr.word, true, cyclic, ti.data());
          for (int s = 0; s < 300; ++s) {
            const uint32_t r = (uint32_t)(rnd() % N1), j = (uint32_t)(rnd() % N2);
            const uint64_t beta = nttp::powmod(root, cyclic ? brv(r, logN1) : 2ull * brv(r, logN1) + 1, q);
            const uint64_t b = nttp::powmod(beta, j, q);
            check_entry(tf.data(), pr.word, (size_t)r * N2 + j, b, q, "twist");
            check_entry(ti.data(), pr.word, (size_t)r * N2 + j, inv(b, q), q, "inverse twist");
          }
          // the row root has order N2 and beta_r^N2 is the row's defining value
          const uint64_t w2 = nttp::row_root(q, root, logN1, cyclic);
          expect(nttp::powmod(w2, N2, q) == 1 && nttp::powmod(w2, N2 / 2, q) == q - 1, "row root", q, logN1);
          (void)order;
        }
      }
    }
  }
  // time of the largest tables a plan builds per limb: 2^17 points, both directions
  const uint64_t q = 1152921504606584833ull;
  const uint64_t psi = nttp::default_psi(q, 1u << 17);
  std::vector<unsigned char> big((1u << 17) * 16);
  const auto t0 = std::chrono::steady_clock::now();
  for (int d = 0; d < 2; ++d) {
    nttp::twiddles(q, psi, 17, 64, d, big.data());
    nttp::twist(q, psi, 17, 8, 64, d, false, big.data());
  }
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (fails) {
    printf("FAILED %d\n", fails);
    return 1;
  }
  printf("ok %.1f ms per limb for the 2^17 twiddle and twist tables\n", ms);
  return 0;
}
