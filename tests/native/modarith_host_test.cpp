// Host unit test of the GPU library's modular arithmetic (modarith.hpp, built
// for the CPU) against exact 128-bit arithmetic: the Shoup quotient estimates,
// the lazy-range invariants of the butterflies (also the unit-twiddle ones of
// the cyclic row transform), canonicalisation and the general products. Prints "ok <checks>" or the first failure; exit code 0/1.
#include <stdint.h>
#include <stdio.h>

#include "modarith.hpp"

using namespace nttk;
typedef unsigned __int128 u128;

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t rnd() {  // xorshift64*: test-only generator
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return rng_state * 0x2545F4914F6CDD1Dull;
}
static long checks = 0;
#define CHECK(c, ...)                                            \
  do {                                                           \
    ++checks;                                                    \
    if (!(c)) {                                                  \
      printf("FAIL line %d: ", __LINE__);                        \
      printf(__VA_ARGS__);                                       \
      printf("\n");                                              \
      return 1;                                                  \
    }                                                            \
  } while (0)

static uint64_t mulm(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }

static int test64(uint64_t q) {
  const uint64_t nq = 0 - q;
  uint64_t inv = q;
  for (int i = 0; i < 6; ++i) inv *= 2 - q * inv;
  ModInfo64 m{};
  m.q = q;
  m.nq = nq;
  m.qinv = inv;
  m.r1 = (uint64_t)(((u128)1 << 64) % q);
  m.r1p = (uint64_t)(((u128)m.r1 << 64) / q);
  m.n2q = 0 - 2 * q;
  m.n4q = 0 - 4 * q;
  Arith64<false> A;
  A.load(m);
  Arith64<true> X;
  X.load(m);
  CHECK(A.L == 4 * q && X.L == 2 * q, "lazy bounds");
  const uint64_t ys_edge[] = {0, 1, 2, q - 1, q, 2 * q - 1, 4 * q - 1, 8 * q - 1, (1ull << 32) - 1, 1ull << 32,
                              (1ull << 32) + 1, ~0ull, ~0ull - 1, 1ull << 63, (1ull << 63) - 1};
  const uint64_t ws_edge[] = {0, 1, 2, q - 1, q - 2, q / 2, (1ull << 32) - 1, 1ull << 32, q / 3};
  for (int it = 0; it < 300000; ++it) {
    const uint64_t y = it < 15 * 9 ? ys_edge[it / 9] : (it & 1 ? rnd() : rnd() % (8 * q));
    const uint64_t w = it < 15 * 9 ? ws_edge[it % 9] % q : rnd() % q;  // twiddles are residues
    const uint64_t wp = (uint64_t)(((u128)w << 64) / q);
    const Tw64 t{w, wp};
    const uint64_t Qt = (uint64_t)(((u128)y * wp) >> 64);
    const uint64_t Qa = shoup_q_approx(y, wp), Qe = shoup_q_exact(y, wp);
    CHECK(Qe == Qt, "exact quotient y=%llu w=%llu", (unsigned long long)y, (unsigned long long)w);
    CHECK(Qa <= Qt && Qt - Qa <= 2, "approx quotient off by %llu", (unsigned long long)(Qt - Qa));
    const uint64_t ra = A.mul(y, t), re = X.mul(y, t);
    const uint64_t want = mulm(y % q, w, q);
    CHECK(ra < 4 * q && ra % q == want, "approx product range/value");
    CHECK(re < 2 * q && re % q == want, "exact product range/value");
    // butterflies: forward inputs anywhere in [0, 2L), inverse in [0, L)
    const uint64_t x8 = rnd() % (8 * q), y8 = rnd() % (8 * q);
    uint64_t a0 = x8, b0 = y8;
    A.ct(a0, b0, t);
    CHECK(a0 < 8 * q && b0 < 8 * q, "ct range");
    CHECK(a0 % q == (x8 % q + mulm(y8 % q, w, q)) % q, "ct sum");
    CHECK(b0 % q == (x8 % q + q - mulm(y8 % q, w, q)) % q, "ct difference");
    const uint64_t x4 = rnd() % (4 * q), y4 = rnd() % (4 * q);
    a0 = x4;
    b0 = y4;
    A.gs(a0, b0, t);
    CHECK(a0 < 4 * q && b0 < 4 * q, "gs range");
    CHECK(a0 % q == (x4 % q + y4 % q) % q, "gs sum");
    CHECK(b0 % q == mulm((x4 % q + q - y4 % q) % q, w, q), "gs difference");
    const uint64_t x4e = rnd() % (4 * q), y4e = rnd() % (4 * q);
    a0 = x4e;
    b0 = y4e;
    X.ct(a0, b0, t);
    CHECK(a0 < 4 * q && b0 < 4 * q, "exact ct range");
    // unit-twiddle butterflies (group 0 of a cyclic stage): the ranges of
    // ct / gs, with y in place of w y, for both lazy bounds
    for (int fl = 0; fl < 2; ++fl) {
      const uint64_t Lz = fl ? 2 * q : 4 * q;
      uint64_t x1 = rnd() % (2 * Lz), y1 = rnd() % (2 * Lz);
      const uint64_t xs1 = x1 % q, ys1 = y1 % q;
      if (fl) X.ct1(x1, y1); else A.ct1(x1, y1);
      CHECK(x1 < 2 * Lz && y1 < 2 * Lz && x1 % q == (xs1 + ys1) % q && y1 % q == (xs1 + q - ys1) % q, "ct1");
      uint64_t x2 = rnd() % Lz, y2 = rnd() % Lz;
      const uint64_t xs2 = x2 % q, ys2 = y2 % q;
      if (fl) X.gs1(x2, y2); else A.gs1(x2, y2);
      CHECK(x2 < Lz && y2 < Lz && x2 % q == (xs2 + ys2) % q && y2 % q == (xs2 + q - ys2) % q, "gs1");
    }
    CHECK(A.canon_fwd(x8) == x8 % q && A.canon_inv(x4) == x4 % q, "canonical (approx)");
    CHECK(X.canon_fwd(x4e) == x4e % q && X.canon_inv(x4e % (2 * q)) == (x4e % (2 * q)) % q, "canonical (exact)");
    // general product
    const uint64_t u = rnd() % q, v = it < 9 ? ws_edge[it] % q : rnd() % q;
    CHECK(mulmod_general(u, v, m) == mulm(u, v, q), "general product");
    // Montgomery product: x y 2^-64, for x y < q 2^64 (here x lazy below 8q)
    const uint64_t u8 = it < 9 ? 8 * q - 1 - it : rnd() % (8 * q);
    const uint64_t mt = mulmod_mont(u8, v, m);
    CHECK(mt < q && mulm(mt, m.r1, q) == mulm(u8 % q, v, q), "Montgomery product");
    CHECK(mulmod_general(u8, v, m) == mulm(u8 % q, v, q), "general product, lazy first operand");
  }
  return 0;
}

// the wide range (q < 2^60, forward values in [0, 16q)): a reducing CT
// butterfly takes x anywhere below 16q and leaves both outputs below 12q; a
// skipping one needs x below 12q and leaves them below 16q. Then whole
// chains of stages under the two reduction patterns, from inputs at the top
// of their ranges, against the 128-bit value of each output.
// the canonicalisation's reciprocal word, from its definition: b = bit
// length of q, (s, e) = (b - 28, 26) for b >= 28 else (0, b - 1),
// c = floor(2^(s + 32 + e) / q)
static uint64_t canon_word(uint64_t q) {
  int b = 0;
  while (b < 64 && (q >> b)) ++b;
  const int s = b >= 28 ? b - 28 : 0, e = b >= 28 ? 26 : b - 1;
  const u128 c = ((u128)1 << (s + 32 + e)) / q;
  if (c >> 32) return 0;  // fails the checks below
  return (uint64_t)c | ((uint64_t)s << 32) | ((uint64_t)e << 40);
}

// the wide range's canonicalisation alone, for moduli of every size class
// around the estimate's switch at 28 bits: x below 16q (the wide range) and
// up to 2^(b+4) (the estimate's own limit)
static int test_canon(uint64_t q) {
  ModInfo64 m{};
  m.q = q;
  m.nq = 0 - q;
  m.n8q = 0 - 8 * q;
  m.cf = canon_word(q);
  Arith64<false, true> W;
  W.load(m);
  int b = 0;
  while (q >> b) ++b;
  const uint64_t top = b + 4 >= 64 ? ~0ull : (1ull << (b + 4)) - 1;
  for (int it = 0; it < 100000; ++it) {
    const uint64_t x = it == 0 ? 16 * q - 1 : it == 1 ? top : it & 1 ? rnd() % (16 * q) : rnd() % top;
    CHECK(W.canon_fwd(x) == x % q, "canonical q=%llu x=%llu", (unsigned long long)q, (unsigned long long)x);
  }
  return 0;
}

static int test_wide(uint64_t q) {
  ModInfo64 m{};
  m.q = q;
  m.nq = 0 - q;
  m.n2q = 0 - 2 * q;
  m.n4q = 0 - 4 * q;
  m.n8q = 0 - 8 * q;
  m.cf = canon_word(q);
  Arith64<false, true> W;
  W.load(m);
  // canonicalisation at every multiple of q in the range and its neighbours
  for (uint64_t k = 0; k <= 16; ++k) {
    for (int d = -2; d <= 2; ++d) {
      const uint64_t x = k * q + (uint64_t)(int64_t)d;
      if ((k == 0 && d < 0) || (k == 16 && d >= 0)) continue;
      CHECK(W.canon_fwd(x) == x % q, "wide canonical at %llu q %+d", (unsigned long long)k, d);
    }
  }
  for (int it = 0; it < 200000; ++it) {
    const uint64_t w = rnd() % q;
    const Tw64 t{w, (uint64_t)(((u128)w << 64) / q)};
    const uint64_t y = it & 1 ? rnd() : rnd() % (16 * q);
    const uint64_t x16 = it < 4 ? 16 * q - 1 - it : rnd() % (16 * q);
    const uint64_t x12 = it < 4 ? 12 * q - 1 - it : rnd() % (12 * q);
    const uint64_t T = mulm(y % q, w, q);
    uint64_t a = x16, b = y;
    W.ct<true>(a, b, t);
    CHECK(a < 12 * q && b < 12 * q, "wide reducing ct range");
    CHECK(a % q == (x16 % q + T) % q && b % q == (x16 % q + q - T) % q, "wide reducing ct value");
    a = x12;
    b = y;
    W.ct<false>(a, b, t);
    CHECK(a < 16 * q && b < 16 * q, "wide skipping ct range");
    CHECK(a % q == (x12 % q + T) % q && b % q == (x12 % q + q - T) % q, "wide skipping ct value");
    const uint64_t y16 = rnd() % (16 * q);
    a = x16;
    b = y16;
    W.ct1<true>(a, b);
    CHECK(a < 12 * q && b < 12 * q && a % q == (x16 % q + y16 % q) % q && b % q == (x16 % q + q - y16 % q) % q,
          "wide reducing ct1");
    a = x12;
    b = y16;
    W.ct1<false>(a, b);
    CHECK(a < 16 * q && b < 16 * q && a % q == (x12 % q + y16 % q) % q && b % q == (x12 % q + q - y16 % q) % q,
          "wide skipping ct1");
    CHECK(W.canon_fwd(x16) == x16 % q, "wide canonical");
  }
  // chains: stage j of a pass reduces iff reduces_x(pattern, j); every value
  // meets the precondition of the butterfly it enters (checked inside by the
  // ranges above: here the bound before each stage and the final values)
  for (int pat = RP_FRESH; pat <= RP_LAZY; ++pat) {
    for (int trial = 0; trial < 2000; ++trial) {
      uint64_t v[2], ref[2];
      for (int i = 0; i < 2; ++i) {
        v[i] = pat == RP_FRESH ? (trial < 2 ? 4 * q - 1 : rnd() % (4 * q)) : (trial < 2 ? 16 * q - 1 : rnd() % (16 * q));
        ref[i] = v[i] % q;
      }
      for (int j = 0; j < 20; ++j) {
        const uint64_t w = rnd() % q;
        const Tw64 t{w, (uint64_t)(((u128)w << 64) / q)};
        const bool red = reduces_x(pat, j);
        CHECK(v[0] < 16 * q && v[1] < 16 * q, "chain bound before stage %d", j);
        CHECK(red || v[0] < 12 * q, "chain: stage %d skips with x >= 12q", j);
        if (red) W.ct<true>(v[0], v[1], t);
        else W.ct<false>(v[0], v[1], t);
        const uint64_t T = mulm(ref[1], w, q);
        const uint64_t r0 = (ref[0] + T) % q, r1 = (ref[0] + q - T) % q;
        ref[0] = r0;
        ref[1] = r1;
        CHECK(v[0] % q == ref[0] && v[1] % q == ref[1], "chain value at stage %d", j);
        // the next stage's x is either output: alternate which one continues
        if (trial & 1) {
          const uint64_t s = v[0];
          v[0] = v[1];
          v[1] = s;
          const uint64_t sr = ref[0];
          ref[0] = ref[1];
          ref[1] = sr;
        }
      }
      CHECK(W.canon_fwd(v[0]) == ref[0] && W.canon_fwd(v[1]) == ref[1], "chain canonical");
    }
  }
  return 0;
}

static int test32(uint32_t q) {
  uint32_t inv = q;
  for (int i = 0; i < 5; ++i) inv *= 2u - q * inv;
  ModInfo32 m{};
  m.q = q;
  m.qinv = inv;
  m.r1 = (uint32_t)((1ull << 32) % q);
  m.r1p = (uint32_t)(((uint64_t)m.r1 << 32) / q);
  Arith32 A;
  A.load(m);
  for (int it = 0; it < 300000; ++it) {
    const uint32_t y = (uint32_t)rnd(), w = (uint32_t)(rnd() % q);
    const Tw32 t{w, (uint32_t)(((uint64_t)w << 32) / q)};
    const uint32_t r = A.mul(y, t);
    CHECK(r < 2 * q && r % q == (uint32_t)((uint64_t)(y % q) * w % q), "32-bit product");
    const uint32_t x4 = (uint32_t)(rnd() % (4ull * q)), y4 = (uint32_t)(rnd() % (4ull * q));
    uint32_t a0 = x4, b0 = y4;
    A.ct(a0, b0, t);
    CHECK(a0 < 4 * q && b0 < 4 * q, "32-bit ct range");
    CHECK(a0 % q == (uint32_t)((x4 % q + (uint64_t)(y4 % q) * w % q) % q), "32-bit ct sum");
    const uint32_t x2 = (uint32_t)(rnd() % (2ull * q)), y2 = (uint32_t)(rnd() % (2ull * q));
    a0 = x2;
    b0 = y2;
    A.gs(a0, b0, t);
    CHECK(a0 < 2 * q && b0 < 2 * q, "32-bit gs range");
    a0 = x4;
    b0 = y4;
    A.ct1(a0, b0);
    CHECK(a0 < 4 * q && b0 < 4 * q && a0 % q == (x4 % q + y4 % q) % q && b0 % q == (x4 % q + q - y4 % q) % q,
          "32-bit ct1");
    a0 = x2;
    b0 = y2;
    A.gs1(a0, b0);
    CHECK(a0 < 2 * q && b0 < 2 * q && a0 % q == (x2 % q + y2 % q) % q && b0 % q == (x2 % q + q - y2 % q) % q,
          "32-bit gs1");
    CHECK(A.canon_fwd(x4) == x4 % q && A.canon_inv(x2) == x2 % q, "32-bit canonical");
    const uint32_t u = (uint32_t)(rnd() % q), v = (uint32_t)(rnd() % q);
    CHECK(mulmod_general(u, v, m) == (uint32_t)((uint64_t)u * v % q), "32-bit general product");
    const uint32_t mt = mulmod_mont(u, v, m);
    CHECK(mt < q && (uint64_t)mt * m.r1 % q == (uint64_t)u * v % q, "32-bit Montgomery product");
  }
  return 0;
}

int main() {
  // largest supported 64-bit size class (just below 2^61) and the workload primes
  const uint64_t q64[] = {2305843009213693951ull /* 2^61 - 1 (prime) */, 1152921504606584833ull,
                          1152921504606748673ull, 1152921504605798401ull, 998244353ull, 12289ull};
  for (uint64_t q : q64)
    if (test64(q)) return 1;
  // the wide range: the largest prime below 2^60, the workload primes, small ones
  const uint64_t qw[] = {1152921504606846883ull, 1152921504606584833ull, 1152921504605798401ull, 998244353ull,
                         12289ull};
  for (uint64_t q : qw)
    if (test_wide(q)) return 1;
  // largest and smallest primes of bit lengths 2 .. 60
  const uint64_t qc[] = {3ull, 7ull, 5ull, 509ull, 257ull, 131071ull, 65537ull, 134217689ull, 67108879ull,
                         268435399ull, 134217757ull, 536870909ull, 268435459ull, 2147483647ull, 1073741827ull,
                         4294967291ull, 2147483659ull, 8589934583ull, 4294967311ull, 35184372088777ull,
                         17592186044423ull, 576460752303423433ull, 288230376151711813ull, 1152921504606846883ull,
                         576460752303423619ull};
  for (uint64_t q : qc)
    if (test_canon(q)) return 1;
  const uint32_t q32[] = {998244353u, 469762049u, 167772161u, 1073479681u /* < 2^30 */, 12289u};
  for (uint32_t q : q32)
    if (test32(q)) return 1;
  printf("ok %ld\n", checks);
  return 0;
}
