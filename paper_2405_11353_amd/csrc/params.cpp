#include "params.hpp"

#include <string.h>

namespace nttp {

using u128 = unsigned __int128;

uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }

uint64_t powmod(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  a %= q;
  for (; e; e >>= 1) {
    if (e & 1) r = mulmod(r, a, q);
    a = mulmod(a, a, q);
  }
  return r;
}

// Miller-Rabin with the first twelve primes as bases: deterministic below 3.3e24.
bool is_prime(uint64_t n) {
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (uint64_t p : bases)
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int r = 0;
  while ((d & 1) == 0) { d >>= 1; ++r; }
  for (uint64_t a : bases) {
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < r && comp; ++i) {
      x = mulmod(x, x, n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}

uint64_t smallest_qnr(uint64_t q) {
  for (uint64_t c = 2; c < 1000 && c < q; ++c)
    if (powmod(c, (q - 1) / 2, q) == q - 1) return c;
  return 0;
}

uint64_t default_psi(uint64_t q, uint32_t N) {
  if ((q - 1) % (2ull * N)) return 0;
  const uint64_t c = smallest_qnr(q);
  return c ? powmod(c, (q - 1) / (2ull * N), q) : 0;
}

uint64_t default_omega(uint64_t q, uint32_t N) {
  if ((q - 1) % N) return 0;
  const uint64_t c = smallest_qnr(q);
  return c ? powmod(c, (q - 1) / N, q) : 0;
}

static uint32_t bitrev(uint32_t x, uint32_t bits) {
  if (bits == 0) return 0;
  x = ((x >> 1) & 0x55555555u) | ((x & 0x55555555u) << 1);
  x = ((x >> 2) & 0x33333333u) | ((x & 0x33333333u) << 2);
  x = ((x >> 4) & 0x0F0F0F0Fu) | ((x & 0x0F0F0F0Fu) << 4);
  x = ((x >> 8) & 0x00FF00FFu) | ((x & 0x00FF00FFu) << 8);
  x = (x >> 16) | (x << 16);
  return x >> (32 - bits);
}

// x * w mod q by Shoup's product with wp = floor(w * 2^64 / q): for x, w < q
// < 2^63, x * w - hi64(x * wp) * q lies in [0, 2q).
static inline uint64_t mul_shoup(uint64_t x, uint64_t w, uint64_t wp, uint64_t q) {
  const uint64_t Q = (uint64_t)(((u128)x * wp) >> 64);
  const uint64_t r = x * w - Q * q;
  return r >= q ? r - q : r;
}

// root^0 .. root^(count-1) mod q with no division per step: eight
// interleaved chains, each advanced by the fixed factor root^8.
static void powers(uint64_t q, uint64_t root, size_t count, std::vector<uint64_t>& pw) {
  pw.resize(count);
  const uint64_t rp = (uint64_t)(((u128)root << 64) / q);
  uint64_t x = 1 % q;
  for (size_t e = 0; e < count && e < 8; ++e) {
    pw[e] = x;
    x = mul_shoup(x, root, rp, q);
  }
  const uint64_t r8 = x, r8p = (uint64_t)(((u128)r8 << 64) / q);  // root^8
  for (size_t e = 8; e < count; ++e) pw[e] = mul_shoup(pw[e - 8], r8, r8p, q);
}

// Shoup companions floor(w * 2^64 / q) for w < q from v = floor((2^128 - 1) /
// q), one division per table instead of one per entry: v > 2^128/q - 2, so
// w * v / 2^64 > w * 2^64 / q - 2q / 2^64 > w * 2^64 / q - 1 (q < 2^63), and
// floor(w * v / 2^64) = w * v_hi + hi64(w * v_lo) is the companion or one
// below it; the remainder w * 2^64 - e * q says which.
struct Recip {
  uint64_t q, vhi, vlo;
};
static Recip recip(uint64_t q) {
  const u128 v = ~(u128)0 / q;
  return Recip{q, (uint64_t)(v >> 64), (uint64_t)v};
}
static uint64_t companion64(uint64_t w, const Recip& R) {
  const uint64_t e = w * R.vhi + (uint64_t)(((u128)w * R.vlo) >> 64);
  const u128 r = ((u128)w << 64) - (u128)e * R.q;
  return e + (r >= R.q ? 1 : 0);
}

static void put_entry(uint64_t w, const Recip& R, int word, void* out, size_t k) {
  if (word == 32) {
    uint32_t* o = (uint32_t*)out + 2 * k;
    o[0] = (uint32_t)w;
    o[1] = (uint32_t)(((uint64_t)w << 32) / R.q);
  } else {
    uint64_t* o = (uint64_t*)out + 2 * k;
    o[0] = w;
    o[1] = companion64(w, R);
  }
}

size_t tw_entry_bytes(int word) { return word == 32 ? 8 : 16; }
size_t modinfo_bytes(int word) { return word == 32 ? 32 : 72; }

void twiddles(uint64_t q, uint64_t root, uint32_t logN, int word, bool inverse, void* out, bool cyclic) {
  const uint32_t N = 1u << logN;
  // powers of the root; the root has order 2N (negacyclic) or N (cyclic)
  const size_t order = cyclic ? (size_t)N : 2 * (size_t)N;
  std::vector<uint64_t> pw;
  powers(q, root, order, pw);
  const uint64_t n_inv = powmod(N % q, q - 2, q);
  const Recip R = recip(q);
  auto exponent = [&](uint32_t k) -> size_t {  // k >= 1
    if (!cyclic) return bitrev(k, logN);
    uint32_t s = 0;
    while ((2u << s) <= k) ++s;
    const uint32_t i = k - (1u << s);
    return (size_t)(N >> (s + 1)) * bitrev(i, s);
  };
  auto value = [&](uint32_t k) -> uint64_t {
    if (!inverse) return k == 0 ? 1 : pw[exponent(k)];
    if (k == 0) return n_inv;
    const uint64_t w = pw[(order - exponent(k)) % order];
    return k == 1 ? mulmod(w, n_inv, q) : w;
  };
  for (uint32_t k = 0; k < N; ++k) put_entry(value(k), R, word, out, k);
}


void twist(uint64_t q, uint64_t root, uint32_t logN, uint32_t logN1, int word, bool inverse, bool cyclic, void* out) {
  const uint32_t N = 1u << logN, N1 = 1u << logN1, N2 = N >> logN1;
  const size_t order = cyclic ? (size_t)N : 2 * (size_t)N;
  std::vector<uint64_t> pw;
  powers(q, root, order, pw);
  const Recip R = recip(q);
  for (uint32_t r = 0; r < N1; ++r) {
    const size_t eb = cyclic ? bitrev(r, logN1) : 2 * (size_t)bitrev(r, logN1) + 1;
    size_t e = 0;  // eb * j mod order
    for (uint32_t j = 0; j < N2; ++j) {
      put_entry(pw[inverse ? (order - e) % order : e], R, word, out, (size_t)r * N2 + j);
      e += eb;
      if (e >= order) e -= order;
    }
  }
}

void mont_scale(uint64_t q, int word, const void* inv_table, void* out) {
  const Recip R = recip(q);
  const uint64_t r = word == 32 ? (1ull << 32) % q : (uint64_t)(((u128)1 << 64) % q);
  for (size_t k = 0; k < 2; ++k) {
    const uint64_t w = word == 32 ? ((const uint32_t*)inv_table)[2 * k] : ((const uint64_t*)inv_table)[2 * k];
    put_entry(mulmod(w, r, q), R, word, out, k);
  }
}

uint64_t row_root(uint64_t q, uint64_t root, uint32_t logN1, bool cyclic) {
  return powmod(root, (cyclic ? 1ull : 2ull) << logN1, q);
}

void modinfo(uint64_t q, int word, void* out) {
  if (word == 32) {
    uint32_t m[8] = {0};
    uint32_t q32 = (uint32_t)q, inv = q32;  // Newton iteration for q^-1 mod 2^32
    for (int i = 0; i < 5; ++i) inv *= 2u - q32 * inv;
    const uint32_t r1 = (uint32_t)((1ull << 32) % q);
    m[0] = q32;
    m[2] = inv;
    m[3] = r1;
    m[4] = (uint32_t)(((uint64_t)r1 << 32) / q);
    memcpy(out, m, sizeof m);
  } else {
    uint64_t m[9] = {0};
    uint64_t inv = q;  // Newton iteration for q^-1 mod 2^64
    for (int i = 0; i < 6; ++i) inv *= 2u - q * inv;
    const uint64_t r1 = (uint64_t)(((u128)1 << 64) % q);
    m[0] = q;
    m[1] = 0 - 8 * q;  // wraps for q >= 2^61, where the wide range is not used
    m[2] = 0 - q;
    m[3] = inv;
    m[4] = r1;
    m[5] = (uint64_t)(((u128)r1 << 64) / q);
    m[6] = 0 - 2 * q;
    m[7] = 0 - 4 * q;
    // wide-range canonicalisation: floor(x / q) from x >> s times c >> e
    const int b = 64 - __builtin_clzll(q);
    const int s = b >= 28 ? b - 28 : 0, e = b >= 28 ? 26 : b - 1;
    const uint64_t c = (uint64_t)(((u128)1 << (s + 32 + e)) / q);  // < 2^32
    m[8] = c | ((uint64_t)s << 32) | ((uint64_t)e << 40);
    memcpy(out, m, sizeof m);
  }
}

}  // namespace nttp
