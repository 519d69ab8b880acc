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
  uint32_t r = 0;
  for (uint32_t b = 0; b < bits; ++b) r |= ((x >> b) & 1u) << (bits - 1 - b);
  return r;
}

size_t tw_entry_bytes(int word) { return word == 32 ? 8 : 16; }
size_t modinfo_bytes(int word) { return word == 32 ? 32 : 64; }

void twiddles(uint64_t q, uint64_t root, uint32_t logN, int word, bool inverse, void* out, bool cyclic) {
  const uint32_t N = 1u << logN;
  // powers of the root; the root has order 2N (negacyclic) or N (cyclic)
  const size_t order = cyclic ? (size_t)N : 2 * (size_t)N;
  std::vector<uint64_t> pw(order);
  pw[0] = 1;
  for (size_t e = 1; e < order; ++e) pw[e] = mulmod(pw[e - 1], root, q);
  const uint64_t n_inv = powmod(N % q, q - 2, q);
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
  for (uint32_t k = 0; k < N; ++k) {
    const uint64_t w = value(k);
    if (word == 32) {
      uint32_t* o = (uint32_t*)out + 2 * (size_t)k;
      o[0] = (uint32_t)w;
      o[1] = (uint32_t)(((uint64_t)w << 32) / q);
    } else {
      uint64_t* o = (uint64_t*)out + 2 * (size_t)k;
      o[0] = w;
      o[1] = (uint64_t)(((u128)w << 64) / q);
    }
  }
}

static void put_entry(uint64_t w, uint64_t q, int word, void* out, size_t k) {
  if (word == 32) {
    uint32_t* o = (uint32_t*)out + 2 * k;
    o[0] = (uint32_t)w;
    o[1] = (uint32_t)(((uint64_t)w << 32) / q);
  } else {
    uint64_t* o = (uint64_t*)out + 2 * k;
    o[0] = w;
    o[1] = (uint64_t)(((u128)w << 64) / q);
  }
}

void twist(uint64_t q, uint64_t root, uint32_t logN, uint32_t logN1, int word, bool inverse, bool cyclic, void* out) {
  const uint32_t N = 1u << logN, N1 = 1u << logN1, N2 = N >> logN1;
  const size_t order = cyclic ? (size_t)N : 2 * (size_t)N;
  std::vector<uint64_t> pw(order);
  pw[0] = 1;
  for (size_t e = 1; e < order; ++e) pw[e] = mulmod(pw[e - 1], root, q);
  for (uint32_t r = 0; r < N1; ++r) {
    const size_t eb = cyclic ? bitrev(r, logN1) : 2 * (size_t)bitrev(r, logN1) + 1;
    for (uint32_t j = 0; j < N2; ++j) {
      const size_t e = (eb * j) % order;
      put_entry(pw[inverse ? (order - e) % order : e], q, word, out, (size_t)r * N2 + j);
    }
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
    uint64_t m[8] = {0};
    uint64_t inv = q;  // Newton iteration for q^-1 mod 2^64
    for (int i = 0; i < 6; ++i) inv *= 2u - q * inv;
    const uint64_t r1 = (uint64_t)(((u128)1 << 64) % q);
    m[0] = q;
    m[2] = 0 - q;
    m[3] = inv;
    m[4] = r1;
    m[5] = (uint64_t)(((u128)r1 << 64) / q);
    memcpy(out, m, sizeof m);
  }
}

}  // namespace nttp
