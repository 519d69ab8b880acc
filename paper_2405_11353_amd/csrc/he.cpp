// C ABI of the HE steps: ciphertext tensor product on an NTT plan, and
// conversion plans (fast RNS basis conversion, ModDown).
#include <hip/hip_runtime.h>
#include <string.h>

#include <new>
#include <vector>

#include "he.hpp"
#include "ntt.h"
#include "ntt_internal.hpp"
#include "params.hpp"
#include "trace.hpp"

typedef unsigned __int128 u128;

struct ntt_bconv {
  uint32_t N = 0, L = 0, K = 0;
  int device = 0;
  std::vector<uint64_t> src, dst;
  void* d_src = nullptr;  // BcSrc[L]
  void* d_mat = nullptr;  // [K][Lp] (shat_i mod t_j) 2^64 mod t_j, split at bit 30 (m0 | m1 << 32)
  void* d_dst = nullptr;  // BcDst[K]
  uint32_t G = 4;         // terms per group of the kernel's column sums
  uint32_t hi_reduce = 0; // sum_i (s_i - 1) >= 2^64
};

static int fail(int code) {
  ntt_set_last_error(code);
  return code;
}

static void bconv_release(ntt_bconv* c) {
  if (!c) return;
  (void)hipFree(c->d_src);
  (void)hipFree(c->d_mat);
  (void)hipFree(c->d_dst);
  delete c;
}

static uint64_t shoup_companion(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }

// prod_{k != skip} s_k mod m (skip = L for the whole product)
static uint64_t partial_product(const std::vector<uint64_t>& s, uint32_t skip, uint64_t m) {
  uint64_t r = 1 % m;
  for (uint32_t k = 0; k < s.size(); ++k)
    if (k != skip) r = nttp::mulmod(r, s[k] % m, m);
  return r;
}

extern "C" {

int ntt_tensor_product(const ntt_plan* p, const void* a, const void* b, void* d, uint32_t batch, void* stream) {
  ntti::Range r("ntt_tensor_product");
  if (!p || !a || !b || !d || batch == 0) return fail(NTT_ERR_ARG);
  if ((uint64_t)batch * p->L * p->N * 3 > (1ull << 40)) return fail(NTT_ERR_ARG);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(NTT_ERR_HIP);
  if (dev != p->device) return fail(NTT_ERR_ARG);
  int rc;
  if ((rc = ntti::debug_range(p, a, 2 * batch, stream)) != NTT_OK ||
      (rc = ntti::debug_range(p, b, 2 * batch, stream)) != NTT_OK)
    return fail(rc);
  const hipError_t e = nttk::launch_tensor(p->word, a, b, d, p->d_mod, p->L, p->logN, batch, (hipStream_t)stream);
  return e == hipSuccess ? NTT_OK : fail(NTT_ERR_HIP);
}

ntt_bconv* ntt_bconv_create(uint32_t N, const uint64_t* src, uint32_t L, const uint64_t* dst, uint32_t K) {
  ntt_set_last_error(NTT_OK);
  if (!src || !dst || L == 0 || K == 0 || L > (uint32_t)nttk::BCONV_MAX_L || K > 4096) {
    fail(NTT_ERR_ARG);
    return nullptr;
  }
  if (N < 2 || (N & 1) || N > (1u << 28)) {
    fail(NTT_ERR_N);
    return nullptr;
  }
  std::vector<uint64_t> all(src, src + L);
  all.insert(all.end(), dst, dst + K);
  for (size_t i = 0; i < all.size(); ++i) {
    if (all[i] < 3 || all[i] >= (1ull << 61) || !nttp::is_prime(all[i])) {
      fail(NTT_ERR_MODULUS);
      return nullptr;
    }
    for (size_t k = 0; k < i; ++k)
      if (all[k] == all[i]) {
        fail(NTT_ERR_MODULUS);
        return nullptr;
      }
  }
  ntt_bconv* c = new (std::nothrow) ntt_bconv;
  if (!c) {
    fail(NTT_ERR_NOMEM);
    return nullptr;
  }
  c->N = N;
  c->L = L;
  c->K = K;
  c->src.assign(src, src + L);
  c->dst.assign(dst, dst + K);
  if (hipGetDevice(&c->device) != hipSuccess) {
    bconv_release(c);
    fail(NTT_ERR_HIP);
    return nullptr;
  }
  std::vector<nttk::BcSrc> hs(L);
  for (uint32_t i = 0; i < L; ++i) {
    const uint64_t q = src[i];
    const uint64_t w = nttp::powmod(partial_product(c->src, i, q), q - 2, q);
    hs[i] = nttk::BcSrc{q, 0 - q, w, shoup_companion(w, q)};
  }
  uint64_t max_prime = 0;
  u128 src_sum = 0;
  for (uint64_t q : all) max_prime = q > max_prime ? q : max_prime;
  for (uint64_t q : c->src) src_sum += q - 1;
  c->G = nttk::bconv_group(max_prime);
  c->hi_reduce = src_sum >> 64 ? 1u : 0u;
  const uint32_t Lp = nttk::bconv_row(L, c->G);
  std::vector<uint64_t> hm((size_t)K * Lp, 0);
  std::vector<nttk::BcDst> hd(K);
  for (uint32_t j = 0; j < K; ++j) {
    const uint64_t t = dst[j];
    const uint64_t r64 = (uint64_t)(((u128)1 << 64) % t);  // 2^64 mod t
    // times 2^64, split at bit 30 for the kernel's column sums: m0 | m1 << 32
    for (uint32_t i = 0; i < L; ++i) {
      const uint64_t m = nttp::mulmod(partial_product(c->src, i, t), r64, t);
      hm[(size_t)j * Lp + i] = (m & ((1ull << 30) - 1)) | ((m >> 30) << 32);
    }
    uint64_t inv = t;  // Newton iteration for t^-1 mod 2^64
    for (int k = 0; k < 6; ++k) inv *= 2u - t * inv;
    const uint64_t sinv = nttp::powmod(partial_product(c->src, L, t), t - 2, t);
    hd[j] = nttk::BcDst{t, 0 - t, 0 - inv, (uint64_t)(((u128)1 << 64) / t), sinv, shoup_companion(sinv, t), 0, 0};
  }
  if (ntti::dev_malloc(&c->d_src, hs.size() * sizeof(nttk::BcSrc)) != hipSuccess ||
      ntti::dev_malloc(&c->d_mat, hm.size() * sizeof(uint64_t)) != hipSuccess ||
      ntti::dev_malloc(&c->d_dst, hd.size() * sizeof(nttk::BcDst)) != hipSuccess) {
    bconv_release(c);
    fail(NTT_ERR_NOMEM);
    return nullptr;
  }
  if (hipMemcpy(c->d_src, hs.data(), hs.size() * sizeof(nttk::BcSrc), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_mat, hm.data(), hm.size() * sizeof(uint64_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_dst, hd.data(), hd.size() * sizeof(nttk::BcDst), hipMemcpyHostToDevice) != hipSuccess) {
    bconv_release(c);
    fail(NTT_ERR_HIP);
    return nullptr;
  }
  return c;
}

void ntt_bconv_destroy(ntt_bconv* c) { bconv_release(c); }

static int bconv_run(const ntt_bconv* c, const void* x, const void* y, void* out, uint32_t batch, void* stream) {
  if (!c || !x || !out || batch == 0) return fail(NTT_ERR_ARG);
  if ((uint64_t)batch * c->N > 0x7FFFFFFFull) return fail(NTT_ERR_ARG);
  // 16-byte vector accesses
  if (((uintptr_t)x | (uintptr_t)out | (uintptr_t)y) & 15) return fail(NTT_ERR_ARG);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(NTT_ERR_HIP);
  if (dev != c->device) return fail(NTT_ERR_ARG);
  const hipError_t e = nttk::launch_bconv((const uint64_t*)x, (const uint64_t*)y, (uint64_t*)out,
                                          (const nttk::BcSrc*)c->d_src, (const uint64_t*)c->d_mat,
                                          (const nttk::BcDst*)c->d_dst, c->L, c->K, c->N, batch, c->G,
                                          c->hi_reduce, (hipStream_t)stream);
  return e == hipSuccess ? NTT_OK : fail(NTT_ERR_HIP);
}

int ntt_base_conv(const ntt_bconv* c, const void* d_x, void* d_out, uint32_t batch, void* stream) {
  ntti::Range r("ntt_base_conv");
  return bconv_run(c, d_x, nullptr, d_out, batch, stream);
}

int ntt_mod_down(const ntt_bconv* c, const void* d_x, const void* d_y, void* d_out, uint32_t batch,
                 void* stream) {
  ntti::Range r("ntt_mod_down");
  if (!d_y) return fail(NTT_ERR_ARG);
  return bconv_run(c, d_x, d_y, d_out, batch, stream);
}

int ntt_bconv_get_info(const ntt_bconv* c, uint32_t* N, uint32_t* L, uint32_t* K) {
  if (!c) return NTT_ERR_ARG;
  if (N) *N = c->N;
  if (L) *L = c->L;
  if (K) *K = c->K;
  return NTT_OK;
}

}  // extern "C"
