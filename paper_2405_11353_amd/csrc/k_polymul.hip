// Polynomial product, four-step shapes: the forward row passes of both
// operands, their elementwise product and the first inverse pass, fused into
// one kernel per row tile. Between the column passes the spectra never reach
// HBM.
#include "polymul.hpp"
#include "launch.hpp"
#include "ntt_core.hpp"

namespace nttk {

// 16 rows per workgroup, N2/V threads per row (V = 2^LV values each; a row
// lies inside one wave, so every exchange is wave-local). The forward phases leave thread t holding
// positions pos(last phase, t, i) of each row, which is the layout the
// inverse phases start from, so the product needs no exchange.
// IND: items come from a descriptor table (data: a's column-pass output,
// overwritten with the product; aux: b's; twiddles and modulus per item), as
// in the server's batches.
template <class A, int LOGN2, bool IND = false, int LV = 4>
__global__ void __launch_bounds__(16 << (LOGN2 - LV))
k_row_polymul(typename A::word* sa, const typename A::word* __restrict__ sb,
              const typename A::tw_t* __restrict__ twf_all, const typename A::tw_t* __restrict__ twi_all,
              const typename ModOf<A>::type* __restrict__ mods, uint32_t L, uint32_t logN, uint32_t batch,
              const ItemDesc* __restrict__ desc = nullptr) {
  using W = typename A::word;
  using TW = typename A::tw_t;
  using M = typename ModOf<A>::type;
  using S = Sched<LOGN2, LV>;
  constexpr int V = 1 << LV;
  constexpr uint32_t N2 = 1u << LOGN2, TPR = N2 / V, RSTR = N2 + N2 / 16 + 1;
  static_assert(TPR <= 64, "a row must fit in one wavefront");
  __shared__ W lds[16 * RSTR];
  __shared__ TW tw0[16][17];  // first-phase twiddles of the 16 rows: forward, then inverse
  const uint32_t logN1 = logN - LOGN2, N1 = 1u << logN1;
  const uint32_t tiles = N1 / 16;
  const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t t = threadIdx.x % TPR, rl = threadIdx.x / TPR;
  uint32_t tile;
  M m;
  const TW* twf;
  const TW* twi;
  W* rowa;
  const W* rowb;
  if constexpr (IND) {
    // logical order (item, tile): an item's tiles run back to back on one XCD
    const uint32_t item = bid / tiles;
    tile = bid % tiles;
    if (item >= batch) return;
    const ItemDesc d = desc[item];
    m = *(const M*)d.mod;
    twf = (const TW*)d.tw_fwd;
    twi = (const TW*)d.tw_inv;
    rowa = (W*)d.data + (size_t)(tile * 16 + rl) * N2;
    rowb = (const W*)d.aux + (size_t)(tile * 16 + rl) * N2;
  } else {
    // logical order (limb, tile, pair): the pairs sharing a limb's twiddles
    // run back to back on one XCD
    const uint32_t b = bid % batch, rest = bid / batch;
    tile = rest % tiles;
    const uint32_t l = rest / tiles;
    if (l >= L) return;
    m = mods[l];
    twf = twf_all + ((size_t)l << logN);
    twi = twi_all + ((size_t)l << logN);
    const size_t off = (((size_t)b * L + l) << logN) + (size_t)(tile * 16 + rl) * N2;
    rowa = sa + off;
    rowb = sb + off;
  }
  const uint32_t r = tile * 16 + rl;
  A a;
  a.load(m);
  W* sh = lds + rl * RSTR;
  auto row_of = [&](uint32_t row) { return tile * 16 + row; };

  W va[V], vb[V];
  // the first-phase twiddles are loaded ahead of the row and written to LDS
  // after the row's loads are issued (loads complete in order)
  FirstPhaseStage<LOGN2, LV, TW> first;
  first.load(twf, logN1, row_of);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int i = 0; i < V; ++i) va[i] = rowa[i * TPR + t];
  first.put(tw0);
  wave_lds_sync();

  auto forward = [&](W (&v)[V], const TW* twf) {
    static_for<0, S::NPH>([&](auto P_) {
      constexpr int p = decltype(P_)::value;
      if constexpr (p > 0) {
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < V; ++i) sh[pad16(pos<LOGN2, LV>(p - 1, t, i))] = v[i];
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = sh[pad16(pos<LOGN2, LV>(p, t, i))];
        ct_phase<A, S::rs(p)>(a, v, twf, logN1 + S::s0(p), (r << S::s0(p)) + grp<LOGN2, LV>(p, t));
      } else {
        ct_phase<A, S::rs(p)>(a, v, &tw0[rl][0], 0u, 0u);
      }
    });
  };
  // one operand at a time, so that only one row's working set is live: a's
  // transform is made canonical before b's row is loaded (the product needs
  // a * b below q * 2^w, which a lazy a below 8q would also meet, but leaving
  // a lazy measured slower: the loop gives b's loads their latency)
  forward(va, twf);
#pragma unroll
  for (int i = 0; i < V; ++i) va[i] = a.canon_fwd(va[i]);
#pragma unroll
  for (int i = 0; i < V; ++i) vb[i] = rowb[i * TPR + t];
  // b's transform reads the same twiddles; an opaque copy of the table
  // pointer makes the compiler load them again (cache hits) instead of
  // keeping all of a's twiddles live across both transforms
  const TW* twf_b = twf;
  asm volatile("" : "+v"(twf_b));
  forward(vb, twf_b);
#pragma unroll
  for (int i = 0; i < V; ++i) {
    // direct mode: Montgomery product, the factor 2^-w multiplied back in by
    // the inverse column pass; descriptor mode (no scaled pair there): exact
    if constexpr (IND) va[i] = mulmod_general(va[i], a.canon_fwd(vb[i]), m);
    else va[i] = mulmod_mont(va[i], a.canon_fwd(vb[i]), m);
  }
  // the wave's rows switch to the inverse table's first-phase twiddles; the
  // inverse phases' exchanges order the copy before their use
  wave_lds_sync();
  stage_first_phase<LOGN2, LV>(tw0, twi, logN1, row_of);
  static_for_down<S::NPH - 1, 0>([&](auto P_) {
    constexpr int p = decltype(P_)::value;
    if constexpr (p < S::NPH - 1) {
      wave_lds_sync();
#pragma unroll
      for (int i = 0; i < V; ++i) sh[pad16(pos<LOGN2, LV>(p + 1, t, i))] = va[i];
      wave_lds_sync();
#pragma unroll
      for (int i = 0; i < V; ++i) va[i] = sh[pad16(pos<LOGN2, LV>(p, t, i))];
    }
    if constexpr (p == 0) gs_phase<A, S::rs(p), false>(a, va, &tw0[rl][0], 0u, 0u);
    else gs_phase<A, S::rs(p), false>(a, va, twi, logN1 + S::s0(p), (r << S::s0(p)) + grp<LOGN2, LV>(p, t));
  });
  // phase 0 leaves thread t with positions i * TPR + t
#pragma unroll
  for (int i = 0; i < V; ++i) rowa[i * TPR + t] = va[i];
}

// values per thread (2^LV) of the fused product kernel; rows of 2^9 keep 16
// values per thread: at 8 a workgroup has 1024 threads, which caps a thread
// at 128 registers, fewer than the two operands' rows need without spilling
#ifndef NTT_LV_POLYMUL
#define NTT_LV_POLYMUL 4
#endif
static_assert(NTT_LV_POLYMUL == 3 || NTT_LV_POLYMUL == 4, "8 or 16 values per thread");
constexpr int pm_lv(int lg2) { return lg2 >= 9 ? 4 : NTT_LV_POLYMUL; }

template <class A>
static hipError_t go(int logN, int logN1, void* sa, const void* sb, const void* twf, const void* twi,
                     const void* mods, uint32_t L, uint32_t batch, hipStream_t s) {
  using W = typename A::word;
  using TW = typename A::tw_t;
  using M = typename ModOf<A>::type;
  const int lg2 = logN - logN1;
  if (logN1 < 6 || logN1 > 9 || lg2 < 6 || lg2 > 9) return hipErrorNotSupported;
  const uint32_t tiles = (1u << logN1) / 16;
  const dim3 grid(batch * L * tiles);
#define POLYMUL_CASE(LG2)                                                                                  \
  case LG2:                                                                                                \
    hipLaunchKernelGGL((k_row_polymul<A, LG2, false, pm_lv(LG2)>), grid, dim3(16u << (LG2 - pm_lv(LG2))), 0, s, \
                       (W*)sa, (const W*)sb, (const TW*)twf, (const TW*)twi, (const M*)mods, L, (uint32_t)logN,   \
                       batch);                                                                             \
    break;
  switch (lg2) {
    POLYMUL_CASE(6)
    POLYMUL_CASE(7)
    POLYMUL_CASE(8)
    POLYMUL_CASE(9)
    default: return hipErrorNotSupported;
  }
#undef POLYMUL_CASE
  return hipGetLastError();
}

hipError_t launch_row_polymul(int word, int logN, int logN1, void* sa, const void* sb, const void* tw_fwd,
                              const void* tw_inv, const void* mods, uint32_t L, uint32_t batch, hipStream_t s) {
  if (word == 32) return go<Arith32>(logN, logN1, sa, sb, tw_fwd, tw_inv, mods, L, batch, s);
  return go<Arith64<false>>(logN, logN1, sa, sb, tw_fwd, tw_inv, mods, L, batch, s);
}

hipError_t launch_ind_row_polymul(const ItemDesc* desc, uint32_t items, int logN, int logN1, hipStream_t s) {
  using A = Arith64<false>;
  const int lg2 = logN - logN1;
  if (items == 0) return hipSuccess;
  if (logN1 < 6 || logN1 > 9 || lg2 < 6 || lg2 > 9) return hipErrorNotSupported;
  const dim3 grid(items * ((1u << logN1) / 16));
#define IND_CASE(LG2)                                                                                      \
  case LG2:                                                                                                \
    hipLaunchKernelGGL((k_row_polymul<A, LG2, true, pm_lv(LG2)>), grid, dim3(16u << (LG2 - pm_lv(LG2))), 0, s,  \
                       nullptr, nullptr, nullptr, nullptr, nullptr, 1u, (uint32_t)logN, items, desc);      \
    break;
  switch (lg2) {
    IND_CASE(6)
    IND_CASE(7)
    IND_CASE(8)
    IND_CASE(9)
    default: return hipErrorNotSupported;
  }
#undef IND_CASE
  return hipGetLastError();
}

}  // namespace nttk
