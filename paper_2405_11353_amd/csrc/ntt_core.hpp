// Kernel templates for the negacyclic NTT on gfx950.
//
// Transform: the merged-twiddle Cooley-Tukey form of the negacyclic NTT. Stage
// s (0-based) pairs positions p and p + N/2^(s+1) and multiplies by
// psi^brv(2^s + (p >> (logN - s))); after logN stages position p holds
// X[brv(p)], the evaluation at psi^(2 brv(p) + 1). The inverse runs the stages
// backwards as Gentleman-Sande butterflies with psi^-brv(k), and the factor
// N^-1 is folded into the two twiddles of the last stage (table slots 0, 1).
// Compared with the paper's DIT (Alg. 1) the psi^j twist is absorbed into the
// twiddles and the bit reversal is done by the store, through LDS.
//
// Work split: each thread holds V = 2^LV values (16, or 8 in the four-step
// kernels that take LV = 3) and applies up to LV stages to them in registers
// (a "phase"); values are exchanged through LDS between phases. A remainder
// phase of logN mod LV stages comes first, so that in every phase the V values
// of a thread sit at a power-of-two stride with the stride of the phase's last
// stage. Twiddles are read from global memory (L1/L2 hits:
// the per-limb table is shared by all polynomials of that limb).
//
// Kernel shapes:
//  * k_lds   : the whole transform in one workgroup (N <= 2^14 for 64-bit words)
//  * k_col/k_row : the four-step split N = N1 x N2 (the paper's six-step idea
//    without the explicit transposes): the first logN1 stages act on the N2
//    columns of the N1 x N2 row-major matrix with the shared twiddles
//    psi^brv(k), k < N1; the last logN2 stages act on each row r with the
//    twiddles of the subtree under node N1 + r. The natural-order output
//    position of row element (r, c) is brv(c) * N1 + brv(r), so a tile of 16
//    rows with consecutive brv(r) is written as 128-byte segments.
//  * k_tiny  : N < 16, one thread per transform.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "launch.hpp"
#include "modarith.hpp"

namespace nttk {

// compile-time loops: f(integral_constant<int, k>) for k = B..E-1 / B down to E
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(static_cast<F&&>(f));
  }
}
template <int B, int E, class F>
__device__ __forceinline__ void static_for_down(F&& f) {
  if constexpr (B >= E) {
    f(std::integral_constant<int, B>{});
    static_for_down<B - 1, E>(static_cast<F&&>(f));
  }
}

template <class A> struct ModOf;
template <bool E, bool W> struct ModOf<Arith64<E, W>> { using type = ModInfo64; };
template <> struct ModOf<Arith32> { using type = ModInfo32; };

__device__ __forceinline__ uint32_t brv(uint32_t x, uint32_t bits) {
  return bits ? (__builtin_bitreverse32(x) >> (32 - bits)) : 0u;
}

// Blocks are dispatched round-robin over the 8 XCDs of the chip; this maps
// consecutive logical work items onto the same XCD (and so the same L2).
// A permutation of [0, G) for any G, so correctness does not depend on the
// hardware's dispatch order.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t G) {
  const uint32_t x = bid & 7u, i = bid >> 3;
  const uint32_t q = G >> 3, r = G & 7u;
  return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// ----------------------------------------------------------- phase schedule
// A thread holds V = 2^LV values (16 by default, 8 where more threads pay)
// and applies up to LV stages to them per phase.
template <int LOGN, int LV = 4> struct Sched {
  static_assert(LOGN >= LV, "N must hold at least V values per thread");
  static constexpr int R0 = LOGN % LV;
  static constexpr int NPH = LOGN / LV + (R0 ? 1 : 0);
  __host__ __device__ static constexpr int rs(int p) { return (R0 && p == 0) ? R0 : LV; }
  __host__ __device__ static constexpr int s0(int p) { return p == 0 ? 0 : (R0 ? R0 + LV * (p - 1) : LV * p); }
  __host__ __device__ static constexpr int lgs(int p) { return LOGN - s0(p) - LV; }  // log2 of the stride
};

// position of value i of thread t in phase p (transform-local)
template <int LOGN, int LV = 4>
__device__ __forceinline__ uint32_t pos(int p, uint32_t t, int i) {
  const int lg = Sched<LOGN, LV>::lgs(p);
  const uint32_t H = t >> lg, low = t & ((1u << lg) - 1u);
  return (H << (lg + LV)) + ((uint32_t)i << lg) + low;
}
// group index of thread t at the first stage of phase p (transform-local)
template <int LOGN, int LV = 4>
__device__ __forceinline__ uint32_t grp(int p, uint32_t t) { return t >> Sched<LOGN, LV>::lgs(p); }

// which forward stages reduce x: RP_* and reduces_x in modarith.hpp
template <class A>
constexpr int rp_of(int wide_rp) { return A::kWide ? wide_rp : RP_ALL; }

// ----------------------------------------------------------- register phases
// RS stages starting at global stage S0; Hg = global group index at S0. RP
// and J0 (the pass-relative index of the phase's first stage) decide which
// stages reduce x.
template <class A, int RS, int RP = RP_ALL, int J0 = 0, int V>
__device__ __forceinline__ void ct_phase(const A& a, typename A::word (&v)[V],
                                         const typename A::tw_t* __restrict__ tw, uint32_t S0, uint32_t Hg) {
  static_for<0, RS>([&](auto K_) {
    constexpr int k = decltype(K_)::value;
    constexpr bool RED = reduces_x(RP, J0 + k);
    const typename A::tw_t* tk = tw + (1u << (S0 + k)) + (Hg << k);
#pragma unroll
    for (int j = 0; j < (1 << k); ++j) {
      const typename A::tw_t w = tk[j];
#pragma unroll
      for (int m = 0; m < ((V / 2) >> k); ++m) {
        const int i0 = j * (V >> k) + m;
        a.template ct<RED>(v[i0], v[i0 + ((V / 2) >> k)], w);
      }
    }
  });
}

// Inverse: the same pairs, stages in reverse order. HAS0: this phase contains
// global stage 0, whose two outputs are both scaled (tables slots 0 and 1, or
// the pair at t01 when given).
template <class A, int RS, bool HAS0, int V>
__device__ __forceinline__ void gs_phase(const A& a, typename A::word (&v)[V],
                                         const typename A::tw_t* __restrict__ tw, uint32_t S0, uint32_t Hg,
                                         const typename A::tw_t* t01 = nullptr) {
#pragma unroll
  for (int k = RS - 1; k >= 0; --k) {
    if (HAS0 && k == 0) {
      const typename A::tw_t* p01 = t01 ? t01 : tw;
      const typename A::tw_t w0 = p01[0], w1 = p01[1];
#pragma unroll
      for (int m = 0; m < V / 2; ++m) a.gs_last(v[m], v[m + V / 2], w0, w1);
    } else {
      const typename A::tw_t* tk = tw + (1u << (S0 + k)) + (Hg << k);
#pragma unroll
      for (int j = 0; j < (1 << k); ++j) {
        const typename A::tw_t w = tk[j];
#pragma unroll
        for (int m = 0; m < ((V / 2) >> k); ++m) {
          const int i0 = j * (V >> k) + m;
          a.gs(v[i0], v[i0 + ((V / 2) >> k)], w);
        }
      }
    }
  }
}

__device__ __forceinline__ uint32_t pad16(uint32_t x) { return x + (x >> 4); }

// ordering of LDS traffic inside one wavefront (no workgroup barrier needed)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ============================================================ k_lds
// P transforms per workgroup, N/16 threads each, whole transform in LDS.
// IND: items come from a descriptor table (batched executor) instead of the
// contiguous [batch][L][N] layout.
template <class A, int LOGN, int P, bool FWD, bool NATURAL, bool IND = false>
__global__ void __launch_bounds__(P << (LOGN - 4))
k_lds(typename A::word* __restrict__ data, const typename A::tw_t* __restrict__ tw_all,
      const typename ModOf<A>::type* __restrict__ mods, uint32_t L, uint32_t items,
      const ItemDesc* __restrict__ desc = nullptr) {
  using W = typename A::word;
  using TW = typename A::tw_t;
  using M = typename ModOf<A>::type;
  using S = Sched<LOGN>;
  constexpr uint32_t N = 1u << LOGN, T = N / 16, SPAN = N + N / 16;
  __shared__ W lds[P * SPAN];
  const uint32_t g = threadIdx.x / T, t = threadIdx.x % T;
  const uint32_t item = blockIdx.x * P + g;
  const bool valid = item < items;
  const uint32_t vi = valid ? item : 0;
  A a;
  const TW* tw;
  W* x;
  if constexpr (IND) {
    const ItemDesc d = desc[vi];
    a.load(*(const M*)d.mod);
    tw = (const TW*)(FWD ? d.tw_fwd : d.tw_inv);
    x = (W*)d.data;
  } else {
    const uint32_t l = vi % L;
    a.load(mods[l]);
    tw = tw_all + ((size_t)l << LOGN);
    x = data + ((size_t)vi << LOGN);
  }
  W* sh = lds + g * SPAN;
  W v[16];
  if constexpr (FWD) {
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = valid ? x[i * T + t] : W(0);
    static_for<0, S::NPH>([&](auto P_) {
      constexpr int p = decltype(P_)::value;
      if constexpr (p > 0) {
        if constexpr (p > 1) __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; ++i) sh[pad16(pos<LOGN>(p - 1, t, i))] = v[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = sh[pad16(pos<LOGN>(p, t, i))];
      }
      // phase 0 has one group per transform: its twiddle addresses are
      // uniform and the compiler reads them with scalar loads
      ct_phase<A, S::rs(p), rp_of<A>(RP_FRESH), S::s0(p)>(a, v, tw, S::s0(p), p == 0 ? 0u : grp<LOGN>(p, t));
    });
    if (S::NPH > 1) __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const uint32_t ps = pos<LOGN>(S::NPH - 1, t, i);
      sh[pad16(NATURAL ? brv(ps, LOGN) : ps)] = a.canon_fwd(v[i]);
    }
    __syncthreads();
    if (valid) {
#pragma unroll
      for (int i = 0; i < 16; ++i) x[i * T + t] = sh[pad16(i * T + t)];
    }
  } else {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const uint32_t m = i * T + t;
      sh[pad16(NATURAL ? brv(m, LOGN) : m)] = valid ? x[m] : W(0);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = sh[pad16(pos<LOGN>(S::NPH - 1, t, i))];
    static_for_down<S::NPH - 1, 0>([&](auto P_) {
      constexpr int p = decltype(P_)::value;
      if constexpr (p < S::NPH - 1) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; ++i) sh[pad16(pos<LOGN>(p + 1, t, i))] = v[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = sh[pad16(pos<LOGN>(p, t, i))];
      }
      gs_phase<A, S::rs(p), p == 0>(a, v, tw, S::s0(p), p == 0 ? 0u : grp<LOGN>(p, t));
    });
    if (valid) {
#pragma unroll
      for (int i = 0; i < 16; ++i) x[i * T + t] = a.canon_inv(v[i]);
    }
  }
}

// ============================================================ data access
// Loads and stores of polynomial data, by role: IN (first read of a
// transform's input), MID (the four-step intermediate, written by one pass
// and re-read by the next while it is still in the last-level cache) and OUT
// (a transform's final output). Each access kind can carry the nontemporal
// (streaming) hint.
#ifndef NTT_NT_LD_IN
#define NTT_NT_LD_IN 0
#endif
#ifndef NTT_NT_ST_MID
#define NTT_NT_ST_MID 0
#endif
#ifndef NTT_NT_LD_MID
#define NTT_NT_LD_MID 0
#endif
#ifndef NTT_NT_ST_OUT
#define NTT_NT_ST_OUT 0
#endif
// the inverse column pass's output alone (the end of an inverse transform):
// on by default. Nothing later in a transform reads it, so it need not stay in
// the caches, where it would displace what the next kernels read (the inverse
// column pass of 48 transforms at 2^16: 16.4-16.6 -> 13.2-14.4 us)
#ifndef NTT_NT_ST_INV_OUT
#define NTT_NT_ST_INV_OUT 1
#endif
constexpr bool NT_LD_IN = NTT_NT_LD_IN, NT_ST_MID = NTT_NT_ST_MID, NT_LD_MID = NTT_NT_LD_MID,
               NT_ST_OUT = NTT_NT_ST_OUT, NT_ST_INV_OUT = NTT_NT_ST_OUT || NTT_NT_ST_INV_OUT;

template <bool NT, class T>
__device__ __forceinline__ T ld_data(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, class T>
__device__ __forceinline__ void st_data(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}
// The same at a per-lane 32-bit byte offset from a workgroup-uniform base:
// the global instruction then takes the base from SGPRs and the offset as is,
// instead of a 64-bit address computed per lane and per access.
template <bool NT, class T>
__device__ __forceinline__ T ld_off(const T* ubase, uint32_t boff) {
  return ld_data<NT>((const T*)((const char*)ubase + boff));
}
template <bool NT, class T>
__device__ __forceinline__ void st_off(T* ubase, uint32_t boff, T v) {
  st_data<NT>((T*)((char*)ubase + boff), v);
}

// ============================================================ column pass
// NC columns per workgroup, N1/V threads per column (V = 2^LV values each);
// columns are adjacent so each row segment read or written is NC words.
// Forward: global stages [0, logN1), out-of-place allowed (in == out is fine).
// Inverse: global stages [logN1-1 .. 0] with the N^-1 fold, canonical output;
// with scale (direct mode), limb l's last stage takes the pair scale[2l],
// scale[2l + 1] in place of table slots 0 and 1 (they also carry the
// Montgomery factor that the fused product left in its input).
template <class A, int LOGN1, int NC, bool FWD, bool IND = false, int LV = 4>
__global__ void __launch_bounds__(NC << (LOGN1 - LV))
k_col(const typename A::word* in, typename A::word* out, const typename A::tw_t* __restrict__ tw_all,
      const typename ModOf<A>::type* __restrict__ mods, uint32_t L, uint32_t logN, uint32_t items,
      const ItemDesc* __restrict__ desc = nullptr, int io = 0,
      const typename A::tw_t* __restrict__ scale = nullptr) {
  using W = typename A::word;
  using TW = typename A::tw_t;
  using M = typename ModOf<A>::type;
  using S = Sched<LOGN1, LV>;
  constexpr int V = 1 << LV;
  constexpr uint32_t N1 = 1u << LOGN1, TPC = N1 / V, LD = NC + 1;
  __shared__ W lds[N1 * LD];
  // forward: the table slots [0, N1) in LDS for the phases after the first,
  // written at the start and published by the first exchange's barrier
  constexpr bool TWL = FWD && S::NPH > 1;
  __shared__ TW twl[TWL ? N1 : 1];
  const uint32_t N2 = 1u << (logN - LOGN1);
  const uint32_t tiles = N2 / NC;
  const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t tile = bid % tiles, item = bid / tiles;
  if (item >= items) return;  // whole workgroup leaves together
  const uint32_t c = threadIdx.x % NC, t = threadIdx.x / NC;
  A a;
  // the column stages use table slots [0, N1) only. In the first phase every
  // thread of the workgroup reads the same slots, which the compiler turns into
  // scalar loads; the forward pass reads the later phases' slots from LDS.
  const TW* tw;
  const TW* t01 = nullptr;
  // src / dst: the tile's first column of the item (workgroup-uniform); a
  // lane's words lie at byte offsets (row * N2 + c) * 8 from them
  const W* src;
  W* dst;
  const size_t off = tile * NC;
  if constexpr (IND) {
    const ItemDesc d = desc[item];
    a.load(*(const M*)d.mod);
    tw = (const TW*)(FWD ? d.tw_fwd : d.tw_inv);
    src = (const W*)(io == IO_SCRATCH_DATA ? d.scratch : d.data) + off;
    dst = (W*)(io == IO_DATA_SCRATCH ? d.scratch : d.data) + off;
  } else {
    const uint32_t l = item % L;
    a.load(mods[l]);
    tw = tw_all + ((size_t)l << logN);
    if (!FWD && scale) t01 = scale + 2 * l;
    const size_t base = ((size_t)item << logN) + off;
    src = in + base;
    dst = out + base;
  }
  // value i of a lane sits in row i * TPC + t (natural) or pos(last phase, t,
  // i) = pos(last phase, t, 0) + (i << lgs): a uniform row step per i and one
  // per-lane byte offset
  constexpr int LGL = S::lgs(S::NPH - 1);
  const uint32_t off_nat = (t * N2 + c) * (uint32_t)sizeof(W);
  const uint32_t off_pos = (pos<LOGN1, LV>(S::NPH - 1, t, 0) * N2 + c) * (uint32_t)sizeof(W);
  W v[V];
  if constexpr (FWD) {
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] = ld_off<NT_LD_IN>(src + (size_t)(i * TPC) * N2, off_nat);
    if constexpr (TWL) {
      for (uint32_t k = threadIdx.x; k < N1; k += blockDim.x) twl[k] = tw[k];
    }
    static_for<0, S::NPH>([&](auto P_) {
      constexpr int p = decltype(P_)::value;
      if constexpr (p > 0) {
        if constexpr (p > 1) __syncthreads();
#pragma unroll
        for (int i = 0; i < V; ++i) lds[pos<LOGN1, LV>(p - 1, t, i) * LD + c] = v[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = lds[pos<LOGN1, LV>(p, t, i) * LD + c];
        ct_phase<A, S::rs(p), rp_of<A>(RP_FRESH), S::s0(p)>(a, v, twl, S::s0(p), grp<LOGN1, LV>(p, t));
      } else {
        ct_phase<A, S::rs(p), rp_of<A>(RP_FRESH), 0>(a, v, tw, 0u, 0u);
      }
    });
#pragma unroll
    for (int i = 0; i < V; ++i) st_off<NT_ST_MID>(dst + ((size_t)i << LGL) * N2, off_pos, v[i]);
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] = ld_off<NT_LD_MID>(src + ((size_t)i << LGL) * N2, off_pos);
    static_for_down<S::NPH - 1, 0>([&](auto P_) {
      constexpr int p = decltype(P_)::value;
      if constexpr (p < S::NPH - 1) {
        if constexpr (p < S::NPH - 2) __syncthreads();
#pragma unroll
        for (int i = 0; i < V; ++i) lds[pos<LOGN1, LV>(p + 1, t, i) * LD + c] = v[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = lds[pos<LOGN1, LV>(p, t, i) * LD + c];
      }
      gs_phase<A, S::rs(p), p == 0>(a, v, tw, S::s0(p), p == 0 ? 0u : grp<LOGN1, LV>(p, t), t01);
    });
#pragma unroll
    for (int i = 0; i < V; ++i) st_off<NT_ST_INV_OUT>(dst + (size_t)(i * TPC) * N2, off_nat, a.canon_inv(v[i]));
  }
}

// ------------------------------------------- first-phase twiddles of a row
// The first phase of a row (stages logN1 .. logN1 + rs(0) - 1) uses the
// 2^rs(0) - 1 twiddles of the row's own subtree: slot 2^k + j of row r is
// table entry 2^(logN1 + k) + (r << k) + j. Each wave copies those of its own
// 64 / TPR rows into LDS (lane q * 2^rs(0) + u: row q, slot u; at most 64
// lanes for every LOGN2 from 6 to 9 and 8 or 16 values per thread; rows
// padded to 17 entries so the wave's rows fall in different LDS banks) and
// orders the copy with the wavefront sync it already needs, so that phase
// reads no twiddle from global memory between butterflies. row_of(rl) is the
// matrix row of workgroup row rl. The copy comes in two halves: load() reads
// this lane's entry (if it has one) and put() writes it to LDS, so that the
// data loads can be issued in between: loads complete in order, and the write
// then waits for the twiddle alone.
template <int LOGN2, int LV, class TW>
struct FirstPhaseStage {
  static constexpr uint32_t TPR = (1u << LOGN2) >> LV, RPW = 64 / TPR, RS0 = Sched<LOGN2, LV>::rs(0),
                            SL = 1u << RS0;
  static_assert(RPW * SL <= 64 && SL <= 16, "one lane per first-phase twiddle of the wave's rows");
  uint32_t rl = 0, u = 0;
  bool has = false;
  TW e{};
  template <class F>
  __device__ __forceinline__ void load(const TW* tw, uint32_t logN1, F row_of) {
    const uint32_t lane = threadIdx.x & 63u, q = lane / SL;
    u = lane % SL;
    rl = (threadIdx.x >> 6) * RPW + q;  // the rows this wave transforms
    has = q < RPW && u;
    if (has) {
      const uint32_t k = 31u - (uint32_t)__builtin_clz(u), j = u - (1u << k);
      e = tw[(1u << (logN1 + k)) + (row_of(rl) << k) + j];
    }
  }
  __device__ __forceinline__ void put(TW (*tw0)[17]) const {
    if (has) tw0[rl][u] = e;
  }
  // the same, with row rl's entries at row_base(rl) (see row_tw0)
  template <class F>
  __device__ __forceinline__ void put_rows(F row_base) const {
    if (has) row_base(rl)[u] = e;
  }
};

// Where the forward split-twist row pass keeps the 17 first-phase twiddles of
// workgroup row rl: inside that row's own exchange area (RSTR words from
// rl * RSTR), which only the wave that owns the row touches, and only before
// its first exchange write. That saves a separate array of 16 * 17 entries,
// and so admits a fourth workgroup per CU at N2 = 2^8 (3.5% faster). The
// entries start 16-byte aligned, at dword bank 8 * (rl mod 4), so that the
// rows of a wave read them in different banks. (The inverse pass could keep
// them there too, after its last exchange read; its extra workgroup made it
// 2% slower, and the two-stream step too.)
template <uint32_t RSTR, class TW, class W>
__device__ __forceinline__ TW* row_tw0(W* lds, uint32_t rl) {
  constexpr uint32_t RB = RSTR * sizeof(W);
  static_assert(RB >= 15 + 112 + 17 * sizeof(TW), "room for 17 entries in a row's area");
  const uint32_t b0 = (rl * RB + 15u) & ~15u;
  const uint32_t shift = (32u * (rl & 3u) - b0) & 127u;
  return reinterpret_cast<TW*>(reinterpret_cast<char*>(lds) + b0 + shift);
}
template <int LOGN2, int LV, class TW, class F>
__device__ __forceinline__ void stage_first_phase(TW (*tw0)[17], const TW* tw, uint32_t logN1, F row_of) {
  FirstPhaseStage<LOGN2, LV, TW> st;
  st.load(tw, logN1, row_of);
  st.put(tw0);
}

// ============================================================ row pass
// 16 rows per workgroup, N2/V threads per row (V = 2^LV values each; a row
// never spans two waves, so exchanges between phases only need wavefront
// ordering).
// Forward: global stages [logN1, logN), canonical output; NATURAL writes
// element (r, c) to brv(c) * N1 + brv(r) with rows r = brv(k1), k1 in the tile.
// Inverse: reads that layout (or rows in place), runs the row stages
// backwards and writes rows in lazy range for the column pass.
// MULIN (inverse only, direct mode): the input is in * in2 * 2^-w elementwise
// mod q (the pointwise product fused into the load as a Montgomery product,
// w the word size), read from two buffers; the column pass that follows
// multiplies the factor 2^w back in with its scaled last-stage pair.
template <class A, int LOGN2, bool FWD, bool NATURAL, bool MULIN = false, bool IND = false, int LV = 4>
__global__ void __launch_bounds__(16 << (LOGN2 - LV))
k_row(const typename A::word* in, typename A::word* out, const typename A::tw_t* __restrict__ tw_all,
      const typename ModOf<A>::type* __restrict__ mods, uint32_t L, uint32_t logN, uint32_t items,
      uint32_t batch, const typename A::word* in2 = nullptr, const ItemDesc* __restrict__ desc = nullptr,
      int io = 0) {
  using W = typename A::word;
  using TW = typename A::tw_t;
  using M = typename ModOf<A>::type;
  using S = Sched<LOGN2, LV>;
  constexpr int V = 1 << LV;
  constexpr uint32_t N2 = 1u << LOGN2, TPR = N2 / V, RSTR = N2 + N2 / 16 + 1;
  static_assert(TPR <= 64, "a row must fit in one wavefront");
  static_assert(!(MULIN && (FWD || IND)), "the fused product runs with the direct-mode inverse");
  __shared__ W lds[16 * RSTR];
  __shared__ TW tw0[16][17];  // first-phase twiddles of the 16 rows
  const uint32_t logN1 = logN - LOGN2, N1 = 1u << logN1;
  const uint32_t tiles = N1 / 16;
  // logical order (limb, tile, poly): the polynomials sharing a limb's row
  // twiddles run back to back on one XCD
  const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t b = bid % batch, rest = bid / batch;
  const uint32_t tile = rest % tiles, l = rest / tiles;
  if (l >= L) return;
  const uint32_t item = b * L + l;
  const uint32_t t = threadIdx.x % TPR, rl = threadIdx.x / TPR;
  const uint32_t k1 = tile * 16 + rl;
  const uint32_t r = NATURAL ? brv(k1, logN1) : k1;
  A a;
  const M* mi;
  const TW* tw;
  size_t pbase;
  if constexpr (IND) {
    // indirect mode: in/out are rebased per item, pbase = 0
    const ItemDesc d = desc[item];
    mi = (const M*)d.mod;
    tw = (const TW*)(FWD ? d.tw_fwd : d.tw_inv);
    in = (const W*)(io == IO_SCRATCH_DATA ? d.scratch : d.data);
    out = (W*)(io == IO_DATA_SCRATCH ? d.scratch : d.data);
    pbase = 0;
  } else {
    mi = mods + l;
    tw = tw_all + ((size_t)l << logN);
    pbase = (size_t)item << logN;
  }
  a.load(*mi);
  W* sh = lds + rl * RSTR;
  W v[V];
  // the first-phase twiddles are loaded before the data and written to LDS
  // after the data loads are issued, so that neither waits for the other
  FirstPhaseStage<LOGN2, LV, TW> first;
  first.load(tw, logN1, [&](uint32_t row) { return NATURAL ? brv(tile * 16 + row, logN1) : tile * 16 + row; });
  __builtin_amdgcn_sched_barrier(0);
  auto stage = [&]() { first.put(tw0); };
  if constexpr (FWD) {
    const W* src = in + pbase + (size_t)r * N2;
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] = ld_data<NT_LD_MID>(src + i * TPR + t);
    stage();
    wave_lds_sync();
    static_for<0, S::NPH>([&](auto P_) {
      constexpr int p = decltype(P_)::value;
      if constexpr (p > 0) {
        if constexpr (p > 1) wave_lds_sync();
#pragma unroll
        for (int i = 0; i < V; ++i) sh[pad16(pos<LOGN2, LV>(p - 1, t, i))] = v[i];
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = sh[pad16(pos<LOGN2, LV>(p, t, i))];
        ct_phase<A, S::rs(p), rp_of<A>(RP_LAZY), S::s0(p)>(a, v, tw, logN1 + S::s0(p),
                                                           (r << S::s0(p)) + grp<LOGN2, LV>(p, t));
      } else {
        ct_phase<A, S::rs(p), rp_of<A>(RP_LAZY), 0>(a, v, &tw0[rl][0], 0u, 0u);
      }
    });
    if constexpr (NATURAL) {
      if (S::NPH > 1) wave_lds_sync();
#pragma unroll
      for (int i = 0; i < V; ++i) sh[pad16(pos<LOGN2, LV>(S::NPH - 1, t, i))] = a.canon_fwd(v[i]);
      __syncthreads();
      const uint32_t rr = threadIdx.x % 16, cg = threadIdx.x / 16;
      // column cc = cg + TPR j goes to row brv(cc) = brv(cg) + brv(TPR j) (disjoint
      // bits): a uniform base per j and one byte offset per lane
      W* dst = out + pbase + tile * 16;
      const uint32_t lane_off = (rr + brv(cg, LOGN2) * N1) * (uint32_t)sizeof(W);
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const uint32_t cc = cg + TPR * j;
        st_off<NT_ST_OUT>(dst + (size_t)brv(TPR * j, LOGN2) * N1, lane_off, lds[rr * RSTR + pad16(cc)]);
      }
    } else {
      if (S::NPH > 1) wave_lds_sync();
#pragma unroll
      for (int i = 0; i < V; ++i) sh[pad16(pos<LOGN2, LV>(S::NPH - 1, t, i))] = a.canon_fwd(v[i]);
      wave_lds_sync();
      W* dst = out + pbase + (size_t)r * N2;
#pragma unroll
      for (int i = 0; i < V; ++i) st_data<NT_ST_OUT>(dst + i * TPR + t, sh[pad16(i * TPR + t)]);
    }
  } else {
    if constexpr (NATURAL) {
      const uint32_t rr = threadIdx.x % 16, cg = threadIdx.x / 16;
      // row brv(cg + TPR j) = brv(cg) + brv(TPR j): a uniform base per j and one
      // byte offset per lane
      const size_t off = pbase + tile * 16;
      const W* src = in + off;
      const uint32_t lane_off = (rr + brv(cg, LOGN2) * N1) * (uint32_t)sizeof(W);
      // every load is issued before the first product, so that a wave has all
      // of its loads in flight at once rather than one pair per product
      W xa[V], xb[MULIN ? V : 1];
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const size_t e = (size_t)brv(TPR * j, LOGN2) * N1;
        xa[j] = ld_off<NT_LD_IN>(src + e, lane_off);
        if constexpr (MULIN) xb[j] = ld_off<NT_LD_IN>(in2 + off + e, lane_off);
      }
      stage();
#pragma unroll
      for (int j = 0; j < V; ++j) {
        W val = xa[j];
        if constexpr (MULIN) val = mulmod_mont(val, xb[j], *mi);
        lds[rr * RSTR + pad16(cg + TPR * j)] = val;
      }
      __syncthreads();
    } else {
      const size_t off = pbase + (size_t)r * N2;
      const W* src = in + off;
      W xa[V], xb[MULIN ? V : 1];
#pragma unroll
      for (int i = 0; i < V; ++i) {
        xa[i] = ld_data<NT_LD_IN>(src + i * TPR + t);
        if constexpr (MULIN) xb[i] = ld_data<NT_LD_IN>(in2 + off + i * TPR + t);
      }
      stage();
#pragma unroll
      for (int i = 0; i < V; ++i) {
        W val = xa[i];
        if constexpr (MULIN) val = mulmod_mont(val, xb[i], *mi);
        sh[pad16(i * TPR + t)] = val;
      }
      wave_lds_sync();
    }
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] = sh[pad16(pos<LOGN2, LV>(S::NPH - 1, t, i))];
    static_for_down<S::NPH - 1, 0>([&](auto P_) {
      constexpr int p = decltype(P_)::value;
      if constexpr (p < S::NPH - 1) {
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < V; ++i) sh[pad16(pos<LOGN2, LV>(p + 1, t, i))] = v[i];
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = sh[pad16(pos<LOGN2, LV>(p, t, i))];
      }
      if constexpr (p == 0) gs_phase<A, S::rs(p), false>(a, v, &tw0[rl][0], 0u, 0u);
      else gs_phase<A, S::rs(p), false>(a, v, tw, logN1 + S::s0(p), (r << S::s0(p)) + grp<LOGN2, LV>(p, t));
    });
    W* dst = out + pbase + (size_t)r * N2;
#pragma unroll
    for (int i = 0; i < V; ++i) st_data<NT_ST_MID>(dst + i * TPR + t, v[i]);
  }
}

// ============================================================ twisted row pass
// The rows of k_row by another factorisation. After the column stages, row r
// holds the input reduced modulo x^N2 - beta_r^N2 with beta_r =
// psi^(2 brv(r) + 1), and its outputs are the values at beta_r * omega^brv(c),
// omega = psi^(2 N1). So the row is multiplied elementwise by beta_r^j (the
// twist: one table entry per element) and then transformed by a cyclic NTT of
// length N2 whose twiddles are the same for every row. Those N2 entries are
// staged once per workgroup in LDS, so no twiddle is fetched from global
// memory between butterflies (the merged-twiddle row pass reads a different
// subtree of twiddles for every row, too many for LDS). In the first phase
// every group 0 has twiddle 1 and takes the unit butterfly, which pays for the
// twist's products. The forward pass multiplies by the twist on load (those
// loads join the data loads); the inverse multiplies by beta_r^-j before the
// store, so its twist loads overlap the last phase.
// Tables: twist[l][N], entry r * N2 + j = beta_r^j (forward) or beta_r^-j
// (inverse); cyc[l][N2], the cyclic table of length N2 for omega (forward) or
// its inverse (slots 0 and 1 are never read). The inverse runs the cyclic
// inverse and multiplies by beta_r^-j before the store; the factor N^-1 stays
// with the column pass.
// LDS position of cyclic-table slot m = 2^s + g for a row of 2^LOGN2. Stage s
// lies in the phase that starts at stage S0 (k = s - S0); there the thread of
// phase group Hg reads group g = (Hg << k) + j, so the groups are stored as
// (j << S0) + Hg: for each j, the lanes of a row read consecutive entries
// instead of entries 2^k apart (which fall in the same LDS banks).
template <int LOGN2, int LV = 4>
__device__ __forceinline__ uint32_t cyc_pos(uint32_t m) {
  using S = Sched<LOGN2, LV>;
  if (m < 2) return m;
  const uint32_t s = 31u - (uint32_t)__builtin_clz(m);
  const uint32_t S0 = (S::R0 && s < (uint32_t)S::R0) ? 0u : (S::R0 ? S::R0 + ((s - S::R0) / LV) * LV : (s / LV) * LV);
  const uint32_t k = s - S0, g = m - (1u << s);
  return (1u << s) + ((g & ((1u << k) - 1u)) << S0) + (g >> k);
}

template <class A, int RS, bool FIRST, int RP = RP_ALL, int J0 = 0, int V>
__device__ __forceinline__ void ct_phase_cyc(const A& a, typename A::word (&v)[V], const typename A::tw_t* tw,
                                             uint32_t S0, uint32_t Hg) {
  static_for<0, RS>([&](auto K_) {
    constexpr int k = decltype(K_)::value;
    constexpr bool RED = reduces_x(RP, J0 + k);
#pragma unroll
    for (int j = 0; j < (1 << k); ++j) {
      if (FIRST && j == 0) {
#pragma unroll
        for (int m = 0; m < ((V / 2) >> k); ++m) a.template ct1<RED>(v[m], v[m + ((V / 2) >> k)]);
      } else {
        const typename A::tw_t w = tw[(1u << (S0 + k)) + ((uint32_t)j << S0) + Hg];  // see cyc_pos
#pragma unroll
        for (int m = 0; m < ((V / 2) >> k); ++m) {
          const int i0 = j * (V >> k) + m;
          a.template ct<RED>(v[i0], v[i0 + ((V / 2) >> k)], w);
        }
      }
    }
  });
}
template <class A, int RS, bool FIRST, int V>
__device__ __forceinline__ void gs_phase_cyc(const A& a, typename A::word (&v)[V], const typename A::tw_t* tw,
                                             uint32_t S0, uint32_t Hg) {
#pragma unroll
  for (int k = RS - 1; k >= 0; --k) {
#pragma unroll
    for (int j = 0; j < (1 << k); ++j) {
      if (FIRST && j == 0) {
#pragma unroll
        for (int m = 0; m < ((V / 2) >> k); ++m) a.gs1(v[m], v[m + ((V / 2) >> k)]);
      } else {
        const typename A::tw_t w = tw[(1u << (S0 + k)) + ((uint32_t)j << S0) + Hg];  // see cyc_pos
#pragma unroll
        for (int m = 0; m < ((V / 2) >> k); ++m) {
          const int i0 = j * (V >> k) + m;
          a.gs(v[i0], v[i0 + ((V / 2) >> k)], w);
        }
      }
    }
  }
}

template <class A, int LOGN2, bool FWD, bool NATURAL, bool MULIN = false, int LV = 4>
__global__ void __launch_bounds__(16 << (LOGN2 - LV))
k_row_tw(const typename A::word* in, typename A::word* out, const typename A::tw_t* __restrict__ twist_all,
         const typename A::tw_t* __restrict__ cyc_all, const typename ModOf<A>::type* __restrict__ mods,
         uint32_t L, uint32_t logN, uint32_t batch, const typename A::word* in2 = nullptr) {
  using W = typename A::word;
  using TW = typename A::tw_t;
  using S = Sched<LOGN2, LV>;
  constexpr int V = 1 << LV;
  constexpr uint32_t N2 = 1u << LOGN2, TPR = N2 / V, RSTR = N2 + N2 / 16 + 1;
  static_assert(TPR <= 64, "a row must fit in one wavefront");
  __shared__ W lds[16 * RSTR];
  __shared__ TW cyc[N2];  // entry k written by thread k (the workgroup has N2 or 2 N2 threads)
  const uint32_t logN1 = logN - LOGN2, N1 = 1u << logN1;
  const uint32_t tiles = N1 / 16;
  const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t b = bid % batch, rest = bid / batch;
  const uint32_t tile = rest % tiles, l = rest / tiles;
  if (l >= L) return;  // whole workgroup leaves together
  const uint32_t item = b * L + l;
  const uint32_t t = threadIdx.x % TPR, rl = threadIdx.x / TPR;
  const uint32_t k1 = tile * 16 + rl;
  const uint32_t r = NATURAL ? brv(k1, logN1) : k1;
  A a;
  const auto* mi = mods + l;
  a.load(*mi);
  const bool has_entry = threadIdx.x < N2;
  const TW cyc_entry = cyc_all[((size_t)l << LOGN2) + (has_entry ? threadIdx.x : 0u)];
  const TW* twist = twist_all + ((size_t)l << logN) + (size_t)r * N2;
  const size_t pbase = (size_t)item << logN;
  W* sh = lds + rl * RSTR;
  W v[V];
  if constexpr (FWD) {
    const W* src = in + pbase + (size_t)r * N2;
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] = ld_data<NT_LD_MID>(src + i * TPR + t);
    if (has_entry) cyc[cyc_pos<LOGN2, LV>(threadIdx.x)] = cyc_entry;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] = a.mul(v[i], twist[i * TPR + t]);
    static_for<0, S::NPH>([&](auto P_) {
      constexpr int p = decltype(P_)::value;
      if constexpr (p > 0) {
        if constexpr (p > 1) wave_lds_sync();
#pragma unroll
        for (int i = 0; i < V; ++i) sh[pad16(pos<LOGN2, LV>(p - 1, t, i))] = v[i];
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = sh[pad16(pos<LOGN2, LV>(p, t, i))];
      }
      ct_phase_cyc<A, S::rs(p), p == 0, rp_of<A>(RP_FRESH), S::s0(p)>(a, v, cyc, S::s0(p), grp<LOGN2, LV>(p, t));
    });
    if constexpr (NATURAL) {
      if (S::NPH > 1) wave_lds_sync();
#pragma unroll
      for (int i = 0; i < V; ++i) sh[pad16(pos<LOGN2, LV>(S::NPH - 1, t, i))] = a.canon_fwd(v[i]);
      __syncthreads();
      const uint32_t rr = threadIdx.x % 16, cg = threadIdx.x / 16;
      // column cc = cg + TPR j goes to row brv(cc) = brv(cg) + brv(TPR j) (disjoint
      // bits): a uniform base per j and one byte offset per lane
      W* dst = out + pbase + tile * 16;
      const uint32_t lane_off = (rr + brv(cg, LOGN2) * N1) * (uint32_t)sizeof(W);
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const uint32_t cc = cg + TPR * j;
        st_off<NT_ST_OUT>(dst + (size_t)brv(TPR * j, LOGN2) * N1, lane_off, lds[rr * RSTR + pad16(cc)]);
      }
    } else {
      if (S::NPH > 1) wave_lds_sync();
#pragma unroll
      for (int i = 0; i < V; ++i) sh[pad16(pos<LOGN2, LV>(S::NPH - 1, t, i))] = a.canon_fwd(v[i]);
      wave_lds_sync();
      W* dst = out + pbase + (size_t)r * N2;
#pragma unroll
      for (int i = 0; i < V; ++i) st_data<NT_ST_OUT>(dst + i * TPR + t, sh[pad16(i * TPR + t)]);
    }
  } else {
    if (has_entry) cyc[cyc_pos<LOGN2, LV>(threadIdx.x)] = cyc_entry;
    if constexpr (NATURAL) {
      const uint32_t rr = threadIdx.x % 16, cg = threadIdx.x / 16;
      // row brv(cg + TPR j) = brv(cg) + brv(TPR j): a uniform base per j and one
      // byte offset per lane
      const size_t off = pbase + tile * 16;
      const W* src = in + off;
      const uint32_t lane_off = (rr + brv(cg, LOGN2) * N1) * (uint32_t)sizeof(W);
      // every load is issued before the first product, so that a wave has all
      // of its loads in flight at once rather than one pair per product
      W xa[V], xb[MULIN ? V : 1];
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const size_t e = (size_t)brv(TPR * j, LOGN2) * N1;
        xa[j] = ld_off<NT_LD_IN>(src + e, lane_off);
        if constexpr (MULIN) xb[j] = ld_off<NT_LD_IN>(in2 + off + e, lane_off);
      }
#pragma unroll
      for (int j = 0; j < V; ++j) {
        W val = xa[j];
        if constexpr (MULIN) val = mulmod_mont(val, xb[j], *mi);
        lds[rr * RSTR + pad16(cg + TPR * j)] = val;
      }
      __syncthreads();
    } else {
      const size_t off = pbase + (size_t)r * N2;
      const W* src = in + off;
      W xa[V], xb[MULIN ? V : 1];
#pragma unroll
      for (int i = 0; i < V; ++i) {
        xa[i] = ld_data<NT_LD_IN>(src + i * TPR + t);
        if constexpr (MULIN) xb[i] = ld_data<NT_LD_IN>(in2 + off + i * TPR + t);
      }
#pragma unroll
      for (int i = 0; i < V; ++i) {
        W val = xa[i];
        if constexpr (MULIN) val = mulmod_mont(val, xb[i], *mi);
        sh[pad16(i * TPR + t)] = val;
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] = sh[pad16(pos<LOGN2, LV>(S::NPH - 1, t, i))];
    static_for_down<S::NPH - 1, 0>([&](auto P_) {
      constexpr int p = decltype(P_)::value;
      if constexpr (p < S::NPH - 1) {
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < V; ++i) sh[pad16(pos<LOGN2, LV>(p + 1, t, i))] = v[i];
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = sh[pad16(pos<LOGN2, LV>(p, t, i))];
      }
      gs_phase_cyc<A, S::rs(p), p == 0>(a, v, cyc, S::s0(p), grp<LOGN2, LV>(p, t));
    });
    // first-phase layout: value i of thread t is row element i * TPR + t
    W* dst = out + pbase + (size_t)r * N2;
#pragma unroll
    for (int i = 0; i < V; ++i) st_data<NT_ST_MID>(dst + i * TPR + t, a.mul(v[i], twist[i * TPR + t]));
  }
}

#ifndef NTT_ROW_SHUFFLE
#define NTT_ROW_SHUFFLE 0
#endif
#if NTT_ROW_SHUFFLE
// 32-bit value of lane (lane ^ m) within a row of 16 lanes
template <int M>
__device__ __forceinline__ uint32_t xor_lane32(uint32_t x) {
  if constexpr (M == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, true);  // quad_perm 1,0,3,2
  else if constexpr (M == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, true);  // 2,3,0,1
  else return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, (M << 10) | 0x1F);  // bit mode, xor M
}
// the 16 x 16 transpose between phases done across lanes instead of through
// LDS: lane t's value j becomes lane j's value t, in four swap stages
__device__ __forceinline__ void transpose_lanes16(uint64_t (&v)[16], uint32_t t) {
  static_for<0, 4>([&](auto K_) {
    constexpr int m = 8 >> decltype(K_)::value;
    const bool hi = (t & m) != 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (j & m) continue;
      const uint64_t send = hi ? v[j] : v[j | m];
      const uint64_t recv = ((uint64_t)xor_lane32<m>((uint32_t)(send >> 32)) << 32) | xor_lane32<m>((uint32_t)send);
      v[j] = hi ? recv : v[j];
      v[j | m] = hi ? v[j | m] : recv;
    }
  });
}
#endif

// ============================================================ split-twist row passes
// The rows of k_row_tw with the twist split in two. After the first P row
// stages (P: those of the first register phase), the twisted row's state is
// the merged row's state times beta_r^(c mod 2^(LOGN2 - P)) at row position c
// (checked numerically for several splits). So the forward pass runs its
// first phase merged, with the row's own subtree of twiddles staged in LDS as
// in k_row; multiplies each value by beta_r^(c mod 2^(LOGN2 - P)); and runs
// the later phases as the cyclic transform of k_row_tw, whose twiddles every
// row shares and which sit in LDS. In the first phase's layout value i of
// thread t is row position (i << lg) + t with lg = LOGN2 - LV, so its factor
// is entry (f << lg) + t of the row's twist table, f = i mod NF, NF =
// 2^(LV - P): one or a few entries per thread instead of one per value. The
// inverse runs the same steps backwards: the cyclic inverse phases, the
// factors beta_r^-(...), and the first phase merged. No twiddle is read from
// global memory between butterflies, and a row reads 2^P - 1 + NF * TPR
// table entries instead of N2.
template <int LOGN2, int LV>
struct SplitTwist {
  using S = Sched<LOGN2, LV>;
  static constexpr int P = S::rs(0);           // stages of the merged first phase
  static constexpr int NF = 1 << (LV - P);     // distinct twist factors per thread
  static constexpr uint32_t LG = LOGN2 - LV;   // log2 of the first phase's stride
};

template <class A, int LOGN2, bool NATURAL, int LV = 4>
__global__ void __launch_bounds__(16 << (LOGN2 - LV))
k_row_st(const typename A::word* in, typename A::word* out, const typename A::tw_t* __restrict__ tw_all,
         const typename A::tw_t* __restrict__ twist_all, const typename A::tw_t* __restrict__ cyc_all,
         const typename ModOf<A>::type* __restrict__ mods, uint32_t L, uint32_t logN, uint32_t batch) {
  using W = typename A::word;
  using TW = typename A::tw_t;
  using S = Sched<LOGN2, LV>;
  using ST = SplitTwist<LOGN2, LV>;
  constexpr int V = 1 << LV;
  constexpr uint32_t N2 = 1u << LOGN2, TPR = N2 / V, RSTR = N2 + N2 / 16 + 1;
  static_assert(TPR <= 64, "a row must fit in one wavefront");
  __shared__ __align__(16) W lds[16 * RSTR];  // also the rows' first-phase twiddles (row_tw0)
  __shared__ TW cyc[N2];                      // cyclic twiddles, entry k written by thread k
  const uint32_t logN1 = logN - LOGN2, N1 = 1u << logN1;
  const uint32_t tiles = N1 / 16;
  const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t b = bid % batch, rest = bid / batch;
  const uint32_t tile = rest % tiles, l = rest / tiles;
  if (l >= L) return;  // whole workgroup leaves together
  const uint32_t item = b * L + l;
  const uint32_t t = threadIdx.x % TPR, rl = threadIdx.x / TPR;
  const uint32_t k1 = tile * 16 + rl;
  const uint32_t r = NATURAL ? brv(k1, logN1) : k1;
  A a;
  a.load(mods[l]);
  const TW* tw = tw_all + ((size_t)l << logN);
  const bool has_entry = threadIdx.x < N2;
  const TW cyc_entry = cyc_all[((size_t)l << LOGN2) + (has_entry ? threadIdx.x : 0u)];
  const TW* trow = twist_all + ((size_t)l << logN) + (size_t)r * N2 + t;
  TW bt[ST::NF];  // beta_r^((f << lg) + t)
#pragma unroll
  for (int f = 0; f < ST::NF; ++f) bt[f] = trow[f << ST::LG];
  FirstPhaseStage<LOGN2, LV, TW> first;
  first.load(tw, logN1, [&](uint32_t row) { return NATURAL ? brv(tile * 16 + row, logN1) : tile * 16 + row; });
  __builtin_amdgcn_sched_barrier(0);
  const size_t pbase = (size_t)item << logN;
  W* sh = lds + rl * RSTR;
  W v[V];
  const W* src = in + pbase + (size_t)r * N2;
#pragma unroll
  for (int i = 0; i < V; ++i) v[i] = ld_data<NT_LD_MID>(src + i * TPR + t);
  first.put_rows([&](uint32_t row) { return row_tw0<RSTR, TW>(lds, row); });
  if (has_entry) cyc[cyc_pos<LOGN2, LV>(threadIdx.x)] = cyc_entry;
  __syncthreads();
  // the merged first phase (input anywhere in the column pass's output range);
  // its twiddle reads precede the row's first exchange write below, in the
  // same wave and on the same array, so they keep their order
  ct_phase<A, ST::P, rp_of<A>(RP_LAZY), 0>(a, v, row_tw0<RSTR, TW>(lds, rl), 0u, 0u);
  // the rest of the twist: now below L
#pragma unroll
  for (int i = 0; i < V; ++i) v[i] = a.mul(v[i], bt[i & (ST::NF - 1)]);
  static_for<1, S::NPH>([&](auto P_) {
    constexpr int p = decltype(P_)::value;
#if NTT_ROW_SHUFFLE
    if constexpr (p == 1 && S::NPH == 2 && V == 16 && TPR == 16 && sizeof(W) == 8) {
      transpose_lanes16(v, t);
    } else
#endif
    {
      if constexpr (p > 1) wave_lds_sync();
#pragma unroll
      for (int i = 0; i < V; ++i) sh[pad16(pos<LOGN2, LV>(p - 1, t, i))] = v[i];
      wave_lds_sync();
#pragma unroll
      for (int i = 0; i < V; ++i) v[i] = sh[pad16(pos<LOGN2, LV>(p, t, i))];
    }
    ct_phase_cyc<A, S::rs(p), false, rp_of<A>(RP_FRESH), S::s0(p) - ST::P>(a, v, cyc, S::s0(p),
                                                                           grp<LOGN2, LV>(p, t));
  });
  if constexpr (NATURAL) {
    if (S::NPH > 1) wave_lds_sync();
#pragma unroll
    for (int i = 0; i < V; ++i) sh[pad16(pos<LOGN2, LV>(S::NPH - 1, t, i))] = a.canon_fwd(v[i]);
    __syncthreads();
    const uint32_t rr = threadIdx.x % 16, cg = threadIdx.x / 16;
    // column cc = cg + TPR j goes to row brv(cc) = brv(cg) + brv(TPR j) (disjoint
    // bits): a uniform base per j and one byte offset per lane
    W* dst = out + pbase + tile * 16;
    const uint32_t lane_off = (rr + brv(cg, LOGN2) * N1) * (uint32_t)sizeof(W);
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const uint32_t cc = cg + TPR * j;
      st_off<NT_ST_OUT>(dst + (size_t)brv(TPR * j, LOGN2) * N1, lane_off, lds[rr * RSTR + pad16(cc)]);
    }
  } else {
    if (S::NPH > 1) wave_lds_sync();
#pragma unroll
    for (int i = 0; i < V; ++i) sh[pad16(pos<LOGN2, LV>(S::NPH - 1, t, i))] = a.canon_fwd(v[i]);
    wave_lds_sync();
    W* dst = out + pbase + (size_t)r * N2;
#pragma unroll
    for (int i = 0; i < V; ++i) st_data<NT_ST_OUT>(dst + i * TPR + t, sh[pad16(i * TPR + t)]);
  }
}

// Lane map of the inverse row pass's phases. A phase whose groups hold 8
// offsets (stride 2^3) with 8 values per thread places, under the identity
// t = (group << 3) + offset, two groups in each 16-lane LDS cycle: their
// 8-word runs lie 64 + 4 padded words apart and share half their banks. The
// map below gives each 16 lanes two offset bits and two group bits, so the
// four groups' runs start 0, 4, 8 and 12 words apart (mod 16) and the 16
// 64-bit accesses cover the 32 banks once. It is a permutation of [0, TPR):
// lane bits 0-1 -> offset bits 0-1, 4 -> offset bit 2, 2-3 -> group bits 0-1,
// 5 -> group bit 2. Rows of 16 lanes (one 16-lane cycle per row whatever the
// map) keep the identity.
#ifndef NTT_ROW_INV_LANES
#define NTT_ROW_INV_LANES 1
#endif
template <int LOGN2, int LV>
__device__ __forceinline__ uint32_t row_inv_lane(int p, uint32_t t) {
  constexpr uint32_t TPR = (1u << LOGN2) >> LV;
  if (!NTT_ROW_INV_LANES || LV != 3 || TPR < 32 || Sched<LOGN2, LV>::lgs(p) != 3) return t;
  const uint32_t off = (t & 3u) | (((t >> 4) & 1u) << 2);
  const uint32_t g = ((t >> 2) & 3u) | ((t >> 5) << 2);
  return (g << 3) | off;
}

// Inverse: the spectrum rows (or with MULIN the Montgomery product of two, as
// in k_row) through the cyclic inverse phases, the factors beta_r^-(...), and
// the merged inverse first phase; rows written in place, in the lazy range the
// column pass takes.
template <class A, int LOGN2, bool NATURAL, bool MULIN, int LV = 3>
__global__ void __launch_bounds__(16 << (LOGN2 - LV))
k_row_st_inv(const typename A::word* in, typename A::word* out, const typename A::tw_t* __restrict__ tw_all,
             const typename A::tw_t* __restrict__ twist_all, const typename A::tw_t* __restrict__ cyc_all,
             const typename ModOf<A>::type* __restrict__ mods, uint32_t L, uint32_t logN, uint32_t batch,
             const typename A::word* in2 = nullptr) {
  using W = typename A::word;
  using TW = typename A::tw_t;
  using S = Sched<LOGN2, LV>;
  using ST = SplitTwist<LOGN2, LV>;
  constexpr int V = 1 << LV;
  constexpr uint32_t N2 = 1u << LOGN2, TPR = N2 / V, RSTR = N2 + N2 / 16 + 1;
  static_assert(TPR <= 64, "a row must fit in one wavefront");
  static_assert(S::NPH > 1, "a cyclic phase before the merged one");
  __shared__ W lds[16 * RSTR];
  __shared__ TW tw0[16][17];
  __shared__ TW cyc[N2];
  const uint32_t logN1 = logN - LOGN2, N1 = 1u << logN1;
  const uint32_t tiles = N1 / 16;
  const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t b = bid % batch, rest = bid / batch;
  const uint32_t tile = rest % tiles, l = rest / tiles;
  if (l >= L) return;  // whole workgroup leaves together
  const uint32_t item = b * L + l;
  const uint32_t t = threadIdx.x % TPR, rl = threadIdx.x / TPR;
  const uint32_t k1 = tile * 16 + rl;
  const uint32_t r = NATURAL ? brv(k1, logN1) : k1;
  A a;
  const auto* mi = mods + l;
  a.load(*mi);
  const TW* tw = tw_all + ((size_t)l << logN);
  const bool has_entry = threadIdx.x < N2;
  const TW cyc_entry = cyc_all[((size_t)l << LOGN2) + (has_entry ? threadIdx.x : 0u)];
  FirstPhaseStage<LOGN2, LV, TW> first;
  first.load(tw, logN1, [&](uint32_t row) { return NATURAL ? brv(tile * 16 + row, logN1) : tile * 16 + row; });
  __builtin_amdgcn_sched_barrier(0);
  const size_t pbase = (size_t)item << logN;
  W* sh = lds + rl * RSTR;
  W v[V];
  if constexpr (NATURAL) {
    const uint32_t rr = threadIdx.x % 16, cg = threadIdx.x / 16;
    // row brv(cg + TPR j) = brv(cg) + brv(TPR j): a uniform base per j and one
    // byte offset per lane
    const size_t off = pbase + tile * 16;
    const W* src = in + off;
    const uint32_t lane_off = (rr + brv(cg, LOGN2) * N1) * (uint32_t)sizeof(W);
    W xa[V], xb[MULIN ? V : 1];
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const size_t e = (size_t)brv(TPR * j, LOGN2) * N1;
      xa[j] = ld_off<NT_LD_IN>(src + e, lane_off);
      if constexpr (MULIN) xb[j] = ld_off<NT_LD_IN>(in2 + off + e, lane_off);
    }
    first.put(tw0);
    if (has_entry) cyc[cyc_pos<LOGN2, LV>(threadIdx.x)] = cyc_entry;
#pragma unroll
    for (int j = 0; j < V; ++j) {
      W val = xa[j];
      if constexpr (MULIN) val = mulmod_mont(val, xb[j], *mi);
      lds[rr * RSTR + pad16(cg + TPR * j)] = val;
    }
  } else {
    const size_t off = pbase + (size_t)r * N2;
    const W* src = in + off;
    W xa[V], xb[MULIN ? V : 1];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      xa[i] = ld_data<NT_LD_IN>(src + i * TPR + t);
      if constexpr (MULIN) xb[i] = ld_data<NT_LD_IN>(in2 + off + i * TPR + t);
    }
    first.put(tw0);
    if (has_entry) cyc[cyc_pos<LOGN2, LV>(threadIdx.x)] = cyc_entry;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      W val = xa[i];
      if constexpr (MULIN) val = mulmod_mont(val, xb[i], *mi);
      sh[pad16(i * TPR + t)] = val;
    }
  }
  __syncthreads();
  // twist factors beta_r^-((f << lg) + t), read while the cyclic phases run
  const TW* trow = twist_all + ((size_t)l << logN) + (size_t)r * N2 + t;
  TW bt[ST::NF];
#pragma unroll
  for (int f = 0; f < ST::NF; ++f) bt[f] = trow[f << ST::LG];
#pragma unroll
  for (int i = 0; i < V; ++i) v[i] = sh[pad16(pos<LOGN2, LV>(S::NPH - 1, row_inv_lane<LOGN2, LV>(S::NPH - 1, t), i))];
  static_for_down<S::NPH - 1, 1>([&](auto P_) {
    constexpr int p = decltype(P_)::value;
    const uint32_t tp = row_inv_lane<LOGN2, LV>(p, t);
    if constexpr (p < S::NPH - 1) {
      const uint32_t tq = row_inv_lane<LOGN2, LV>(p + 1, t);
      wave_lds_sync();
#pragma unroll
      for (int i = 0; i < V; ++i) sh[pad16(pos<LOGN2, LV>(p + 1, tq, i))] = v[i];
      wave_lds_sync();
#pragma unroll
      for (int i = 0; i < V; ++i) v[i] = sh[pad16(pos<LOGN2, LV>(p, tp, i))];
    }
    gs_phase_cyc<A, S::rs(p), false>(a, v, cyc, S::s0(p), grp<LOGN2, LV>(p, tp));
  });
  wave_lds_sync();
#pragma unroll
  for (int i = 0; i < V; ++i) sh[pad16(pos<LOGN2, LV>(1, row_inv_lane<LOGN2, LV>(1, t), i))] = v[i];
  wave_lds_sync();
#pragma unroll
  for (int i = 0; i < V; ++i) v[i] = a.mul(sh[pad16(pos<LOGN2, LV>(0, t, i))], bt[i & (ST::NF - 1)]);
  gs_phase<A, ST::P, false>(a, v, &tw0[rl][0], 0u, 0u);
  // first-phase layout: value i of thread t is row element i * TPR + t
  W* dst = out + pbase + (size_t)r * N2;
#pragma unroll
  for (int i = 0; i < V; ++i) st_data<NT_ST_MID>(dst + i * TPR + t, v[i]);
}

// ============================================================ tiny N
// N in {2, 4, 8}: one thread per transform, the same stage structure.
template <class A, int LOGN, bool FWD, bool NATURAL>
__global__ void __launch_bounds__(256)
k_tiny(typename A::word* __restrict__ data, const typename A::tw_t* __restrict__ tw_all,
       const typename ModOf<A>::type* __restrict__ mods, uint32_t L, uint32_t items) {
  using W = typename A::word;
  constexpr uint32_t N = 1u << LOGN;
  const uint32_t item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= items) return;
  const uint32_t l = item % L;
  A a;
  a.load(mods[l]);
  const typename A::tw_t* tw = tw_all + ((size_t)l << LOGN);
  W* x = data + ((size_t)item << LOGN);
  W v[N];
  if constexpr (FWD) {
#pragma unroll
    for (uint32_t i = 0; i < N; ++i) v[i] = x[i];
#pragma unroll
    for (int s = 0; s < LOGN; ++s) {
      const uint32_t h = N >> (s + 1);
#pragma unroll
      for (uint32_t g = 0; g < (1u << s); ++g) {
        const typename A::tw_t w = tw[(1u << s) + g];
#pragma unroll
        for (uint32_t m = 0; m < h; ++m) a.template ct<!A::kWide>(v[g * 2 * h + m], v[g * 2 * h + m + h], w);
      }
    }
#pragma unroll
    for (uint32_t i = 0; i < N; ++i) x[NATURAL ? brv(i, LOGN) : i] = a.canon_fwd(v[i]);
  } else {
#pragma unroll
    for (uint32_t i = 0; i < N; ++i) v[i] = x[NATURAL ? brv(i, LOGN) : i];
#pragma unroll
    for (int s = LOGN - 1; s >= 0; --s) {
      const uint32_t h = N >> (s + 1);
      if (s == 0) {
        const typename A::tw_t w0 = tw[0], w1 = tw[1];
#pragma unroll
        for (uint32_t m = 0; m < h; ++m) a.gs_last(v[m], v[m + h], w0, w1);
      } else {
#pragma unroll
        for (uint32_t g = 0; g < (1u << s); ++g) {
          const typename A::tw_t w = tw[(1u << s) + g];
#pragma unroll
          for (uint32_t m = 0; m < h; ++m) a.gs(v[g * 2 * h + m], v[g * 2 * h + m + h], w);
        }
      }
    }
#pragma unroll
    for (uint32_t i = 0; i < N; ++i) x[i] = a.canon_inv(v[i]);
  }
}

// ============================================================ pointwise
// c = a * b mod q_l elementwise over [items][N]; two words per thread per step.
template <class M, class W>
__global__ void __launch_bounds__(256)
k_pointwise(const W* __restrict__ a, const W* __restrict__ b, W* c, const M* __restrict__ mods,
            uint32_t L, uint32_t logN, size_t n_pairs) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pairs; i += stride) {
    const size_t e = 2 * i;
    const uint32_t l = (uint32_t)((e >> logN) % L);
    const M m = mods[l];
    const W a0 = a[e], a1 = a[e + 1], b0 = b[e], b1 = b[e + 1];
    c[e] = mulmod_general(a0, b0, m);
    c[e + 1] = mulmod_general(a1, b1, m);
  }
}

}  // namespace nttk
