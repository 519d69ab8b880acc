// The paper's algorithm variants as GPU kernels, for comparison with the
// fused kernels: one launch per stage over global memory, one thread per
// butterfly (the two inner loops flattened into the thread index, the
// Flat-NTT idea), canonical arithmetic after every operation as in
// modulo_add (Alg. 4) and modulo_mult (Alg. 5). Cyclic transform (Eq. 3).
//   DIT       Alg. 1: bit_reverse, then stages s = 1..L in place
//   DIF       Alg. 2: stages s = L..1 in place, then bit_reverse
//   PEASE     Alg. 3: bit_reverse, then constant-geometry stages into a second
//             array, copied back after every stage
//   PEASE_NC  Pease_nc: the same stages, swapping the two arrays instead of copying
//   STOCKHAM  autosort: two arrays, no bit reversal
// Twiddles: W[i] = omega^i for i < N/2 (the inverse uses omega^-i and a
// final scaling by N^-1).
#include "launch.hpp"
#include "ntt_core.hpp"

namespace nttk {
namespace {

template <class A>
struct Canon {
  using W = typename A::word;
  using TW = typename A::tw_t;
  A a;
  W q;
  __device__ void load(const typename ModOf<A>::type& m) {
    a.load(m);
    q = a.q;
  }
  __device__ W add(W x, W y) const {
    const W s = x + y;
    return s >= q ? s - q : s;
  }
  __device__ W sub(W x, W y) const { return x >= y ? x - y : x + q - y; }
  // exact-quotient Shoup product in [0, 2q), then one conditional subtraction
  __device__ W mul(W y, const TW& t) const {
    const W r = a.mul(y, t);
    return r >= q ? r - q : r;
  }
};

template <class W>
__global__ void __launch_bounds__(256) k_pbitrev(W* data, uint32_t items, uint32_t logN) {
  const size_t total = (size_t)items << logN, stride = (size_t)gridDim.x * blockDim.x;
  const uint32_t mask = (1u << logN) - 1;
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
    const uint32_t i = (uint32_t)(g & mask), j = brv(i, logN);
    if (i < j) {
      W* x = data + (g - i);
      const W t = x[i];
      x[i] = x[j];
      x[j] = t;
    }
  }
}

template <class W>
__global__ void __launch_bounds__(256) k_pcopy(W* dst, const W* src, size_t total) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) dst[g] = src[g];
}

// one stage of DIT (DIF = false) or DIF (DIF = true), in place
template <class A, bool DIF>
__global__ void __launch_bounds__(256)
k_pstage(typename A::word* data, const typename A::tw_t* __restrict__ Wt, const typename ModOf<A>::type* __restrict__ mods,
         uint32_t L, uint32_t logN, uint32_t s, uint32_t items) {
  using W = typename A::word;
  const uint32_t half = (1u << logN) >> 1;
  const size_t total = (size_t)items * half, stride = (size_t)gridDim.x * blockDim.x;
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
    const uint32_t item = (uint32_t)(g / half), b = (uint32_t)(g % half), l = item % L;
    Canon<A> c;
    c.load(mods[l]);
    const uint32_t h = 1u << (s - 1);
    const uint32_t k = b & (h - 1), i0 = ((b >> (s - 1)) << s) + k;
    const typename A::tw_t tw = Wt[(size_t)l * half + ((size_t)k << (logN - s))];  // W[(N/m) k]
    W* x = data + ((size_t)item << logN);
    const W f1 = x[i0], g2 = x[i0 + h];
    if (!DIF) {
      const W f2 = c.mul(g2, tw);
      x[i0] = c.add(f1, f2);
      x[i0 + h] = c.sub(f1, f2);
    } else {
      x[i0] = c.add(f1, g2);
      x[i0 + h] = c.mul(c.sub(f1, g2), tw);
    }
  }
}

// one constant-geometry stage (Pease), x -> y
template <class A>
__global__ void __launch_bounds__(256)
k_ppease(const typename A::word* xin, typename A::word* yout, const typename A::tw_t* __restrict__ Wt,
         const typename ModOf<A>::type* __restrict__ mods, uint32_t L, uint32_t logN, uint32_t s, uint32_t items) {
  using W = typename A::word;
  const uint32_t half = (1u << logN) >> 1;
  const size_t total = (size_t)items * half, stride = (size_t)gridDim.x * blockDim.x;
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
    const uint32_t item = (uint32_t)(g / half), r = (uint32_t)(g % half), l = item % L;
    Canon<A> c;
    c.load(mods[l]);
    const uint32_t base = (1u << (s - 1)) - 1;
    const W* x = xin + ((size_t)item << logN);
    W* y = yout + ((size_t)item << logN);
    const W f1 = x[2 * r], f2 = c.mul(x[2 * r + 1], Wt[(size_t)l * half + (r & ~base)]);
    y[r] = c.add(f1, f2);
    y[r + half] = c.sub(f1, f2);
  }
}

// one Stockham autosort stage t, x -> y
template <class A>
__global__ void __launch_bounds__(256)
k_pstockham(const typename A::word* xin, typename A::word* yout, const typename A::tw_t* __restrict__ Wt,
            const typename ModOf<A>::type* __restrict__ mods, uint32_t L, uint32_t logN, uint32_t t, uint32_t items) {
  using W = typename A::word;
  const uint32_t half = (1u << logN) >> 1;
  const size_t total = (size_t)items * half, stride = (size_t)gridDim.x * blockDim.x;
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
    const uint32_t item = (uint32_t)(g / half), b = (uint32_t)(g % half), l = item % L;
    Canon<A> c;
    c.load(mods[l]);
    const uint32_t Lt = 1u << t, h = Lt >> 1, r = (1u << logN) >> t;
    const uint32_t j = b & (h - 1), k = b >> (t - 1);
    const typename A::tw_t om = Wt[(size_t)l * half + ((size_t)j << (logN - t))];  // W^((N/Lt) j)
    const W* x = xin + ((size_t)item << logN);
    W* y = yout + ((size_t)item << logN);
    const W u = x[j + h * k], v = c.mul(x[j + h * (k + r)], om);
    y[j + Lt * k] = c.add(u, v);
    y[j + h + Lt * k] = c.sub(u, v);
  }
}

template <class A>
__global__ void __launch_bounds__(256)
k_pscale(typename A::word* data, const typename A::tw_t* __restrict__ ninv, const typename ModOf<A>::type* __restrict__ mods,
         uint32_t L, uint32_t logN, uint32_t items) {
  const size_t total = (size_t)items << logN, stride = (size_t)gridDim.x * blockDim.x;
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
    const uint32_t l = (uint32_t)((g >> logN) % L);
    Canon<A> c;
    c.load(mods[l]);
    data[g] = c.mul(data[g], ninv[l]);
  }
}

dim3 grid_for(size_t threads) {
  size_t b = (threads + 255) / 256;
  return dim3((unsigned)(b < 8192 ? (b ? b : 1) : 8192));
}

template <class A>
hipError_t run(const PaperLaunch& c, bool fwd) {
  using W = typename A::word;
  using TW = typename A::tw_t;
  using M = typename ModOf<A>::type;
  W* d = (W*)c.data;
  W* s = (W*)c.scratch;
  const TW* Wt = (const TW*)(fwd ? c.tw_fwd : c.tw_inv);
  const M* m = (const M*)c.mods;
  const uint32_t lg = (uint32_t)c.logN, Lg = c.L, it = c.items;
  const size_t total = (size_t)it << lg;
  const dim3 gb = grid_for(total / 2 ? total / 2 : 1), ge = grid_for(total), blk(256);
  const hipStream_t st = c.stream;
  W* cur = d;
  W* other = s;
  switch (c.path) {
    case PAPER_DIT:
      hipLaunchKernelGGL(k_pbitrev<W>, ge, blk, 0, st, d, it, lg);
      for (uint32_t k = 1; k <= lg; ++k) hipLaunchKernelGGL((k_pstage<A, false>), gb, blk, 0, st, d, Wt, m, Lg, lg, k, it);
      break;
    case PAPER_DIF:
      for (uint32_t k = lg; k >= 1; --k) hipLaunchKernelGGL((k_pstage<A, true>), gb, blk, 0, st, d, Wt, m, Lg, lg, k, it);
      hipLaunchKernelGGL(k_pbitrev<W>, ge, blk, 0, st, d, it, lg);
      break;
    case PAPER_PEASE:
    case PAPER_PEASE_NC:
      if (!s) return hipErrorInvalidValue;
      hipLaunchKernelGGL(k_pbitrev<W>, ge, blk, 0, st, d, it, lg);
      for (uint32_t k = lg; k >= 1; --k) {
        hipLaunchKernelGGL(k_ppease<A>, gb, blk, 0, st, cur, other, Wt, m, Lg, lg, k, it);
        if (c.path == PAPER_PEASE) {
          hipLaunchKernelGGL(k_pcopy<W>, ge, blk, 0, st, cur, (const W*)other, total);  // the copy Pease_nc removes
        } else {
          W* t = cur;
          cur = other;
          other = t;
        }
      }
      if (cur != d) hipLaunchKernelGGL(k_pcopy<W>, ge, blk, 0, st, d, (const W*)cur, total);
      break;
    case PAPER_STOCKHAM:
      if (!s) return hipErrorInvalidValue;
      for (uint32_t k = 1; k <= lg; ++k) {
        hipLaunchKernelGGL(k_pstockham<A>, gb, blk, 0, st, cur, other, Wt, m, Lg, lg, k, it);
        W* t = cur;
        cur = other;
        other = t;
      }
      if (cur != d) hipLaunchKernelGGL(k_pcopy<W>, ge, blk, 0, st, d, (const W*)cur, total);
      break;
    default:
      return hipErrorNotSupported;
  }
  if (!fwd) hipLaunchKernelGGL(k_pscale<A>, ge, blk, 0, st, d, (const TW*)c.ninv, m, Lg, lg, it);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_paper(const PaperLaunch& c, bool forward) {
  if (c.items == 0 || c.logN < 1) return hipErrorInvalidValue;
  return c.word == 32 ? run<Arith32>(c, forward) : run<Arith64<true>>(c, forward);
}

}  // namespace nttk
