// HE steps on either side of the transform (elementwise over coefficients,
// bound by HBM bandwidth): ciphertext tensor product, fast RNS basis
// conversion, ModDown.
#include "he.hpp"
#include "modarith.hpp"

namespace nttk {

// ------------------------------------------------------------ tensor product
// For each of [batch] ciphertext pairs a, b ([2][L][N] each):
//   d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1  (d is [3][L][N]).
// Canonical inputs give canonical outputs.
template <class M, class W>
__global__ void __launch_bounds__(256)
k_tensor(const W* __restrict__ a, const W* __restrict__ b, W* __restrict__ d, const M* __restrict__ mods,
         uint32_t L, uint32_t logN, uint32_t batch) {
  const size_t per = (size_t)L << logN;  // words per component
  const size_t total = per * batch, stride = (size_t)gridDim.x * blockDim.x;
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
    const size_t ct = g / per, e = g - ct * per;
    const M m = mods[e >> logN];
    const W* ac = a + 2 * per * ct;
    const W* bc = b + 2 * per * ct;
    W* dc = d + 3 * per * ct;
    const W a0 = ac[e], a1 = ac[per + e], b0 = bc[e], b1 = bc[per + e];
    const W p01 = mulmod_general(a0, b1, m), p10 = mulmod_general(a1, b0, m);
    const W s = p01 + p10;
    dc[e] = mulmod_general(a0, b0, m);
    dc[per + e] = s >= m.q ? s - m.q : s;
    dc[2 * per + e] = mulmod_general(a1, b1, m);
  }
}

hipError_t launch_tensor(int word, const void* a, const void* b, void* d, const void* mods, uint32_t L,
                         uint32_t logN, uint32_t batch, hipStream_t s) {
  const size_t total = ((size_t)L << logN) * batch;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const size_t want = (total + 255) / 256, cap = (size_t)cus * 16;
  const dim3 grid((unsigned)(want < cap ? want : cap)), block(256);
  if (word == 32)
    hipLaunchKernelGGL((k_tensor<ModInfo32, uint32_t>), grid, block, 0, s, (const uint32_t*)a, (const uint32_t*)b,
                       (uint32_t*)d, (const ModInfo32*)mods, L, logN, batch);
  else
    hipLaunchKernelGGL((k_tensor<ModInfo64, uint64_t>), grid, block, 0, s, (const uint64_t*)a, (const uint64_t*)b,
                       (uint64_t*)d, (const ModInfo64*)mods, L, logN, batch);
  return hipGetLastError();
}

// ------------------------------------------------------------ basis conversion
// Exact sum of up to 64 products y*m with y, m below 2^61. Both factors are
// split at bit 30 (y = y0 + y1 2^30, y0 < 2^30, y1 < 2^31; m likewise), so
// one product contributes to three columns
//   A: y0 m0 < 2^60,  B: y0 m1 + y1 m0 < 2^62,  C: y1 m1 < 2^62
// and four terms of a column fit 64 bits; with every prime below 2^60 (y1,
// m1 < 2^30) the bounds are 2^60, 2^61, 2^60 and eight terms fit. The kernel
// adds G products into plain 64-bit group sums with multiply-adds and folds
// each group into 96-bit column totals (64-bit sum + carry count).
struct Col96 {
  uint64_t s;
  uint32_t c;
};

__device__ __forceinline__ void col_add(Col96& a, uint64_t g) {
  const uint64_t t = a.s + g;
  a.c += t < g ? 1u : 0u;
  a.s = t;
}

// T = A + B 2^30 + C 2^60 (below 2^128) as hi 2^64 + lo, then T 2^-64 mod t
// by one Montgomery reduction: with u = lo (-t^-1) mod 2^64, T + u t is a
// multiple of 2^64 and (T + u t) / 2^64 = hi + hi64(u t) + (lo != 0), below
// 2t when hi < t. hi < t holds when sum_i (s_i - 1) < 2^64; otherwise
// (hi_reduce) hi is first reduced mod t, which keeps T mod t.
__device__ __forceinline__ uint64_t cols_redc(const Col96& A, const Col96& B, const Col96& C, const BcDst& d,
                                              uint32_t hi_reduce) {
  uint64_t lo = A.s, hi = A.c;
  const uint64_t bl = B.s << 30, bh = (B.s >> 34) | ((uint64_t)B.c << 30);
  lo += bl;
  hi += bh + (lo < bl ? 1u : 0u);
  const uint64_t cl = C.s << 60, ch = (C.s >> 4) | ((uint64_t)C.c << 60);
  lo += cl;
  hi += ch + (lo < cl ? 1u : 0u);
  if (hi_reduce) {
    hi = shoup_r(hi, 1, shoup_q_exact(hi, d.onep), d.nq);  // [0, 2t)
    hi = hi >= d.q ? hi - d.q : hi;
  }
  const uint64_t u = lo * d.ninv;
  uint64_t r = hi + shoup_q_exact(u, d.q) + (lo != 0 ? 1u : 0u);  // [0, 2t)
  return r >= d.q ? r - d.q : r;
}

// A block of W waves (W = blockDim.x / 64, 1 to 4) owns 64 x CPT adjacent
// coefficients of one polynomial. The waves first scale the L source
// residues by shat_i^-1 (Shoup, canonical) between them, split at bit 30,
// into LDS; then every wave copies all L scaled residues of its lanes into
// registers and computes the outputs j = wave, wave + W, ...: a dot product
// with row j of the matrix (read through the scalar cache, the row being the
// same for the whole wave) in groups of G terms, one Montgomery reduction,
// and for ModDown the scaled difference with y_j, whose loads are issued OC
// outputs at a time ahead of the arithmetic (the first OC before the scaling
// step) so that their latency overlaps work. LMAX bounds L at compile time so
// the residues stay in registers; the rows past L are zero, so every group
// is whole. For ModDown out may be yin: each element is read and then
// written by one thread.
template <int LMAX, int CPT, int G, bool DOWN>
__global__ void __launch_bounds__(256)
k_bconv(const uint64_t* __restrict__ x, const uint64_t* yin, uint64_t* out, const BcSrc* __restrict__ src,
        const uint64_t* __restrict__ mat, const BcDst* __restrict__ dst, uint32_t L, uint32_t K, uint32_t N,
        uint32_t batch, uint32_t hi_reduce) {
  static_assert(LMAX % G == 0, "whole groups");
  using V = typename std::conditional<CPT == 2, ulonglong2, uint64_t>::type;
  constexpr int OC = DOWN ? (CPT == 2 ? 6 : 8) : 1;  // outputs per prefetch chunk
  struct Split {
    uint32_t v[2 * CPT];  // (y0, y1) per coefficient
  };
  __shared__ Split ys[LMAX][64];
  constexpr uint32_t M30 = (1u << 30) - 1;
  // the wave index is uniform across the wave; saying so keeps the matrix
  // rows and per-prime constants on scalar loads (vector loads here would
  // need waits that also drain this wave's outstanding stores)
  const uint32_t lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t W = blockDim.x >> 6;
  const uint32_t slots = N / CPT, tiles = (slots + 63) / 64;
  const uint32_t b = blockIdx.x / tiles;
  const uint32_t slot = (blockIdx.x - b * tiles) * 64 + lane;
  const bool live = slot < slots;
  const uint32_t n = slot * CPT;
  const uint32_t Lp = (L + G - 1) / G * G;
  const size_t ob = (size_t)b * K * N + n;

  uint64_t pre[OC][CPT];
  auto prefetch = [&](uint32_t jb) {
    if (DOWN && live) {
#pragma unroll
      for (int t = 0; t < OC; ++t) {
        const uint32_t j = jb + t * W;
        if (j < K) *(V*)pre[t] = *(const V*)(yin + ob + (size_t)j * N);
      }
    }
  };
  prefetch(wave);

  const uint64_t* xb = x + (size_t)b * L * N + n;
  for (uint32_t i = wave; i < Lp; i += W) {
    Split e;
    if (i < L && live) {
      const BcSrc s = src[i];
      uint64_t v[CPT];
      *(V*)v = *(const V*)(xb + (size_t)i * N);
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        uint64_t r = shoup_r(v[c], s.w, shoup_q_exact(v[c], s.wp), s.nq);  // [0, 2 s_i)
        r = r >= s.q ? r - s.q : r;
        e.v[2 * c] = (uint32_t)r & M30;
        e.v[2 * c + 1] = (uint32_t)(r >> 30);
      }
    } else {
#pragma unroll
      for (int c = 0; c < 2 * CPT; ++c) e.v[c] = 0;
    }
    ys[i][lane] = e;
  }
  __syncthreads();
  if (!live) return;

  uint32_t y0[LMAX][CPT], y1[LMAX][CPT];
#pragma unroll
  for (int i0 = 0; i0 < LMAX; i0 += G) {
    if (i0 < (int)L) {
#pragma unroll
      for (int k = 0; k < G; ++k) {
        const Split e = ys[i0 + k][lane];
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
          y0[i0 + k][c] = e.v[2 * c];
          y1[i0 + k][c] = e.v[2 * c + 1];
        }
      }
    }
  }

  for (uint32_t jb = wave; jb < K; jb += OC * W) {
    if (jb != wave) prefetch(jb);
#pragma unroll
    for (int t = 0; t < OC; ++t) {
      const uint32_t j = jb + t * W;
      if (j >= K) break;
      const uint64_t* mj = mat + (size_t)j * Lp;
      Col96 A[CPT], B[CPT], C[CPT];
#pragma unroll
      for (int c = 0; c < CPT; ++c) A[c] = B[c] = C[c] = Col96{0, 0};
#pragma unroll
      for (int i0 = 0; i0 < LMAX; i0 += G) {
        if (i0 < (int)L) {
          uint64_t ga[CPT], gb[CPT], gc[CPT];
#pragma unroll
          for (int c = 0; c < CPT; ++c) ga[c] = gb[c] = gc[c] = 0;
#pragma unroll
          for (int k = 0; k < G; ++k) {
            const uint64_t m = mj[i0 + k];
            const uint32_t m0 = lo32(m), m1 = hi32(m);
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
              ga[c] = mad32(y0[i0 + k][c], m0, ga[c]);
              gb[c] = mad32(y1[i0 + k][c], m0, mad32(y0[i0 + k][c], m1, gb[c]));
              gc[c] = mad32(y1[i0 + k][c], m1, gc[c]);
            }
          }
#pragma unroll
          for (int c = 0; c < CPT; ++c) {
            col_add(A[c], ga[c]);
            col_add(B[c], gb[c]);
            col_add(C[c], gc[c]);
          }
        }
      }
      const BcDst d = dst[j];
      uint64_t r[CPT];
#pragma unroll
      for (int c = 0; c < CPT; ++c) r[c] = cols_redc(A[c], B[c], C[c], d, hi_reduce);
      if (DOWN) {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
          const uint64_t v = pre[t][c];
          const uint64_t diff = v >= r[c] ? v - r[c] : v + d.q - r[c];
          const uint64_t z = shoup_r(diff, d.sinv, shoup_q_exact(diff, d.sinvp), d.nq);
          r[c] = z >= d.q ? z - d.q : z;
        }
      }
      *(V*)(out + ob + (size_t)j * N) = *(V*)r;
    }
  }
}

// Waves per block: the largest W in 1..4 whose grid fits the GPU in one
// round at the kernel's occupancy (a second, partial round would run a few
// blocks alone at full latency); 4 when no W fits.
template <class F>
static uint32_t bconv_waves(F kernel, uint32_t blocks) {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
  }
  for (uint32_t w = 4; w >= 1; --w) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, (int)(64 * w), 0) != hipSuccess) break;
    if ((uint64_t)per_cu * cus >= blocks) return w;
  }
  return 4;
}

template <int LMAX, int CPT, int G>
static hipError_t bconv_go(const uint64_t* x, const uint64_t* y, uint64_t* out, const BcSrc* src,
                           const uint64_t* mat, const BcDst* dst, uint32_t L, uint32_t K, uint32_t N,
                           uint32_t batch, uint32_t hi_reduce, hipStream_t s) {
  const uint32_t tiles = (N / CPT + 63) / 64;
  const dim3 grid(tiles * batch);
  if (y) {
    auto k = k_bconv<LMAX, CPT, G, true>;
    const dim3 block(64 * bconv_waves(k, grid.x));
    hipLaunchKernelGGL(k, grid, block, 0, s, x, y, out, src, mat, dst, L, K, N, batch, hi_reduce);
  } else {
    auto k = k_bconv<LMAX, CPT, G, false>;
    const dim3 block(64 * bconv_waves(k, grid.x));
    hipLaunchKernelGGL(k, grid, block, 0, s, x, y, out, src, mat, dst, L, K, N, batch, hi_reduce);
  }
  return hipGetLastError();
}

hipError_t launch_bconv(const uint64_t* x, const uint64_t* y, uint64_t* out, const BcSrc* src,
                        const uint64_t* mat, const BcDst* dst, uint32_t L, uint32_t K, uint32_t N, uint32_t batch,
                        uint32_t G, uint32_t hi_reduce, hipStream_t s) {
  if (G == 8) {
    if (L <= 8) return bconv_go<8, 2, 8>(x, y, out, src, mat, dst, L, K, N, batch, hi_reduce, s);
    if (L <= 16) return bconv_go<16, 2, 8>(x, y, out, src, mat, dst, L, K, N, batch, hi_reduce, s);
    if (L <= 24) return bconv_go<24, 2, 8>(x, y, out, src, mat, dst, L, K, N, batch, hi_reduce, s);
    if (L <= 32) return bconv_go<32, 1, 8>(x, y, out, src, mat, dst, L, K, N, batch, hi_reduce, s);
    if (L <= 48) return bconv_go<48, 1, 8>(x, y, out, src, mat, dst, L, K, N, batch, hi_reduce, s);
    if (L <= 64) return bconv_go<64, 1, 8>(x, y, out, src, mat, dst, L, K, N, batch, hi_reduce, s);
  } else if (G == 4) {
    if (L <= 4) return bconv_go<4, 2, 4>(x, y, out, src, mat, dst, L, K, N, batch, hi_reduce, s);
    if (L <= 8) return bconv_go<8, 2, 4>(x, y, out, src, mat, dst, L, K, N, batch, hi_reduce, s);
    if (L <= 16) return bconv_go<16, 2, 4>(x, y, out, src, mat, dst, L, K, N, batch, hi_reduce, s);
    if (L <= 32) return bconv_go<32, 1, 4>(x, y, out, src, mat, dst, L, K, N, batch, hi_reduce, s);
    if (L <= 64) return bconv_go<64, 1, 4>(x, y, out, src, mat, dst, L, K, N, batch, hi_reduce, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace nttk
