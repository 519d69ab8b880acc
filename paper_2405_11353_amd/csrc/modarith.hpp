// Modular arithmetic for the gfx950 NTT kernels.
//
// The multiply-by-twiddle is Shoup's precomputed-quotient product (the paper's
// modulo_mult, Alg. 5, with tw_h = floor(tw * 2^w / q)), here at w = 64 built
// from 32-bit integer operations, and at w = 32 for moduli below 2^30. The
// add/sub of each butterfly follows modulo_add (Alg. 4) but keeps values in a
// lazy range [0, k*q) and reduces with one conditional subtraction of a
// multiple of q, as in Harvey's NTT butterflies; results are made canonical
// once, before they are stored.
//
// Measured on MI355X: v_mul_lo/hi_u32 and v_mad_u64_u32 issue at the same rate
// as 64-bit adds and compares (about one wave instruction per 4 clocks per
// SIMD), so the cost of a butterfly is its instruction count. The "approx"
// quotient below saves the lowest 32x32 partial product and two carries.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nttk {

// The arithmetic is __host__ __device__ so that the host build can be unit
// tested against 128-bit integer arithmetic on the CPU.
#define NTT_HD __host__ __device__ __forceinline__

NTT_HD uint32_t umulhi32(uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umulhi(a, b);
#else
  return (uint32_t)(((uint64_t)a * b) >> 32);
#endif
}

// ---------------------------------------------------------------- 64-bit
struct ModInfo64 {
  uint64_t q;     // modulus, q < 2^62
  uint64_t n8q;   // 2^64 - 8q: the wide range's reduction (q < 2^60)
  uint64_t nq;    // 2^64 - q, so that lo64(Q*q) is subtracted by an add
  uint64_t qinv;  // q^-1 mod 2^64 (Montgomery reduction in the pointwise product)
  uint64_t r1;    // 2^64 mod q
  uint64_t r1p;   // floor(r1 * 2^64 / q), Shoup companion of r1
  uint64_t n2q;   // 2^64 - 2q and 2^64 - 4q: the lazy reductions subtract 2q or
  uint64_t n4q;   // 4q by one 64-bit add of these (no borrow chain)
  uint64_t cf;    // quotient estimate of the wide range's canonicalisation:
                  // bits 0-31 c = floor(2^(s + 32 + e) / q), bits 32-39 s,
                  // bits 40-47 e, where b = bit length of q and (s, e) =
                  // (b - 28, 26) if b >= 28, else (0, b - 1)
};

static_assert(sizeof(ModInfo64) == 72, "the table generator writes 9 words per modulus");

struct Tw64 {
  uint64_t w;   // twiddle in [0, q)
  uint64_t wp;  // floor(w * 2^64 / q)
};

NTT_HD uint32_t lo32(uint64_t x) { return (uint32_t)x; }
NTT_HD uint32_t hi32(uint64_t x) { return (uint32_t)(x >> 32); }
NTT_HD uint64_t mad32(uint32_t a, uint32_t b, uint64_t c) {
  return (uint64_t)a * b + c;  // v_mad_u64_u32
}

// Quotient estimate floor(y * wp / 2^64) minus 0, 1 or 2: drops the low half
// of the two cross products and the whole low product (each < 2^64 in weight,
// so the sum dropped is < 3 * 2^64).
NTT_HD uint64_t shoup_q_approx(uint64_t y, uint64_t wp) {
  uint32_t y0 = lo32(y), y1 = hi32(y), p0 = lo32(wp), p1 = hi32(wp);
  uint64_t s = (uint64_t)umulhi32(y1, p0) + umulhi32(y0, p1);
  return mad32(y1, p1, s);
}
// Exact high half of y * wp.
NTT_HD uint64_t shoup_q_exact(uint64_t y, uint64_t wp) {
  uint32_t y0 = lo32(y), y1 = hi32(y), p0 = lo32(wp), p1 = hi32(wp);
  uint64_t t = mad32(y1, p0, umulhi32(y0, p0));
  uint64_t u = mad32(y0, p1, lo32(t));
  return mad32(y1, p1, (uint64_t)hi32(t) + hi32(u));
}
// r = y*w - Q*q mod 2^64, computed as y*w + Q*(2^64 - q): the true value is
// below 2^64 whenever Q is one of the estimates above.
NTT_HD uint64_t shoup_r(uint64_t y, uint64_t w, uint64_t Q, uint64_t nq) {
  uint32_t y0 = lo32(y), y1 = hi32(y), w0 = lo32(w), w1 = hi32(w);
  uint32_t Q0 = lo32(Q), Q1 = hi32(Q), n0 = lo32(nq), n1 = hi32(nq);
  uint64_t lo = mad32(Q0, n0, mad32(y0, w0, 0));
  uint32_t hi = hi32(lo) + y1 * w0 + y0 * w1 + Q1 * n0 + Q0 * n1;
#if defined(__HIP_DEVICE_COMPILE__)
  // An empty asm (no instruction) that hides hi's value, so that the compiler
  // keeps the 32-bit add of hi32(lo) instead of turning the result into a
  // 64-bit add of lo and hi << 32, which costs a move to zero the low half
  asm("" : "+v"(hi));
#endif
  return ((uint64_t)hi << 32) | lo32(lo);
}

// x + y*w - Q*q mod 2^64: the remainder above with its multiply-add chain
// seeded by x, so that a butterfly's sum x + (y*w mod q) costs no add of its
// own. Any x < 2^64; the caller knows the true value is below 2^64.
NTT_HD uint64_t shoup_r_plus(uint64_t y, uint64_t w, uint64_t Q, uint64_t nq, uint64_t x) {
  uint32_t y0 = lo32(y), y1 = hi32(y), w0 = lo32(w), w1 = hi32(w);
  uint32_t Q0 = lo32(Q), Q1 = hi32(Q), n0 = lo32(nq), n1 = hi32(nq);
  uint64_t lo = mad32(Q0, n0, mad32(y0, w0, x));
  uint32_t hi = hi32(lo) + y1 * w0 + y0 * w1 + Q1 * n0 + Q0 * n1;
#if defined(__HIP_DEVICE_COMPILE__)
  asm("" : "+v"(hi));  // keep the 32-bit add, as in shoup_r
#endif
  return ((uint64_t)hi << 32) | lo32(lo);
}

// Which forward stages reduce x before the CT butterfly, by the stage's index
// j within its pass. Outside the wide range every stage does. In the wide
// range ([0, 16q), q < 2^60) a butterfly may skip the reduction while x is
// below 12q, each skipped stage adding 4q to the bound and each reducing one
// leaving it at 12q:
//  RP_FRESH, a pass whose input is below 4q (coefficients, or twisted rows):
//    bounds 8q, 12q, 16q after stages 0..2 skip, then stages 3, 5, 7, ...
//    reduce and the even ones after them skip;
//  RP_LAZY, a pass whose input is anywhere in [0, 16q) (the row pass after the
//    column pass): stages 0, 2, 4, ... reduce and the odd ones skip.
enum { RP_ALL = 0, RP_FRESH = 1, RP_LAZY = 2 };
NTT_HD constexpr bool reduces_x(int rp, int j) {
  return rp == RP_ALL ? true : rp == RP_FRESH ? (j >= 3 && ((j - 3) & 1) == 0) : ((j & 1) == 0);
}

// 1: the CT butterfly takes its sum from shoup_r_plus and its difference as
// 2 x + L - sum (one 64-bit shift-add and a subtraction); 0: from the product
// T, as x + T and x + L - T
#ifndef NTT_CT_FOLD
#define NTT_CT_FOLD 1
#endif

// 1: the wide range's canonicalisation subtracts an estimated multiple of q
// (ModInfo64::cf) and then q at most once; 0: four conditional subtractions
#ifndef NTT_CANON_EST
#define NTT_CANON_EST 1
#endif

// WIDE (approximate quotient, every q < 2^60): forward values live in
// [0, 16q) instead of [0, 8q). A CT butterfly whose x is below 12q needs no
// reduction (x + T and x + 4q - T stay below 16q), and one that reduces
// subtracts 8q from x < 16q and leaves both outputs below 12q; so the stages
// of a forward pass can alternate between reducing and not (see
// reduces_x in ntt_core.hpp), and about half the reductions go away. The
// inverse (GS) butterflies are the same as without WIDE.
template <bool EXACT, bool WIDE = false>
struct Arith64 {
  static_assert(!(EXACT && WIDE), "the wide range is for the approximate quotient");
  using word = uint64_t;
  using tw_t = Tw64;
  static constexpr bool kExact = EXACT;
  static constexpr bool kWide = WIDE;
  uint64_t q, L, nq, nL, n2q, n4q, R, nR;
  uint32_t cc, cs, ce;  // the wide range's canonicalisation (ModInfo64::cf)

  NTT_HD void load(const ModInfo64& m) {
    q = m.q;
    L = EXACT ? 2 * m.q : 4 * m.q;
    nq = m.nq;
    nL = EXACT ? m.n2q : m.n4q;
    n2q = m.n2q;
    n4q = m.n4q;
    R = WIDE ? 8 * m.q : L;     // what a reducing CT butterfly subtracts from x
    nR = WIDE ? m.n8q : nL;
    cc = lo32(m.cf);
    cs = hi32(m.cf) & 0xffu;
    ce = (hi32(m.cf) >> 8) & 0xffu;
  }

  // y * w mod q, result in [0, L) (L = 4q approx, 2q exact), any y < 2^64
  NTT_HD uint64_t mul(uint64_t y, const Tw64& t) const {
    uint64_t Q = EXACT ? shoup_q_exact(y, t.wp) : shoup_q_approx(y, t.wp);
    return shoup_r(y, t.w, Q, nq);
  }
  // x - m if x >= m, else x; nm = 2^64 - m, so that the subtraction is a single
  // 64-bit add instead of a subtract with borrow, whose carry register also
  // costs wait states before the select can read it
  NTT_HD static uint64_t csub(uint64_t x, uint64_t m, uint64_t nm) { return x >= m ? x + nm : x; }

  // Cooley-Tukey butterfly (x, y) -> (x + w y, x - w y); values in [0, 2L),
  // or with WIDE in [0, 16q): RED reduces x from [0, 16q) (outputs below 12q),
  // !RED needs x below 12q
  template <bool RED = true>
  NTT_HD void ct(uint64_t& x, uint64_t& y, const Tw64& t) const {
    static_assert(RED || WIDE, "every butterfly reduces outside the wide range");
    uint64_t xr = RED ? csub(x, R, nR) : x;
#if NTT_CT_FOLD
    // s = xr + T with T = y w mod q in [0, L); the difference xr + L - T is
    // 2 xr + L - s, exact mod 2^64 since its true value is in (0, 2L)
    uint64_t Q = EXACT ? shoup_q_exact(y, t.wp) : shoup_q_approx(y, t.wp);
    uint64_t s = shoup_r_plus(y, t.w, Q, nq, xr);
    y = (xr << 1) + L - s;
    x = s;
#else
    uint64_t T = mul(y, t);
    x = xr + T;
    y = xr + L - T;
#endif
  }
  // Gentleman-Sande butterfly (x, y) -> (x + y, (x - y) w); values in [0, L)
  NTT_HD void gs(uint64_t& x, uint64_t& y, const Tw64& t) const {
    uint64_t s = x + y;
    uint64_t d = x + L - y;
    x = csub(s, L, nL);
    y = mul(d, t);
  }
  // butterflies whose twiddle is 1 (group 0 of a cyclic transform): both
  // inputs are reduced instead of multiplied, same ranges as ct / gs (with
  // WIDE, y is brought below 4q, where a product would leave it)
  template <bool RED = true>
  NTT_HD void ct1(uint64_t& x, uint64_t& y) const {
    static_assert(RED || WIDE, "every butterfly reduces outside the wide range");
    uint64_t xr = RED ? csub(x, R, nR) : x;
    uint64_t yr = WIDE ? csub(csub(y, R, nR), L, nL) : csub(y, L, nL);
    x = xr + yr;
    y = xr + L - yr;
  }
  NTT_HD void gs1(uint64_t& x, uint64_t& y) const {
    uint64_t s = x + y;
    uint64_t d = x + L - y;
    x = csub(s, L, nL);
    y = csub(d, L, nL);
  }
  // last inverse stage: both outputs scaled (N^-1 folded into two twiddles)
  NTT_HD void gs_last(uint64_t& x, uint64_t& y, const Tw64& t0, const Tw64& t1) const {
    uint64_t s = x + y;
    uint64_t d = x + L - y;
    x = mul(s, t0);
    y = mul(d, t1);
  }
  // canonical from [0, 2L) (forward; [0, 16q) with WIDE) or [0, L) (inverse)
  NTT_HD uint64_t canon_fwd(uint64_t x) const {
    if (WIDE && NTT_CANON_EST) {
      // k = floor(x / q) or one less: the top 32 bits of x (x >> s, below
      // 2^32 for every x < 2^(b+4), which covers 16q) times the 32-bit
      // reciprocal c. Truncating x and c each loses less than 2^-26 of a
      // unit of x / q, so x - k q lies in [0, 2q) and one subtraction of q
      // finishes; x - k q is formed as x + k (2^64 - q) mod 2^64.
      const uint32_t k = umulhi32((uint32_t)(x >> cs), cc) >> ce;
      const uint64_t lo = mad32(k, lo32(nq), x);
      uint32_t hi = hi32(lo) + k * hi32(nq);
#if defined(__HIP_DEVICE_COMPILE__)
      asm("" : "+v"(hi));  // keep the 32-bit add, as in shoup_r
#endif
      return csub(((uint64_t)hi << 32) | lo32(lo), q, nq);
    }
    if (WIDE) x = csub(x, R, nR);
    x = csub(x, L, nL);
    if (!EXACT) x = csub(x, 2 * q, n2q);
    return csub(x, q, nq);
  }
  NTT_HD uint64_t canon_inv(uint64_t x) const {
    if (!EXACT) x = csub(x, 2 * q, n2q);
    return csub(x, q, nq);
  }
};

// Montgomery product x*y*2^-64 mod q in [0, q), for any x*y < q*2^64 (so
// that the 128-bit product's high word is below q): u = lo64(x*y) * q^-1 makes
// x*y - u*q divisible by 2^64, and the quotient, hi64(x*y) - hi64(u*q), lies in
// (-q, q). The fused product + inverse takes this and leaves the factor 2^-64
// to the last inverse stage, whose N^-1 twiddles then carry 2^64 as well.
NTT_HD uint64_t mulmod_mont(uint64_t x, uint64_t y, const ModInfo64& m) {
  uint32_t x0 = lo32(x), x1 = hi32(x), y0 = lo32(y), y1 = hi32(y);
  // 128-bit product t = th:tl
  uint64_t p00 = mad32(x0, y0, 0);
  uint64_t p10 = mad32(x1, y0, hi32(p00));
  uint64_t p01 = mad32(x0, y1, lo32(p10));
  uint64_t th = mad32(x1, y1, (uint64_t)hi32(p10) + hi32(p01));
  uint64_t tl = ((uint64_t)lo32(p01) << 32) | lo32(p00);
  // u = tl * q^-1 mod 2^64; then t - u*q = 0 mod 2^64 and (t - u*q)/2^64 = th - hi64(u*q)
  uint32_t u0 = lo32(tl), u1 = hi32(tl), i0 = lo32(m.qinv), i1 = hi32(m.qinv);
  uint64_t u = mad32(u0, i0, 0);
  u = ((uint64_t)(hi32(u) + u1 * i0 + u0 * i1) << 32) | lo32(u);
  uint64_t uq_hi;
  {
    uint32_t a0 = lo32(u), a1 = hi32(u), q0 = lo32(m.q), q1 = hi32(m.q);
    uint64_t s00 = mad32(a0, q0, 0);
    uint64_t s10 = mad32(a1, q0, hi32(s00));
    uint64_t s01 = mad32(a0, q1, lo32(s10));
    uint64_t s11 = mad32(a1, q1, (uint64_t)hi32(s10) + hi32(s01));
    uq_hi = s11;
  }
  uint64_t r = th - uq_hi;            // in (-q, q) as a signed value
  return (th < uq_hi) ? r + m.q : r;  // [0, q)
}

// General product x*y mod q for the pointwise kernel (neither operand known in
// advance): the Montgomery product above, then a Shoup product by 2^64 mod q
// restores the factor.
NTT_HD uint64_t mulmod_general(uint64_t x, uint64_t y, const ModInfo64& m) {
  const uint64_t r = mulmod_mont(x, y, m);
  // times 2^64 mod q (Shoup, exact quotient): [0, 2q) then canonical
  uint64_t Q = shoup_q_exact(r, m.r1p);
  uint64_t z = shoup_r(r, m.r1, Q, m.nq);
  return z >= m.q ? z - m.q : z;
}

// ---------------------------------------------------------------- 32-bit
struct ModInfo32 {
  uint32_t q;     // q < 2^30
  uint32_t rsv;   // reserved
  uint32_t qinv;  // q^-1 mod 2^32
  uint32_t r1;    // 2^32 mod q
  uint32_t r1p;   // floor(r1 * 2^32 / q)
  uint32_t pad[3];
};
struct Tw32 {
  uint32_t w, wp;  // wp = floor(w * 2^32 / q)
};

struct Arith32 {
  using word = uint32_t;
  using tw_t = Tw32;
  static constexpr bool kExact = true;
  uint32_t q, L;
  NTT_HD void load(const ModInfo32& m) { q = m.q; L = 2 * m.q; }
  // Shoup at w = 32 (Alg. 5 with the paper's word size): result in [0, 2q)
  NTT_HD uint32_t mul(uint32_t y, const Tw32& t) const {
    uint32_t Q = umulhi32(y, t.wp);
    return y * t.w - Q * q;
  }
  NTT_HD static uint32_t csub(uint32_t x, uint32_t m) { return x >= m ? x - m : x; }
  static constexpr bool kWide = false;
  template <bool RED = true>
  NTT_HD void ct(uint32_t& x, uint32_t& y, const Tw32& t) const {
    static_assert(RED, "every butterfly reduces");
    uint32_t xr = csub(x, L);
    uint32_t T = mul(y, t);
    x = xr + T;
    y = xr + L - T;
  }
  NTT_HD void gs(uint32_t& x, uint32_t& y, const Tw32& t) const {
    uint32_t s = x + y;
    uint32_t d = x + L - y;
    x = csub(s, L);
    y = mul(d, t);
  }
  template <bool RED = true>
  NTT_HD void ct1(uint32_t& x, uint32_t& y) const {
    static_assert(RED, "every butterfly reduces");
    uint32_t xr = csub(x, L), yr = csub(y, L);
    x = xr + yr;
    y = xr + L - yr;
  }
  NTT_HD void gs1(uint32_t& x, uint32_t& y) const {
    uint32_t s = x + y;
    uint32_t d = x + L - y;
    x = csub(s, L);
    y = csub(d, L);
  }
  NTT_HD void gs_last(uint32_t& x, uint32_t& y, const Tw32& t0, const Tw32& t1) const {
    uint32_t s = x + y;
    uint32_t d = x + L - y;
    x = mul(s, t0);
    y = mul(d, t1);
  }
  NTT_HD uint32_t canon_fwd(uint32_t x) const { return csub(csub(x, L), q); }
  NTT_HD uint32_t canon_inv(uint32_t x) const { return csub(x, q); }
};

// x*y*2^-32 mod q in [0, q) for x*y < q*2^32 (Montgomery, as at 64 bits)
NTT_HD uint32_t mulmod_mont(uint32_t x, uint32_t y, const ModInfo32& m) {
  uint64_t t = (uint64_t)x * y;
  uint32_t u = (uint32_t)t * m.qinv;                 // t - u q = 0 mod 2^32
  uint32_t uq_hi = umulhi32(u, m.q);
  uint32_t th = (uint32_t)(t >> 32);
  uint32_t r = th - uq_hi;
  return (th < uq_hi) ? r + m.q : r;                 // x y 2^-32 mod q
}

NTT_HD uint32_t mulmod_general(uint32_t x, uint32_t y, const ModInfo32& m) {
  const uint32_t r = mulmod_mont(x, y, m);
  uint32_t Q = umulhi32(r, m.r1p);
  uint32_t z = r * m.r1 - Q * m.q;                   // [0, 2q)
  return z >= m.q ? z - m.q : z;
}

}  // namespace nttk
