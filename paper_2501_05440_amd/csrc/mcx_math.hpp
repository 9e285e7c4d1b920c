// mcx_math.hpp - counter-based random numbers and correctly rounded
// transcendental functions for the transport kernels (host + device).
//
// Random numbers: Philox4x64-10 (Salmon et al., SC'11), the counter-based
// generator named by the method's replicable-RNG requirement (paper Sec. 1).
// A draw d of a stream keyed (seed, tag) reads word d % 4 of the block at
// counter (d / 4, particle id, generation, problem), mapped to
// (top 52 bits + 1/2) * 2^-52 in (0, 1).
//
// ln(x) and cos/sin(2 pi t) are evaluated in double-double arithmetic with a
// relative error near 2^-100 and rounded once, which yields the correctly
// rounded binary64 result except with a probability of order 2^-45 per call.
// Every other operation of the path is a single IEEE-754 operation, so the
// value of every quantity of a history is defined independently of any math
// library.  Build with -ffp-contract=off: the compiler must not fuse the
// products and sums written here.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mcx_tables.inc"

#define MCX_HD __host__ __device__ __forceinline__

namespace mcx {

// Double-double tables: ln(j / 256), j = 181..362, and sin, cos(pi k / 64),
// k = 0..16.  One copy lives in device constant memory, one in host memory.
static __constant__ double c_log_tab[2 * MCX_LOG_TAB_N] = MCX_LOG_TAB_INIT;
static __constant__ double c_sc_tab[4 * MCX_SINCOS_TAB_N] = MCX_SINCOS_TAB_INIT;
static const double h_log_tab[2 * MCX_LOG_TAB_N] = MCX_LOG_TAB_INIT;
static const double h_sc_tab[4 * MCX_SINCOS_TAB_N] = MCX_SINCOS_TAB_INIT;

MCX_HD const double* log_tab() {
#if defined(__HIP_DEVICE_COMPILE__)
  return c_log_tab;
#else
  return h_log_tab;
#endif
}

MCX_HD const double* sc_tab() {
#if defined(__HIP_DEVICE_COMPILE__)
  return c_sc_tab;
#else
  return h_sc_tab;
#endif
}

// ---------------------------------------------------------------------------
// Philox4x64-10
// ---------------------------------------------------------------------------

struct u64x4 {
  uint64_t v[4];
};

// Full 64 x 64 -> 128-bit product.  On the device, from four 32 x 32 + 64
// multiply-adds (each partial sum below fits in 64 bits), which yields the
// low and the high word together.
MCX_HD void mul128(uint64_t a, uint64_t b, uint64_t* lo, uint64_t* hi) {
#if defined(__HIP_DEVICE_COMPILE__)
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  const uint64_t p00 = (uint64_t)a0 * b0;
  const uint64_t t = (uint64_t)a0 * b1 + (p00 >> 32);
  const uint64_t u = (uint64_t)a1 * b0 + (uint32_t)t;
  *lo = (u << 32) | (uint32_t)p00;
  *hi = (uint64_t)a1 * b1 + (t >> 32) + (u >> 32);
#else
  const unsigned __int128 p = (unsigned __int128)a * b;
  *lo = (uint64_t)p;
  *hi = (uint64_t)(p >> 64);
#endif
}

MCX_HD u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                           uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0, lo0, hi1, lo1;
    mul128(M0, c0, &lo0, &hi0);
    mul128(M1, c2, &lo1, &hi1);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  return u64x4{{c0, c1, c2, c3}};
}

MCX_HD double u01(uint64_t w) { return ((double)(w >> 12) + 0.5) * 0x1p-52; }

enum : uint64_t { TAG_SRC = 1, TAG_TRANSPORT = 2, TAG_RESAMPLE = 3 };

// One stream position: (seed, tag) key plus (id, gen, problem) counter words.
// The block of the current counter is cached, so consecutive draws cost one
// Philox evaluation per four draws.
struct Stream {
  uint64_t k0, k1, id, gen, prob;
  uint32_t draw;
  uint32_t blk_idx;  // draw >> 2 of the cached block, or ~0u
  u64x4 blk;

  MCX_HD Stream(uint64_t seed, uint64_t tag, uint64_t id_, uint64_t gen_, uint64_t prob_,
                uint32_t draw_)
      : k0(seed), k1(tag), id(id_), gen(gen_), prob(prob_), draw(draw_), blk_idx(~0u) {}

  MCX_HD double next() {
    const uint32_t b = draw >> 2;
    if (b != blk_idx) {
      blk = philox4x64_10(b, id, gen, prob, k0, k1);
      blk_idx = b;
    }
    const uint32_t k = draw & 3u;
    const uint64_t w = k == 0 ? blk.v[0] : k == 1 ? blk.v[1] : k == 2 ? blk.v[2] : blk.v[3];
    draw += 1u;
    return u01(w);
  }
};

// ---------------------------------------------------------------------------
// double-double arithmetic (hi + lo, |lo| <= ulp(hi) / 2 after renormalising)
// ---------------------------------------------------------------------------

struct dd {
  double hi, lo;
};

MCX_HD dd two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  const double e = (a - (s - bb)) + (b - bb);
  return dd{s, e};
}

MCX_HD dd fast_two_sum(double a, double b) {  // |a| >= |b| or a == 0
  const double s = a + b;
  const double e = b - (s - a);
  return dd{s, e};
}

MCX_HD dd two_prod(double a, double b) {
  const double p = a * b;
  const double e = fma(a, b, -p);
  return dd{p, e};
}

MCX_HD dd dd_add(dd x, dd y) {
  dd s = two_sum(x.hi, y.hi);
  dd t = two_sum(x.lo, y.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}

MCX_HD dd dd_neg(dd x) { return dd{-x.hi, -x.lo}; }

MCX_HD dd dd_mul(dd x, dd y) {
  dd p = two_prod(x.hi, y.hi);
  p.lo += x.hi * y.lo + x.lo * y.hi;
  return fast_two_sum(p.hi, p.lo);
}

MCX_HD dd dd_mul_d(dd x, double y) {
  dd p = two_prod(x.hi, y);
  p.lo += x.lo * y;
  return fast_two_sum(p.hi, p.lo);
}

MCX_HD uint64_t as_u64(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return (uint64_t)__double_as_longlong(x);
#else
  uint64_t u;
  __builtin_memcpy(&u, &x, 8);
  return u;
#endif
}

MCX_HD double as_f64(uint64_t u) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __longlong_as_double((long long)u);
#else
  double x;
  __builtin_memcpy(&x, &u, 8);
  return x;
#endif
}

// ---------------------------------------------------------------------------
// ln(x), correctly rounded, for positive finite x.
//
// x = 2^e m with m in [181/256, 362/256); j = round(256 m), F = j / 256,
// u = (m - F) / F (|u| <= 2^-8.5), and
//   ln x = e ln2 + ln F + 2 atanh(s),  s = u / (2 + u),  |s| <= 2^-9.5,
//   atanh(s) = s + s^3/3 + s^5 (1/5 + s^2/7 + s^4/9 + s^6/11) + O(s^13).
// The terms whose rounding error could reach 2^-100 relative are carried in
// double-double; the table holds ln F as double-double.
// ---------------------------------------------------------------------------

MCX_HD double cr_log(double x, const double* log_tab) {
  if (!(x > 0.0)) return x == 0.0 ? -__builtin_inf() : __builtin_nan("");
  if (x == __builtin_inf()) return x;
  int e_adj = 0;
  if (x < 0x1p-1022) {
    x *= 0x1p54;
    e_adj = -54;
  }
  const uint64_t ix = as_u64(x);
  int e = (int)((ix >> 52) & 0x7ff) - 1023 + e_adj;
  double m = as_f64((ix & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull);
  if (m >= 1.4140625) {
    m *= 0.5;
    e += 1;
  }
  const int j = (int)rint(m * 256.0);
  const double F = (double)j * 0x1p-8;
  const double f = m - F;  // exact
  // s = u / (2 + u) = f / (m + F) in double-double: D = m + F exactly as a
  // pair and one reciprocal of its high part; the quotient's residual comes
  // from an fma (exact up to a rounding of relative size 2^-105), and the low
  // part takes one more residual step, so that it is within about half an
  // ulp of the true remainder quotient (the reciprocal alone is off by up to
  // 2^-53 relative, too much for arguments next to 1)
  const dd D = two_sum(m, F);
  const double rD = 1.0 / D.hi;
  const double sh = f * rD;
  const double rem = fma(-sh, D.hi, f) - sh * D.lo;
  const double sl1 = rem * rD;
  const double rem2 = fma(-sl1, D.hi, rem) - sl1 * D.lo;
  const dd s = fast_two_sum(sh, sl1 + rem2 * rD);
  const int k = j - MCX_LOG_TAB_J0;
  const double lnF_hi = log_tab[2 * k], lnF_lo = log_tab[2 * k + 1];
  {
    // Quick evaluation: the leading terms e ln2_hi + ln F_hi + 2 s.hi summed
    // exactly, everything else (2 atanh(s) - 2 s and the low parts) in plain
    // double.  Its error stays below 2^-69 of the result (the low-part sum
    // and the series are under 2^-19 of it and carry relative errors near
    // 2^-51), so if the remainder of the rounded sum keeps 2^-67 of the
    // result away from the rounding boundary (half an ulp, a quarter below
    // a power of two), that rounding is the correct one; else the
    // double-double evaluation below decides.
    const double z = s.hi * s.hi;
    const double tail =
        s.hi * z *
        (2.0 / 3.0 + z * (2.0 / 5.0 + z * (2.0 / 7.0 + z * (2.0 / 9.0 + z * (2.0 / 11.0)))));
    const dd a = fast_two_sum((double)e * MCX_LN2_HI, lnF_hi);  // e ln2_hi is exact
    const dd b = two_sum(a.hi, 2.0 * s.hi);
    const double small = ((a.lo + lnF_lo) + (double)e * MCX_LN2_LO) + (2.0 * s.lo + tail);
    const dd q = fast_two_sum(b.hi, b.lo + small);
    if (q.hi == 0.0) return 0.0;  // x = 1
    const uint64_t qb = as_u64(q.hi);
    double half = as_f64((((qb >> 52) & 0x7FFull) - 53ull) << 52);
    if ((qb & 0x000FFFFFFFFFFFFFull) == 0 && (q.lo < 0.0) == (q.hi > 0.0)) half *= 0.5;
    if (fabs(q.lo) + fabs(q.hi) * 0x1p-67 < half) return q.hi;
  }
  const dd s2 = dd_mul(s, s);
  const dd s3 = dd_mul(s2, s);
  const double z = s2.hi;
  const double p = z * (0.2 + z * (1.0 / 7.0 + z * (1.0 / 9.0 + z * (1.0 / 11.0))));
  const dd third{MCX_THIRD_HI, MCX_THIRD_LO};
  dd at = dd_add(s, dd_mul(s3, third));
  at = dd_add(at, dd{s3.hi * p, 0.0});
  const dd l1p{2.0 * at.hi, 2.0 * at.lo};
  const dd lnF{lnF_hi, lnF_lo};
  const dd eln2 = fast_two_sum((double)e * MCX_LN2_HI, (double)e * MCX_LN2_LO);
  const dd r = dd_add(dd_add(eln2, lnF), l1p);
  return r.hi + r.lo;
}

// ---------------------------------------------------------------------------
// cos(2 pi t) and sin(2 pi t) for the exact real 2 pi t, 0 <= t < 1,
// correctly rounded.  The angle pi x (x = 2t) is folded exactly into pi y,
// 0 <= y <= 1/4; y = k/64 + r with |r| <= 1/128, theta = pi r, and
//   sin(pi y) = S_k cos(theta) + C_k sin(theta),
//   cos(pi y) = C_k cos(theta) - S_k sin(theta),
// with S_k, C_k = sin, cos(pi k / 64) from a double-double table and Taylor
// series in theta (|theta| <= pi/128) carried in double-double where needed.
// ---------------------------------------------------------------------------

MCX_HD void cr_cossin_2pi(double t, const double* sc_tab, double* c_out, double* s_out) {
  double x = 2.0 * t;
  bool neg_s = false, neg_c = false, swap = false;
  if (x >= 1.0) {
    x = x - 1.0;
    neg_s = !neg_s;
    neg_c = !neg_c;
  }
  if (x > 0.5) {
    x = 1.0 - x;
    neg_c = !neg_c;
  }
  if (x > 0.25) {
    x = 0.5 - x;
    swap = true;
  }
  const double kf = rint(x * 64.0);
  const double r = x - kf * 0x1p-6;  // exact
  const int k = (int)kf;
  const double th_hi = MCX_PI_HI * r;
  const dd th = fast_two_sum(th_hi, fma(MCX_PI_HI, r, -th_hi) + MCX_PI_LO * r);
  const dd t2 = dd_mul(th, th);
  const dd t3 = dd_mul(t2, th);
  const double z = t2.hi;
  // sin(theta) = theta - theta^3/6 + theta^5/120 - theta^7/5040 + ...
  const dd sixth{MCX_SIXTH_HI, MCX_SIXTH_LO};
  const dd r120{MCX_R120_HI, MCX_R120_LO};
  const double ts = t3.hi * (z * z) * (-1.0 / 5040.0 + z * (1.0 / 362880.0 - z * (1.0 / 39916800.0)));
  dd sn = dd_add(th, dd_neg(dd_mul(t3, sixth)));
  sn = dd_add(sn, dd_mul(dd_mul(t3, t2), r120));
  sn = dd_add(sn, dd{ts, 0.0});
  // cos(theta) = 1 - theta^2/2 + theta^4/24 - theta^6/720 + ...
  const dd r24{MCX_R24_HI, MCX_R24_LO};
  const double tc = (z * z * z) * (-1.0 / 720.0 + z * (1.0 / 40320.0 - z * (1.0 / 3628800.0)));
  dd cs = dd_add(dd{1.0, 0.0}, dd{-0.5 * t2.hi, -0.5 * t2.lo});
  cs = dd_add(cs, dd_mul(dd_mul(t2, t2), r24));
  cs = dd_add(cs, dd{tc, 0.0});
  const dd S{sc_tab[4 * k + 0], sc_tab[4 * k + 1]};
  const dd C{sc_tab[4 * k + 2], sc_tab[4 * k + 3]};
  const dd sy = dd_add(dd_mul(S, cs), dd_mul(C, sn));
  const dd cy = dd_add(dd_mul(C, cs), dd_neg(dd_mul(S, sn)));
  double sv = sy.hi + sy.lo;
  double cv = cy.hi + cy.lo;
  if (swap) {
    const double tmp = sv;
    sv = cv;
    cv = tmp;
  }
  *s_out = neg_s ? -sv : sv;
  *c_out = neg_c ? -cv : cv;
}

}  // namespace mcx
