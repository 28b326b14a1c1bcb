// ee_dd.hpp -- correctly rounded exp and log in double-double arithmetic,
// for the FP64 step of the estimator (App. A: Delta F = -log <exp(-W)>).
//
// The estimator kernel evaluates the exponentials of the works and the
// logarithms of their sums with these functions, so that its results do not
// depend on the accuracy of the device math library: each returns the
// double nearest to the exact value (ties to even), apart from the cases
// noted below.  The same source compiles for the host (plain C++, no device
// builtins), which is how it is tested against a 60-digit decimal
// evaluation.
//
// Method.
//   Error-free transformations (Knuth's two-sum, Dekker's fast two-sum, the
//   fused-multiply-add two-product) give double-double numbers h + l with
//   about 106 bits.
//   exp(x): x = k ln2 + r with |r| <= ln2/2 (Cody and Waite's reduction,
//   ln2 split into three doubles C1 + C2 + C3 with C1 rounded to 42 bits so
//   that k C1 is exact for |k| < 2^11).  expm1(r / 2^8) by its Taylor
//   series to the 10th power in double-double, then eight doublings
//   expm1(2a) = 2 expm1(a) + expm1(a)^2, and exp(x) = 2^k (1 + expm1(r)).
//   The double-double result has a relative error of about 2^-100, so its
//   rounding to double is the correctly rounded exp(x) unless exp(x) lies
//   within that distance of a rounding boundary.
//   log(s): one Newton step for y = log s from y0 = log(s) of the math
//   library: with exp(y0) = 2^k (1 + m) in double-double,
//   d = s exp(-y0) - 1 = (s 2^-k - 1 - m) / (1 + m) (the subtraction is
//   exact), and y = y0 + log1p(d) with log1p(d) = d - d^2/2 to the precision
//   needed (|d| <= 2^-51).
//
// Domain: exp for every double (results below 2^-1022 are rounded twice,
// which can move them by one unit of the subnormal grid; the estimator's
// exponentials are relative to the largest term, 1, so such terms change no
// sum).  log for positive normal numbers and +inf.
//
// Compile with floating-point contraction off: the error-free
// transformations need every product and sum rounded as written.
#pragma once
#include <cmath>

#if defined(__HIPCC__)
#define EE_HD __host__ __device__
#else
#define EE_HD
#endif

#pragma clang fp contract(off)

namespace ee {
namespace dd {

struct DD {
  double h, l;
};

EE_HD inline DD two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return DD{s, (a - (s - bb)) + (b - bb)};
}

// |a| >= |b| (or a = 0)
EE_HD inline DD fast_two_sum(double a, double b) {
  const double s = a + b;
  return DD{s, b - (s - a)};
}

EE_HD inline DD two_prod(double a, double b) {
  const double p = a * b;
  return DD{p, ::fma(a, b, -p)};
}

EE_HD inline DD add(DD a, DD b) {
  DD s = two_sum(a.h, b.h);
  const DD t = two_sum(a.l, b.l);
  s.l += t.h;
  s = fast_two_sum(s.h, s.l);
  s.l += t.l;
  return fast_two_sum(s.h, s.l);
}

EE_HD inline DD mul(DD a, DD b) {
  DD p = two_prod(a.h, b.h);
  p.l += a.h * b.l + a.l * b.h;
  return fast_two_sum(p.h, p.l);
}

// ln 2 = C1 + C2 + C3 (C1: 42 significant bits; C2, C3: the next doubles of
// the remainder), and 1/ln 2 (only used to pick k).
constexpr double kC1 = 0x1.62e42fefa3800p-1;
constexpr double kC2 = 0x1.ef35793c76730p-45;
constexpr double kC3 = 0x1.f97b57a079a19p-103;
constexpr double kInvLn2 = 0x1.71547652b82fep+0;

// 1/n! for n = 2..10 as double-double (nearest double, then the nearest
// double to the remainder).
EE_HD inline DD inv_fact(int n) {
  switch (n) {
    case 2: return DD{0x1.0000000000000p-1, 0.0};
    case 3: return DD{0x1.5555555555555p-3, 0x1.5555555555555p-57};
    case 4: return DD{0x1.5555555555555p-5, 0x1.5555555555555p-59};
    case 5: return DD{0x1.1111111111111p-7, 0x1.1111111111111p-63};
    case 6: return DD{0x1.6c16c16c16c17p-10, -0x1.f49f49f49f49fp-65};
    case 7: return DD{0x1.a01a01a01a01ap-13, 0x1.a01a01a01a01ap-73};
    case 8: return DD{0x1.a01a01a01a01ap-16, 0x1.a01a01a01a01ap-76};
    case 9: return DD{0x1.71de3a556c734p-19, -0x1.c154f8ddc6c00p-73};
    default: return DD{0x1.27e4fb7789f5cp-22, 0x1.cbbc05b4fa99ap-76};  // n = 10
  }
}

// r - k ln 2 as double-double, for x = the double argument, k integral with
// |k| < 2^11 and |x - k ln2| small.  x - k C1 is exact (k C1 needs at most
// 53 bits, and the two are within a factor of two when k != 0).
EE_HD inline DD reduce_ln2(double x, double k) {
  const double a = x - k * kC1;
  const DD p = two_prod(k, kC2);
  DD r = two_sum(a, -p.h);
  r.l = (r.l - p.l) - k * kC3;
  return fast_two_sum(r.h, r.l);
}

// expm1(r) for |r| <= ln2/2 (a little more is fine), relative error ~2^-100.
EE_HD inline DD expm1_reduced(DD r) {
  const DD x{::ldexp(r.h, -8), ::ldexp(r.l, -8)};
  DD p = inv_fact(10);
  for (int n = 9; n >= 2; --n) p = add(mul(p, x), inv_fact(n));
  p = add(mul(p, x), DD{1.0, 0.0});
  DD m = mul(p, x);
  for (int i = 0; i < 8; ++i) m = add(add(m, m), mul(m, m));
  return m;
}

// The double nearest to exp(x).
EE_HD inline double exp_cr(double x) {
  if (x != x) return x;
  if (x > 0x1.62e42fefa39efp+9) return HUGE_VAL;   // above log(DBL_MAX)
  if (x < -0x1.74910d52d3052p+9) return 0.0;      // below log(2^-1075)
  if (x == 0.0) return 1.0;
  const double k = ::rint(x * kInvLn2);
  const DD m = expm1_reduced(reduce_ln2(x, k));
  DD e = two_sum(1.0, m.h);
  e.l += m.l;
  e = fast_two_sum(e.h, e.l);
  return ::ldexp(e.h, (int)k);
}

// The double nearest to log(s), s positive and normal (or +inf).
EE_HD inline double log_cr(double s) {
  if (!(s > 0.0)) return (s == 0.0) ? -HUGE_VAL : (s - s) / (s - s);
  if (s == 1.0) return 0.0;
  if (s > 1.7976931348623157e308) return s;
  const double y0 = ::log(s);
  const double k = ::rint(y0 * kInvLn2);
  const DD m = expm1_reduced(reduce_ln2(y0, k));  // exp(y0) = 2^k (1 + m)
  const double f = ::ldexp(s, -(int)k) - 1.0;     // exact: s 2^-k is in [1/2, 2]
  const double num = (f - m.h) - m.l;              // f - m.h is exact (Sterbenz)
  const double d = num / (1.0 + m.h);
  return y0 + (d - 0.5 * d * d);
}

}  // namespace dd
}  // namespace ee
