// Power x^y of a positive normal FP64 x for the equation of state
// p = p_ref (R_d rho theta / p_ref)^(C_p / C_v) (Eq. pressure) and its
// inverse, written from the series definitions:
//   ln x = e ln 2 + 2 atanh(f),  x = m 2^e, m in [1/sqrt 2, sqrt 2),
//          f = (m - 1) / (m + 1), |f| <= 0.1716,
//          atanh f = f (1 + f^2/3 + f^4/5 + ... + f^24/25)  (truncation < 3e-19);
//   e^t  = 2^k e^r,  k = round(t / ln 2), |r| <= ln 2 / 2,
//          e^r = sum_{n=0}^{15} r^n / n!                    (truncation < 4e-19).
// ln 2 is split into a 32-bit-exact high part and the remainder, so that
// k ln 2 and e ln 2 carry no rounding.  Every product-sum is an explicit
// fma, so the host and device builds of this header round identically.
// Relative error against a correctly rounded pow: a few units in the last
// place times |y ln x| (checked on the host over the ranges the model
// uses).  Not for x <= 0, subnormal x, or results outside the normal range.
#pragma once

#include <cmath>

namespace thor {

__host__ __device__ __forceinline__ double powd_ln(double x) {
  int e;
  double m = std::frexp(x, &e);              // x = m 2^e, m in [0.5, 1)
  if (m < 0.70710678118654752440) {          // into [1/sqrt 2, sqrt 2)
    m *= 2.0;
    e -= 1;
  }
  const double f = (m - 1.0) / (m + 1.0);
  const double f2 = f * f;
  // 1 + f^2/3 + ... + f^24/25, Horner in f^2
  double s = 1.0 / 25.0;
  s = std::fma(s, f2, 1.0 / 23.0);
  s = std::fma(s, f2, 1.0 / 21.0);
  s = std::fma(s, f2, 1.0 / 19.0);
  s = std::fma(s, f2, 1.0 / 17.0);
  s = std::fma(s, f2, 1.0 / 15.0);
  s = std::fma(s, f2, 1.0 / 13.0);
  s = std::fma(s, f2, 1.0 / 11.0);
  s = std::fma(s, f2, 1.0 / 9.0);
  s = std::fma(s, f2, 1.0 / 7.0);
  s = std::fma(s, f2, 1.0 / 5.0);
  s = std::fma(s, f2, 1.0 / 3.0);
  const double lnm = std::fma(2.0 * f * f2, s, 2.0 * f);   // 2 f + 2 f^3 (s without its leading 1)
  const double ln2_hi = 0.693147180369123816490;            // low 21 mantissa bits zero
  const double ln2_lo = 1.90821492927058770002e-10;         // ln 2 - ln2_hi
  const double de = (double)e;
  return std::fma(de, ln2_hi, std::fma(de, ln2_lo, lnm));
}

__host__ __device__ __forceinline__ double powd_exp(double t) {
  const double inv_ln2 = 1.44269504088896340736;
  const double ln2_hi = 0.693147180369123816490;
  const double ln2_lo = 1.90821492927058770002e-10;
  const double k = std::rint(t * inv_ln2);
  const double r = std::fma(-k, ln2_lo, std::fma(-k, ln2_hi, t));
  // sum_{n=0}^{15} r^n / n!, Horner
  double s = 1.0 / 1307674368000.0;          // 1/15!
  s = std::fma(s, r, 1.0 / 87178291200.0);   // 1/14!
  s = std::fma(s, r, 1.0 / 6227020800.0);
  s = std::fma(s, r, 1.0 / 479001600.0);
  s = std::fma(s, r, 1.0 / 39916800.0);
  s = std::fma(s, r, 1.0 / 3628800.0);
  s = std::fma(s, r, 1.0 / 362880.0);
  s = std::fma(s, r, 1.0 / 40320.0);
  s = std::fma(s, r, 1.0 / 5040.0);
  s = std::fma(s, r, 1.0 / 720.0);
  s = std::fma(s, r, 1.0 / 120.0);
  s = std::fma(s, r, 1.0 / 24.0);
  s = std::fma(s, r, 1.0 / 6.0);
  s = std::fma(s, r, 0.5);
  s = std::fma(s, r, 1.0);
  s = std::fma(s, r, 1.0);
  return std::ldexp(s, (int)k);
}

// x^y for positive normal x.
__host__ __device__ __forceinline__ double powd(double x, double y) { return powd_exp(y * powd_ln(x)); }

}  // namespace thor
