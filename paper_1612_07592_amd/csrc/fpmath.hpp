// exp, log and expm1 in FP64 for the FP64 path, host and device.
//
// The method needs these functions to double precision only, but math
// libraries differ in the last bit, and in a chaotic run a single differing
// bit (say, in the photon energy of one emission) grows until two runs part.
// These are written as short series whose every operation is an IEEE-rounded
// add, multiply or divide in a fixed order (built without FMA contraction),
// so that any IEEE platform gives the same bits:
//   exp(x):   x = k ln2 + r with k = rint(x/ln2) and r = (x - k L_HI) - k L_LO,
//             ln2 = L_HI + L_LO with 42 significant bits in L_HI (k L_HI is
//             exact); exp(r) = sum_{n<=14} r^n/n! by Horner (|r| <= ln2/2, the
//             first omitted term below 2^-60); scaled by 2^k.
//   log(x):   x = m 2^e with m in [sqrt(1/2), sqrt(2)), s = (m-1)/(m+1);
//             log m = 2 atanh s = 2 s sum_{j<=11} s^(2j)/(2j+1) (|s| <= 0.1716);
//             log x = e L_HI + (e L_LO + log m).
//   expm1(x): x sum_{n<=13} x^n/(n+1)! for |x| < ln2/2, else exp(x) - 1.
// Accuracy against the platform libm: exp 1 ulp, log 3 ulp, expm1 4 ulp.
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>

namespace pic {

constexpr double kL2Hi = 0x1.62e42fefa38p-1;
constexpr double kL2Lo = 0x1.ef35793c7673p-45;
constexpr double kInvLn2 = 0x1.71547652b82fep+0;

// sum_{n=0}^{14} r^n / n! by Horner from the highest term
__host__ __device__ inline double exp_series(double r) {
  double p = 1.0 / 87178291200.0;
  p = p * r + 1.0 / 6227020800.0;
  p = p * r + 1.0 / 479001600.0;
  p = p * r + 1.0 / 39916800.0;
  p = p * r + 1.0 / 3628800.0;
  p = p * r + 1.0 / 362880.0;
  p = p * r + 1.0 / 40320.0;
  p = p * r + 1.0 / 5040.0;
  p = p * r + 1.0 / 720.0;
  p = p * r + 1.0 / 120.0;
  p = p * r + 1.0 / 24.0;
  p = p * r + 1.0 / 6.0;
  p = p * r + 1.0 / 2.0;
  p = p * r + 1.0;
  p = p * r + 1.0;
  return p;
}

__host__ __device__ inline double fp_exp(double x) {
  if (x != x) return x;
  if (x > 709.8) return HUGE_VAL;
  if (x < -745.2) return 0.0;
  const double k = rint(x * kInvLn2);
  const double r = (x - k * kL2Hi) - k * kL2Lo;
  return ldexp(exp_series(r), (int)k);
}

__host__ __device__ inline double fp_log(double x) {
  if (x != x) return x;
  if (!(x > 0.0)) return x == 0.0 ? -HUGE_VAL : (double)NAN;
  if (x == HUGE_VAL) return x;
  int e = 0;
  double m = frexp(x, &e);  // x = m 2^e, m in [1/2, 1)
  if (m < 0x1.6a09e667f3bcdp-1) {
    m = m * 2.0;
    e = e - 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  // sum_{j=0}^{11} z^j / (2j + 1) by Horner from the highest term
  double p = 1.0 / 23.0;
  p = p * z + 1.0 / 21.0;
  p = p * z + 1.0 / 19.0;
  p = p * z + 1.0 / 17.0;
  p = p * z + 1.0 / 15.0;
  p = p * z + 1.0 / 13.0;
  p = p * z + 1.0 / 11.0;
  p = p * z + 1.0 / 9.0;
  p = p * z + 1.0 / 7.0;
  p = p * z + 1.0 / 5.0;
  p = p * z + 1.0 / 3.0;
  p = p * z + 1.0;
  const double lm = (2.0 * s) * p;
  const double de = (double)e;
  return de * kL2Hi + (de * kL2Lo + lm);
}

__host__ __device__ inline double fp_expm1(double x) {
  if (fabs(x) < 0x1.62e42fefa39efp-2) {  // |x| < ln2/2
    // sum_{n=0}^{13} x^n / (n+1)! by Horner from the highest term, times x
    double p = 1.0 / 87178291200.0;
    p = p * x + 1.0 / 6227020800.0;
    p = p * x + 1.0 / 479001600.0;
    p = p * x + 1.0 / 39916800.0;
    p = p * x + 1.0 / 3628800.0;
    p = p * x + 1.0 / 362880.0;
    p = p * x + 1.0 / 40320.0;
    p = p * x + 1.0 / 5040.0;
    p = p * x + 1.0 / 720.0;
    p = p * x + 1.0 / 120.0;
    p = p * x + 1.0 / 24.0;
    p = p * x + 1.0 / 6.0;
    p = p * x + 1.0 / 2.0;
    p = p * x + 1.0;
    return x * p;
  }
  return fp_exp(x) - 1.0;
}

}  // namespace pic
