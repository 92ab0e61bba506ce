// gs_exp.h -- FP64 exponential for the per-pair response evaluation.
//
// exp(x) = 2^n p(r), x = n ln2 + r, |r| <= ln2/2 (Cody & Waite argument
// reduction): ln2 is split into a head with 40 significant bits, so n * head
// is exact for |n| < 2^13, and a tail.  n is rounded by adding 1.5 * 2^52
// to x / ln2 in one fused operation: the sum has unit spacing, so it holds
// the nearest integer n, whose two's complement is its low 32 bits.  p is the degree-11 polynomial that
// minimises the relative error of exp(r) on [-ln2/2, ln2/2], fitted with
// the Remez exchange algorithm in 60-digit arithmetic (maximum relative
// error 3.1e-18 before the coefficients are rounded to double).
//
// Arguments below -1000 are raised to -1000 (the result underflows to 0
// either way), so far-tail exponents never reach a saturated integer
// conversion.  A NaN argument is not propagated; callers flag invalid
// inputs separately.  Arguments above ~709.78 overflow to +inf.
//
// The coefficients are passed in as an array so that device code can keep
// them in scalar registers (a __constant__ table read with scalar loads)
// and the polynomial issues as plain FMAs.
#pragma once
#include <math.h>

#ifdef __HIPCC__
#define GS_HD __host__ __device__
#else
#define GS_HD
#endif

namespace gs {

// c[0..11]: polynomial coefficients of r^11 .. r^0 (Horner order);
// c[12] = 1/ln2, c[13] = ln2 head, c[14] = ln2 tail, c[15] = 1.5 * 2^52.
#define GS_EXP_COEFS                                                                                 \
  {                                                                                                  \
    2.499430488481720730096538e-8, 2.763229327945987537523749e-7, 2.755762253087225465714744e-6,    \
        2.480148652142746394884348e-5, 1.984126943267923686630193e-4, 1.388888895122398829076301e-3, \
        8.333333333559271335728342e-3, 4.166666666649276729475066e-2, 1.666666666666616866446141e-1, \
        5.000000000000017685649359e-1, 1.000000000000000030360381e0, 9.999999999999999971003972e-1,  \
        1.4426950408889634074, 0.6931471805592082, 7.371002565167799e-13, 6755399441055744.0         \
  }

// c0 = c[0] and mg = c[15], passed separately so that a caller can hold them
// in vector registers: an instruction may read only one scalar register, and
// these two meet another scalar operand.
GS_HD inline double exp_cw(double x, const double *c, double c0, double mg) {
  x = fmax(x, -1000.0);
  const double t = fma(x, c[12], mg);
  const double n = t - mg;
  double r = fma(-n, c[13], x);
  r = fma(-n, c[14], r);
  double p = fma(c0, r, c[1]);
  p = fma(p, r, c[2]);
  p = fma(p, r, c[3]);
  p = fma(p, r, c[4]);
  p = fma(p, r, c[5]);
  p = fma(p, r, c[6]);
  p = fma(p, r, c[7]);
  p = fma(p, r, c[8]);
  p = fma(p, r, c[9]);
  p = fma(p, r, c[10]);
  p = fma(p, r, c[11]);
  return ldexp(p, (int)(unsigned)__builtin_bit_cast(unsigned long long, t));
}

GS_HD inline double exp_cw(double x, const double *c) { return exp_cw(x, c, c[0], c[15]); }

}  // namespace gs
