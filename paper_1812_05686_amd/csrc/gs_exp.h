// gs_exp.h -- FP64 exponential for the per-pair response evaluation.
//
// exp(x) = 2^n p(r), x = n ln2 + r, |r| <= ln2/2 (Cody & Waite argument
// reduction, with a one-term ln2): n is rounded by adding 1.5 * 2^52 to
// x / ln2 in one fused operation (the sum has unit spacing, so it holds the
// nearest integer n, whose two's complement is its low 32 bits), and
// r = x - n ln2 is formed in one FMA with ln2 rounded to double.  The product
// is exact inside the FMA; the rounding of ln2 (2.3e-17) shifts r by
// |n| 2.3e-17, so the relative error grows with |x|: below 6e-16 + |n| 2.4e-17,
// i.e. 2.6e-15 for the log-densities above -60 that a banded fold keeps and
// 2.5e-14 at the bottom of the normal range.  Pair exponents never need more:
// a bin's value is set by its largest pairs.  p is the degree-10 polynomial
// that minimises the relative error of exp(r) on [-ln2/2, ln2/2], from the
// Remez exchange algorithm in 80-digit arithmetic (remez_exp.py; 2.1e-16
// before and 3.1e-16 after its coefficients are rounded to double).
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

// c[0..10]: polynomial coefficients of r^10 .. r^0 (Horner order);
// c[11] = 1/ln2, c[12] = ln2 (rounded to double), c[13] = 1.5 * 2^52.
#define GS_EXP_COEFS                                                                             \
  {                                                                                              \
    2.748844159545267e-07, 2.763976828264541e-06, 2.4801917693499152e-05, 0.00019841171384145565, \
        0.0013888888499132617, 0.00833333338466586, 0.04166666666842604, 0.16666666666557742,     \
        0.49999999999997286, 1.0000000000000064, 1.0, 1.4426950408889634074,                      \
        0.69314718055994530942, 6755399441055744.0                                                \
  }
#define GS_EXP_NCOEF 14

// c0 = c[0] and mg = c[13], passed separately so that a caller can hold them
// in vector registers: an instruction may read only one scalar register, and
// these two meet another scalar operand.
GS_HD inline double exp_cw(double x, const double *c, double c0, double mg) {
  x = fmax(x, -1000.0);
  const double t = fma(x, c[11], mg);
  const double n = t - mg;
  const double r = fma(-n, c[12], x);
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
  return ldexp(p, (int)(unsigned)__builtin_bit_cast(unsigned long long, t));
}

GS_HD inline double exp_cw(double x, const double *c) { return exp_cw(x, c, c[0], c[13]); }

}  // namespace gs
