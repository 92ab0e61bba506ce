// gs_exp.h -- FP64 exponential for the per-pair response evaluation.
//
// exp(x) = 2^n p(r), x = n ln2 + r, |r| <= ln2/2 (Cody & Waite argument
// reduction, with a one-term ln2): n is rounded by adding 1.5 * 2^52 to
// x / ln2 in one fused operation (the sum has unit spacing, so it holds the
// nearest integer n, whose two's complement is its low 32 bits), and
// r = x - n ln2 is formed in one FMA with ln2 rounded to double.  The product
// is exact inside the FMA; the rounding of ln2 (2.3e-17) shifts r by
// |n| 2.3e-17, so the relative error grows with |x|.  p is the degree-9
// polynomial that minimises the relative error of exp(r) on [-ln2/2, ln2/2],
// from the Remez exchange algorithm in 80-digit arithmetic (remez_exp.py;
// 1.34e-14 before and 1.36e-14 after its coefficients are rounded to double).
// In all the relative error is below 1.45e-14 + |n| 2.4e-17: 1.7e-14 for
// log-densities above -60 (a banded fold keeps those above its cut, -52 by
// default) and 4e-14 at the bottom of the normal range.
//
// Degree 9 matches the accuracy of the argument: a pair exponent formed from
// a cell's tile-relative constants carries a rounding error of up to ~4e-14
// (absolute, so relative in the density), which one more polynomial term
// (degree 10: 3.1e-16) would not remove.  A bin's value is set by its largest
// pairs, so either sits far inside the per-bin bound of 1e-12.
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

// c[0..GS_EXP_DEG]: polynomial coefficients of r^9 .. r^0 (Horner order),
// then 1/ln2, ln2 (rounded to double) and 1.5 * 2^52.
#define GS_EXP_DEG 9
#define GS_EXP_COEFS                                                                                    \
  {                                                                                                     \
    2.7482187570947232e-06, 2.488401002622006e-05, 0.00019841596395523973, 0.0013888802828792976,       \
        0.008333333002823906, 0.04166666703246359, 0.16666666667826951, 0.4999999999945797,            \
        0.9999999999998928, 1.0000000000000127, 1.4426950408889634074, 0.69314718055994530942,         \
        6755399441055744.0                                                                              \
  }
#define GS_EXP_NCOEF (GS_EXP_DEG + 4)
#define GS_EXP_INV_LN2 (GS_EXP_DEG + 1)
#define GS_EXP_LN2 (GS_EXP_DEG + 2)
#define GS_EXP_SHIFT (GS_EXP_DEG + 3)

// Arguments at or above kExpNoClampMin may skip the lower clamp: there
// x / ln2 rounds to an integer of magnitude below 2^31 (the low 32 bits of t
// are that integer) and the result already underflows to 0 below about -745.
// A caller that can show every argument of a loop is finite and at least
// kExpNoClampMin (a concave exponent checked at the ends of its range) uses
// exp_cw_unclamped; the two agree bit for bit there.
constexpr double kExpNoClampMin = -1.0e9;

// c0 = c[0] and mg = c[GS_EXP_SHIFT], passed separately so that a caller can
// hold them in vector registers: an instruction may read only one scalar
// register, and these two meet another scalar operand.
GS_HD inline double exp_cw_unclamped(double x, const double *c, double c0, double mg) {
  const double t = fma(x, c[GS_EXP_INV_LN2], mg);
  const double n = t - mg;
  const double r = fma(-n, c[GS_EXP_LN2], x);
  double p = c0;
#pragma unroll
  for (int i = 1; i <= GS_EXP_DEG; i++) p = fma(p, r, c[i]);
  return ldexp(p, (int)(unsigned)__builtin_bit_cast(unsigned long long, t));
}

GS_HD inline double exp_cw(double x, const double *c, double c0, double mg) {
  return exp_cw_unclamped(fmax(x, -1000.0), c, c0, mg);
}

GS_HD inline double exp_cw(double x, const double *c) { return exp_cw(x, c, c[0], c[GS_EXP_SHIFT]); }

}  // namespace gs
