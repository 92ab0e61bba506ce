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

// Table-driven variant, used by the pair loops: x = n ln2/64 + r with n =
// 64 e + j (0 <= j < 64) rounded as above and |r| <= ln2/128, so
// exp(x) = 2^e 2^(j/64) q(r).  q is the degree-4 polynomial that minimises
// the relative error of exp(r) on [-ln2/128, ln2/128] (remez_exp.py 4 64:
// 2.44e-15 after its coefficients are rounded; its constant term rounds to
// 1), and the table holds 2^(j/64) rounded to double (remez_exp.py prints it
// from 80-digit values).  ln2/64 is rounded to double (error 3.6e-19), so
// the relative error is below 2.9e-15 + |n| 3.7e-19: 5e-15 for arguments
// above -60 (exp_cw: 1.7e-14), in four FP64 operations fewer than exp_cw.
// The table index is the low six bits of n, so every argument, NaN
// included, reads inside the table.  Arguments below -1000 are raised to
// -1000 as for exp_cw (a NaN argument gives 0).
#define GS_EXPT_COEFS                                                                                   \
  { 0.041666615756061516, 0.1666669721299421, 0.5000000000026126, 0.9999999999977606,                 \
    92.33248261689366, 0.010830424696249145, 6755399441055744.0 }
#define GS_EXPT_NCOEF 7
#define GS_EXPT_INV (4)    // 64 / ln2
#define GS_EXPT_LN2 (5)    // ln2 / 64
#define GS_EXPT_SHIFT (6)  // 1.5 * 2^52
#define GS_EXPT_TABLE                                                                                   \
  {                                                                                                     \
        1.0, 1.0108892860517005, 1.0218971486541166, 1.0330248790212284,                          \
        1.0442737824274138, 1.0556451783605572, 1.0671404006768237, 1.0787607977571199,           \
        1.0905077326652577, 1.102382583307841, 1.1143867425958924, 1.1265216186082418,            \
        1.1387886347566916, 1.1511892299529827, 1.1637248587775775, 1.1763969916502812,           \
        1.189207115002721, 1.202156731452703, 1.215247359980469, 1.22848053610687,                \
        1.241857812073484, 1.255380757024691, 1.2690509571917332, 1.2828700160787783,             \
        1.2968395546510096, 1.3109612115247644, 1.3252366431597413, 1.339667524053303,            \
        1.3542555469368927, 1.3690024229745905, 1.383909881963832, 1.3989796725383112,            \
        1.4142135623730951, 1.42961333839197, 1.4451808069770467, 1.460917794180647,              \
        1.4768261459394993, 1.4929077282912648, 1.5091644275934228, 1.5255981507445384,           \
        1.5422108254079407, 1.559004400237837, 1.5759808451078865, 1.593142151342267,             \
        1.6104903319492543, 1.6280274218573478, 1.645755478153965, 1.6636765803267364,            \
        1.681792830507429, 1.7001063537185235, 1.718619298122478, 1.7373338352737062,             \
        1.7562521603732995, 1.7753764925265212, 1.7947090750031072, 1.8142521755003989,           \
        1.8340080864093424, 1.8539791250833855, 1.8741676341103, 1.8945759815869656,              \
        1.9152065613971474, 1.9360617934922943, 1.9571441241754002, 1.978456026387951             \
  }

// Arguments at or above kExpTbNoClampMin may skip the lower clamp: there n
// is below 2^31 in magnitude (64 |x| / ln2 < 2^31) and the result already
// underflows to 0 below about -745.
constexpr double kExpTbNoClampMin = -1.0e7;

// c: the coefficients (c[0] = the degree-4 one, meeting another scalar operand,
// is passed again as c4), tb: the table, mg = c[GS_EXPT_SHIFT].
GS_HD inline double exp_tb_unclamped(double x, const double *c, double c4, const double *tb, double mg) {
  const double t = fma(x, c[GS_EXPT_INV], mg);
  const double n = t - mg;
  const double r = fma(-n, c[GS_EXPT_LN2], x);
  double q = fma(c4, r, c[1]);
  q = fma(q, r, c[2]);
  q = fma(q, r, c[3]);
  q = fma(q, r, 1.0);
  const int ni = (int)(unsigned)__builtin_bit_cast(unsigned long long, t);
  return ldexp(q * tb[ni & 63], ni >> 6);
}

GS_HD inline double exp_tb(double x, const double *c, double c4, const double *tb, double mg) {
  return exp_tb_unclamped(fmax(x, -1000.0), c, c4, tb, mg);
}

}  // namespace gs
