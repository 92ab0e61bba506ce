// gs_exp.h -- FP64 exponentials for the per-pair response evaluation: exp_tb
// (below; table-driven, what the pair loops call) and exp_cw, the plain
// Cody-Waite form it replaced (no table), kept with its own host accuracy
// test.
//
// exp_cw: exp(x) = 2^n p(r), x = n ln2 + r, |r| <= ln2/2 (Cody & Waite argument
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

// Table-driven variant, used by the pair loops: x = n ln2/256 + r with n =
// 256 e + j (0 <= j < 256) rounded as above and |r| <= ln2/512, so
// exp(x) = 2^e 2^(j/256) q(r).  q is the degree-3 polynomial that minimises
// the relative error of exp(r) on [-ln2/512, ln2/512] (remez_exp.py 3 256:
// 1.75e-14 after its coefficients are rounded), and the table holds
// 2^(j/256) rounded to double (remez_exp.py prints it from 80-digit values).
// ln2/256 is rounded to double (error 9.1e-20), so the relative error is
// below 1.8e-14 + |n| 1.0e-19: 2e-14 for arguments above -60, in five FP64
// operations fewer than exp_cw.  The table index is the low eight bits of n,
// so every argument, NaN included, reads inside the table.  Arguments below
// -1000 are raised to -1000 as for exp_cw (a NaN argument gives 0).
#define GS_EXPT_COEFS                                                                                   \
  { 0.1666666513934773, 0.5000000763659402, 1.0000000000000384, 0.9999999999999825,                   \
    369.3299304675746, 0.0027076061740622863, 6755399441055744.0 }
#define GS_EXPT_NCOEF 7
#define GS_EXPT_INV (4)    // 256 / ln2
#define GS_EXPT_LN2 (5)    // ln2 / 256
#define GS_EXPT_SHIFT (6)  // 1.5 * 2^52
#define GS_EXPT_N 256
#define GS_EXPT_TABLE                                                                                   \
  {                                                                                                     \
        1.0, 1.0027112750502025, 1.0054299011128027, 1.0081558981184175,                          \
        1.0108892860517005, 1.0136300849514894, 1.016378314910953, 1.019133996077738,             \
        1.0218971486541166, 1.0246677928971357, 1.0274459491187637, 1.030231637686041,            \
        1.0330248790212284, 1.0358256936019572, 1.0386341019613787, 1.041450124688316,            \
        1.0442737824274138, 1.0471050958792898, 1.0499440858006872, 1.0527907730046264,           \
        1.0556451783605572, 1.0585073227945128, 1.061377227289262, 1.0642549128844645,            \
        1.0671404006768237, 1.0700337118202419, 1.0729348675259756, 1.075843889062791,            \
        1.0787607977571199, 1.0816856149932152, 1.0846183622133092, 1.0875590609177697,           \
        1.0905077326652577, 1.0934643990728858, 1.0964290818163769, 1.099401802630222,            \
        1.102382583307841, 1.1053714457017412, 1.1083684117236787, 1.1113735033448175,            \
        1.1143867425958924, 1.1174081515673693, 1.1204377524096067, 1.12347556733302,             \
        1.1265216186082418, 1.129575928566288, 1.1326385195987192, 1.1357094141578055,            \
        1.1387886347566916, 1.1418762039695616, 1.1449721444318042, 1.148076478840179,            \
        1.1511892299529827, 1.154310420590216, 1.1574400736337511, 1.1605782120274988,            \
        1.1637248587775775, 1.1668800369524817, 1.1700437696832502, 1.1732160801636373,           \
        1.1763969916502812, 1.1795865274628758, 1.182784710984341, 1.1859915656609938,            \
        1.189207115002721, 1.1924313825831512, 1.1956643920398273, 1.1989061670743806,            \
        1.202156731452703, 1.2054161090051239, 1.2086843236265816, 1.2119613992768012,            \
        1.215247359980469, 1.2185422298274085, 1.2218460329727576, 1.2251587936371455,            \
        1.22848053610687, 1.2318112847340759, 1.2351510639369334, 1.2384998981998165,             \
        1.241857812073484, 1.245224830175258, 1.2486009771892048, 1.2519862778663162,             \
        1.255380757024691, 1.2587844395497165, 1.2621973503942507, 1.2656195145788063,            \
        1.2690509571917332, 1.2724917033894028, 1.275941778396392, 1.2794012075056693,            \
        1.2828700160787783, 1.2863482295460256, 1.2898358734066657, 1.2933329732290895,           \
        1.2968395546510096, 1.3003556433796506, 1.3038812651919358, 1.3074164459346773,           \
        1.3109612115247644, 1.3145155879493546, 1.318079601266064, 1.3216532776031575,            \
        1.3252366431597413, 1.3288297242059544, 1.3324325470831615, 1.3360451382041458,           \
        1.339667524053303, 1.3432997311868353, 1.3469417862329458, 1.3505937158920345,            \
        1.3542555469368927, 1.3579273062129011, 1.3616090206382248, 1.365300717204012,            \
        1.3690024229745905, 1.3727141650876684, 1.3764359707545302, 1.380167867260238,            \
        1.383909881963832, 1.387662042298529, 1.3914243757719262, 1.3951969099662003,             \
        1.3989796725383112, 1.4027726912202048, 1.4065759938190154, 1.4103896082172707,           \
        1.4142135623730951, 1.4180478843204152, 1.4218926021691656, 1.4257477441054942,           \
        1.42961333839197, 1.433489413367789, 1.4373759974489824, 1.4412731191286257,              \
        1.4451808069770467, 1.449099089642035, 1.4530279958490526, 1.4569675544014438,            \
        1.460917794180647, 1.4648787441464057, 1.4688504333369818, 1.4728328908693675,            \
        1.4768261459394993, 1.4808302278224719, 1.4848451658727524, 1.488870989524397,            \
        1.4929077282912648, 1.4969554117672355, 1.5010140696264256, 1.5050837316234065,           \
        1.5091644275934228, 1.5132561874526098, 1.5173590411982147, 1.5214730189088146,           \
        1.5255981507445384, 1.529734466947287, 1.533881997840956, 1.5380407738316568,             \
        1.5422108254079407, 1.5463921831410214, 1.550584877685, 1.5547889397770887,               \
        1.559004400237837, 1.5632312899713576, 1.567469639965553, 1.5717194812923414,             \
        1.5759808451078865, 1.5802537626528246, 1.5845382652524937, 1.588834384317164,            \
        1.593142151342267, 1.597461597908627, 1.6017927556826934, 1.606135656416771,              \
        1.6104903319492543, 1.6148568142048607, 1.6192351351948637, 1.6236253270173289,           \
        1.6280274218573478, 1.632441451987275, 1.6368674497669644, 1.6413054476440063,            \
        1.645755478153965, 1.6502175739206177, 1.6546917676561943, 1.6591780921616162,            \
        1.6636765803267364, 1.6681872651305825, 1.6727101796415966, 1.6772453570178785,           \
        1.681792830507429, 1.6863526334483934, 1.6909247992693053, 1.6955093614893326,            \
        1.7001063537185235, 1.7047158096580513, 1.709337763100463, 1.713972247929926,             \
        1.718619298122478, 1.723278947746274, 1.7279512309618377, 1.732636182022311,              \
        1.7373338352737062, 1.7420442251551564, 1.746767386199169, 1.7515033530318782,            \
        1.7562521603732995, 1.761013843037584, 1.7657884359332727, 1.7705759740635547,            \
        1.7753764925265212, 1.7801900265154245, 1.785016611318935, 1.789856282321401,             \
        1.7947090750031072, 1.7995750249405351, 1.804454167806624, 1.809346539371032,             \
        1.8142521755003989, 1.8191711121586085, 1.8241033854070534, 1.8290490314048973,           \
        1.8340080864093424, 1.8389805867758937, 1.843966568958626, 1.8489660695104508,            \
        1.8539791250833855, 1.8590057724288205, 1.864046048397789, 1.8690999899412386,            \
        1.8741676341103, 1.8792490180565602, 1.8843441790323345, 1.8894531543909392,              \
        1.8945759815869656, 1.8997126981765553, 1.9048633418176741, 1.9100279502703899,           \
        1.9152065613971474, 1.9203992131630474, 1.925605943636125, 1.930826790987627,             \
        1.9360617934922943, 1.9413109895286405, 1.9465744175792332, 1.9518521162309783,           \
        1.9571441241754002, 1.9624504802089273, 1.9677712232331759, 1.9731063922552343,           \
        1.978456026387951, 1.9838201648502194, 1.9891988469672663, 1.9945921121709402             \
  }

// Arguments at or above kExpTbNoClampMin may skip the lower clamp: there n
// is below 2^31 in magnitude (256 |x| / ln2 < 2^31) and the result already
// underflows to 0 below about -745.
constexpr double kExpTbNoClampMin = -1.0e6;

// c: the coefficients (c[0] = the degree-3 one, meeting another scalar operand,
// is passed again as c3), tb: the table, mg = c[GS_EXPT_SHIFT].
GS_HD inline double exp_tb_unclamped(double x, const double *c, double c3, const double *tb, double mg) {
  const double t = fma(x, c[GS_EXPT_INV], mg);
  const double n = t - mg;
  const double r = fma(-n, c[GS_EXPT_LN2], x);
  double q = fma(c3, r, c[1]);
  q = fma(q, r, c[2]);
  q = fma(q, r, c[3]);
  const int ni = (int)(unsigned)__builtin_bit_cast(unsigned long long, t);
  return ldexp(q * tb[ni & (GS_EXPT_N - 1)], ni >> 8);
}

GS_HD inline double exp_tb(double x, const double *c, double c3, const double *tb, double mg) {
  return exp_tb_unclamped(fmax(x, -1000.0), c, c3, tb, mg);
}

}  // namespace gs
