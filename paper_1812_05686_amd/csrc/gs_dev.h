// gs_dev.h -- device-side arithmetic of the fold likelihood for gfx950.
//
// Per-cell response constants and per-pair response evaluation
// (section 2.3 response families, section 2.5 mesh evaluation).  The gamma
// family's log-density has terms of size ~k ln x (~10^4 at k ~ 10^3) that
// cancel to O(1); the per-pair exponent is therefore evaluated from
// double-double per-cell and per-bin constants with error-free products,
// so one FP64 exp per pair keeps the per-bin relative error near 1e-15.
#pragma once
#ifdef __HIPCC__
#include <hip/hip_runtime.h>
#endif
#include <math.h>
#include <stdint.h>

#include "gs_exp.h"

// The error-free transformations below (two_sum, the hi/lo splits of the
// per-pair exponent) are only exact when every product and sum is rounded
// on its own; contracting a product into a neighbouring add (allowed by the
// device compiler's default) silently double-counts the rounding error
// terms.  Contraction is therefore switched off in this header: the fused
// operations it needs are written as explicit fma() calls.  The includer's
// setting is restored at the end of the header.
#pragma clang fp contract(off)

namespace gs {

constexpr int kRecLen = 8;  // doubles per cell record
constexpr int kBinLen = 4;     // doubles per static bin record: xbar, dx, ln xbar (hi, lo)
constexpr int kBinRecLen = 8;  // doubles per evaluated window bin: x, ln x (hi, lo), G, G ln x, G x, u, v
constexpr double kHalfLn2Pi = 0.91893853320467274178032973640561764;  // ln(2 pi)/2
// ln 2 as an unevaluated sum hi + lo (hi = nearest double)
constexpr double kLn2Hi = 0.6931471805599453094;   // 0x1.62e42fefa39efp-1
constexpr double kLn2Lo = 2.319046813846299558e-17;

enum Family : int {
  kGaussE = 0, kGaussPE = 1, kGammaPE = 2, kTemplate = 3,
  kGenGammaPE = 4, kSPoisPE = 5, kEmgPE = 6  // evaluated by the direct per-pair path (gs_gen.h)
};

struct dd {
  double hi, lo;
};

GS_HD inline dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}

GS_HD inline dd two_prod(double a, double b) {
  double p = a * b;
  return {p, fma(a, b, -p)};
}

// Natural log of a positive double as hi + lo with |error| ~ 1e-19 relative.
// x = 2^e f, f in [1/sqrt2, sqrt2); ln f = 2 atanh(s), s = (f - 1)/(f + 1),
// |s| <= 0.1716, with s carried as a double-double quotient.
GS_HD inline dd dd_log(double x) {
  int e;
  double f = frexp(x, &e);  // f in [0.5, 1)
  if (f < 0.70710678118654752440) {
    f *= 2.0;
    e -= 1;
  }
  double num = f - 1.0;  // exact for f in [0.5, 2]
  dd den = two_sum(f, 1.0);
  double sh = num / den.hi;
  double rem = fma(-sh, den.hi, num) - sh * den.lo;
  double sl = rem / den.hi;
  double s2 = sh * sh;
  // atanh(s)/s - 1 = s^2/3 + s^4/5 + ... through s^24/25
  double t = 1.0 / 25;
  t = fma(t, s2, 1.0 / 23);
  t = fma(t, s2, 1.0 / 21);
  t = fma(t, s2, 1.0 / 19);
  t = fma(t, s2, 1.0 / 17);
  t = fma(t, s2, 1.0 / 15);
  t = fma(t, s2, 1.0 / 13);
  t = fma(t, s2, 1.0 / 11);
  t = fma(t, s2, 1.0 / 9);
  t = fma(t, s2, 1.0 / 7);
  t = fma(t, s2, 1.0 / 5);
  t = fma(t, s2, 1.0 / 3);
  t *= s2;
  // 2 atanh(sh + sl) = 2 sh + 2 (sh t + sl (1 + sh^2)) + O(sl^2)
  double tail = 2.0 * fma(sh, t, sl * (1.0 + s2));
  dd le = two_prod((double)e, kLn2Hi);
  le.lo = fma((double)e, kLn2Lo, le.lo);
  dd r = two_sum(le.hi, 2.0 * sh);
  double lo = r.lo + le.lo + tail;
  return two_sum(r.hi, lo);
}

// Remainder of Stirling's formula, s(k) = lgamma(k) - (k - 1/2) ln k + k - ln(2 pi)/2.
// For k >= 12 the asymptotic series sum_n B_2n / (2n (2n-1) k^(2n-1)); below,
// the exact recurrence s(k) = s(k+1) + (k + 1/2) ln(1 + 1/k) - 1.
GS_HD inline double stirling_rem(double k) {
  double acc = 0.0;
  while (k < 12.0) {
    acc += fma(k + 0.5, log1p(1.0 / k), -1.0);
    k += 1.0;
  }
  double r = 1.0 / k, r2 = r * r;
  double p = -3617.0 / 122400.0;
  p = fma(p, r2, 1.0 / 156.0);
  p = fma(p, r2, -691.0 / 360360.0);
  p = fma(p, r2, 1.0 / 1188.0);
  p = fma(p, r2, -1.0 / 1680.0);
  p = fma(p, r2, 1.0 / 1260.0);
  p = fma(p, r2, -1.0 / 360.0);
  p = fma(p, r2, 1.0 / 12.0);
  return acc + p * r;
}

// ln k - psi(k): asymptotic series for k >= 8 (no cancellation), else shifted
// up with psi(k) = psi(k + n) - sum_{j<n} 1/(k + j).
GS_HD inline double log_minus_digamma(double k) {
  double acc = 0.0, k0 = k;
  while (k < 8.0) {
    acc += 1.0 / k;
    k += 1.0;
  }
  double r = 1.0 / k, r2 = r * r;
  // ln k - psi(k) = 1/(2k) + 1/(12k^2) - 1/(120k^4) + 1/(252k^6) - 1/(240k^8) + 1/(132k^10)
  //                 - 691/(32760k^12) + 1/(12k^14)
  double p = 1.0 / 12.0;
  p = fma(p, r2, -691.0 / 32760.0);
  p = fma(p, r2, 1.0 / 132.0);
  p = fma(p, r2, -1.0 / 240.0);
  p = fma(p, r2, 1.0 / 252.0);
  p = fma(p, r2, -1.0 / 120.0);
  p = fma(p, r2, 1.0 / 12.0);
  double v = fma(p, r2, 0.5 * r);
  if (k != k0) v += acc - log(k / k0);  // ln k0 - psi(k0) = [ln k - psi(k)] - ln(k/k0) + sum 1/(k0+j)
  return v;
}

// Birks quenching factor Q(E) = 1 - 2/y + 2 ln(1+y)/y^2, y = sqrt(E)/(kB A),
// and dQ/dkB.  Below y = 0.05 the series 2 sum (-1)^(n+1) y^n/(n+2).
GS_HD inline double quench(double E, double kB, double A, double *dQ_dkB) {
  if (!(E > 0.0)) {
    *dQ_dkB = 0.0;
    return 0.0;
  }
  double y = sqrt(E) / (kB * A);
  double Q, dQdy;
  if (y < 0.05) {
    Q = 0.0;
    dQdy = 0.0;
    double yn = 1.0;
    for (int n = 1; n <= 14; n++) {
      double c = ((n & 1) ? 2.0 : -2.0) / (n + 2);
      dQdy = fma(c * n, yn, dQdy);
      yn *= y;
      Q = fma(c, yn, Q);
    }
  } else {
    double iy = 1.0 / y;
    double L = log1p(y);
    Q = 1.0 - 2.0 * iy + 2.0 * L * iy * iy;
    dQdy = 2.0 * iy * iy - 4.0 * L * iy * iy * iy + 2.0 * iy * iy / (1.0 + y);
  }
  *dQ_dkB = -dQdy * y / kB;
  return Q;
}

// Response moments m(E), s(E) and their derivatives w.r.t. the response
// parameters (a, b) or (LY, kB, a, b, c).  Returns false for an invalid response.
struct Moments {
  double m, s;
  double dm[5], ds[5];
};

GS_HD inline bool moments(int fam, const double *resp, double A, double E, Moments &o) {
#pragma unroll
  for (int p = 0; p < 5; p++) o.dm[p] = o.ds[p] = 0.0;
  if (fam == kGaussE) {
    double a = resp[0], b = resp[1];
    double s2 = fma(b, E, a * a);
    o.m = E;
    o.s = sqrt(s2);
    o.ds[0] = a / o.s;
    o.ds[1] = 0.5 * E / o.s;
    return s2 > 0.0 && s2 < 1e300;
  }
  double LY = resp[0], kB = resp[1], a = resp[2], b = resp[3], c = resp[4];
  if (!(kB > 0.0)) {
    o.m = o.s = 0.0;
    return false;
  }
  double dQ;
  double Q = quench(E, kB, A, &dQ);
  double m = LY * Q * E;
  double s2 = a * a + b * m + c * c * m * m;
  double s = sqrt(s2);
  o.m = m;
  o.s = s;
  o.dm[0] = Q * E;
  o.dm[1] = LY * E * dQ;
  double dsdm = (b + 2.0 * c * c * m) / (2.0 * s);
  o.ds[0] = dsdm * o.dm[0];
  o.ds[1] = dsdm * o.dm[1];
  o.ds[2] = a / s;
  o.ds[3] = 0.5 * m / s;
  o.ds[4] = c * m * m / s;
  bool ok = s2 > 0.0 && s2 < 1e300;
  if (fam == kGammaPE || fam == kGenGammaPE || fam == kSPoisPE) ok = ok && m > 0.0;
  return ok;
}

// Per-cell record (8 doubles), consumed by the fold and adjoint loops.
//  gamma:    {k - 1, 1/th hi, 1/th lo, C hi, C lo, W, support, 0}
//            C = -lgamma(k) - k ln th, in double-double
//  gaussian: {m, 1/s, -ln s - ln(2 pi)/2, W, 0, 0, support, 0}
// W = sum_s R_s w_si (1-D combined weight).  Slot 6 holds the cell's bin
// support as two int32 (written by the caller).  Invalid responses are
// flagged by the caller; their records are zeros.
GS_HD inline void cell_record(int fam, double m, double s, double W, bool ok, double *rec) {
  for (int q = 0; q < kRecLen; q++) rec[q] = 0.0;
  if (!ok) return;
  if (fam == kGammaPE) {
    double s2 = s * s;
    double k = m * m / s2;
    double th = s2 / m;
    double bh = 1.0 / th;
    double bl = fma(-bh, th, 1.0) * bh;
    dd mk = two_prod(k, th);             // k th = mean, exactly as hi + lo
    dd lm = dd_log(mk.hi);
    lm.lo += mk.lo / mk.hi;
    // C = -k ln(k th) + k + ln(k)/2 - ln(2 pi)/2 - s(k)
    dd p = two_prod(k, lm.hi);
    p.lo = fma(k, lm.lo, p.lo);
    dd c1 = two_sum(-p.hi, k);
    double small = 0.5 * log(k) - kHalfLn2Pi - stirling_rem(k) - p.lo;
    dd C = two_sum(c1.hi, c1.lo + small);
    rec[0] = k - 1.0;
    rec[1] = bh;
    rec[2] = bl;
    rec[3] = C.hi;
    rec[4] = C.lo;
    rec[5] = W;
  } else {
    rec[0] = m;
    rec[1] = 1.0 / s;
    rec[2] = -log(s) - kHalfLn2Pi;
    rec[3] = W;
  }
}

// Per-pair log-density: gamma uses the bin's x and ln x as double-double.
GS_HD inline double gamma_exponent(double K, double Bh, double Bl, double Ch, double Cl,
                                                 double x, double Lh, double Ll) {
  double p = K * Lh;
  double ep = fma(K, Lh, -p);
  double q = x * Bh;
  double eq = fma(x, Bh, -q);
  double t = (p + Ch) - q;
  double corr = fma(K, Ll, ep) - eq;
  corr = fma(-x, Bl, corr) + Cl;
  return t + corr;
}

GS_HD inline double gauss_exponent(double m, double is, double c0, double x, double &z) {
  z = (x - m) * is;
  return fma(-0.5 * z, z, c0);
}

// Pair exponent relative to a reference point xr (a bin midpoint, with
// ln xr as hi + lo), used where many pairs share xr (a fold tile, an adjoint
// bin block):  E(x) = Eref + A u + B v  with
//   gamma:    u = ln x - ln xr, v = x - xr;      A = k - 1, B = -1/th
//   Gaussian: u = x - xr,      v = (x - xr)^2;   A = (m - xr)/s^2, B = -1/(2 s^2)
// and Eref = E(xr), formed from the cell record (double-double for gamma).
// With u and v small (xr within a tile or block of x), rounding adds about
// u_64 (|A u| + |B v| + |E|) to E, instead of u_64 |(k - 1) ln x| for a
// plain evaluation.
struct RelCell {
  double A, B, Eref;
};

GS_HD inline RelCell rel_cell(int fam, const double *rc, double xr, double Lhr, double Llr) {
  if (fam == kGammaPE) return {rc[0], -rc[1], gamma_exponent(rc[0], rc[1], rc[2], rc[3], rc[4], xr, Lhr, Llr)};
  const double is = rc[1], z = (xr - rc[0]) * is;
  return {-z * is, -0.5 * is * is, fma(-0.5 * z, z, rc[2])};
}

GS_HD inline void rel_offsets(int fam, double x, double Lh, double Ll, double xr, double Lhr, double Llr, double &u,
                              double &v) {
  if (fam == kGammaPE) {
    u = (Lh - Lhr) + (Ll - Llr);
    v = x - xr;
  } else {
    u = x - xr;
    v = u * u;
  }
}

GS_HD inline double rel_exponent(double A, double B, double Eref, double u, double v) {
  return fma(A, u, fma(B, v, Eref));
}

}  // namespace gs

#pragma clang fp contract(fast)
