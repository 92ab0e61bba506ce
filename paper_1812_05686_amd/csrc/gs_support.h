// gs_support.h -- per-cell bin support of the banded fold (host and device).
//
// A pair (bin j, cell i) is evaluated only when the cell's response
// log-density at the bin midpoint can exceed the cut T; the support of a
// cell is the bin range [x, y) where it can.  Everything here is
// conservative: a bin left out has a log-density <= T.
#pragma once
#include <math.h>

#include "gs_dev.h"

namespace gs {

struct Span {
  int x, y;
};

// Reco-bin midpoints xbar_j = bins[j * kBinLen], increasing.  When the
// binning is uniform (bw > 0: xbar_j = bx0 + j bw up to rounding) the index
// is guessed arithmetically and then corrected against the midpoints, so the
// result is the same as the binary search's.

// min { j : xbar_j >= x } (n if none).
GS_HD inline int bin_at_or_above(const double *bins, int n, double x, double bx0, double bw) {
  if (bw > 0.0) {
    int j = (int)fmin(fmax(ceil((x - bx0) / bw), 0.0), (double)n);
    while (j > 0 && bins[(size_t)(j - 1) * kBinLen] >= x) j--;
    while (j < n && bins[(size_t)j * kBinLen] < x) j++;
    return j;
  }
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (bins[(size_t)mid * kBinLen] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// min { j : xbar_j > x } (n if none).
GS_HD inline int bin_above(const double *bins, int n, double x, double bx0, double bw) {
  if (bw > 0.0) {
    int j = (int)fmin(fmax(floor((x - bx0) / bw) + 1.0, 0.0), (double)n);
    while (j > 0 && bins[(size_t)(j - 1) * kBinLen] > x) j--;
    while (j < n && bins[(size_t)j * kBinLen] <= x) j++;
    return j;
  }
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (bins[(size_t)mid * kBinLen] <= x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Interval [xl, xr] outside of which the gamma log-density
// E(x) = (k-1) ln x - x/th + C is at most T; xl = -inf when the interval
// reaches below x_lo (the smallest positive bin midpoint, or 0 if none).
//
// Newton's method on a concave function, started outside a root, approaches
// the root monotonically without crossing it (the tangent lies above the
// function), so every iterate is a conservative end point.  In u = ln x,
// E = (k-1) u - e^u/th + C is concave for every k and nearly linear far to
// the left; for k > 1 it is also concave in x and nearly linear far to the
// right.  So the right end is found in x when k > 1, the left end (k > 1
// only: for k <= 1 the density does not vanish at 0) and the k <= 1 right
// end in u.  Iterating stops once a step moves x by less than 2% of the
// standard deviation, far below a bin at these widths.
//
// For k > 1 the iterations start from the Wilson-Hilferty approximation: the
// cube root of x / (k th) is close to normal with mean 1 - 1/(9k) and
// variance 1/(9k), so the level T lies near z = sqrt(2 (E(mode) - T)) standard
// deviations of it; half a deviation is added outwards, and a start that
// still lies inside is moved outwards (doubling its distance from the mode)
// until E <= T.  From there one or two Newton steps reach the tolerance.
GS_HD inline bool gamma_support(double k, double th, double C, double T, double x_lo, double &xl, double &xr) {
  const double sd = sqrt(k) * th, tol = 0.02 * sd, ith = 1.0 / th;
  auto El = [&](double x, double lx) { return (k - 1.0) * lx - x * ith + C; };  // lx = ln x
  xl = -INFINITY;
  if (k > 1.0) {
    const double xm = (k - 1.0) * th, lxm = log(xm);
    const double Em = El(xm, lxm);
    if (!(Em > T)) return false;
    const double s3 = 1.0 / (3.0 * sqrt(k)), mu3 = 1.0 - s3 * s3, kt = k * th;
    const double z = sqrt(2.0 * (Em - T)) + 0.5;
    // right end, in x
    double y = mu3 + z * s3;
    double x = fmax(kt * y * y * y, xm + sd), lx = log(x), E = El(x, lx);
    for (int i = 0; i < 80 && E > T; i++) {
      x = xm + 2.0 * (x - xm);
      lx = log(x);
      E = El(x, lx);
    }
    for (int i = 0; i < 40; i++) {
      const double nx = x - (E - T) / ((k - 1.0) / x - ith);
      if (!(nx < x)) break;
      const bool done = x - nx < tol;
      x = nx;
      if (done) break;
      lx = log(x);
      E = El(x, lx);
    }
    xr = x;
    // left end, in u, from a point where E <= T that is not below the first bin
    const double floor_x = x_lo > 0.0 ? x_lo : xm * 0x1p-64;
    if (!(floor_x < xm)) return true;  // the support reaches the lowest bin
    const double lf = log(floor_x), Ef = El(floor_x, lf);
    if (Ef > T) return true;
    y = mu3 - z * s3;
    x = y > 0.0 ? fmin(kt * y * y * y, xm - sd) : floor_x;
    if (x > floor_x) {
      lx = log(x);
      E = El(x, lx);
      for (int i = 0; i < 80 && E > T; i++) {
        x = xm - 2.0 * (xm - x);
        if (!(x > floor_x)) break;
        lx = log(x);
        E = El(x, lx);
      }
    }
    if (!(x > floor_x) || E > T) {
      x = floor_x;
      lx = lf;
    }
    double u = lx, ex = x;
    for (int q = 0; q < 40; q++) {
      const double nu = u - ((k - 1.0) * u - ex * ith + C - T) / ((k - 1.0) - ex * ith);
      if (!(nu > u) || !(nu < lxm)) break;
      const double nex = exp(nu);
      const bool done = nex - ex < tol;
      u = nu;
      ex = nex;
      if (done) break;
    }
    xl = ex;
    return true;
  }
  // k <= 1: right end, in u, from just outside x = th (C - T), where the
  // decreasing density meets T if the log term is ignored
  double u = log(th * fmax(C - T, 1.0) + sd);
  double ex = exp(u);
  for (int i = 0; i < 80 && (k - 1.0) * u - ex * ith + C > T; i++) {
    u += 0.6931471805599453;
    ex = exp(u);
  }
  for (int i = 0; i < 60; i++) {
    const double nu = u - ((k - 1.0) * u - ex * ith + C - T) / ((k - 1.0) - ex * ith);
    if (!(nu < u)) break;
    const double nex = exp(nu);
    const bool done = ex - nex < tol;
    u = nu;
    ex = nex;
    if (done) break;
  }
  xr = ex;
  return true;
}

// Reco bins [x, y) whose midpoint log-density can exceed T for a cell with
// record rc (see cell_record) and moments m, s.  An invalid response has an
// empty support; T = -inf gives every bin.
GS_HD inline Span cell_support(int fam, const double *rc, double m, double s, bool ok, const double *bins, int n_reco,
                               double bx0, double bw, double T) {
  if (!ok) return {0, 0};
  if (!(T > -INFINITY)) return {0, n_reco};
  double xl, xr;
  if (fam == kGammaPE) {
    const double s2 = s * s;
    // smallest positive bin midpoint (the midpoints increase)
    const int jp = bin_above(bins, n_reco, 0.0, bx0, bw);
    const double x_lo = jp < n_reco ? bins[(size_t)jp * kBinLen] : 0.0;
    if (!gamma_support(m * m / s2, s2 / m, rc[3] + rc[4], T, x_lo, xl, xr)) return {0, 0};
  } else {
    const double c0 = rc[2];
    if (!(c0 > T)) return {0, 0};
    const double h = s * sqrt(2.0 * (c0 - T));
    xl = m - h;
    xr = m + h;
  }
  return {bin_at_or_above(bins, n_reco, xl, bx0, bw), bin_above(bins, n_reco, xr, bx0, bw)};
}

}  // namespace gs
