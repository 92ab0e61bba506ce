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
// (k-1) ln x - x/th + C is at most T.  In u = ln x it reads
// E(u) = (k-1) u - e^u/th + C, concave for every k (in x it is convex when
// k < 1).  Newton's method on a concave function, started outside a root,
// approaches the root monotonically without crossing it (the tangent lies
// above the function), so every iterate is a conservative end point;
// iterating stops once a step moves x by less than 2% of the standard
// deviation, far below a bin at these widths.
GS_HD inline bool gamma_support(double k, double th, double C, double T, double &xl, double &xr) {
  auto E = [&](double u) { return (k - 1.0) * u - exp(u) / th + C; };
  auto dE = [&](double u) { return (k - 1.0) - exp(u) / th; };
  const double sd = sqrt(k) * th;
  const double tol = 0.02 * sd;
  double xm = 0.0, w = fmax(sd, th);
  if (k > 1.0) {
    xm = (k - 1.0) * th;
    const double Em = E(log(xm));
    if (!(Em > T)) return false;
    w = sd * sqrt(2.0 * (Em - T)) + sd;
  }
  // right end: E decreasing there
  double u = log(xm + w);
  for (int i = 0; i < 80 && E(u) > T; i++) u += 0.6931471805599453;
  for (int i = 0; i < 40; i++) {
    const double nu = u - (E(u) - T) / dE(u);
    if (!(nu < u)) break;
    const bool done = exp(u) - exp(nu) < tol;
    u = nu;
    if (done) break;
  }
  xr = exp(u);
  xl = -INFINITY;
  if (k > 1.0) {  // left end: E increasing below the mode (for k <= 1 the density has no left end)
    const double um = log(xm);
    u = xm - w > 0.0 ? log(xm - w) : um - 0.6931471805599453;
    for (int i = 0; i < 1100 && E(u) > T; i++) u -= 0.6931471805599453;
    if (E(u) <= T) {
      for (int q = 0; q < 40; q++) {
        const double nu = u - (E(u) - T) / dE(u);
        if (!(nu > u) || !(nu < um)) break;
        const bool done = exp(nu) - exp(u) < tol;
        u = nu;
        if (done) break;
      }
      xl = exp(u);
    }
  }
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
    if (!gamma_support(m * m / s2, s2 / m, rc[3] + rc[4], T, xl, xr)) return {0, 0};
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
