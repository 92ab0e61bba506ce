// Host check of the tile-relative pair exponent (rel_cell, rel_offsets,
// rel_exponent in paper_1812_05686_amd/csrc/gs_dev.h) that the 1-D fold and
// the adjoint evaluate per (bin, cell) pair.  For every cell of a response
// grid and every bin of the reco range, with the reference at the middle bin
// of the bin's 32-bin tile (the fold) and, for gamma, of its 64-bin block (the
// adjoint), as the kernels place them, the relative exponent
// is compared with the exponent the cell record defines, evaluated in
// quadruple precision (__float128; the gamma terms K ln x reach ~5e5 and
// cancel to O(10), beyond what long double resolves):
//   gamma:    E* = K ln x - x (Bh + Bl) + (Ch + Cl)
//   Gaussian: E* = c0 - ((x - m) is)^2 / 2
// Reports the worst |E - E*| over pairs with E* > -60 (the pairs a banded
// fold keeps), the worst ratio of that error to the rounding bound
// u (|A u| + |B v| + |Eref| + |E|), and the same error of the plain
// double-double per-pair exponent for comparison.  Prints one JSON line.
#include <quadmath.h>

#include <cmath>
#include <cstdio>
#include <vector>

#include "gs_dev.h"

using namespace gs;
typedef __float128 qd;

struct Res {
  long pairs = 0, tiles = 0;
  double max_err = 0.0, max_ratio = 0.0, max_err_dd = 0.0, max_rel_density = 0.0;
  // worst amount by which a bin inside a tile falls below the lower of the
  // tile's two end bins, in units of u (|A u| + |B v| + |Eref|) of that bin
  double max_below_ends = 0.0;
};

static void run(int fam, const double *resp, double A, int n_true, double e_step, const std::vector<double> &edges,
                Res &r, int W) {
  const int n = (int)edges.size() - 1;
  std::vector<double> x(n), Lh(n), Ll(n);
  for (int j = 0; j < n; j++) {
    x[j] = 0.5 * (edges[j] + edges[j + 1]);
    const dd L = x[j] > 0.0 ? dd_log(x[j]) : dd{0.0, 0.0};
    Lh[j] = L.hi;
    Ll[j] = L.lo;
  }
  const double u64 = std::ldexp(1.0, -53);
  for (int i = 0; i < n_true; i++) {
    const double E = (i + 0.5) * e_step;
    Moments mo;
    if (!moments(fam, resp, A, E, mo)) continue;
    double rc[kRecLen];
    cell_record(fam, mo.m, mo.s, 1.0, true, rc);
    // the pair loops' range check: within a tile the relative exponent is lowest
    // at one of the two end bins (checked on every tile of positive midpoints)
    for (int t0 = 0; t0 < n; t0 += W) {
      const int t1 = t0 + W < n ? t0 + W : n;
      if (fam == kGammaPE && !(x[t0] > 0.0)) continue;
      const int jr = t0 + W / 2 < t1 - 1 ? t0 + W / 2 : t1 - 1;
      const RelCell c = rel_cell(fam, rc, x[jr], Lh[jr], Ll[jr]);
      auto Eat = [&](int j, double &scale) {
        double u, v;
        rel_offsets(fam, x[j], Lh[j], Ll[j], x[jr], Lh[jr], Ll[jr], u, v);
        scale = u64 * (std::fabs(c.A * u) + std::fabs(c.B * v) + std::fabs(c.Eref)) + 1e-300;
        return rel_exponent(c.A, c.B, c.Eref, u, v);
      };
      double sf, sl;
      const double ends = std::fmin(Eat(t0, sf), Eat(t1 - 1, sl));
      for (int j = t0 + 1; j < t1 - 1; j++) {
        double sc;
        const double Ej = Eat(j, sc);
        if (ends - Ej > 0.0 && (ends - Ej) / sc > r.max_below_ends) r.max_below_ends = (ends - Ej) / sc;
      }
      r.tiles++;
    }
    for (int j = 0; j < n; j++) {
      if (fam == kGammaPE && !(x[j] > 0.0)) continue;
      qd Es;
      if (fam == kGammaPE)
        Es = (qd)rc[0] * logq((qd)x[j]) - (qd)x[j] * ((qd)rc[1] + (qd)rc[2]) + ((qd)rc[3] + (qd)rc[4]);
      else {
        const qd z = ((qd)x[j] - (qd)rc[0]) * (qd)rc[1];
        Es = (qd)rc[2] - (qd)0.5 * z * z;
      }
      if (!(Es > (qd)-60.0)) continue;
      const int t0 = j / W * W, last = (t0 + W < n ? t0 + W : n) - 1;
      int jr = t0 + W / 2 < last ? t0 + W / 2 : last;
      if (fam == kGammaPE && !(x[jr] > 0.0)) jr = last;
      const RelCell c = rel_cell(fam, rc, x[jr], Lh[jr], Ll[jr]);
      double u, v;
      rel_offsets(fam, x[j], Lh[j], Ll[j], x[jr], Lh[jr], Ll[jr], u, v);
      const double Er = rel_exponent(c.A, c.B, c.Eref, u, v);
      const double err = (double)fabsq((qd)Er - Es);
      const double bound = u64 * (std::fabs(c.A * u) + std::fabs(c.B * v) + std::fabs(c.Eref) + std::fabs(Er));
      double Edd, z;
      if (fam == kGammaPE)
        Edd = gamma_exponent(rc[0], rc[1], rc[2], rc[3], rc[4], x[j], Lh[j], Ll[j]);
      else
        Edd = gauss_exponent(rc[0], rc[1], rc[2], x[j], z);
      r.pairs++;
      if (err > r.max_err) r.max_err = err;
      if (bound > 0 && err / bound > r.max_ratio) r.max_ratio = err / bound;
      const double ed = (double)fabsq((qd)Edd - Es);
      if (ed > r.max_err_dd) r.max_err_dd = ed;
      const double rel = (double)fabsq(expm1q((qd)Er - Es));
      if (rel > r.max_rel_density) r.max_rel_density = rel;
    }
  }
}

int main() {
  Res g, k;
  // photoelectron families: the Borexino-scale response and a sharper one
  const double pe[5] = {500.0, 0.011, 2.0, 1.15, 0.015};
  const double pe2[5] = {1500.0, 0.011, 0.5, 0.3, 0.004};
  std::vector<double> u900(901), nonu(301), u200(201);
  for (int j = 0; j <= 900; j++) u900[j] = 1.6 * j;
  for (int j = 0; j <= 300; j++) nonu[j] = 1440.0 * std::pow(j / 300.0, 1.5);
  for (int j = 0; j <= 200; j++) u200[j] = 10.0 * j;
  const double ke[2] = {10.0, 5.0};
  // gamma: the fold's tiles and the adjoint's blocks; the Gaussian families use the
  // relative form in the fold only (the adjoint forms their exponent per pair)
  for (int W : {32, 64}) {
    run(kGammaPE, pe, 2.0, 4000, 0.00075, u900, g, W);
    run(kGammaPE, pe2, 2.0, 1000, 0.003, u900, g, W);
    run(kGammaPE, pe, 2.0, 1000, 0.003, nonu, g, W);
  }
  run(kGaussE, ke, 0.0, 500, 5.0, u200, k, 32);
  run(kGaussPE, pe, 2.0, 1000, 0.003, u900, k, 32);
  std::printf(
      "{\"gamma\": {\"pairs\": %ld, \"max_err\": %.3e, \"max_ratio\": %.3f, \"max_err_dd\": %.3e, "
      "\"max_rel_density\": %.3e, \"tiles\": %ld, \"max_below_ends\": %.3f}, \"gauss\": {\"pairs\": %ld, "
      "\"max_err\": %.3e, \"max_ratio\": %.3f, \"max_err_dd\": %.3e, \"max_rel_density\": %.3e, "
      "\"tiles\": %ld, \"max_below_ends\": %.3f}}\n",
      g.pairs, g.max_err, g.max_ratio, g.max_err_dd, g.max_rel_density, g.tiles, g.max_below_ends, k.pairs,
      k.max_err, k.max_ratio, k.max_err_dd, k.max_rel_density, k.tiles, k.max_below_ends);
  return 0;
}
