// Host check of the banded fold's per-cell supports (paper_1812_05686_amd/csrc/gs_support.h):
// every bin whose midpoint log-density exceeds the cut lies inside the support
// (brute force over all bins, log-density in long double), the support is at
// most a few bins wider than needed, and the arithmetic bin search for uniform
// binnings returns the binary search's index.  Prints one JSON line.
#include <cmath>
#include <cstdio>
#include <vector>

#include "gs_support.h"

using namespace gs;
typedef long double ld;

static ld logdens(int fam, ld x, ld m, ld s) {
  if (fam == kGammaPE) {
    if (!(x > 0)) return -INFINITY;
    const ld k = m * m / (s * s), th = s * s / m;
    return (k - 1) * logl(x) - x / th - lgammal(k) - k * logl(th);
  }
  const ld z = (x - m) / s;
  return -0.5L * z * z - logl(s) - 0.5L * logl(2 * 3.14159265358979323846264338327950288L);
}

struct Res {
  long cells = 0, missed = 0, empty_bad = 0, idx_mismatch = 0;
  int max_extra = 0;
};

static void run(int fam, const double *resp, double A, int n_true, double e_step, const std::vector<double> &edges,
                bool uniform, double T, Res &r) {
  const int n = (int)edges.size() - 1;
  std::vector<double> bins((size_t)n * kBinLen);
  for (int j = 0; j < n; j++) {
    const double x = (edges[j] + edges[j + 1]) * 0.5;
    bins[(size_t)j * kBinLen] = x;
    bins[(size_t)j * kBinLen + 1] = edges[j + 1] - edges[j];
  }
  const double bx0 = bins[0], bw = uniform ? (bins[(size_t)(n - 1) * kBinLen] - bins[0]) / (n - 1) : 0.0;
  // index search equivalence on a sweep of points, including the midpoints themselves
  if (uniform)
    for (int q = -40; q < 40 * n + 40; q++) {
      const double x = bins[0] - 3 * bw + q * (bw / 40.0) * 1.0000001;
      if (bin_at_or_above(bins.data(), n, x, bx0, bw) != bin_at_or_above(bins.data(), n, x, 0, 0)) r.idx_mismatch++;
      if (bin_above(bins.data(), n, x, bx0, bw) != bin_above(bins.data(), n, x, 0, 0)) r.idx_mismatch++;
    }
  for (int i = 0; i < n_true; i++) {
    const double E = (i + 0.5) * e_step;
    Moments mo;
    const bool ok = moments(fam, resp, A, E, mo);
    double rec[kRecLen];
    cell_record(fam, mo.m, mo.s, 1.0, ok, rec);
    const Span sp = cell_support(fam, rec, mo.m, mo.s, ok, bins.data(), n, bx0, bw, T);
    if (!ok) continue;
    r.cells++;
    int lo = n, hi = 0;
    for (int j = 0; j < n; j++)
      if (logdens(fam, bins[(size_t)j * kBinLen], mo.m, mo.s) > T) {
        lo = j < lo ? j : lo;
        hi = j + 1;
        if (j < sp.x || j >= sp.y) r.missed++;
      }
    if (hi <= lo) {
      if (sp.y - sp.x > 4) r.empty_bad++;
      continue;
    }
    const int extra = (lo - sp.x) > (sp.y - hi) ? lo - sp.x : sp.y - hi;
    if (extra > r.max_extra) r.max_extra = extra;
  }
}

int main() {
  Res r;
  const double pe[5] = {500.0, 0.011, 2.0, 1.15, 0.015};
  const double pe2[5] = {480.0, 0.013, 1.2, 0.6, 0.03};
  const double ke[2] = {10.0, 5.0};
  std::vector<double> u900(901), u200(201), nonu(301);
  for (int j = 0; j <= 900; j++) u900[j] = 1.6 * j;
  for (int j = 0; j <= 200; j++) u200[j] = 10.0 * j;
  for (int j = 0; j <= 300; j++) nonu[j] = 1440.0 * std::pow(j / 300.0, 1.5);
  for (double T : {-60.0, -20.0}) {
    run(kGammaPE, pe, 2.0, 4000, 0.00075, u900, true, T, r);
    run(kGammaPE, pe2, 2.0, 1000, 0.003, u900, true, T, r);
    run(kGaussPE, pe, 2.0, 4000, 0.00075, u900, true, T, r);
    run(kGaussE, ke, 2.0, 500, 5.0, u200, true, T, r);
    run(kGammaPE, pe, 2.0, 1000, 0.003, nonu, false, T, r);
  }
  printf("{\"cells\": %ld, \"missed\": %ld, \"empty_bad\": %ld, \"idx_mismatch\": %ld, \"max_extra\": %d}\n", r.cells,
         r.missed, r.empty_bad, r.idx_mismatch, r.max_extra);
  return 0;
}
