// Host build of the device exponential (gs_exp.h) checked against long-double expl:
// the relative error over the log-densities a banded fold keeps ([-60, 1]), its
// growth with |n| (x = n ln2 + r) over the whole normal range against the bound
// 1.45e-14 + |n| 2.4e-17 the header states, the subnormal range (that bound plus
// the rounding to a subnormal, in units of the smallest subnormal), special
// values, and that the unclamped variant agrees with it bit for bit on
// [kExpNoClampMin, 709].
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>

#include "gs_exp.h"

int main() {
  const double c[GS_EXP_NCOEF] = GS_EXP_COEFS;
  double max_rel = 0, worst = 0, max_rel_kept = 0, max_ratio = 0, max_sub = 0;
  long n_bad_special = 0, n = 0;
  std::mt19937_64 rng(1812);
  std::uniform_real_distribution<double> U(-708.0, 709.0), V(-1.0, 1.0), K(-60.0, 1.0);
  auto check = [&](double x) {
    const long double ref = expl((long double)x);
    const double got = gs::exp_cw(x, c);
    n++;
    if (x >= -708.0) {
      const double rel = (double)fabsl((got - ref) / ref);
      if (rel > max_rel) {
        max_rel = rel;
        worst = x;
      }
      if (x >= -60.0 && x <= 1.0 && rel > max_rel_kept) max_rel_kept = rel;
      const double bound = 1.45e-14 + std::fabs(std::nearbyint(x / 0.6931471805599453)) * 2.4e-17;
      if (rel / bound > max_ratio) max_ratio = rel / bound;
    } else {
      // subnormal / underflow range: error beyond the relative bound, in units of the
      // smallest subnormal
      const double bound = 1.45e-14 + std::fabs(std::nearbyint(x / 0.6931471805599453)) * 2.4e-17;
      const double ab = (double)((fabsl(got - ref) - bound * ref) / 4.9406564584124654e-324L);
      if (ab > max_sub) max_sub = ab;
    }
  };
  for (int i = 0; i < 2000000; i++) check(U(rng));
  for (int i = 0; i < 2000000; i++) check(V(rng));
  for (int i = 0; i < 2000000; i++) check(K(rng));
  for (double x = -0.5; x <= 0.5; x += 1.0 / 4096) check(x);
  for (double x = -760.0; x < -700.0; x += 0.01) check(x);
  if (gs::exp_cw(-746.0, c) != 0.0) n_bad_special++;
  if (gs::exp_cw(-1.0e6, c) != 0.0) n_bad_special++;
  if (gs::exp_cw(-1.0e30, c) != 0.0) n_bad_special++;
  if (!(std::fabs(gs::exp_cw(0.0, c) - 1.0) <= 1.45e-14)) n_bad_special++;
  if (!std::isinf(gs::exp_cw(710.0, c))) n_bad_special++;
  // the unclamped variant on its stated domain, including far below the underflow
  long n_unclamped_diff = 0;
  std::uniform_real_distribution<double> W(gs::kExpNoClampMin, 709.0), Z(-1.0e6, -700.0);
  auto same = [&](double x) {
    const double a = gs::exp_cw(x, c), b = gs::exp_cw_unclamped(x, c, c[0], c[GS_EXP_SHIFT]);
    if (std::memcmp(&a, &b, sizeof a) != 0) n_unclamped_diff++;
  };
  for (int i = 0; i < 1000000; i++) same(W(rng));
  for (int i = 0; i < 1000000; i++) same(Z(rng));
  for (int i = 0; i < 1000000; i++) same(K(rng));
  same(gs::kExpNoClampMin);
  same(-1000.0);
  same(0.0);
  printf(
      "{\"n\": %ld, \"max_rel\": %.6e, \"worst_x\": %.17g, \"max_rel_kept\": %.6e, \"max_bound_ratio\": %.3f, "
      "\"max_subnormal_ulps\": %.3f, \"bad_special\": %ld, \"unclamped_diff\": %ld}\n",
      n, max_rel, worst, max_rel_kept, max_ratio, max_sub, n_bad_special, n_unclamped_diff);
  return 0;
}
