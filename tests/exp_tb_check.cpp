// Host build of the table-driven device exponential (gs_exp.h, exp_tb) checked
// against long-double expl: the relative error over the log-densities a banded
// fold keeps ([-60, 1]), its growth with |n| (x = n ln2/256 + r) over the whole
// normal range against the bound 1.8e-14 + |n| 1.0e-19 the header states, the
// subnormal range (that bound plus the rounding to a subnormal, in units of the
// smallest subnormal), every table entry (x = j ln2/256), special values (NaN
// included: the index stays inside the table), and that the unclamped
// variant agrees with it bit for bit on [kExpTbNoClampMin, 709].
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <random>

#include "gs_exp.h"

int main() {
  const double c[GS_EXPT_NCOEF] = GS_EXPT_COEFS;
  const double tb[GS_EXPT_N] = GS_EXPT_TABLE;
  const double c3 = c[0], mg = c[GS_EXPT_SHIFT];
  auto e = [&](double x) { return gs::exp_tb(x, c, c3, tb, mg); };
  double max_rel = 0, worst = 0, max_rel_kept = 0, max_ratio = 0, max_sub = 0, max_table = 0;
  long n_bad_special = 0, n = 0;
  std::mt19937_64 rng(1812);
  std::uniform_real_distribution<double> U(-708.0, 709.0), V(-1.0, 1.0), K(-60.0, 1.0);
  auto bound = [](double x) { return 1.8e-14 + std::fabs(std::nearbyint(x * 256.0 / 0.6931471805599453)) * 1.0e-19; };
  auto check = [&](double x) {
    const long double ref = expl((long double)x);
    const double got = e(x);
    n++;
    if (x >= -708.0) {
      const double rel = (double)fabsl((got - ref) / ref);
      if (rel > max_rel) {
        max_rel = rel;
        worst = x;
      }
      if (x >= -60.0 && x <= 1.0 && rel > max_rel_kept) max_rel_kept = rel;
      if (rel / bound(x) > max_ratio) max_ratio = rel / bound(x);
    } else {
      const double ab = (double)((fabsl(got - ref) - bound(x) * ref) / 4.9406564584124654e-324L);
      if (ab > max_sub) max_sub = ab;
    }
  };
  for (int i = 0; i < 2000000; i++) check(U(rng));
  for (int i = 0; i < 2000000; i++) check(V(rng));
  for (int i = 0; i < 2000000; i++) check(K(rng));
  for (double x = -0.5; x <= 0.5; x += 1.0 / 4096) check(x);
  for (double x = -760.0; x < -700.0; x += 0.01) check(x);
  // each table entry is 2^(j/256) to within half an ulp
  for (int j = 0; j < GS_EXPT_N; j++) {
    const long double ref = exp2l((long double)j / GS_EXPT_N);
    const double rel = (double)fabsl((tb[j] - ref) / ref);
    if (rel > max_table) max_table = rel;
    check(j * 0.6931471805599453 / GS_EXPT_N);
    check(-j * 0.6931471805599453 / GS_EXPT_N - 1.0);
  }
  if (e(-746.0) != 0.0) n_bad_special++;
  if (e(-1.0e6) != 0.0) n_bad_special++;
  if (e(-1.0e30) != 0.0) n_bad_special++;
  if (!(std::fabs(e(0.0) - 1.0) <= 1.8e-14)) n_bad_special++;
  if (!std::isinf(e(710.0))) n_bad_special++;
  // NaN: the clamp turns it into -1000 (result 0, as exp_cw); unclamped, the
  // index is masked and the result is NaN
  if (e(std::numeric_limits<double>::quiet_NaN()) != 0.0) n_bad_special++;
  if (!std::isnan(gs::exp_tb_unclamped(std::numeric_limits<double>::quiet_NaN(), c, c3, tb, mg))) n_bad_special++;
  long n_unclamped_diff = 0;
  std::uniform_real_distribution<double> W(gs::kExpTbNoClampMin, 709.0), Z(-1.0e6, -700.0);
  auto same = [&](double x) {
    const double a = e(x), b = gs::exp_tb_unclamped(x, c, c3, tb, mg);
    if (std::memcmp(&a, &b, sizeof a) != 0) n_unclamped_diff++;
  };
  for (int i = 0; i < 1000000; i++) same(W(rng));
  for (int i = 0; i < 1000000; i++) same(Z(rng));
  for (int i = 0; i < 1000000; i++) same(K(rng));
  same(gs::kExpTbNoClampMin);
  same(-1000.0);
  same(0.0);
  printf(
      "{\"n\": %ld, \"max_rel\": %.6e, \"worst_x\": %.17g, \"max_rel_kept\": %.6e, \"max_bound_ratio\": %.3f, "
      "\"max_subnormal_ulps\": %.3f, \"max_table_rel\": %.3e, \"bad_special\": %ld, \"unclamped_diff\": %ld}\n",
      n, max_rel, worst, max_rel_kept, max_ratio, max_sub, max_table, n_bad_special, n_unclamped_diff);
  return 0;
}
