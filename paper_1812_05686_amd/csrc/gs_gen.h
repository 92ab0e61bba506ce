// gs_gen.h -- device arithmetic of the further response families and of
// exact reco-bin contents (section 2.3 names the modified Gaussian, the
// generalized gamma and the scaled Poisson; section 2.5 evaluates the
// response on the visible x true mesh).
//
// These responses go through a direct per-pair path (k_foldg, k_adjg): each
// pair evaluates the bin content K_ji of one cell in one reco bin and, in the
// adjoint, dK/dm and dK/ds, in FP64 without the tile-relative exponent of the
// Gaussian / gamma fast path.  The Poisson-type normalisations
// e^-u u^k / Gamma(k+1), whose terms k ln u and ln Gamma(k+1) reach ~1e5 and
// cancel to O(1), are formed in Loader's saddle-point form
// exp(-bd0(k, u) - s(k)) / sqrt(2 pi k) (bd0 = k ln(k/u) + u - k by its own
// series near u = k, s = Stirling's remainder), so that no large terms cancel.
//
// Families (mean m, standard deviation s per cell):
//  Gaussian (exact bins only)  N(m, s^2), K = Phi(z_hi) - Phi(z_lo) by erfc
//  gamma (exact bins only)     k = m^2/s^2, th = s^2/m, K from P(k, x/th)
//  generalized gamma           Stacy's density with power p (the model's
//                              shape), k = m^2/(p^2 s^2), th = m Gamma(k) /
//                              Gamma(k + 1/p); K from P(k, (x/th)^p)
//  scaled Poisson              Poisson(x/g; lambda)/g continued to real x by
//                              Gamma, g = s^2/m, lambda = m^2/s^2; midpoint
//                              rule only
//  modified Gaussian           N(mu_g, sg^2) convolved with an exponential of
//                              mean tau = f s (f: the model's shape),
//                              sg = s sqrt(1 - f^2), mu_g = m - tau
// P(k, u) is the regularised incomplete gamma, by its series below
// u = k + 1 and Legendre's continued fraction above, each with its
// derivative w.r.t. k carried term by term.
#pragma once
#include "gs_dev.h"

namespace gs {

constexpr double kSqrt2 = 1.41421356237309504880;
constexpr double kInvSqrt2Pi = 0.39894228040143267794;
constexpr int kIgamMaxIter = 20000;  // a bound only: the admitted shapes converge in a few hundred steps

// Loader's deviance term bd0(k, u) = k ln(k/u) + u - k >= 0, by the series in
// v = (k - u)/(k + u) where the direct form would cancel.
__device__ inline double bd0(double k, double u) {
  const double d = k - u;
  if (fabs(d) < 0.1 * (k + u)) {
    const double v = d / (k + u), v2 = v * v;
    double s = d * v, ej = 2.0 * k * v;
    for (int j = 1; j < 200; j++) {
      ej *= v2;
      const double s1 = s + ej / (2 * j + 1);
      if (s1 == s) break;
      s = s1;
    }
    return s;
  }
  return k * log(k / u) + u - k;
}

// ln of e^-u u^k / Gamma(k + 1) for k, u > 0 (sk = stirling_rem(k)).
__device__ inline double ln_pois(double k, double u, double sk) { return -bd0(k, u) - sk - kHalfLn2Pi - 0.5 * log(k); }

// lgamma(k + a) - lgamma(k) for k > 0, a > 0 without cancellation:
// s(k + a) - s(k) + (k - 1/2) ln(1 + a/k) + a ln(k + a) - a.
__device__ inline double lgamma_diff(double k, double a) {
  return stirling_rem(k + a) - stirling_rem(k) + (k - 0.5) * log1p(a / k) + a * log(k + a) - a;
}

struct Igam {
  double P, Q, dP;  // P(k, u), 1 - P, dP/dk
};

// Regularised incomplete gamma and (if deriv) its k-derivative; sk = stirling_rem(k).
__device__ inline Igam igam(double k, double u, double sk, bool deriv) {
  Igam o{0.0, 1.0, 0.0};
  if (!(u > 0.0)) return o;
  const double pre = exp(ln_pois(k, u, sk));  // e^-u u^k / Gamma(k+1)
  const double lku = log(k / u);
  if (u < k + 1.0) {
    double c = 1.0, S = 1.0, H = 0.0, dS = 0.0;
    for (int n = 1; n < kIgamMaxIter; n++) {
      const double r = 1.0 / (k + n);
      c *= u * r;
      S += c;
      if (deriv) {
        H += r;
        dS = fma(-c, H, dS);
      }
      if (c < 1e-17 * S && (!deriv || c * H <= 1e-17 * fabs(dS))) break;
    }
    o.P = pre * S;
    o.Q = 1.0 - o.P;
    // ln u - psi(k + 1) = -ln(k/u) - (psi(k+1) - ln k),  psi(k+1) - ln k = 1/k - (ln k - psi(k))
    if (deriv) o.dP = pre * fma(-lku - (1.0 / k - log_minus_digamma(k)), S, dS);
    return o;
  }
  // Gamma(k, u) e^u u^-k = 1/(b1 + a2/(b2 + ...)), b_i = u + 2i - 1 - k, a_i = -(i-1)(i-1-k):
  // modified Lentz, each convergent's k-derivative alongside
  const double tiny = 1e-300;
  double b = u + 1.0 - k, db = -1.0;
  double c = 1.0 / tiny, dc = 0.0;
  double d = 1.0 / b, dd = d * d;
  double h = d, dh = dd;
  for (int i = 1; i < kIgamMaxIter; i++) {
    const double an = -i * (i - k), dan = i;
    b += 2.0;
    double den = fma(an, d, b);
    const double dden = dan * d + an * dd + db;
    if (fabs(den) < tiny) den = tiny;
    const double dn = 1.0 / den, ddn = -dden * dn * dn;
    double cn = b + an / c;
    const double dcn = db + dan / c - an * dc / (c * c);
    if (fabs(cn) < tiny) cn = tiny;
    d = dn;
    dd = ddn;
    c = cn;
    dc = dcn;
    const double del = d * c, ddel = dd * c + d * dc;
    dh = dh * del + h * ddel;
    h *= del;
    if (fabs(del - 1.0) < 1e-16 && (!deriv || fabs(ddel * h) <= 1e-16 * fabs(dh))) break;
  }
  const double preQ = k * pre;  // e^-u u^k / Gamma(k)
  o.Q = preQ * h;
  o.P = 1.0 - o.Q;
  // ln u - psi(k) = -ln(k/u) + (ln k - psi(k))
  if (deriv) o.dP = -preQ * fma(-lku + log_minus_digamma(k), h, dh);
  return o;
}

// u = (x/th)^p, rounded once (x/th) or through pow: forming it as exp(p (ln x - ln th))
// would carry the ~1e-16 |ln x| error of the logarithms into u.
__device__ inline double gen_u(double p, double x, double th) { return p == 1.0 ? x / th : pow(x / th, p); }

// Per-cell constants of the direct path: {m, s, a, b, c, d} with
//  Gaussian: -;  gamma / gen. gamma: a = k, b = th, c = ln th, d = s(k);
//  scaled Poisson: a = g, b = lambda, c = ln lambda;  modified Gaussian: a = mu_g, b = sg, c = tau.
struct GenCell {
  double m, s, a, b, c, d;
};

__device__ inline bool gen_gamma_type(int fam) { return fam == kGammaPE || fam == kGenGammaPE; }

__device__ inline bool gen_cell(int fam, double p, double m, double s, GenCell &g) {
  g = {m, s, 0.0, 0.0, 0.0, 0.0};
  if (!(s > 0.0) || !isfinite(m) || !isfinite(s)) return false;
  if (gen_gamma_type(fam) || fam == kSPoisPE) {
    if (!(m > 0.0)) return false;
  }
  if (fam == kGammaPE) {
    g.a = (m / s) * (m / s);
    g.b = s * s / m;
  } else if (fam == kGenGammaPE) {
    const double q = m / (p * s);
    g.a = q * q;
    g.b = m * exp(-lgamma_diff(g.a, 1.0 / p));
  } else if (fam == kSPoisPE) {
    g.a = s * s / m;
    g.b = (m / s) * (m / s);
    g.c = log(g.b);
  } else if (fam == kEmgPE) {
    g.c = p * s;
    g.b = s * sqrt(1.0 - p * p);
    g.a = m - g.c;
  }
  if (gen_gamma_type(fam)) {
    g.c = log(g.b);
    g.d = stirling_rem(g.a);
  }
  return true;
}

// d(k, th)/d(m, s) of the gamma-type families (th = m Gamma(k)/Gamma(k + 1/p)).
struct GenChain {
  double k_m, k_s, t_m, t_s;
};

__device__ inline GenChain gen_chain(int fam, double p, const GenCell &g) {
  GenChain c{0.0, 0.0, 0.0, 0.0};
  if (!gen_gamma_type(fam)) return c;
  const double k = g.a, th = g.b;
  const double a = fam == kGammaPE ? 1.0 : 1.0 / p;
  // psi(k + a) - psi(k) = ln(1 + a/k) - (ln - psi)(k + a) + (ln - psi)(k)
  const double dD = log1p(a / k) - log_minus_digamma(k + a) + log_minus_digamma(k);
  c.k_m = 2.0 * k / g.m;
  c.k_s = -2.0 * k / g.s;
  c.t_m = th / g.m - th * dD * c.k_m;
  c.t_s = -th * dD * c.k_s;
  return c;
}

// Modified Gaussian: density r, the Gaussian factor phi(y) = N(y; 0, sg^2)
// (y = x - mu_g) and dr/d(mu_g, sg, tau).  Above y = sg^2/tau the erfc
// factor is at least 1 and the exponential decays; below it the two are
// combined as exp(-y^2 / 2 sg^2) erfcx(.) so that neither over- nor underflows.
__device__ inline double emg_r(const GenCell &g, double x, double &phi, double &rm, double &rsg, double &rt) {
  const double y = x - g.a, sg = g.b, t = g.c;
  const double z = y / sg, ik = sg / t;  // 1/K with K = tau / sg
  const double w = (ik - z) / kSqrt2;
  const double e2 = exp(-0.5 * z * z);
  const double r = w >= 0.0 ? e2 * erfcx(w) / (2.0 * t) : exp(fma(0.5 * ik, ik, -z * ik)) * erfc(w) / (2.0 * t);
  phi = e2 * kInvSqrt2Pi / sg;
  rm = (r - phi) / t;
  rsg = sg / (t * t) * (r - phi) - y / (sg * t) * phi;
  rt = r * (-1.0 / t + y / (t * t) - sg * sg / (t * t * t)) + sg * sg / (t * t * t) * phi;
  return r;
}

// ln r(x) of a cell (support search); -inf outside the density's support.
__device__ inline double gen_lnr(int fam, double p, const GenCell &g, double x) {
  switch (fam) {
    case kGammaPE:
    case kGenGammaPE: {
      if (!(x > 0.0)) return -INFINITY;
      const double pp = fam == kGammaPE ? 1.0 : p;
      const double u = gen_u(pp, x, g.b);
      return log(pp * g.a / x) + ln_pois(g.a, u, g.d);
    }
    case kSPoisPE: {
      if (x < 0.0) return -INFINITY;
      if (x == 0.0) return -g.b - log(g.a);
      const double t = x / g.a;
      return ln_pois(t, g.b, stirling_rem(t)) - log(g.a);
    }
    case kEmgPE: {  // the two forms of emg_r, in logarithms (no under- or overflow)
      const double z = (x - g.a) / g.b, ik = g.b / g.c, w = (ik - z) / kSqrt2;
      if (w >= 0.0) return -0.5 * z * z + log(erfcx(w)) - log(2.0 * g.c);
      return fma(0.5 * ik, ik, -z * ik) + log(erfc(w)) - log(2.0 * g.c);
    }
    default: {
      const double z = (x - g.m) / g.s;
      return -0.5 * z * z - log(g.s) - kHalfLn2Pi;
    }
  }
}

// Density r(x) and (if deriv) dr/dm, dr/ds.
__device__ inline double gen_density(int fam, double p, const GenCell &g, const GenChain &ch, double x, bool deriv,
                                double &dm, double &ds) {
  dm = ds = 0.0;
  switch (fam) {
    case kGammaPE:
    case kGenGammaPE: {
      if (!(x > 0.0)) return 0.0;
      const double pp = fam == kGammaPE ? 1.0 : p, k = g.a, th = g.b;
      const double u = gen_u(pp, x, g.b);
      const double r = pp * k * exp(ln_pois(k, u, g.d)) / x;
      if (deriv) {
        const double lk = -log(k / u) + log_minus_digamma(k);  // d ln r / dk = ln u - psi(k)
        const double lt = pp * (u - k) / th;                    // d ln r / dth
        dm = r * (lk * ch.k_m + lt * ch.t_m);
        ds = r * (lk * ch.k_s + lt * ch.t_s);
      }
      return r;
    }
    case kSPoisPE: {
      if (x < 0.0) return 0.0;
      const double gg = g.a, lam = g.b;
      double r, lg, ll;
      if (x == 0.0) {
        r = exp(-lam) / gg;
        lg = -1.0 / gg;
        ll = -1.0;
      } else {
        const double t = x / gg;
        r = exp(ln_pois(t, lam, stirling_rem(t))) / gg;
        // ln lambda - psi(t + 1) = -ln(t/lambda) - 1/t + (ln t - psi(t))
        const double lpsi = -log(t / lam) - 1.0 / t + log_minus_digamma(t);
        lg = -1.0 / gg - t / gg * lpsi;
        ll = t / lam - 1.0;
      }
      if (deriv) {
        dm = r * (lg * (-gg / g.m) + ll * (2.0 * lam / g.m));
        ds = r * (lg * (2.0 * gg / g.s) + ll * (-2.0 * lam / g.s));
      }
      return r;
    }
    case kEmgPE: {
      double phi, rm, rsg, rt;
      const double r = emg_r(g, x, phi, rm, rsg, rt);
      if (deriv) {
        const double f = g.c / g.s, cf = g.b / g.s;
        dm = rm;
        ds = -f * rm + cf * rsg + f * rt;
      }
      return r;
    }
    default: {
      const double z = (x - g.m) / g.s;
      const double r = exp(-0.5 * z * z) * kInvSqrt2Pi / g.s;
      if (deriv) {
        dm = r * z / g.s;
        ds = r * (z * z - 1.0) / g.s;
      }
      return r;
    }
  }
}

// Distribution function at x: F, Fc = 1 - F (each without cancellation) and
// (if deriv) dF/dm, dF/ds.  Not for the scaled Poisson.
__device__ inline void gen_cdf(int fam, double p, const GenCell &g, const GenChain &ch, double x, bool deriv, double &F,
                          double &Fc, double &dm, double &ds) {
  dm = ds = 0.0;
  switch (fam) {
    case kGammaPE:
    case kGenGammaPE: {
      if (!(x > 0.0)) {
        F = 0.0;
        Fc = 1.0;
        return;
      }
      const double pp = fam == kGammaPE ? 1.0 : p, k = g.a, th = g.b;
      const double u = gen_u(pp, x, g.b);
      const Igam I = igam(k, u, g.d, deriv);
      F = I.P;
      Fc = I.Q;
      if (deriv) {
        const double Ft = -pp * k * exp(ln_pois(k, u, g.d)) / th;  // dP(k, u)/dth
        dm = I.dP * ch.k_m + Ft * ch.t_m;
        ds = I.dP * ch.k_s + Ft * ch.t_s;
      }
      return;
    }
    case kEmgPE: {
      double phi, rm, rsg, rt;
      const double r = emg_r(g, x, phi, rm, rsg, rt), y = x - g.a, sg = g.b, t = g.c;
      F = 0.5 * erfc(-y / (kSqrt2 * sg)) - t * r;
      Fc = 0.5 * erfc(y / (kSqrt2 * sg)) + t * r;
      if (deriv) {
        const double f = t / g.s, cf = sg / g.s;
        const double Fm = -r, Fsg = -y / sg * phi - t * rsg, Ft = -r - t * rt;
        dm = Fm;
        ds = -f * Fm + cf * Fsg + f * Ft;
      }
      return;
    }
    default: {
      const double z = (x - g.m) / g.s;
      F = 0.5 * erfc(-z / kSqrt2);
      Fc = 0.5 * erfc(z / kSqrt2);
      if (deriv) {
        const double r = exp(-0.5 * z * z) * kInvSqrt2Pi / g.s;
        dm = -r;
        ds = -z * r;
      }
      return;
    }
  }
}

// One edge of an exact bin: the distribution function there.
struct Edge {
  double F, Fc, dm, ds;
};

__device__ inline Edge gen_edge(int fam, double p, const GenCell &g, const GenChain &ch, double x, bool deriv) {
  Edge e;
  gen_cdf(fam, p, g, ch, x, deriv, e.F, e.Fc, e.dm, e.ds);
  return e;
}

// Exact bin content from its two edges: on the lower tail's distribution
// function while the bin lies below the median, on the upper tail's above.
__device__ inline double edge_content(const Edge &lo, const Edge &hi, double &dm, double &ds) {
  dm = hi.dm - lo.dm;
  ds = hi.ds - lo.ds;
  return hi.F < 0.5 ? hi.F - lo.F : lo.Fc - hi.Fc;
}

// Support of a cell: the reco bins [lo, hi) on which ln r reaches
// ln r(m) + cut somewhere.  Every family here is unimodal with its mode at or
// below the mean, so above the mean's bin ln r falls with x and below it
// "ln r(edge) >= target" holds from some edge on: two binary searches over the
// bin edges (about 2 log2(n_reco) density evaluations).  Bin j is kept when
// its lower edge (above the mean) or its upper edge (below it) reaches the
// target, i.e. exactly when it meets the x range where ln r >= target.
__device__ inline int2 gen_support(int fam, double p, const GenCell &g, const double *edges, int n_reco, double cut) {
  const double target = gen_lnr(fam, p, g, g.m) + cut;
  // jm: the bin holding the mean (clamped to the binning)
  int a = 0, b = n_reco;
  while (a < b) {
    const int c = (a + b) >> 1;
    if (edges[c + 1] > g.m) b = c; else a = c + 1;
  }
  const int jm = min(a, n_reco - 1);
  // hi: the first edge above the mean's bin whose density is below the target (n_reco if none)
  a = jm + 1;
  b = n_reco;
  while (a < b) {
    const int c = (a + b) >> 1;
    if (gen_lnr(fam, p, g, edges[c]) < target) b = c; else a = c + 1;
  }
  const int hi = a;
  // lo: one past the last edge at or below the mean's bin whose density is below the target
  a = 0;
  b = jm + 1;
  while (a < b) {
    const int c = (a + b) >> 1;
    if (gen_lnr(fam, p, g, edges[c]) >= target) b = c; else a = c + 1;
  }
  const int lo = max(a - 1, 0);
  return make_int2(lo, max(hi, lo));
}

}  // namespace gs
