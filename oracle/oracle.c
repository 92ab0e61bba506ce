/* oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * The plain CPU definition of what the GPU library computes: the binned
 * multi-observable Poisson negative log-likelihood of GooStats
 * (arXiv:1812.05686), its gradient, and a BFGS fit driver.  Everything is
 * plain nested loops in the order the definitions are written, in long
 * double where the gamma-family exponent cancels.  Only tests, the smoke
 * check and the CPU-baseline leg of the benchmark use it; it shares no
 * code, header or table with the GPU library.
 *
 * Readings of points the paper leaves open (each is listed in the design doc):
 *  R1  -ln L = sum (mu - n ln mu) + 1/2 sum ((p - c)/sigma)^2 (Eq.4 with the
 *      sign fixed, ln n! dropped, and the factor 1/2 so that a change of 0.5
 *      in -ln L is one standard deviation).
 *  R2  n = 0 contributes mu (0 ln 0 = 0); mu < 0, or mu = 0 with n > 0, is a
 *      domain error: -ln L = +inf and status DOMAIN.  Every mu > 0 gives the
 *      finite Eq.4 term, however small mu is.  Where n > 0 and the FP64 seed
 *      1 - n/mu of the gradient overflows (n/mu above DBL_MAX, decided in FP64
 *      from the bin's FP64 mu) the gradient has no FP64 value: status
 *      GRAD_RANGE, gradient NaN, -ln L still finite.
 *  R3  reco bin content = bin width x response at the bin midpoint (the
 *      response evaluated on the visible x true energy mesh, section 2.5).
 *  R4  true spectra are histograms on a uniform cell-centred grid with rows
 *      summing to 1; a rate is the expected count at unit exposure.
 *  R5  a monoenergetic (AnaPeak, section 4.3) species is a delta at exactly
 *      its line energy.
 *  R6  exposure multiplies all rates of a dataset (section 4.1 input list).
 *  R7  quenching: Birks' law integrated with dE/dx = A/sqrt(E):
 *      Q = 1 - 2/y + 2 ln(1+y)/y^2, y = sqrt(E)/(kB A); light m = LY Q E.
 *  R8  response shapes (section 2.3 names the families without formulas):
 *      Gaussian N(x; m, s^2), or the gamma density with the same mean and
 *      variance (generalized gamma with unit power).
 *  R9  resolution: s^2 = a^2 + b E (energy family), s^2 = a^2 + b m + c^2 m^2
 *      (photoelectron families).
 *  R12 secondary observable (section 2.4): per-species two-Gaussian mixture at
 *      the bin midpoint, renormalised over the bins, with nuisances
 *      (mean shift delta, width scale kappa, logit shift eta of weight 1).
 *  R17 multivariate slice likelihood (section 2.4, cost model Eq.3): the energy
 *      histogram's Poisson likelihood plus, per energy slice, the likelihood of
 *      the slice's secondary-observable histogram given its total (multinomial:
 *      n_i. ln mu_i. - sum_k n_ik ln mu_ik), so that the energy information is
 *      not counted twice; with one slice per energy bin it equals the joint 2-D
 *      likelihood.
 *  R18 exact bin contents (section 2.5 evaluates the response on the mesh; a
 *      model may ask for the bin integral instead of the midpoint rule): the
 *      difference of the distribution function at the bin edges (erfc for the
 *      Gaussian families, the regularised incomplete gamma for the gamma
 *      families, a closed form for the modified Gaussian); none for the
 *      scaled Poisson, whose continued density has no closed-form integral.
 *  R19 generalized gamma (section 2.3 cites it without a formula): Stacy's
 *      three-parameter form with the power p fixed per model, shape
 *      k = m^2/(p^2 s^2) and the scale that makes the mean m.
 *  R20 scaled Poisson (cited without a formula): x/g ~ Poisson(lambda) with
 *      g = s^2/m, lambda = m^2/s^2, continued to real x >= 0 through the Gamma
 *      function and not renormalised.
 *  R21 modified Gaussian (cited without a formula): the exponentially
 *      modified Gaussian with tail fraction f = tau/s fixed per model, mean m
 *      and variance s^2.
 */
#include "oracle.h"

#include <math.h>
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>

typedef long double ld;
static const ld PI_L = 3.141592653589793238462643383279502884L;

static int n_resp(int fam) { return fam == ORC_TEMPLATE ? 0 : fam == ORC_GAUSS_E ? 2 : 5; }

int32_t orc_num_params(const orc_model *M) {
  return M->n_species + n_resp(M->family) + (M->n_psd > 0 ? 3 : 0);
}

/* ---------------------------------------------------------------- R7 ---- */
/* Q(E) = (1/E) int_0^E dE' / (1 + kB A / sqrt(E')).  With u = sqrt(E')/(kB A)
 * this is (2/y^2) int_0^y u^2/(1+u) du = 1 - 2/y + 2 ln(1+y)/y^2.  For tiny y
 * the power series 2 sum_n (-1)^(n+1) y^n/(n+2) avoids the cancellation. */
static ld quench_l(ld E, ld kB, ld A, ld *dQ_dkB) {
  if (!(E > 0)) {
    if (dQ_dkB) *dQ_dkB = 0;
    return 0;
  }
  ld y = sqrtl(E) / (kB * A);
  ld Q, dQdy;
  if (y < 1e-3L) {
    ld yn = 1;
    Q = 0;
    dQdy = 0;
    for (int n = 1; n <= 12; n++) {
      ld sgn = (n & 1) ? 1 : -1;
      dQdy += sgn * 2.0L * n * yn / (n + 2);
      yn *= y;
      Q += sgn * 2.0L * yn / (n + 2);
    }
  } else {
    ld L = log1pl(y);
    Q = 1 - 2 / y + 2 * L / (y * y);
    dQdy = 2 / (y * y) - 4 * L / (y * y * y) + 2 / (y * y * (1 + y));
  }
  if (dQ_dkB) *dQ_dkB = dQdy * (-y / kB); /* dy/dkB = -y/kB */
  return Q;
}

double orc_quench(double e, double kB, double A) { return (double)quench_l(e, kB, A, NULL); }
double orc_dquench_dkB(double e, double kB, double A) {
  ld d;
  quench_l(e, kB, A, &d);
  return (double)d;
}

/* Digamma: recurrence psi(x) = psi(x+1) - 1/x up to x >= 10 (Abramowitz &
 * Stegun 6.3.5), then the asymptotic series A&S 6.3.18 through x^-14. */
static ld digamma_l(ld x) {
  ld r = 0;
  while (x < 10) {
    r -= 1 / x;
    x += 1;
  }
  ld f = 1 / (x * x);
  ld tail = f * (1.0L / 12 - f * (1.0L / 120 - f * (1.0L / 252 - f * (1.0L / 240 - f * (1.0L / 132 - f * (691.0L / 32760 - f / 12))))));
  return r + logl(x) - 0.5L / x - tail;
}
double orc_digamma(double x) { return (double)digamma_l(x); }

/* ------------------------------------------------------- R7, R9 moments -- */
typedef struct {
  ld m, s;
  ld dm[5], ds[5]; /* derivatives w.r.t. the response parameters */
} mom_t;

/* Mean m and width s of the response to a deposit of true energy E, with
 * their derivatives (section 4.3: light yield, non-linearity and resolution
 * are fit parameters).  Returns 0 when the parameters give no valid response. */
static int moments_l(int fam, const double *resp, double A, ld E, mom_t *o) {
  memset(o, 0, sizeof *o);
  if (fam == ORC_GAUSS_E) {
    ld a = resp[0], b = resp[1];
    ld s2 = a * a + b * E;
    if (!(s2 > 0) || !isfinite((double)s2)) return 0;
    o->m = E;
    o->s = sqrtl(s2);
    o->ds[0] = a / o->s;
    o->ds[1] = E / (2 * o->s);
    return 1;
  }
  ld LY = resp[0], kB = resp[1], a = resp[2], b = resp[3], c = resp[4];
  if (!(kB > 0)) return 0;
  ld dQ;
  ld Q = quench_l(E, kB, A, &dQ);
  ld m = LY * Q * E;
  ld s2 = a * a + b * m + c * c * m * m;
  if (!(s2 > 0) || !isfinite((double)s2)) return 0;
  if ((fam == ORC_GAMMA_PE || fam == ORC_GENGAMMA_PE || fam == ORC_SPOIS_PE) && !(m > 0)) return 0;
  ld s = sqrtl(s2);
  o->m = m;
  o->s = s;
  o->dm[0] = Q * E;
  o->dm[1] = LY * E * dQ;
  ld dsdm = (b + 2 * c * c * m) / (2 * s);
  o->ds[0] = dsdm * o->dm[0];
  o->ds[1] = dsdm * o->dm[1];
  o->ds[2] = a / s;
  o->ds[3] = m / (2 * s);
  o->ds[4] = c * m * m / s;
  return 1;
}

int32_t orc_moments(int32_t family, const double *resp, double A, double E, double *m, double *s) {
  mom_t o;
  int ok = moments_l(family, resp, A, E, &o);
  *m = (double)o.m;
  *s = (double)o.s;
  return ok;
}

/* ------------------------------------------------------------ R8 shapes -- */
/* Regularised incomplete gamma P(k, u) = int_0^u t^(k-1) e^-t dt / Gamma(k),
 * Q = 1 - P, and dP/dk (R18: the exact bin content of the gamma-type
 * families).  Below u = k + 1 the series
 *   P = e^-u u^k / Gamma(k+1) * sum_n prod_{i=1..n} u / (k + i)
 * whose k-derivative is taken term by term; above it Legendre's continued
 * fraction for Gamma(k, u) e^u u^-k, evaluated by the modified Lentz method
 * with the derivative of every convergent w.r.t. k carried along. */
static void igam_l(ld k, ld u, ld *P, ld *Q, ld *dP) {
  if (!(u > 0)) {
    *P = 0;
    *Q = 1;
    *dP = 0;
    return;
  }
  const ld lu = logl(u);
  if (u < k + 1) {
    ld c = 1, S = 1, H = 0, dS = 0;
    for (int n = 1; n < 100000; n++) {
      H += 1 / (k + n);
      c *= u / (k + n);
      S += c;
      dS -= c * H;
      if (c < 1e-21L * S && c * H <= 1e-21L * fabsl(dS)) break;
    }
    const ld pre = expl(k * lu - u - lgammal(k + 1));
    *P = pre * S;
    *Q = 1 - *P;
    *dP = pre * ((lu - digamma_l(k + 1)) * S + dS);
    return;
  }
  const ld tiny = 1e-4000L;
  ld b = u + 1 - k, db = -1;
  ld c = 1 / tiny, dc = 0;
  ld d = 1 / b, dd = 1 / (b * b);
  ld h = d, dh = dd;
  for (int i = 1; i < 100000; i++) {
    const ld an = -(ld)i * (i - k), dan = i;
    b += 2;
    ld den = an * d + b;
    const ld dden = dan * d + an * dd + db;
    if (fabsl(den) < tiny) den = tiny;
    const ld dn = 1 / den, ddn = -dden * dn * dn;
    ld cn = b + an / c;
    const ld dcn = db + dan / c - an * dc / (c * c);
    if (fabsl(cn) < tiny) cn = tiny;
    d = dn;
    dd = ddn;
    c = cn;
    dc = dcn;
    const ld del = d * c, ddel = dd * c + d * dc;
    dh = dh * del + h * ddel;
    h *= del;
    if (fabsl(del - 1) < 1e-21L && fabsl(ddel * h) <= 1e-21L * fabsl(dh)) break;
  }
  const ld pre = expl(k * lu - u - lgammal(k));
  *Q = pre * h;
  *P = 1 - *Q;
  *dP = -pre * ((lu - digamma_l(k)) * h + dh);
}

/* Per-cell constants of the response density, computed once per true cell.
 * Families (R8, R19-R21), all with mean m and standard deviation s:
 *  Gaussian        N(x; m, s^2)
 *  gamma           shape k = m^2/s^2, scale th = s^2/m
 *  gen. gamma      p x^(kp-1) exp(-(x/th)^p) / (Gamma(k) th^(kp)), power p
 *                  (the model's shape parameter), k = m^2/(p^2 s^2),
 *                  th = m Gamma(k) / Gamma(k + 1/p) (mean exactly m; the
 *                  variance is s^2 up to O(1/k); p = 1 is the gamma family)
 *  scaled Poisson  Poisson(x/g; lambda) / g continued to real x >= 0 by the
 *                  Gamma function, g = s^2/m, lambda = m^2/s^2, not
 *                  renormalised (its integral falls short of 1 by
 *                  e^-lambda int_0^inf e^-lambda t / (t (pi^2 + ln^2 t)) dt)
 *  mod. Gaussian   exponentially modified Gaussian: N(mu_g, sg^2) convolved
 *                  with an exponential of mean tau, tau = f s,
 *                  sg = s sqrt(1 - f^2), mu_g = m - tau (f: the model's
 *                  shape parameter, 0 < f < 1). */
typedef struct {
  int fam;
  ld m, s;
  ld k, th, lgk, lth, psik; /* gamma, generalized gamma */
  ld p, dk_dm, dk_ds, dth_dm, dth_ds; /* generalized gamma */
  ld g, lam, llam;          /* scaled Poisson */
  ld mug, sg, tau, f;       /* modified Gaussian */
  ld norm;                  /* Gaussian: 1/(s sqrt(2 pi)) */
} dens_t;

static int pe_positive(int fam) {
  return fam == ORC_GAMMA_PE || fam == ORC_GENGAMMA_PE || fam == ORC_SPOIS_PE;
}

static int dens_prep(int fam, ld shape, ld m, ld s, dens_t *d) {
  memset(d, 0, sizeof *d);
  d->fam = fam;
  d->m = m;
  d->s = s;
  if (!(s > 0) || !isfinite((double)m) || !isfinite((double)s)) return 0;
  if (pe_positive(fam) && !(m > 0)) return 0;
  ld s2 = s * s;
  switch (fam) {
    case ORC_GAMMA_PE:
      d->k = m * m / s2;
      d->th = s2 / m;
      d->lgk = lgammal(d->k);
      d->lth = logl(d->th);
      d->psik = digamma_l(d->k);
      d->dk_dm = 2 * m / s2;
      d->dk_ds = -2 * m * m / (s2 * s);
      d->dth_dm = -s2 / (m * m);
      d->dth_ds = 2 * s / m;
      return 1;
    case ORC_GENGAMMA_PE: {
      if (!(shape > 0) || !isfinite((double)shape)) return 0;
      ld p = shape, k = m * m / (p * p * s2);
      /* ln Gamma(k + 1/p) - ln Gamma(k) in quadruple precision: the two terms
       * reach ~k ln k and cancel to ~ln(k)/p */
      ld D = (ld)(lgammaq((__float128)k + (__float128)(1 / p)) - lgammaq((__float128)k));
      ld dD = digamma_l(k + 1 / p) - digamma_l(k);
      d->p = p;
      d->k = k;
      d->th = m * expl(-D);
      d->lgk = lgammal(k);
      d->lth = logl(d->th);
      d->psik = digamma_l(k);
      d->dk_dm = 2 * k / m;
      d->dk_ds = -2 * k / s;
      d->dth_dm = d->th / m - d->th * dD * d->dk_dm;
      d->dth_ds = -d->th * dD * d->dk_ds;
      return 1;
    }
    case ORC_SPOIS_PE:
      d->g = s2 / m;
      d->lam = m * m / s2;
      d->llam = logl(d->lam);
      return 1;
    case ORC_EMG_PE:
      if (!(shape > 0 && shape < 1)) return 0;
      d->f = shape;
      d->tau = shape * s;
      d->sg = s * sqrtl(1 - shape * shape);
      d->mug = m - d->tau;
      return 1;
    default:
      d->norm = 1 / (s * sqrtl(2 * PI_L));
      return 1;
  }
}

/* Modified Gaussian: density r, the Gaussian factor phi = N(x; mu_g, sg^2)
 * and dr / d(mu_g, sg, tau). */
static ld emg_r(const dens_t *d, ld x, ld *phi, ld *rm, ld *rsg, ld *rt) {
  const ld y = x - d->mug, sg = d->sg, t = d->tau;
  const ld r = expl(-y / t + sg * sg / (2 * t * t)) * erfcl((sg * sg / t - y) / (sqrtl(2) * sg)) / (2 * t);
  const ld ph = expl(-y * y / (2 * sg * sg)) / (sg * sqrtl(2 * PI_L));
  *phi = ph;
  *rm = (r - ph) / t;
  *rsg = sg / (t * t) * (r - ph) - y / (sg * t) * ph;
  *rt = r * (-1 / t + y / (t * t) - sg * sg / (t * t * t)) + sg * sg / (t * t * t) * ph;
  return r;
}

/* r(x | m, s) and dr/dm, dr/ds. */
static ld dens_eval(const dens_t *d, ld x, ld *dm, ld *ds) {
  ld r, a, b;
  switch (d->fam) {
    case ORC_GAMMA_PE:
    case ORC_GENGAMMA_PE: {
      if (!(x > 0)) {
        *dm = *ds = 0;
        return 0;
      }
      const ld p = d->fam == ORC_GAMMA_PE ? 1 : d->p;
      const ld y = logl(x) - d->lth, xp = expl(p * y); /* (x/th)^p */
      r = p * expl((d->k * p - 1) * y - xp - d->lgk - d->lth);
      a = p * y - d->psik;                   /* d ln r / dk     */
      b = (p * xp - d->k * p) / d->th;       /* d ln r / dtheta */
      *dm = r * (a * d->dk_dm + b * d->dth_dm);
      *ds = r * (a * d->dk_ds + b * d->dth_ds);
      return r;
    }
    case ORC_SPOIS_PE: {
      if (x < 0) {
        *dm = *ds = 0;
        return 0;
      }
      const ld t = x / d->g, g = d->g, lam = d->lam;
      r = expl(t * d->llam - lam - lgammal(t + 1)) / g;
      a = -1 / g - t / g * (d->llam - digamma_l(t + 1)); /* d ln r / dg      */
      b = t / lam - 1;                                  /* d ln r / dlambda */
      *dm = r * (a * (-g / d->m) + b * (2 * lam / d->m));
      *ds = r * (a * (2 * g / d->s) + b * (-2 * lam / d->s));
      return r;
    }
    case ORC_EMG_PE: {
      ld ph, rm, rsg, rt;
      r = emg_r(d, x, &ph, &rm, &rsg, &rt);
      *dm = rm;
      *ds = -d->f * rm + sqrtl(1 - d->f * d->f) * rsg + d->f * rt;
      return r;
    }
    default: {
      const ld z = (x - d->m) / d->s;
      r = d->norm * expl(-0.5L * z * z);
      *dm = r * z / d->s;
      *ds = r * (z * z - 1) / d->s;
      return r;
    }
  }
}

/* Distribution function at x: F, Fc = 1 - F (each formed without
 * cancellation), and dF/dm, dF/ds.  Returns 0 for the scaled Poisson, whose
 * continued density has no closed-form integral (R18 offers it no exact bin
 * content). */
static int cdf_eval(const dens_t *d, ld x, ld *F, ld *Fc, ld *dm, ld *ds) {
  switch (d->fam) {
    case ORC_GAMMA_PE:
    case ORC_GENGAMMA_PE: {
      if (!(x > 0)) {
        *F = 0;
        *Fc = 1;
        *dm = *ds = 0;
        return 1;
      }
      const ld p = d->fam == ORC_GAMMA_PE ? 1 : d->p;
      const ld u = expl(p * (logl(x) - d->lth));
      ld dPk;
      igam_l(d->k, u, F, Fc, &dPk);
      const ld dPth = -p * expl(d->k * logl(u) - u - d->lgk) / d->th;
      *dm = dPk * d->dk_dm + dPth * d->dth_dm;
      *ds = dPk * d->dk_ds + dPth * d->dth_ds;
      return 1;
    }
    case ORC_EMG_PE: {
      ld ph, rm, rsg, rt;
      const ld r = emg_r(d, x, &ph, &rm, &rsg, &rt), y = x - d->mug, sg = d->sg, t = d->tau;
      *F = 0.5L * erfcl(-y / (sqrtl(2) * sg)) - t * r;
      *Fc = 0.5L * erfcl(y / (sqrtl(2) * sg)) + t * r;
      const ld Fm = -r, Fsg = -y / sg * ph - t * rsg, Ft = -r - t * rt;
      *dm = Fm;
      *ds = -d->f * Fm + sqrtl(1 - d->f * d->f) * Fsg + d->f * Ft;
      return 1;
    }
    case ORC_SPOIS_PE:
      return 0;
    default: {
      const ld z = (x - d->m) / d->s, r = d->norm * expl(-0.5L * z * z);
      *F = 0.5L * erfcl(-z / sqrtl(2));
      *Fc = 0.5L * erfcl(z / sqrtl(2));
      *dm = -r;
      *ds = -z * r;
      return 1;
    }
  }
}

/* Content of reco bin [xlo, xhi) (midpoint xm, width dx) of a unit deposit,
 * K = dx r(xm) (R3), or with exact bins (R18) the integral of r over the bin
 * as a difference of distribution functions (taken on the lower or upper
 * tail, whichever is the smaller); dK/dm, dK/ds.  Returns 0 if the family has
 * no exact bin content. */
static int bin_content(const dens_t *d, int exact, ld xlo, ld xhi, ld xm, ld dx, ld *K, ld *dm, ld *ds) {
  if (!exact) {
    ld a, b;
    *K = dx * dens_eval(d, xm, &a, &b);
    *dm = dx * a;
    *ds = dx * b;
    return 1;
  }
  ld Fl, Fcl, ml, sl, Fh, Fch, mh, sh;
  if (!cdf_eval(d, xlo, &Fl, &Fcl, &ml, &sl) || !cdf_eval(d, xhi, &Fh, &Fch, &mh, &sh)) return 0;
  *K = Fh < 0.5L ? Fh - Fl : Fcl - Fch;
  *dm = mh - ml;
  *ds = sh - sl;
  return 1;
}

double orc_density(int32_t family, double x, double m, double s) { return orc_density3(family, 0.0, x, m, s); }

double orc_density3(int32_t family, double shape, double x, double m, double s) {
  dens_t d;
  ld a, b;
  if (!dens_prep(family, shape, m, s, &d)) return NAN;
  return (double)dens_eval(&d, x, &a, &b);
}

void orc_density_dms(int32_t family, double x, double m, double s, double *dm, double *ds) {
  orc_density_dms3(family, 0.0, x, m, s, dm, ds);
}

void orc_density_dms3(int32_t family, double shape, double x, double m, double s, double *dm, double *ds) {
  dens_t d;
  ld a = NAN, b = NAN;
  ld r = dens_prep(family, shape, m, s, &d) ? dens_eval(&d, x, &a, &b) : NAN;
  *dm = r != 0 ? (double)(a / r) : 0.0;
  *ds = r != 0 ? (double)(b / r) : 0.0;
}

int32_t orc_bin_content(int32_t family, double shape, int32_t exact, double xlo, double xhi, double m, double s,
                        double *K, double *dKdm, double *dKds) {
  dens_t d;
  ld k, a, b;
  if (!dens_prep(family, shape, m, s, &d)) return 0;
  if (!bin_content(&d, exact, xlo, xhi, ((ld)xlo + xhi) / 2, (ld)xhi - xlo, &k, &a, &b)) return 0;
  *K = (double)k;
  *dKdm = (double)a;
  *dKds = (double)b;
  return 1;
}

int32_t orc_igam(double k, double u, double *P, double *Q, double *dPdk) {
  ld p, q, d;
  igam_l(k, u, &p, &q, &d);
  *P = (double)p;
  *Q = (double)q;
  *dPdk = (double)d;
  return 1;
}

/* ---------------------------------------------------------- fold (Eq.2) -- */
/* K_ji = dx_j * r(xbar_j | m_i, s_i) on the visible x true mesh (section 2.5),
 * then F[j][s] = sum_i w_si K_ji over the grid cells of species s; a line
 * species is a single cell at its energy with weight 1 (R5).  If dF is given
 * it receives d F[j][s] / d resp_p as dF[(j*S + s)*nr + p].  Returns 0 if the
 * response is invalid somewhere on the grid. */
static int fold_l(const orc_model *M, const double *theta, ld *F, ld *dF) {
  const int S = M->n_species, J = M->n_reco, fam = M->family, nr = n_resp(fam);
  const double *resp = theta + S;
  memset(F, 0, sizeof(ld) * (size_t)J * S);
  if (dF && nr > 0) memset(dF, 0, sizeof(ld) * (size_t)J * S * nr);
  if (fam == ORC_TEMPLATE) {
    /* Monte Carlo fit (section 3.2): the template is the species' reco spectrum */
    for (int j = 0; j < J; j++)
      for (int s = 0; s < S; s++) F[(size_t)j * S + s] = M->spectra[(size_t)s * M->n_true + j];
    return 1;
  }
  ld *xb = malloc(sizeof(ld) * J), *dx = malloc(sizeof(ld) * J);
  ld *w = malloc(sizeof(ld) * S);
  for (int j = 0; j < J; j++) {
    xb[j] = (M->reco_edges[j] + M->reco_edges[j + 1]) * 0.5;
    dx[j] = (ld)M->reco_edges[j + 1] - (ld)M->reco_edges[j];
  }
  int n_grid = 0;
  for (int s = 0; s < S; s++) n_grid += isnan(M->line_energy[s]) ? 1 : 0;
  int ok = 1;
  /* cells 0..n_true-1 are the grid; then one cell per line species */
  for (int i = 0; i < M->n_true + S && ok; i++) {
    int line_s = -1;
    ld E;
    if (i < M->n_true) {
      if (n_grid == 0) continue;
      int any = 0;
      for (int s = 0; s < S; s++) {
        w[s] = isnan(M->line_energy[s]) ? (ld)M->spectra[(size_t)s * M->n_true + i] : 0;
        any |= w[s] != 0;
      }
      if (!any) continue;
      E = (ld)(M->e_lo + (i + 0.5) * M->e_step);
    } else {
      line_s = i - M->n_true;
      if (isnan(M->line_energy[line_s])) continue;
      for (int s = 0; s < S; s++) w[s] = s == line_s;
      E = (ld)M->line_energy[line_s];
    }
    mom_t mo;
    if (!moments_l(fam, resp, M->birks_A, E, &mo)) {
      ok = 0;
      break;
    }
    dens_t d;
    if (!dens_prep(fam, M->shape, mo.m, mo.s, &d)) {
      ok = 0;
      break;
    }
    for (int j = 0; j < J && ok; j++) {
      ld K, dKm, dKs;
      ok = bin_content(&d, M->exact_bins, M->reco_edges[j], M->reco_edges[j + 1], xb[j], dx[j], &K, &dKm, &dKs);
      for (int s = 0; s < S && ok; s++) {
        if (w[s] == 0) continue;
        F[(size_t)j * S + s] += w[s] * K;
        if (dF)
          for (int p = 0; p < nr; p++)
            dF[((size_t)j * S + s) * nr + p] += w[s] * (dKm * mo.dm[p] + dKs * mo.ds[p]);
      }
    }
  }
  free(xb);
  free(dx);
  free(w);
  return ok;
}

int32_t orc_species_fold(const orc_model *M, const double *theta, double *F) {
  size_t n = (size_t)M->n_reco * M->n_species;
  ld *f = malloc(sizeof(ld) * n);
  int ok = fold_l(M, theta, f, NULL);
  for (size_t i = 0; i < n; i++) F[i] = (double)f[i];
  free(f);
  return ok;
}

/* ------------------------------------------------ secondary obs. (R12) -- */
/* P[s][k] = p_sk / sum_k' p_sk', p_sk = dy_k (w1' N(ybar_k; mu1+delta, (kappa s1)^2)
 * + (1-w1') N(ybar_k; mu2+delta, (kappa s2)^2)), w1' = sigmoid(logit(w1) + eta).
 * dP[(s*K + k)*3 + v] = d P_sk / d (delta, kappa, eta)_v. */
static int psd_l(const orc_model *M, const double *nu, ld *P, ld *dP) {
  const int S = M->n_species, K = M->n_psd;
  ld delta = nu[0], kappa = nu[1], eta = nu[2];
  if (!(kappa > 0)) return 0;
  ld *p = malloc(sizeof(ld) * K), *dp = malloc(sizeof(ld) * K * 3);
  int ok = 1;
  for (int s = 0; s < S; s++) {
    const double *mx = M->psd_mix + 5 * s;
    ld w1 = mx[0];
    if (!(w1 > 0 && w1 < 1)) {
      ok = 0;
      break;
    }
    ld wp = 1 / (1 + expl(-(logl(w1 / (1 - w1)) + eta)));
    ld Z = 0, dZ[3] = {0, 0, 0};
    for (int k = 0; k < K; k++) {
      ld y = (M->psd_edges[k] + M->psd_edges[k + 1]) * 0.5;
      ld dy = (ld)M->psd_edges[k + 1] - (ld)M->psd_edges[k];
      ld Nc[2], dd[2], dk[2];
      for (int c = 0; c < 2; c++) {
        ld mu = mx[1 + 2 * c] + delta, sg = mx[2 + 2 * c] * kappa;
        ld z = (y - mu) / sg;
        Nc[c] = expl(-0.5L * z * z) / (sg * sqrtl(2 * PI_L));
        dd[c] = Nc[c] * z / sg;
        dk[c] = Nc[c] * (z * z - 1) / kappa;
      }
      p[k] = dy * (wp * Nc[0] + (1 - wp) * Nc[1]);
      dp[3 * k + 0] = dy * (wp * dd[0] + (1 - wp) * dd[1]);
      dp[3 * k + 1] = dy * (wp * dk[0] + (1 - wp) * dk[1]);
      dp[3 * k + 2] = dy * wp * (1 - wp) * (Nc[0] - Nc[1]);
      Z += p[k];
      for (int v = 0; v < 3; v++) dZ[v] += dp[3 * k + v];
    }
    for (int k = 0; k < K; k++) {
      P[(size_t)s * K + k] = p[k] / Z;
      if (dP)
        for (int v = 0; v < 3; v++)
          dP[((size_t)s * K + k) * 3 + v] = (dp[3 * k + v] - p[k] / Z * dZ[v]) / Z;
    }
  }
  free(p);
  free(dp);
  return ok;
}

int32_t orc_psd_probs(const orc_model *M, const double *theta, double *P) {
  if (M->n_psd <= 0) return 0;
  size_t n = (size_t)M->n_species * M->n_psd;
  ld *q = malloc(sizeof(ld) * n);
  int ok = psd_l(M, theta + M->n_species + n_resp(M->family), q, NULL);
  for (size_t i = 0; i < n; i++) P[i] = (double)q[i];
  free(q);
  return ok;
}

/* ------------------------------------------------- expectation (Eq.2/3) -- */
/* mu[d][j][k] = eps_d sum_s R_s F_js P_sk  (P = 1 in one dimension). */
static void expected_l(const orc_model *M, const double *theta, const ld *F, const ld *P, ld *mu) {
  const int S = M->n_species, J = M->n_reco, K = M->n_psd > 0 ? M->n_psd : 1;
  for (int d = 0; d < M->n_datasets; d++)
    for (int j = 0; j < J; j++)
      for (int k = 0; k < K; k++) {
        ld acc = 0;
        for (int s = 0; s < S; s++)
          acc += (ld)theta[s] * F[(size_t)j * S + s] * (P ? P[(size_t)s * K + k] : 1);
        mu[((size_t)d * J + j) * K + k] = M->exposure[d] * acc;
      }
}

static int theta_finite(const orc_model *M, const double *theta) {
  int P = orc_num_params(M);
  for (int p = 0; p < P; p++)
    if (!isfinite(theta[p])) return 0;
  return 1;
}

int32_t orc_expected(const orc_model *M, const double *theta, double *mu) {
  const int S = M->n_species, J = M->n_reco, K = M->n_psd > 0 ? M->n_psd : 1;
  size_t nb = (size_t)M->n_datasets * J * K;
  ld *F = malloc(sizeof(ld) * (size_t)J * S), *P = NULL, *m = malloc(sizeof(ld) * nb);
  int ok = theta_finite(M, theta) && fold_l(M, theta, F, NULL);
  if (ok && M->n_psd > 0) {
    P = malloc(sizeof(ld) * (size_t)S * K);
    ok = psd_l(M, theta + S + n_resp(M->family), P, NULL);
  }
  if (ok) expected_l(M, theta, F, P, m);
  for (size_t i = 0; i < nb; i++) mu[i] = ok ? (double)m[i] : NAN;
  free(F);
  free(P);
  free(m);
  return ok;
}

/* ------------------------------------------------------ -ln L (Eq.4) ----- */
/* R1/R2 per-bin term.  Returns 0 on a domain error; *range is set when n > 0
 * and the FP64 value of n/mu (mu is the bin's FP64 expectation) overflows. */
static int poisson_term(ld mu, ld n, ld *term, ld *g, int *range) {
  if (mu > 0) {
    *term = n > 0 ? mu - n * logl(mu) : mu;
    *g = 1 - n / mu;
    if (n > 0 && !isfinite((double)n / (double)mu)) *range = 1;
    return 1;
  }
  if (mu == 0 && n == 0) {
    *term = 0;
    *g = 1;
    return 1;
  }
  return 0;
}

/* R17: the multivariate slice likelihood, added into *nll and (if gr) the
 * gradient.  Energy part: mu_dj = eps_d sum_s R_s F_js against n_dj = sum_k
 * n_djk; slice i: N_si = sum_{j in i} F_js, mu_dik = eps_d sum_s R_s N_si P_sk,
 * mu_di. = sum_k mu_dik, n_dik = sum_{j in i} n_djk, piece
 * n_di. ln mu_di. - sum_k n_dik ln mu_dik.  Returns 0 on a domain error. */
static int mv_terms(const orc_model *M, const double *theta, const ld *F, const ld *dF, const ld *P, const ld *dP,
                    ld *nll, ld *gr, int *range) {
  const int S = M->n_species, J = M->n_reco, K = M->n_psd, nr = n_resp(M->family);
  for (int d = 0; d < M->n_datasets; d++) {
    const ld eps = M->exposure[d];
    for (int j = M->win_lo; j < M->win_hi; j++) {
      ld mu = 0, n = 0;
      for (int s = 0; s < S; s++) mu += (ld)theta[s] * F[(size_t)j * S + s];
      mu = (double)(eps * mu);
      for (int k = 0; k < K; k++) n += M->counts[((size_t)d * J + j) * K + k];
      ld term, g;
      if (!poisson_term(mu, n, &term, &g, range)) return 0;
      *nll += term;
      if (!gr) continue;
      for (int s = 0; s < S; s++) {
        gr[s] += g * eps * F[(size_t)j * S + s];
        for (int p = 0; p < nr; p++) gr[S + p] += g * eps * theta[s] * dF[((size_t)j * S + s) * nr + p];
      }
    }
    for (int i = 0; i < M->n_slices; i++) {
      const int j0 = M->slice_edges[i], j1 = M->slice_edges[i + 1];
      for (int k0 = 0; k0 <= K; k0++) {
        /* k0 < K: the bin k0 of the slice's histogram (weight -n_ik); k0 = K: its
         * total (weight +n_i.) */
        ld mu = 0, n = 0;
        for (int s = 0; s < S; s++) {
          ld Ns = 0;
          for (int j = j0; j < j1; j++) Ns += F[(size_t)j * S + s];
          mu += (ld)theta[s] * Ns * (k0 < K ? P[(size_t)s * K + k0] : 1);
        }
        mu = (double)(eps * mu);
        for (int j = j0; j < j1; j++)
          for (int k = 0; k < K; k++)
            if (k0 == K || k == k0) n += M->counts[((size_t)d * J + j) * K + k];
        if (n == 0) continue;
        if (!(mu > 0)) return 0;
        if (!isfinite((double)n / (double)mu)) *range = 1;
        const ld sign = k0 < K ? -1 : 1;
        *nll += sign * n * logl(mu);
        if (!gr) continue;
        const ld g = sign * n / mu; /* d piece / d mu */
        for (int s = 0; s < S; s++) {
          const ld pk = k0 < K ? P[(size_t)s * K + k0] : 1;
          ld Ns = 0;
          for (int j = j0; j < j1; j++) Ns += F[(size_t)j * S + s];
          gr[s] += g * eps * Ns * pk;
          for (int p = 0; p < nr; p++) {
            ld dN = 0;
            for (int j = j0; j < j1; j++) dN += dF[((size_t)j * S + s) * nr + p];
            gr[S + p] += g * eps * theta[s] * dN * pk;
          }
          if (k0 < K)
            for (int v = 0; v < 3; v++) gr[S + nr + v] += g * eps * theta[s] * Ns * dP[((size_t)s * K + k0) * 3 + v];
        }
      }
    }
  }
  return 1;
}

double orc_nll_grad(const orc_model *M, const double *theta, double *grad, uint32_t *st) {
  const int S = M->n_species, J = M->n_reco, fam = M->family, nr = n_resp(fam);
  const int K = M->n_psd > 0 ? M->n_psd : 1, Pn = orc_num_params(M);
  *st = 0;
  if (!theta_finite(M, theta)) {
    *st = ORC_ST_NONFINITE;
    if (grad)
      for (int p = 0; p < Pn; p++) grad[p] = NAN;
    return NAN;
  }
  ld *F = malloc(sizeof(ld) * (size_t)J * S);
  ld *dF = grad ? malloc(sizeof(ld) * (size_t)J * S * nr) : NULL;
  ld *P = NULL, *dP = NULL;
  int ok = fold_l(M, theta, F, dF);
  if (ok && M->n_psd > 0) {
    P = malloc(sizeof(ld) * (size_t)S * K);
    dP = malloc(sizeof(ld) * (size_t)S * K * 3);
    ok = psd_l(M, theta + S + nr, P, dP);
  }
  ld nll = 0;
  int range = 0;
  ld *gr = calloc((size_t)Pn, sizeof(ld));
  if (ok && M->n_slices > 0) {
    ok = mv_terms(M, theta, F, dF, P, dP, &nll, grad ? gr : NULL, &range);
  } else
  for (int d = 0; d < M->n_datasets && ok; d++) {
    ld eps = M->exposure[d];
    for (int j = M->win_lo; j < M->win_hi && ok; j++)
      for (int k = 0; k < K; k++) {
        ld mu = 0;
        for (int s = 0; s < S; s++) mu += (ld)theta[s] * F[(size_t)j * S + s] * (P ? P[(size_t)s * K + k] : 1);
        /* mu is an FP64 quantity: round the long-double sum to double (so a tail
         * that underflows in FP64 is exactly 0 here too) */
        mu = (double)(eps * mu);
        ld n = M->counts[((size_t)d * J + j) * K + k];
        ld term, g;
        if (!poisson_term(mu, n, &term, &g, &range)) {
          ok = 0;
          break;
        }
        nll += term;
        if (!grad) continue;
        /* d mu / d theta, term by term */
        for (int s = 0; s < S; s++) {
          ld pk = P ? P[(size_t)s * K + k] : 1;
          gr[s] += g * eps * F[(size_t)j * S + s] * pk;
          for (int p = 0; p < nr; p++) gr[S + p] += g * eps * theta[s] * pk * dF[((size_t)j * S + s) * nr + p];
          if (P)
            for (int v = 0; v < 3; v++)
              gr[S + nr + v] += g * eps * theta[s] * F[(size_t)j * S + s] * dP[((size_t)s * K + k) * 3 + v];
        }
      }
  }
  if (ok)
    for (int p = 0; p < Pn; p++)
      if (M->pull_sigma && M->pull_sigma[p] > 0) {
        ld z = ((ld)theta[p] - M->pull_centre[p]) / M->pull_sigma[p];
        nll += 0.5L * z * z;
        gr[p] += z / M->pull_sigma[p];
      }
  if (!ok) *st = ORC_ST_DOMAIN;
  else if (range) *st = ORC_ST_GRAD_RANGE;
  if (grad)
    for (int p = 0; p < Pn; p++) grad[p] = ok && !range ? (double)gr[p] : NAN;
  free(gr);
  free(F);
  free(dF);
  free(P);
  free(dP);
  return ok ? (double)nll : INFINITY;
}

double orc_nll(const orc_model *M, const double *theta, uint32_t *st) {
  return orc_nll_grad(M, theta, NULL, st);
}

/* ------------------------------------------------------------- BFGS ------ */
/* The minimizer step (MINUIT's variable-metric role in section 3.2): BFGS on
 * the inverse Hessian with a backtracking Armijo line search.  Gradient is
 * either analytic or central finite differences with steps 1e-4 * scale. */
typedef struct {
  const orc_model *M;
  const orc_fit_opts *o;
  int P, nf;
  int *idx;      /* free parameter indices */
  double *full;  /* full parameter vector workspace */
  int n_eval;
} fitctx;

static double f_eval(fitctx *c, const double *x, double *g, uint32_t *st) {
  for (int q = 0; q < c->nf; q++) c->full[c->idx[q]] = x[q];
  c->n_eval++;
  if (!g) return orc_nll(c->M, c->full, st);
  if (!c->o->use_fd) {
    double *gf = malloc(sizeof(double) * c->P);
    double f = orc_nll_grad(c->M, c->full, gf, st);
    for (int q = 0; q < c->nf; q++) g[q] = gf[c->idx[q]];
    free(gf);
    return f;
  }
  double f = orc_nll(c->M, c->full, st);
  for (int q = 0; q < c->nf; q++) {
    int p = c->idx[q];
    double h = 1e-4 * c->o->scale[p], x0 = c->full[p];
    uint32_t s1, s2;
    c->full[p] = x0 + h;
    double fp = orc_nll(c->M, c->full, &s1);
    c->full[p] = x0 - h;
    double fm = orc_nll(c->M, c->full, &s2);
    c->full[p] = x0;
    c->n_eval += 2;
    g[q] = (fp - fm) / (2 * h);
    *st |= s1 | s2;
  }
  return f;
}

/* Gauss-Jordan inverse with partial pivoting of an n x n matrix. */
static int invert(int n, double *a, double *inv) {
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) inv[i * n + j] = i == j;
  for (int c = 0; c < n; c++) {
    int piv = c;
    for (int r = c + 1; r < n; r++)
      if (fabs(a[r * n + c]) > fabs(a[piv * n + c])) piv = r;
    if (a[piv * n + c] == 0) return 0;
    for (int j = 0; j < n; j++) {
      double t = a[c * n + j];
      a[c * n + j] = a[piv * n + j];
      a[piv * n + j] = t;
      t = inv[c * n + j];
      inv[c * n + j] = inv[piv * n + j];
      inv[piv * n + j] = t;
    }
    double d = a[c * n + c];
    for (int j = 0; j < n; j++) {
      a[c * n + j] /= d;
      inv[c * n + j] /= d;
    }
    for (int r = 0; r < n; r++)
      if (r != c && a[r * n + c] != 0) {
        double f = a[r * n + c];
        for (int j = 0; j < n; j++) {
          a[r * n + j] -= f * a[c * n + j];
          inv[r * n + j] -= f * inv[c * n + j];
        }
      }
  }
  return 1;
}

int32_t orc_fit(const orc_model *M, const double *theta0, const orc_fit_opts *o, double *theta_hat,
                double *sigma, orc_fit_result *res) {
  fitctx c = {M, o, orc_num_params(M), 0, NULL, NULL, 0};
  c.idx = malloc(sizeof(int) * c.P);
  c.full = malloc(sizeof(double) * c.P);
  memcpy(c.full, theta0, sizeof(double) * c.P);
  for (int p = 0; p < c.P; p++)
    if (!o->free_mask || o->free_mask[p]) c.idx[c.nf++] = p;
  const int n = c.nf;
  double *x = malloc(sizeof(double) * n), *g = malloc(sizeof(double) * n), *H = malloc(sizeof(double) * n * n);
  double *pd = malloc(sizeof(double) * n), *xn = malloc(sizeof(double) * n), *gn = malloc(sizeof(double) * n);
  double *sv = malloc(sizeof(double) * n), *yv = malloc(sizeof(double) * n), *Hy = malloc(sizeof(double) * n);
  for (int q = 0; q < n; q++) x[q] = theta0[c.idx[q]];
  uint32_t st = 0, est;
  double f = f_eval(&c, x, g, &est);
  st |= est & (ORC_ST_NONFINITE | ORC_ST_GRAD_RANGE);
  /* a start without an FP64 gradient (R2) cannot begin a quasi-Newton step */
  const int no_grad = (est & ORC_ST_GRAD_RANGE) != 0;
#define RESET_H()                                                            \
  for (int i = 0; i < n; i++)                                                \
    for (int j = 0; j < n; j++) H[i * n + j] = i == j ? o->scale[c.idx[i]] * o->scale[c.idx[i]] : 0;
  RESET_H();
  int it = 0;
  double edm = INFINITY;
  if (!isfinite(f)) st |= est;
  while (isfinite(f) && !no_grad) {
    edm = 0;
    for (int i = 0; i < n; i++)
      for (int j = 0; j < n; j++) edm += 0.5 * g[i] * H[i * n + j] * g[j];
    if (edm < o->edm_tol) break;
    if (it >= o->max_iter) {
      st |= ORC_ST_MAXITER;
      break;
    }
    double slope = 0;
    for (int i = 0; i < n; i++) {
      pd[i] = 0;
      for (int j = 0; j < n; j++) pd[i] -= H[i * n + j] * g[j];
      slope += g[i] * pd[i];
    }
    if (!(slope < 0)) {
      RESET_H();
      st |= ORC_ST_BFGS_RESET;
      slope = 0;
      for (int i = 0; i < n; i++) {
        pd[i] = -H[i * n + i] * g[i];
        slope += g[i] * pd[i];
      }
    }
    double alpha = 1, fn = INFINITY;
    int accepted = 0;
    for (int ls = 0; ls < 40; ls++) {
      for (int i = 0; i < n; i++) xn[i] = x[i] + alpha * pd[i];
      fn = f_eval(&c, xn, NULL, &est);
      /* a trial point whose gradient has no FP64 value (R2) is not taken */
      const int usable = isfinite(fn) && !(est & ORC_ST_GRAD_RANGE);
      if (usable && fn <= f + 1e-4 * alpha * slope + 1e-14 * fabs(f)) {
        accepted = 1;
        break;
      }
      if (usable) {
        double aq = -slope * alpha * alpha / (2 * (fn - f - slope * alpha));
        alpha = fmin(fmax(aq, 0.1 * alpha), 0.5 * alpha);
      } else {
        alpha *= 0.25;
      }
    }
    if (!accepted) {
      st |= ORC_ST_LS_FAIL;
      break;
    }
    fn = f_eval(&c, xn, gn, &est);
    double sy = 0, ss = 0, yy = 0;
    for (int i = 0; i < n; i++) {
      sv[i] = xn[i] - x[i];
      yv[i] = gn[i] - g[i];
      sy += sv[i] * yv[i];
      ss += sv[i] * sv[i];
      yy += yv[i] * yv[i];
    }
    if (sy > 1e-12 * sqrt(ss * yy)) {
      /* H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T */
      double rho = 1 / sy, yHy = 0;
      for (int i = 0; i < n; i++) {
        Hy[i] = 0;
        for (int j = 0; j < n; j++) Hy[i] += H[i * n + j] * yv[j];
        yHy += yv[i] * Hy[i];
      }
      for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
          H[i * n + j] += -rho * (sv[i] * Hy[j] + Hy[i] * sv[j]) + (rho * rho * yHy + rho) * sv[i] * sv[j];
    } else {
      RESET_H();
      st |= ORC_ST_BFGS_RESET;
    }
    memcpy(x, xn, sizeof(double) * n);
    memcpy(g, gn, sizeof(double) * n);
    f = fn;
    it++;
  }
#undef RESET_H
  for (int p = 0; p < c.P; p++) theta_hat[p] = theta0[p];
  for (int q = 0; q < n; q++) theta_hat[c.idx[q]] = x[q];
  if (sigma) {
    for (int p = 0; p < c.P; p++) sigma[p] = 0;
    if (o->hesse && isfinite(f)) {
      /* Hessian by central differences of the analytic gradient, then inverse */
      double *Hs = malloc(sizeof(double) * n * n), *Hi = malloc(sizeof(double) * n * n);
      double *full = malloc(sizeof(double) * c.P), *gp = malloc(sizeof(double) * c.P), *gm = malloc(sizeof(double) * c.P);
      memcpy(full, theta_hat, sizeof(double) * c.P);
      for (int q = 0; q < n; q++) {
        int p = c.idx[q];
        double h = 1e-4 * o->scale[p], x0 = full[p];
        uint32_t s1;
        full[p] = x0 + h;
        orc_nll_grad(M, full, gp, &s1);
        full[p] = x0 - h;
        orc_nll_grad(M, full, gm, &s1);
        full[p] = x0;
        for (int r = 0; r < n; r++) Hs[r * n + q] = (gp[c.idx[r]] - gm[c.idx[r]]) / (2 * h);
      }
      for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++) Hs[i * n + j] = Hs[j * n + i] = 0.5 * (Hs[i * n + j] + Hs[j * n + i]);
      if (invert(n, Hs, Hi))
        for (int q = 0; q < n; q++) sigma[c.idx[q]] = Hi[q * n + q] > 0 ? sqrt(Hi[q * n + q]) : NAN;
      free(Hs);
      free(Hi);
      free(full);
      free(gp);
      free(gm);
    } else {
      for (int q = 0; q < n; q++) sigma[c.idx[q]] = sqrt(fmax(H[q * n + q], 0));
    }
  }
  res->nll = f;
  res->edm = edm;
  res->iters = it;
  res->n_eval = c.n_eval;
  res->status = st;
  free(c.idx);
  free(c.full);
  free(x);
  free(g);
  free(H);
  free(pd);
  free(xn);
  free(gn);
  free(sv);
  free(yv);
  free(Hy);
  return isfinite(f) && !no_grad && !(st & (ORC_ST_LS_FAIL | ORC_ST_MAXITER));
}

/* ------------------------------------------------- discovery test (Eq.5) -- */
/* Eq.5 writes the profile likelihood ratio with the free fit in the numerator
 * and a minus sign in front, which would make t <= 0; read as the ratio of the
 * null fit's likelihood to the free fit's, t = -2 ln(L_null / L_free) =
 * 2 (NLL_null - NLL_free) >= 0, the form the paper's own recipe prints (the
 * difference of the two fits' likelihoods).  Two plain fits, one after the
 * other. */
int32_t orc_discovery(const orc_model *M, const double *theta0, const orc_fit_opts *o, int32_t signal,
                      double *t, double *theta_free, double *theta_null, orc_fit_result *res_free,
                      orc_fit_result *res_null) {
  const int P = orc_num_params(M);
  if (signal < 0 || signal >= P) return 0;
  int ok_free = orc_fit(M, theta0, o, theta_free, NULL, res_free);
  double *th0 = malloc(sizeof(double) * P);
  uint8_t *fm = malloc((size_t)P);
  memcpy(th0, theta0, sizeof(double) * P);
  th0[signal] = 0.0;
  for (int p = 0; p < P; p++) fm[p] = (uint8_t)((!o->free_mask || o->free_mask[p]) && p != signal);
  orc_fit_opts on = *o;
  on.free_mask = fm;
  int ok_null = orc_fit(M, th0, &on, theta_null, NULL, res_null);
  *t = 2.0 * (res_null->nll - res_free->nll);
  free(th0);
  free(fm);
  return ok_free && ok_null;
}

