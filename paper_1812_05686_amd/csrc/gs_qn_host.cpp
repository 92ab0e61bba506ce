// gs_qn_host.cpp -- host quasi-Newton driver over the device evaluations.
//
// BFGS on the inverse Hessian with a backtracking Armijo line search: the
// minimizer role that MINUIT's variable-metric method plays in the paper
// (sections 3.2 and 4.1).  Two gradient sources:
//   adjoint: gs_nll_grad at every trial point (the gradient of an accepted
//            trial is reused, so a step costs one evaluation when the full
//            step is accepted);
//   plain:   central differences of gs_nll, 2 calls per free parameter, where
//            rate-only perturbations hit the cached per-species fold.
#include <cmath>
#include <cstring>
#include <vector>

#include "gs.h"

namespace {

struct Ctx {
  gs_model *M;
  const gs_fit_opts *o;
  int P;
  std::vector<int> idx;
  std::vector<double> full;
  int n_eval = 0;
  gs_status err = GS_OK;
};

// f at free-parameter vector x; gradient into g (size n_free) when g != nullptr.
double evaluate(Ctx &c, const double *x, double *g, uint32_t &st) {
  const int n = (int)c.idx.size();
  for (int q = 0; q < n; q++) c.full[c.idx[q]] = x[q];
  double f = NAN;
  st = 0;
  if (!c.o->use_fd || !g) {
    std::vector<double> gf(c.P);
    gs_status s = (!c.o->use_fd && g) ? gs_nll_grad(c.M, c.full.data(), &f, gf.data(), &st)
                                      : gs_nll(c.M, c.full.data(), &f, &st);
    c.n_eval++;
    if (s != GS_OK) c.err = s;
    if (g)
      for (int q = 0; q < n; q++) g[q] = gf[c.idx[q]];
    return f;
  }
  gs_status s = gs_nll(c.M, c.full.data(), &f, &st);
  c.n_eval++;
  if (s != GS_OK) c.err = s;
  for (int q = 0; q < n; q++) {
    const int p = c.idx[q];
    const double h = 1e-4 * c.o->scale[p], x0 = c.full[p];
    double fp, fm;
    uint32_t s1 = 0, s2 = 0;
    c.full[p] = x0 + h;
    if (gs_nll(c.M, c.full.data(), &fp, &s1) != GS_OK) c.err = GS_ERR_DEVICE;
    c.full[p] = x0 - h;
    if (gs_nll(c.M, c.full.data(), &fm, &s2) != GS_OK) c.err = GS_ERR_DEVICE;
    c.full[p] = x0;
    c.n_eval += 2;
    g[q] = (fp - fm) / (2.0 * h);
    st |= s1 | s2;
  }
  return f;
}

bool invert(int n, std::vector<double> a, std::vector<double> &inv) {
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; i++) inv[(size_t)i * n + i] = 1.0;
  for (int c = 0; c < n; c++) {
    int piv = c;
    for (int r = c + 1; r < n; r++)
      if (std::fabs(a[(size_t)r * n + c]) > std::fabs(a[(size_t)piv * n + c])) piv = r;
    if (a[(size_t)piv * n + c] == 0.0) return false;
    if (piv != c)
      for (int j = 0; j < n; j++) {
        std::swap(a[(size_t)c * n + j], a[(size_t)piv * n + j]);
        std::swap(inv[(size_t)c * n + j], inv[(size_t)piv * n + j]);
      }
    const double d = a[(size_t)c * n + c];
    for (int j = 0; j < n; j++) {
      a[(size_t)c * n + j] /= d;
      inv[(size_t)c * n + j] /= d;
    }
    for (int r = 0; r < n; r++) {
      if (r == c) continue;
      const double f = a[(size_t)r * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; j++) {
        a[(size_t)r * n + j] -= f * a[(size_t)c * n + j];
        inv[(size_t)r * n + j] -= f * inv[(size_t)c * n + j];
      }
    }
  }
  return true;
}

}  // namespace

extern "C" gs_status gs_fit(gs_model *M, const double *theta0, const gs_fit_opts *o, double *theta_hat,
                            double *sigma, gs_fit_result *res) {
  if (!M || !theta0 || !o || !o->scale || !theta_hat || !res) return GS_ERR_ARG;
  Ctx c{M, o, gs_model_num_params(M)};
  c.full.assign(theta0, theta0 + c.P);
  for (int p = 0; p < c.P; p++) {
    if (!(o->scale[p] > 0)) return GS_ERR_ARG;
    if (!o->free_mask || o->free_mask[p]) c.idx.push_back(p);
  }
  const int n = (int)c.idx.size();
  std::vector<double> x(n), g(n), H((size_t)n * n), H0((size_t)n * n, 0.0), d(n), xt(n), gt(n), s(n), y(n), Hy(n);
  for (int q = 0; q < n; q++) {
    x[q] = theta0[c.idx[q]];
    H0[(size_t)q * n + q] = o->scale[c.idx[q]] * o->scale[c.idx[q]];
  }
  H = H0;
  uint32_t st = 0, est = 0;
  double f = evaluate(c, x.data(), g.data(), est);
  st |= est & (GS_ST_NONFINITE | GS_ST_DOMAIN | GS_ST_UNRESOLVED | GS_ST_GRAD_RANGE);
  // a start without an FP64 gradient cannot begin a quasi-Newton step
  const bool no_grad = (est & GS_ST_GRAD_RANGE) != 0;
  double edm = INFINITY;
  int it = 0;
  while (std::isfinite(f) && !no_grad && c.err == GS_OK) {
    edm = 0.0;
    for (int i = 0; i < n; i++) {
      double hg = 0.0;
      for (int j = 0; j < n; j++) hg += H[(size_t)i * n + j] * g[j];
      d[i] = -hg;
      edm += 0.5 * g[i] * hg;
    }
    if (edm < o->edm_tol) {
      st |= GS_ST_CONVERGED;
      break;
    }
    if (it >= o->max_iter) {
      st |= GS_ST_MAXITER;
      break;
    }
    double slope = 0.0;
    for (int i = 0; i < n; i++) slope += g[i] * d[i];
    if (!(slope < 0.0)) {  // not a descent direction: restart from the diagonal metric
      H = H0;
      st |= GS_ST_BFGS_RESET;
      slope = 0.0;
      for (int i = 0; i < n; i++) {
        d[i] = -H0[(size_t)i * n + i] * g[i];
        slope += g[i] * d[i];
      }
    }
    double alpha = 1.0, ft = INFINITY;
    bool ok = false, have_g = false;
    for (int ls = 0; ls < 40; ls++) {
      for (int i = 0; i < n; i++) xt[i] = x[i] + alpha * d[i];
      // adjoint path: take the gradient with the trial value; plain path: value only
      have_g = !o->use_fd;
      ft = evaluate(c, xt.data(), have_g ? gt.data() : nullptr, est);
      if (c.err != GS_OK) break;
      // a trial point whose gradient has no FP64 value is not taken
      const bool usable = std::isfinite(ft) && !(est & GS_ST_GRAD_RANGE);
      if (usable && ft <= f + 1e-4 * alpha * slope + 1e-14 * std::fabs(f)) {
        ok = true;
        break;
      }
      if (usable) {
        const double aq = -slope * alpha * alpha / (2.0 * (ft - f - slope * alpha));
        alpha = std::fmin(std::fmax(aq, 0.1 * alpha), 0.5 * alpha);
      } else {
        alpha *= 0.25;
      }
    }
    if (!ok) {
      st |= GS_ST_LS_FAIL;
      break;
    }
    if (!have_g) ft = evaluate(c, xt.data(), gt.data(), est);
    double sy = 0.0, ss = 0.0, yy = 0.0;
    for (int i = 0; i < n; i++) {
      s[i] = xt[i] - x[i];
      y[i] = gt[i] - g[i];
      sy += s[i] * y[i];
      ss += s[i] * s[i];
      yy += y[i] * y[i];
    }
    if (sy > 1e-12 * std::sqrt(ss * yy)) {
      double yHy = 0.0;
      for (int i = 0; i < n; i++) {
        double a = 0.0;
        for (int j = 0; j < n; j++) a += H[(size_t)i * n + j] * y[j];
        Hy[i] = a;
        yHy += y[i] * a;
      }
      const double rho = 1.0 / sy, k2 = rho + rho * rho * yHy;
      for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
          H[(size_t)i * n + j] += k2 * s[i] * s[j] - rho * (Hy[i] * s[j] + s[i] * Hy[j]);
    } else {
      H = H0;
      st |= GS_ST_BFGS_RESET;
    }
    x = xt;
    g = gt;
    f = ft;
    it++;
  }
  if (c.err != GS_OK) return c.err;
  for (int p = 0; p < c.P; p++) theta_hat[p] = theta0[p];
  for (int q = 0; q < n; q++) theta_hat[c.idx[q]] = x[q];
  if (sigma) {
    for (int p = 0; p < c.P; p++) sigma[p] = 0.0;
    if (o->hesse && std::isfinite(f)) {
      std::vector<double> Hs((size_t)n * n), Hi, full(theta_hat, theta_hat + c.P), gp(c.P), gm(c.P);
      for (int q = 0; q < n; q++) {
        const int p = c.idx[q];
        const double h = 1e-4 * o->scale[p], x0 = full[p];
        double fv;
        uint32_t s1;
        full[p] = x0 + h;
        gs_status e1 = gs_nll_grad(M, full.data(), &fv, gp.data(), &s1);
        full[p] = x0 - h;
        gs_status e2 = gs_nll_grad(M, full.data(), &fv, gm.data(), &s1);
        full[p] = x0;
        if (e1 != GS_OK || e2 != GS_OK) return GS_ERR_DEVICE;
        for (int r = 0; r < n; r++) Hs[(size_t)r * n + q] = (gp[c.idx[r]] - gm[c.idx[r]]) / (2.0 * h);
      }
      for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++)
          Hs[(size_t)i * n + j] = Hs[(size_t)j * n + i] = 0.5 * (Hs[(size_t)i * n + j] + Hs[(size_t)j * n + i]);
      if (invert(n, Hs, Hi))
        for (int q = 0; q < n; q++) {
          const double v = Hi[(size_t)q * n + q];
          sigma[c.idx[q]] = v > 0 ? std::sqrt(v) : NAN;
        }
    } else {
      for (int q = 0; q < n; q++) sigma[c.idx[q]] = std::sqrt(std::fmax(H[(size_t)q * n + q], 0.0));
    }
  }
  res->nll = f;
  res->edm = edm;
  res->iters = it;
  res->n_eval = c.n_eval;
  res->status = st;
  return GS_OK;
}
