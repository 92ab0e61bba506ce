/* oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 (long double where cancellation demands it) CPU
 * definition of the binned multi-observable Poisson likelihood with an
 * analytic detector-response fold, as described in "GooStats: A GPU-based
 * framework for multi-variate analysis in particle physics" (arXiv:1812.05686):
 *   - detector response (section 2.3), evaluated on the visible-energy x
 *     true-energy mesh and then summed against the true spectrum (section 2.5,
 *     and the analytical-fit cost model Eq.2);
 *   - multivariate likelihood over a secondary observable (section 2.4, Eq.3);
 *   - Poisson log-likelihood plus Gaussian pull terms (section 4.1, Eq.4);
 *   - exposure as a per-dataset multiplier (section 4.1 input list).
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may call this library.  It shares no code with the GPU library.
 */
#ifndef GS_ORACLE_H
#define GS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ORC_TEMPLATE: Monte Carlo templates (section 3.2, the Monte Carlo fit): each
 * species' spectrum is already its reco histogram at unit rate, spectra
 * [n_species][n_reco] (n_true = n_reco), so there is no fold and no response
 * parameter. */
enum { ORC_GAUSS_E = 0, ORC_GAUSS_PE = 1, ORC_GAMMA_PE = 2, ORC_TEMPLATE = 3,
       ORC_GENGAMMA_PE = 4, ORC_SPOIS_PE = 5, ORC_EMG_PE = 6 };
enum { ORC_ST_DOMAIN = 1u, ORC_ST_NONFINITE = 2u, ORC_ST_LS_FAIL = 4u,
       ORC_ST_MAXITER = 8u, ORC_ST_BFGS_RESET = 16u, ORC_ST_GRAD_RANGE = 64u };

typedef struct {
  int32_t n_true;            /* true-energy cells, centres e_lo + (i + 1/2) e_step   */
  double e_lo, e_step;
  int32_t n_species;
  const double *spectra;     /* [n_species][n_true]; ignored for line species         */
  const double *line_energy; /* [n_species]; NaN = grid species, else the line energy */
  int32_t n_reco;
  const double *reco_edges;  /* [n_reco + 1]                                          */
  int32_t n_psd;             /* 0 = one-dimensional                                   */
  const double *psd_edges;   /* [n_psd + 1]                                           */
  const double *psd_mix;     /* [n_species][5] = w1, mean1, sigma1, mean2, sigma2     */
  int32_t n_datasets;
  const double *exposure;    /* [n_datasets]                                          */
  const double *counts;      /* [n_datasets][n_reco][max(n_psd,1)]                    */
  int32_t win_lo, win_hi;    /* energy-bin window [lo, hi)                            */
  int32_t family;
  double birks_A;
  const double *pull_centre; /* [n_params]                                            */
  const double *pull_sigma;  /* [n_params]; <= 0 means no pull                        */
  /* Multivariate slice likelihood (section 2.4; n_psd > 0): 0 = the joint 2-D
   * likelihood over every (energy, pulse-shape) bin; n > 0 = the energy
   * likelihood plus one secondary-observable piece per energy slice, slice i
   * covering reco bins [slice_edges[i], slice_edges[i+1]), the slices tiling
   * the window. */
  int32_t n_slices;
  const int32_t *slice_edges;  /* [n_slices + 1]                                        */
  /* Reco-bin content (section 2.5 mesh): 0 = bin width x density at the
   * midpoint, 1 = the density's integral over the bin (distribution-function
   * differences; not for the scaled Poisson). */
  int32_t exact_bins;
  /* Shape parameter of the family: the power p of the generalized gamma,
   * the tail fraction f = tau/s of the modified Gaussian; unused otherwise. */
  double shape;
} orc_model;

int32_t orc_num_params(const orc_model *M);

/* Building blocks, exported for the pins. */
double orc_quench(double e_mev, double kB, double A);
double orc_dquench_dkB(double e_mev, double kB, double A);
double orc_digamma(double x);
/* Response moments at true energy E for response parameters resp[]. Returns 0 if invalid. */
int32_t orc_moments(int32_t family, const double *resp, double birks_A, double E,
                    double *m, double *s);
double orc_density(int32_t family, double x, double m, double s);
void orc_density_dms(int32_t family, double x, double m, double s, double *dlnr_dm, double *dlnr_ds);
double orc_density3(int32_t family, double shape, double x, double m, double s);
void orc_density_dms3(int32_t family, double shape, double x, double m, double s, double *dlnr_dm, double *dlnr_ds);
/* Content of reco bin [xlo, xhi) for a deposit with response moments (m, s), and its derivatives. */
int32_t orc_bin_content(int32_t family, double shape, int32_t exact, double xlo, double xhi, double m, double s,
                        double *K, double *dKdm, double *dKds);
/* Regularised incomplete gamma P(k, u), Q = 1 - P and dP/dk. */
int32_t orc_igam(double k, double u, double *P, double *Q, double *dPdk);

/* F[j][s]: per-species reco spectrum at unit rate and exposure, all reco bins. */
int32_t orc_species_fold(const orc_model *M, const double *theta, double *F);
/* P[s][k]: per-species pulse-shape bin probabilities (2-D models only). */
int32_t orc_psd_probs(const orc_model *M, const double *theta, double *P);
/* mu[d][j][k] for all reco bins j (window ignored). */
int32_t orc_expected(const orc_model *M, const double *theta, double *mu);
/* -ln L over the window, plus pulls; status bits in *st. grad may be NULL. */
double orc_nll(const orc_model *M, const double *theta, uint32_t *st);
double orc_nll_grad(const orc_model *M, const double *theta, double *grad, uint32_t *st);

typedef struct {
  int32_t max_iter;     /* accepted BFGS steps                                     */
  double edm_tol;       /* stop when 0.5 g^T H^-1 g < edm_tol                       */
  int32_t use_fd;       /* 1: central finite-difference gradient (plain path)       */
  const double *scale;  /* [P] parameter scales: initial metric, FD steps 1e-4*s     */
  const uint8_t *free_mask; /* [P]; NULL = all free                               */
  int32_t hesse;        /* 1: sigma from finite differences of the analytic gradient */
} orc_fit_opts;

typedef struct {
  double nll, edm;
  int32_t iters, n_eval;
  uint32_t status;
} orc_fit_result;

int32_t orc_fit(const orc_model *M, const double *theta0, const orc_fit_opts *o,
                double *theta_hat, double *sigma, orc_fit_result *res);

/* Profile-likelihood discovery statistic (section 4.2, Eq.5): t = 2 (-ln L of the
 * fit with parameter `signal` fixed at 0  -  -ln L of the fit with it free), the
 * other free parameters profiled in both.  The free fit starts at theta0; the
 * null fit at theta0 with theta0[signal] set to 0.  o->free_mask (or all) gives
 * the free parameters of the free fit.  Returns 1 when both fits converged. */
int32_t orc_discovery(const orc_model *M, const double *theta0, const orc_fit_opts *o, int32_t signal,
                      double *t, double *theta_free, double *theta_null, orc_fit_result *res_free,
                      orc_fit_result *res_null);

#ifdef __cplusplus
}
#endif
#endif
