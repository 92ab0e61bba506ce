/* gs.h -- C ABI of libgs: the binned multi-observable Poisson likelihood with
 * an analytic detector-response fold, on AMD Instinct MI355X (gfx950).
 *
 * What is computed (GooStats, arXiv:1812.05686):
 *   - each species' true-energy spectrum (a histogram on a uniform grid of
 *     true-energy cells, or a single line energy for monoenergetic species,
 *     the "AnaPeak" type of section 4.3) is folded through a parametrised
 *     analytic detector response (section 2.3): the response is evaluated on
 *     the visible-energy x true-energy mesh at reco-bin midpoints, times the
 *     bin width, and summed against the spectrum (section 2.5; cost model
 *     Eq.2);
 *   - the folded spectra are scaled by rate x exposure and summed (section 4.1
 *     input list); with a secondary observable each species carries a
 *     pulse-shape distribution and the expectation is a 2-D histogram
 *     (section 2.4, Eq.3 class of fits);
 *   - -ln L = sum over window bins of (mu - n ln mu) + 1/2 sum over pulls of
 *     ((theta_p - c_p)/sigma_p)^2 (Eq.4 with ln n! dropped; n = 0 contributes
 *     mu; mu < 0, or mu = 0 with n > 0, gives +inf and GS_ST_DOMAIN; every
 *     mu > 0 gives the finite term, however small).
 *
 * Admitted responses: the pair evaluation holds the per-bin bound (1e-12
 * relative for expected counts >= 1e-3) only for responses that FP64 can
 * resolve on the binning.  With m and s the mean and width of a cell's
 * response and w the largest width of the reco bins its response covers (the
 * bins where its log-density is above the banding cut; for the gamma family
 * those at x > 0), every cell whose response reaches the fit window must
 * satisfy
 *   GAUSS_E:   s >= w / 4.5
 *   GAUSS_PE:  s >= w / 4.5 and m <= 600 s
 *   GAMMA_PE:  m <= 300 s   and w m <= 300 s^2
 * (set from the measured error of the tile-relative exponent, which grows as
 * (w/s)^2 for the Gaussian families and with w m / s^2 for gamma, and of the
 * density's conditioning on an FP64 mean, ~1e-15 m/s; the Borexino-scale
 * model has s >= 2 pe = 1.25 w, m/s <= 31 and w m / s^2 <= 1.2).  Outside it
 * the evaluation is refused: -ln L and the gradient are NaN with
 * GS_ST_UNRESOLVED.
 *
 * Parameter vector theta (FP64), same layout for gradients:
 *   [ R_0 .. R_{S-1} | response parameters | delta, kappa, eta (2-D only) ]
 *   GS_RESP_GAUSS_E  : (a, b)            m = E, s^2 = a^2 + b E
 *   GS_RESP_GAUSS_PE : (LY, kB, a, b, c) m = LY Q(E; kB) E, s^2 = a^2 + b m + c^2 m^2
 *   GS_RESP_GAMMA_PE : same moments, gamma density with mean m, variance s^2
 *   GS_RESP_GENGAMMA_PE, GS_RESP_SPOIS_PE, GS_RESP_EMG_PE: same parameters
 *                      and moments, the further densities of gs_family
 *   GS_RESP_TEMPLATE : none (Monte Carlo templates, see gs_family)
 *   Q(E; kB) = 1 - 2/y + 2 ln(1 + y)/y^2, y = sqrt(E)/(kB * birks_A)  (Birks'
 *   law integrated with dE/dx = birks_A/sqrt(E); E in MeV for the pe families).
 *   Pulse shape of species s (2-D): two Gaussians (w1, mean1, sigma1) and
 *   (1 - w1, mean2, sigma2) at the bin midpoints, means shifted by delta,
 *   widths scaled by kappa, odds of component 1 multiplied by exp(eta),
 *   renormalised over the pulse-shape bins.
 *
 * Conventions: all floating point is FP64, sizes int32, arrays row-major.
 * No C++ exception crosses the ABI.  A gs_status return reports API or
 * device failures (message via gs_last_error()); mathematical conditions are
 * reported as status bits alongside values, never as a gs_status.
 */
#ifndef GS_H
#define GS_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GS_OK = 0,
  GS_ERR_ARG = 1,         /* invalid argument or descriptor                 */
  GS_ERR_DEVICE = 2,      /* HIP runtime error, or no usable gfx950 device  */
  GS_ERR_OOM = 3,         /* device or pinned host allocation failed        */
  GS_ERR_UNSUPPORTED = 4  /* valid but outside the implemented limits       */
} gs_status;

/* Per-evaluation / per-toy status bits. */
#define GS_ST_DOMAIN 1u      /* mu < 0, mu = 0 with n > 0, or invalid response: -ln L = +inf */
#define GS_ST_NONFINITE 2u   /* non-finite parameter: -ln L = NaN                              */
#define GS_ST_LS_FAIL 4u     /* fit: line search exhausted                                     */
#define GS_ST_MAXITER 8u     /* fit: iteration limit reached                                   */
#define GS_ST_BFGS_RESET 16u /* fit: inverse Hessian reset (curvature y^T s <= 0)              */
#define GS_ST_CONVERGED 32u  /* fit: EDM below tolerance                                       */
/* A bin with n > 0 has mu so small that the gradient seed 1 - n/mu overflows
 * FP64 (n/mu > DBL_MAX, decided in FP64): -ln L is finite and valid, the
 * gradient has no FP64 value and is NaN.  Fits do not step to such points. */
#define GS_ST_GRAD_RANGE 64u
/* A response outside the admitted range (see above) reaches the window: the
 * evaluation is refused, -ln L and the gradient are NaN. */
#define GS_ST_UNRESOLVED 128u

/* GS_RESP_TEMPLATE: the Monte Carlo fit of section 3.2 (cost model Eq.1): each
 * species' reco spectrum at unit rate and exposure is given as a template, so
 * there is no response and no fold: mu_dj = eps_d sum_s R_s T_sj.  The
 * descriptor's spectra hold the templates [n_species][n_reco] (n_true =
 * n_reco; e_lo, e_step and birks_A are not used, every line_energy is NaN,
 * n_psd = 0), and theta holds the rates alone. */
/* Section 2.3 names three further response functions without formulas; the
 * library takes them as follows (mean m and width s from the photoelectron
 * moments above, `shape` from the descriptor):
 *   GS_RESP_GENGAMMA_PE: the generalized gamma p x^(kp-1) exp(-(x/th)^p) /
 *     (Gamma(k) th^(kp)), power p = shape > 0, k = m^2/(p^2 s^2),
 *     th = m Gamma(k)/Gamma(k + 1/p): mean m, variance s^2 up to O(1/k);
 *     p = 1 is GS_RESP_GAMMA_PE.
 *   GS_RESP_SPOIS_PE: the scaled Poisson, x/g ~ Poisson(lambda) with
 *     g = s^2/m, lambda = m^2/s^2, continued to real x >= 0 through the
 *     Gamma function and not renormalised (its integral falls short of 1 by
 *     e^-lambda int_0^inf e^(-lambda t) dt / (t (pi^2 + ln^2 t))).
 *   GS_RESP_EMG_PE: the modified Gaussian, a Gaussian convolved with an
 *     exponential of mean tau = f s, f = shape in (0, 1), Gaussian width
 *     s sqrt(1 - f^2) and mean m - tau.
 * These families, and any model with exact_bins = 1, go through a direct
 * per-pair evaluation (one-dimensional models only, GS_ERR_ARG for
 * n_psd > 0).  Their admitted range (GS_ST_UNRESOLVED outside, as above):
 * m <= 300 s for the gamma-type families and the scaled Poisson, m <= 600 s
 * for the Gaussian photoelectron family and the modified Gaussian, none for
 * the energy family (its mean is the cell energy); the bin width is not
 * limited. */
typedef enum {
  GS_RESP_GAUSS_E = 0,
  GS_RESP_GAUSS_PE = 1,
  GS_RESP_GAMMA_PE = 2,
  GS_RESP_TEMPLATE = 3,
  GS_RESP_GENGAMMA_PE = 4,
  GS_RESP_SPOIS_PE = 5,
  GS_RESP_EMG_PE = 6
} gs_family;

/* Limits of this implementation (GS_ERR_UNSUPPORTED beyond them). */
#define GS_MAX_SPECIES 16
#define GS_MAX_DATASETS 8
#define GS_MAX_PARAMS (GS_MAX_SPECIES + 5 + 3)
#define GS_MAX_PSD 128

/* Description of one fit problem (section 4.1 lists its inputs: data
 * histogram, components and their types, rates and response parameters,
 * pull terms, exposure; section 2.1: several datasets).  The library copies
 * everything it needs; the caller keeps ownership of every array. */
typedef struct {
  int32_t n_true;             /* true-energy cells, centres e_lo + (i + 1/2) e_step      */
  double e_lo, e_step;        /* e_step > 0                                                */
  int32_t n_species;          /* 1 .. GS_MAX_SPECIES                                       */
  const double *spectra;      /* [n_species][n_true]; row ignored for line species         */
  const double *line_energy;  /* [n_species]; NaN = grid species, else line energy         */
  int32_t n_reco;             /* energy (reco) bins                                        */
  const double *reco_edges;   /* [n_reco + 1], finite, strictly increasing                 */
  int32_t n_psd;              /* 0 = one-dimensional; else pulse-shape bins                */
  const double *psd_edges;    /* [n_psd + 1] finite, strictly increasing (n_psd > 0)       */
  const double *psd_mix;      /* [n_species][5] = w1, mean1, sigma1, mean2, sigma2         */
  int32_t n_datasets;         /* 1 .. GS_MAX_DATASETS, sharing every parameter             */
  const double *exposure;     /* [n_datasets], > 0                                         */
  const double *counts;       /* [n_datasets][n_reco][max(n_psd,1)], finite, >= 0          */
  int32_t win_lo, win_hi;     /* energy-bin window [win_lo, win_hi), 0 <= lo < hi <= n_reco */
  int32_t family;             /* gs_family                                                 */
  double birks_A;             /* stopping-power constant of the quenching model (> 0)      */
  const double *pull_centre;  /* [n_params] or NULL (no pulls)                             */
  const double *pull_sigma;   /* [n_params] or NULL; sigma <= 0 means no pull on that one  */
  /* Multivariate slice likelihood (section 2.4, cost model Eq.3), for n_psd > 0:
   * n_slices = 0 gives the joint likelihood over every (energy, pulse-shape)
   * bin; n_slices > 0 gives the energy histogram's likelihood (counts summed
   * over the pulse-shape bins) plus, for each energy slice i (reco bins
   * [slice_edges[i], slice_edges[i+1]), the slices tiling [win_lo, win_hi)),
   * the likelihood of the slice's pulse-shape histogram given its total:
   * n_i. ln mu_i. - sum_k n_ik ln mu_ik with mu_ik = eps sum_s R_s P_sk
   * sum_{j in i} F_js.  With one slice per bin this equals the joint
   * likelihood; fewer slices cost fewer bins. */
  int32_t n_slices;
  const int32_t *slice_edges; /* [n_slices + 1] or NULL (n_slices = 0)                     */
  /* Reco-bin content of a deposit (section 2.5 evaluates the response on the
   * visible x true mesh): 0 = bin width x density at the bin midpoint; 1 = the
   * density's integral over the bin, as a difference of the distribution
   * function at the edges (erfc for the Gaussian families, the regularised
   * incomplete gamma for the gamma-type families, a closed form for the
   * modified Gaussian).  Not for GS_RESP_SPOIS_PE or templates. */
  int32_t exact_bins;
  double shape;               /* GENGAMMA_PE: the power p; EMG_PE: the tail fraction f     */
} gs_model_desc;

typedef struct gs_model gs_model;
typedef struct gs_batch gs_batch;

/* Message for the last non-OK return on the calling thread ("" if none). */
const char *gs_last_error(void);

/* Host-only descriptor check (no device needed).  Returns the number of
 * parameters (> 0) or -1 with the reason in gs_last_error(). */
int32_t gs_desc_validate(const gs_model_desc *d);

/* ------------------------------------------------------- single model --- */
/* Create a model on HIP device `device` (must be gfx950).  Deep-copies the
 * descriptor into device memory; `*out` is owned by the caller and released
 * with gs_model_destroy.  GS_ERR_ARG for an invalid descriptor,
 * GS_ERR_DEVICE/GS_ERR_OOM for runtime failures. */
gs_status gs_model_create(const gs_model_desc *d, int32_t device, gs_model **out);
void gs_model_destroy(gs_model *m);
int32_t gs_model_num_params(const gs_model *m);

/* -ln L at host parameters theta[n_params] (section 4.1, Eq.4), synchronous.
 * This is the plain path: per-species folded spectra are cached on the
 * device and re-folded only when a response parameter changed (the value
 * cache of section 2.5); rate-only changes cost one combine-and-reduce
 * pass.  *nll = +inf with GS_ST_DOMAIN, or NaN with GS_ST_NONFINITE. */
gs_status gs_nll(gs_model *m, const double *theta, double *nll, uint32_t *st);

/* -ln L and its gradient grad[n_params] from one forward fold and one
 * adjoint (reverse-mode) pass over the same visible x true mesh,
 * synchronous.  On GS_ST_DOMAIN / GS_ST_NONFINITE / GS_ST_UNRESOLVED /
 * GS_ST_GRAD_RANGE the gradient is NaN. */
gs_status gs_nll_grad(gs_model *m, const double *theta, double *nll, double *grad, uint32_t *st);

/* Expected counts mu[n_datasets][win_hi - win_lo][max(n_psd,1)] (host) at
 * theta (Eq.2 fold, scaled by rates and exposure).  Synchronous.  NaN where
 * gs_nll_grad would report GS_ST_UNRESOLVED or GS_ST_NONFINITE. */
gs_status gs_expected(gs_model *m, const double *theta, double *mu);

/* Per-species expected reco spectra at unit rate and exposure,
 * F[win_hi - win_lo][n_species] (host), species in descriptor order: the
 * folded component spectra that the expectation combines (Eq.2).  Synchronous. */
gs_status gs_species_spectra(gs_model *m, const double *theta, double *F);

/* Per-species pulse-shape bin probabilities P[n_species][n_psd] (host) at
 * theta (2-D models only; GS_ERR_ARG otherwise).  Synchronous. */
gs_status gs_psd_probs(gs_model *m, const double *theta, double *P);

/* Fit controls for gs_fit and gs_fit_batched. */
typedef struct {
  int32_t max_iter;         /* accepted quasi-Newton steps (e.g. 500)                         */
  double edm_tol;           /* stop when 1/2 g^T H^-1 g < edm_tol (e.g. 1e-9)                 */
  int32_t use_fd;           /* gs_fit only: 1 = central finite-difference gradient (plain path) */
  const double *scale;      /* [n_params] > 0: initial inverse Hessian diag(scale^2), FD step 1e-4*scale */
  const uint8_t *free_mask; /* [n_params] or NULL (all free)                                  */
  int32_t hesse;            /* gs_fit only: 1 = sigma from finite differences of the gradient */
} gs_fit_opts;

typedef struct {
  double nll, edm;
  int32_t iters, n_eval;
  uint32_t status;          /* GS_ST_* bits                                                    */
} gs_fit_result;

/* Quasi-Newton (BFGS, backtracking Armijo line search) minimisation on the
 * host driving the device evaluations: the minimizer role MINUIT plays in
 * section 3.2.  use_fd = 0 uses gs_nll_grad (adjoint); use_fd = 1 uses
 * central differences of gs_nll (2 calls per free parameter per gradient,
 * with the rate-only cache).  theta_hat[n_params], sigma[n_params] (sigma may
 * be NULL) are host arrays.  Returns GS_OK even if the fit did not converge:
 * check res->status. */
gs_status gs_fit(gs_model *m, const double *theta0, const gs_fit_opts *o, double *theta_hat,
                 double *sigma, gs_fit_result *res);

/* --------------------------------------------------------- batches ----- */
/* A batch of independent fit problems (pseudo-experiments), each with its
 * own data, window, exposures, pulls and parameters (section 4.2 fits many
 * fake datasets; here they run concurrently).  descs[t] describes toy t;
 * toys whose descriptors point at the same spectra, line_energy, reco_edges,
 * psd_edges and psd_mix arrays (same addresses) and agree on family, grid
 * and sizes share one device copy of that structure.  Every array is copied.
 * n_toys >= 1.  The batch is created on `device`. */
gs_status gs_batch_create(const gs_model_desc *descs, int32_t n_toys, int32_t device, gs_batch **out);
void gs_batch_destroy(gs_batch *b);
int32_t gs_batch_num_toys(const gs_batch *b);
/* Row stride of the batched parameter / gradient arrays (= max n_params). */
int32_t gs_batch_param_stride(const gs_batch *b);

/* Batched -ln L and gradient.  All pointers are DEVICE pointers on the
 * batch's device, caller-owned, FP64 contiguous: d_theta[n_toys][stride],
 * d_nll[n_toys], d_grad[n_toys][stride] (entries past a toy's n_params are
 * left 0), d_status[n_toys].  Enqueued on `hip_stream` (a hipStream_t; NULL =
 * the default stream) and returns without synchronising.  Concurrent calls on
 * one batch must be ordered by the caller (they share work buffers). */
gs_status gs_nll_grad_batched(gs_batch *b, const double *d_theta, double *d_nll, double *d_grad,
                              uint32_t *d_status, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as gs_nll_grad_batched (same kernels, same layout, bitwise the
 * same results), with the split-K and block partials of the evaluation in a
 * fixed workspace of 64 MiB that the loaded library holds on every device it
 * runs on until the process ends, instead of the batch's own buffers.  It
 * calls no allocating routine.  Batches whose partials do not fit (more than
 * a few hundred Borexino-scale toys) return GS_ERR_UNSUPPORTED.  Every call
 * on one device shares that device's workspace: calls that overlap in time on
 * one device (different streams, threads or batches) race and must be ordered
 * by the caller.  Pointers and stream as for gs_nll_grad_batched. */
gs_status gs_nll_grad_batched_noalloc(gs_batch *b, const double *d_theta, double *d_nll, double *d_grad,
                                      uint32_t *d_status, void *hip_stream);

/* Batched fits: every toy runs its own BFGS state machine on the device;
 * the evaluation and update kernels of several iterations are captured in
 * one HIP graph that is replayed until all toys stop.  Device pointers as
 * above: d_theta0[n_toys][stride] (start), d_free[n_toys][stride] (uint8,
 * NULL = all free), outputs d_theta_hat[n_toys][stride], d_nll_hat[n_toys],
 * d_sigma[n_toys][stride] (sqrt of the BFGS inverse-Hessian diagonal, may be
 * NULL), d_iters[n_toys], d_status[n_toys].  Parameter scales (the initial
 * metric is diag(scale^2)): d_scale[n_toys][stride] on the device, one row
 * per toy, or, when d_scale is NULL, o->scale, a HOST array [stride] used for
 * every toy (each entry > 0, else GS_ERR_ARG); a non-positive or non-finite
 * entry of d_scale is taken as 1.  o->use_fd and o->hesse are ignored.
 * Synchronises `hip_stream` before returning. */
gs_status gs_fit_batched(gs_batch *b, const double *d_theta0, const uint8_t *d_free, const double *d_scale,
                         const gs_fit_opts *o,
                         double *d_theta_hat, double *d_nll_hat, double *d_sigma, int32_t *d_iters,
                         uint32_t *d_status, void *hip_stream);

/* Profile-likelihood discovery test over the batch's toys (section 4.2,
 * Eq.5): per toy, a fit with every free parameter free (start d_theta0, mask
 * d_free) and a fit with the toy's signal parameter d_signal[t] (an index into
 * its theta) fixed at 0 (same start otherwise), and the statistic
 * t = -2 ln(L_null / L_free) = 2 (-ln L_null - (-ln L_free)) >= 0, NaN unless
 * both fits converged.  (Eq.5 prints the ratio the other way up; the paper's
 * own recipe takes the difference of the two fits' likelihoods, which this
 * follows.)  Device arrays as for gs_fit_batched: d_signal[n_toys] (int32),
 * d_t[n_toys], d_theta_free / d_theta_null [n_toys][stride], d_nll_free /
 * d_nll_null [n_toys], d_status_free / d_status_null [n_toys] (GS_ST_* of
 * each fit).  Scales as for gs_fit_batched.  The first call on a batch
 * allocates the null fit's start and mask.  Synchronises `hip_stream`. */
gs_status gs_discovery_batched(gs_batch *b, const double *d_theta0, const uint8_t *d_free, const double *d_scale,
                               const int32_t *d_signal, const gs_fit_opts *o, double *d_t, double *d_theta_free,
                               double *d_nll_free, uint32_t *d_status_free, double *d_theta_null, double *d_nll_null,
                               uint32_t *d_status_null, void *hip_stream);

/* ------------------------------------------------------- mesh banding --- */
/* Pairs (reco bin j, true cell i) whose log-density ln r(xbar_j | E_i) is
 * below log_cut are skipped (default -52).  Each cell's support, the bins
 * where the log-density can exceed log_cut, is solved per evaluation, so the
 * absolute error of every expected count is at most
 * sum_s |R_s| eps_d dx_j exp(log_cut) (1.6e-17 counts for the 4000-cell,
 * 900-bin model at its nominal rates: 1.6e-14 of a bin holding 1e-3 counts,
 * the smallest the 1e-12 relative bound applies to).  -INFINITY evaluates the full mesh.
 * The setting applies to later calls on the batch / model. */
gs_status gs_batch_set_log_cut(gs_batch *b, double log_cut);
gs_status gs_model_set_log_cut(gs_model *m, double log_cut);

/* --------------------------------------------------------- profiling --- */
/* Kernel ids for gs_batch_kernel_times. */
#define GS_K_CELLS 0   /* per-cell response moments and records           */
#define GS_K_FOLD 1    /* fold of the combined spectrum (adjoint path)     */
#define GS_K_NLL 2     /* Poisson terms, reduction, adjoint seeds          */
#define GS_K_ADJ 3     /* adjoint pass over the mesh (one-dimensional toys) */
#define GS_K_GRAD 4    /* chain rule to the parameter gradient             */
#define GS_K_FOLDS 5   /* per-species fold (plain path, 2-D)               */
#define GS_K_REDF 6    /* per-species split-K reduction                    */
#define GS_K_NLLF 7    /* -ln L from per-species spectra                   */
#define GS_K_QN 8      /* device quasi-Newton step                         */
#define GS_K_FINISH 9  /* per-problem totals, pulls, status                */
#define GS_K_ADJS 10   /* per-species adjoint (secondary-observable toys)   */
#define GS_K_TMPL 11   /* Monte Carlo template likelihood and rate gradient */
#define GS_K_COUNT 12

/* Work layout of a batch (the batch scheduler's tuning knobs for the toy
 * studies of section 4.2): the split-K target (work-groups the fold and the
 * adjoint aim for, by splitting each toy's cells / bins into chunks when the
 * batch alone gives fewer), cells per gradient-kernel block (256: one per
 * thread, or 1024: four per thread), rounds per block of the secondary-
 * observable likelihood and seed kernels (1 or 8), and waves per adjoint
 * workgroup (1 or 4).  The work buffers are sized at creation for every
 * candidate in the product {2048, 1024, 4096, 8192} x {256, 1024} x {1, 8
 * (secondary-observable batches only)} x {1, 4}, where a target that splits
 * the batch into the same chunk counts as an earlier one is left out; the
 * default is target 2048 with the other three chosen from the batch's size
 * (four waves per adjoint workgroup whenever the batch holds both 1-D and
 * secondary-observable toys).  Results do not depend on the layout beyond
 * the order of floating-point sums.
 *
 * gs_batch_set_layout puts one candidate in force (GS_ERR_ARG if it is not a
 * candidate).  gs_batch_autotune times gs_nll_grad_batched at d_theta under
 * every candidate (after three warm-up evaluations: two passes, the second in
 * reverse order, of one warm-up and `reps` timed evaluations each, HIP events
 * on `hip_stream`, each candidate's faster pass kept; the outputs d_nll,
 * d_grad, d_status as for gs_nll_grad_batched hold the last evaluation's
 * values) and puts the fastest in force, or the default layout when no
 * candidate beats it by more than 1%; choice (host, 5 entries, may be NULL) receives its target, cells
 * per gradient block, rounds, adjoint waves, and mean milliseconds per
 * evaluation.  gs_batch_layout reports the layout in force (the same four
 * knobs) and the number of candidates (host, 5 entries).  All three synchronise the device; a captured batched-
 * fit graph is rebuilt on the next gs_fit_batched. */
gs_status gs_batch_set_layout(gs_batch *b, int32_t target_wg, int32_t grad_cells, int32_t iter2,
                              int32_t adj_waves);
gs_status gs_batch_autotune(gs_batch *b, const double *d_theta, double *d_nll, double *d_grad, uint32_t *d_status,
                            int32_t reps, void *hip_stream, double *choice);
gs_status gs_batch_layout(const gs_batch *b, int32_t *out);
/* When on, each kernel launch of the batch is bracketed by HIP events
 * recorded on the stream the kernel is launched on (small overhead). */
gs_status gs_batch_set_profiling(gs_batch *b, int32_t on);
/* Accumulated device milliseconds and launch counts per kernel id since the
 * last reset (host arrays of GS_K_COUNT entries).  Waits for the recorded
 * events; reset != 0 clears the accumulators afterwards. */
gs_status gs_batch_kernel_times(gs_batch *b, double *ms, int64_t *launches, int32_t reset);
/* Mesh pairs (window bin x cell) of the most recent evaluation of the batch,
 * host array of 6: out[0] pairs the fold evaluated (every bin of a tile per
 * visited cell and tile: 32-bin tiles for 1-D toys, 64-bin tiles for
 * secondary-observable toys, idle lanes of a partial tile included), out[1] pairs the
 * adjoint evaluated, out[2] the full mesh sum_t (window bins x cells), out[3]
 * the banded mesh: pairs whose bin lies in the cell's support, i.e. the
 * pairs the method needs at the current log-density cut; out[4] the banded
 * pairs of secondary-observable toys (folded per species), out[5] those pairs
 * weighted by the number of species their cell carries (the grid species for
 * a grid cell, 1 for a line): the per-species contraction's multiply-adds.
 * Synchronises the device. */
gs_status gs_batch_mesh_pairs(gs_batch *b, int64_t *out);
/* Convergence profile of the most recent gs_fit_batched on this batch: after
 * each launch of the captured fit graph (a fixed number of evaluation + BFGS
 * steps), the number of toys still running and the host milliseconds since
 * the call began.  Copies min(cap, count) entries into the host arrays
 * active[] and ms[] and sets *n to the full count. */
gs_status gs_batch_fit_trace(gs_batch *b, int32_t *active, double *ms, int32_t cap, int32_t *n);

#ifdef __cplusplus
}
#endif
#endif /* GS_H */
