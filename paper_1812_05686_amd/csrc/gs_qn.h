// gs_qn.h -- per-toy quasi-Newton state on the device.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs.h"

namespace gs {

enum QNPhase : int { kPhaseInit = 0, kPhaseSearch = 1 };

// Arrays indexed [toy][P] (P = the batch parameter stride) or [toy][P][P] (H).
struct QNView {
  int P, stride;
  double *x, *xt, *g, *d, *H, *h0;  // accepted point, trial point (evaluated next), gradient, direction, inverse Hessian
  double *f, *edm, *alpha, *slope;  // per toy
  int *phase, *iter, *nls, *n_par;  // per toy
  uint32_t *status;
  uint8_t *active, *freep;
};

hipError_t launch_qn_init(const QNView &q, int n, const double *theta0, const uint8_t *free_mask,
                          const double *scale, int scale_stride, hipStream_t st);
// Grid rows are toys 0 .. n-1, or toy_list[0 .. n) when toy_list is not NULL.
hipError_t launch_qn_step(const QNView &q, int n, const int *toy_list, const double *nll_eval,
                          const double *grad_eval, const uint32_t *st_eval, double edm_tol, int max_iter,
                          hipStream_t st);
hipError_t launch_qn_count(const uint8_t *active, int n, int *out, hipStream_t st);
// Start of the null fit of the discovery test: theta0 and the free mask with
// each toy's signal parameter set to 0 and fixed.
hipError_t launch_null_start(int n, int stride, const double *theta0, const uint8_t *free_mask, const int32_t *signal,
                             double *theta0_null, uint8_t *free_null, hipStream_t st);
// t = 2 (nll_null - nll_free) where both fits converged, else NaN.
hipError_t launch_discovery_t(int n, const double *nll_free, const uint32_t *st_free, const double *nll_null,
                              const uint32_t *st_null, double *t, hipStream_t st);
hipError_t launch_qn_final(const QNView &q, int n, double *theta_hat, double *nll, double *sigma, int32_t *iters,
                           uint32_t *status, hipStream_t st);

}  // namespace gs
