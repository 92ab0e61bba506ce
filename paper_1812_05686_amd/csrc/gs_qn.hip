// gs_qn.hip -- device-resident quasi-Newton minimisation of many toys.
//
// Every toy runs the same BFGS method as the host driver (inverse-Hessian
// update, backtracking Armijo line search with safeguarded quadratic
// interpolation, EDM = 1/2 g^T H g stopping rule): the minimizer that fits
// each pseudo-experiment of the paper's toy studies (section 4.2), run for
// all toys at once.  One 64-lane wavefront per toy; lane p owns parameter p
// and row p of the inverse Hessian.  Each call of k_qn_step consumes the
// evaluation at the toy's trial point and writes the next trial point, so a
// fit is a fixed sequence [evaluate, step] that can be captured in a graph.
#include "gs_qn.h"

namespace gs {

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// scale: row t at scale + t * scale_stride (scale_stride 0: one row for every
// toy); a non-positive or non-finite entry is taken as 1.
__global__ __launch_bounds__(64) void k_qn_init(QNView q, const double *__restrict__ theta0,
                                                const uint8_t *__restrict__ free_mask, const double *__restrict__ scale,
                                                int scale_stride) {
  const int t = blockIdx.x, p = threadIdx.x, P = q.P;
  const size_t r = (size_t)t * P;
  const bool fr = p < q.n_par[t] && (!free_mask || free_mask[r + p]);
  if (p < P) {
    double sc = scale[(size_t)t * scale_stride + p];
    if (!(sc > 0.0 && sc < INFINITY)) sc = 1.0;
    q.x[r + p] = theta0[r + p];
    q.xt[r + p] = theta0[r + p];
    q.freep[r + p] = fr ? 1 : 0;
    q.h0[r + p] = fr ? sc * sc : 0.0;
    for (int c = 0; c < P; c++) q.H[(r + p) * P + c] = (c == p && fr) ? sc * sc : 0.0;
  }
  if (p == 0) {
    q.phase[t] = kPhaseInit;
    q.iter[t] = 0;
    q.nls[t] = 0;
    q.status[t] = 0;
    q.active[t] = 1;
  }
}

__global__ __launch_bounds__(64) void k_qn_step(QNView q, const int *__restrict__ toy_list,
                                                const double *__restrict__ nll_eval,
                                                const double *__restrict__ grad_eval,
                                                const uint32_t *__restrict__ st_eval, double edm_tol, int max_iter) {
  const int t = toy_list ? toy_list[blockIdx.x] : (int)blockIdx.x, p = threadIdx.x, P = q.P;
  if (!q.active[t]) return;
  const size_t r = (size_t)t * P;
  const bool lane = p < P;
  const bool fr = lane && q.freep[r + p];
  const double ft = nll_eval[t];
  const double gtp = fr ? grad_eval[(size_t)t * q.stride + p] : 0.0;
  double xp = lane ? q.x[r + p] : 0.0, xtp = lane ? q.xt[r + p] : 0.0;
  double gp = lane ? q.g[r + p] : 0.0;
  double f = q.f[t];
  uint32_t status = q.status[t];
  int phase = q.phase[t], iter = q.iter[t];
  bool new_direction = false;
  // lane p's row of the inverse Hessian, held in registers from its first use
  // in this step to its one write-back (P <= GS_MAX_PARAMS)
  double Hr[GS_MAX_PARAMS];
  bool have_row = false;
  auto load_row = [&] {
#pragma unroll
    for (int c = 0; c < GS_MAX_PARAMS; c++) Hr[c] = lane && c < P ? q.H[(r + p) * P + c] : 0.0;
    have_row = true;
  };
  auto store_row = [&] {
#pragma unroll
    for (int c = 0; c < GS_MAX_PARAMS; c++)
      if (lane && c < P) q.H[(r + p) * P + c] = Hr[c];
  };
  auto reset_row = [&] {  // the diagonal metric (lanes past P read nothing)
    const double h0p = lane ? q.h0[r + p] : 0.0;
#pragma unroll
    for (int c = 0; c < GS_MAX_PARAMS; c++) Hr[c] = c == p ? h0p : 0.0;
  };
  // a point whose gradient has no FP64 value (GS_ST_GRAD_RANGE) is not taken
  const bool usable = isfinite(ft) && !(st_eval[t] & GS_ST_GRAD_RANGE);
  if (phase == kPhaseInit) {
    if (!usable) {
      if (p == 0) {
        q.status[t] = status | (st_eval[t] & (GS_ST_DOMAIN | GS_ST_NONFINITE | GS_ST_UNRESOLVED | GS_ST_GRAD_RANGE));
        q.active[t] = 0;
      }
      return;
    }
    xp = xtp;
    f = ft;
    gp = gtp;
    new_direction = true;
  } else {
    const double alpha = q.alpha[t], slope = q.slope[t];
    if (usable && ft <= f + 1e-4 * alpha * slope + 1e-14 * fabs(f)) {
      // accept the trial point; BFGS update of the inverse Hessian
      const double s = fr ? xtp - xp : 0.0, y = fr ? gtp - gp : 0.0;
      const double sy = wave_sum(s * y), ss = wave_sum(s * s), yy = wave_sum(y * y);
      load_row();
      if (sy > 1e-12 * sqrt(ss * yy)) {
        // Hy_p = sum_c H_pc y_c: lane p needs every y_c, read through shuffles
        double hy = 0.0;
#pragma unroll
        for (int c = 0; c < GS_MAX_PARAMS; c++)
          if (c < P) {
            const double yc = __shfl(y, c, 64);
            if (lane) hy = __fma_rn(Hr[c], yc, hy);
          }
        const double yHy = wave_sum(y * hy);
        const double rho = 1.0 / sy, k2 = rho + rho * rho * yHy;
#pragma unroll
        for (int c = 0; c < GS_MAX_PARAMS; c++)
          if (c < P) {
            const double sc = __shfl(s, c, 64), hyc = __shfl(hy, c, 64);
            if (lane) Hr[c] += k2 * s * sc - rho * (hy * sc + s * hyc);
          }
      } else {
        reset_row();
        status |= GS_ST_BFGS_RESET;
      }
      store_row();
      xp = xtp;
      f = ft;
      gp = gtp;
      iter += 1;
      new_direction = true;
    } else {
      const int nls = q.nls[t] + 1;
      if (nls >= 40) {
        if (p == 0) {
          q.status[t] = status | GS_ST_LS_FAIL;
          q.active[t] = 0;
        }
        return;
      }
      double a;
      if (usable) {
        const double aq = -slope * alpha * alpha / (2.0 * (ft - f - slope * alpha));
        a = fmin(fmax(aq, 0.1 * alpha), 0.5 * alpha);
      } else {
        a = 0.25 * alpha;
      }
      if (lane) q.xt[r + p] = fr ? xp + a * q.d[r + p] : xp;
      if (p == 0) {
        q.alpha[t] = a;
        q.nls[t] = nls;
      }
      return;
    }
  }
  // new search direction d = -H g from the accepted point
  if (new_direction) {
    if (!have_row) load_row();
    double hg = 0.0;
#pragma unroll
    for (int c = 0; c < GS_MAX_PARAMS; c++)
      if (c < P) {
        const double gc = __shfl(gp, c, 64);
        if (lane) hg = __fma_rn(Hr[c], gc, hg);
      }
    double d = fr ? -hg : 0.0;
    const double edm = -0.5 * wave_sum(gp * d);
    uint32_t done = 0;
    if (edm < edm_tol)
      done = GS_ST_CONVERGED;
    else if (iter >= max_iter)
      done = GS_ST_MAXITER;
    double slope = wave_sum(gp * d);
    if (!done && !(slope < 0.0)) {  // not a descent direction: restart from the diagonal metric
      reset_row();
      store_row();
      status |= GS_ST_BFGS_RESET;
      d = fr ? -q.h0[r + p] * gp : 0.0;
      slope = wave_sum(gp * d);
    }
    if (lane) {
      q.x[r + p] = xp;
      q.g[r + p] = gp;
      q.d[r + p] = d;
      q.xt[r + p] = fr ? xp + d : xp;
    }
    if (p == 0) {
      q.f[t] = f;
      q.edm[t] = edm;
      q.iter[t] = iter;
      q.phase[t] = kPhaseSearch;
      q.alpha[t] = 1.0;
      q.slope[t] = slope;
      q.nls[t] = 0;
      q.status[t] = status | done;
      if (done) q.active[t] = 0;
    }
  }
}

// Deterministic count of the toys still running (one block).
__global__ __launch_bounds__(256) void k_qn_count(const uint8_t *__restrict__ active, int n, int *__restrict__ out) {
  __shared__ int part[4];
  int c = 0;
  for (int t = threadIdx.x; t < n; t += blockDim.x) c += active[t];
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = part[0] + part[1] + part[2] + part[3];
}

// Results: theta_hat = x, nll = f, sigma = sqrt(diag H) (the BFGS estimate of
// the covariance), iterations, status.
__global__ __launch_bounds__(64) void k_qn_final(QNView q, double *__restrict__ theta_hat, double *__restrict__ nll,
                                                 double *__restrict__ sigma, int32_t *__restrict__ iters,
                                                 uint32_t *__restrict__ status) {
  const int t = blockIdx.x, p = threadIdx.x, P = q.P;
  const size_t r = (size_t)t * P;
  if (p < P) {
    theta_hat[(size_t)t * q.stride + p] = q.phase[t] == kPhaseInit ? q.xt[r + p] : q.x[r + p];
    if (sigma) sigma[(size_t)t * q.stride + p] = q.freep[r + p] ? sqrt(fmax(q.H[(r + p) * P + p], 0.0)) : 0.0;
  }
  if (p == 0) {
    nll[t] = q.phase[t] == kPhaseInit ? __builtin_nan("") : q.f[t];
    iters[t] = q.iter[t];
    status[t] = q.status[t] | (q.active[t] ? GS_ST_MAXITER : 0u);
  }
}

// ------------------------------------------------------- discovery test --
// Profile-likelihood ratio of section 4.2 (Eq.5): a fit with every free
// parameter free and a fit with the signal parameter fixed at zero, per toy.
__global__ __launch_bounds__(64) void k_null_start(int stride, const double *__restrict__ theta0,
                                                   const uint8_t *__restrict__ free_mask,
                                                   const int32_t *__restrict__ signal, double *__restrict__ theta0_null,
                                                   uint8_t *__restrict__ free_null) {
  const int t = blockIdx.x, sig = signal[t];
  for (int p = threadIdx.x; p < stride; p += 64) {
    const size_t r = (size_t)t * stride + p;
    theta0_null[r] = p == sig ? 0.0 : theta0[r];
    free_null[r] = p == sig ? 0 : (free_mask ? free_mask[r] : 1);
  }
}

// t = -2 ln(L_null / L_free) = 2 (NLL_null - NLL_free); NaN unless both fits converged.
__global__ __launch_bounds__(256) void k_discovery_t(int n, const double *__restrict__ nll_free,
                                                     const uint32_t *__restrict__ st_free,
                                                     const double *__restrict__ nll_null,
                                                     const uint32_t *__restrict__ st_null, double *__restrict__ t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool ok = (st_free[i] & GS_ST_CONVERGED) && (st_null[i] & GS_ST_CONVERGED);
  t[i] = ok ? 2.0 * (nll_null[i] - nll_free[i]) : __builtin_nan("");
}

hipError_t launch_null_start(int n, int stride, const double *theta0, const uint8_t *free_mask, const int32_t *signal,
                             double *theta0_null, uint8_t *free_null, hipStream_t st) {
  hipLaunchKernelGGL(k_null_start, dim3(n), dim3(64), 0, st, stride, theta0, free_mask, signal, theta0_null, free_null);
  return hipGetLastError();
}

hipError_t launch_discovery_t(int n, const double *nll_free, const uint32_t *st_free, const double *nll_null,
                              const uint32_t *st_null, double *t, hipStream_t st) {
  hipLaunchKernelGGL(k_discovery_t, dim3((n + 255) / 256), dim3(256), 0, st, n, nll_free, st_free, nll_null, st_null, t);
  return hipGetLastError();
}

hipError_t launch_qn_init(const QNView &q, int n, const double *theta0, const uint8_t *free_mask,
                          const double *scale, int scale_stride, hipStream_t st) {
  hipLaunchKernelGGL(k_qn_init, dim3(n), dim3(64), 0, st, q, theta0, free_mask, scale, scale_stride);
  return hipGetLastError();
}

hipError_t launch_qn_step(const QNView &q, int n, const int *toy_list, const double *nll_eval,
                          const double *grad_eval, const uint32_t *st_eval, double edm_tol, int max_iter,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_qn_step, dim3(n), dim3(64), 0, st, q, toy_list, nll_eval, grad_eval, st_eval, edm_tol,
                     max_iter);
  return hipGetLastError();
}

hipError_t launch_qn_count(const uint8_t *active, int n, int *out, hipStream_t st) {
  hipLaunchKernelGGL(k_qn_count, dim3(1), dim3(256), 0, st, active, n, out);
  return hipGetLastError();
}

hipError_t launch_qn_final(const QNView &q, int n, double *theta_hat, double *nll, double *sigma, int32_t *iters,
                           uint32_t *status, hipStream_t st) {
  hipLaunchKernelGGL(k_qn_final, dim3(n), dim3(64), 0, st, q, theta_hat, nll, sigma, iters, status);
  return hipGetLastError();
}

}  // namespace gs
