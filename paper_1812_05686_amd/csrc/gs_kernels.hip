// gs_kernels.hip -- gfx950 kernels of the fold likelihood and its adjoint.
//
// One evaluation (section 2.5: the response on the visible x true mesh is
// evaluated and smeared against the true spectrum; Eq.2 cost ~ N_vis N_true):
//   k_cells  per (toy, cell): response moments and the per-cell record
//   k_fold1  per wave: 64 window bins (one per lane) x a cell range; the cell
//            records are wave-uniform and come through scalar loads, so the
//            VALU only does the per-pair exponent, one exp and one FMA
//   k_nll1   per toy: split-K partial sums in fixed order, Poisson terms of
//            Eq.4, adjoint seeds G_j = dx_j sum_d eps_d (1 - n_dj/mu_dj)
//   k_adj1   per wave: 64 cells (one per lane) x a window-bin range; bins are
//            wave-uniform; per-cell sums of G r {1, t1, t2}
//   k_grad1  per toy: chain rule from per-cell sums to d(-ln L)/d theta
// No floating-point atomics: every reduction has a fixed order, so results
// are bitwise reproducible for a fixed launch configuration.
#include "gs_impl.h"

namespace gs {

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Deterministic block sum of one double per thread (blockDim.x = 256).
__device__ double block_sum(double v, double *lds) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); i++) r += lds[i];
  return r;  // valid on thread 0
}

// ------------------------------------------------------------ k_cells -----
__global__ __launch_bounds__(256) void k_cells(const ToyDev *__restrict__ toys, const ShapeDev *__restrict__ shapes,
                                               const double *__restrict__ theta, int stride,
                                               const uint8_t *__restrict__ active, double *__restrict__ rec) {
  const int t = blockIdx.y;
  if (active && !active[t]) return;
  const ToyDev &T = toys[t];
  const ShapeDev &Sh = shapes[T.shape];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Sh.n_cell) return;
  const double *th = theta + (size_t)t * stride;
  Moments mo;
  bool ok = moments(Sh.family, th + Sh.S, Sh.birks_A, Sh.cellE[i], mo);
  double W = 0.0;
  if (i < Sh.n_true) {
    const double *w = Sh.wcell + (size_t)i * Sh.Sg;
    for (int s = 0; s < Sh.Sg; s++) W = __fma_rn(th[Sh.sp_of[s]], w[s], W);
  } else {
    W = th[Sh.sp_of[Sh.Sg + (i - Sh.n_true)]];
  }
  cell_record(Sh.family, mo.m, mo.s, W, ok, rec + (T.cell_off + i) * kRecLen);
}

hipError_t launch_cells(const BatchView &v, const double *theta, const uint8_t *active, int max_cells, hipStream_t st) {
  dim3 grid((max_cells + 255) / 256, v.n_toys);
  hipLaunchKernelGGL(k_cells, grid, dim3(256), 0, st, v.toys, v.shapes, theta, v.stride, active, v.rec);
  return hipGetLastError();
}

// ------------------------------------------------------------ k_fold1 -----
template <int FAM>
__device__ __forceinline__ double fold_range(const double *__restrict__ R, int c0, int c1, double x, double Lh,
                                             double Ll) {
  double a0 = 0.0, a1 = 0.0;
  int i = c0;
  for (; i + 1 < c1; i += 2) {
    const double *p = R + (size_t)i * kRecLen;
    const double *q = p + kRecLen;
    if (FAM == kGammaPE) {
      double e0 = gamma_exponent(p[0], p[1], p[2], p[3], p[4], x, Lh, Ll);
      double e1 = gamma_exponent(q[0], q[1], q[2], q[3], q[4], x, Lh, Ll);
      a0 = __fma_rn(p[5], exp(e0), a0);
      a1 = __fma_rn(q[5], exp(e1), a1);
    } else {
      double z0, z1;
      double e0 = gauss_exponent(p[0], p[1], p[2], x, z0);
      double e1 = gauss_exponent(q[0], q[1], q[2], x, z1);
      a0 = __fma_rn(p[3], exp(e0), a0);
      a1 = __fma_rn(q[3], exp(e1), a1);
    }
  }
  if (i < c1) {
    const double *p = R + (size_t)i * kRecLen;
    if (FAM == kGammaPE) {
      a0 = __fma_rn(p[5], exp(gamma_exponent(p[0], p[1], p[2], p[3], p[4], x, Lh, Ll)), a0);
    } else {
      double z;
      a0 = __fma_rn(p[3], exp(gauss_exponent(p[0], p[1], p[2], x, z)), a0);
    }
  }
  return a0 + a1;
}

__global__ __launch_bounds__(256) void k_fold1(const FoldItem *__restrict__ items, int n_items,
                                               const ToyDev *__restrict__ toys, const ShapeDev *__restrict__ shapes,
                                               const double *__restrict__ rec, const uint8_t *__restrict__ active,
                                               double *__restrict__ fpart) {
  const int w = wave_uniform((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (w >= n_items) return;
  const int lane = threadIdx.x & 63;
  const FoldItem it = items[w];
  if (active && !active[it.toy]) return;
  const ToyDev &T = toys[it.toy];
  const ShapeDev &Sh = shapes[T.shape];
  const int b = it.bin0 + lane;
  const bool valid = b < T.L;
  const int j = T.lo + (valid ? b : T.L - 1);
  const double *bn = Sh.bins + (size_t)j * kBinLen;
  const double x = bn[0], Lh = bn[2], Ll = bn[3];
  const double *R = rec + T.cell_off * kRecLen;
  double acc;
  if (Sh.family == kGammaPE) {
    acc = fold_range<kGammaPE>(R, it.cell0, it.cell1, x, Lh, Ll);
    if (!(x > 0.0)) acc = 0.0;
  } else {
    acc = fold_range<kGaussE>(R, it.cell0, it.cell1, x, Lh, Ll);
  }
  if (valid) fpart[T.fpart_off + (long long)it.chunk * T.L + b] = acc;
}

hipError_t launch_fold1(const BatchView &v, hipStream_t st) {
  if (v.n_fold_items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fold1, dim3((v.n_fold_items + 3) / 4), dim3(256), 0, st, v.fold_items, v.n_fold_items,
                     v.toys, v.shapes, v.rec, (const uint8_t *)nullptr, v.fpart);
  return hipGetLastError();
}

// ------------------------------------------------------------ k_nll1 ------
// Poisson term of Eq.4 (ln n! dropped).  Returns false on a domain error.
__device__ __forceinline__ bool poisson_term(double mu, double n, double &term, double &g) {
  if (mu > 0.0) {
    term = n > 0.0 ? __fma_rn(-n, log(mu), mu) : mu;
    g = 1.0 - n / mu;
    return isfinite(g);  // mu < n/DBL_MAX: the seed is not representable
  }
  term = 0.0;
  g = 1.0;
  return mu == 0.0 && n == 0.0;
}

// Pulls, parameter finiteness, final status and -ln L of toy t (thread 0).
__device__ void finish_nll(const ToyDev &T, const double *th, const double *pull_c, const double *pull_s,
                           double sum, bool bad, double *nll, uint32_t *status, int t) {
  uint32_t st = 0;
  for (int p = 0; p < T.P; p++)
    if (!isfinite(th[p])) st |= GS_ST_NONFINITE;
  if (bad) st |= GS_ST_DOMAIN;
  for (int p = 0; p < T.P; p++) {
    double s = pull_s[T.pull_off + p];
    if (s > 0.0) {
      double z = (th[p] - pull_c[T.pull_off + p]) / s;
      sum = __fma_rn(0.5 * z, z, sum);
    }
  }
  if (st & GS_ST_NONFINITE)
    sum = __builtin_nan("");
  else if (st & GS_ST_DOMAIN)
    sum = __builtin_inf();
  nll[t] = sum;
  status[t] = st;
}

__global__ __launch_bounds__(256) void k_nll1(const ToyDev *__restrict__ toys, const ShapeDev *__restrict__ shapes,
                                              const double *__restrict__ theta, int stride,
                                              const double *__restrict__ fpart, const double *__restrict__ cnt,
                                              const double *__restrict__ pull_c, const double *__restrict__ pull_s,
                                              const uint8_t *__restrict__ active, double *__restrict__ binrec,
                                              double *__restrict__ nll, uint32_t *__restrict__ status,
                                              double *__restrict__ mu_out) {
  __shared__ double lds[8];
  __shared__ int bad_s;
  const int t = blockIdx.x;
  if (active && !active[t]) return;
  const ToyDev &T = toys[t];
  const ShapeDev &Sh = shapes[T.shape];
  if (threadIdx.x == 0) bad_s = 0;
  __syncthreads();
  double sum = 0.0;
  bool bad = false;
  for (int b = threadIdx.x; b < T.L; b += blockDim.x) {
    const int j = T.lo + b;
    const double *bn = Sh.bins + (size_t)j * kBinLen;
    const double dx = bn[1];
    double s1 = 0.0;
    for (int c = 0; c < T.fold_chunks; c++) s1 += fpart[T.fpart_off + (long long)c * T.L + b];
    const double mu1 = dx * s1;
    double G = 0.0;
    for (int d = 0; d < T.D; d++) {
      const double mu = T.exposure[d] * mu1;
      const double n = cnt[T.cnt_off + (long long)d * T.L + b];
      double term, g;
      if (!poisson_term(mu, n, term, g)) bad = true;
      sum += term;
      G = __fma_rn(T.exposure[d], g, G);
      if (mu_out) mu_out[(long long)d * T.L + b] = mu;
    }
    if (Sh.family == kGammaPE && !(bn[0] > 0.0)) G = 0.0;
    double *br = binrec + (T.win_off + b) * kBinLen;
    br[0] = bn[0];
    br[1] = bn[2];
    br[2] = bn[3];
    br[3] = G * dx;
  }
  if (bad) bad_s = 1;  // benign race: every writer stores 1
  double tot = block_sum(sum, lds);
  __syncthreads();
  if (threadIdx.x == 0)
    finish_nll(T, theta + (size_t)t * stride, pull_c, pull_s, tot, bad_s != 0, nll, status, t);
}

hipError_t launch_nll1(const BatchView &v, const double *theta, double *nll, uint32_t *status, double *mu_out,
                       const uint8_t *active, hipStream_t st) {
  hipLaunchKernelGGL(k_nll1, dim3(v.n_toys), dim3(256), 0, st, v.toys, v.shapes, theta, v.stride, v.fpart, v.cnt,
                     v.pull_c, v.pull_s, active, v.binrec, nll, status, mu_out);
  return hipGetLastError();
}

// ------------------------------------------------------------- k_adj1 -----
template <int FAM>
__device__ __forceinline__ void adj_range(const double *__restrict__ rc, const double *__restrict__ BR, int b0,
                                          int b1, double &A0, double &A1, double &A2) {
  for (int b = b0; b < b1; b++) {
    const double *br = BR + (size_t)b * kBinLen;
    const double x = br[0], G = br[3];
    if (FAM == kGammaPE) {
      if (!(G != 0.0)) continue;  // wave-uniform: bin outside the gamma support
      double r = exp(gamma_exponent(rc[0], rc[1], rc[2], rc[3], rc[4], x, br[1], br[2]));
      double Gr = G * r;
      A0 += Gr;
      A1 = __fma_rn(Gr, br[1] - rc[6], A1);
      A2 = __fma_rn(Gr, x - rc[7], A2);
    } else {
      double z;
      double r = exp(gauss_exponent(rc[0], rc[1], rc[2], x, z));
      double Gr = G * r;
      double Grz = Gr * z;
      A0 += Gr;
      A1 += Grz;
      A2 = __fma_rn(Grz, z, A2);
    }
  }
}

__global__ __launch_bounds__(256) void k_adj1(const AdjItem *__restrict__ items, int n_items,
                                              const ToyDev *__restrict__ toys, const ShapeDev *__restrict__ shapes,
                                              const double *__restrict__ rec, const double *__restrict__ binrec,
                                              const uint8_t *__restrict__ active, double *__restrict__ apart) {
  const int w = wave_uniform((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (w >= n_items) return;
  const int lane = threadIdx.x & 63;
  const AdjItem it = items[w];
  if (active && !active[it.toy]) return;
  const ToyDev &T = toys[it.toy];
  const ShapeDev &Sh = shapes[T.shape];
  const int i = it.cell0 + lane;
  const bool valid = i < T.n_cell;
  const double *rp = rec + (T.cell_off + (valid ? i : T.n_cell - 1)) * kRecLen;
  double rc[kRecLen];
#pragma unroll
  for (int q = 0; q < kRecLen; q++) rc[q] = rp[q];
  const double *BR = binrec + T.win_off * kBinLen;
  double A0 = 0.0, A1 = 0.0, A2 = 0.0;
  if (Sh.family == kGammaPE)
    adj_range<kGammaPE>(rc, BR, it.bin0, it.bin1, A0, A1, A2);
  else
    adj_range<kGaussE>(rc, BR, it.bin0, it.bin1, A0, A1, A2);
  if (valid) {
    double *o = apart + T.apart_off + ((long long)it.chunk * T.n_cell + i) * 3;
    o[0] = A0;
    o[1] = A1;
    o[2] = A2;
  }
}

hipError_t launch_adj1(const BatchView &v, hipStream_t st) {
  if (v.n_adj_items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj1, dim3((v.n_adj_items + 3) / 4), dim3(256), 0, st, v.adj_items, v.n_adj_items, v.toys,
                     v.shapes, v.rec, v.binrec, (const uint8_t *)nullptr, v.apart);
  return hipGetLastError();
}

// ------------------------------------------------------------ k_grad1 -----
__global__ __launch_bounds__(256) void k_grad1(const ToyDev *__restrict__ toys, const ShapeDev *__restrict__ shapes,
                                               const double *__restrict__ theta, int stride,
                                               const double *__restrict__ rec, const double *__restrict__ apart,
                                               const double *__restrict__ pull_c, const double *__restrict__ pull_s,
                                               const uint32_t *__restrict__ status, const uint8_t *__restrict__ active,
                                               double *__restrict__ grad) {
  __shared__ double lds[8];
  __shared__ double res[GS_MAX_PARAMS];
  const int t = blockIdx.x;
  if (active && !active[t]) return;
  const ToyDev &T = toys[t];
  const ShapeDev &Sh = shapes[T.shape];
  const double *th = theta + (size_t)t * stride;
  const int fam = Sh.family, nr = fam == kGaussE ? 2 : 5;
  double gR[GS_MAX_SPECIES], gP[5];
#pragma unroll
  for (int s = 0; s < GS_MAX_SPECIES; s++) gR[s] = 0.0;
#pragma unroll
  for (int p = 0; p < 5; p++) gP[p] = 0.0;
  for (int i = threadIdx.x; i < Sh.n_cell; i += blockDim.x) {
    double A0 = 0.0, A1 = 0.0, A2 = 0.0;
    for (int c = 0; c < T.adj_chunks; c++) {
      const double *a = apart + T.apart_off + ((long long)c * T.n_cell + i) * 3;
      A0 += a[0];
      A1 += a[1];
      A2 += a[2];
    }
    Moments mo;
    moments(fam, th + Sh.S, Sh.birks_A, Sh.cellE[i], mo);
    const double *rc = rec + (T.cell_off + i) * kRecLen;
    double dNdm, dNds;
    if (fam == kGammaPE) {
      const double W = rc[5], m = mo.m, s = mo.s, s2 = s * s;
      const double k = m * m / s2, thg = s2 / m;
      const double dk = W * __fma_rn(log_minus_digamma(k), A0, A1);  // d(-ln L)/dk
      const double dth = W * A2 / (thg * thg);                       // d(-ln L)/dtheta
      dNdm = dk * (2.0 * m / s2) - dth * (s2 / (m * m));
      dNds = -dk * (2.0 * m * m / (s2 * s)) + dth * (2.0 * s / m);
    } else {
      const double W = rc[3], is = 1.0 / mo.s;
      dNdm = W * A1 * is;
      dNds = W * (A2 - A0) * is;
    }
#pragma unroll
    for (int p = 0; p < 5; p++) gP[p] = __fma_rn(dNdm, mo.dm[p], __fma_rn(dNds, mo.ds[p], gP[p]));
    if (i < Sh.n_true) {
      const double *w = Sh.wcell + (size_t)i * Sh.Sg;
#pragma unroll
      for (int s = 0; s < GS_MAX_SPECIES; s++)
        if (s < Sh.Sg) gR[s] = __fma_rn(w[s], A0, gR[s]);
    } else {
      const int q = Sh.Sg + (i - Sh.n_true);
#pragma unroll
      for (int s = 0; s < GS_MAX_SPECIES; s++)
        if (s == q) gR[s] += A0;
    }
  }
  for (int s = 0; s < Sh.S; s++) {
    double v = block_sum(gR[s], lds);
    if (threadIdx.x == 0) res[Sh.sp_of[s]] = v;
  }
  for (int p = 0; p < nr; p++) {
    double v = block_sum(gP[p], lds);
    if (threadIdx.x == 0) res[Sh.S + p] = v;
  }
  __syncthreads();
  if (threadIdx.x < stride) {
    const int p = threadIdx.x;
    double g = 0.0;
    if (p < T.P) {
      g = p < Sh.S + nr ? res[p] : 0.0;
      double s = pull_s[T.pull_off + p];
      if (s > 0.0) g += (th[p] - pull_c[T.pull_off + p]) / (s * s);
      if (status[t] & (GS_ST_DOMAIN | GS_ST_NONFINITE)) g = __builtin_nan("");
    }
    grad[(size_t)t * stride + p] = g;
  }
}

hipError_t launch_grad1(const BatchView &v, const double *theta, const uint32_t *status, double *grad,
                        const uint8_t *active, hipStream_t st) {
  hipLaunchKernelGGL(k_grad1, dim3(v.n_toys), dim3(256), 0, st, v.toys, v.shapes, theta, v.stride, v.rec, v.apart,
                     v.pull_c, v.pull_s, status, active, grad);
  return hipGetLastError();
}

// ------------------------------------------------------- bins setup -------
// Reco-bin constants of a shape: midpoint, width, ln(midpoint) as double-double.
__global__ void k_bins_setup(const double *__restrict__ edges, int n_reco, double *__restrict__ bins) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_reco) return;
  const double a = edges[j], b = edges[j + 1];
  const double x = (a + b) * 0.5;
  dd L = x > 0.0 ? dd_log(x) : dd{0.0, 0.0};
  double *o = bins + (size_t)j * kBinLen;
  o[0] = x;
  o[1] = b - a;
  o[2] = L.hi;
  o[3] = L.lo;
}

hipError_t launch_bins_setup(const ShapeDev *, double *bins, const double *edges, int n_reco, hipStream_t st) {
  hipLaunchKernelGGL(k_bins_setup, dim3((n_reco + 255) / 256), dim3(256), 0, st, edges, n_reco, bins);
  return hipGetLastError();
}

// ---------------------------------------------------- per-species fold ----
// F_js = dx_j sum_i w_si r_ji for every species (plain path cache, 2-D).
// Lanes are bins; grid cells add into Sg accumulators, line cells into their own.
template <int FAM>
__device__ __forceinline__ void folds_range(const double *__restrict__ R, const double *__restrict__ wc, int Sg,
                                            int n_true, int c0, int c1, double x, double Lh, double Ll,
                                            double (&acc)[GS_MAX_SPECIES]) {
  for (int i = c0; i < c1; i++) {
    const double *p = R + (size_t)i * kRecLen;
    double r;
    if (FAM == kGammaPE) {
      r = exp(gamma_exponent(p[0], p[1], p[2], p[3], p[4], x, Lh, Ll));
    } else {
      double z;
      r = exp(gauss_exponent(p[0], p[1], p[2], x, z));
    }
    if (i < n_true) {
      const double *w = wc + (size_t)i * Sg;
#pragma unroll
      for (int s = 0; s < GS_MAX_SPECIES; s++)
        if (s < Sg) acc[s] = __fma_rn(w[s], r, acc[s]);
    } else {
      const int q = Sg + (i - n_true);
#pragma unroll
      for (int s = 0; s < GS_MAX_SPECIES; s++)
        if (s == q) acc[s] += r;
    }
  }
}

__global__ __launch_bounds__(256) void k_foldS(const FoldItem *__restrict__ items, int n_items,
                                               const ToyDev *__restrict__ toys, const ShapeDev *__restrict__ shapes,
                                               const double *__restrict__ rec, const long long *__restrict__ fs_off,
                                               double *__restrict__ fspart) {
  const int w = wave_uniform((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (w >= n_items) return;
  const int lane = threadIdx.x & 63;
  const FoldItem it = items[w];
  const ToyDev &T = toys[it.toy];
  const ShapeDev &Sh = shapes[T.shape];
  const int b = it.bin0 + lane;
  const bool valid = b < T.L;
  const int j = T.lo + (valid ? b : T.L - 1);
  const double *bn = Sh.bins + (size_t)j * kBinLen;
  const double x = bn[0], Lh = bn[2], Ll = bn[3];
  const double *R = rec + T.cell_off * kRecLen;
  double acc[GS_MAX_SPECIES];
#pragma unroll
  for (int s = 0; s < GS_MAX_SPECIES; s++) acc[s] = 0.0;
  if (Sh.family == kGammaPE) {
    folds_range<kGammaPE>(R, Sh.wcell, Sh.Sg, Sh.n_true, it.cell0, it.cell1, x, Lh, Ll, acc);
    if (!(x > 0.0))
#pragma unroll
      for (int s = 0; s < GS_MAX_SPECIES; s++) acc[s] = 0.0;
  } else {
    folds_range<kGaussE>(R, Sh.wcell, Sh.Sg, Sh.n_true, it.cell0, it.cell1, x, Lh, Ll, acc);
  }
  if (valid) {
    double *o = fspart + fs_off[it.toy] + ((long long)it.chunk * T.L + b) * T.S;
#pragma unroll
    for (int s = 0; s < GS_MAX_SPECIES; s++)
      if (s < T.S) o[s] = acc[s];
  }
}

hipError_t launch_foldS(const BatchView &v, hipStream_t st) {
  if (v.n_fold_items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_foldS, dim3((v.n_fold_items + 3) / 4), dim3(256), 0, st, v.fold_items, v.n_fold_items,
                     v.toys, v.shapes, v.rec, v.fs_off, v.fspart);
  return hipGetLastError();
}

// F[(win_off + b) * S + s] = dx_b * sum over chunks (fixed order).
__global__ __launch_bounds__(256) void k_reduceF(const ToyDev *__restrict__ toys, const ShapeDev *__restrict__ shapes,
                                                 const long long *__restrict__ fs_off,
                                                 const double *__restrict__ fspart, double *__restrict__ F) {
  const int t = blockIdx.y;
  const ToyDev &T = toys[t];
  const ShapeDev &Sh = shapes[T.shape];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= T.L * T.S) return;
  const int b = e / T.S;
  double acc = 0.0;
  for (int c = 0; c < T.fold_chunks; c++) acc += fspart[fs_off[t] + (long long)c * T.L * T.S + e];
  F[T.win_off * T.S + e] = Sh.bins[(size_t)(T.lo + b) * kBinLen + 1] * acc;
}

// -ln L from cached per-species spectra: mu_dj = eps_d sum_s R_s F_js.
__global__ __launch_bounds__(256) void k_nllF(const ToyDev *__restrict__ toys, const ShapeDev *__restrict__ shapes,
                                              const double *__restrict__ theta, int stride, const double *__restrict__ F,
                                              const double *__restrict__ cnt, const double *__restrict__ pull_c,
                                              const double *__restrict__ pull_s, double *__restrict__ nll,
                                              uint32_t *__restrict__ status, double *__restrict__ mu_out) {
  __shared__ double lds[8];
  __shared__ int bad_s;
  const int t = blockIdx.x;
  const ToyDev &T = toys[t];
  const ShapeDev &Sh = shapes[T.shape];
  const double *th = theta + (size_t)t * stride;
  if (threadIdx.x == 0) bad_s = 0;
  __syncthreads();
  double sum = 0.0;
  bool bad = false;
  for (int b = threadIdx.x; b < T.L; b += blockDim.x) {
    const double *f = F + (T.win_off + b) * T.S;
    double mu1 = 0.0;
    for (int s = 0; s < Sh.S; s++) mu1 = __fma_rn(th[Sh.sp_of[s]], f[s], mu1);
    for (int d = 0; d < T.D; d++) {
      const double mu = T.exposure[d] * mu1;
      const double n = cnt[T.cnt_off + (long long)d * T.L + b];
      double term, g;
      if (!poisson_term(mu, n, term, g)) bad = true;
      sum += term;
      if (mu_out) mu_out[(long long)d * T.L + b] = mu;
    }
  }
  if (bad) bad_s = 1;
  double tot = block_sum(sum, lds);
  __syncthreads();
  if (threadIdx.x == 0) finish_nll(T, th, pull_c, pull_s, tot, bad_s != 0, nll, status, t);
}

hipError_t launch_nllF(const BatchView &v, const double *theta, double *nll, uint32_t *status, double *mu_out,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_nllF, dim3(v.n_toys), dim3(256), 0, st, v.toys, v.shapes, theta, v.stride, v.F, v.cnt,
                     v.pull_c, v.pull_s, nll, status, mu_out);
  return hipGetLastError();
}

hipError_t launch_reduceF_grid(const BatchView &v, int max_LS, hipStream_t st) {
  dim3 grid((max_LS + 255) / 256, v.n_toys);
  hipLaunchKernelGGL(k_reduceF, grid, dim3(256), 0, st, v.toys, v.shapes, v.fs_off, v.fspart, v.F);
  return hipGetLastError();
}

}  // namespace gs
