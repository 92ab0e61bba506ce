// gs_kernels.hip -- gfx950 kernels of the fold likelihood and its adjoint.
//
// One evaluation (section 2.5: the response on the visible x true mesh is
// evaluated and smeared against the true spectrum; Eq.2 cost ~ N_vis N_true):
//   k_cells     per (toy, cell): response moments, the per-cell record and the
//               cell's support: the reco bins whose midpoint log-density
//               exceeds log_cut (pairs outside it are skipped)
//   k_fold      per workgroup: 64 window bins (one per lane) x a cell range,
//               the 4 waves interleaving the cells; cell records and supports
//               are wave-uniform (scalar loads, scalar skip test), so the VALU
//               only does the per-pair exponent, one exp and the FMAs
//   k_bins1     per (toy, 256 window bins): split-K partials in fixed order,
//               Poisson terms of Eq.4, adjoint seeds G_j = dx_j sum_d eps_d
//               (1 - n_dj/mu_dj), block partial of -ln L
//   k_adj       per workgroup: 64 cells (one per lane) x the window bins inside
//               the union of their supports, the 4 waves interleaving the bins;
//               per-cell sums of G r {1, t1, t2}
//   k_cellgrad  per (toy, 256 cells): chain rule from per-cell sums to
//               d(-ln L)/d theta, block partials
//   k_finish    per toy: -ln L and gradient from the block partials, pulls,
//               status bits
// No floating-point atomics: every reduction has a fixed order, so results
// are bitwise reproducible for a fixed launch configuration.
#include <math.h>

#include "gs_impl.h"
#include "gs_support.h"
#include "gs_gen.h"

namespace gs {

// Coefficients of exp_tb, read through scalar loads so they live in SGPRs,
// and its table of 2^(j/256), which every pair kernel copies into LDS.
__constant__ double kExpC[GS_EXPT_NCOEF] = GS_EXPT_COEFS;
__constant__ double kExpTable[GS_EXPT_N] = GS_EXPT_TABLE;

// exp_tb's constants as the pair loops use them: the coefficients (scalar
// registers) plus the two that meet another scalar operand, copied once per
// thread into vector registers (the empty asm hides the copy from the
// optimiser, which would otherwise rematerialise it inside the loop), and the
// table in LDS.  exp_consts fills the table: every thread of the workgroup
// calls it first, before any return.
struct ExpK {
  const double *c, *tb;
  double c3, mg;
};
__device__ __forceinline__ ExpK exp_consts(double *stb) {
  for (int i = threadIdx.x; i < GS_EXPT_N; i += blockDim.x) stb[i] = kExpTable[i];
  __syncthreads();
  ExpK e{kExpC, stb, kExpC[0], kExpC[GS_EXPT_SHIFT]};
  asm volatile("" : "+v"(e.c3));
  asm volatile("" : "+v"(e.mg));
  return e;
}
__device__ __forceinline__ double dexp(double x, const ExpK &e) { return exp_tb(x, e.c, e.c3, e.tb, e.mg); }
// CLAMP = false: every argument is known to be finite and >= kExpTbNoClampMin.
template <bool CLAMP>
__device__ __forceinline__ double dexp(double x, const ExpK &e) {
  return CLAMP ? exp_tb(x, e.c, e.c3, e.tb, e.mg) : exp_tb_unclamped(x, e.c, e.c3, e.tb, e.mg);
}

// Whether a pair exponent E = Eref + A u + B v stays finite and at or above
// kExpTbNoClampMin over bins whose offsets run from (uf, vf) to (ul, vl) in
// increasing x.  E is concave in x or monotone on the bins in between (gamma
// with k >= 1: (k-1) ln x - x/th; k < 1: decreasing; Gaussian families: a
// downward parabola), so its minimum over them is at one of the two ends.
__device__ __forceinline__ bool exp_args_bounded(double A, double B, double Eref, double uf, double vf, double ul,
                                                 double vl) {
  return rel_exponent(A, B, Eref, uf, vf) >= kExpTbNoClampMin && rel_exponent(A, B, Eref, ul, vl) >= kExpTbNoClampMin;
}

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Toy handled by grid row b: every toy in order, or the b-th entry of a
// compacted list of toys (batched fits drop finished toys from the grids).
__device__ __forceinline__ int toy_of(const int *__restrict__ list, int b) { return list ? list[b] : b; }

// Workgroups are dispatched round-robin over the 8 XCDs; map block b to an
// item so that each XCD works through a contiguous, toy-major range of items
// and the cell records of one toy stay in one XCD's L2.
__device__ __forceinline__ int xcd_item(int b, int n) {
  const int per = (n + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}
inline int xcd_grid(int n) { return ((n + 7) >> 3) * 8; }

// Lane l's value of v at lane (l ^ o), through the LDS crossbar; addr = (l ^ o) * 4
// is formed once per butterfly step and shared by every value reduced in it.
__device__ __forceinline__ double xor_fetch(double v, int addr) {
  const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// Deterministic sum over a wavefront (xor butterfly); result valid on every lane.
__device__ __forceinline__ double wave_sum(double v) {
  const int lane = lane_id();
  for (int o = 32; o > 0; o >>= 1) v += xor_fetch(v, (lane ^ o) << 2);
  return v;
}

// The same for the first n of N values (n wave-uniform): the six butterfly
// addresses are formed once and shared.  G values go through the butterfly
// together (their exchanges in flight at once, for latency); G = 1 keeps only
// one value's partial sums live at a time (for registers).  Every value takes
// the same six steps in the same order whatever G is.
template <int N, int G = 1>
__device__ __forceinline__ void wave_sum_n(double (&v)[N], int n) {
  const int lane = lane_id();
  int addr[6];
#pragma unroll
  for (int k = 0; k < 6; k++) addr[k] = (lane ^ (32 >> k)) << 2;
#pragma unroll
  for (int q0 = 0; q0 < N; q0 += G)
    if (q0 < n) {
#pragma unroll
      for (int k = 0; k < 6; k++) {
        double f[G];
#pragma unroll
        for (int u = 0; u < G; u++)
          if (q0 + u < N && q0 + u < n) f[u] = xor_fetch(v[q0 + u], addr[k]);
#pragma unroll
        for (int u = 0; u < G; u++)
          if (q0 + u < N && q0 + u < n) v[q0 + u] += f[u];
      }
    }
}

// Deterministic sum over a block of kBlock threads; result valid on thread 0.
__device__ double block_sum(double v, double *lds) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); i++) r += lds[i];
  return r;
}

// ------------------------------------------------------------- k_cells ----
// Responses the FP64 pair evaluation resolves to the per-bin bound on bins of
// width up to w (gs.h states the range).  Measured against the oracle: the
// tile-relative Gaussian exponent cancels terms of relative size (w/s)^2
// (per-bin error 4e-13 at w/s = 4.8, 2e-12 at 10); an FP64 mean carries a
// density error of about 5e-16 m/s (Gaussian) and 1.2e-15 m/s (gamma, through
// its shape k = (m/s)^2); the gamma tile term grows with w m/s^2.  A cell
// outside the range whose response reaches the fit window refuses the
// evaluation.
constexpr double kAdmitGaussW = 4.5;      // s >= w / 4.5 (Gaussian families)
constexpr double kAdmitCondGauss = 600.0; // m <= 600 s (GAUSS_PE)
constexpr double kAdmitCondGamma = 300.0; // m <= 300 s (GAMMA_PE)
constexpr double kAdmitGammaW = 300.0;    // w m <= 300 s^2 (GAMMA_PE)
__device__ __forceinline__ bool admitted(int fam, double m, double s, double w) {
  if (fam == kGammaPE) return m <= kAdmitCondGamma * s && w * m <= kAdmitGammaW * s * s;
  if (fam == kGaussPE) return kAdmitGaussW * s >= w && m <= kAdmitCondGauss * s;
  return kAdmitGaussW * s >= w;
}

// Admitted range of the direct per-pair path (no tile-relative exponent, so no
// bin-width limit): the conditioning of a density on its FP64 mean, as for the
// fast path; the energy family's mean is the cell energy itself (no rounding).
__device__ __forceinline__ bool gen_admitted(int fam, double m, double s) {
  if (fam == kGaussE) return true;
  if (fam == kGammaPE || fam == kGenGammaPE || fam == kSPoisPE) return m <= kAdmitCondGamma * s;
  return m <= kAdmitCondGauss * s;
}

// Per-block flags of k_cells (cflag): an invalid response, a refused one.
constexpr uint32_t kCellInvalid = 1u, kCellUnresolved = 2u;

__device__ __forceinline__ void put_support(double *rc, int2 s) { *(int2 *)(rc + 6) = s; }
__device__ __forceinline__ int2 get_support(const double *rc) { return *(const int2 *)(rc + 6); }

// Entry (species s, window bin b) of a toy's per-species window array (F, H):
// rows of the toy's S species from fh_off.
__device__ __forceinline__ long long fh_at(const ToyDev &T, int s, int b) {
  return T.fh_off + (long long)b * T.S + s;
}

// GEN selects the shapes of the direct path (a launch of its own, so that the
// direct path's register use does not lower the fast path's occupancy).
template <bool GEN>
__global__ __launch_bounds__(64) void k_cells(const int *__restrict__ toy_list, const ToyDev *__restrict__ toys, const ShapeDev *__restrict__ shapes,
                                               const double *__restrict__ theta, int stride, double log_cut,
                                               const uint8_t *__restrict__ active, double *__restrict__ rec,
                                               int2 *__restrict__ sup, int2 *__restrict__ ghull,
                                               uint32_t *__restrict__ cflag) {
  const int t = toy_of(toy_list, blockIdx.y);
  if (active && !active[t]) return;
  const ToyDev &T = toys[t];
  if ((int)blockIdx.x >= T.cflag_blocks) return;
  const ShapeDev &Sh = shapes[T.shape];
  if ((Sh.gen != 0) != GEN) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool ok = true, unresolved = false;
  int hx = 0x7fffffff, hy = -1;  // this cell's contribution to its group's support hull
  if (i < Sh.n_cell) {
    const double *th = theta + (size_t)t * stride;
    Moments mo;
    ok = moments(Sh.family, th + Sh.S, Sh.birks_A, Sh.cellE[i], mo);
    double W = 0.0;
    if (i < Sh.n_true) {
      const double *w = Sh.wcellT + i;
#pragma unroll
      for (int s = 0; s < GS_MAX_SPECIES; s++)
        if (s < Sh.Sg) W = __fma_rn(th[Sh.sp_of[s]], w[(size_t)s * Sh.n_true], W);
    } else {
      W = th[Sh.sp_of[Sh.Sg + (i - Sh.n_true)]];
    }
    ok = ok && isfinite(W);
    double r[kRecLen];
    int2 sp;
    if constexpr (GEN) {  // direct path: {m, s, W, a, b, c, support, d} (GenCell constants)
      GenCell gc;
      ok = ok && gen_cell(Sh.family, Sh.shape, mo.m, mo.s, gc);
#pragma unroll
      for (int q = 0; q < kRecLen; q++) r[q] = 0.0;
      if (ok) {
        r[0] = gc.m;
        r[1] = gc.s;
        r[2] = W;
        r[3] = gc.a;
        r[4] = gc.b;
        r[5] = gc.c;
        r[7] = gc.d;
      }
      sp = ok ? gen_support(Sh.family, Sh.shape, gc, Sh.edges, Sh.n_reco, log_cut) : make_int2(0, 0);
      if (ok && sp.y > T.lo && sp.x < T.lo + T.L) unresolved = !gen_admitted(Sh.family, mo.m, mo.s);
    } else {
      cell_record(Sh.family, mo.m, mo.s, W, ok, r);
      const Span spn = cell_support(Sh.family, r, mo.m, mo.s, ok, Sh.bins, Sh.n_reco, Sh.bx0, Sh.bw, log_cut);
      sp = make_int2(spn.x, spn.y);
    }
    if (!GEN && ok && sp.y > T.lo && sp.x < T.lo + T.L) {  // the response reaches the window
      // the widths of the bins the response covers (the binning's width if uniform)
      double w = Sh.bw;
      if (!(w > 0.0)) {
        w = 0.0;
        for (int j = sp.x; j < sp.y; j++) {
          const double *bn = Sh.bins + (size_t)j * kBinLen;
          if (Sh.family != kGammaPE || bn[0] > 0.0) w = fmax(w, bn[1]);  // a gamma density is 0 at x <= 0
        }
      }
      unresolved = !admitted(Sh.family, mo.m, mo.s, w);
    }
    put_support(r, sp);
    double *rc = rec + (T.cell_off + i) * kRecLen;
#pragma unroll
    for (int q = 0; q < kRecLen; q++) rc[q] = r[q];
    sup[T.cell_off + i] = sp;
    if (i < Sh.n_true && sp.y > sp.x) {
      hx = sp.x;
      hy = sp.y;
    }
  }
  // hull of each aligned group of kGroup grid cells (lines are not included)
  for (int o = 1; o < kGroup; o <<= 1) {
    hx = min(hx, __shfl_xor(hx, o, 64));
    hy = max(hy, __shfl_xor(hy, o, 64));
  }
  if ((threadIdx.x & (kGroup - 1)) == 0 && i < Sh.n_true) ghull[T.ghull_off + i / kGroup] = make_int2(hx, hy);
  const int bad = __syncthreads_or(!ok), unres = __syncthreads_or(unresolved);
  if (threadIdx.x == 0) cflag[T.cflag_off + blockIdx.x] = (bad ? kCellInvalid : 0u) | (unres ? kCellUnresolved : 0u);
}

hipError_t launch_cells(const BatchView &v, const double *theta, const uint8_t *active, hipStream_t st) {
  dim3 grid(v.max_cflag_blocks, v.n_list);
  hipLaunchKernelGGL(k_cells<false>, grid, dim3(kCellBlock), 0, st, v.toy_list, v.toys, v.shapes, theta, v.stride, v.log_cut,
                     active, v.rec, v.sup, v.ghull, v.cflag);
  if (v.has_gen)
    hipLaunchKernelGGL(k_cells<true>, grid, dim3(kCellBlock), 0, st, v.toy_list, v.toys, v.shapes, theta, v.stride,
                       v.log_cut, active, v.rec, v.sup, v.ghull, v.cflag);
  return hipGetLastError();
}

// -------------------------------------------------------------- k_fold ----
// ------------------------------------------------------------ 1-D fold ----
// A workgroup owns kFoldTile1 = 32 window bins and a set of cells.  Each
// quarter-wave covers the whole tile, two bins per lane (bins j and j + 16 for
// lane j of the quarter), and the 16 quarter-waves of the workgroup take the
// cells in turn, so one LDS read of a cell (a broadcast to 16 lanes) feeds two
// pairs.  Narrow tiles keep the pairs evaluated outside the cells' supports
// (at the support ends of the cells that meet a tile) few.
//
// Tile-relative exponent (rel_cell, rel_offsets, rel_exponent): within a
// tile the log-density of a cell is written about a reference point xr of the
// tile (a bin midpoint) as E = Eref + A u + B v, with per-lane bin offsets
// (u, v) and per-cell staged values {A, B, Eref, W}.  Eref is evaluated once
// per cell and tile, in double-double for gamma (its terms of size k ln x
// cancel), so a pair costs two FMAs before the exponential.
struct Off2 {
  double u0, v0, u1, v1;  // offsets of the lane's two bins
};
struct TileRef {
  double x, Lh, Ll;  // reference midpoint and its logarithm (hi, lo)
};

// Reference point of the window bins [first, first + n) of a toy (clipped to
// the window, at least one bin): the middle bin, or the last one when the
// middle midpoint is not positive (the gamma density lives on x > 0).
__device__ __forceinline__ TileRef tile_ref(const ShapeDev &Sh, const ToyDev &T, int first, int n) {
  const int last = max(min(first + n, T.L) - 1, 0);
  const double *r = Sh.bins + (size_t)(T.lo + min(first + n / 2, last)) * kBinLen;
  if (Sh.family == kGammaPE && !(r[0] > 0.0)) r = Sh.bins + (size_t)(T.lo + last) * kBinLen;
  return {r[0], r[2], r[3]};
}

template <bool CLAMP>
__device__ __forceinline__ void fold_pair_ref(const double *__restrict__ p, const Off2 &o, const ExpK &ec, double &a0,
                                              double &a1) {
  a0 = __fma_rn(p[3], dexp<CLAMP>(rel_exponent(p[0], p[1], p[2], o.u0, o.v0), ec), a0);
  a1 = __fma_rn(p[3], dexp<CLAMP>(rel_exponent(p[0], p[1], p[2], o.u1, o.v1), ec), a1);
}

// Cell quads wave, wave + kWaves, ... of a staged batch of nb cells (nb a
// multiple of 4: a batch is padded with zero cells); quarter h of the wave
// takes the cell 4k + h of quad k.  A staged cell is 4 doubles.
template <bool CLAMP>
__device__ __forceinline__ void fold_batch(const double *srec, int nb, int wave, const Off2 &o, const ExpK &ec,
                                           double &a0, double &a1) {
  const int h = (threadIdx.x >> 4) & 3;
  const int nq = nb >> 2;
  const double *base = srec + h * 4;
  int k = wave;
  for (; k + kWaves < nq; k += 2 * kWaves) {
    const double2 p0 = *(const double2 *)(base + 16 * k), p1 = *(const double2 *)(base + 16 * k + 2);
    const double2 q0 = *(const double2 *)(base + 16 * (k + kWaves));
    const double2 q1 = *(const double2 *)(base + 16 * (k + kWaves) + 2);
    const double p[4] = {p0.x, p0.y, p1.x, p1.y}, q[4] = {q0.x, q0.y, q1.x, q1.y};
    fold_pair_ref<CLAMP>(p, o, ec, a0, a1);
    fold_pair_ref<CLAMP>(q, o, ec, a0, a1);
  }
  if (k < nq) {
    const double2 p0 = *(const double2 *)(base + 16 * k), p1 = *(const double2 *)(base + 16 * k + 2);
    const double p[4] = {p0.x, p0.y, p1.x, p1.y};
    fold_pair_ref<CLAMP>(p, o, ec, a0, a1);
  }
}

// The staged batch's pairs, through the unclamped exponential unless a cell
// staged into this workgroup so far may reach an exponent below
// kExpTbNoClampMin on the tile (the LDS flag set by stage_store, read after the
// barrier that follows staging, so the branch is uniform).
__device__ __forceinline__ void fold_batch_any(const double *srec, int nb, int wave, const Off2 &o, const ExpK &ec,
                                               const int *sclamp, double &a0, double &a1) {
  if (wave_uniform(*sclamp))
    fold_batch<true>(srec, nb, wave, o, ec, a0, a1);
  else
    fold_batch<false>(srec, nb, wave, o, ec, a0, a1);
}

// The record parts a staged cell is formed from (zeros for cell < 0: a zero
// record has weight 0).
template <int FAM>
__device__ __forceinline__ void stage_load(const double *__restrict__ R, int cell, double2 (&f)[3]) {
  f[0] = f[1] = f[2] = make_double2(0.0, 0.0);
  if (cell < 0) return;
  const double2 *r = (const double2 *)(R + (size_t)cell * kRecLen);
  f[0] = r[0];
  f[1] = r[1];
  if (FAM == kGammaPE) f[2] = r[2];
}

// Offsets of the tile's first and last bins (wave-uniform), for the check of
// the exponent's range at staging.
struct TileEnds {
  double uf, vf, ul, vl;
};
__device__ __forceinline__ double read_lane(double x, int l) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, l), hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Staged cell c = {A, B, Eref, W} about the tile's reference point.  Sets
// *sclamp when the cell's exponent may leave [kExpTbNoClampMin, inf) on the
// tile.
template <int FAM>
__device__ __forceinline__ void stage_store(double *srec, int c, const double2 (&f)[3], const TileRef &ref,
                                            const TileEnds &te, int *sclamp) {
  // record {k - 1, 1/th hi, lo, C hi, lo, W} (gamma) or {m, 1/s, c0, W}
  const double rc[6] = {f[0].x, f[0].y, f[1].x, f[1].y, f[2].x, f[2].y};
  const RelCell q = rel_cell(FAM, rc, ref.x, ref.Lh, ref.Ll);
  const double W = FAM == kGammaPE ? f[2].y : f[1].y;
  ((double2 *)srec)[2 * c] = make_double2(q.A, q.B);
  ((double2 *)srec)[2 * c + 1] = make_double2(q.Eref, W);
  if (!exp_args_bounded(q.A, q.B, q.Eref, te.uf, te.vf, te.ul, te.vl)) *sclamp = 1;  // every writer stores 1
}

// All cells of [c_lo, c_hi) against the tile (block-uniform range; every
// thread of the block calls this), kStage1 cells per batch, one per thread.
template <int FAM>
__device__ __forceinline__ void fold_range(const double *__restrict__ R, int c_lo, int c_hi, double *srec, int wave,
                                           const TileRef &ref, const TileEnds &te, int *sclamp, const Off2 &o,
                                           const ExpK &ec, double &a0, double &a1) {
  static_assert(kStage1 == kWaves * 64, "one staged cell per thread");
  const int tid = threadIdx.x;
  double2 f[3];
  if (c_lo < c_hi) stage_load<FAM>(R, c_lo + tid < c_hi ? c_lo + tid : -1, f);
  for (int base = c_lo; base < c_hi; base += kStage1) {
    const int nb = (min(kStage1, c_hi - base) + 3) & ~3;  // padded to whole cell quads
    __syncthreads();  // every wave is done with the previous batch
    if (tid < nb) stage_store<FAM>(srec, tid, f, ref, te, sclamp);
    __syncthreads();
    const int nxt = base + kStage1 + tid;
    if (base + kStage1 < c_hi) stage_load<FAM>(R, nxt < c_hi ? nxt : -1, f);
    fold_batch_any(srec, nb, wave, o, ec, sclamp, a0, a1);
  }
}

// Compacts, in increasing order, the groups g in [g0, g1) (at most one per
// thread) whose hull meets window bins [j0, j1) into list[]; returns their
// number (block-uniform; every thread of the block calls this).
__device__ __forceinline__ int group_list(const int2 *__restrict__ hull, int g0, int g1, int j0, int j1, int *list,
                                          int *cnt) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = g0 + (int)threadIdx.x;
  bool hit = false;
  if (g < g1) {
    const int2 h = hull[g];
    hit = h.x < j1 && h.y > j0;
  }
  const unsigned long long m = __ballot(hit);
  __syncthreads();  // list and cnt of a previous call are no longer read
  if (lane == 0) cnt[wave] = __popcll(m);
  __syncthreads();
  int off = 0;
  for (int w = 0; w < wave; w++) off += cnt[w];
  if (hit) list[off + __popcll(m & ((1ull << lane) - 1ull))] = g;
  __syncthreads();
  return cnt[0] + cnt[1] + cnt[2] + cnt[3];
}

// All cells of the listed groups, clipped to [c_lo, c_hi), against the tile.
// A batch holds kStage1 / kGroup groups; cells past the clip are staged as
// zero cells (weight 0).
template <int FAM>
__device__ __forceinline__ void fold_groups(const double *__restrict__ R, const int *list, int n_list, int c_lo,
                                            int c_hi, double *srec, int wave, const TileRef &ref, const TileEnds &te,
                                            int *sclamp, const Off2 &o, const ExpK &ec, double &a0, double &a1) {
  constexpr int kGPB = kStage1 / kGroup;
  const int tid = threadIdx.x;
  auto cell_of = [&](int bi) {
    const int li = bi * kGPB + tid / kGroup;
    const int cell = li < n_list ? list[li] * kGroup + tid % kGroup : -1;
    return cell >= c_lo && cell < c_hi ? cell : -1;
  };
  double2 f[3];
  const int n_batch = (n_list + kGPB - 1) / kGPB;
  if (n_batch > 0) stage_load<FAM>(R, cell_of(0), f);
  for (int bi = 0; bi < n_batch; bi++) {
    const int nb = min(kGPB, n_list - bi * kGPB) * kGroup;
    __syncthreads();  // every wave is done with the previous batch
    if (tid < nb) stage_store<FAM>(srec, tid, f, ref, te, sclamp);
    __syncthreads();
    if (bi + 1 < n_batch) stage_load<FAM>(R, cell_of(bi + 1), f);
    fold_batch_any(srec, nb, wave, o, ec, sclamp, a0, a1);
  }
}

__global__ __launch_bounds__(256, 6) void k_fold1(const FoldItem *__restrict__ items, int n_items,
                                               const ToyDev *__restrict__ toys, const ShapeDev *__restrict__ shapes,
                                               const double *__restrict__ rec, const int2 *__restrict__ ghull,
                                               const uint8_t *__restrict__ active, double *__restrict__ out) {
  __shared__ __align__(16) double srec[kStage1 * 4];
  __shared__ double red[kWaves * 4 * kFoldTile1];
  __shared__ int glist[kWaves * 64];
  __shared__ int gcnt[kWaves];
  __shared__ int sclamp;
  __shared__ double s_exp[GS_EXPT_N];
  const ExpK ec = exp_consts(s_exp);
  const int w_item = xcd_item(blockIdx.x, n_items);
  if (w_item >= n_items) return;
  const FoldItem it = items[w_item];
  if (active && !active[it.toy]) return;
  const ToyDev &T = toys[it.toy];
  if (T.two_d || T.gen) return;
  const ShapeDev &Sh = shapes[T.shape];
  // A gamma tile whose first bin lies at x <= 0 always takes the clamped
  // exponential: such a bin's offsets stand in for ln x = 0, so the exponent
  // there is not the concave function the end-bin check relies on.  The flag
  // is first read after the barriers of group_list or staging.
  if (threadIdx.x == 0)
    sclamp = Sh.family == kGammaPE && !(Sh.bins[(size_t)(T.lo + it.bin0) * kBinLen] > 0.0) ? 1 : 0;
  const int wave = wave_uniform(threadIdx.x >> 6), lane = threadIdx.x & 63;
  constexpr int kHalf = kFoldTile1 / 2;
  const bool gamma = Sh.family == kGammaPE;
  const int last = min(it.bin0 + kFoldTile1, T.L) - 1;  // last window bin of the tile
  const int b0 = it.bin0 + (lane & (kHalf - 1)), b1 = b0 + kHalf;
  const double *bp0 = Sh.bins + (size_t)(T.lo + min(b0, last)) * kBinLen;
  const double *bp1 = Sh.bins + (size_t)(T.lo + min(b1, last)) * kBinLen;
  const TileRef ref = tile_ref(Sh, T, it.bin0, kFoldTile1);
  Off2 o;
  rel_offsets(Sh.family, bp0[0], bp0[2], bp0[3], ref.x, ref.Lh, ref.Ll, o.u0, o.v0);
  rel_offsets(Sh.family, bp1[0], bp1[2], bp1[3], ref.x, ref.Lh, ref.Ll, o.u1, o.v1);
  // lane 0 holds the tile's first bin, lane kHalf - 1 its last (b1 clipped to last)
  const TileEnds te{read_lane(o.u0, 0), read_lane(o.v0, 0), read_lane(o.u1, kHalf - 1), read_lane(o.v1, kHalf - 1)};
  const int j0 = T.lo + it.bin0, j1 = T.lo + last + 1;
  const double *R = rec + T.cell_off * kRecLen;
  // grid cells: the groups whose hull meets the tile, up to kWaves * 64 groups per pass
  const int g_end = min(it.cell1, Sh.n_true);
  const int l_lo = max(it.cell0, Sh.n_true), l_hi = it.cell1;  // line cells: few, all evaluated
  double a0 = 0.0, a1 = 0.0;
  for (int gb = it.cell0 / kGroup; gb * kGroup < g_end; gb += kWaves * 64) {
    const int n = group_list(ghull + T.ghull_off, gb, min(gb + kWaves * 64, (g_end + kGroup - 1) / kGroup), j0, j1,
                             glist, gcnt);
    if (gamma)
      fold_groups<kGammaPE>(R, glist, n, it.cell0, g_end, srec, wave, ref, te, &sclamp, o, ec, a0, a1);
    else
      fold_groups<kGaussE>(R, glist, n, it.cell0, g_end, srec, wave, ref, te, &sclamp, o, ec, a0, a1);
  }
  if (gamma) {
    fold_range<kGammaPE>(R, l_lo, l_hi, srec, wave, ref, te, &sclamp, o, ec, a0, a1);
    if (!(bp0[0] > 0.0)) a0 = 0.0;  // outside the gamma support
    if (!(bp1[0] > 0.0)) a1 = 0.0;
  } else {
    fold_range<kGaussE>(R, l_lo, l_hi, srec, wave, ref, te, &sclamp, o, ec, a0, a1);
  }
  // red[stream][bin]: stream = wave * 4 + quarter, bin of the tile
  const int stream = threadIdx.x >> 4, j = lane & (kHalf - 1);
  red[stream * kFoldTile1 + j] = a0;
  red[stream * kFoldTile1 + kHalf + j] = a1;
  __syncthreads();
  if (threadIdx.x < kFoldTile1) {  // thread o: bin o of the tile, summed over the streams in a fixed order
    const int b = it.bin0 + (int)threadIdx.x;
    if (b < T.L) {
      double s = 0.0;
      for (int q = 0; q < kWaves * 4; q++) s += red[q * kFoldTile1 + threadIdx.x];
      out[T.fpart_off + (long long)it.chunk * T.L + b] = s;
    }
  }
}

// Per-species fold (plain path and the secondary-observable model):
// F_js = sum_i K_ji w_si, a dense contraction over the cells, runs on the FP64
// matrix cores.  A workgroup owns kFoldTile = 64 window bins and its 4 waves
// 16 bins each.  Per step the VALU forms the response of the wave's 16 bins x
// 4 cells, one pair per lane, as the A operand (lane l: bin l % 16, cell l / 16
// of the step).  v_mfma_f64_4x4x4f64 takes the A and B operands in the lane
// layouts of the 16x16x4 form but forms only the four diagonal 4 x 4 blocks of
// their product: lane l holds row 4 b + l / 16 and column 4 b + l % 4, with
// b = (l % 16) / 4 (layout checked on the device).  So a B operand that gives
// every column block the same four species g .. g + 3 (lane l: species
// 4 g + l % 4 of cell l / 16: w_si for a grid cell, one-hot on its own species
// for a line cell, zero for the padding of a staged batch) makes one
// instruction F[16 bins][4 species]: a grid cell of the pulse-shape model,
// which weighs 8 species, takes two instead of a 16x16x4 over 16 species
// columns, half of them zero.  The accumulator holds one register per group
// of four species.  Cells come from the compacted hull groups that meet the
// tile and are staged through LDS as in the 1-D fold, each with its
// tile-relative exponent about the reference point of either half-tile (the
// 32 bins that a 1-D fold tile spans): {A, Eref, B} of the lower half-tile,
// then of the upper one (A and B depend on the reference for the Gaussian
// families).
typedef double dbl4 __attribute__((ext_vector_type(4)));

// One staged batch of nb cells (a multiple of 4: padding slots hold zero
// weights) against the wave's 16 bins; sb: the staged records offset to the
// wave's half-tile (3 half), so that a cell's {A, Eref, B} sit at one address
// plus immediate offsets; ng: the groups of four species the batch's cells
// weigh (wave-uniform).
template <bool CLAMP>
__device__ __forceinline__ void folds_batch(const double *sb, const double *swt, int nb, int ng, double u, double v,
                                            const ExpK &ec, double (&acc)[GS_MAX_SPECIES / 4]) {
  const int lane = threadIdx.x & 63, kc = lane >> 4, q = lane & 3;
  for (int c4 = 0; c4 < nb; c4 += 4) {
    const double *r = sb + 6 * (c4 + kc);
    const double k = dexp<CLAMP>(rel_exponent(r[0], r[2], r[1], u, v), ec);
    const double *w = swt + (c4 + kc) * GS_MAX_SPECIES + q;
#pragma unroll
    for (int g = 0; g < GS_MAX_SPECIES / 4; g++)
      if (g < ng) acc[g] = __builtin_amdgcn_mfma_f64_4x4x4f64(k, w[4 * g], acc[g], 0, 0, 0);
  }
}

// Weight vector of cell i over the internal species (grid species, then lines).
__device__ __forceinline__ double cell_weight(const ShapeDev &Sh, int i, int q) {
  if (i < Sh.n_true) return q < Sh.Sg ? Sh.wcell[(size_t)i * Sh.Sg + q] : 0.0;
  return q == Sh.Sg + (i - Sh.n_true) ? 1.0 : 0.0;
}

// Cells of a staged batch: either the listed groups of grid cells (list !=
// NULL, clipped to [c_lo, c_hi)) or the cell range [c_lo, c_hi).  Thread t
// stages cell t % kStage against the reference point rh of its half-tile
// (t / kStage) and a share of the batch's species weights.  Nothing is
// prefetched across the MFMA loop, so it keeps few registers live: the staging
// loads' latency is hidden by the other workgroups on the compute unit.
template <int FAM>
__device__ __forceinline__ void folds_cells(const ShapeDev &Sh, const double *__restrict__ R, const int *list,
                                            int n_list, int c_lo, int c_hi, double *srec, double *swt,
                                            const TileRef &rh, const TileEnds &te, int *sclamp, double u,
                                            double v, const ExpK &ec, int ng, double (&acc)[GS_MAX_SPECIES / 4]) {
  static_assert(2 * kStage == kWaves * 64, "one staged cell and half-tile per thread");
  constexpr int kGPB = kStage / kGroup;
  const int tid = threadIdx.x, cs = tid % kStage, half = tid / kStage;
  auto cell_of = [&](int bi, int c) {  // cell at slot c of batch bi, or -1
    if (list) {
      const int li = bi * kGPB + c / kGroup;
      const int cell = li < n_list ? list[li] * kGroup + c % kGroup : -1;
      return cell >= c_lo && cell < c_hi ? cell : -1;
    }
    const int cell = c_lo + bi * kStage + c;
    return cell < c_hi ? cell : -1;
  };
  const int n_batch = list ? (n_list + kGPB - 1) / kGPB : (c_hi - c_lo + kStage - 1) / kStage;
  for (int bi = 0; bi < n_batch; bi++) {
    const int rem = list ? (n_list - bi * kGPB) * kGroup : c_hi - c_lo - bi * kStage;
    const int nb = (min(kStage, rem) + 3) & ~3;  // whole MFMA steps; padding slots carry zero weights
    double2 f[3];
    const int cell = cell_of(bi, cs);
    stage_load<FAM>(R, cell, f);
    // this thread's half of its cell's weights (species 8 half .. 8 half + 7)
    double2 wq[4];
    const double2 *wsrc = (const double2 *)(Sh.w16 + (size_t)max(cell, 0) * GS_MAX_SPECIES + 8 * half);
#pragma unroll
    for (int e = 0; e < 4; e++) wq[e] = cell >= 0 ? wsrc[e] : make_double2(0.0, 0.0);
    __syncthreads();  // every wave is done with the previous batch
    {
      // record {k - 1, 1/th hi, lo, C hi, lo, W} (gamma) or {m, 1/s, c0, W};
      // staged per half-tile as {A, Eref, B} at slots 3 half .. 3 half + 2
      const double rc[6] = {f[0].x, f[0].y, f[1].x, f[1].y, f[2].x, f[2].y};
      const RelCell q = rel_cell(FAM, rc, rh.x, rh.Lh, rh.Ll);
      double *o = srec + 6 * cs + 3 * half;
      o[0] = q.A;
      o[1] = q.Eref;
      o[2] = q.B;
      // a staged cell whose exponent may leave [kExpTbNoClampMin, inf) on its half-tile
      if (cell >= 0 && !exp_args_bounded(q.A, q.B, q.Eref, te.uf, te.vf, te.ul, te.vl)) *sclamp = 1;
    }
#pragma unroll
    for (int e = 0; e < 4; e++) ((double2 *)swt)[(cs * GS_MAX_SPECIES + 8 * half) / 2 + e] = wq[e];
    __syncthreads();
    const double *sb = srec + 3 * (int)(threadIdx.x >> 6 >> 1);
    if (*sclamp)
      folds_batch<true>(sb, swt, nb, ng, u, v, ec, acc);
    else
      folds_batch<false>(sb, swt, nb, ng, u, v, ec, acc);
  }
}

__global__ __launch_bounds__(256, 6) void k_fold_s(const FoldItem *__restrict__ items, int n_items,
                                                const ToyDev *__restrict__ toys, const ShapeDev *__restrict__ shapes,
                                                const double *__restrict__ rec, const int2 *__restrict__ ghull,
                                                int mode, const uint8_t *__restrict__ active,
                                                double *__restrict__ out) {
  __shared__ __align__(16) double srec[kStage * 6];
  __shared__ __align__(16) double swt[kStage * GS_MAX_SPECIES];
  __shared__ int glist[kWaves * 64];
  __shared__ int gcnt[kWaves];
  __shared__ int sclamp;
  __shared__ double s_exp[GS_EXPT_N];
  const ExpK ec = exp_consts(s_exp);
  const int w_item = xcd_item(blockIdx.x, n_items);
  if (w_item >= n_items) return;
  const FoldItem it = items[w_item];
  if (active && !active[it.toy]) return;
  const ToyDev &T = toys[it.toy];
  if ((mode >= 0 && T.two_d != mode) || T.gen) return;
  const ShapeDev &Sh = shapes[T.shape];
  const int wave = wave_uniform(threadIdx.x >> 6), lane = threadIdx.x & 63;
  // the lane's bin as a row of the A operand, clipped to the window
  const int b = it.bin0 + 16 * wave + (lane & 15);
  const double *bp = Sh.bins + (size_t)(T.lo + min(b, T.L - 1)) * kBinLen;
  // waves 0, 1 take the lower half-tile's reference point, waves 2, 3 the upper's; a thread
  // stages cells against the half-tile threadIdx.x / kStage (the same split)
  const int half = wave >> 1;
  const TileRef rh = tile_ref(Sh, T, it.bin0 + half * (kFoldTile / 2), kFoldTile / 2);
  double u, v;
  rel_offsets(Sh.family, bp[0], bp[2], bp[3], rh.x, rh.Lh, rh.Ll, u, v);
  // offsets of the half-tile's first and last window bins, for the staging's
  // range check; a gamma tile whose first bin lies at x <= 0 always clamps
  // (offsets there stand in for ln x = 0, so the exponent is not concave)
  TileEnds te;
  {
    const int fb = min(it.bin0 + half * (kFoldTile / 2), T.L - 1);
    const int lb = min(it.bin0 + half * (kFoldTile / 2) + kFoldTile / 2 - 1, T.L - 1);
    const double *bf = Sh.bins + (size_t)(T.lo + fb) * kBinLen, *bl = Sh.bins + (size_t)(T.lo + lb) * kBinLen;
    rel_offsets(Sh.family, bf[0], bf[2], bf[3], rh.x, rh.Lh, rh.Ll, te.uf, te.vf);
    rel_offsets(Sh.family, bl[0], bl[2], bl[3], rh.x, rh.Lh, rh.Ll, te.ul, te.vl);
    // wave-uniform: keep them in scalar registers
    te = {read_lane(te.uf, 0), read_lane(te.vf, 0), read_lane(te.ul, 0), read_lane(te.vl, 0)};
  }
  if (threadIdx.x == 0)
    sclamp = Sh.family == kGammaPE && !(Sh.bins[(size_t)(T.lo + it.bin0) * kBinLen] > 0.0) ? 1 : 0;
  const int j0 = T.lo + it.bin0, j1 = T.lo + min(it.bin0 + kFoldTile, T.L);
  const double *R = rec + T.cell_off * kRecLen;
  const int g_end = min(it.cell1, Sh.n_true);
  const int l_lo = max(it.cell0, Sh.n_true), l_hi = it.cell1;  // line cells: few, all evaluated
  const bool gamma = Sh.family == kGammaPE;
  double acc[GS_MAX_SPECIES / 4] = {0.0, 0.0, 0.0, 0.0};
  const int S = T.S, ngg = (Sh.Sg + 3) >> 2, ngl = (S + 3) >> 2;  // species groups of grid / line cells
  for (int gb = it.cell0 / kGroup; gb * kGroup < g_end; gb += kWaves * 64) {
    const int n = group_list(ghull + T.ghull_off, gb, min(gb + kWaves * 64, (g_end + kGroup - 1) / kGroup), j0, j1,
                             glist, gcnt);
    if (gamma)
      folds_cells<kGammaPE>(Sh, R, glist, n, it.cell0, g_end, srec, swt, rh, te, &sclamp, u, v, ec, ngg, acc);
    else
      folds_cells<kGaussE>(Sh, R, glist, n, it.cell0, g_end, srec, swt, rh, te, &sclamp, u, v, ec, ngg, acc);
  }
  if (gamma)
    folds_cells<kGammaPE>(Sh, R, nullptr, 0, l_lo, l_hi, srec, swt, rh, te, &sclamp, u, v, ec, ngl, acc);
  else
    folds_cells<kGaussE>(Sh, R, nullptr, 0, l_lo, l_hi, srec, swt, rh, te, &sclamp, u, v, ec, ngl, acc);
  // lane l, register g: bin 4 ((l % 16) / 4) + l / 16 of the wave's 16, species 4 g + l % 4
  const int bb = it.bin0 + 16 * wave + 4 * ((lane & 15) >> 2) + (lane >> 4);
  if (bb < T.L) {
    const bool outside = gamma && !(Sh.bins[(size_t)(T.lo + bb) * kBinLen] > 0.0);  // outside the gamma support
    double *o = out + T.fs_off + ((long long)it.chunk * T.L + bb) * S;
#pragma unroll
    for (int g = 0; g < GS_MAX_SPECIES / 4; g++) {
      const int sp = 4 * g + (lane & 3);
      if (sp < S) o[sp] = outside ? 0.0 : acc[g];
    }
  }
}

// ------------------------------------------------ direct per-pair fold ----
// Toys of the further response families, or with exact bin contents (gs_gen.h):
// each pair (window bin, cell) evaluates the bin content K_ji itself.  A
// workgroup takes one fold item: `tile` window bins, one per thread of a
// stream, against the item's cells dealt round-robin to the 256 / tile
// streams; the lanes of a stream read the same cell record (a broadcast) and
// skip a cell whose support misses their bin.  The partials are bin contents
// (no width factor): PS = false sums W_i K_ji into fpart, PS = true sums
// w_si K_ji per species into fspart; the streams are added in a fixed order.
template <bool PS>
__global__ __launch_bounds__(256) void k_foldg(const FoldItem *__restrict__ items, int n_items, int tile,
                                               const ToyDev *__restrict__ toys, const ShapeDev *__restrict__ shapes,
                                               const double *__restrict__ rec, const uint8_t *__restrict__ active,
                                               double *__restrict__ out) {
  constexpr int NQ = PS ? GS_MAX_SPECIES : 1;
  __shared__ double red[256 * NQ];
  const int w_item = xcd_item(blockIdx.x, n_items);
  if (w_item >= n_items) return;
  const FoldItem it = items[w_item];
  if (active && !active[it.toy]) return;
  const ToyDev &T = toys[it.toy];
  if (!T.gen) return;
  const ShapeDev &Sh = shapes[T.shape];
  const int nstream = 256 / tile, stream = threadIdx.x / tile, jb = threadIdx.x - stream * tile;
  const int b = it.bin0 + jb;
  const bool in = b < T.L;
  const int j = T.lo + min(b, T.L - 1);
  const double xlo = Sh.edges[j], xhi = Sh.edges[j + 1];
  const double xm = Sh.bins[(size_t)j * kBinLen], dx = Sh.bins[(size_t)j * kBinLen + 1];
  const int fam = Sh.family, S = T.S;
  const bool ex = Sh.exact != 0;
  const double p = Sh.shape;
  const GenChain ch{0.0, 0.0, 0.0, 0.0};  // no derivatives in the forward fold
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; q++) acc[q] = 0.0;
  const double *R = rec + T.cell_off * kRecLen;
  for (int i = it.cell0 + stream; i < it.cell1; i += nstream) {
    const double *rc = R + (size_t)i * kRecLen;
    const int2 sp = get_support(rc);
    if (!in || j < sp.x || j >= sp.y) continue;
    const GenCell g{rc[0], rc[1], rc[3], rc[4], rc[5], rc[7]};
    double K, d1, d2;
    if (ex) {
      const Edge lo = gen_edge(fam, p, g, ch, xlo, false), hi = gen_edge(fam, p, g, ch, xhi, false);
      K = edge_content(lo, hi, d1, d2);
    } else {
      K = dx * gen_density(fam, p, g, ch, xm, false, d1, d2);
    }
    if (PS) {
#pragma unroll
      for (int q = 0; q < NQ; q++)
        if (q < S) acc[q] = fma(cell_weight(Sh, i, q), K, acc[q]);
    } else {
      acc[0] = fma(rc[2], K, acc[0]);
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; q++) red[threadIdx.x * NQ + q] = acc[q];
  __syncthreads();
  if (stream != 0 || !in) return;
  if (PS) {
    for (int q = 0; q < S; q++) {
      double v = red[jb * NQ + q];
      for (int w = 1; w < nstream; w++) v += red[(w * tile + jb) * NQ + q];
      out[T.fs_off + ((long long)it.chunk * T.L + b) * S + q] = v;
    }
  } else {
    double v = red[jb];
    for (int w = 1; w < nstream; w++) v += red[w * tile + jb];
    out[T.fpart_off + (long long)it.chunk * T.L + b] = v;
  }
}

hipError_t launch_fold(const BatchView &v, bool per_species, int mode, const uint8_t *active, hipStream_t st) {
  if (per_species) {
    // the per-species fold serves the 2-D toys, or every toy (plain path)
    const FoldItem *it = mode == kOnly2D ? v.fold2 : v.fold_items;
    const int n = mode == kOnly2D ? v.n_fold2 : mode == kOnly1D ? v.n_fold1s : v.n_fold_items;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fold_s, dim3(xcd_grid(n)), dim3(kWaves * 64), 0, st, it, n, v.toys, v.shapes, v.rec,
                       v.ghull, mode, active, v.fspart);
    if (v.has_gen && mode != kOnly2D)
      hipLaunchKernelGGL(k_foldg<true>, dim3(xcd_grid(n)), dim3(256), 0, st, it, n, kFoldTile, v.toys, v.shapes,
                         v.rec, active, v.fspart);
  } else {
    if (v.n_fold1 == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fold1, dim3(xcd_grid(v.n_fold1)), dim3(kWaves * 64), 0, st, v.fold1, v.n_fold1, v.toys,
                       v.shapes, v.rec, v.ghull, active, v.fpart);
    if (v.has_gen)
      hipLaunchKernelGGL(k_foldg<false>, dim3(xcd_grid(v.n_fold1)), dim3(256), 0, st, v.fold1, v.n_fold1, kFoldTile1,
                         v.toys, v.shapes, v.rec, active, v.fpart);
  }
  return hipGetLastError();
}

// -------------------------------------------- adjoint block references ---
// The adjoint evaluates a cell's log-density relative to a reference point
// per block of kABlock window bins (as the 1-D fold does per tile):
// E(x) = E(xr) + (k - 1) u + (-1/th) v with u = ln x - ln xr, v = x - xr.
// The bin offsets (u, v) go into the window-bin record (slots 6, 7) and the
// reference itself into the block's row of bref; E(xr) is formed per cell
// and block in double-double.  The reference is the block's middle bin, or
// its last bin when that midpoint is not positive (the gamma density lives
// on x > 0).
__device__ __forceinline__ const double *block_ref(const ShapeDev &Sh, const ToyDev &T, int q) {
  const int last = min((q + 1) * kABlock, T.L) - 1;
  const double *r = Sh.bins + (size_t)(T.lo + min(q * kABlock + kABlock / 2, last)) * kBinLen;
  if (Sh.family == kGammaPE && !(r[0] > 0.0)) r = Sh.bins + (size_t)(T.lo + last) * kBinLen;
  return r;
}

// Offsets (u, v) of window bin b (shape bin record bn) from its block's
// reference; the block's first bin also writes the block's bref row.  A bin
// at x <= 0 (outside the gamma support, zero seed) gets v = 1e300: with
// B = -1/th < 0 its exponent is far below -1000, so the clamped exponential
// gives exactly 0 and the zero seed adds exactly zero (an exponent from the
// ln x = 0 stand-in alone can overflow, and 0 * inf is NaN).
__device__ __forceinline__ void block_offsets(const ShapeDev &Sh, const ToyDev &T, int b, const double *bn, double &u,
                                              double &v, double *__restrict__ bref) {
  const double *r = block_ref(Sh, T, b / kABlock);
  rel_offsets(kGammaPE, bn[0], bn[2], bn[3], r[0], r[2], r[3], u, v);
  if (!(bn[0] > 0.0)) v = 1e300;
  if (b % kABlock == 0) {
    double *o = bref + (T.bref_off + b / kABlock) * 4;
    o[0] = r[0];
    o[1] = r[2];
    o[2] = r[3];
    o[3] = 0.0;
  }
}

// ------------------------------------------------------------- k_bins1 ----
// Poisson term of Eq.4 (ln n! dropped) and the adjoint seed g = 1 - n/mu.
// Returns a flag: 0, kBadDomain (mu < 0, or mu = 0 with n > 0: no term), or
// kBadRange (n > 0 with n/mu above DBL_MAX: the term is finite, the seed has
// no FP64 value and is returned as 0).
constexpr uint32_t kBadDomain = 1u, kBadRange = 2u;
__device__ __forceinline__ uint32_t poisson_term(double mu, double n, double &term, double &g) {
  if (mu > 0.0) {
    term = n > 0.0 ? __fma_rn(-n, log(mu), mu) : mu;
    g = 1.0 - n / mu;
    if (isfinite(g)) return 0u;
    g = 0.0;
    return kBadRange;
  }
  term = 0.0;
  g = 1.0;
  return mu == 0.0 && n == 0.0 ? 0u : kBadDomain;
}

__global__ __launch_bounds__(256) void k_bins1(const int *__restrict__ toy_list, const ToyDev *__restrict__ toys, const ShapeDev *__restrict__ shapes,
                                               const double *__restrict__ fpart, const double *__restrict__ cnt,
                                               const uint8_t *__restrict__ active, double *__restrict__ binrec,
                                               double *__restrict__ bref, double *__restrict__ nllp,
                                               uint32_t *__restrict__ badp, double *__restrict__ mu_out) {
  __shared__ double lds[8];
  __shared__ uint32_t bad_s;
  const int t = toy_of(toy_list, blockIdx.y);
  if (active && !active[t]) return;
  const ToyDev &T = toys[t];
  if ((int)blockIdx.x >= T.bin_blocks || T.two_d || T.tmpl) return;
  const ShapeDev &Sh = shapes[T.shape];
  if (threadIdx.x == 0) bad_s = 0u;
  __syncthreads();
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  double sum = 0.0;
  if (b < T.L) {
    const int j = T.lo + b;
    const double *bn = Sh.bins + (size_t)j * kBinLen;
    const double dx = bn[1];
    const double *fp = fpart + T.fpart_off + b;
    double s1 = 0.0;
    int c = 0;
    for (; c + 8 <= T.fold_chunks; c += 8) {  // eight chunks' loads before their adds (in chunk order)
      double pv[8];
#pragma unroll
      for (int u = 0; u < 8; u++) pv[u] = fp[(long long)(c + u) * T.L];
#pragma unroll
      for (int u = 0; u < 8; u++) s1 += pv[u];
    }
    for (; c < T.fold_chunks; c++) s1 += fp[(long long)c * T.L];
    const double mu1 = T.gen ? s1 : dx * s1;  // the direct path's partials are bin contents already
    double G = 0.0;
    uint32_t bad = 0u;
    for (int d = 0; d < T.D; d++) {
      const double mu = T.exposure[d] * mu1;
      const double n = cnt[T.cnt_off + (long long)d * T.L + b];
      double term, g;
      bad |= poisson_term(mu, n, term, g);
      sum += term;
      G = __fma_rn(T.exposure[d], g, G);
      if (mu_out) mu_out[(long long)d * T.L + b] = mu;
    }
    if (Sh.family == kGammaPE && !T.gen && !(bn[0] > 0.0)) G = 0.0;
    double *br = binrec + (T.win_off + b) * kBinRecLen;
    const double Gd = T.gen ? G : G * dx;
    br[0] = bn[0];
    br[1] = bn[2];
    br[2] = bn[3];
    br[3] = Gd;
    br[4] = Gd * bn[2];
    br[5] = Gd * bn[0];
    block_offsets(Sh, T, b, bn, br[6], br[7], bref);
    if (bad) atomicOr(&bad_s, bad);
  }
  const double tot = block_sum(sum, lds);
  __syncthreads();
  if (threadIdx.x == 0) {
    nllp[T.nllp_off + blockIdx.x] = tot;
    badp[T.nllp_off + blockIdx.x] = bad_s;
  }
}

hipError_t launch_bins1(const BatchView &v, double *mu_out, const uint8_t *active, hipStream_t st) {
  if (v.n1d == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bins1, dim3(v.max_bin_blocks1, v.n1d), dim3(kBlock), 0, st, v.list1d, v.toys, v.shapes, v.fpart,
                     v.cnt, active, v.binrec, v.bref, v.nllp, v.badp, mu_out);
  return hipGetLastError();
}

// --------------------------------------------------------------- k_adj ----
// Per-cell sums over window bins of Gr = G_j r_ji times {1, t1, t2}:
//  gamma:    t1 = ln x_j, t2 = x_j (shifted by ln m and m in k_cellgrad)
//  gaussian: t1 = z_ji, t2 = z_ji^2 with z = (x - m)/s
// When NW waves share an item, wave w takes the bins b0 + w, b0 + w + NW, ...
// of [b0, b1); a wave with an item of its own (NW = 1) takes them all.  A
// gamma cell's exponent is formed per kABlock block about the block's
// reference point (see block_ref).
// Reference exponents E(x_r) of a lane's gamma cell for the bin blocks
// [qa, qb) (at most kRefBlocks), formed once per cell and block: wave w takes
// the blocks qa + w, qa + w + NW, ... of the NW waves and the workgroup shares
// them through LDS.  Every thread of the workgroup calls this.
template <int NW>
__device__ __forceinline__ void stage_refs(const double *__restrict__ rc, const double *__restrict__ BF, int qa, int qb,
                                           int wave, double (*sref)[kTile]) {
  const int lane = threadIdx.x & 63;
  __syncthreads();  // the previous round's rows are no longer read
  for (int q = qa + wave; q < qb; q += NW) {
    const double *r = BF + (size_t)q * 4;
    sref[q - qa][lane] = rel_cell(kGammaPE, rc, r[0], r[1], r[2]).Eref;
  }
  __syncthreads();
}

// A lane's gamma cell against the bins b, b + NW, ... of [b, hi) within one
// kABlock block (Eref formed about the block's reference point).  A zero seed
// adds exactly zero, so there is no test per bin; a bin outside the gamma
// support (x <= 0) has a zero seed and offsets whose exponent underflows (see
// block_offsets), and a block holding one takes the clamped exponential.
template <bool CLAMP, int NW>
__device__ __forceinline__ void adj_block(const double *__restrict__ BR, int b, int hi, double A, double B, double Eref,
                                          const ExpK &ec, double &A0, double &A1, double &A2) {
  for (; b + NW < hi; b += 2 * NW) {
    // bin record: x, ln x (hi, lo), G, G ln x, G x, u, v
    const double *p = BR + (size_t)b * kBinRecLen, *p2 = p + NW * kBinRecLen;
    const double r0 = dexp<CLAMP>(rel_exponent(A, B, Eref, p[6], p[7]), ec);
    const double r1 = dexp<CLAMP>(rel_exponent(A, B, Eref, p2[6], p2[7]), ec);
    A0 = __fma_rn(p[3], r0, A0);
    A1 = __fma_rn(p[4], r0, A1);
    A2 = __fma_rn(p[5], r0, A2);
    A0 = __fma_rn(p2[3], r1, A0);
    A1 = __fma_rn(p2[4], r1, A1);
    A2 = __fma_rn(p2[5], r1, A2);
  }
  if (b < hi) {
    const double *p = BR + (size_t)b * kBinRecLen;
    const double r0 = dexp<CLAMP>(rel_exponent(A, B, Eref, p[6], p[7]), ec);
    A0 = __fma_rn(p[3], r0, A0);
    A1 = __fma_rn(p[4], r0, A1);
    A2 = __fma_rn(p[5], r0, A2);
  }
}

// Whether any lane's gamma exponent may leave [kExpTbNoClampMin, inf) on the
// bins [lo, hi) of a block (wave-uniform): checked at the two end bins.  A
// block starting at x <= 0 always needs the clamp: offsets there stand in for
// ln x = 0, so the exponent at that end is not the concave function.
__device__ __forceinline__ bool block_needs_clamp(const double *__restrict__ BR, int lo, int hi, double A, double B,
                                                  double Eref) {
  const double *pl = BR + (size_t)lo * kBinRecLen, *ph = BR + (size_t)(hi - 1) * kBinRecLen;
  if (!(pl[0] > 0.0)) return true;
  return __ballot(!exp_args_bounded(A, B, Eref, pl[6], pl[7], ph[6], ph[7])) != 0ull;
}

template <int FAM, int NW>
__device__ __forceinline__ void adj_bins(const double *__restrict__ rc, const double *__restrict__ BR,
                                         const double *__restrict__ BF, int b0, int b1, int wave, const ExpK &ec,
                                         double (*sref)[kTile], double &A0, double &A1, double &A2) {
  if (b0 >= b1) return;
  if (FAM == kGammaPE) {
    const int lane = threadIdx.x & 63;
    const double A = rc[0], B = -rc[1];
    const int q_end = (b1 + kABlock - 1) / kABlock;
    for (int qa = b0 / kABlock; qa < q_end; qa += kRefBlocks) {
      const int qb = min(qa + kRefBlocks, q_end);
      if (NW > 1) stage_refs<NW>(rc, BF, qa, qb, wave, sref);
      for (int q = qa; q < qb; q++) {
        const int lo = max(b0, q * kABlock), hi = min(b1, (q + 1) * kABlock);
        int b = lo + ((b0 + wave - lo) & (NW - 1));  // first bin of this wave in the block
        if (b >= hi) continue;
        double Eref;
        if (NW > 1) {
          Eref = sref[q - qa][lane];
        } else {  // a wave on its own forms its references itself
          const double *r = BF + (size_t)q * 4;
          Eref = rel_cell(kGammaPE, rc, r[0], r[1], r[2]).Eref;
        }
        if (block_needs_clamp(BR, lo, hi, A, B, Eref))
          adj_block<true, NW>(BR, b, hi, A, B, Eref, ec, A0, A1, A2);
        else
          adj_block<false, NW>(BR, b, hi, A, B, Eref, ec, A0, A1, A2);
      }
    }
    return;
  }
  const double *br = BR + (size_t)(b0 + wave) * kBinRecLen;
  double x = br[0], G = br[3];
  for (int b = b0 + wave; b < b1; b += NW) {
    const double *bn = BR + (size_t)min(b + NW, b1 - 1) * kBinRecLen;  // next bin, fetched early
    const double nx = bn[0], nG = bn[3];
    double z;
    const double Gr = G * dexp(gauss_exponent(rc[0], rc[1], rc[2], x, z), ec);
    const double Grz = Gr * z;
    A0 += Gr;
    A1 += Grz;
    A2 = __fma_rn(Grz, z, A2);
    x = nx;
    G = nG;
  }
}

// NW = kWaves waves of a workgroup share one item (interleaving its bins), or,
// for NW = 1, each of the kAdjGroupWaves waves takes an item of its own and
// walks all of its bins (no LDS and no barrier).
template <int NW>
__global__ __launch_bounds__((NW > 1 ? kWaves : kAdjGroupWaves) * 64) void k_adj(const AdjItem *__restrict__ items, int n_items,
                                             const ToyDev *__restrict__ toys, const ShapeDev *__restrict__ shapes,
                                             const double *__restrict__ rec, const double *__restrict__ binrec,
                                             const double *__restrict__ bref, const uint8_t *__restrict__ active,
                                             double *__restrict__ apart) {
  __shared__ double red[NW * kTile * 3];
  __shared__ double sref[NW > 1 ? kRefBlocks : 1][kTile];
  __shared__ double s_exp[GS_EXPT_N];
  const ExpK ec = exp_consts(s_exp);
  const int lane = threadIdx.x & 63;
  const int w_item = NW > 1 ? xcd_item(blockIdx.x, n_items)
                            : xcd_item(blockIdx.x, (n_items + kAdjGroupWaves - 1) / kAdjGroupWaves) * kAdjGroupWaves +
                                  wave_uniform(threadIdx.x >> 6);
  if (w_item >= n_items) return;
  const AdjItem it = items[w_item];
  if (active && !active[it.toy]) return;
  const int wave = NW > 1 ? wave_uniform(threadIdx.x >> 6) : 0;  // this wave's place within its item
  const ToyDev &T = toys[it.toy];
  if (T.two_d || T.gen) return;
  const ShapeDev &Sh = shapes[T.shape];
  const int i = it.cell0 + lane;
  const bool valid = i < T.n_cell;
  const int ic = valid ? i : T.n_cell - 1;
  const double *rp = rec + (T.cell_off + ic) * kRecLen;
  double rc[kRecLen];
#pragma unroll
  for (int q = 0; q < kRecLen; q++) rc[q] = rp[q];
  // union of the 64 cells' supports, as window-relative bins, clipped to the chunk
  const int2 s = get_support(rc);
  int lo = valid ? s.x : 0x7fffffff, hi = valid ? s.y : -1;
  for (int o = 32; o > 0; o >>= 1) {
    lo = min(lo, __shfl_xor(lo, o, 64));
    hi = max(hi, __shfl_xor(hi, o, 64));
  }
  const int b0 = max(it.bin0, wave_uniform(lo) - T.lo), b1 = min(it.bin1, wave_uniform(hi) - T.lo);
  const double *BR = binrec + T.win_off * kBinRecLen, *BF = bref + T.bref_off * 4;
  double A0 = 0.0, A1 = 0.0, A2 = 0.0;
  if (Sh.family == kGammaPE)
    adj_bins<kGammaPE, NW>(rc, BR, BF, b0, b1, wave, ec, sref, A0, A1, A2);
  else
    adj_bins<kGaussE, NW>(rc, BR, BF, b0, b1, wave, ec, sref, A0, A1, A2);
  if (NW == 1) {
    if (valid) {
      double *o = apart + T.apart_off + ((long long)it.chunk * T.n_cell + i) * 3;
      o[0] = A0;
      o[1] = A1;
      o[2] = A2;
    }
    return;
  }
  red[(wave * 3 + 0) * kTile + lane] = A0;
  red[(wave * 3 + 1) * kTile + lane] = A1;
  red[(wave * 3 + 2) * kTile + lane] = A2;
  __syncthreads();
  if (wave == 0 && valid) {
    double *o = apart + T.apart_off + ((long long)it.chunk * T.n_cell + i) * 3;
    for (int q = 0; q < 3; q++) {
      double v = red[q * kTile + lane];
      for (int ww = 1; ww < NW; ww++) v += red[(ww * 3 + q) * kTile + lane];
      o[q] = v;
    }
  }
}

// ---------------------------------------------------- per-species adjoint --
// Secondary-observable toys: the seed of pair (j, i) is
// Z_ji = sum_s H_js R_s w_si (H_js = dx_j sum_k P_sk Gam_jk, from k_bins2), a
// dense contraction over the species that runs on the FP64 matrix cores.  A
// workgroup takes an adjoint item (64 cells x a window-bin range) and each of
// its 4 waves 16 of the cells; a wave walks the union of its cells' supports
// in steps of 16 bins.  Per step, v_mfma_f64_16x16x4f64 forms Z for 16 bins x
// 16 cells from H (A operand, lane l: bin l % 16, species 4 k + l / 16) and
// R_s w_si (B operand, lane l: species 4 k + l / 16, cell l % 16; held in
// registers), k over the species in fours.  Lane l then holds Z for its cell
// l % 16 at the bins l / 16 + 4 v (v = 0..3), evaluates those four pairs'
// responses on the VALU and adds Z r {1, ln x, x} (gamma) or Z r {1, z, z^2}
// (Gaussian) to its cell's sums; the four lanes of a cell are combined at the
// end.  A gamma cell's exponent is formed about the reference point of each
// kABlock-bin block (as in the 1-D adjoint); bins outside the walked range
// carry a zero seed.
// One step of the walk: 16 bins from jb against the wave's 16 cells.  The
// lane's four bin records (bins jb + grp + 4 v; rows past the window are
// zero padding, and their Z is zero) are loaded before the contraction, so
// their latency overlaps the MFMA chain.
template <int FAM>
__device__ __forceinline__ void adj_s_walk(const double *__restrict__ BR, const double *__restrict__ BF,
                                           const double *__restrict__ HR, int S, int nk, int b0, int b1,
                                           const double (&rc)[kRecLen], const double (&rwk)[4], const ExpK &ec,
                                           double &A0, double &A1, double &A2) {
  const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
  double Eref = 0.0;
  int qref = -1;
  for (int jb = b0 & ~15; jb < b1; jb += 16) {
    const double *br = BR + (size_t)(jb + grp) * kBinRecLen;
    double2 xl[4], uv[4];
#pragma unroll
    for (int v = 0; v < 4; v++) {
      xl[v] = *(const double2 *)(br + 4 * v * kBinRecLen);  // x, ln x (hi)
      if (FAM == kGammaPE) uv[v] = *(const double2 *)(br + 4 * v * kBinRecLen + 6);  // block offsets u, v
    }
    const int ja = jb + col;  // the A operand's bin
    const bool in = ja >= b0 && ja < b1;
    dbl4 Z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 4; k++)
      if (k < nk) {
        const int s4 = 4 * k + grp;
        const double h = in && s4 < S ? HR[(size_t)ja * S + s4] : 0.0;
        Z = __builtin_amdgcn_mfma_f64_16x16x4f64(h, rwk[k], Z, 0, 0, 0);
      }
    if (FAM == kGammaPE && jb / kABlock != qref) {  // a 16-bin step lies inside one reference block
      qref = jb / kABlock;
      const double *r = BF + (size_t)qref * 4;
      Eref = rel_cell(kGammaPE, rc, r[0], r[1], r[2]).Eref;
    }
#pragma unroll
    for (int v = 0; v < 4; v++) {
      if (FAM == kGammaPE) {
        const double Gr = Z[v] * dexp(rel_exponent(rc[0], -rc[1], Eref, uv[v].x, uv[v].y), ec);
        A0 += Gr;
        A1 = __fma_rn(Gr, xl[v].y, A1);
        A2 = __fma_rn(Gr, xl[v].x, A2);
      } else {
        double z;
        const double Gr = Z[v] * dexp(gauss_exponent(rc[0], rc[1], rc[2], xl[v].x, z), ec);
        const double Grz = Gr * z;
        A0 += Gr;
        A1 += Grz;
        A2 = __fma_rn(Grz, z, A2);
      }
    }
  }
}

__global__ __launch_bounds__(kWaves * 64) void k_adj_s(const AdjItem *__restrict__ items, int n_items,
                                                       const ToyDev *__restrict__ toys,
                                                       const ShapeDev *__restrict__ shapes,
                                                       const double *__restrict__ theta, int stride,
                                                       const double *__restrict__ rec,
                                                       const double *__restrict__ binrec,
                                                       const double *__restrict__ bref, const double *__restrict__ H,
                                                       const uint8_t *__restrict__ active,
                                                       double *__restrict__ apart) {
  __shared__ double s_exp[GS_EXPT_N];
  const ExpK ec = exp_consts(s_exp);
  const int w_item = xcd_item(blockIdx.x, n_items);
  if (w_item >= n_items) return;
  const AdjItem it = items[w_item];
  if (active && !active[it.toy]) return;
  const ToyDev &T = toys[it.toy];
  if (!T.two_d) return;
  const ShapeDev &Sh = shapes[T.shape];
  const int wave = wave_uniform(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  const int c0 = it.cell0 + 16 * wave;  // the wave's first cell
  const int i = c0 + col;               // the lane's cell
  const bool valid = i < T.n_cell;
  const int ic = valid ? i : T.n_cell - 1;
  const double *rp = rec + (T.cell_off + ic) * kRecLen;
  double rc[kRecLen];
#pragma unroll
  for (int q = 0; q < kRecLen; q++) rc[q] = rp[q];
  // B operand: R_s w_si of the lane's cell for the species 4 k + grp; grid
  // cells weigh only the grid species, a line cell its own species alone
  const double *th = theta + (size_t)it.toy * stride;
  const int nq = c0 + 16 <= Sh.n_true ? Sh.Sg : T.S;
  const int nk = (nq + 3) >> 2;
  double rwk[4];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int sp = 4 * k + grp;
    double w = 0.0;
    if (valid && sp < T.S) {
      if (ic < Sh.n_true)
        w = sp < Sh.Sg ? th[Sh.sp_of[sp]] * Sh.wcellT[(size_t)sp * Sh.n_true + ic] : 0.0;
      else
        w = sp == Sh.Sg + (ic - Sh.n_true) ? th[Sh.sp_of[sp]] : 0.0;
    }
    rwk[k] = w;
  }
  // union of the wave's 16 cells' supports, as window-relative bins, clipped to the chunk
  const int2 sp = get_support(rc);
  int lo = valid ? sp.x : 0x7fffffff, hi = valid ? sp.y : -1;
  for (int o = 8; o > 0; o >>= 1) {
    lo = min(lo, __shfl_xor(lo, o, 64));
    hi = max(hi, __shfl_xor(hi, o, 64));
  }
  const int b0 = max(it.bin0, wave_uniform(lo) - T.lo), b1 = min(it.bin1, wave_uniform(hi) - T.lo);
  const double *BR = binrec + T.win_off * kBinRecLen, *BF = bref + T.bref_off * 4, *HR = H + T.fh_off;
  double A0 = 0.0, A1 = 0.0, A2 = 0.0;
  if (Sh.family == kGammaPE)
    adj_s_walk<kGammaPE>(BR, BF, HR, T.S, nk, b0, b1, rc, rwk, ec, A0, A1, A2);
  else
    adj_s_walk<kGaussE>(BR, BF, HR, T.S, nk, b0, b1, rc, rwk, ec, A0, A1, A2);
  // the four lanes of a cell (l, l ^ 16, l ^ 32, l ^ 48) in a fixed order
  A0 += __shfl_xor(A0, 16, 64);
  A1 += __shfl_xor(A1, 16, 64);
  A2 += __shfl_xor(A2, 16, 64);
  A0 += __shfl_xor(A0, 32, 64);
  A1 += __shfl_xor(A1, 32, 64);
  A2 += __shfl_xor(A2, 32, 64);
  if (grp == 0 && valid) {
    double *o = apart + T.apart_off + ((long long)it.chunk * T.n_cell + i) * 3;
    o[0] = A0;
    o[1] = A1;
    o[2] = A2;
  }
}

// --------------------------------------------- direct per-pair adjoint ----
// One wave per adjoint item, lane = cell, walking the window bins of the
// cell's own support inside the item's range: per-cell sums G K, G dK/dm and
// G dK/ds (G = sum_d eps_d (1 - n/mu) from the window-bin record, without a
// width factor), which k_cellgrad chains to the parameters.  With exact bins
// a bin's upper edge is the next bin's lower edge, evaluated once.
__global__ __launch_bounds__(256) void k_adjg(const AdjItem *__restrict__ items, int n_items,
                                              const ToyDev *__restrict__ toys, const ShapeDev *__restrict__ shapes,
                                              const double *__restrict__ rec, const double *__restrict__ binrec,
                                              const uint8_t *__restrict__ active, double *__restrict__ apart) {
  const int w_item = blockIdx.x * 4 + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (w_item >= n_items) return;
  const AdjItem it = items[w_item];
  if (active && !active[it.toy]) return;
  const ToyDev &T = toys[it.toy];
  if (!T.gen) return;
  const ShapeDev &Sh = shapes[T.shape];
  const int i = it.cell0 + lane;
  if (i >= T.n_cell) return;
  const double *rc = rec + (T.cell_off + i) * kRecLen;
  const int2 sp = get_support(rc);
  const int b0 = max(it.bin0, sp.x - T.lo), b1 = min(it.bin1, sp.y - T.lo);
  double A0 = 0.0, A1 = 0.0, A2 = 0.0;
  if (b0 < b1) {
    const int fam = Sh.family;
    const double p = Sh.shape;
    const GenCell g{rc[0], rc[1], rc[3], rc[4], rc[5], rc[7]};
    const GenChain ch = gen_chain(fam, p, g);
    const double *BR = binrec + T.win_off * kBinRecLen;
    if (Sh.exact) {
      Edge lo = gen_edge(fam, p, g, ch, Sh.edges[T.lo + b0], true);
      for (int b = b0; b < b1; b++) {
        const Edge hi = gen_edge(fam, p, g, ch, Sh.edges[T.lo + b + 1], true);
        double dm, ds;
        const double K = edge_content(lo, hi, dm, ds), G = BR[(size_t)b * kBinRecLen + 3];
        A0 = fma(G, K, A0);
        A1 = fma(G, dm, A1);
        A2 = fma(G, ds, A2);
        lo = hi;
      }
    } else {
      for (int b = b0; b < b1; b++) {
        const double *bn = Sh.bins + (size_t)(T.lo + b) * kBinLen;
        double dm, ds;
        const double r = gen_density(fam, p, g, ch, bn[0], true, dm, ds);
        const double Gd = BR[(size_t)b * kBinRecLen + 3] * bn[1];
        A0 = fma(Gd, r, A0);
        A1 = fma(Gd, dm, A1);
        A2 = fma(Gd, ds, A2);
      }
    }
  }
  double *o = apart + T.apart_off + ((long long)it.chunk * T.n_cell + i) * 3;
  o[0] = A0;
  o[1] = A1;
  o[2] = A2;
}

hipError_t launch_adj(const BatchView &v, bool per_species, const uint8_t *active, hipStream_t st) {
  const AdjItem *it = per_species ? v.adj2 : v.adj1;
  const int n = per_species ? v.n_adj2 : v.n_adj1;
  if (n == 0) return hipSuccess;
  if (per_species) {
    hipLaunchKernelGGL(k_adj_s, dim3(xcd_grid(n)), dim3(kWaves * 64), 0, st, it, n, v.toys, v.shapes, v.theta_dev,
                       v.stride, v.rec, v.binrec, v.bref, v.H, active, v.apart);
    return hipGetLastError();
  }
  // one wave per item walks all bins of its cells, kAdjGroupWaves items per
  // workgroup (large batches: the fixed per-wave work spreads over four times
  // the pairs); kWaves waves interleave an item's bins (small batches, where
  // the grid must fill the GPU)
  if (v.has_gen)
    hipLaunchKernelGGL(k_adjg, dim3((n + 3) / 4), dim3(256), 0, st, it, n, v.toys, v.shapes, v.rec, v.binrec, active,
                       v.apart);
  const int groups = (n + kAdjGroupWaves - 1) / kAdjGroupWaves;
  if (v.adj_waves == 1)
    hipLaunchKernelGGL((k_adj<1>), dim3(xcd_grid(groups)), dim3(kAdjGroupWaves * 64), 0, st, it, n, v.toys, v.shapes,
                       v.rec, v.binrec, v.bref, active, v.apart);
  else
    hipLaunchKernelGGL((k_adj<kWaves>), dim3(xcd_grid(n)), dim3(kWaves * 64), 0, st, it, n, v.toys, v.shapes, v.rec,
                       v.binrec, v.bref, active, v.apart);
  return hipGetLastError();
}

// ----------------------------------------------------------- k_cellgrad ---
template <int CPT>
__global__ __launch_bounds__(256, 4) void k_cellgrad(const int *__restrict__ toy_list, const ToyDev *__restrict__ toys, const ShapeDev *__restrict__ shapes,
                                                  const double *__restrict__ theta, int stride,
                                                  const double *__restrict__ rec, const double *__restrict__ apart,
                                                  const uint8_t *__restrict__ active, double *__restrict__ gpart) {
  __shared__ double part[kBlock / 64][kGradLen];
  const int t = toy_of(toy_list, blockIdx.y);
  if (active && !active[t]) return;
  const ToyDev &T = toys[t];
  if ((int)blockIdx.x >= T.cell_blocks || T.tmpl) return;
  const ShapeDev &Sh = shapes[T.shape];
  const double *th = theta + (size_t)t * stride;
  const int fam = Sh.family, nr = fam == kGaussE ? 2 : 5;
  double gR[GS_MAX_SPECIES], gP[5], R[GS_MAX_SPECIES];  // R: grid species' rates (uniform)
#pragma unroll
  for (int s = 0; s < GS_MAX_SPECIES; s++) {
    gR[s] = 0.0;
    R[s] = s < Sh.Sg ? th[Sh.sp_of[s]] : 0.0;
  }
#pragma unroll
  for (int p = 0; p < 5; p++) gP[p] = 0.0;
  // CPT * kBlock consecutive cells per block: cells threadIdx.x, + kBlock, ... per thread
  for (int c = 0; c < CPT; c++) {
    const int i = (blockIdx.x * CPT + c) * kBlock + threadIdx.x;
    if (i >= Sh.n_cell) break;
    // the adjoint chunks' partials, summed in chunk order; U chunks' loads are
    // issued before their adds, so a single model's many chunks (split-K) do not
    // wait out one load latency each
    constexpr int U = CPT == 1 ? 8 : 2;
    const double *ap = apart + T.apart_off + (long long)i * 3;
    const long long cs = (long long)T.n_cell * 3;
    double A0 = 0.0, A1 = 0.0, A2 = 0.0;
    int k = 0;
    for (; k + U <= T.adj_chunks; k += U) {
      double a[U][3];
#pragma unroll
      for (int u = 0; u < U; u++)
#pragma unroll
        for (int q = 0; q < 3; q++) a[u][q] = ap[(k + u) * cs + q];
#pragma unroll
      for (int u = 0; u < U; u++) {
        A0 += a[u][0];
        A1 += a[u][1];
        A2 += a[u][2];
      }
    }
    for (; k < T.adj_chunks; k++) {
      A0 += ap[k * cs];
      A1 += ap[k * cs + 1];
      A2 += ap[k * cs + 2];
    }
    Moments mo;
    moments(fam, th + Sh.S, Sh.birks_A, Sh.cellE[i], mo);
    // 1-D toys: the combined weight W_i = sum_s R_s w_si, recomputed from the shape's
    // weights (shared by every toy of the shape) rather than read back from the cell
    // record, and in the same walk the rate gradients sum_i w_si A0_i; a line cell
    // weighs its own species alone
    double W = 1.0;
    if (!T.two_d) {
      if (i < Sh.n_true) {
        const double *w = Sh.wcellT + i;
        W = 0.0;
#pragma unroll
        for (int s = 0; s < GS_MAX_SPECIES; s++)
          if (s < Sh.Sg) {
            const double ws = w[(size_t)s * Sh.n_true];
            W = __fma_rn(R[s], ws, W);
            gR[s] = __fma_rn(ws, A0, gR[s]);
          }
      } else {
        const int q = Sh.Sg + (i - Sh.n_true);
        W = th[Sh.sp_of[q]];
#pragma unroll
        for (int s = 0; s < GS_MAX_SPECIES; s++)
          if (s == q) gR[s] += A0;
      }
    }
    double dNdm, dNds;
    if (Sh.gen) {  // direct path: the sums are of G dK/dm and G dK/ds themselves
      dNdm = W * A1;
      dNds = W * A2;
    } else if (fam == kGammaPE) {
      const double m = mo.m, s = mo.s, s2 = s * s;
      const double k = m * m / s2, thg = s2 / m, mk = k * thg;
      // shift the sums of ln x and x to ln x - ln(k th) and x - k th
      const double B1 = __fma_rn(-log(mk), A0, A1), B2 = __fma_rn(-mk, A0, A2);
      const double dk = W * __fma_rn(log_minus_digamma(k), A0, B1);  // d(-ln L)/dk
      const double dth = W * B2 / (thg * thg);                       // d(-ln L)/dtheta
      dNdm = dk * (2.0 * m / s2) - dth * (s2 / (m * m));
      dNds = -dk * (2.0 * m * m / (s2 * s)) + dth * (2.0 * s / m);
    } else {
      const double is = 1.0 / mo.s;
      dNdm = W * A1 * is;
      dNds = W * (A2 - A0) * is;
    }
#pragma unroll
    for (int p = 0; p < 5; p++) gP[p] = __fma_rn(dNdm, mo.dm[p], __fma_rn(dNds, mo.ds[p], gP[p]));
    // (rate gradients of 2-D models come from the pulse-shape contraction, k_bins2)
  }
  // every entry summed over the wave, then over the block's waves in a fixed order
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // (one cell per thread: a small batch or one model, where the reduction's
  // latency shows; four values go through the butterfly together)
  wave_sum_n<GS_MAX_SPECIES, CPT == 1 ? 4 : 1>(gR, Sh.S);
  wave_sum_n<5, CPT == 1 ? 4 : 1>(gP, nr);
  if (lane == 0) {
#pragma unroll
    for (int s = 0; s < GS_MAX_SPECIES; s++)
      if (s < Sh.S) part[wv][s] = gR[s];
#pragma unroll
    for (int p = 0; p < 5; p++)
      if (p < nr) part[wv][Sh.S + p] = gP[p];
  }
  __syncthreads();
  const int q = threadIdx.x;
  if (q < Sh.S + nr) {
    double v = part[0][q];
    for (int w = 1; w < kBlock / 64; w++) v += part[w][q];
    gpart[(T.gpart_off + blockIdx.x) * kGradLen + (q < Sh.S ? Sh.sp_of[q] : q)] = v;
  }
}

hipError_t launch_cellgrad(const BatchView &v, const double *theta, const uint8_t *active, hipStream_t st) {
  // one cell per thread keeps the kernel's registers low (no accumulators
  // carried across cells); four per thread amortise the block reductions
  if (v.grad_cells == kBlock)
    hipLaunchKernelGGL(k_cellgrad<1>, dim3(v.max_cell_blocks, v.n_list), dim3(kBlock), 0, st, v.toy_list, v.toys,
                       v.shapes, theta, v.stride, v.rec, v.apart, active, v.gpart);
  else
    hipLaunchKernelGGL(k_cellgrad<kGradCellsLarge / kBlock>, dim3(v.max_cell_blocks, v.n_list), dim3(kBlock), 0, st,
                       v.toy_list, v.toys, v.shapes, theta, v.stride, v.rec, v.apart, active, v.gpart);
  return hipGetLastError();
}

// ------------------------------------------------------------- k_finish ---
// Thread p < stride: gradient entry p; thread 0 also -ln L and status.
__global__ __launch_bounds__(256) void k_finish(const int *__restrict__ toy_list, const ToyDev *__restrict__ toys, const ShapeDev *__restrict__ shapes,
                                               const double *__restrict__ theta, int stride,
                                               const double *__restrict__ nllp, const uint32_t *__restrict__ badp,
                                               const uint32_t *__restrict__ cflag, const double *__restrict__ gpart,
                                               const double *__restrict__ vpart, const uint32_t *__restrict__ pflag,
                                               const double *__restrict__ pull_c,
                                               const double *__restrict__ pull_s, const uint8_t *__restrict__ active,
                                               double *__restrict__ nll, double *__restrict__ grad,
                                               uint32_t *__restrict__ status) {
  __shared__ uint32_t st_s;
  __shared__ double gsum[kGradLen];
  const int t = toy_of(toy_list, blockIdx.x);
  if (active && !active[t]) return;
  const ToyDev &T = toys[t];
  const ShapeDev &Sh = shapes[T.shape];
  const double *th = theta + (size_t)t * stride;
  // wave 0: -ln L and status; every wave: gradient entries wave, wave + 4, ...
  // Every sum over block partials runs across the lanes (lane-strided, then a
  // fixed butterfly), so no lane walks a long serial chain of loads.
  const int p = threadIdx.x & 63, wave = wave_uniform(threadIdx.x >> 6);
  if (grad) {
    const int nr = Sh.family == kTemplate ? 0 : Sh.family == kGaussE ? 2 : 5;
    const double *vp = vpart + T.vpart_off * kVLen;
    // this wave's entries pp = wave + kWaves q, q < nq; the cell-gradient block
    // partials of all of them are loaded in one pass over the blocks, so their
    // loads are in flight together
    constexpr int kPW = (kGradLen + kWaves - 1) / kWaves;
    const int nq = T.P > wave ? (T.P - wave + kWaves - 1) / kWaves : 0;
    double a[kPW];
#pragma unroll
    for (int q = 0; q < kPW; q++) a[q] = 0.0;
    for (int b = p; b < T.cell_blocks; b += 64) {
      const double *g = gpart + (T.gpart_off + b) * kGradLen;
#pragma unroll
      for (int q = 0; q < kPW; q++)
        if (q < nq && wave + kWaves * q < Sh.S + nr) a[q] += g[wave + kWaves * q];
    }
    if (T.two_d) {  // pieces that need no fold, from the 2-D block partials
#pragma unroll
      for (int q = 0; q < kPW; q++) {
        const int pp = wave + kWaves * q;
        int e = -1;  // the entry's column of the 2-D partials (none past this wave's entries)
        if (q < nq && pp < Sh.S) {
          for (int r = 0; r < Sh.S; r++)
            if (Sh.sp_of[r] == pp) e = r;
        } else if (q < nq && pp >= Sh.S + nr) {
          e = GS_MAX_SPECIES + (pp - Sh.S - nr);
        }
        if (e >= 0 && e < GS_MAX_SPECIES)  // rate pieces: the first hblocks rows
          for (int blk = p; blk < T.hblocks; blk += 64) a[q] += vp[(size_t)blk * kVLen + e];
        else if (e >= 0)  // nuisance pieces: the next bin_blocks rows
          for (int blk = p; blk < T.bin_blocks; blk += 64) a[q] += vp[(size_t)(T.hblocks + blk) * kVLen + e];
      }
    }
    wave_sum_n<kPW, 3>(a, nq);
    if (p == 0)
#pragma unroll
      for (int q = 0; q < kPW; q++)
        if (q < nq) gsum[wave + kWaves * q] = a[q];
  }
  if (wave == 0) {
    double part = 0.0;
    for (int b = p; b < T.bin_blocks; b += 64) part += nllp[T.nllp_off + b];
    const double nll_bins = wave_sum(part);
    // flags and pull terms spread over the lanes (no serial chain of loads)
    bool nonfin = false;
    uint32_t bb = 0u, cf = 0u;
    for (int b = p; b < T.bin_blocks; b += 64) bb |= badp[T.nllp_off + b];
    for (int b = p; b < T.cflag_blocks; b += 64) cf |= cflag[T.cflag_off + b];
    const bool dom = (bb & kBadDomain) || (cf & kCellInvalid);  // kCellInvalid: invalid response on the grid
    const bool range = bb & kBadRange, unres = cf & kCellUnresolved;
    double pull = 0.0;
    if (p < T.P) {
      nonfin = !isfinite(th[p]);
      const double s = pull_s[T.pull_off + p];
      if (s > 0.0) {
        const double z = (th[p] - pull_c[T.pull_off + p]) / s;
        pull = 0.5 * z * z;
      }
    }
    pull = wave_sum(pull);
    const bool any_dom = __ballot(dom) != 0ull, any_nonfin = __ballot(nonfin) != 0ull;
    const bool any_range = __ballot(range) != 0ull, any_unres = __ballot(unres) != 0ull;
    if (p == 0) {
      uint32_t st = 0;
      double sum = nll_bins + pull - T.cnl;  // cnl: the parameter-free part k_bins2 leaves out
      if (any_dom || (T.two_d && pflag[t])) st |= GS_ST_DOMAIN;  // pflag: invalid pulse-shape nuisance
      if (any_nonfin) st |= GS_ST_NONFINITE;
      if (any_unres) st |= GS_ST_UNRESOLVED;
      if (any_range) st |= GS_ST_GRAD_RANGE;
      if (st & GS_ST_NONFINITE) {
        st = GS_ST_NONFINITE;  // a non-finite parameter explains every other symptom
        sum = __builtin_nan("");
      } else if (st & GS_ST_UNRESOLVED) {
        sum = __builtin_nan("");  // refused: no value is claimed
      } else if (st & GS_ST_DOMAIN) {
        sum = __builtin_inf();
      }
      nll[t] = sum;
      status[t] = st;
      st_s = st;
    }
  }
  __syncthreads();
  if (grad && threadIdx.x < stride) {
    double g = 0.0;
    if (p < T.P) {
      g = gsum[p];
      const double s = pull_s[T.pull_off + p];
      if (s > 0.0) g += (th[p] - pull_c[T.pull_off + p]) / (s * s);
      if (st_s & (GS_ST_DOMAIN | GS_ST_NONFINITE | GS_ST_UNRESOLVED | GS_ST_GRAD_RANGE)) g = __builtin_nan("");
    }
    grad[(size_t)t * stride + p] = g;
  }
}

hipError_t launch_finish(const BatchView &v, const double *theta, double *nll, double *grad, uint32_t *status,
                         const uint8_t *active, hipStream_t st) {
  hipLaunchKernelGGL(k_finish, dim3(v.n_list), dim3(kBlock), 0, st, v.toy_list, v.toys, v.shapes, theta, v.stride, v.nllp, v.badp,
                     v.cflag, v.gpart, v.vpart, v.pflag, v.pull_c, v.pull_s, active, nll, grad, status);
  return hipGetLastError();
}

// ------------------------------------------------------- bins setup -------
// Reco-bin constants of a shape: midpoint, width, ln(midpoint) as double-double.
__global__ void k_bins_setup(const double *__restrict__ edges, int n_reco, double *__restrict__ bins) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_reco) return;
  const double a = edges[j], b = edges[j + 1];
  const double x = (a + b) * 0.5;
  const dd L = x > 0.0 ? dd_log(x) : dd{0.0, 0.0};
  double *o = bins + (size_t)j * kBinLen;
  o[0] = x;
  o[1] = b - a;
  o[2] = L.hi;
  o[3] = L.lo;
}

hipError_t launch_bins_setup(double *bins, const double *edges, int n_reco, hipStream_t st) {
  hipLaunchKernelGGL(k_bins_setup, dim3((n_reco + 255) / 256), dim3(256), 0, st, edges, n_reco, bins);
  return hipGetLastError();
}

// ---------------------------------------------- per-species (plain path) --
// F (species s, window bin b) = dx_b * sum over chunks (fixed order); one thread per (bin, species).
__global__ __launch_bounds__(256) void k_reduceF(const int *__restrict__ toy_list, const ToyDev *__restrict__ toys,
                                                 const ShapeDev *__restrict__ shapes,
                                                 const double *__restrict__ fspart, int mode,
                                                 const uint8_t *__restrict__ active, double *__restrict__ F) {
  const int t = toy_of(toy_list, blockIdx.y);
  if (active && !active[t]) return;
  const ToyDev &T = toys[t];
  if (mode >= 0 && T.two_d != mode) return;
  const ShapeDev &Sh = shapes[T.shape];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= T.L * T.S) return;
  const int b = e / T.S, sp = e - b * T.S;
  const double dx = Sh.bins[(size_t)(T.lo + b) * kBinLen + 1];
  // the fold chunks' partials in chunk order, eight chunks' loads issued before their adds
  const double *fp = fspart + T.fs_off + (long long)b * T.S + sp;
  const long long cs = (long long)T.L * T.S;
  double acc = 0.0;
  int c = 0;
  for (; c + 8 <= T.fold_chunks; c += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; u++) v[u] = fp[(c + u) * cs];
#pragma unroll
    for (int u = 0; u < 8; u++) acc += v[u];
  }
  for (; c < T.fold_chunks; c++) acc += fp[c * cs];
  F[fh_at(T, sp, b)] = T.gen ? acc : dx * acc;
}

hipError_t launch_reduceF(const BatchView &v, int mode, const uint8_t *active, hipStream_t st) {
  const int *list = mode == kOnly2D ? v.list2d : mode == kOnly1D ? v.list1d : v.toy_list;
  const int n = mode == kOnly2D ? v.n2d : mode == kOnly1D ? v.n1d : v.n_list;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduceF, dim3(v.max_ls_blocks, n), dim3(kBlock), 0, st, list, v.toys, v.shapes, v.fspart,
                     mode, active, v.F);
  return hipGetLastError();
}

// -ln L block partials from cached per-species spectra: mu_dj = eps_d sum_s R_s F_js.
__global__ __launch_bounds__(256) void k_binsF(const int *__restrict__ toy_list, const ToyDev *__restrict__ toys, const ShapeDev *__restrict__ shapes,
                                               const double *__restrict__ theta, int stride,
                                               const double *__restrict__ F, const double *__restrict__ cnt,
                                               double *__restrict__ nllp, uint32_t *__restrict__ badp,
                                               double *__restrict__ mu_out) {
  __shared__ double lds[8];
  __shared__ uint32_t bad_s;
  const int t = toy_of(toy_list, blockIdx.y);
  const ToyDev &T = toys[t];
  if ((int)blockIdx.x >= T.bin_blocks || T.two_d || T.tmpl) return;
  const ShapeDev &Sh = shapes[T.shape];
  const double *th = theta + (size_t)t * stride;
  if (threadIdx.x == 0) bad_s = 0u;
  __syncthreads();
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  double sum = 0.0;
  if (b < T.L) {
    const double *f = F + fh_at(T, 0, b);
    double mu1 = 0.0;
    for (int s = 0; s < Sh.S; s++) mu1 = __fma_rn(th[Sh.sp_of[s]], f[s], mu1);
    uint32_t bad = 0u;
    for (int d = 0; d < T.D; d++) {
      const double mu = T.exposure[d] * mu1;
      const double n = cnt[T.cnt_off + (long long)d * T.L + b];
      double term, g;
      bad |= poisson_term(mu, n, term, g);
      sum += term;
      if (mu_out) mu_out[(long long)d * T.L + b] = mu;
    }
    if (bad) atomicOr(&bad_s, bad);
  }
  const double tot = block_sum(sum, lds);
  __syncthreads();
  if (threadIdx.x == 0) {
    nllp[T.nllp_off + blockIdx.x] = tot;
    badp[T.nllp_off + blockIdx.x] = bad_s;
  }
}

hipError_t launch_binsF(const BatchView &v, const double *theta, double *mu_out, hipStream_t st) {
  if (v.n1d == 0) return hipSuccess;
  hipLaunchKernelGGL(k_binsF, dim3(v.max_bin_blocks1, v.n1d), dim3(kBlock), 0, st, v.list1d, v.toys, v.shapes, theta,
                     v.stride, v.F, v.cnt, v.nllp, v.badp, mu_out);
  return hipGetLastError();
}


// ---------------------------------------------------- Monte Carlo templates --
// The Monte Carlo fit (section 3.2, cost model Eq.1): each species' reco
// spectrum at unit rate is a template T_sj (the response is already in it),
// so mu_dj = eps_d sum_s R_s T_sj needs no fold.  Toys that share a template
// and window (a group of at most 16, formed on the host) make both sums dense
// contractions over the shared T, which run on v_mfma_f64_16x16x4f64:
//   mu^T[j][q]  = sum_s T[s][j] R[s][q]              (bins x toys, K = species)
//   grad[s][q] += sum_j T[s][j] G[q][j],  G = sum_d eps_d (1 - n_dj/mu_dj)
// A wave walks WB bins of its group in chunks of 16.  Chunk row r
// (0..15) stands for bin 4 (r % 4) + r / 4, so that the first product leaves
// lane l with toy l % 16 at the four consecutive bins 4 (l / 16) + v of its
// registers v (its counts are one 32-byte run), and register v is then the
// B operand of the second product's step v as it stands (k = l / 16 is bin
// 4k + v).  Padding species, bins past the window and empty toy slots carry
// zeros into both products.  The four waves of a block cover 4 WB
// consecutive bins and fold their partials through LDS in a fixed order into
// one row per toy and block.
template <int WB>
__global__ __launch_bounds__(256) void k_tmpl(const int *__restrict__ toy_list, const int *__restrict__ groups,
                                              const ToyDev *__restrict__ toys, const ShapeDev *__restrict__ shapes,
                                              const double *__restrict__ theta, int stride,
                                              const double *__restrict__ cnt, const uint8_t *__restrict__ active,
                                              double *__restrict__ nllp, uint32_t *__restrict__ badp,
                                              double *__restrict__ gpart, double *__restrict__ mu_out) {
  __shared__ double gsh[kWaves][4][64];
  __shared__ double nsh[kWaves][16];
  __shared__ uint32_t bsh[kWaves][16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, q = lane & 15, k4 = lane >> 4;
  const int first = groups[2 * blockIdx.x], count = groups[2 * blockIdx.x + 1];
  const int blk = blockIdx.y;
  const ToyDev &L0 = toys[toy_of(toy_list, first)];  // the group shares shape, window and datasets
  if (blk >= L0.bin_blocks) return;
  const ShapeDev &Sh = shapes[L0.shape];
  const int S = Sh.S, L = L0.L, D = L0.D;
  // this lane's toy (column q of both products)
  const int t = q < count ? toy_of(toy_list, first + q) : -1;
  const bool live = t >= 0 && !(active && !active[t]);
  const ToyDev &T = toys[live ? t : toy_of(toy_list, first)];
  const double *tT = Sh.wcellT + L0.lo;  // T[s][j] at tT[s * n_true + j]
  const size_t nt = (size_t)Sh.n_true;
  // B operand of the first product: R[s = 4i + l/16][q]
  double rB[4];
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const int s = 4 * i + k4;
    rB[i] = live && s < S ? theta[(size_t)t * stride + Sh.sp_of[s]] : 0.0;
  }
  const double *cq = cnt + T.cnt_off;
  const int nsteps = (S + 3) >> 2;  // first-product steps of 4 species
  // first-product row r = l % 16 is bin 4 (r % 4) + r / 4 of the chunk
  const int jA = 4 * (q & 3) + (q >> 2);
  dbl4 gacc = {0.0, 0.0, 0.0, 0.0};
  double sum = 0.0;
  uint32_t bad = 0u;
  static_assert(WB % 16 == 0, "template chunks are 16 bins");
  const int w0 = blk * kWaves * WB + wv * WB;
  // loads use clamped (in-bounds) indices and are unconditional, so that a
  // chunk's loads issue together; what lies outside is zeroed by selects
  const int sA[4] = {min(k4, S - 1), min(4 + k4, S - 1), min(8 + k4, S - 1), min(12 + k4, S - 1)};
  const int sq = min(q, S - 1);
  for (int c = 0; c < WB; c += 16) {
    const int n0 = w0 + c;
    if (n0 >= L) break;
    const int jb = n0 + 4 * k4;  // lane l: toy q at bins jb + v, v = 0..3
    const bool inA = n0 + jA < L;
    const int jAc = min(n0 + jA, L - 1);
    double a[4], tA[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const double x = tT[sA[i] * nt + jAc];
      a[i] = inA && 4 * i + k4 < S ? x : 0.0;
    }
#pragma unroll
    for (int v = 0; v < 4; v++) {
      const double x = tT[sq * nt + min(jb + v, L - 1)];
      tA[v] = jb + v < L && q < S ? x : 0.0;
    }
    dbl4 mu1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 4; i++)
      if (i < nsteps) mu1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], rB[i], mu1, 0, 0, 0);
    double G[4] = {0.0, 0.0, 0.0, 0.0};
    for (int d = 0; d < D; d++) {
      const double e = T.exposure[d];
      const double *cd = cq + (long long)d * L;
      double n[4];
#pragma unroll
      for (int v = 0; v < 4; v++) n[v] = cd[min(jb + v, L - 1)];
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const bool ok = live && jb + v < L;
        const double mu = e * mu1[v];
        double term, gg;
        const uint32_t f = poisson_term(mu, n[v], term, gg);
        bad |= ok ? f : 0u;
        sum += ok ? term : 0.0;
        G[v] = ok ? __fma_rn(e, gg, G[v]) : 0.0;
        if (mu_out && q == 0 && ok) mu_out[(long long)d * L + jb + v] = mu;
      }
    }
#pragma unroll
    for (int v = 0; v < 4; v++) gacc = __builtin_amdgcn_mfma_f64_16x16x4f64(tA[v], G[v], gacc, 0, 0, 0);
  }
  // toy q's -ln L and flags over the four lanes that hold it
  sum += __shfl_xor(sum, 16);
  sum += __shfl_xor(sum, 32);
  bad |= __shfl_xor(bad, 16);
  bad |= __shfl_xor(bad, 32);
#pragma unroll
  for (int v = 0; v < 4; v++) gsh[wv][v][lane] = gacc[v];
  if (k4 == 0) {
    nsh[wv][q] = sum;
    bsh[wv][q] = bad;
  }
  __syncthreads();
  if (wv != 0 || !live) return;
  // gacc register v of lane l is grad[s = l/16 + 4v][toy q]
#pragma unroll
  for (int v = 0; v < 4; v++) {
    const int s = k4 + 4 * v;
    if (s < S) {
      double g = gsh[0][v][lane];
      for (int w = 1; w < kWaves; w++) g += gsh[w][v][lane];
      gpart[(T.gpart_off + blk) * kGradLen + Sh.sp_of[s]] = g;
    }
  }
  if (k4 == 0) {
    double tot = nsh[0][q];
    uint32_t b = bsh[0][q];
    for (int w = 1; w < kWaves; w++) {
      tot += nsh[w][q];
      b |= bsh[w][q];
    }
    nllp[T.nllp_off + blk] = tot;
    badp[T.nllp_off + blk] = b;
  }
}

hipError_t launch_tmpl(const BatchView &v, const double *theta, double *mu_out, const uint8_t *active, hipStream_t st) {
  if (v.nt == 0 || v.n_tgroup == 0) return hipSuccess;
  const dim3 grid(v.n_tgroup, v.max_bin_blocks_t), block(kBlock);
  if (v.tmpl_bins == kTmplBlockBins)
    hipLaunchKernelGGL(k_tmpl<kTmplBlockBins / kWaves>, grid, block, 0, st, v.listt, v.tgroup, v.toys, v.shapes,
                       theta, v.stride, v.cnt, active, v.nllp, v.badp, v.gpart, mu_out);
  else if (v.tmpl_bins == 256)
    hipLaunchKernelGGL(k_tmpl<64>, grid, block, 0, st, v.listt, v.tgroup, v.toys, v.shapes, theta, v.stride, v.cnt,
                       active, v.nllp, v.badp, v.gpart, mu_out);
  else
    hipLaunchKernelGGL(k_tmpl<16>, grid, block, 0, st, v.listt, v.tgroup, v.toys, v.shapes, theta, v.stride, v.cnt,
                       active, v.nllp, v.badp, v.gpart, mu_out);
  return hipGetLastError();
}

// ------------------------------------------- secondary observable (2-D) --
// Pulse-shape probabilities of every species (section 2.4): a two-Gaussian
// mixture at the bin midpoints, means shifted by delta, widths scaled by
// kappa, odds of component 1 multiplied by exp(eta), renormalised over the
// bins; with their derivatives w.r.t. (delta, kappa, eta).  One wave per
// (toy, species), lanes over the bins (at most GS_MAX_PSD = 2 x 64).
__global__ __launch_bounds__(64) void k_psd(const int *__restrict__ toy_list, const ToyDev *__restrict__ toys,
                                            const ShapeDev *__restrict__ shapes, const double *__restrict__ theta,
                                            int stride, const uint8_t *__restrict__ active, double *__restrict__ P,
                                            double *__restrict__ dP, uint32_t *__restrict__ pflag) {
  const int t = toy_of(toy_list, blockIdx.y), s = blockIdx.x, lane = threadIdx.x;
  if (active && !active[t]) return;
  const ToyDev &T = toys[t];
  if (!T.two_d) return;
  const ShapeDev &Sh = shapes[T.shape];
  const double *nu = theta + (size_t)t * stride + Sh.S + (Sh.family == kGaussE ? 2 : 5);
  const double delta = nu[0], kappa = nu[1], eta = nu[2];
  const bool ok = kappa > 0.0 && isfinite(kappa) && isfinite(delta) && isfinite(eta);
  if (s == 0 && lane == 0) pflag[t] = ok ? 0u : 1u;
  if (!ok || s >= Sh.S) return;
  const double *mx = Sh.mix + 5 * s;
  const double w1 = mx[0];
  const double wp = 1.0 / (1.0 + exp(-(log(w1 / (1.0 - w1)) + eta)));
  const double inv_root2pi = 0.39894228040143267794;
  auto comp = [&](double y, int c, double &N, double &dd, double &dk) {
    const double sg = mx[2 + 2 * c] * kappa;
    const double z = (y - (mx[1 + 2 * c] + delta)) / sg;
    N = exp(-0.5 * z * z) * inv_root2pi / sg;
    dd = N * z / sg;
    dk = N * (z * z - 1.0) / kappa;
  };
  const int K = Sh.n_psd;
  double p[2] = {0.0, 0.0}, q0[2] = {0.0, 0.0}, q1[2] = {0.0, 0.0}, q2[2] = {0.0, 0.0};
  double Z = 0.0, dZ0 = 0.0, dZ1 = 0.0, dZ2 = 0.0;
#pragma unroll
  for (int h = 0; h < 2; h++) {
    const int k = lane + 64 * h;
    if (k < K) {
      const double y = Sh.psd[2 * k], dy = Sh.psd[2 * k + 1];
      double N0, d0, k0, N1, d1, k1;
      comp(y, 0, N0, d0, k0);
      comp(y, 1, N1, d1, k1);
      p[h] = dy * (wp * N0 + (1.0 - wp) * N1);
      q0[h] = dy * (wp * d0 + (1.0 - wp) * d1);
      q1[h] = dy * (wp * k0 + (1.0 - wp) * k1);
      q2[h] = dy * wp * (1.0 - wp) * (N0 - N1);
      Z += p[h];
      dZ0 += q0[h];
      dZ1 += q1[h];
      dZ2 += q2[h];
    }
  }
  Z = wave_sum(Z);
  dZ0 = wave_sum(dZ0);
  dZ1 = wave_sum(dZ1);
  dZ2 = wave_sum(dZ2);
  const double iZ = 1.0 / Z;
#pragma unroll
  for (int h = 0; h < 2; h++) {
    const int k = lane + 64 * h;
    if (k < K) {
      const double pk = p[h] * iZ;
      const long long o = T.psd_off + (long long)s * T.K + k;
      P[o] = pk;
      dP[3 * o + 0] = (q0[h] - pk * dZ0) * iZ;
      dP[3 * o + 1] = (q1[h] - pk * dZ1) * iZ;
      dP[3 * o + 2] = (q2[h] - pk * dZ2) * iZ;
    }
  }
}

hipError_t launch_psd(const BatchView &v, const double *theta, const uint8_t *active, hipStream_t st) {
  if (v.n2d == 0) return hipSuccess;
  hipLaunchKernelGGL(k_psd, dim3(GS_MAX_SPECIES, v.n2d), dim3(64), 0, st, v.list2d, v.toys, v.shapes, theta,
                     v.stride, active, v.P, v.dP, v.pflag);
  return hipGetLastError();
}

// Joint 2-D likelihood of a toy (section 2.4) with its adjoint seeds, on
// v_mfma_f64_16x16x4f64.  With RF_js = R_s F_js the expected counts of the
// (window bin j, pulse-shape bin k) cells are mu_djk = eps_d M_jk, M = RF P (a
// sum over species), and Gam_jk = sum_d eps_d (1 - n_djk/mu_djk).  A wave takes
// 16 window bins at a time and, per tile of 16 pulse-shape bins, forms
//   M^T = P^T RF^T  (A: P from LDS; B: rows of F times the rates),
//   the Poisson terms and Gam^T, in M^T's accumulator layout (lane l, register
//        v: k = l/16 + 4v, j = l%16),
//   h^T += P Gam^T: that accumulator layout is this product's B operand
//        layout (lane l: k = l/16 + 4c, j = l%16), so Gam stays in registers,
//   D_v^T = dP_v^T RF^T and A_v += sum_jk D_v^T Gam^T, the pieces of the
//        pulse-shape nuisance gradient that need no fold (v: delta, kappa, eta),
// then H_js = dx_j h_js (h_js = sum_k P_sk Gam_jk), the bin record, and the
// rate-gradient piece a_s = sum_j F_js h_js.  Pulse-shape bins past K and
// window bins past the window take Gam = 0 and zero B operands; their A
// operands are clamped (finite) reads.  Block blk covers iter2 rounds of
// kWaves x 16 window bins; it writes the -ln L partial nllp[blk], the rate
// pieces to vpart row blk and the nuisance pieces to row hblocks + blk.
// SPLIT (one round per block: small batches, where one model must fill the
// GPU): the block's waves share 16 window bins and take its pulse-shape tiles
// in turn (wave w: tiles w, w + kWaves, ...); wave 0 adds their h^T in wave
// order through LDS and writes the seeds.  P and dP are staged in LDS as
// [s][4][k].
template <bool SPLIT>
__global__ __launch_bounds__(256, 3) void k_bins2(const int *__restrict__ toy_list, const ToyDev *__restrict__ toys,
                                               const ShapeDev *__restrict__ shapes,
                                               const double *__restrict__ theta, int stride,
                                               const double *__restrict__ F, const double *__restrict__ P,
                                               const double *__restrict__ dP, const double *__restrict__ cnt,
                                               const double *__restrict__ nsum, int iter2,
                                               const uint8_t *__restrict__ active,
                                               double *__restrict__ nllp, uint32_t *__restrict__ badp,
                                               double *__restrict__ binrec, double *__restrict__ bref,
                                               double *__restrict__ H, double *__restrict__ vpart,
                                               double *__restrict__ mu_out) {
  extern __shared__ double pd[];  // [S][4][K]: P_sk, dP_sk/d(delta, kappa, eta)
  __shared__ double red[kWaves][kVLen];
  __shared__ double lds[8];
  __shared__ double leps[GS_MAX_DATASETS];
  __shared__ dbl4 hred[SPLIT ? kWaves * 64 : 1];
  __shared__ uint32_t bad_s;
  const int t = toy_of(toy_list, blockIdx.y);
  if (active && !active[t]) return;
  const ToyDev &T = toys[t];
  if ((int)blockIdx.x >= T.bin_blocks || !T.two_d || T.mv) return;
  const ShapeDev &Sh = shapes[T.shape];
  const int S = T.S, K = T.K, L = T.L;
  const int wave = wave_uniform(threadIdx.x >> 6), lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
  if (threadIdx.x == 0) bad_s = 0u;
  if (threadIdx.x < T.D) leps[threadIdx.x] = log(T.exposure[threadIdx.x]);
  for (int e = threadIdx.x; e < S * K; e += blockDim.x) {
    const long long o = T.psd_off + e;
    const int q = e / K, k = e - q * K;
    double *d = pd + (size_t)q * 4 * K + k;
    d[0] = P[o];
    d[K] = dP[3 * o];
    d[2 * K] = dP[3 * o + 1];
    d[3 * K] = dP[3 * o + 2];
  }
  __syncthreads();
  const double *th = theta + (size_t)t * stride;
  const int QS = (S + 3) >> 2, NT = (K + 15) >> 4;
  // With mu_d = eps_d M: sum_d (mu_d - n_d ln mu_d) = E M - N ln M - sum_d n_d ln eps_d
  // and Gam = sum_d eps_d (1 - n_d / mu_d) = E - N / M (E = sum_d eps_d, N = sum_d n_d,
  // from nsum): one load, one logarithm and one division per cell.  The last sum
  // does not depend on the parameters: T.cnl holds it over the whole window and
  // k_finish subtracts it.  Cells with M <= 0, or a quotient n_d / mu_d that may
  // overflow, take the terms dataset by dataset (poisson_term) and add their own
  // sum_d n_d ln eps_d back.
  double E = 0.0, emin = T.exposure[0];
  for (int d = 0; d < T.D; d++) {
    E += T.exposure[d];
    emin = fmin(emin, T.exposure[d]);
  }
  const double q_max = 1e300 * emin;
  const long long LK = (long long)L * K;
  double R[4];  // rates of this lane's B-operand species s = 4q + grp
#pragma unroll
  for (int q = 0; q < 4; q++) R[q] = 4 * q + grp < S ? th[Sh.sp_of[4 * q + grp]] : 0.0;
  const int sa = min(col, S - 1);  // A row (species) of P Gam^T
  const double *F0 = F + T.fh_off;
  double *H0 = H + T.fh_off;
  const double *cn = cnt + T.cnt_off, *ns = nsum + T.nsum_off;
  double sum = 0.0, A0 = 0.0, A1 = 0.0, A2 = 0.0, a[4] = {0.0, 0.0, 0.0, 0.0};
  uint32_t bad = 0u;
  const int nt0 = SPLIT ? wave : 0, nts = SPLIT ? kWaves : 1;  // this wave's pulse-shape tiles
  for (int r = 0; r < (SPLIT ? 1 : iter2); r++) {
    const int j0 = SPLIT ? blockIdx.x * 16 : ((blockIdx.x * iter2 + r) * kWaves + wave) * 16;
    if (j0 >= L) break;  // wave-uniform (block-uniform with SPLIT)
    const int jb = j0 + col;  // this lane's window bin (B column, accumulator column)
    const bool jin = jb < L;
    double f[4], rf[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      f[q] = jin && 4 * q + grp < S ? F0[(size_t)jb * S + 4 * q + grp] : 0.0;
      rf[q] = R[q] * f[q];
    }
    dbl4 hT = {0.0, 0.0, 0.0, 0.0};
    // summed counts of the lane's cells (clamped addresses): the wave's first tile now, its
    // next tile during the current one
    const double *nr = ns + (size_t)min(jb, L - 1) * K;
    double Nn[4];
#pragma unroll
    for (int v = 0; v < 4; v++) Nn[v] = nr[min(16 * nt0 + grp + 4 * v, K - 1)];
    for (int nt = nt0; nt < NT; nt += nts) {
      const int ka = min(16 * nt + col, K - 1);  // A row (pulse-shape bin) of P^T and dP^T
      double Nc[4];
#pragma unroll
      for (int v = 0; v < 4; v++) {
        Nc[v] = Nn[v];
        if (nt + nts < NT) Nn[v] = nr[min(16 * (nt + nts) + grp + 4 * v, K - 1)];
      }
      dbl4 Mt = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < 4; q++)
        if (q < QS) Mt = __builtin_amdgcn_mfma_f64_16x16x4f64(pd[(size_t)min(4 * q + grp, S - 1) * 4 * K + ka], rf[q], Mt, 0, 0, 0);
      double gam[4];
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int k = 16 * nt + grp + 4 * v;
        double gs = 0.0;
        if (jin && k < K) {
          const double M = Mt[v], N = Nc[v];
          const long long o0 = (long long)jb * K + k;
          const double q = N / M;
          if (M > 0.0 && q <= q_max) {
            sum += E * M - N * log(M);
            gs = E - q;
          } else {
            for (int d = 0; d < T.D; d++) {
              const double n = cn[o0 + d * LK];
              double term, g;
              bad |= poisson_term(T.exposure[d] * M, n, term, g);
              sum += __fma_rn(n, leps[d], term);
              gs = __fma_rn(T.exposure[d], g, gs);
            }
          }
          if (mu_out)
            for (int d = 0; d < T.D; d++) mu_out[o0 + d * LK] = T.exposure[d] * M;
        }
        gam[v] = gs;
      }
#pragma unroll
      for (int w = 0; w < 3; w++) {
        dbl4 Dt = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 4; q++)
          if (q < QS)
            Dt = __builtin_amdgcn_mfma_f64_16x16x4f64(pd[((size_t)min(4 * q + grp, S - 1) * 4 + 1 + w) * K + ka], rf[q],
                                                      Dt, 0, 0, 0);
        double acc = Dt[0] * gam[0];
        acc = __fma_rn(Dt[1], gam[1], acc);
        acc = __fma_rn(Dt[2], gam[2], acc);
        acc = __fma_rn(Dt[3], gam[3], acc);
        if (w == 0) A0 += acc;
        if (w == 1) A1 += acc;
        if (w == 2) A2 += acc;
      }
#pragma unroll
      for (int c = 0; c < 4; c++)
        hT = __builtin_amdgcn_mfma_f64_16x16x4f64(pd[(size_t)sa * 4 * K + min(16 * nt + 4 * c + grp, K - 1)], gam[c], hT,
                                                  0, 0, 0);
    }
    if (SPLIT) {  // the waves' partial h^T, added in wave order
      hred[wave * 64 + lane] = hT;
      __syncthreads();
      if (wave == 0) {
        hT = hred[lane];
        for (int w = 1; w < kWaves; w++) hT += hred[w * 64 + lane];
      }
    }
    if (jin && (!SPLIT || wave == 0)) {  // hT register v: species grp + 4v of bin jb
      const double *bn = Sh.bins + (size_t)(T.lo + jb) * kBinLen;
      const bool outside = Sh.family == kGammaPE && !(bn[0] > 0.0);
#pragma unroll
      for (int v = 0; v < 4; v++)
        if (grp + 4 * v < S) {
          H0[(size_t)jb * S + grp + 4 * v] = outside ? 0.0 : bn[1] * hT[v];
          a[v] = __fma_rn(f[v], hT[v], a[v]);
        }
      if (grp == 0) {
        double *br = binrec + (T.win_off + jb) * kBinRecLen;
        br[0] = bn[0];
        br[1] = bn[2];
        br[2] = bn[3];
        br[3] = outside ? 0.0 : 1.0;  // the seed itself is per species (H)
        br[4] = 0.0;
        br[5] = 0.0;
        block_offsets(Sh, T, jb, bn, br[6], br[7], bref);
      }
    }
  }
  // rate pieces: sum over the 16 bins (lanes col) of each species grp + 4v
#pragma unroll
  for (int v = 0; v < 4; v++)
    for (int o = 1; o < 16; o <<= 1) a[v] += __shfl_xor(a[v], o, 64);
  A0 = wave_sum(A0);
  A1 = wave_sum(A1);
  A2 = wave_sum(A2);
  if (col == 0) {
#pragma unroll
    for (int v = 0; v < 4; v++) red[wave][grp + 4 * v] = a[v];
  }
  if (lane == 0) {
    red[wave][GS_MAX_SPECIES] = A0;
    red[wave][GS_MAX_SPECIES + 1] = A1;
    red[wave][GS_MAX_SPECIES + 2] = A2;
  }
  if (bad) atomicOr(&bad_s, bad);
  const double tot = block_sum(sum, lds);  // its barriers also order red and bad_s
  if (threadIdx.x == 0) {
    nllp[T.nllp_off + blockIdx.x] = tot;
    badp[T.nllp_off + blockIdx.x] = bad_s;
  }
  const int e = threadIdx.x;
  if (e < S || (e >= GS_MAX_SPECIES && e < GS_MAX_SPECIES + 3)) {
    const double s = red[0][e] + red[1][e] + red[2][e] + red[3][e];
    const long long row = T.vpart_off + (e < GS_MAX_SPECIES ? 0 : T.hblocks) + blockIdx.x;
    vpart[row * kVLen + e] = s;
  }
}

hipError_t launch_bins2(const BatchView &v, const double *theta, double *mu_out, const uint8_t *active,
                        hipStream_t st) {
  if (v.n2d == 0 || v.max_bin_blocks2 == 0) return hipSuccess;  // no joint 2-D toys (all multivariate)
  const size_t lds = sizeof(double) * 4 * v.max_psd_sk;
  if (v.iter2 == 1)
    hipLaunchKernelGGL(k_bins2<true>, dim3(v.max_bin_blocks2, v.n2d), dim3(kBlock), lds, st, v.list2d, v.toys, v.shapes,
                       theta, v.stride, v.F, v.P, v.dP, v.cnt, v.nsum, v.iter2, active, v.nllp, v.badp, v.binrec, v.bref,
                       v.H, v.vpart, mu_out);
  else
    hipLaunchKernelGGL(k_bins2<false>, dim3(v.max_bin_blocks2, v.n2d), dim3(kBlock), lds, st, v.list2d, v.toys,
                       v.shapes, theta, v.stride, v.F, v.P, v.dP, v.cnt, v.nsum, v.iter2, active, v.nllp, v.badp,
                       v.binrec, v.bref, v.H, v.vpart, mu_out);
  return hipGetLastError();
}

// ------------------------------------------ multivariate slice likelihood --
// The paper's multivariate likelihood (section 2.4, cost model Eq.3): the
// energy histogram's Poisson likelihood (counts summed over the pulse-shape
// bins) plus, per energy slice i, the likelihood of the slice's pulse-shape
// histogram n_ik given its total n_i.: n_i. ln mu_i. - sum_k n_ik ln mu_ik with
// mu_ik = eps sum_s R_s N_si P_sk and N_si = sum_{j in i} F_js.  Its gradient
// with respect to F_js is R_s c_js, c_js = sum_d eps_d (1 - n_dj/mu_dj) +
// sigma_s(slice of j), so the per-species adjoint takes H_js = dx_j c_js as
// for the joint 2-D likelihood.  Counts of a multivariate toy are stored as
// its energy histogram [d][j] followed by its slices' histograms [d][i][k].

// Deterministic OR over a wavefront.
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
  uint32_t r = 0u;
  for (uint32_t bit = 1u; bit <= 2u; bit <<= 1)
    if (__ballot((v & bit) != 0u) != 0ull) r |= bit;
  return r;
}

// One wave per (toy, slice): lane s sums N_si over the slice's bins; lanes over
// k form the piece, the seeds sigma_si = sum_d eps_d (n_di./mu_di. -
// sum_k n_dik P_sk/mu_dik) and the slice's partial of the pulse-shape
// nuisance gradient, -sum_dk eps_d (n_dik/mu_dik) sum_s R_s N_si dP_sk/dnu.
__global__ __launch_bounds__(64) void k_mv_slice(const int *__restrict__ toy_list, const ToyDev *__restrict__ toys,
                                                 const ShapeDev *__restrict__ shapes, const double *__restrict__ theta,
                                                 int stride, const double *__restrict__ F, const double *__restrict__ P,
                                                 const double *__restrict__ dP, const double *__restrict__ cnt,
                                                 const int *__restrict__ sedge, const uint8_t *__restrict__ active,
                                                 double *__restrict__ sig, double *__restrict__ nllp,
                                                 uint32_t *__restrict__ badp, double *__restrict__ vpart) {
  const int t = toy_of(toy_list, blockIdx.y), i = blockIdx.x, lane = threadIdx.x;
  if (active && !active[t]) return;
  const ToyDev &T = toys[t];
  if (!T.mv || i >= T.n_slices) return;
  const ShapeDev &Sh = shapes[T.shape];
  const int S = T.S, K = T.K;
  const double *th = theta + (size_t)t * stride;
  const int j0 = sedge[T.slice_off + i], j1 = sedge[T.slice_off + i + 1];
  double N = 0.0;
  if (lane < S)
    for (int j = j0; j < j1; j++) N += F[fh_at(T, lane, j)];
  const double RN = lane < S ? th[Sh.sp_of[lane]] * N : 0.0;
  double rn[GS_MAX_SPECIES];
#pragma unroll
  for (int s = 0; s < GS_MAX_SPECIES; s++) rn[s] = __shfl(RN, s, 64);  // R_s N_si, wave-uniform
  const double *Pt = P + T.psd_off, *dPt = dP + 3 * T.psd_off;
  const double *sc = cnt + T.cnt_off + (long long)T.D * T.L;  // the slices' histograms [d][slice][k]
  double piece = 0.0, a[3] = {0.0, 0.0, 0.0}, sigma[GS_MAX_SPECIES];
#pragma unroll
  for (int s = 0; s < GS_MAX_SPECIES; s++) sigma[s] = 0.0;
  uint32_t bad = 0u;
  for (int d = 0; d < T.D; d++) {
    const double eps = T.exposure[d];
    double sg[GS_MAX_SPECIES], nsum = 0.0;
#pragma unroll
    for (int s = 0; s < GS_MAX_SPECIES; s++) sg[s] = 0.0;
    for (int k = lane; k < K; k += 64) {
      const double n = sc[((long long)d * T.n_slices + i) * K + k];
      nsum += n;
      if (!(n > 0.0)) continue;
      double m = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0;
#pragma unroll
      for (int s = 0; s < GS_MAX_SPECIES; s++)
        if (s < S) {
          m = __fma_rn(rn[s], Pt[(size_t)s * K + k], m);
          const double *dp = dPt + ((size_t)s * K + k) * 3;
          m0 = __fma_rn(rn[s], dp[0], m0);
          m1 = __fma_rn(rn[s], dp[1], m1);
          m2 = __fma_rn(rn[s], dp[2], m2);
        }
      const double mu = eps * m;
      if (!(mu > 0.0)) {
        bad |= kBadDomain;
        continue;
      }
      piece = __fma_rn(-n, log(mu), piece);
      double q = n / mu;
      if (!isfinite(q)) {
        bad |= kBadRange;
        q = 0.0;
      }
#pragma unroll
      for (int s = 0; s < GS_MAX_SPECIES; s++)
        if (s < S) sg[s] = __fma_rn(-q, Pt[(size_t)s * K + k], sg[s]);
      a[0] = __fma_rn(-q * eps, m0, a[0]);
      a[1] = __fma_rn(-q * eps, m1, a[1]);
      a[2] = __fma_rn(-q * eps, m2, a[2]);
    }
    wave_sum_n(sg, S);
    const double nd = wave_sum(nsum);  // n_di.
    double tot = 0.0;
#pragma unroll
    for (int s = 0; s < GS_MAX_SPECIES; s++) tot += rn[s];
    const double mud = eps * tot;       // mu_di.
    double q0 = 0.0;
    if (nd > 0.0) {
      if (!(mud > 0.0)) {
        bad |= kBadDomain;
      } else {
        if (lane == 0) piece = __fma_rn(nd, log(mud), piece);
        q0 = nd / mud;
        if (!isfinite(q0)) {
          bad |= kBadRange;
          q0 = 0.0;
        }
      }
    }
#pragma unroll
    for (int s = 0; s < GS_MAX_SPECIES; s++) sigma[s] = __fma_rn(eps, sg[s] + q0, sigma[s]);
  }
  piece = wave_sum(piece);
  a[0] = wave_sum(a[0]);
  a[1] = wave_sum(a[1]);
  a[2] = wave_sum(a[2]);
  bad = wave_or(bad);
  if (lane < S) {
    double v = 0.0;
#pragma unroll
    for (int s = 0; s < GS_MAX_SPECIES; s++) v = s == lane ? sigma[s] : v;
    sig[T.sig_off + (long long)i * S + lane] = v;
  }
  if (lane == 0) {
    nllp[T.nllp_off + T.eblocks + i] = piece;
    badp[T.nllp_off + T.eblocks + i] = bad;
    double *vp = vpart + (T.vpart_off + T.hblocks + T.eblocks + i) * kVLen + GS_MAX_SPECIES;
    vp[0] = a[0];
    vp[1] = a[1];
    vp[2] = a[2];
  }
}

// One thread per (window bin j, species slot q), kHTile bins per block: the
// energy histogram's Poisson terms (block partial of -ln L), the per-species
// seeds H_jq = dx_j c_jq for the adjoint, the bin record, and the block
// partial of the rate gradient sum_j F_jq c_jq.
__global__ __launch_bounds__(256) void k_mv_bins(const int *__restrict__ toy_list, const ToyDev *__restrict__ toys,
                                                 const ShapeDev *__restrict__ shapes, const double *__restrict__ theta,
                                                 int stride, const double *__restrict__ F, const double *__restrict__ cnt,
                                                 const int *__restrict__ sedge, const double *__restrict__ sig,
                                                 const uint8_t *__restrict__ active, double *__restrict__ binrec,
                                                 double *__restrict__ bref, double *__restrict__ H,
                                                 double *__restrict__ nllp, uint32_t *__restrict__ badp,
                                                 double *__restrict__ vpart) {
  __shared__ double red[kHTile][GS_MAX_SPECIES];
  __shared__ double lds[8];
  __shared__ uint32_t bad_s;
  const int t = toy_of(toy_list, blockIdx.y), blk = blockIdx.x;
  if (active && !active[t]) return;
  const ToyDev &T = toys[t];
  if (!T.mv || blk >= T.eblocks) return;
  const ShapeDev &Sh = shapes[T.shape];
  const int S = T.S, jj = threadIdx.x / GS_MAX_SPECIES, q = threadIdx.x % GS_MAX_SPECIES;
  const double *th = theta + (size_t)t * stride;
  if (threadIdx.x == 0) bad_s = 0u;
  __syncthreads();
  const int b = blk * kHTile + jj;
  double a = 0.0, term_sum = 0.0;
  if (b < T.L) {
    const double *Fr = F + fh_at(T, 0, b);
    double mu1 = 0.0;
    for (int s = 0; s < S; s++) mu1 = __fma_rn(th[Sh.sp_of[s]], Fr[s], mu1);
    double e = 0.0;
    uint32_t bad = 0u;
    for (int d = 0; d < T.D; d++) {
      const double mu = T.exposure[d] * mu1;
      const double n = cnt[T.cnt_off + (long long)d * T.L + b];
      double term, g;
      bad |= poisson_term(mu, n, term, g);
      if (q == 0) term_sum += term;
      e = __fma_rn(T.exposure[d], g, e);
    }
    if (bad && q == 0) atomicOr(&bad_s, bad);
    // the slice of bin b: the last slice edge at or below it
    int lo = 0, hi = T.n_slices;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (sedge[T.slice_off + mid] <= b) lo = mid; else hi = mid;
    }
    const double *bn = Sh.bins + (size_t)(T.lo + b) * kBinLen;
    const bool outside = Sh.family == kGammaPE && !(bn[0] > 0.0);
    if (q < S) {
      const double c = e + sig[T.sig_off + (long long)lo * S + q];
      H[fh_at(T, q, b)] = outside ? 0.0 : bn[1] * c;
      a = Fr[q] * c;
    }
    if (q == 0) {
      double *br = binrec + (T.win_off + b) * kBinRecLen;
      br[0] = bn[0];
      br[1] = bn[2];
      br[2] = bn[3];
      br[3] = outside ? 0.0 : 1.0;  // the seed itself is per species (H)
      br[4] = 0.0;
      br[5] = 0.0;
      block_offsets(Sh, T, b, bn, br[6], br[7], bref);
    }
  }
  red[jj][q] = a;
  const double tot = block_sum(term_sum, lds);  // its barriers also order red and bad_s
  if (threadIdx.x < S) {
    double v = red[0][threadIdx.x];
    for (int j = 1; j < kHTile; j++) v += red[j][threadIdx.x];
    vpart[(T.vpart_off + blk) * kVLen + threadIdx.x] = v;
  }
  if (threadIdx.x < 3) vpart[(T.vpart_off + T.hblocks + blk) * kVLen + GS_MAX_SPECIES + threadIdx.x] = 0.0;
  if (threadIdx.x == 0) {
    nllp[T.nllp_off + blk] = tot;
    badp[T.nllp_off + blk] = bad_s;
  }
}

// Expected counts of multivariate toys (the same joint expectation mu_djk as the
// 2-D model's), for gs_expected: one thread per (window bin, pulse-shape bin).
__global__ __launch_bounds__(256) void k_mv_expect(const int *__restrict__ toy_list, const ToyDev *__restrict__ toys,
                                                   const ShapeDev *__restrict__ shapes,
                                                   const double *__restrict__ theta, int stride,
                                                   const double *__restrict__ F, const double *__restrict__ P,
                                                   double *__restrict__ mu_out) {
  const int t = toy_of(toy_list, blockIdx.y);
  const ToyDev &T = toys[t];
  if (!T.mv) return;
  const ShapeDev &Sh = shapes[T.shape];
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)T.L * T.K) return;
  const int b = (int)(e / T.K), k = (int)(e - (long long)b * T.K);
  const double *th = theta + (size_t)t * stride;
  double M = 0.0;
  for (int s = 0; s < T.S; s++)
    M = __fma_rn(th[Sh.sp_of[s]] * F[fh_at(T, s, b)], P[T.psd_off + (long long)s * T.K + k], M);
  for (int d = 0; d < T.D; d++) mu_out[((long long)d * T.L + b) * T.K + k] = T.exposure[d] * M;
}

hipError_t launch_mv(const BatchView &v, const double *theta, double *mu_out, const uint8_t *active, hipStream_t st) {
  if (!v.has_mv || v.n2d == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mv_slice, dim3(v.max_slices, v.n2d), dim3(64), 0, st, v.list2d, v.toys, v.shapes, theta,
                     v.stride, v.F, v.P, v.dP, v.cnt, v.sedge, active, v.sig, v.nllp, v.badp, v.vpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mv_bins, dim3(v.max_eblocks, v.n2d), dim3(kHTile * GS_MAX_SPECIES), 0, st, v.list2d, v.toys,
                     v.shapes, theta, v.stride, v.F, v.cnt, v.sedge, v.sig, active, v.binrec, v.bref, v.H, v.nllp,
                     v.badp, v.vpart);
  e = hipGetLastError();
  if (e != hipSuccess || !mu_out) return e;
  hipLaunchKernelGGL(k_mv_expect, dim3((v.max_mv_cells + kBlock - 1) / kBlock, v.n2d), dim3(kBlock), 0, st,
                     v.list2d, v.toys, v.shapes, theta, v.stride, v.F, v.P, mu_out);
  return hipGetLastError();
}

}  // namespace gs

