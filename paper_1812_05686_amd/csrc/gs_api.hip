// gs_api.hip -- host side of libgs: descriptor validation, device layout of
// models and batches, synchronous single-model calls, batched calls and the
// host quasi-Newton driver.  Every step of an evaluation runs in the kernels
// of gs_kernels.hip; this file only allocates, copies and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <tuple>
#include <chrono>
#include <vector>

#include "gs_impl.h"
#include "gs_qn.h"

using namespace gs;

namespace {

thread_local std::string g_err;

gs_status fail(gs_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(e_ == hipErrorOutOfMemory ? GS_ERR_OOM : GS_ERR_DEVICE, "%s: %s (%s:%d)", #expr, \
                  hipGetErrorString(e_), __FILE__, __LINE__);                            \
  } while (0)

int n_resp(int fam) { return fam == GS_RESP_TEMPLATE ? 0 : fam == GS_RESP_GAUSS_E ? 2 : 5; }

int num_params(const gs_model_desc *d) {
  return d->n_species + n_resp(d->family) + (d->n_psd > 0 ? 3 : 0);
}

// Host-side descriptor check; returns n_params or -1 with g_err set.
int validate(const gs_model_desc *d) {
  auto bad = [](const char *fmt, auto... a) {
    char b[256];
    snprintf(b, sizeof b, fmt, a...);
    g_err = b;
    return -1;
  };
  if (!d) return bad("null descriptor");
  if (d->family < 0 || d->family > GS_RESP_EMG_PE) return bad("unknown response family %d", d->family);
  if (d->exact_bins != 0 && d->exact_bins != 1) return bad("exact_bins must be 0 or 1");
  if (d->family >= GS_RESP_GENGAMMA_PE || d->exact_bins) {
    if (d->n_psd != 0) return bad("family %d / exact bins: one-dimensional models only", d->family);
    if (d->family == GS_RESP_TEMPLATE) return bad("templates have no bin integrals");
    if (d->family == GS_RESP_SPOIS_PE && d->exact_bins) return bad("the scaled Poisson has no exact bin content");
  }
  if (d->family == GS_RESP_GENGAMMA_PE && !(d->shape > 0 && std::isfinite(d->shape)))
    return bad("generalized gamma power %g must be positive", d->shape);
  if (d->family == GS_RESP_EMG_PE && !(d->shape > 0 && d->shape < 1))
    return bad("modified Gaussian tail fraction %g outside (0, 1)", d->shape);
  if (d->n_species < 1 || d->n_species > GS_MAX_SPECIES)
    return bad("n_species %d outside 1..%d", d->n_species, GS_MAX_SPECIES);
  if (d->n_true < 1) return bad("n_true %d < 1", d->n_true);
  if (!(d->e_step > 0) || !std::isfinite(d->e_lo) || !std::isfinite(d->e_step)) return bad("bad true grid");
  if (!d->line_energy) return bad("line_energy is NULL");
  int n_grid = 0;
  for (int s = 0; s < d->n_species; s++) {
    if (std::isnan(d->line_energy[s])) {
      n_grid++;
    } else if (!std::isfinite(d->line_energy[s])) {
      return bad("line energy of species %d is not finite", s);
    }
  }
  if (n_grid > 0 && !d->spectra) return bad("spectra is NULL");
  if (d->family == GS_RESP_TEMPLATE) {
    if (n_grid != d->n_species) return bad("template models have no line species");
    if (d->n_true != d->n_reco) return bad("templates need n_true == n_reco (%d != %d)", d->n_true, d->n_reco);
    if (d->n_psd != 0) return bad("template models are one-dimensional (n_psd = 0)");
  }
  for (int s = 0; s < d->n_species; s++) {
    if (!std::isnan(d->line_energy[s])) continue;
    for (int i = 0; i < d->n_true; i++) {
      double w = d->spectra[(size_t)s * d->n_true + i];
      if (!(w >= 0) || !std::isfinite(w)) return bad("spectrum %d cell %d is negative or not finite", s, i);
    }
  }
  if (d->n_reco < 1 || !d->reco_edges) return bad("no reco bins");
  if (!std::isfinite(d->reco_edges[0])) return bad("reco_edges[0] is not finite");
  for (int j = 0; j < d->n_reco; j++)
    if (!(d->reco_edges[j + 1] > d->reco_edges[j]) || !std::isfinite(d->reco_edges[j + 1]))
      return bad("reco_edges not strictly increasing at %d", j);
  if (d->n_psd < 0) return bad("n_psd < 0");
  if (d->n_psd > 0) {
    if (!d->psd_edges || !d->psd_mix) return bad("psd_edges / psd_mix is NULL");
    if (!std::isfinite(d->psd_edges[0]) || !std::isfinite(d->psd_edges[d->n_psd]))
      return bad("psd_edges not finite");
    for (int k = 0; k < d->n_psd; k++)
      if (!(d->psd_edges[k + 1] > d->psd_edges[k])) return bad("psd_edges not strictly increasing at %d", k);
    for (int s = 0; s < d->n_species; s++) {
      const double *m = d->psd_mix + 5 * s;
      if (!(m[0] > 0 && m[0] < 1) || !(m[2] > 0) || !(m[4] > 0) || !std::isfinite(m[1]) || !std::isfinite(m[3]))
        return bad("psd_mix of species %d invalid", s);
    }
  }
  if (d->n_slices < 0) return bad("n_slices < 0");
  if (d->n_slices > 0) {
    if (d->n_psd < 1) return bad("energy slices need a secondary observable (n_psd > 0)");
    if (!d->slice_edges) return bad("slice_edges is NULL");
    if (d->slice_edges[0] != d->win_lo || d->slice_edges[d->n_slices] != d->win_hi)
      return bad("slice_edges must start at win_lo and end at win_hi");
    for (int i = 0; i < d->n_slices; i++)
      if (!(d->slice_edges[i + 1] > d->slice_edges[i])) return bad("slice_edges not strictly increasing at %d", i);
  }
  if (d->n_datasets < 1 || d->n_datasets > GS_MAX_DATASETS)
    return bad("n_datasets %d outside 1..%d", d->n_datasets, GS_MAX_DATASETS);
  if (!d->exposure) return bad("exposure is NULL");
  for (int k = 0; k < d->n_datasets; k++)
    if (!(d->exposure[k] > 0) || !std::isfinite(d->exposure[k])) return bad("exposure %d not positive", k);
  if (!(d->win_lo >= 0 && d->win_lo < d->win_hi && d->win_hi <= d->n_reco))
    return bad("window [%d, %d) invalid for %d bins", d->win_lo, d->win_hi, d->n_reco);
  if (!d->counts) return bad("counts is NULL");
  const int K = std::max(d->n_psd, 1);
  for (int k = 0; k < d->n_datasets; k++)
    for (int j = d->win_lo; j < d->win_hi; j++)
      for (int q = 0; q < K; q++) {
        double n = d->counts[((size_t)k * d->n_reco + j) * K + q];
        if (!(n >= 0) || !std::isfinite(n)) return bad("count (%d,%d,%d) negative or not finite", k, j, q);
      }
  if (d->family != GS_RESP_GAUSS_E && d->family != GS_RESP_TEMPLATE && !(d->birks_A > 0))
    return bad("birks_A must be > 0");
  const int P = num_params(d);
  if (d->pull_sigma)
    for (int p = 0; p < P; p++)
      if (d->pull_sigma[p] > 0 && (!d->pull_centre || !std::isfinite(d->pull_centre[p])))
        return bad("pull %d has no finite centre", p);
  return P;
}

// ------------------------------------------------------------- batch ----
struct ShapeKey {
  const void *spectra, *lines, *edges, *pe, *pm;
  int fam, n_true, S, n_reco, n_psd;
  double e_lo, e_step, A;
  int exact;
  double shape;
  bool operator<(const ShapeKey &o) const {
    return std::tie(spectra, lines, edges, pe, pm, fam, n_true, S, n_reco, n_psd, e_lo, e_step, A, exact, shape) <
           std::tie(o.spectra, o.lines, o.edges, o.pe, o.pm, o.fam, o.n_true, o.S, o.n_reco, o.n_psd, o.e_lo,
                    o.e_step, o.A, o.exact, o.shape);
  }
};

struct DevBuf {
  void *p = nullptr;
  size_t n = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

// Layout knobs of a batch: the split-K target (work-groups the fold and the
// adjoint aim for when the batch alone is smaller), cells per k_cellgrad block,
// rounds of window bins per k_bins2 block, and waves per adjoint workgroup.
struct Knobs {
  int target_wg, grad_cells, iter2, adj_waves;
};
// Work-buffer sizes (elements) and item counts a layout needs.
struct LayoutSizes {
  long long fpart, fspart, apart, nllp, gpart, vpart;
  size_t n_fold, n_adj;
};

struct gs_batch {
  int device = 0;
  int n_toys = 0, stride = 0;
  std::vector<ShapeDev> shapes_h;
  std::vector<ToyDev> toys_h;
  std::vector<FoldItem> fold_h;   // per-species fold items, every toy
  std::vector<FoldItem> fold1_h;  // 1-D fold items, 1-D toys
  std::vector<AdjItem> adj_h;
  // layout knobs in force, the candidates the autotuner tries, and the
  // capacities (largest candidate) the work buffers and item arrays hold
  Knobs knobs{};
  std::vector<Knobs> candidates;
  LayoutSizes cap{}, cur{};  // largest candidate; the layout in force
  FoldItem *d_fold_items = nullptr;
  AdjItem *d_adj_items = nullptr;
  ToyDev *d_toys = nullptr;
  std::vector<void *> allocs;
  BatchView v{};
  bool has_2d = false;
  // kernel timing (gs_batch_set_profiling): event pairs around each launch
  bool prof = false;
  struct Timed {
    int kernel;
    hipEvent_t a, b;
  };
  std::vector<Timed> pending;
  std::vector<hipEvent_t> ev_free;
  double prof_ms[GS_K_COUNT] = {};
  long long prof_n[GS_K_COUNT] = {};
  // batched fits: device quasi-Newton state and the captured iteration graph
  bool qn_ready = false;
  QNView q{};
  double *e_nll = nullptr, *e_grad = nullptr, *d_scale = nullptr;
  uint32_t *e_st = nullptr;
  int *d_count = nullptr, *h_count = nullptr;
  std::vector<int> trace_active;  // last gs_fit_batched: toys still running after each graph launch
  std::vector<double> trace_ms;   // and the host time since the call started
  hipStream_t fit_stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // batches with both 1-D and 2-D toys: the 2-D chain runs on a stream of its
  // own, forked from the caller's stream after the cell records and joined
  // before the gradient chain (default priority, as every stream here)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipGraphExec_t graph = nullptr;
  int graph_k = 0, graph_max_iter = -1;
  double graph_tol = -1.0;
  bool graph_compact = false;  // the instantiated graph covers a compacted toy list
  // compacted toy and work-item lists of a batched fit (device copies)
  int *d_toy_list = nullptr, *d_list1 = nullptr, *d_list2 = nullptr, *d_listt = nullptr, *d_tgroup = nullptr;
  // discovery test: the null fit's start and free mask, iteration counts
  double *d_th0_null = nullptr;
  uint8_t *d_free_null = nullptr;
  int32_t *d_iters_tmp = nullptr;
  FoldItem *d_fold_c = nullptr;
  AdjItem *d_adj_c = nullptr;

  ~gs_batch() {
    if (graph) (void)hipGraphExecDestroy(graph);
    if (fit_stream) (void)hipStreamDestroy(fit_stream);
    if (side) (void)hipStreamDestroy(side);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (h_count) (void)hipHostFree(h_count);
    for (auto &t : pending) {
      (void)hipEventDestroy(t.a);
      (void)hipEventDestroy(t.b);
    }
    for (auto e : ev_free) (void)hipEventDestroy(e);
    for (void *p : allocs) (void)hipFree(p);
  }
  hipEvent_t event() {
    hipEvent_t e = nullptr;
    if (!ev_free.empty()) {
      e = ev_free.back();
      ev_free.pop_back();
    } else {
      (void)hipEventCreate(&e);
    }
    return e;
  }
  template <class T>
  hipError_t alloc(T **p, size_t n) {
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void **)p, n * sizeof(T));
    if (e == hipSuccess) allocs.push_back(*p);
    return e;
  }
};

struct gs_model {
  gs_batch *b = nullptr;
  hipStream_t stream = nullptr;
  int P = 0;
  double *d_theta = nullptr, *d_nll = nullptr, *d_grad = nullptr, *d_mu = nullptr;
  uint32_t *d_status = nullptr;
  double *h_theta = nullptr, *h_out = nullptr;  // pinned staging
  uint32_t *h_status = nullptr;
  std::vector<double> cached_resp;  // response params of the cached per-species fold
  bool cache_valid = false;
  int n_mu = 0;
};

namespace {

// Split-K choice: about 8 workgroups per CU when a batch is small; large
// batches keep whole tiles (one chunk) so no partial sums are needed.
constexpr int kTargetWG = 2048;
// Default banding cut: the skipped mass per bin, sum_s |R_s| eps dx e^cut, is
// then at most about 3e-17 counts at the largest rates and bin widths here,
// 3% of the 1e-12 relative budget of a bin holding 1e-3 counts.
constexpr double kDefaultLogCut = -52.0;

// Splits work items by the kind of their toy (1-D first, then 2-D: items of a
// toy stay contiguous and in order) and uploads them to dst; sets the view's
// per-kind pointers into dst.  fi: per-species fold items (every toy), fi1:
// 1-D fold items (1-D toys), stored after them; dst_f holds both.
static gs_status upload_items(gs_batch *B, const std::vector<FoldItem> &fi, const std::vector<FoldItem> &fi1,
                              const std::vector<AdjItem> &ai, FoldItem *dst_f, AdjItem *dst_a, BatchView &v,
                              hipStream_t st) {
  std::vector<FoldItem> f;
  std::vector<AdjItem> a;
  for (int kind = 0; kind < 2; kind++) {
    for (const FoldItem &it : fi)
      if (B->toys_h[it.toy].two_d == kind) f.push_back(it);
    for (const AdjItem &it : ai)
      if (B->toys_h[it.toy].two_d == kind) a.push_back(it);
    if (kind == 0) {
      v.n_fold1s = (int)f.size();
      v.n_adj1 = (int)a.size();
    }
  }
  v.n_fold_items = (int)f.size();
  v.n_fold2 = v.n_fold_items - v.n_fold1s;
  v.n_adj2 = (int)a.size() - v.n_adj1;
  for (const FoldItem &it : fi1)
    if (!B->toys_h[it.toy].two_d) f.push_back(it);
  v.n_fold1 = (int)f.size() - v.n_fold_items;
  if (!f.empty()) HIP_TRY(hipMemcpyAsync(dst_f, f.data(), sizeof(FoldItem) * f.size(), hipMemcpyHostToDevice, st));
  if (!a.empty()) HIP_TRY(hipMemcpyAsync(dst_a, a.data(), sizeof(AdjItem) * a.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));  // the host vectors go out of scope
  v.fold_items = dst_f;
  v.adj_items = dst_a;
  v.n_adj_items = (int)a.size();
  v.fold2 = dst_f + v.n_fold1s;
  v.fold1 = dst_f + v.n_fold_items;
  v.adj1 = dst_a;
  v.adj2 = dst_a + v.n_adj1;
  return GS_OK;
}

// The layout knobs the autotuner tries: split-K targets, one or four cells per
// k_cellgrad thread, one or kIter2Large rounds per 2-D block (2-D batches),
// one or kWaves waves per adjoint workgroup.
static std::vector<Knobs> layout_candidates(const gs_batch *B) {
  // split-K targets that give the same chunk counts as an earlier one give the
  // same layout: only the first (the default target comes first) is kept
  long long tiles_f = 0, tiles_a = 0;
  for (const ToyDev &T : B->toys_h) {
    tiles_f += (T.L + kFoldTile - 1) / kFoldTile;
    tiles_a += (T.n_cell + kTile - 1) / kTile;
  }
  tiles_f = std::max(tiles_f, 1LL);  // template toys have no cells (and a batch of them no fold)
  tiles_a = std::max(tiles_a, 1LL);
  std::vector<std::pair<long long, long long>> seen;
  std::vector<Knobs> c;
  for (int wg : {kTargetWG, 1024, 4096, 8192}) {
    const std::pair<long long, long long> nch{std::max<long long>(1, (wg + tiles_f - 1) / tiles_f),
                                              std::max<long long>(1, (wg + tiles_a - 1) / tiles_a)};
    if (std::find(seen.begin(), seen.end(), nch) != seen.end()) continue;
    seen.push_back(nch);
    for (int gc : {kBlock, kGradCellsLarge})
      for (int it : {1, kIter2Large})
        for (int aw : {1, kWaves}) {
          if (it != 1 && !B->v.has_2d) continue;
          c.push_back({wg, gc, it, aw});
        }
  }
  return c;
}

// The default layout: a split-K target of kTargetWG work-groups; four cells per
// k_cellgrad thread, kIter2Large 2-D rounds and one-wave adjoint workgroups
// once the batch gives at least kGradLargeBlocks blocks of kBlock cells, cell
// tiles of the adjoint (so one model still fills the GPU).  A batch with both
// 1-D and 2-D toys keeps four-wave adjoint workgroups: beside the 2-D chain on
// the second stream they gave the faster step and, by more, the faster batched
// fits (their graphs run the same layout).
static Knobs default_knobs(const gs_batch *B) {
  long long grad_blocks = 0, bins2_blocks = 0, adj_tiles = 0;
  bool has_1d = false;
  for (const ToyDev &T : B->toys_h) {
    grad_blocks += (T.n_cell + kBlock - 1) / kBlock;
    adj_tiles += (T.n_cell + kTile - 1) / kTile;
    if (T.two_d) bins2_blocks += ((long long)T.L * T.K + kBlock - 1) / kBlock;
    has_1d = has_1d || (!T.two_d && !T.tmpl);
  }
  const bool forked = has_1d && bins2_blocks > 0;
  return {kTargetWG, grad_blocks >= kGradLargeBlocks ? kGradCellsLarge : kBlock,
          bins2_blocks >= kGradLargeBlocks ? kIter2Large : 1,
          adj_tiles >= kGradLargeBlocks && !forked ? 1 : kWaves};
}

static void grow(LayoutSizes &a, const LayoutSizes &b) {
  a.fpart = std::max(a.fpart, b.fpart);
  a.fspart = std::max(a.fspart, b.fspart);
  a.apart = std::max(a.apart, b.apart);
  a.nllp = std::max(a.nllp, b.nllp);
  a.gpart = std::max(a.gpart, b.gpart);
  a.vpart = std::max(a.vpart, b.vpart);
  a.n_fold = std::max(a.n_fold, b.n_fold);
  a.n_adj = std::max(a.n_adj, b.n_adj);
}

// Lays the batch out for knobs k on the host: every toy's chunk and block
// counts and partial-buffer offsets, the work items, and the view's largest
// grid sizes.  Returns the buffer sizes and item counts this layout needs.
static LayoutSizes layout(gs_batch *B, const Knobs &k) {
  BatchView &v = B->v;
  long long tiles_f = 0, tiles_a = 0;
  for (const ToyDev &T : B->toys_h) {
    tiles_f += (T.L + kFoldTile - 1) / kFoldTile;
    tiles_a += (T.n_cell + kTile - 1) / kTile;
  }
  tiles_f = std::max(tiles_f, 1LL);  // template toys have no cells (and a batch of them no fold)
  tiles_a = std::max(tiles_a, 1LL);
  const int nch_f = (int)std::max<long long>(1, (k.target_wg + tiles_f - 1) / tiles_f);
  const int nch_a = (int)std::max<long long>(1, (k.target_wg + tiles_a - 1) / tiles_a);
  v.grad_cells = k.grad_cells;
  v.iter2 = k.iter2;
  v.adj_waves = k.adj_waves;
  v.max_cell_blocks = v.max_bin_blocks = v.max_bin_blocks1 = v.max_bin_blocks2 = v.max_hblocks = 0;
  v.max_bin_blocks_t = 0;
  v.max_eblocks = 0;
  B->fold_h.clear();
  B->fold1_h.clear();
  B->adj_h.clear();
  LayoutSizes z{};
  // template blocks: the largest size whose launch still has kTmplMinBlocks
  // blocks (toys in groups of up to 16 share a block)
  v.tmpl_bins = kTmplBlockBins;
  for (int tb : {kTmplBlockBins, 256, 64}) {
    long long nb = 0;
    for (const ToyDev &T : B->toys_h)
      if (T.tmpl) nb += (T.L + tb - 1) / tb;
    v.tmpl_bins = tb;
    if (nb / kTmplGroup >= kTmplMinBlocks) break;
  }
  for (int t = 0; t < (int)B->toys_h.size(); t++) {
    ToyDev &T = B->toys_h[t];
    const ShapeDev &sh = B->shapes_h[T.shape];
    // chunk sizes: at least 128 cells (a multiple of the hull group) / 64 bins per chunk
    const int cpc = std::max(128, ((sh.n_cell + nch_f - 1) / nch_f + kGroup - 1) / kGroup * kGroup);
    T.fold_chunks = (sh.n_cell + cpc - 1) / cpc;
    const int bpc = std::max(64, (T.L + nch_a - 1) / nch_a);
    T.adj_chunks = (T.L + bpc - 1) / bpc;
    // 2-D: k_bins2 blocks of iter2 rounds of kWaves x 16 window bins (one round: 16 bins, the
    // waves splitting the pulse-shape tiles); each writes a row of rate pieces (the first
    // hblocks rows) and a row of nuisance pieces (the next bin_blocks)
    const int c2 = k.iter2 == 1 ? 16 : kWaves * 16 * k.iter2;
    T.bin_blocks = T.two_d  ? (T.L + c2 - 1) / c2
                   : T.tmpl ? (T.L + v.tmpl_bins - 1) / v.tmpl_bins
                            : (T.L + kBlock - 1) / kBlock;
    T.hblocks = T.two_d ? T.bin_blocks : 0;
    if (T.mv) {  // rows of k_mv_bins (energy blocks), then one per slice (k_mv_slice)
      T.eblocks = (T.L + kHTile - 1) / kHTile;
      T.hblocks = T.eblocks;
      T.bin_blocks = T.eblocks + T.n_slices;
    }
    // template toys keep one rate-gradient row per bin block where other toys keep one per cell block
    T.cell_blocks = T.tmpl ? T.bin_blocks : (sh.n_cell + k.grad_cells - 1) / k.grad_cells;
    T.vpart_off = z.vpart;
    T.fpart_off = z.fpart;
    T.fs_off = z.fspart;
    T.apart_off = z.apart;
    T.nllp_off = z.nllp;
    T.gpart_off = z.gpart;
    for (int b0 = 0; b0 < T.L; b0 += kFoldTile)
      for (int c = 0; c < T.fold_chunks; c++)
        B->fold_h.push_back({t, b0, c * cpc, std::min(sh.n_cell, (c + 1) * cpc), c});
    if (!T.two_d)
      for (int b0 = 0; b0 < T.L; b0 += kFoldTile1)
        for (int c = 0; c < T.fold_chunks; c++)
          B->fold1_h.push_back({t, b0, c * cpc, std::min(sh.n_cell, (c + 1) * cpc), c});
    for (int c0 = 0; c0 < sh.n_cell; c0 += kTile)
      for (int c = 0; c < T.adj_chunks; c++)
        B->adj_h.push_back({t, c0, c * bpc, std::min(T.L, (c + 1) * bpc), c});
    if (T.two_d) z.vpart += T.hblocks + T.bin_blocks;
    z.fpart += (long long)T.fold_chunks * T.L;
    z.fspart += (long long)T.fold_chunks * T.L * T.S;
    z.apart += (long long)T.adj_chunks * sh.n_cell * 3;
    z.nllp += T.bin_blocks;
    z.gpart += T.cell_blocks;
    if (!T.tmpl) v.max_cell_blocks = std::max(v.max_cell_blocks, T.cell_blocks);
    v.max_bin_blocks = std::max(v.max_bin_blocks, T.bin_blocks);
    if (T.mv) {
      v.max_eblocks = std::max(v.max_eblocks, T.eblocks);
    } else {
      int &mb = T.two_d ? v.max_bin_blocks2 : T.tmpl ? v.max_bin_blocks_t : v.max_bin_blocks1;
      mb = std::max(mb, T.bin_blocks);
      v.max_hblocks = std::max(v.max_hblocks, T.hblocks);
    }
  }
  z.n_fold = B->fold_h.size() + B->fold1_h.size();
  z.n_adj = B->adj_h.size();
  return z;
}

// Template toys in the order k_tmpl takes them: stably sorted by (shape,
// window, datasets), cut into groups of at most kTmplGroup that agree on all
// three; grp receives (first position in lt, count) per group.
static void tmpl_groups(const std::vector<ToyDev> &toys, std::vector<int> &lt, std::vector<int> &grp) {
  auto key = [&](int t) {
    const ToyDev &T = toys[t];
    return std::make_tuple(T.shape, T.lo, T.L, T.D);
  };
  std::stable_sort(lt.begin(), lt.end(), [&](int a, int b) { return key(a) < key(b); });
  grp.clear();
  for (int i = 0; i < (int)lt.size(); i++) {
    if (!grp.empty() && grp.back() < kTmplGroup && key(lt[grp[grp.size() - 2]]) == key(lt[i])) {
      grp.back()++;
    } else {
      grp.push_back(i);
      grp.push_back(1);
    }
  }
}

gs_status build_batch(const gs_model_desc *descs, int n_toys, int device, gs_batch **out) {
  if (!descs || n_toys < 1) return fail(GS_ERR_ARG, "need at least one descriptor");
  std::vector<int> P(n_toys);
  for (int t = 0; t < n_toys; t++) {
    P[t] = validate(&descs[t]);
    if (P[t] < 0) return fail(GS_ERR_ARG, "toy %d: %s", t, g_err.c_str());
    if (descs[t].n_psd > GS_MAX_PSD) return fail(GS_ERR_UNSUPPORTED, "toy %d: more than %d pulse-shape bins", t, GS_MAX_PSD);
  }
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(GS_ERR_DEVICE, "device %d not present (%d devices)", device, ndev);
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(GS_ERR_DEVICE, "device %d is %s; this library is built for gfx950", device, prop.gcnArchName);
  HIP_TRY(hipSetDevice(device));

  auto *B = new gs_batch();
  std::unique_ptr<gs_batch> guard(B);
  B->device = device;
  B->n_toys = n_toys;
  B->stride = *std::max_element(P.begin(), P.end());

  // ---- shapes (deduplicated by array identity) ----
  std::map<ShapeKey, int> shape_of;
  std::vector<int> toy_shape(n_toys);
  for (int t = 0; t < n_toys; t++) {
    const gs_model_desc &d = descs[t];
    const bool shaped = d.family == GS_RESP_GENGAMMA_PE || d.family == GS_RESP_EMG_PE;
    ShapeKey k{d.spectra, d.line_energy, d.reco_edges, d.psd_edges, d.psd_mix, d.family, d.n_true,
               d.n_species, d.n_reco, d.n_psd, d.e_lo, d.e_step, d.family == GS_RESP_GAUSS_E ? 0.0 : d.birks_A,
               d.exact_bins, shaped ? d.shape : 0.0};
    auto it = shape_of.find(k);
    if (it != shape_of.end()) {
      toy_shape[t] = it->second;
      continue;
    }
    const int id = (int)B->shapes_h.size();
    shape_of[k] = id;
    toy_shape[t] = id;
    ShapeDev sh{};
    sh.family = d.family;
    sh.n_true = d.n_true;
    sh.S = d.n_species;
    sh.n_reco = d.n_reco;
    sh.n_psd = d.n_psd;
    sh.birks_A = d.birks_A;
    sh.exact = d.exact_bins;
    sh.shape = d.shape;
    sh.gen = d.family >= GS_RESP_GENGAMMA_PE || d.exact_bins ? 1 : 0;
    std::vector<int> grid, line;
    for (int q = 0; q < d.n_species; q++) (std::isnan(d.line_energy[q]) ? grid : line).push_back(q);
    sh.Sg = (int)grid.size();
    sh.n_line = (int)line.size();
    sh.n_cell = d.family == GS_RESP_TEMPLATE ? 0 : d.n_true + sh.n_line;  // templates: no cells
    for (int q = 0; q < sh.Sg; q++) sh.sp_of[q] = grid[q];
    for (int q = 0; q < sh.n_line; q++) sh.sp_of[sh.Sg + q] = line[q];
    std::vector<double> cellE(sh.n_cell), wcell((size_t)d.n_true * std::max(sh.Sg, 1), 0.0);
    std::vector<double> wcellT(wcell.size(), 0.0);
    if (sh.n_cell > 0) {  // template shapes have no cells
      for (int i = 0; i < d.n_true; i++) cellE[i] = d.e_lo + (i + 0.5) * d.e_step;
      for (int q = 0; q < sh.n_line; q++) cellE[d.n_true + q] = d.line_energy[line[q]];
    }
    for (int i = 0; i < d.n_true; i++)
      for (int q = 0; q < sh.Sg; q++) {
        wcell[(size_t)i * sh.Sg + q] = d.spectra[(size_t)grid[q] * d.n_true + i];
        wcellT[(size_t)q * d.n_true + i] = d.spectra[(size_t)grid[q] * d.n_true + i];
      }
    double *cE, *wc, *wct, *bins, *edges;
    HIP_TRY(B->alloc(&cE, cellE.size()));
    HIP_TRY(B->alloc(&wc, wcell.size()));
    HIP_TRY(B->alloc(&wct, wcellT.size()));
    HIP_TRY(B->alloc(&bins, (size_t)d.n_reco * kBinLen));
    HIP_TRY(B->alloc(&edges, (size_t)d.n_reco + 1));
    HIP_TRY(hipMemcpy(cE, cellE.data(), cellE.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(wc, wcell.data(), wcell.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(wct, wcellT.data(), wcellT.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(edges, d.reco_edges, ((size_t)d.n_reco + 1) * 8, hipMemcpyHostToDevice));
    HIP_TRY(launch_bins_setup(bins, edges, d.n_reco, nullptr));
    sh.cellE = cE;
    sh.wcell = wc;
    sh.wcellT = wct;
    {  // padded per-cell weights over the internal species, for the per-species fold's staging
      std::vector<double> w16((size_t)std::max(sh.n_cell, 1) * GS_MAX_SPECIES, 0.0);
      for (int i = 0; i < d.n_true && i < sh.n_cell; i++)
        for (int q = 0; q < sh.Sg; q++) w16[(size_t)i * GS_MAX_SPECIES + q] = wcell[(size_t)i * sh.Sg + q];
      for (int q = 0; q < sh.n_line; q++) w16[(size_t)(d.n_true + q) * GS_MAX_SPECIES + sh.Sg + q] = 1.0;
      double *wd;
      HIP_TRY(B->alloc(&wd, w16.size()));
      HIP_TRY(hipMemcpy(wd, w16.data(), w16.size() * 8, hipMemcpyHostToDevice));
      sh.w16 = wd;
    }
    sh.bins = bins;
    sh.edges = edges;
    // uniform binning (midpoints within 1e-6 of a bin width of a lattice): the
    // support search guesses bin indices arithmetically
    sh.bx0 = 0.5 * (d.reco_edges[0] + d.reco_edges[1]);
    sh.bw = 0.0;
    if (d.n_reco > 1) {
      const double xl = 0.5 * (d.reco_edges[d.n_reco - 1] + d.reco_edges[d.n_reco]);
      const double w = (xl - sh.bx0) / (d.n_reco - 1);
      bool uni = w > 0.0;
      for (int j = 0; uni && j < d.n_reco; j++)
        uni = std::fabs(0.5 * (d.reco_edges[j] + d.reco_edges[j + 1]) - (sh.bx0 + j * w)) <= 1e-6 * w;
      if (uni) sh.bw = w;
    }
    if (d.n_psd > 0) {
      std::vector<double> psd(2 * (size_t)d.n_psd), mix(5 * (size_t)d.n_species);
      for (int k = 0; k < d.n_psd; k++) {
        psd[2 * k] = (d.psd_edges[k] + d.psd_edges[k + 1]) * 0.5;
        psd[2 * k + 1] = d.psd_edges[k + 1] - d.psd_edges[k];
      }
      for (int q = 0; q < d.n_species; q++)
        for (int c = 0; c < 5; c++) mix[5 * q + c] = d.psd_mix[5 * sh.sp_of[q] + c];
      double *pd, *mx;
      HIP_TRY(B->alloc(&pd, psd.size()));
      HIP_TRY(B->alloc(&mx, mix.size()));
      HIP_TRY(hipMemcpy(pd, psd.data(), psd.size() * 8, hipMemcpyHostToDevice));
      HIP_TRY(hipMemcpy(mx, mix.data(), mix.size() * 8, hipMemcpyHostToDevice));
      sh.psd = pd;
      sh.mix = mx;
    }
    B->shapes_h.push_back(sh);
  }

  // ---- toys: the fields and offsets that do not depend on the layout knobs ----
  long long cell_off = 0, win_off = 0, fh_off = 0, bref_off = 0, cnt_off = 0, pull_off = 0;
  long long cflag_off = 0, psd_off = 0, ghull_off = 0, slice_off = 0, sig_n = 0;
  std::vector<double> cnt_h, nsum_h, pc_h, ps_h;
  std::vector<int> sedge_h;
  BatchView &v = B->v;
  for (int t = 0; t < n_toys; t++) {
    const gs_model_desc &d = descs[t];
    const ShapeDev &sh = B->shapes_h[toy_shape[t]];
    ToyDev T{};
    T.shape = toy_shape[t];
    T.D = d.n_datasets;
    T.lo = d.win_lo;
    T.L = d.win_hi - d.win_lo;
    T.P = P[t];
    T.K = std::max(d.n_psd, 1);
    T.two_d = d.n_psd > 0 ? 1 : 0;
    T.tmpl = d.family == GS_RESP_TEMPLATE ? 1 : 0;
    T.mv = d.n_slices > 0 ? 1 : 0;
    T.n_slices = d.n_slices;
    T.slice_off = slice_off;
    T.sig_off = sig_n;
    if (T.mv) {
      sig_n += (long long)d.n_slices * sh.S;
      for (int i = 0; i <= d.n_slices; i++) sedge_h.push_back(d.slice_edges[i] - d.win_lo);
      slice_off += d.n_slices + 1;
      v.has_mv = true;
      v.max_slices = std::max(v.max_slices, d.n_slices);
      v.max_mv_cells = std::max(v.max_mv_cells, (d.win_hi - d.win_lo) * d.n_psd);
    }
    T.psd_off = psd_off;
    if (T.two_d) {
      psd_off += (long long)sh.S * T.K;
      v.has_2d = true;
    } else if (T.tmpl) {
      v.has_tmpl = true;
    } else {
      v.has_1d = true;
    }
    T.gen = sh.gen;
    if (T.gen) v.has_gen = true;
    T.n_cell = sh.n_cell;
    T.S = sh.S;
    for (int k = 0; k < T.D; k++) T.exposure[k] = d.exposure[k];
    T.cflag_blocks = (sh.n_cell + kCellBlock - 1) / kCellBlock;
    T.cflag_off = cflag_off;
    T.ghull_off = ghull_off;
    T.cell_off = cell_off;
    T.win_off = win_off;
    T.fh_off = fh_off;
    T.bref_off = bref_off;
    T.cnt_off = cnt_off;
    T.pull_off = pull_off;
    if (T.mv) {
      // the energy histogram [d][j], then each slice's pulse-shape histogram [d][i][k]
      for (int k = 0; k < T.D; k++)
        for (int j = d.win_lo; j < d.win_hi; j++) {
          double n = 0.0;
          for (int q = 0; q < T.K; q++) n += d.counts[((size_t)k * d.n_reco + j) * T.K + q];
          cnt_h.push_back(n);
        }
      for (int k = 0; k < T.D; k++)
        for (int i = 0; i < d.n_slices; i++)
          for (int q = 0; q < T.K; q++) {
            double n = 0.0;
            for (int j = d.slice_edges[i]; j < d.slice_edges[i + 1]; j++)
              n += d.counts[((size_t)k * d.n_reco + j) * T.K + q];
            cnt_h.push_back(n);
          }
    } else {
      for (int k = 0; k < T.D; k++)
        for (int j = d.win_lo; j < d.win_hi; j++)
          for (int q = 0; q < T.K; q++) cnt_h.push_back(d.counts[((size_t)k * d.n_reco + j) * T.K + q]);
    }
    T.nsum_off = (long long)nsum_h.size();
    T.cnl = 0.0;
    if (T.two_d && !T.mv) {  // the constants k_bins2 takes: summed counts, sum of n ln eps (long double)
      long double c = 0.0L;
      for (int j = d.win_lo; j < d.win_hi; j++)
        for (int q = 0; q < T.K; q++) {
          double n = 0.0;
          for (int k = 0; k < T.D; k++) {
            const double nk = d.counts[((size_t)k * d.n_reco + j) * T.K + q];
            n += nk;
            c += (long double)nk * std::log((long double)d.exposure[k]);
          }
          nsum_h.push_back(n);
        }
      T.cnl = (double)c;
    }
    for (int p = 0; p < T.P; p++) {
      const bool has = d.pull_sigma && d.pull_sigma[p] > 0;
      pc_h.push_back(has ? d.pull_centre[p] : 0.0);
      ps_h.push_back(has ? d.pull_sigma[p] : 0.0);
    }
    cell_off += sh.n_cell;
    win_off += win_rows(T.L);
    fh_off += (long long)win_rows(T.L) * T.S;
    bref_off += (T.L + kABlock - 1) / kABlock;
    cnt_off += T.mv ? (long long)T.D * (T.L + (long long)T.n_slices * T.K) : (long long)T.D * T.L * T.K;
    cflag_off += T.cflag_blocks;
    ghull_off += (sh.n_true + kGroup - 1) / kGroup;
    pull_off += T.P;
    v.max_cells = std::max(v.max_cells, sh.n_cell);
    v.max_cflag_blocks = std::max(v.max_cflag_blocks, T.cflag_blocks);
    v.max_ls_blocks = std::max(v.max_ls_blocks, (int)(((long long)T.L * T.S + kBlock - 1) / kBlock));
    if (T.two_d) v.max_psd_sk = std::max(v.max_psd_sk, T.S * T.K);
    B->toys_h.push_back(T);
  }
  // ---- layout: the work buffers hold the largest candidate layout; the default is in force ----
  B->candidates = layout_candidates(B);
  B->knobs = default_knobs(B);
  LayoutSizes cap{};
  for (const Knobs &k : B->candidates) grow(cap, layout(B, k));
  B->cur = layout(B, B->knobs);
  grow(cap, B->cur);
  B->cap = cap;
  v.n_toys = n_toys;
  v.toy_list = nullptr;
  v.n_list = n_toys;
  v.list1d = v.list2d = v.listt = nullptr;
  v.n1d = v.n2d = v.nt = 0;
  for (const ToyDev &T : B->toys_h) (T.two_d ? v.n2d : T.tmpl ? v.nt : v.n1d)++;
  v.stride = B->stride;
  v.log_cut = kDefaultLogCut;
  ShapeDev *shd;
  ToyDev *tod;
  FoldItem *fi;
  AdjItem *ai;
  double *cnt, *pc, *ps;
  HIP_TRY(B->alloc(&shd, B->shapes_h.size()));
  HIP_TRY(B->alloc(&tod, B->toys_h.size()));
  HIP_TRY(B->alloc(&fi, cap.n_fold));
  HIP_TRY(B->alloc(&ai, cap.n_adj));
  HIP_TRY(B->alloc(&cnt, cnt_h.size()));
  HIP_TRY(B->alloc(&pc, pc_h.size()));
  HIP_TRY(B->alloc(&ps, ps_h.size()));
  HIP_TRY(B->alloc(&v.rec, (size_t)cell_off * kRecLen));
  HIP_TRY(B->alloc(&v.cflag, (size_t)cflag_off));
  HIP_TRY(B->alloc(&v.sup, (size_t)cell_off));
  HIP_TRY(B->alloc(&v.ghull, (size_t)std::max<long long>(ghull_off, 1)));
  HIP_TRY(B->alloc(&v.pflag, (size_t)n_toys));
  if (v.has_mv) {
    int *se;
    HIP_TRY(B->alloc(&se, sedge_h.size()));
    HIP_TRY(hipMemcpy(se, sedge_h.data(), sizeof(int) * sedge_h.size(), hipMemcpyHostToDevice));
    v.sedge = se;
    HIP_TRY(B->alloc(&v.sig, (size_t)sig_n));
  }
  if (v.has_2d) {
    HIP_TRY(B->alloc(&v.H, (size_t)fh_off));
    HIP_TRY(B->alloc(&v.P, (size_t)psd_off));
    HIP_TRY(B->alloc(&v.dP, (size_t)psd_off * 3));
    HIP_TRY(B->alloc(&v.vpart, (size_t)cap.vpart * kVLen));
  }
  HIP_TRY(B->alloc(&v.fpart, (size_t)cap.fpart));
  HIP_TRY(B->alloc(&v.fspart, (size_t)cap.fspart));
  HIP_TRY(B->alloc(&v.F, (size_t)std::max<long long>(fh_off, 1)));
  HIP_TRY(B->alloc(&v.apart, (size_t)cap.apart));
  HIP_TRY(B->alloc(&v.binrec, (size_t)win_off * kBinRecLen));
  HIP_TRY(hipMemset(v.binrec, 0, (size_t)win_off * kBinRecLen * sizeof(double)));  // the padding rows stay zero
  HIP_TRY(B->alloc(&v.bref, (size_t)bref_off * 4));
  HIP_TRY(B->alloc(&v.nllp, (size_t)cap.nllp));
  HIP_TRY(B->alloc(&v.badp, (size_t)cap.nllp));
  HIP_TRY(B->alloc(&v.gpart, (size_t)cap.gpart * kGradLen));
  HIP_TRY(hipMemcpy(shd, B->shapes_h.data(), B->shapes_h.size() * sizeof(ShapeDev), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(tod, B->toys_h.data(), B->toys_h.size() * sizeof(ToyDev), hipMemcpyHostToDevice));
  B->d_toys = tod;
  B->d_fold_items = fi;
  B->d_adj_items = ai;
  {
    gs_status us = upload_items(B, B->fold_h, B->fold1_h, B->adj_h, fi, ai, v, nullptr);
    if (us != GS_OK) return us;
  }
  if ((v.n1d > 0) + (v.n2d > 0) + (v.nt > 0) > 1) {  // a mixed batch: kernels of one kind take their toys from a list
    std::vector<int> l1, l2;
    for (int t = 0; t < n_toys; t++)
      if (!B->toys_h[t].tmpl) (B->toys_h[t].two_d ? l2 : l1).push_back(t);
    int *d1, *d2;
    HIP_TRY(B->alloc(&d1, l1.size()));
    HIP_TRY(B->alloc(&d2, l2.size()));
    if (!l1.empty()) HIP_TRY(hipMemcpy(d1, l1.data(), sizeof(int) * l1.size(), hipMemcpyHostToDevice));
    if (!l2.empty()) HIP_TRY(hipMemcpy(d2, l2.data(), sizeof(int) * l2.size(), hipMemcpyHostToDevice));
    v.list1d = d1;
    v.list2d = d2;
  }
  v.tgroup = nullptr;
  v.n_tgroup = 0;
  if (v.nt > 0) {  // template toys always go through a list: k_tmpl groups them by template
    std::vector<int> lt, grp;
    for (int t = 0; t < n_toys; t++)
      if (B->toys_h[t].tmpl) lt.push_back(t);
    tmpl_groups(B->toys_h, lt, grp);
    int *dt, *dg;
    HIP_TRY(B->alloc(&dt, lt.size()));
    HIP_TRY(B->alloc(&dg, grp.size()));
    HIP_TRY(hipMemcpy(dt, lt.data(), sizeof(int) * lt.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dg, grp.data(), sizeof(int) * grp.size(), hipMemcpyHostToDevice));
    v.listt = dt;
    v.tgroup = dg;
    v.n_tgroup = (int)grp.size() / 2;
  }
  HIP_TRY(hipMemcpy(cnt, cnt_h.data(), cnt_h.size() * 8, hipMemcpyHostToDevice));
  if (v.has_1d && v.has_2d) {
    HIP_TRY(hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&B->ev_join, hipEventDisableTiming));
  }
  if (!nsum_h.empty()) {
    double *ns;
    HIP_TRY(B->alloc(&ns, nsum_h.size()));
    HIP_TRY(hipMemcpy(ns, nsum_h.data(), nsum_h.size() * 8, hipMemcpyHostToDevice));
    v.nsum = ns;
  }
  HIP_TRY(hipMemcpy(pc, pc_h.data(), pc_h.size() * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ps, ps_h.data(), ps_h.size() * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipDeviceSynchronize());
  v.shapes = shd;
  v.toys = tod;
  v.cnt = cnt;
  v.pull_c = pc;
  v.pull_s = ps;
  *out = guard.release();
  return GS_OK;
}

// Launch through `f`, bracketed by timing events when profiling is on.
template <class F>
hipError_t timed(gs_batch *B, int kernel, hipStream_t st, F f) {
  if (!B->prof) return f();
  hipEvent_t a = B->event(), b = B->event();
  hipError_t e = hipEventRecord(a, st);
  if (e == hipSuccess) e = f();
  if (e == hipSuccess) e = hipEventRecord(b, st);
  B->pending.push_back({kernel, a, b});
  return e;
}

// One adjoint-path evaluation of every toy: cells, fold, -ln L, adjoint,
// gradient.  One-dimensional toys fold with the combined weight; toys with a
// secondary observable fold per species and expand over the pulse-shape bins.
// The two chains write disjoint parts of every buffer (each toy its own), so
// in a batch that has both the 2-D chain runs on the side stream alongside
// the 1-D one: the per-species kernels lean on the matrix cores, the 1-D ones
// on the vector units.  Kernel timing keeps them in one stream.
// view: the batch's own (every toy) or a compacted copy of it.
gs_status enqueue_nll_grad(gs_batch *B, const double *d_theta, double *d_nll, double *d_grad, uint32_t *d_status,
                           double *d_mu, hipStream_t st, const uint8_t *active = nullptr,
                           const BatchView *view = nullptr) {
  BatchView v = view ? *view : B->v;
  v.theta_dev = d_theta;
  B->v.theta_dev = d_theta;
  if (v.has_1d || v.has_2d) HIP_TRY(timed(B, GS_K_CELLS, st, [&] { return launch_cells(v, d_theta, active, st); }));
  if (v.has_tmpl) HIP_TRY(timed(B, GS_K_TMPL, st, [&] { return launch_tmpl(v, d_theta, d_mu, active, st); }));
  const bool fork = B->side && !B->prof && v.has_1d && v.has_2d;
  hipStream_t s2 = fork ? B->side : st;  // the 2-D chain's stream
  if (fork) {
    HIP_TRY(hipEventRecord(B->ev_fork, st));
    HIP_TRY(hipStreamWaitEvent(s2, B->ev_fork, 0));
  }
  if (v.has_2d) {
    HIP_TRY(timed(B, GS_K_FOLDS, s2, [&] { return launch_fold(v, true, kOnly2D, active, s2); }));
    HIP_TRY(timed(B, GS_K_REDF, s2, [&] { return launch_reduceF(v, kOnly2D, active, s2); }));
    HIP_TRY(launch_psd(v, d_theta, active, s2));
    HIP_TRY(timed(B, GS_K_NLL, s2, [&] { return launch_bins2(v, d_theta, d_mu, active, s2); }));
    if (v.has_mv) HIP_TRY(timed(B, GS_K_NLL, s2, [&] { return launch_mv(v, d_theta, d_mu, active, s2); }));
    if (d_grad) HIP_TRY(timed(B, GS_K_ADJS, s2, [&] { return launch_adj(v, true, active, s2); }));
  }
  if (v.has_1d) {
    HIP_TRY(timed(B, GS_K_FOLD, st, [&] { return launch_fold(v, false, kOnly1D, active, st); }));
    HIP_TRY(timed(B, GS_K_NLL, st, [&] { return launch_bins1(v, d_mu, active, st); }));
    if (d_grad) HIP_TRY(timed(B, GS_K_ADJ, st, [&] { return launch_adj(v, false, active, st); }));
  }
  if (fork) {
    HIP_TRY(hipEventRecord(B->ev_join, s2));
    HIP_TRY(hipStreamWaitEvent(st, B->ev_join, 0));
  }
  if (d_grad && (v.has_1d || v.has_2d))
    HIP_TRY(timed(B, GS_K_GRAD, st, [&] { return launch_cellgrad(v, d_theta, active, st); }));
  HIP_TRY(timed(B, GS_K_FINISH, st,
                [&] { return launch_finish(v, d_theta, d_nll, d_grad, d_status, active, st); }));
  return GS_OK;
}

}  // namespace

// ================================================================ C ABI ===
extern "C" {

const char *gs_last_error(void) { return g_err.c_str(); }

int32_t gs_desc_validate(const gs_model_desc *d) { return validate(d); }

gs_status gs_batch_create(const gs_model_desc *descs, int32_t n_toys, int32_t device, gs_batch **out) {
  if (!out) return fail(GS_ERR_ARG, "out is NULL");
  *out = nullptr;
  return build_batch(descs, n_toys, device, out);
}

void gs_batch_destroy(gs_batch *b) { delete b; }
int32_t gs_batch_num_toys(const gs_batch *b) { return b ? b->n_toys : 0; }
int32_t gs_batch_param_stride(const gs_batch *b) { return b ? b->stride : 0; }

gs_status gs_nll_grad_batched(gs_batch *b, const double *d_theta, double *d_nll, double *d_grad, uint32_t *d_status,
                              void *hip_stream) {
  if (!b || !d_theta || !d_nll || !d_status) return fail(GS_ERR_ARG, "null argument");
  HIP_TRY(hipSetDevice(b->device));
  return enqueue_nll_grad(b, d_theta, d_nll, d_grad, d_status, nullptr, (hipStream_t)hip_stream);
}

// ------------------------------------------- evaluation without allocation ---
// Workspace of gs_nll_grad_batched_noalloc: the split-K and block partials of
// one evaluation live in this fixed array instead of the batch's own buffers.
// The loaded library holds one copy on every device it runs on until the
// process ends.  In host code `scratch` names a host-side stand-in, never the
// device memory: kernels get the address that hipGetSymbolAddress returns for
// the current device (kept per device below).
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, unsigned char *> g_scratch_ptr;  // device -> address of its copy of scratch

// The device address of this device's scratch (looked up once per device, with
// the device current).
gs_status scratch_ptr(int device, unsigned char **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return GS_OK;
  }
  void *p = nullptr;
  HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  g_scratch_ptr[device] = (unsigned char *)p;
  *out = (unsigned char *)p;
  return GS_OK;
}
}  // namespace

gs_status gs_nll_grad_batched_noalloc(gs_batch *b, const double *d_theta, double *d_nll, double *d_grad,
                                      uint32_t *d_status, void *hip_stream) {
  if (!b || !d_theta || !d_nll || !d_status) return fail(GS_ERR_ARG, "null argument");
  HIP_TRY(hipSetDevice(b->device));
  unsigned char *base = nullptr;
  gs_status s = scratch_ptr(b->device, &base);
  if (s != GS_OK) return s;
  // carve the partials of the layout in force out of the array, each 256-byte aligned
  const LayoutSizes &z = b->cur;
  const auto al = [](size_t n) { return (n + 255) & ~size_t(255); };
  const size_t nb[8] = {al(8 * (size_t)std::max<long long>(z.fpart, 1)), al(8 * (size_t)std::max<long long>(z.fspart, 1)),
                        al(8 * (size_t)std::max<long long>(z.apart, 1)), al(8 * (size_t)std::max<long long>(z.nllp, 1)),
                        al(4 * (size_t)std::max<long long>(z.nllp, 1)),
                        al(8 * (size_t)std::max<long long>(z.gpart, 1) * kGradLen),
                        al(8 * (size_t)std::max<long long>(z.vpart, 1) * kVLen), 0};
  size_t need = 0;
  for (int k = 0; k < 7; k++) need += nb[k];
  if (need > kScratchBytes)
    return fail(GS_ERR_UNSUPPORTED, "gs_nll_grad_batched_noalloc: this batch's partials need %zu bytes, more than "
                "the %zu of the fixed workspace; use gs_nll_grad_batched", need, kScratchBytes);
  BatchView v = b->v;
  size_t off = 0;
  v.fpart = (double *)(base + off), off += nb[0];
  v.fspart = (double *)(base + off), off += nb[1];
  v.apart = (double *)(base + off), off += nb[2];
  v.nllp = (double *)(base + off), off += nb[3];
  v.badp = (uint32_t *)(base + off), off += nb[4];
  v.gpart = (double *)(base + off), off += nb[5];
  v.vpart = (double *)(base + off), off += nb[6];
  return enqueue_nll_grad(b, d_theta, d_nll, d_grad, d_status, nullptr, (hipStream_t)hip_stream, nullptr, &v);
}

// Puts layout k in force: host layout, then the toys and work items uploaded
// (synchronously); a captured fit graph, which holds the old layout, is dropped.
static gs_status apply_layout(gs_batch *B, const Knobs &k) {
  const LayoutSizes z = layout(B, k);
  if (z.fpart > B->cap.fpart || z.fspart > B->cap.fspart || z.apart > B->cap.apart || z.nllp > B->cap.nllp ||
      z.gpart > B->cap.gpart || z.vpart > B->cap.vpart || z.n_fold > B->cap.n_fold || z.n_adj > B->cap.n_adj)
    return fail(GS_ERR_ARG, "layout exceeds the batch's work buffers");
  HIP_TRY(hipMemcpy(B->d_toys, B->toys_h.data(), B->toys_h.size() * sizeof(ToyDev), hipMemcpyHostToDevice));
  gs_status us = upload_items(B, B->fold_h, B->fold1_h, B->adj_h, B->d_fold_items, B->d_adj_items, B->v, nullptr);
  if (us != GS_OK) return us;
  B->knobs = k;
  B->cur = z;
  if (B->graph) {
    HIP_TRY(hipGraphExecDestroy(B->graph));
    B->graph = nullptr;
  }
  return GS_OK;
}

gs_status gs_batch_set_layout(gs_batch *b, int32_t target_wg, int32_t grad_cells, int32_t iter2,
                              int32_t adj_waves) {
  if (!b) return fail(GS_ERR_ARG, "null batch");
  HIP_TRY(hipSetDevice(b->device));
  for (const Knobs &k : b->candidates)
    if (k.target_wg == target_wg && k.grad_cells == grad_cells && k.iter2 == iter2 && k.adj_waves == adj_waves) {
      HIP_TRY(hipDeviceSynchronize());  // no evaluation of the old layout may still run
      return apply_layout(b, k);
    }
  return fail(GS_ERR_ARG, "layout (%d, %d, %d, %d) is not one of the batch's candidates", target_wg, grad_cells,
              iter2, adj_waves);
}

gs_status gs_batch_autotune(gs_batch *b, const double *d_theta, double *d_nll, double *d_grad, uint32_t *d_status,
                            int32_t reps, void *hip_stream, double *choice) {
  if (!b || !d_theta || !d_nll || !d_status || reps < 1) return fail(GS_ERR_ARG, "bad argument");
  HIP_TRY(hipSetDevice(b->device));
  hipStream_t st = (hipStream_t)hip_stream;
  HIP_TRY(hipDeviceSynchronize());
  const Knobs dflt = default_knobs(b);
  const int nc = (int)b->candidates.size();
  std::vector<double> ms(nc, INFINITY);
  hipEvent_t e0 = b->event(), e1 = b->event();
  gs_status s = GS_OK;
  // warm the device up at the layout in force, then time every candidate in
  // two passes (the second in reverse order, so that a drift of the clocks
  // favours no candidate) and keep each candidate's faster time
  for (int r = 0; r < 3 && s == GS_OK; r++) s = enqueue_nll_grad(b, d_theta, d_nll, d_grad, d_status, nullptr, st);
  for (int pass = 0; pass < 2 && s == GS_OK; pass++)
    for (int c = 0; c < nc && s == GS_OK; c++) {
      const int ci = pass == 0 ? c : nc - 1 - c;
      s = apply_layout(b, b->candidates[ci]);
      if (s == GS_OK) s = enqueue_nll_grad(b, d_theta, d_nll, d_grad, d_status, nullptr, st);  // warm-up
      if (s != GS_OK) break;
      hipError_t e = hipEventRecord(e0, st);
      for (int r = 0; r < reps && s == GS_OK && e == hipSuccess; r++)
        s = enqueue_nll_grad(b, d_theta, d_nll, d_grad, d_status, nullptr, st);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float t = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
      if (e != hipSuccess) s = fail(GS_ERR_DEVICE, "autotune timing: %s", hipGetErrorString(e));
      if (s == GS_OK) ms[ci] = std::min(ms[ci], (double)t / reps);
    }
  b->ev_free.push_back(e0);
  b->ev_free.push_back(e1);
  if (s != GS_OK) return s;
  // the fastest candidate, kept only if it beats the default layout by more than 1%
  int best = 0, di = -1;
  for (int c = 0; c < nc; c++) {
    if (ms[c] < ms[best]) best = c;
    const Knobs &k = b->candidates[c];
    if (k.target_wg == dflt.target_wg && k.grad_cells == dflt.grad_cells && k.iter2 == dflt.iter2 &&
        k.adj_waves == dflt.adj_waves)
      di = c;
  }
  if (di >= 0 && !(ms[best] < 0.99 * ms[di])) best = di;
  s = apply_layout(b, b->candidates[best]);
  if (s != GS_OK) return s;
  if (choice) {
    const Knobs &k = b->candidates[best];
    choice[0] = k.target_wg;
    choice[1] = k.grad_cells;
    choice[2] = k.iter2;
    choice[3] = k.adj_waves;
    choice[4] = ms[best];
  }
  return GS_OK;
}

gs_status gs_batch_layout(const gs_batch *b, int32_t *out) {
  if (!b || !out) return fail(GS_ERR_ARG, "null argument");
  out[0] = b->knobs.target_wg;
  out[1] = b->knobs.grad_cells;
  out[2] = b->knobs.iter2;
  out[3] = b->knobs.adj_waves;
  out[4] = (int32_t)b->candidates.size();
  return GS_OK;
}

gs_status gs_batch_set_log_cut(gs_batch *b, double log_cut) {
  if (!b || std::isnan(log_cut)) return fail(GS_ERR_ARG, "bad argument");
  b->v.log_cut = log_cut;
  if (b->graph) {  // a captured fit graph holds the old cut
    HIP_TRY(hipGraphExecDestroy(b->graph));
    b->graph = nullptr;
  }
  return GS_OK;
}

gs_status gs_model_set_log_cut(gs_model *m, double log_cut) {
  if (!m) return fail(GS_ERR_ARG, "null model");
  m->cache_valid = false;
  return gs_batch_set_log_cut(m->b, log_cut);
}

gs_status gs_batch_mesh_pairs(gs_batch *b, int64_t *out) {
  if (!b || !out) return fail(GS_ERR_ARG, "null argument");
  HIP_TRY(hipSetDevice(b->device));
  HIP_TRY(hipDeviceSynchronize());
  long long n_cells = 0;
  for (const ToyDev &T : b->toys_h) n_cells = std::max(n_cells, T.cell_off + T.n_cell);
  std::vector<int2> sup((size_t)n_cells);
  HIP_TRY(hipMemcpy(sup.data(), b->v.sup, sizeof(int2) * (size_t)n_cells, hipMemcpyDeviceToHost));
  long long fold = 0, adj = 0, full = 0, band = 0, band2 = 0, band2s = 0;
  for (const ToyDev &T : b->toys_h) {
    const ShapeDev &Sh = b->shapes_h[T.shape];
    full += (long long)T.L * T.n_cell;
    for (int i = 0; i < T.n_cell; i++) {
      const int2 s = sup[T.cell_off + i];
      const int x = std::max(s.x, T.lo), y = std::min(s.y, T.lo + T.L);
      if (y <= x) continue;
      band += y - x;
      if (T.two_d) {
        band2 += y - x;
        band2s += (long long)(y - x) * (i < Sh.n_true ? Sh.Sg : 1);
      }
    }
  }
  // the fold evaluates every cell of the hull groups that meet its tile
  // (partial groups padded to kGroup), plus the chunk's line cells, on every
  // bin of the tile: kFoldTile1 bins for 1-D toys, kFoldTile for 2-D toys
  std::vector<FoldItem> fitems;
  for (const FoldItem &it : b->fold1_h)
    if (!b->toys_h[it.toy].two_d) fitems.push_back(it);
  for (const FoldItem &it : b->fold_h)
    if (b->toys_h[it.toy].two_d) fitems.push_back(it);
  for (const FoldItem &it : fitems) {
    const ToyDev &T = b->toys_h[it.toy];
    const ShapeDev &Sh = b->shapes_h[T.shape];
    const int tile = T.two_d ? kFoldTile : kFoldTile1;
    const int j0 = T.lo + it.bin0, j1 = T.lo + std::min(it.bin0 + tile, T.L);
    const int g_end = std::min(it.cell1, Sh.n_true);
    long long cells = std::max(0, it.cell1 - std::max(it.cell0, Sh.n_true));
    for (int g = it.cell0 / kGroup; g * kGroup < g_end; g++) {
      int hx = 0x7fffffff, hy = -1;
      for (int i = g * kGroup; i < std::min((g + 1) * kGroup, Sh.n_true); i++) {
        const int2 s = sup[T.cell_off + i];
        if (s.y > s.x) {
          hx = std::min(hx, s.x);
          hy = std::max(hy, s.y);
        }
      }
      if (hx < j1 && hy > j0) cells += kGroup;
    }
    fold += cells * tile;
  }
  for (const AdjItem &it : b->adj_h) {
    const ToyDev &T = b->toys_h[it.toy];
    // 1-D toys: one walk over the union of the item's 64 cells' supports; 2-D toys: one walk
    // per 16 cells, in whole steps of 16 bins (the per-species adjoint's matrix tiles)
    const int per = T.two_d ? 16 : kTile;
    for (int c0 = it.cell0; c0 < std::min(it.cell0 + kTile, T.n_cell); c0 += per) {
      int lo = 0x7fffffff, hi = -1;
      for (int i = c0; i < std::min(c0 + per, T.n_cell); i++) {
        lo = std::min(lo, sup[T.cell_off + i].x);
        hi = std::max(hi, sup[T.cell_off + i].y);
      }
      const int b0 = std::max(it.bin0, lo - T.lo), b1 = std::min(it.bin1, hi - T.lo);
      if (b1 > b0) adj += (long long)(T.two_d ? (b1 - (b0 & ~15) + 15) / 16 * 16 : b1 - b0) * per;
    }
  }
  out[0] = fold;
  out[1] = adj;
  out[2] = full;
  out[3] = band;
  out[4] = band2;
  out[5] = band2s;
  return GS_OK;
}

gs_status gs_batch_fit_trace(gs_batch *b, int32_t *active, double *ms, int32_t cap, int32_t *n) {
  if (!b || !n || cap < 0 || (cap > 0 && (!active || !ms))) return fail(GS_ERR_ARG, "bad argument");
  const int m = (int)b->trace_active.size();
  for (int i = 0; i < std::min(m, (int)cap); i++) {
    active[i] = b->trace_active[i];
    ms[i] = b->trace_ms[i];
  }
  *n = m;
  return GS_OK;
}

gs_status gs_batch_set_profiling(gs_batch *b, int32_t on) {
  if (!b) return fail(GS_ERR_ARG, "null batch");
  b->prof = on != 0;
  return GS_OK;
}

gs_status gs_batch_kernel_times(gs_batch *b, double *ms, int64_t *launches, int32_t reset) {
  if (!b || !ms || !launches) return fail(GS_ERR_ARG, "null argument");
  HIP_TRY(hipSetDevice(b->device));
  for (auto &t : b->pending) {
    float el = 0.f;
    HIP_TRY(hipEventSynchronize(t.b));
    HIP_TRY(hipEventElapsedTime(&el, t.a, t.b));
    b->prof_ms[t.kernel] += el;
    b->prof_n[t.kernel] += 1;
    b->ev_free.push_back(t.a);
    b->ev_free.push_back(t.b);
  }
  b->pending.clear();
  for (int k = 0; k < GS_K_COUNT; k++) {
    ms[k] = b->prof_ms[k];
    launches[k] = b->prof_n[k];
    if (reset) {
      b->prof_ms[k] = 0.0;
      b->prof_n[k] = 0;
    }
  }
  return GS_OK;
}

gs_status gs_model_create(const gs_model_desc *d, int32_t device, gs_model **out) {
  if (!out) return fail(GS_ERR_ARG, "out is NULL");
  *out = nullptr;
  gs_batch *b = nullptr;
  gs_status s = build_batch(d, 1, device, &b);
  if (s != GS_OK) return s;
  auto *M = new gs_model();
  M->b = b;
  M->P = b->toys_h[0].P;
  const ToyDev &T = b->toys_h[0];
  M->n_mu = T.D * T.L * T.K;
  auto cleanup = [&](gs_status e) {
    gs_model_destroy(M);
    return e;
  };
#define MTRY(expr)                                                                                    \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess)                                                                             \
      return cleanup(fail(GS_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)));                   \
  } while (0)
  MTRY(hipStreamCreateWithFlags(&M->stream, hipStreamNonBlocking));
  MTRY(hipMalloc((void **)&M->d_theta, sizeof(double) * b->stride));
  MTRY(hipMalloc((void **)&M->d_nll, sizeof(double)));
  MTRY(hipMalloc((void **)&M->d_grad, sizeof(double) * b->stride));
  MTRY(hipMalloc((void **)&M->d_mu, sizeof(double) * std::max(M->n_mu, 1)));
  MTRY(hipMalloc((void **)&M->d_status, sizeof(uint32_t)));
  MTRY(hipHostMalloc((void **)&M->h_theta, sizeof(double) * b->stride, hipHostMallocDefault));
  MTRY(hipHostMalloc((void **)&M->h_out, sizeof(double) * (1 + b->stride + std::max(M->n_mu, 1)), hipHostMallocDefault));
  MTRY(hipHostMalloc((void **)&M->h_status, sizeof(uint32_t), hipHostMallocDefault));
#undef MTRY
  *out = M;
  return GS_OK;
}

void gs_model_destroy(gs_model *m) {
  if (!m) return;
  if (m->b) (void)hipSetDevice(m->b->device);
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  (void)hipFree(m->d_theta);
  (void)hipFree(m->d_nll);
  (void)hipFree(m->d_grad);
  (void)hipFree(m->d_mu);
  (void)hipFree(m->d_status);
  (void)hipHostFree(m->h_theta);
  (void)hipHostFree(m->h_out);
  (void)hipHostFree(m->h_status);
  if (m->stream) (void)hipStreamDestroy(m->stream);
  delete m->b;
  delete m;
}

int32_t gs_model_num_params(const gs_model *m) { return m ? m->P : 0; }

static gs_status upload_theta(gs_model *M, const double *theta) {
  std::memcpy(M->h_theta, theta, sizeof(double) * M->P);
  for (int p = M->P; p < M->b->stride; p++) M->h_theta[p] = 0.0;
  HIP_TRY(hipMemcpyAsync(M->d_theta, M->h_theta, sizeof(double) * M->b->stride, hipMemcpyHostToDevice, M->stream));
  return GS_OK;
}

gs_status gs_nll_grad(gs_model *M, const double *theta, double *nll, double *grad, uint32_t *st) {
  if (!M || !theta || !nll) return fail(GS_ERR_ARG, "null argument");
  gs_batch *B = M->b;
  HIP_TRY(hipSetDevice(B->device));
  if (B->v.has_2d) M->cache_valid = false;  // the per-species fold below overwrites gs_nll's cached F
  gs_status s = upload_theta(M, theta);
  if (s != GS_OK) return s;
  s = enqueue_nll_grad(B, M->d_theta, M->d_nll, grad ? M->d_grad : nullptr, M->d_status, nullptr, M->stream);
  if (s != GS_OK) return s;
  HIP_TRY(hipMemcpyAsync(M->h_out, M->d_nll, sizeof(double), hipMemcpyDeviceToHost, M->stream));
  if (grad)
    HIP_TRY(hipMemcpyAsync(M->h_out + 1, M->d_grad, sizeof(double) * M->P, hipMemcpyDeviceToHost, M->stream));
  HIP_TRY(hipMemcpyAsync(M->h_status, M->d_status, sizeof(uint32_t), hipMemcpyDeviceToHost, M->stream));
  HIP_TRY(hipStreamSynchronize(M->stream));
  *nll = M->h_out[0];
  if (grad) std::memcpy(grad, M->h_out + 1, sizeof(double) * M->P);
  if (st) *st = *M->h_status;
  return GS_OK;
}

gs_status gs_expected(gs_model *M, const double *theta, double *mu) {
  if (!M || !theta || !mu) return fail(GS_ERR_ARG, "null argument");
  gs_batch *B = M->b;
  HIP_TRY(hipSetDevice(B->device));
  if (B->v.has_2d) M->cache_valid = false;  // the per-species fold below overwrites gs_nll's cached F
  gs_status s = upload_theta(M, theta);
  if (s != GS_OK) return s;
  s = enqueue_nll_grad(B, M->d_theta, M->d_nll, nullptr, M->d_status, M->d_mu, M->stream);
  if (s != GS_OK) return s;
  HIP_TRY(hipMemcpyAsync(M->h_out, M->d_mu, sizeof(double) * M->n_mu, hipMemcpyDeviceToHost, M->stream));
  HIP_TRY(hipMemcpyAsync(M->h_status, M->d_status, sizeof(uint32_t), hipMemcpyDeviceToHost, M->stream));
  HIP_TRY(hipStreamSynchronize(M->stream));
  // a refused evaluation (response outside the admitted range) claims no value
  const bool refused = (*M->h_status & (GS_ST_UNRESOLVED | GS_ST_NONFINITE)) != 0;
  for (int i = 0; i < M->n_mu; i++) mu[i] = refused ? NAN : M->h_out[i];
  return GS_OK;
}

gs_status gs_species_spectra(gs_model *M, const double *theta, double *F) {
  if (!M || !theta || !F) return fail(GS_ERR_ARG, "null argument");
  gs_batch *B = M->b;
  HIP_TRY(hipSetDevice(B->device));
  gs_status s = upload_theta(M, theta);
  if (s != GS_OK) return s;
  const ToyDev &T = B->toys_h[0];
  const ShapeDev &sh = B->shapes_h[0];
  std::vector<double> f((size_t)T.L * T.S);  // the device's F rows (fh_off = 0: the model's only toy)
  if (B->v.has_tmpl) {  // the species spectra are the templates themselves
    std::vector<double> w((size_t)sh.Sg * sh.n_true);
    HIP_TRY(hipMemcpy(w.data(), sh.wcellT, sizeof(double) * w.size(), hipMemcpyDeviceToHost));
    for (int b = 0; b < T.L; b++)
      for (int q = 0; q < T.S; q++) f[(size_t)b * T.S + q] = w[(size_t)q * sh.n_true + T.lo + b];
  } else {
    HIP_TRY(launch_cells(B->v, M->d_theta, nullptr, M->stream));
    HIP_TRY(launch_fold(B->v, true, kAllToys, nullptr, M->stream));
    HIP_TRY(launch_reduceF(B->v, kAllToys, nullptr, M->stream));
    HIP_TRY(hipMemcpyAsync(f.data(), B->v.F, sizeof(double) * f.size(), hipMemcpyDeviceToHost, M->stream));
    HIP_TRY(hipStreamSynchronize(M->stream));
  }
  M->cache_valid = false;
  for (int b = 0; b < T.L; b++)
    for (int q = 0; q < T.S; q++) F[(size_t)b * T.S + sh.sp_of[q]] = f[(size_t)b * T.S + q];
  return GS_OK;
}

gs_status gs_psd_probs(gs_model *M, const double *theta, double *P) {
  if (!M || !theta || !P) return fail(GS_ERR_ARG, "null argument");
  gs_batch *B = M->b;
  if (!B->v.has_2d) return fail(GS_ERR_ARG, "model has no secondary observable");
  HIP_TRY(hipSetDevice(B->device));
  gs_status s = upload_theta(M, theta);
  if (s != GS_OK) return s;
  const ToyDev &T = B->toys_h[0];
  const ShapeDev &sh = B->shapes_h[0];
  HIP_TRY(launch_psd(B->v, M->d_theta, nullptr, M->stream));
  std::vector<double> p((size_t)T.S * T.K);
  HIP_TRY(hipMemcpyAsync(p.data(), B->v.P, sizeof(double) * p.size(), hipMemcpyDeviceToHost, M->stream));
  HIP_TRY(hipStreamSynchronize(M->stream));
  for (int q = 0; q < T.S; q++)
    for (int k = 0; k < T.K; k++) P[(size_t)sh.sp_of[q] * T.K + k] = p[(size_t)q * T.K + k];
  return GS_OK;
}

gs_status gs_nll(gs_model *M, const double *theta, double *nll, uint32_t *st) {
  if (!M || !theta || !nll) return fail(GS_ERR_ARG, "null argument");
  gs_batch *B = M->b;
  HIP_TRY(hipSetDevice(B->device));
  const ShapeDev &sh = B->shapes_h[0];
  const int nr = n_resp(sh.family);
  std::vector<double> resp(theta + sh.S, theta + sh.S + nr);
  gs_status s = upload_theta(M, theta);
  if (s != GS_OK) return s;
  if (B->v.has_tmpl) {  // templates: nothing to fold or cache; one pass gives -ln L
    s = enqueue_nll_grad(B, M->d_theta, M->d_nll, nullptr, M->d_status, nullptr, M->stream);
    if (s != GS_OK) return s;
    HIP_TRY(hipMemcpyAsync(M->h_out, M->d_nll, sizeof(double), hipMemcpyDeviceToHost, M->stream));
    HIP_TRY(hipMemcpyAsync(M->h_status, M->d_status, sizeof(uint32_t), hipMemcpyDeviceToHost, M->stream));
    HIP_TRY(hipStreamSynchronize(M->stream));
    *nll = M->h_out[0];
    if (st) *st = *M->h_status;
    return GS_OK;
  }
  const bool refold = !M->cache_valid || std::memcmp(resp.data(), M->cached_resp.data(), nr * 8) != 0;
  B->v.theta_dev = M->d_theta;
  if (refold) {
    HIP_TRY(timed(B, GS_K_CELLS, M->stream, [&] { return launch_cells(B->v, M->d_theta, nullptr, M->stream); }));
    HIP_TRY(timed(B, GS_K_FOLDS, M->stream, [&] { return launch_fold(B->v, true, kAllToys, nullptr, M->stream); }));
    HIP_TRY(timed(B, GS_K_REDF, M->stream, [&] { return launch_reduceF(B->v, kAllToys, nullptr, M->stream); }));
    M->cached_resp = resp;
    M->cache_valid = true;
  }
  if (B->v.has_2d) {
    HIP_TRY(launch_psd(B->v, M->d_theta, nullptr, M->stream));
    HIP_TRY(timed(B, GS_K_NLLF, M->stream,
                  [&] { return launch_bins2(B->v, M->d_theta, nullptr, nullptr, M->stream); }));
    HIP_TRY(launch_mv(B->v, M->d_theta, nullptr, nullptr, M->stream));
  } else {
    HIP_TRY(timed(B, GS_K_NLLF, M->stream, [&] { return launch_binsF(B->v, M->d_theta, nullptr, M->stream); }));
  }
  HIP_TRY(timed(B, GS_K_FINISH, M->stream, [&] {
    return launch_finish(B->v, M->d_theta, M->d_nll, nullptr, M->d_status, nullptr, M->stream);
  }));
  HIP_TRY(hipMemcpyAsync(M->h_out, M->d_nll, sizeof(double), hipMemcpyDeviceToHost, M->stream));
  HIP_TRY(hipMemcpyAsync(M->h_status, M->d_status, sizeof(uint32_t), hipMemcpyDeviceToHost, M->stream));
  HIP_TRY(hipStreamSynchronize(M->stream));
  *nll = M->h_out[0];
  if (st) *st = *M->h_status;
  return GS_OK;
}

gs_status gs_fit(gs_model *M, const double *theta0, const gs_fit_opts *o, double *theta_hat, double *sigma,
                 gs_fit_result *res);

static gs_status qn_setup(gs_batch *B) {
  if (B->qn_ready) return GS_OK;
  const int n = B->n_toys, P = B->stride;
  if (P > GS_MAX_PARAMS) return fail(GS_ERR_UNSUPPORTED, "%d parameters per toy (at most %d)", P, GS_MAX_PARAMS);
  QNView &q = B->q;
  q.P = P;
  q.stride = P;
  HIP_TRY(B->alloc(&q.x, (size_t)n * P));
  HIP_TRY(B->alloc(&q.xt, (size_t)n * P));
  HIP_TRY(B->alloc(&q.g, (size_t)n * P));
  HIP_TRY(B->alloc(&q.d, (size_t)n * P));
  HIP_TRY(B->alloc(&q.h0, (size_t)n * P));
  HIP_TRY(B->alloc(&q.H, (size_t)n * P * P));
  HIP_TRY(B->alloc(&q.f, (size_t)n));
  HIP_TRY(B->alloc(&q.edm, (size_t)n));
  HIP_TRY(B->alloc(&q.alpha, (size_t)n));
  HIP_TRY(B->alloc(&q.slope, (size_t)n));
  HIP_TRY(B->alloc(&q.phase, (size_t)n));
  HIP_TRY(B->alloc(&q.iter, (size_t)n));
  HIP_TRY(B->alloc(&q.nls, (size_t)n));
  HIP_TRY(B->alloc(&q.n_par, (size_t)n));
  HIP_TRY(B->alloc(&q.status, (size_t)n));
  HIP_TRY(B->alloc(&q.active, (size_t)n));
  HIP_TRY(B->alloc(&q.freep, (size_t)n * P));
  HIP_TRY(B->alloc(&B->e_nll, (size_t)n));
  HIP_TRY(B->alloc(&B->e_grad, (size_t)n * P));
  HIP_TRY(B->alloc(&B->e_st, (size_t)n));
  HIP_TRY(B->alloc(&B->d_scale, (size_t)P));
  HIP_TRY(B->alloc(&B->d_count, 1));
  HIP_TRY(hipHostMalloc((void **)&B->h_count, sizeof(int), hipHostMallocDefault));
  HIP_TRY(B->alloc(&B->d_toy_list, (size_t)n));
  HIP_TRY(B->alloc(&B->d_list1, (size_t)n));
  HIP_TRY(B->alloc(&B->d_list2, (size_t)n));
  HIP_TRY(B->alloc(&B->d_listt, (size_t)n));
  HIP_TRY(B->alloc(&B->d_tgroup, (size_t)n * 2));
  HIP_TRY(B->alloc(&B->d_fold_c, std::max<size_t>(B->cap.n_fold, 1)));
  HIP_TRY(B->alloc(&B->d_adj_c, std::max<size_t>(B->cap.n_adj, 1)));
  std::vector<int> np(n);
  for (int t = 0; t < n; t++) np[t] = B->toys_h[t].P;
  HIP_TRY(hipMemcpy(q.n_par, np.data(), sizeof(int) * n, hipMemcpyHostToDevice));
  HIP_TRY(hipStreamCreateWithFlags(&B->fit_stream, hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming));
  B->qn_ready = true;
  return GS_OK;
}

// Capture K iterations of [evaluate every active toy at its trial point,
// quasi-Newton step] followed by a count of the active toys.
// Captures K x [evaluate the trial points, BFGS step] plus the active count.
// view == NULL: every toy; else a compacted view (toy list and work items of
// the toys still running), captured afresh.
static gs_status qn_graph(gs_batch *B, int K, double tol, int max_iter, const BatchView *view = nullptr) {
  if (!view && B->graph && !B->graph_compact && B->graph_k == K && B->graph_tol == tol &&
      B->graph_max_iter == max_iter)
    return GS_OK;
  if (B->graph) {
    HIP_TRY(hipGraphExecDestroy(B->graph));
    B->graph = nullptr;
  }
  const bool prof = B->prof;
  B->prof = false;  // no timing events inside the graph
  hipStream_t st = B->fit_stream;
  const int n_rows = view ? view->n_list : B->n_toys;
  const int *list = view ? view->toy_list : nullptr;
  HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  gs_status s = GS_OK;
  for (int k = 0; k < K && s == GS_OK; k++) {
    s = enqueue_nll_grad(B, B->q.xt, B->e_nll, B->e_grad, B->e_st, nullptr, st, B->q.active, view);
    if (s == GS_OK &&
        launch_qn_step(B->q, n_rows, list, B->e_nll, B->e_grad, B->e_st, tol, max_iter, st) != hipSuccess)
      s = fail(GS_ERR_DEVICE, "launch_qn_step failed during capture");
  }
  if (s == GS_OK && launch_qn_count(B->q.active, B->n_toys, B->d_count, st) != hipSuccess)
    s = fail(GS_ERR_DEVICE, "launch_qn_count failed during capture");
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(st, &g);
  B->prof = prof;
  if (s != GS_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return fail(GS_ERR_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&B->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(GS_ERR_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  B->graph_k = K;
  B->graph_tol = tol;
  B->graph_max_iter = max_iter;
  B->graph_compact = view != nullptr;
  return GS_OK;
}

// The toys still running and their fold / adjoint items, uploaded to the
// batch's compaction buffers; returns the view that covers only them.
static gs_status compact_view(gs_batch *B, hipStream_t st, BatchView &out) {
  std::vector<uint8_t> act((size_t)B->n_toys);
  HIP_TRY(hipMemcpyAsync(act.data(), B->q.active, act.size(), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  std::vector<int> list, l1, l2, lt;
  for (int t = 0; t < B->n_toys; t++)
    if (act[t]) {
      list.push_back(t);
      (B->toys_h[t].two_d ? l2 : B->toys_h[t].tmpl ? lt : l1).push_back(t);
    }
  std::vector<FoldItem> fi, fi1;
  std::vector<AdjItem> ai;
  for (const FoldItem &it : B->fold_h)
    if (act[it.toy]) fi.push_back(it);
  for (const FoldItem &it : B->fold1_h)
    if (act[it.toy]) fi1.push_back(it);
  for (const AdjItem &it : B->adj_h)
    if (act[it.toy]) ai.push_back(it);
  out = B->v;
  if (!list.empty())
    HIP_TRY(hipMemcpyAsync(B->d_toy_list, list.data(), sizeof(int) * list.size(), hipMemcpyHostToDevice, st));
  if (!l1.empty()) HIP_TRY(hipMemcpyAsync(B->d_list1, l1.data(), sizeof(int) * l1.size(), hipMemcpyHostToDevice, st));
  if (!l2.empty()) HIP_TRY(hipMemcpyAsync(B->d_list2, l2.data(), sizeof(int) * l2.size(), hipMemcpyHostToDevice, st));
  std::vector<int> grp;
  tmpl_groups(B->toys_h, lt, grp);
  if (!lt.empty()) HIP_TRY(hipMemcpyAsync(B->d_listt, lt.data(), sizeof(int) * lt.size(), hipMemcpyHostToDevice, st));
  if (!grp.empty()) HIP_TRY(hipMemcpyAsync(B->d_tgroup, grp.data(), sizeof(int) * grp.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));  // host vectors go out of scope
  gs_status us = upload_items(B, fi, fi1, ai, B->d_fold_c, B->d_adj_c, out, st);
  if (us != GS_OK) return us;
  out.toy_list = B->d_toy_list;
  out.n_list = (int)list.size();
  out.list1d = B->d_list1;
  out.n1d = (int)l1.size();
  out.list2d = B->d_list2;
  out.n2d = (int)l2.size();
  out.listt = B->d_listt;
  out.nt = (int)lt.size();
  out.tgroup = B->d_tgroup;
  out.n_tgroup = (int)grp.size() / 2;
  return GS_OK;
}

gs_status gs_fit_batched(gs_batch *B, const double *d_theta0, const uint8_t *d_free, const double *d_scale,
                         const gs_fit_opts *o,
                         double *d_theta_hat, double *d_nll_hat, double *d_sigma, int32_t *d_iters,
                         uint32_t *d_status, void *hip_stream) {
  if (!B || !d_theta0 || !o || (!o->scale && !d_scale) || !d_theta_hat || !d_nll_hat || !d_iters || !d_status)
    return fail(GS_ERR_ARG, "null argument");
  if (o->max_iter < 1 || !(o->edm_tol > 0)) return fail(GS_ERR_ARG, "max_iter >= 1 and edm_tol > 0 required");
  if (!d_scale)
    for (int p = 0; p < B->stride; p++)
      if (!(o->scale[p] > 0)) return fail(GS_ERR_ARG, "scale[%d] must be > 0", p);
  HIP_TRY(hipSetDevice(B->device));
  gs_status s = qn_setup(B);
  if (s != GS_OK) return s;
  hipStream_t caller = (hipStream_t)hip_stream, st = B->fit_stream;
  if (!d_scale) HIP_TRY(hipMemcpyAsync(B->d_scale, o->scale, sizeof(double) * B->stride, hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(B->ev_in, caller));
  HIP_TRY(hipStreamWaitEvent(st, B->ev_in, 0));
  HIP_TRY(launch_qn_init(B->q, B->n_toys, d_theta0, d_free, d_scale ? d_scale : B->d_scale, d_scale ? B->stride : 0,
                         st));
  constexpr int K = 8;
  constexpr int kCompactMin = 16;  // below this many toys a smaller graph no longer pays
  s = qn_graph(B, K, o->edm_tol, o->max_iter);
  if (s != GS_OK) return s;
  // an iteration is one evaluation; a fit needs max_iter accepted steps plus line-search trials
  const long long cap = 4LL * o->max_iter + 64;
  B->trace_active.clear();
  B->trace_ms.clear();
  const auto t0 = std::chrono::steady_clock::now();
  int rows = B->n_toys;  // toys the current graph's grids cover
  for (long long done = 0; done < cap; done += K) {
    HIP_TRY(hipGraphLaunch(B->graph, st));
    HIP_TRY(hipMemcpyAsync(B->h_count, B->d_count, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const int running = *B->h_count;
    B->trace_active.push_back(running);
    B->trace_ms.push_back(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
    if (running == 0) break;
    // once half of the covered toys have stopped, re-capture the graph over the rest
    if (2 * running <= rows && rows > kCompactMin) {
      BatchView cv;
      s = compact_view(B, st, cv);
      if (s == GS_OK) s = qn_graph(B, K, o->edm_tol, o->max_iter, &cv);
      if (s != GS_OK) return s;
      rows = running;
    }
  }
  HIP_TRY(launch_qn_final(B->q, B->n_toys, d_theta_hat, d_nll_hat, d_sigma, d_iters, d_status, st));
  HIP_TRY(hipEventRecord(B->ev_out, st));
  HIP_TRY(hipStreamWaitEvent(caller, B->ev_out, 0));
  HIP_TRY(hipStreamSynchronize(caller));
  return GS_OK;
}

gs_status gs_discovery_batched(gs_batch *B, const double *d_theta0, const uint8_t *d_free, const double *d_scale,
                               const int32_t *d_signal, const gs_fit_opts *o, double *d_t, double *d_theta_free,
                               double *d_nll_free, uint32_t *d_status_free, double *d_theta_null, double *d_nll_null,
                               uint32_t *d_status_null, void *hip_stream) {
  if (!B || !d_theta0 || !d_signal || !o || !d_t || !d_theta_free || !d_nll_free || !d_status_free || !d_theta_null ||
      !d_nll_null || !d_status_null)
    return fail(GS_ERR_ARG, "null argument");
  HIP_TRY(hipSetDevice(B->device));
  const int n = B->n_toys, P = B->stride;
  if (!B->d_th0_null) {
    HIP_TRY(B->alloc(&B->d_th0_null, (size_t)n * P));
    HIP_TRY(B->alloc(&B->d_free_null, (size_t)n * P));
    HIP_TRY(B->alloc(&B->d_iters_tmp, (size_t)n));
  }
  hipStream_t st = (hipStream_t)hip_stream;
  HIP_TRY(launch_null_start(n, P, d_theta0, d_free, d_signal, B->d_th0_null, B->d_free_null, st));
  gs_status s = gs_fit_batched(B, d_theta0, d_free, d_scale, o, d_theta_free, d_nll_free, nullptr, B->d_iters_tmp,
                               d_status_free, hip_stream);
  if (s != GS_OK) return s;
  s = gs_fit_batched(B, B->d_th0_null, B->d_free_null, d_scale, o, d_theta_null, d_nll_null, nullptr, B->d_iters_tmp,
                     d_status_null, hip_stream);
  if (s != GS_OK) return s;
  HIP_TRY(launch_discovery_t(n, d_nll_free, d_status_free, d_nll_null, d_status_null, d_t, st));
  HIP_TRY(hipStreamSynchronize(st));
  return GS_OK;
}

}  // extern "C"
