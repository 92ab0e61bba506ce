// gs_impl.h -- internal layout of models and batches on the device.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs.h"
#include "gs_dev.h"

namespace gs {

constexpr int kTile = 64;       // cells per adjoint tile (one per lane); bins per per-species fold tile
constexpr int kFoldTile = 64;   // window bins per per-species fold item (two per lane of each half-wave)
constexpr int kFoldTile1 = 32;  // window bins per 1-D fold item (two per lane of each quarter-wave)
constexpr int kABlock = 64;     // window bins per adjoint exponent reference block
constexpr int kRefBlocks = 16;  // reference blocks whose per-cell exponents the adjoint stages in LDS at once
constexpr int kStage = 128;     // cell records staged in LDS per batch of the per-species fold
constexpr int kStage1 = 256;    // cells staged in LDS per batch of the 1-D fold (one per thread)
constexpr int kGroup = 16;      // grid cells per support hull
constexpr int kVLen = GS_MAX_SPECIES + 4;  // 2-D gradient partials per block: species, 3 nuisances, pad
constexpr int kWaves = 4;       // wavefronts per workgroup cooperating on one tile
constexpr int kAdjGroupWaves = 2;  // workgroup size of the adjoint that gives each wave its own item
constexpr int kBlock = 256;     // threads per reduction block
constexpr int kHTile = kBlock / GS_MAX_SPECIES;  // energy bins per k_mv_bins block (multivariate models)
// k_bins2 rounds per block (BatchView::iter2): each block stages the toy's
// pulse-shape table, so large batches give a block kIter2Large rounds
// (kWaves x 16 window bins each) to pay for it; small ones one round, so that
// one model still fills the GPU
constexpr int kIter2Large = 8;
constexpr int kGradLen = GS_MAX_PARAMS;
// Zeroed window-bin rows after each toy's window: kernels that walk bins in
// steps of 16 read whole steps without clamping the bin index
constexpr int kWinPad = 16;
// Window rows a toy owns (binrec, F, H): its window, at least kWinPad zeroed
// rows, rounded up to a multiple of 16
constexpr int win_rows(int L) { return (L + kWinPad + 15) & ~15; }
constexpr int kCellBlock = 64;  // cells per k_cells block (one invalid-response flag each)
// cells per k_cellgrad block: kBlock (one per thread) for small batches, where
// the grid must fill the GPU, 4 * kBlock for large ones (one reduction per
// 1024 cells); BatchView::grad_cells holds the choice
constexpr int kGradCellsLarge = 1024;
constexpr int kGradLargeBlocks = 16384;
// window bins per k_tmpl block (one partial row per toy and block): 1024 for
// large template batches, 256 or 64 when fewer blocks would leave the GPU idle
constexpr int kTmplBlockBins = 1024;
constexpr int kTmplMinBlocks = 1024;  // blocks a template launch aims for before it shrinks the block
constexpr int kTmplGroup = 16;        // toys per k_tmpl group (the columns of its matrix products)

// Structure shared by every toy of one shape (spectra, grid, binning).
// Species are stored in internal order: grid species first, then lines;
// sp_of maps an internal species to its index in theta.
struct ShapeDev {
  int family, n_true, n_line, n_cell, S, Sg, n_reco, n_psd;
  double birks_A;
  const double *cellE;  // [n_cell]: grid-cell centres, then line energies
  const double *wcell;   // [n_true][Sg]: grid-species weights, cell-major
  const double *wcellT;  // [Sg][n_true]: the same, species-major (lanes on consecutive cells read coalesced)
  const double *w16;     // [n_cell][GS_MAX_SPECIES]: every cell's weights over the internal species (lines one-hot), zero-padded
  const double *bins;   // [n_reco][kBinLen]: xbar, dx, ln xbar (hi, lo)
  double bx0, bw;       // uniform binning: xbar_j = bx0 + j bw (bw = 0: not uniform)
  const double *edges;  // [n_reco + 1] reco-bin edges
  int gen;              // 1: the direct per-pair path (families >= kGenGammaPE, or exact bins)
  int exact;            // 1: reco-bin contents are the response's bin integrals
  double shape;         // generalized gamma power / modified Gaussian tail fraction
  const double *psd;    // [n_psd][2]: ybar, dy
  const double *mix;    // [S][5], internal species order
  int sp_of[GS_MAX_SPECIES];
};

// One toy (fit problem) of a batch; offsets index the batch-wide buffers.
struct ToyDev {
  int shape, D, lo, L, P, K, n_cell, S;
  int two_d;                    // 1: pulse-shape (secondary observable) model
  int tmpl;                     // 1: Monte Carlo template model (no fold, no response)
  int mv;                       // 1: multivariate slice likelihood (2-D toys with energy slices)
  int gen;                      // 1: response through the direct per-pair path (k_foldg, k_adjg)
  int n_slices, eblocks;        // mv: energy slices; k_mv_bins blocks (kHTile window bins each)
  int fold_chunks, adj_chunks;
  int bin_blocks, cell_blocks;  // reduction blocks over window bins (2-D: k_bins2 blocks) / cells (k_cellgrad)
  int hblocks;                  // 2-D: rows of rate pieces in vpart (joint: bin_blocks; multivariate: eblocks)
  int cflag_blocks;             // k_cells blocks (kCellBlock cells each)
  long long cell_off;   // rec[(cell_off + i) * kRecLen]
  long long win_off;    // binrec[(win_off + b) * kBinRecLen]
  long long fh_off;     // per-species window arrays: F[fh_off + b * S + s], H likewise (win_rows(L) rows of S)
  long long bref_off;   // adjoint block references: bref[(bref_off + q) * 4], q = b / kABlock
  long long cnt_off;    // counts of the window: cnt[cnt_off + (d * L + b) * K + k]
  long long nsum_off;   // joint 2-D: nsum[nsum_off + b * K + k] = sum_d n_dbk
  double cnl;           // joint 2-D: sum over the window's cells and datasets of n ln eps_d (k_finish subtracts it)
  long long fpart_off;  // fold partials: fpart[fpart_off + chunk * L + b]
  long long fs_off;     // per-species fold partials: fspart[fs_off + (chunk * L + b) * S + s]
  long long apart_off;  // adjoint partials: apart[apart_off + (chunk * n_cell + i) * 3 + q]
  long long nllp_off;   // -ln L partials per bin block
  long long gpart_off;  // per cell block: gpart[(gpart_off + blk) * kGradLen + p]
  long long cflag_off;  // per k_cells block: cflag[cflag_off + blk]
  long long ghull_off;  // per kGroup grid cells: union of their supports, ghull[ghull_off + g]
  long long pull_off;   // pull centres / widths [P]
  long long vpart_off;  // 2-D: vpart[(vpart_off + r) * kVLen + e], rows: hblocks of rate pieces, then bin_blocks of nuisance pieces
  long long psd_off;    // 2-D: P[psd_off + s * K + k], dP[(psd_off + s * K + k) * 3 + v]
  long long slice_off;  // mv: slice edges sedge[slice_off + i] (window bins, n_slices + 1)
  long long sig_off;    // mv: slice seeds sig[sig_off + i * S + s]
  double exposure[GS_MAX_DATASETS];
};

// One workgroup of the fold: kFoldTile (per-species fold) or kFoldTile1 (1-D
// fold) window bins of one toy against a cell range.
struct FoldItem {
  int toy, bin0, cell0, cell1, chunk;
};
// One workgroup of the adjoint: 64 cells of one toy against a window-bin range.
struct AdjItem {
  int toy, cell0, bin0, bin1, chunk;
};

// Device views of one batch, passed by value to the launchers.
struct BatchView {
  int n_toys, stride;
  const int *toy_list;  // per-toy grids cover toy_list[0 .. n_list) (NULL: every toy, n_list = n_toys)
  int n_list;
  // the same toys split by kind, for kernels of one kind (NULL list: toy_list / n_list)
  const int *list1d, *list2d, *listt;
  // k_tmpl groups: pairs (first position in listt, count) of toys sharing
  // shape, window and datasets
  const int *tgroup;
  int n_tgroup;
  int tmpl_bins;  // window bins per k_tmpl block (kTmplBlockBins, 256 or 64)
  int n1d, n2d, nt;  // 1-D analytic, 2-D and template toys
  int max_cells, max_cell_blocks, max_bin_blocks;
  int grad_cells;  // cells per k_cellgrad block (kBlock or kGradCellsLarge)
  int iter2;       // rounds per k_bins2 block (1 or kIter2Large)
  int adj_waves;   // waves per adjoint workgroup (1 or kWaves)
  int max_bin_blocks1, max_bin_blocks2;  // the same over 1-D / 2-D toys
  int max_ls_blocks;  // kBlock blocks over (window bin, species) pairs
  int max_psd_sk;     // largest S x K of a 2-D toy (P, dP are staged in LDS)
  int max_hblocks;    // largest hblocks over the joint 2-D toys
  double log_cut;   // pairs whose log-density is below this are skipped
  const ToyDev *toys;
  const ShapeDev *shapes;
  double *rec;      // cell records
  uint32_t *cflag;  // per k_cells block: an invalid response was met
  int2 *sup;        // per cell: reco-bin support [x, y) (also in slot 6 of the record)
  int2 *ghull;      // per kGroup grid cells: smallest x and largest y of their non-empty supports
  int max_cflag_blocks;
  double *fpart;    // fold partials (combined weight)
  double *fspart;   // fold partials per species
  double *F;        // per toy [win_rows(L)][S] from fh_off: per-species spectra of the window, bin width included
  double *apart;    // adjoint partials
  double *binrec;   // window bins: xbar, ln xbar hi, lo, G, G ln xbar, G xbar, block offsets u, v
  double *bref;     // per block of kABlock window bins: reference xbar, ln xbar (hi, lo), 0
  double *nllp;     // -ln L partials
  double *gpart;    // gradient partials
  uint32_t *badp;   // domain flags per bin block
  const double *cnt;
  const double *nsum;  // joint 2-D toys: counts summed over the datasets
  const double *pull_c, *pull_s;
  const FoldItem *fold_items;  // every toy's per-species fold items (kFoldTile bins): 1-D toys first, then 2-D
  int n_fold_items, n_fold1s;  // all of them / those of 1-D toys
  const AdjItem *adj_items;
  int n_adj_items;
  // by kind (1-D: k_fold1 on kFoldTile1-bin items, k_adj<false>; 2-D: k_fold_s, k_adj<true>)
  const FoldItem *fold1, *fold2;
  const AdjItem *adj1, *adj2;
  int n_fold1, n_fold2, n_adj1, n_adj2;
  // secondary observable (2-D) models
  double *H;        // per toy [win_rows(L)][S] from fh_off: dx_j sum_k P_sk Gam_jk
  double *P, *dP;   // pulse-shape probabilities and their nuisance derivatives
  double *vpart;    // per k_bins2 block: sum_j F_js sum_k P_sk Gam_jk (s), nuisance pieces
  uint32_t *pflag;  // [toy]: invalid pulse-shape nuisance
  const double *theta_dev;  // parameters of the evaluation in flight (per-species adjoint)
  int max_bin_blocks_t;  // k_tmpl grid
  int max_slices, max_eblocks, max_mv_cells;  // mv grids (slices; energy blocks; window bins x pulse-shape bins)
  const int *sedge;      // mv: slice edges per toy
  double *sig;           // mv: per (slice, species) seeds of the slice pieces
  bool has_mv;
  bool has_1d, has_2d, has_tmpl, has_gen;
};

// Which toys a launch covers.
enum ModeFilter : int { kAllToys = -1, kOnly1D = 0, kOnly2D = 1 };

// Launchers (gs_kernels.hip).  All enqueue on `st` and return the launch status.
hipError_t launch_bins_setup(double *bins, const double *edges, int n_reco, hipStream_t st);
hipError_t launch_cells(const BatchView &v, const double *theta, const uint8_t *active, hipStream_t st);
hipError_t launch_fold(const BatchView &v, bool per_species, int mode, const uint8_t *active, hipStream_t st);
hipError_t launch_bins1(const BatchView &v, double *mu_out, const uint8_t *active, hipStream_t st);
hipError_t launch_adj(const BatchView &v, bool per_species, const uint8_t *active, hipStream_t st);
hipError_t launch_cellgrad(const BatchView &v, const double *theta, const uint8_t *active, hipStream_t st);
hipError_t launch_finish(const BatchView &v, const double *theta, double *nll, double *grad, uint32_t *status,
                         const uint8_t *active, hipStream_t st);
hipError_t launch_reduceF(const BatchView &v, int mode, const uint8_t *active, hipStream_t st);
hipError_t launch_binsF(const BatchView &v, const double *theta, double *mu_out, hipStream_t st);
hipError_t launch_psd(const BatchView &v, const double *theta, const uint8_t *active, hipStream_t st);
hipError_t launch_mv(const BatchView &v, const double *theta, double *mu_out, const uint8_t *active, hipStream_t st);
hipError_t launch_tmpl(const BatchView &v, const double *theta, double *mu_out, const uint8_t *active, hipStream_t st);
hipError_t launch_bins2(const BatchView &v, const double *theta, double *mu_out, const uint8_t *active,
                        hipStream_t st);

}  // namespace gs
