// gs_impl.h -- internal layout of models and batches on the device.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs.h"
#include "gs_dev.h"

namespace gs {

// Structure shared by every toy of one shape (spectra, grid, binning).
// Species are stored in internal order: grid species first, then lines;
// sp_of maps an internal species to its index in theta.
struct ShapeDev {
  int family, n_true, n_line, n_cell, S, Sg, n_reco, n_psd;
  double birks_A;
  const double *cellE;  // [n_cell]: grid-cell centres, then line energies
  const double *wcell;  // [n_true][Sg]: grid-species weights, cell-major
  const double *bins;   // [n_reco][kBinLen]: xbar, dx, ln xbar (hi, lo)
  const double *psd;    // [n_psd][2]: ybar, dy
  const double *mix;    // [S][5], internal species order
  int sp_of[GS_MAX_SPECIES];
};

// One toy (fit problem) of a batch; offsets index the batch-wide buffers.
struct ToyDev {
  int shape, D, lo, L, P, K, n_cell, S;
  int fold_chunks, adj_chunks;
  long long cell_off;   // cell records: rec[(cell_off + i) * kRecLen]
  long long win_off;    // window bins: binrec[(win_off + b) * kBinLen], F[(win_off + b) * S]
  long long cnt_off;    // counts of the window: cnt[cnt_off + (d * L + b) * K + k]
  long long fpart_off;  // fold partials
  long long apart_off;  // adjoint partials: apart[apart_off + (chunk * n_cell + i) * 3 + q]
  long long pull_off;   // pull centres / widths [P]
  double exposure[GS_MAX_DATASETS];
};

// One wavefront of the fold: 64 window bins of one toy against a cell range.
struct FoldItem {
  int toy, bin0, cell0, cell1, chunk;
};
// One wavefront of the adjoint: 64 cells of one toy against a window-bin range.
struct AdjItem {
  int toy, cell0, bin0, bin1, chunk;
};

// Device views of one batch, passed by value to the launchers.
struct BatchView {
  int n_toys, stride;
  const ToyDev *toys;
  const ShapeDev *shapes;
  double *rec;      // cell records
  double *fpart;    // fold partials (combined weight)
  double *apart;    // adjoint partials
  double *binrec;   // per toy window bins: xbar, ln xbar hi, lo, G
  const double *cnt;
  const double *pull_c, *pull_s;
  const FoldItem *fold_items;
  int n_fold_items;
  const AdjItem *adj_items;
  int n_adj_items;
  // per-species fold (plain path and 2-D)
  double *fspart;   // [toy][chunk][L][S]
  double *F;        // [toy][L][S], includes the bin width
  long long *fs_off;  // per toy offset into fspart
};

// Launchers (gs_kernels.hip).  All enqueue on `st` and return hipSuccess or the launch error.
hipError_t launch_cells(const BatchView &v, const double *theta, const uint8_t *active, int max_cells, hipStream_t st);
hipError_t launch_fold1(const BatchView &v, hipStream_t st);
hipError_t launch_nll1(const BatchView &v, const double *theta, double *nll, uint32_t *status, double *mu_out,
                       const uint8_t *active, hipStream_t st);
hipError_t launch_adj1(const BatchView &v, hipStream_t st);
hipError_t launch_grad1(const BatchView &v, const double *theta, const uint32_t *status, double *grad,
                        const uint8_t *active, hipStream_t st);
hipError_t launch_bins_setup(const ShapeDev *shape_d, double *bins, const double *edges, int n_reco, hipStream_t st);
hipError_t launch_foldS(const BatchView &v, hipStream_t st);
hipError_t launch_reduceF_grid(const BatchView &v, int max_LS, hipStream_t st);
hipError_t launch_nllF(const BatchView &v, const double *theta, double *nll, uint32_t *status, double *mu_out,
                       hipStream_t st);

}  // namespace gs
