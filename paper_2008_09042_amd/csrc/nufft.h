// Arguments and launchers of the Kaiser-Bessel NUFFT kernels (2D).
#pragma once

#include "common.h"

namespace mx {

struct NufftArgs {
  int n0, n1;                 // image
  int g0, g1;                 // oversampled grid (sigma * n)
  int J, W;                   // coils, kernel width (taps per axis, <= 8)
  int64_t M;                  // samples per coil
  const float* iphi0;         // [n0] 1 / Phi((r0 - n0/2) / g0)
  const float* iphi1;         // [n1]
  // the samples sorted by the cell (row-major) of their first tap (spread and degrid)
  const int32_t* cell_ptr;    // [g0 * g1 + 1] CSR offsets of the cells into the sorted order
  const int32_t* s_perm;      // [M] original index of each sorted sample
  const int32_t* s_inv;       // [M] sorted position of each sample (s_perm's inverse)
  const int32_t* s_col;       // [M] first-tap column of each sorted sample
  const int2* s_base;         // [M] first-tap (row, column) of each sorted sample
  const float* s_wts;         // [M][16] tap weights of each sorted sample: axis 0 in [0, W), axis 1 in [8, 8 + W)
  // spread blocks (SPREAD_ROWS grid rows, 64 columns) in which some lane's sample sequence
  // exceeds the split threshold: skipped by the plain kernels, their rows taken one by one
  // by the split-row workgroups
  const uint8_t* s_heavy;     // [ceil(g0 / SPREAD_ROWS) * ceil(g1 / 64)] 1 for a split block (may be null)
  const int32_t* s_hlist;     // [n_heavy] split rows: row * ceil(g1 / 64) + column block; the
                              // first n_med from blocks at most 4x over the threshold
  int n_heavy, n_med;
  int split_pm, split_ph;     // column parts of a split row: rows of moderately long blocks, of the longest
  int spread_lds;             // plain spread blocks: 1 stage the samples through LDS, 0 walk them from memory
  float cscale;               // sqrt(g0 g1 / (n0 n1)): unitary DFT -> the operator's scaling
};

// Coils per spread workgroup, and the bytes of the staging buffer the spread needs.
int spread_group(int J);
// Grid columns per spread block, and the default length of a grid point's sample sequence
// above which its block is split (MAXWELL_SPREAD_SPLIT in the environment at plan creation
// overrides it).
constexpr int SPREAD_COLS = 64;
#ifndef SPREAD_ROWS
#define SPREAD_ROWS 2   // grid rows per wave of the plain spread kernel
#endif
constexpr int SPREAD_SPLIT_DEFAULT = 48;
// Column parts of a split row (each a workgroup over 64 / P columns): rows of blocks at most
// four times over the threshold, and the longest (MAXWELL_SPREAD_SPLIT_PARTS=pm,ph overrides).
constexpr int SPREAD_SPLIT_PM = 4, SPREAD_SPLIT_PH = 16;
size_t spread_stage_bytes(int J, int64_t M);
hipError_t degrid_launch(const NufftArgs& a, const float2* grid, float2* y, hipStream_t st);
// grid = alpha * (*scale_dev) * spread(y); ys is a staging buffer of spread_stage_bytes(J, M).
// With `staged`, y is already in the staging layout (sorted samples, coils innermost, J a
// multiple of the coil group: ys[s][j] = y[j][perm[s]]) and ys is not used.
hipError_t spread_launch(const NufftArgs& a, const float2* y, float alpha, const float* scale_dev, float2* ys,
                         float2* grid, hipStream_t st, bool staged = false);

}  // namespace mx
