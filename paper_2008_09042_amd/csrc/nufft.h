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
  const int2* base;           // [M] grid index of the first tap on each axis (wrapped)
  const float* wts;           // [M][2][W] tap weights phi(u - g) per axis
  const int32_t* tile_ptr;    // [ntiles + 1] CSR offsets of the spread tiles
  const int32_t* tile_idx;    // samples whose footprint meets each tile
  float cscale;               // sqrt(g0 g1 / (n0 n1)): unitary DFT -> the operator's scaling
};

int nufft_tiles(int g0, int g1);
int nufft_tile_edge();
hipError_t pad_deapod_launch(const NufftArgs& a, const float2* S, const float2* x, float2* grid, hipStream_t st);
hipError_t crop_deapod_launch(const NufftArgs& a, const float2* grid, float2* out, hipStream_t st);
hipError_t degrid_launch(const NufftArgs& a, const float2* grid, float2* y, hipStream_t st);
hipError_t spread_launch(const NufftArgs& a, const float2* y, float alpha, const float* scale_dev, float2* grid,
                         hipStream_t st);

}  // namespace mx
