// Kaiser-Bessel non-uniform FFT for non-Cartesian (radial) sampling.
//
// The paper uses the same operator for non-Cartesian trajectories once F is
// available (Sec. III-B); F is approximated by the standard gridding NUFFT
// with an oversampled grid (sigma * n) and a width-W Kaiser-Bessel kernel:
//
//   type 2 (image -> samples)   deapodise and zero-pad (pad kernel), centred DFT
//                               on the oversampled grid (per-axis FFT kernel),
//                               interpolate W x W taps per sample (degrid kernel)
//   type 1 (samples -> image)   exact transpose: spread (grid kernel), inverse
//                               DFT, crop and deapodise (crop kernel)
//
// The spread is output-stationary: the grid is cut into 32 x 32 tiles; at plan
// time every sample is listed under each tile its footprint touches (with the
// periodic wrap of the grid); a workgroup stages its tile's samples through
// LDS and every thread sums the contributions to its own grid points in list
// order.  No atomics, so results are bitwise reproducible.
//
// Per-sample tap weights phi(u - g) are computed on the host in FP64 at plan
// time (I0 from its power series), so the kernels only multiply and add.
#include "common.h"
#include "nufft.h"

namespace mx {

namespace {

constexpr int NT = 256;

// Grid[j][a][b] = S[j][r0][r1] x[r0][r1] / (Phi0[r0] Phi1[r1]) inside the centred
// window of the oversampled grid, zero elsewhere.
__global__ void pad_deapod_kernel(NufftArgs a, const float2* __restrict__ S, const float2* __restrict__ x,
                                  float2* __restrict__ grid) {
  const int64_t G = (int64_t)a.g0 * a.g1;
  const int64_t total = G * a.J;
  const int off0 = a.g0 / 2 - a.n0 / 2, off1 = a.g1 / 2 - a.n1 / 2;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t j = e / G, q = e % G;
    const int ga = (int)(q / a.g1), gb = (int)(q % a.g1);
    const int r0 = ga - off0, r1 = gb - off1;
    float2 v = make_float2(0.f, 0.f);
    if (r0 >= 0 && r0 < a.n0 && r1 >= 0 && r1 < a.n1) {
      const int64_t r = (int64_t)r0 * a.n1 + r1;
      v = cscale(cmul(S[j * (int64_t)a.n0 * a.n1 + r], x[r]), a.iphi0[r0] * a.iphi1[r1]);
    }
    grid[e] = v;
  }
}

// out[j][r] = scale * Grid[j][r + off] / (Phi0 Phi1)
__global__ void crop_deapod_kernel(NufftArgs a, const float2* __restrict__ grid, float2* __restrict__ out) {
  const int64_t N = (int64_t)a.n0 * a.n1, G = (int64_t)a.g0 * a.g1;
  const int64_t total = N * a.J;
  const int off0 = a.g0 / 2 - a.n0 / 2, off1 = a.g1 / 2 - a.n1 / 2;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t j = e / N, r = e % N;
    const int r0 = (int)(r / a.n1), r1 = (int)(r % a.n1);
    const float2 v = grid[j * G + (int64_t)(r0 + off0) * a.g1 + (r1 + off1)];
    out[e] = cscale(v, a.iphi0[r0] * a.iphi1[r1]);
  }
}

// y[j][m] = c * sum_{t0, t1} w0[m][t0] w1[m][t1] Grid[j][(b0 + t0) mod g0][(b1 + t1) mod g1]
__global__ void degrid_kernel(NufftArgs a, const float2* __restrict__ grid, float2* __restrict__ y) {
  const int64_t G = (int64_t)a.g0 * a.g1;
  const int64_t total = a.M * a.J;
  const int W = a.W;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t j = e / a.M, m = e % a.M;
    const int2 b = a.base[m];
    const float* w0 = a.wts + m * 2 * W;
    const float* w1 = w0 + W;
    const float2* gj = grid + j * G;
    float2 acc = make_float2(0.f, 0.f);
    for (int t0 = 0; t0 < W; ++t0) {
      int ga = b.x + t0;
      if (ga >= a.g0) ga -= a.g0;
      float2 row = make_float2(0.f, 0.f);
      for (int t1 = 0; t1 < W; ++t1) {
        int gb = b.y + t1;
        if (gb >= a.g1) gb -= a.g1;
        const float2 gv = gj[(int64_t)ga * a.g1 + gb];
        row.x += w1[t1] * gv.x;
        row.y += w1[t1] * gv.y;
      }
      acc.x += w0[t0] * row.x;
      acc.y += w0[t0] * row.y;
    }
    y[e] = cscale(acc, a.cscale);
  }
}

// Output-stationary spread: one workgroup per (coil, tile).
constexpr int TILE = 32;            // tile edge (grid cells)
constexpr int BATCH = 256;          // samples staged per LDS round

__global__ __launch_bounds__(NT) void spread_kernel(NufftArgs a, const float2* __restrict__ y, float alpha,
                                                    const float* __restrict__ scale_dev, float2* __restrict__ grid) {
  __shared__ int2 sb[BATCH];
  __shared__ float sw[BATCH][2 * 8];
  __shared__ float2 sy[BATCH];
  const int tiles1 = (a.g1 + TILE - 1) / TILE;
  const int ntiles = ((a.g0 + TILE - 1) / TILE) * tiles1;
  const int j = blockIdx.x / ntiles, tile = blockIdx.x % ntiles;
  const int ta = (tile / tiles1) * TILE, tb = (tile % tiles1) * TILE;
  const int W = a.W;
  float s = alpha * a.cscale;
  if (scale_dev) s *= *scale_dev;
  // each thread owns 4 grid points of the tile: rows ta + (threadIdx.x / 32) + 8 q, column tb + threadIdx.x % 32
  const int cb = tb + (threadIdx.x % TILE);
  float2 acc[4];
  int ra[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    acc[q] = make_float2(0.f, 0.f);
    ra[q] = ta + (threadIdx.x / TILE) + 8 * q;
  }
  const int beg = a.tile_ptr[tile], end = a.tile_ptr[tile + 1];
  for (int b0 = beg; b0 < end; b0 += BATCH) {
    const int nb = (end - b0) < BATCH ? (end - b0) : BATCH;
    __syncthreads();
    for (int e = threadIdx.x; e < nb; e += NT) {
      const int m = a.tile_idx[b0 + e];
      sb[e] = a.base[m];
      for (int t = 0; t < 2 * W; ++t) sw[e][t] = a.wts[(int64_t)m * 2 * W + t];
      sy[e] = y[(int64_t)j * a.M + m];
    }
    __syncthreads();
    for (int e = 0; e < nb; ++e) {
      const int2 b = sb[e];
      int t1 = cb - b.y;
      if (t1 < 0) t1 += a.g1;
      if (t1 >= W) continue;
      const float w1 = sw[e][W + t1];
      const float2 yv = sy[e];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int t0 = ra[q] - b.x;
        if (t0 < 0) t0 += a.g0;
        if (t0 < W) {
          const float w = sw[e][t0] * w1;
          acc[q].x += w * yv.x;
          acc[q].y += w * yv.y;
        }
      }
    }
  }
  const int64_t G = (int64_t)a.g0 * a.g1;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (ra[q] < a.g0 && cb < a.g1) grid[(int64_t)j * G + (int64_t)ra[q] * a.g1 + cb] = cscale(acc[q], s);
}

inline unsigned grid_for(int64_t total) {
  int64_t b = (total + NT - 1) / NT;
  if (b > 16384) b = 16384;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

int nufft_tiles(int g0, int g1) { return ((g0 + TILE - 1) / TILE) * ((g1 + TILE - 1) / TILE); }
int nufft_tile_edge() { return TILE; }

hipError_t pad_deapod_launch(const NufftArgs& a, const float2* S, const float2* x, float2* grid, hipStream_t st) {
  hipLaunchKernelGGL(pad_deapod_kernel, dim3(grid_for((int64_t)a.g0 * a.g1 * a.J)), dim3(NT), 0, st, a, S, x, grid);
  return hipGetLastError();
}

hipError_t crop_deapod_launch(const NufftArgs& a, const float2* grid, float2* out, hipStream_t st) {
  hipLaunchKernelGGL(crop_deapod_kernel, dim3(grid_for((int64_t)a.n0 * a.n1 * a.J)), dim3(NT), 0, st, a, grid, out);
  return hipGetLastError();
}

hipError_t degrid_launch(const NufftArgs& a, const float2* grid, float2* y, hipStream_t st) {
  if (a.M * a.J == 0) return hipSuccess;
  hipLaunchKernelGGL(degrid_kernel, dim3(grid_for(a.M * a.J)), dim3(NT), 0, st, a, grid, y);
  return hipGetLastError();
}

hipError_t spread_launch(const NufftArgs& a, const float2* y, float alpha, const float* scale_dev, float2* grid,
                         hipStream_t st) {
  const int nt = nufft_tiles(a.g0, a.g1);
  hipLaunchKernelGGL(spread_kernel, dim3((unsigned)(nt * a.J)), dim3(NT), 0, st, a, y, alpha, scale_dev, grid);
  return hipGetLastError();
}

}  // namespace mx
