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
// The spread is output-stationary: every grid point gathers the samples whose
// W x W footprint covers it, found through a plan-time sort of the samples by
// grid cell, and sums them in a fixed order.  No atomics, so results are
// bitwise reproducible.
//
// Per-sample tap weights phi(u - g) are computed on the host in FP64 at plan
// time (I0 from its power series), so the kernels only multiply and add.
#include "common.h"
#include "nufft.h"

namespace mx {

namespace {

constexpr int NT = 256;

constexpr int SREC = 16;            // floats per sorted-sample weight record: w0 [0, 8), w1 [8, 16)

// y[j][m] = c * sum_{t0, t1} w0[m][t0] w1[m][t1] Grid[j][(b0 + t0) mod g0][(b1 + t1) mod g1],
// b the first tap per axis and w the tap weights of sample m.
// The width is a template argument so the W x W taps unroll and their loads are all in
// flight together.
template <int W>
__global__ __launch_bounds__(NT) void degrid_kernel(NufftArgs a, const float2* __restrict__ grid,
                                                    float2* __restrict__ y) {
  const int64_t G = (int64_t)a.g0 * a.g1;
  const int64_t total = a.M * a.J;
  // consecutive blocks (neighbouring samples, which read the same grid rows) go to one XCD:
  // the hardware deals workgroups round-robin over the 8 XCDs, each with its own L2
  const int64_t nb = gridDim.x;
  int64_t bid = blockIdx.x;
  if ((nb & 7) == 0) bid = (bid & 7) * (nb >> 3) + (bid >> 3);
  for (int64_t e = bid * NT + threadIdx.x; e < total; e += nb * NT) {
    // samples in first-tap cell order, so the lanes of a wave read overlapping grid rows
    // (against sample order: 40 -> 24 us at 512^2, 16 coils, 64 spokes x 512)
    const int64_t j = e / a.M, s = e % a.M;
    const int64_t m = a.s_perm[s];
    const int2 b = a.s_base[s];
    const float* w0 = a.s_wts + s * SREC;
    const float* w1 = w0 + 8;
    const float2* gj = grid + j * G;
    int col[W];
#pragma unroll
    for (int t1 = 0; t1 < W; ++t1) col[t1] = b.y + t1 < a.g1 ? b.y + t1 : b.y + t1 - a.g1;
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int t0 = 0; t0 < W; ++t0) {
      const int ga = b.x + t0 < a.g0 ? b.x + t0 : b.x + t0 - a.g0;
      const float2* gr = gj + (int64_t)ga * a.g1;
      float2 row = make_float2(0.f, 0.f);
#pragma unroll
      for (int t1 = 0; t1 < W; ++t1) {
        const float2 gv = gr[col[t1]];
        row.x += w1[t1] * gv.x;
        row.y += w1[t1] * gv.y;
      }
      acc.x += w0[t0] * row.x;
      acc.y += w0[t0] * row.y;
    }
    y[j * a.M + m] = cscale(acc, a.cscale);
  }
}

// Spread, gather form.  Samples are sorted at plan time by the grid cell of their first
// tap (row-major), with a CSR over the cells; grid point (r, c) receives the samples whose
// first tap lies in rows r-W+1..r and columns c-W+1..c (periodic): for each row offset t0 a
// window of W consecutive cells, which is one contiguous range of sorted samples (two at
// the column wrap).  A staging pass first gathers the samples' values into sorted order,
// coil-minor and padded to a whole number of coil groups, so a thread reads each sample's
// JG values as one contiguous run.
//
// A wave covers one grid row, 64 columns (one per lane) and JG coils: each lane takes the W
// row windows of its column in t0 order as one sequence of samples, with two samples' loads in
// flight, and writes its sums (fixed order, no atomics, no LDS).  Most grid points see a few
// samples, so the wave's time is the latency of a few dependent loads; one wave per block
// keeps the whole grid resident at once.  The blocks whose longest sequence is long (the
// dense centre of a radial trajectory, where a grid point sees hundreds of samples) are
// marked at plan time; their rows are split over many lanes per grid point (split rows,
// below), in the same launch as the plain blocks when those are staged through LDS.
constexpr int SPC = SPREAD_COLS;    // grid columns per workgroup (one per lane)

// ys[inv[m]][j] = y[j][m] for j < J, 0 for J <= j < Jp.  A thread per sample m reads its
// coils down the columns of y (coalesced over m across a wave; the inverse permutation's load
// does not hold them up) and writes its Jp values as one contiguous run (a 128-byte line at 16
// coils), 16 bytes at a time where Jp is even.
__global__ __launch_bounds__(NT) void spread_stage_kernel(NufftArgs a, const float2* __restrict__ y, int Jp,
                                                          float2* __restrict__ ys) {
  const int64_t m = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (m >= a.M) return;
  float2* dst = ys + (int64_t)a.s_inv[m] * Jp;
  for (int j0 = 0; j0 < Jp; j0 += 8) {
    float2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = min(j0 + u, a.J - 1);  // in range; the value is dropped past J
      v[u] = y[(int64_t)j * a.M + m];
      if (j0 + u >= a.J) v[u] = make_float2(0.f, 0.f);
    }
    if ((Jp & 1) == 0) {
#pragma unroll
      for (int u = 0; u < 8; u += 2)
        if (j0 + u < Jp) reinterpret_cast<float4*>(dst + j0)[u / 2] = make_float4(v[u].x, v[u].y, v[u + 1].x, v[u + 1].y);
    } else {
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (j0 + u < Jp) dst[j0 + u] = v[u];
    }
  }
}

__device__ __forceinline__ float pick8(float4 lo, float4 hi, int t) {
  float v = lo.x;
  v = t == 1 ? lo.y : v;
  v = t == 2 ? lo.z : v;
  v = t == 3 ? lo.w : v;
  v = t == 4 ? hi.x : v;
  v = t == 5 ? hi.y : v;
  v = t == 6 ? hi.z : v;
  v = t == 7 ? hi.w : v;
  return v;
}

// acc += sum over the sorted samples s + k step + u (u < U, k >= 0) in [s, e) of
// w0[t0] w1[c - col] ys[.][jo .. jo + JG).  The loads of U samples depend on the position
// only and are all issued before any is used; the whole w1 record is loaded and the tap
// picked in registers (the empty asm keeps the compiler from turning the pick back into a
// load that waits on col).
template <int JG, int U>
__device__ __forceinline__ void spread_range(const NufftArgs& a, const float2* __restrict__ ys, int Jp, int jo,
                                             int c, int t0, int s, int e, int step, float2 (&acc)[JG]) {
  const float4* rec = reinterpret_cast<const float4*>(a.s_wts);
  constexpr int YV = JG >= 2 ? JG / 2 : 1;
  for (; s < e; s += step) {
    int col[U];
    float w0[U];
    float4 w1l[U], w1h[U];
    float4 yv[U][YV];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int su = min(s + u, e - 1);
      col[u] = a.s_col[su];
      w0[u] = a.s_wts[(int64_t)su * SREC + t0];
      w1l[u] = rec[(int64_t)su * (SREC / 4) + 2];
      w1h[u] = rec[(int64_t)su * (SREC / 4) + 3];
      const float2* yr = ys + (int64_t)su * Jp + jo;
      if constexpr (JG == 1) {
        const float2 v = yr[0];
        yv[u][0] = make_float4(v.x, v.y, 0.f, 0.f);
      } else {
#pragma unroll
        for (int q = 0; q < YV; ++q) yv[u][q] = reinterpret_cast<const float4*>(yr)[q];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      asm volatile("" : "+v"(w1l[u].x), "+v"(w1l[u].y), "+v"(w1l[u].z), "+v"(w1l[u].w));
      asm volatile("" : "+v"(w1h[u].x), "+v"(w1h[u].y), "+v"(w1h[u].z), "+v"(w1h[u].w));
      int t1 = c - col[u];
      if (t1 < 0) t1 += a.g1;
      const float w = (s + u < e ? w0[u] : 0.f) * pick8(w1l[u], w1h[u], t1);
      if constexpr (JG == 1) {
        acc[0].x += w * yv[u][0].x;
        acc[0].y += w * yv[u][0].y;
      } else {
#pragma unroll
        for (int q = 0; q < YV; ++q) {
          acc[2 * q].x += w * yv[u][q].x;
          acc[2 * q].y += w * yv[u][q].y;
          acc[2 * q + 1].x += w * yv[u][q].z;
          acc[2 * q + 1].y += w * yv[u][q].w;
        }
      }
    }
  }
}

// Split rows: the rows of the blocks in which some grid point sees more samples than the
// split threshold (the dense centre of a radial trajectory, where it sees hundreds).  One
// workgroup of four waves takes one split row, SCOL = 64 / P of its block's columns and JG
// coils, with P = split_pm for the rows of blocks at most four times over the threshold and
// split_ph for the longest.  A column is shared by 4 P lanes (P per wave): a lane walks the
// column's W row windows (cell row r - t0 for tap t0 = 0 .. W - 1, each the W cells ending at
// the column) as one sequence of samples and takes every (4 P)-th group of U consecutive
// positions.  The 4 P partial sums of an output are added through LDS (spart, 256 JG
// entries) in share order: fixed, no atomics.  Used by the LDS plain kernel's launch (its
// workgroups after the plain ones) and by spread_split_kernel, so both paths add the same
// products in the same order.
template <int JG, int W, int U>
__device__ __forceinline__ void spread_split_block(const NufftArgs& a, const float2* __restrict__ ys, int Jp,
                                                   float alpha, const float* __restrict__ scale_dev,
                                                   float2* __restrict__ grid, int bid, float2* spart) {
  const int bc = (a.g1 + SPC - 1) / SPC;
  const int per_g = a.split_pm * a.n_med + a.split_ph * (a.n_heavy - a.n_med);
  const int jg = bid / per_g;
  int rem = bid - jg * per_g, P, h;
  if (rem < a.split_pm * a.n_med) {
    P = a.split_pm;
    h = rem / P;
    rem -= h * P;
  } else {
    rem -= a.split_pm * a.n_med;
    P = a.split_ph;
    h = a.n_med + rem / P;
    rem -= (h - a.n_med) * P;
  }
  const int SCOL = SPC / P;
  const int blk = a.s_hlist[h];
  const int r = blk / bc, c0 = (blk % bc) * SPC + rem * SCOL;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int cc = lane % SCOL, ls = lane / SCOL;
  const int share = wave * P + ls, nshare = 4 * P;
  const bool live = c0 + cc < a.g1;
  const int c = live ? c0 + cc : a.g1 - 1;  // a lane past the last column walks nothing
  const int jo = jg * JG;
  // row window t0 contributes [rb[2 t0], + len) then [rb[2 t0 + 1], + len) (the second one
  // non-empty only at the column wrap); all offsets are loaded unconditionally
  int rb[2 * W], cum[2 * W + 1];
  {
    const int lo = c - W + 1;
    const int i0 = lo >= 0 ? lo : a.g1 + lo, i1 = lo >= 0 ? c + 1 : a.g1, i3 = lo >= 0 ? 0 : c + 1;
    int v0[W], v1[W], v2[W], v3[W];
#pragma unroll
    for (int t = 0; t < W; ++t) {
      const int row = ((r - t) % a.g0 + a.g0) % a.g0;
      const int32_t* cp = a.cell_ptr + (int64_t)row * a.g1;
      v0[t] = cp[i0];
      v1[t] = cp[i1];
      v2[t] = cp[0];
      v3[t] = cp[i3];
    }
    cum[0] = 0;
#pragma unroll
    for (int t = 0; t < W; ++t) {
      rb[2 * t] = v0[t];
      cum[2 * t + 1] = cum[2 * t] + (v1[t] - v0[t]);
      rb[2 * t + 1] = v2[t];
      cum[2 * t + 2] = cum[2 * t + 1] + (v3[t] - v2[t]);
    }
  }
  const int total = live ? cum[2 * W] : 0;
  const float4* rec = reinterpret_cast<const float4*>(a.s_wts);
  constexpr int YV = JG >= 2 ? JG / 2 : 1;
  float2 acc[JG];
#pragma unroll
  for (int q = 0; q < JG; ++q) acc[q] = make_float2(0.f, 0.f);
  for (int k = U * share; k < total; k += U * nshare) {
    int col[U];
    float w0[U];
    float4 w1l[U], w1h[U];
    float4 yv[U][YV];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int kk = min(k + u, total - 1);
      // the last range whose start is at or before kk holds it (empty ranges are passed over)
      int su = rb[0] + kk, t = 0;
#pragma unroll
      for (int j = 1; j < 2 * W; ++j)
        if (kk >= cum[j]) {
          su = rb[j] + (kk - cum[j]);
          t = j / 2;
        }
      col[u] = a.s_col[su];
      w0[u] = a.s_wts[(int64_t)su * SREC + t];
      w1l[u] = rec[(int64_t)su * (SREC / 4) + 2];
      w1h[u] = rec[(int64_t)su * (SREC / 4) + 3];
      const float2* yr = ys + (int64_t)su * Jp + jo;
      if constexpr (JG == 1) {
        const float2 v = yr[0];
        yv[u][0] = make_float4(v.x, v.y, 0.f, 0.f);
      } else {
#pragma unroll
        for (int q = 0; q < YV; ++q) yv[u][q] = reinterpret_cast<const float4*>(yr)[q];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      asm volatile("" : "+v"(w1l[u].x), "+v"(w1l[u].y), "+v"(w1l[u].z), "+v"(w1l[u].w));
      asm volatile("" : "+v"(w1h[u].x), "+v"(w1h[u].y), "+v"(w1h[u].z), "+v"(w1h[u].w));
      int t1 = c - col[u];
      if (t1 < 0) t1 += a.g1;
      const float w = (k + u < total ? w0[u] : 0.f) * pick8(w1l[u], w1h[u], t1);
      if constexpr (JG == 1) {
        acc[0].x += w * yv[u][0].x;
        acc[0].y += w * yv[u][0].y;
      } else {
#pragma unroll
        for (int q = 0; q < YV; ++q) {
          acc[2 * q].x += w * yv[u][q].x;
          acc[2 * q].y += w * yv[u][q].y;
          acc[2 * q + 1].x += w * yv[u][q].z;
          acc[2 * q + 1].y += w * yv[u][q].w;
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < JG; ++q) spart[(int)threadIdx.x * JG + q] = acc[q];
  __syncthreads();
  float sc = alpha * a.cscale;
  if (scale_dev) sc *= *scale_dev;
  const int64_t G = (int64_t)a.g0 * a.g1;
  for (int o = threadIdx.x; o < JG * SCOL; o += 256) {
    const int q = o / SCOL, l = o % SCOL;
    if (c0 + l >= a.g1 || jo + q >= a.J) continue;
    float2 v = make_float2(0.f, 0.f);
    for (int w = 0; w < 4; ++w)
      for (int s2 = 0; s2 < P; ++s2) {
        const float2 p = spart[(w * 64 + s2 * SCOL + l) * JG + q];
        v.x += p.x;
        v.y += p.y;
      }
    grid[(int64_t)(jo + q) * G + (int64_t)r * a.g1 + c0 + l] = cscale(v, sc);
  }
}

template <int JG, int W>
__global__ __launch_bounds__(256) void spread_split_kernel(NufftArgs a, const float2* __restrict__ ys, int Jp,
                                                           float alpha, const float* __restrict__ scale_dev,
                                                           float2* __restrict__ grid) {
  __shared__ float2 spart[256 * JG];
  spread_split_block<JG, W, 2>(a, ys, Jp, alpha, scale_dev, grid, (int)blockIdx.x, spart);
}

// One wave per (coil group, R grid rows, 64 columns); four waves per workgroup.  Output row
// r0 + i of a lane takes the samples of cell rows r0 + i - t0 (t0 < W); over its R rows the
// lane walks the W + R - 1 cell rows r0 + R - 1 - t (t = 0 .. W + R - 2) once, in t order,
// and adds each sample to every row i with tap t0 = i - R + 1 + t in [0, W): one load of a
// sample's values serves up to R outputs.
template <int JG, int W, int R, int U>
__global__ __launch_bounds__(256) void spread_flat_kernel(NufftArgs a, const float2* __restrict__ ys, int Jp,
                                                          float alpha, const float* __restrict__ scale_dev,
                                                          float2* __restrict__ grid) {
  constexpr int NW = W + R - 1;  // cell rows walked
  const int bc = (a.g1 + SPC - 1) / SPC;
  const int64_t nblk = (int64_t)((a.g0 + R - 1) / R) * bc;
  const int64_t id = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (id >= nblk * (Jp / JG)) return;
  const int jg = (int)(id / nblk), blk = (int)(id % nblk);
  if (a.s_heavy && a.s_heavy[blk]) return;  // split rows, taken by spread_split_kernel
  const int r0 = (blk / bc) * R, c = (blk % bc) * SPC + threadIdx.x % 64;
  if (c >= a.g1) return;  // no barrier or cross-lane operation follows
  const int jo = jg * JG;
  // cell row t contributes [rb[2 t], + len) then [rb[2 t + 1], + len) (the second one
  // non-empty only at the column wrap); all offsets are loaded unconditionally
  int rb[2 * NW], cum[2 * NW + 1];
  {
    const int lo = c - W + 1;
    const int i0 = lo >= 0 ? lo : a.g1 + lo, i1 = lo >= 0 ? c + 1 : a.g1, i3 = lo >= 0 ? 0 : c + 1;
    int v0[NW], v1[NW], v2[NW], v3[NW];
#pragma unroll
    for (int t = 0; t < NW; ++t) {
      const int row = ((r0 + R - 1 - t) % a.g0 + a.g0) % a.g0;
      const int32_t* cp = a.cell_ptr + (int64_t)row * a.g1;
      v0[t] = cp[i0];
      v1[t] = cp[i1];
      v2[t] = cp[0];
      v3[t] = cp[i3];
    }
    cum[0] = 0;
#pragma unroll
    for (int t = 0; t < NW; ++t) {
      rb[2 * t] = v0[t];
      cum[2 * t + 1] = cum[2 * t] + (v1[t] - v0[t]);
      rb[2 * t + 1] = v2[t];
      cum[2 * t + 2] = cum[2 * t + 1] + (v3[t] - v2[t]);
    }
  }
  const int total = cum[2 * NW];
  const float4* rec = reinterpret_cast<const float4*>(a.s_wts);
  constexpr int YV = JG >= 2 ? JG / 2 : 1;
  float2 acc[R][JG];
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int q = 0; q < JG; ++q) acc[i][q] = make_float2(0.f, 0.f);
  for (int k = 0; k < total; k += U) {
    int col[U], tw[U];
    float4 w0l[U], w0h[U], w1l[U], w1h[U];
    float4 yv[U][YV];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int kk = min(k + u, total - 1);
      // the last range whose start is at or before kk holds it (empty ranges are passed over)
      int su = rb[0] + kk, t = 0;
#pragma unroll
      for (int j = 1; j < 2 * NW; ++j)
        if (kk >= cum[j]) {
          su = rb[j] + (kk - cum[j]);
          t = j / 2;
        }
      tw[u] = t;
      col[u] = a.s_col[su];
      if constexpr (R == 1) {
        w0l[u] = make_float4(a.s_wts[(int64_t)su * SREC + t], 0.f, 0.f, 0.f);
        w0h[u] = w0l[u];
      } else {
        w0l[u] = rec[(int64_t)su * (SREC / 4) + 0];
        w0h[u] = rec[(int64_t)su * (SREC / 4) + 1];
      }
      w1l[u] = rec[(int64_t)su * (SREC / 4) + 2];
      w1h[u] = rec[(int64_t)su * (SREC / 4) + 3];
      const float2* yr = ys + (int64_t)su * Jp + jo;
      if constexpr (JG == 1) {
        const float2 v = yr[0];
        yv[u][0] = make_float4(v.x, v.y, 0.f, 0.f);
      } else {
#pragma unroll
        for (int q = 0; q < YV; ++q) yv[u][q] = reinterpret_cast<const float4*>(yr)[q];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      asm volatile("" : "+v"(w0l[u].x), "+v"(w0l[u].y), "+v"(w0l[u].z), "+v"(w0l[u].w));
      asm volatile("" : "+v"(w0h[u].x), "+v"(w0h[u].y), "+v"(w0h[u].z), "+v"(w0h[u].w));
      asm volatile("" : "+v"(w1l[u].x), "+v"(w1l[u].y), "+v"(w1l[u].z), "+v"(w1l[u].w));
      asm volatile("" : "+v"(w1h[u].x), "+v"(w1h[u].y), "+v"(w1h[u].z), "+v"(w1h[u].w));
      int t1 = c - col[u];
      if (t1 < 0) t1 += a.g1;
      const float w1 = (k + u < total ? 1.f : 0.f) * pick8(w1l[u], w1h[u], t1);
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int t0 = i - R + 1 + tw[u];
        float w0;
        if constexpr (R == 1) {
          w0 = w0l[u].x;
        } else {
          w0 = (t0 >= 0 && t0 < W) ? pick8(w0l[u], w0h[u], t0) : 0.f;
        }
        const float w = w0 * w1;
        if constexpr (JG == 1) {
          acc[i][0].x += w * yv[u][0].x;
          acc[i][0].y += w * yv[u][0].y;
        } else {
#pragma unroll
          for (int q = 0; q < YV; ++q) {
            acc[i][2 * q].x += w * yv[u][q].x;
            acc[i][2 * q].y += w * yv[u][q].y;
            acc[i][2 * q + 1].x += w * yv[u][q].z;
            acc[i][2 * q + 1].y += w * yv[u][q].w;
          }
        }
      }
    }
  }
  float sc = alpha * a.cscale;
  if (scale_dev) sc *= *scale_dev;
  const int64_t G = (int64_t)a.g0 * a.g1;
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int q = 0; q < JG; ++q)
      if (r0 + i < a.g0 && jo + q < a.J)
        grid[(int64_t)(jo + q) * G + (int64_t)(r0 + i) * a.g1 + c] = cscale(acc[i][q], sc);
}

// The same blocks with the samples staged through LDS.  A wave's samples are the sorted
// ranges of its W + R - 1 cell rows over the columns [c0 - W + 1, c0 + 64) (two ranges in a
// row whose window wraps past column 0), taken as one sequence of `total` records.  The
// wave stages 64 consecutive records at a time (one per lane, coalesced: column, the tap of
// each of its R output rows, the W column taps, the JG coil values), the next chunk loaded
// into registers while the current one is used; each lane then adds the records of its own
// window, which are consecutive in every range.  Fixed order per grid point: ranges in
// (cell row, wrapped part first) order, samples in sorted order, as in the plain kernel.
template <int JG, int W, int R>
__global__ __launch_bounds__(256, 4) void spread_lds_kernel(NufftArgs a, const float2* __restrict__ ys, int Jp,
                                                         float alpha, const float* __restrict__ scale_dev,
                                                         float2* __restrict__ grid) {
  constexpr int NW = W + R - 1;  // cell rows
  constexpr int NS = 2 * NW;     // ranges: (cell row t, part p), p = 0 wrapped columns, 1 the rest
  constexpr int YV = JG >= 2 ? JG / 2 : 1;
  struct Chunk {
    float2 y[SPC][JG];
    float w1[W][SPC];
    float w0[R][SPC];
    int col[SPC];
  };
  __shared__ Chunk chunks[4];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  Chunk& ck = chunks[wave];
  const int bc = (a.g1 + SPC - 1) / SPC;
  const int64_t nblk = (int64_t)((a.g0 + R - 1) / R) * bc;
  // workgroups past the plain blocks' take the split rows, with the chunk staging as their
  // partial sums (uniform per workgroup, so the split rows' barrier is reached by all)
  const int64_t nplain = (nblk * (Jp / JG) + 3) / 4;
  if ((int64_t)blockIdx.x >= nplain) {
    static_assert(sizeof(chunks) >= 256 * JG * sizeof(float2), "split partial sums fit the staging");
    spread_split_block<JG, W, 2>(a, ys, Jp, alpha, scale_dev, grid, (int)(blockIdx.x - nplain),
                                 reinterpret_cast<float2*>(chunks));
    return;
  }
  // consecutive plain workgroups (neighbouring row blocks, which read the same cell rows'
  // samples) go to one XCD: the hardware deals workgroups round-robin over the 8 XCDs
  int64_t bx = blockIdx.x;
  const int64_t np8 = nplain & ~(int64_t)7;
  if (bx < np8) bx = (bx & 7) * (np8 >> 3) + (bx >> 3);
  const int64_t id = bx * 4 + wave;
  if (id >= nblk * (Jp / JG)) return;  // whole waves only: no workgroup barrier follows
  const int jg = (int)(id / nblk), blk = (int)(id % nblk);
  if (a.s_heavy && a.s_heavy[blk]) return;  // split rows, taken by the workgroups after these
  const int r0 = (blk / bc) * R, c0 = (blk % bc) * SPC, c = c0 + lane;
  const bool live = c < a.g1;
  const int jo = jg * JG;
  const int lo_w = c0 - W + 1, hi_w = min(c0 + SPC, a.g1);
  // range starts, lengths and the lane's part of each (as offsets into the range)
  int S[NS], cum[NS + 1];
  unsigned lr[NS];  // the lane's part of range q: [lr & 0xffff, lr >> 16) (ranges hold < 65536 samples)
  cum[0] = 0;
#pragma unroll
  for (int t = 0; t < NW; ++t) {
    const int row = ((r0 + R - 1 - t) % a.g0 + a.g0) % a.g0;
    const int32_t* cp = a.cell_ptr + (int64_t)row * a.g1;
    const int lo = c - W + 1;
    // part 0: columns [g1 + lo_w, g1), present when the wave's window wraps
    const int s0 = lo_w < 0 ? cp[a.g1 + lo_w] : 0, e0 = lo_w < 0 ? cp[a.g1] : 0;
    const int l0 = (live && lo < 0) ? cp[a.g1 + lo] : e0;
    // part 1: columns [max(lo_w, 0), hi_w)
    const int s1 = cp[max(lo_w, 0)], e1 = cp[hi_w];
    const int l1 = live ? cp[max(lo, 0)] : e1, m1 = live ? cp[c + 1] : e1;
    S[2 * t] = __builtin_amdgcn_readfirstlane(s0);
    cum[2 * t + 1] = cum[2 * t] + __builtin_amdgcn_readfirstlane(e0 - s0);
    lr[2 * t] = (unsigned)(l0 - s0) | ((unsigned)(e0 - s0) << 16);
    S[2 * t + 1] = __builtin_amdgcn_readfirstlane(s1);
    cum[2 * t + 2] = cum[2 * t + 1] + __builtin_amdgcn_readfirstlane(e1 - s1);
    lr[2 * t + 1] = (unsigned)(l1 - s1) | ((unsigned)(m1 - s1) << 16);
  }
  const int total = cum[NS];
  // one record into registers: the sequence position v (clamped) of this lane's chunk slot.
  // The R row taps and W column taps it uses are packed into whole vectors, so the record
  // stays in registers.
  constexpr int NP = (R + W + 3) / 4;
  struct Rec {
    int col;
    float4 w[NP];  // row taps [0, R), column taps [R, R + W)
    float4 y[YV];
  };
  const auto fetch = [&](int v) __attribute__((always_inline)) {
    Rec r;
    v = min(v, total - 1);
    int sidx = S[0] + v, tr = 0;
#pragma unroll
    for (int q = 1; q < NS; ++q)
      if (v >= cum[q]) {
        sidx = S[q] + (v - cum[q]);
        tr = q / 2;
      }
    r.col = a.s_col[sidx];
    const float4* wr = reinterpret_cast<const float4*>(a.s_wts) + (int64_t)sidx * (SREC / 4);
    const float4 w0l = wr[0], w0h = wr[1], w1l = wr[2], w1h = wr[3];
    const float w1[8] = {w1l.x, w1l.y, w1l.z, w1l.w, w1h.x, w1h.y, w1h.z, w1h.w};
    float t[4 * NP];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int t0 = i - R + 1 + tr;
      t[i] = (t0 >= 0 && t0 < W) ? pick8(w0l, w0h, t0) : 0.f;
    }
#pragma unroll
    for (int k = 0; k < W; ++k) t[R + k] = w1[k];
#pragma unroll
    for (int k = R + W; k < 4 * NP; ++k) t[k] = 0.f;
#pragma unroll
    for (int p = 0; p < NP; ++p) r.w[p] = make_float4(t[4 * p], t[4 * p + 1], t[4 * p + 2], t[4 * p + 3]);
    const float2* yr = ys + (int64_t)sidx * Jp + jo;
    if constexpr (JG == 1) {
      const float2 v2 = yr[0];
      r.y[0] = make_float4(v2.x, v2.y, 0.f, 0.f);
    } else {
#pragma unroll
      for (int q = 0; q < YV; ++q) r.y[q] = reinterpret_cast<const float4*>(yr)[q];
    }
    return r;
  };
  const auto put = [&](const Rec& r) __attribute__((always_inline)) {
    ck.col[lane] = r.col;
    float t[4 * NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      t[4 * p] = r.w[p].x;
      t[4 * p + 1] = r.w[p].y;
      t[4 * p + 2] = r.w[p].z;
      t[4 * p + 3] = r.w[p].w;
    }
#pragma unroll
    for (int i = 0; i < R; ++i) ck.w0[i][lane] = t[i];
#pragma unroll
    for (int k = 0; k < W; ++k) ck.w1[k][lane] = t[R + k];
    if constexpr (JG == 1) {
      ck.y[lane][0] = make_float2(r.y[0].x, r.y[0].y);
    } else {
#pragma unroll
      for (int q = 0; q < YV; ++q) reinterpret_cast<float4*>(ck.y[lane])[q] = r.y[q];
    }
  };
  float2 acc[R][JG];
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int q = 0; q < JG; ++q) acc[i][q] = make_float2(0.f, 0.f);
  if (total > 0) {
    // the loads of a chunk slot past the sequence repeat its last record (the index is
    // clamped), so the fetch is unconditional: the one after the last chunk goes unused
    Rec nx = fetch(lane);
    for (int v0 = 0; v0 < total; v0 += SPC) {
      put(nx);
      asm volatile("" ::: "memory");  // the wave's LDS accesses run in program order
      nx = fetch(v0 + SPC + lane);
      // this lane's records in the chunk, range by range
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        const int b = max(cum[q] + (int)(lr[q] & 0xffffu), v0), e = min(cum[q] + (int)(lr[q] >> 16), v0 + SPC);
        for (int k = b; k < e; ++k) {
          const int l = k - v0;
          int t1 = c - ck.col[l];
          if (t1 < 0) t1 += a.g1;
          const float w1 = ck.w1[t1][l];
#pragma unroll
          for (int i = 0; i < R; ++i) {
            const float w = ck.w0[i][l] * w1;
            if constexpr (JG == 1) {
              const float2 y = ck.y[l][0];
              acc[i][0].x += w * y.x;
              acc[i][0].y += w * y.y;
            } else {
#pragma unroll
              for (int h = 0; h < YV; ++h) {
                const float4 y = reinterpret_cast<const float4*>(ck.y[l])[h];
                acc[i][2 * h].x += w * y.x;
                acc[i][2 * h].y += w * y.y;
                acc[i][2 * h + 1].x += w * y.z;
                acc[i][2 * h + 1].y += w * y.w;
              }
            }
          }
        }
      }
      asm volatile("" ::: "memory");
    }
  }
  if (!live) return;
  float sc = alpha * a.cscale;
  if (scale_dev) sc *= *scale_dev;
  const int64_t G = (int64_t)a.g0 * a.g1;
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int q = 0; q < JG; ++q)
      if (r0 + i < a.g0 && jo + q < a.J)
        grid[(int64_t)(jo + q) * G + (int64_t)(r0 + i) * a.g1 + c] = cscale(acc[i][q], sc);
}

template <int JG, int W>
void launch_flat(const NufftArgs& a, const float2* ys, int Jp, float alpha, const float* scale_dev, float2* grid,
                 hipStream_t st) {
  constexpr int R = SPREAD_ROWS;
  const int64_t waves = (int64_t)((a.g0 + R - 1) / R) * ((a.g1 + SPC - 1) / SPC) * (Jp / JG);
  const int64_t plain = (waves + 3) / 4;
  const int64_t split =
      a.n_heavy > 0 ? (int64_t)(a.split_pm * a.n_med + a.split_ph * (a.n_heavy - a.n_med)) * (Jp / JG) : 0;
  bool lds = false;
  if constexpr (JG <= 8) lds = a.spread_lds != 0;  // the LDS form takes at most 8 coils per lane
  if (lds) {  // one launch: the plain blocks' workgroups, then the split rows'
    if constexpr (JG <= 8)
      hipLaunchKernelGGL((spread_lds_kernel<JG, W, R>), dim3((unsigned)(plain + split)), dim3(256), 0, st, a, ys, Jp,
                         alpha, scale_dev, grid);
  } else {
    hipLaunchKernelGGL((spread_flat_kernel<JG, W, R, 2>), dim3((unsigned)plain), dim3(256), 0, st, a, ys, Jp, alpha,
                       scale_dev, grid);
    if (split > 0)
      hipLaunchKernelGGL((spread_split_kernel<JG, W>), dim3((unsigned)split), dim3(256), 0, st, a, ys, Jp, alpha,
                         scale_dev, grid);
  }
}

template <int JG>
void launch_flat_w(const NufftArgs& a, const float2* ys, int Jp, float alpha, const float* scale_dev, float2* grid,
                   hipStream_t st) {
  switch (a.W) {
    case 1: launch_flat<JG, 1>(a, ys, Jp, alpha, scale_dev, grid, st); break;
    case 2: launch_flat<JG, 2>(a, ys, Jp, alpha, scale_dev, grid, st); break;
    case 3: launch_flat<JG, 3>(a, ys, Jp, alpha, scale_dev, grid, st); break;
    case 4: launch_flat<JG, 4>(a, ys, Jp, alpha, scale_dev, grid, st); break;
    case 5: launch_flat<JG, 5>(a, ys, Jp, alpha, scale_dev, grid, st); break;
    case 6: launch_flat<JG, 6>(a, ys, Jp, alpha, scale_dev, grid, st); break;
    case 7: launch_flat<JG, 7>(a, ys, Jp, alpha, scale_dev, grid, st); break;
    default: launch_flat<JG, 8>(a, ys, Jp, alpha, scale_dev, grid, st); break;
  }
}

inline unsigned grid_for(int64_t total) {
  int64_t b = (total + NT - 1) / NT;
  if (b > 16384) b = 16384;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

int spread_group(int J) { return J >= 8 ? 8 : J > 2 ? 4 : J; }

size_t spread_stage_bytes(int J, int64_t M) {
  const int jg = spread_group(J);
  return (size_t)M * (size_t)((J + jg - 1) / jg * jg) * sizeof(float2);
}

hipError_t degrid_launch(const NufftArgs& a, const float2* grid, float2* y, hipStream_t st) {
  if (a.M * a.J == 0) return hipSuccess;
  const dim3 gr(grid_for(a.M * a.J));
  switch (a.W) {
    case 2: hipLaunchKernelGGL(degrid_kernel<2>, gr, dim3(NT), 0, st, a, grid, y); break;
    case 3: hipLaunchKernelGGL(degrid_kernel<3>, gr, dim3(NT), 0, st, a, grid, y); break;
    case 4: hipLaunchKernelGGL(degrid_kernel<4>, gr, dim3(NT), 0, st, a, grid, y); break;
    case 5: hipLaunchKernelGGL(degrid_kernel<5>, gr, dim3(NT), 0, st, a, grid, y); break;
    case 6: hipLaunchKernelGGL(degrid_kernel<6>, gr, dim3(NT), 0, st, a, grid, y); break;
    case 7: hipLaunchKernelGGL(degrid_kernel<7>, gr, dim3(NT), 0, st, a, grid, y); break;
    case 8: hipLaunchKernelGGL(degrid_kernel<8>, gr, dim3(NT), 0, st, a, grid, y); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t spread_launch(const NufftArgs& a, const float2* y, float alpha, const float* scale_dev, float2* ys,
                         float2* grid, hipStream_t st, bool staged) {
  const int jg = spread_group(a.J);
  const int Jp = (a.J + jg - 1) / jg * jg;
  if (a.W < 1 || a.W > 8) return hipErrorInvalidValue;
  if (staged) {
    if (Jp != a.J) return hipErrorInvalidValue;
    ys = const_cast<float2*>(y);  // read only
  } else if (a.M > 0)
    hipLaunchKernelGGL(spread_stage_kernel, dim3((unsigned)((a.M + NT - 1) / NT)), dim3(NT), 0, st, a, y, Jp, ys);
  // the plain kernel from memory takes 16 coils per lane where the padded coil count allows
  // (one walk of a sample sequence serves twice the coils; 150 vs 156 us at 32 coils, 128
  // spokes); through LDS, at most 8 (twice the waves in flight: 31 vs 43 us at 16 coils,
  // 64 spokes; 4 coils take 39 us)
  switch (a.spread_lds ? jg : Jp % 16 == 0 ? 16 : jg) {
    case 1: launch_flat_w<1>(a, ys, Jp, alpha, scale_dev, grid, st); break;
    case 2: launch_flat_w<2>(a, ys, Jp, alpha, scale_dev, grid, st); break;
    case 4: launch_flat_w<4>(a, ys, Jp, alpha, scale_dev, grid, st); break;
    case 8: launch_flat_w<8>(a, ys, Jp, alpha, scale_dev, grid, st); break;
    default: launch_flat_w<16>(a, ys, Jp, alpha, scale_dev, grid, st); break;
  }
  return hipGetLastError();
}

}  // namespace mx
