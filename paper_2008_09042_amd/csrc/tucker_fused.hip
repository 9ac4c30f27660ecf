// Fused path for a 3D Tucker basis with Cartesian sampling of full lines along
// the last axis (readout).  Paper: the bilinear operator of Sec. II-B, Eq. (5)
// with the Tucker-factored basis of Sec. II-E.
//
// Geometry: image (n0, n1, n2), ranks (r0, r1, r2), sampled lines L = {(k0, k1)}
// each with every k2, so y_j is [L][n2].  Because the mask is a product of a
// plane pattern and the full readout axis, the 3D centred DFT followed by the
// gather factors into (a) a 2D DFT of every (i0, i1) plane followed by a gather
// of the L sampled points, then (b) a 1D DFT along i2 of each sampled line.
// The coil map of plane i2 is
//     s_j[:, :, i2] = U0 W U1^T,   W = T3[j][i2] = (core x_4 c_j x_3 U2)[:, :, i2]
// (mode products of Sec. II-E), so no [J][N] array is ever written to memory:
//
//   forward   T1 = core x_4 c,  T3 = T1 x_3 U2                 (MFMA GEMM kernel)
//             plane kernel per (i2, coil): V = W U1^T, P = U0 V (MFMA, P kept in
//             registers), m = x (.) P, 2D DFT in LDS, gather L points -> Z[j][i2][L]
//             line kernel per (coil, 32 lines): DFT along i2, residual / loss -> y or r
//   adjoint   line kernel: inverse DFT along k2 (scaled) -> Zb[j][i2][L]
//             plane kernel per (i2, group of coils): recompute P, scatter Zb, inverse
//             2D DFT -> g;  gx partial += conj(P) (.) g;  h = conj(x) (.) g;
//             Wb = U0^H h conj(U1) -> T3b[j][i2]
//             T1b = T3b x_3 U2^H,  gc = core^H T1b              (MFMA GEMM kernel)
//             gx = sum of the per-group partials (fixed order, no atomics)
//
// Complex products on MFMA use v_mfma_f32_16x16x4_f32 (FP32) as four real
// products, or BF16 hi/lo splits on v_mfma_f32_16x16x32_bf16 (BF16_SPLIT).
#include "fft_device.h"
#include "fused.h"

namespace mx {

typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int PT = 512;                          // threads per plane workgroup
constexpr int NWAVE = PT / 64;
constexpr int PMAX = 128;                        // max n0, n1 on this path
constexpr int PSMAX = PMAX + 1;                  // padded plane row stride
constexpr int PLANE_ELEMS = PMAX * PSMAX;        // 16,512 complex = 132 KB of LDS
constexpr int W_OFF = 0;                         // W  [r0p][r1p]  (<= 64 x 64)
constexpr int V_OFF = 64 * 64;                   // V  [r0p][n1]   (<= 64 x 128)

__device__ inline void cmfma(f32x4& cr, f32x4& ci, float2 a, float2 b) {
  cr = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, cr, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, b.y, cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.y, ci, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.x, ci, 0, 0, 0);
}

__device__ inline f32x4 z4() { return f32x4{0.f, 0.f, 0.f, 0.f}; }

// W (r0 x r1 of T3[j][i2]) into LDS, zero-padded to r0p x r1p.
__device__ inline void load_W(const PlaneArgs& a, int j, int i2, float2* lds) {
  const float2* src = a.T3 + ((size_t)j * a.n2 + i2) * a.r0 * a.r1;
  for (int e = threadIdx.x; e < a.r0p * a.r1p; e += PT) {
    const int p0 = e / a.r1p, p1 = e % a.r1p;
    lds[W_OFF + e] = (p0 < a.r0 && p1 < a.r1) ? src[p0 * a.r1 + p1] : make_float2(0.f, 0.f);
  }
}

// V = W U1^T  ([r0p][n1], row stride n1) in LDS.
__device__ inline void compute_V(const PlaneArgs& a, float2* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int mbl = a.r0p / 16, nbl = a.n1 / 16;
  for (int blk = wave; blk < mbl * nbl; blk += NWAVE) {
    const int mb = blk / nbl, nb = blk % nbl;
    f32x4 cr = z4(), ci = z4();
    const int row = 16 * mb + (lane & 15), col = 16 * nb + (lane & 15);
    for (int k = 0; k < a.r1p; k += 4) {
      const int kk = k + (lane >> 4);
      const float2 av = lds[W_OFF + row * a.r1p + kk];
      const float2 bv = kk < a.r1 ? a.U1[(size_t)col * a.r1 + kk] : make_float2(0.f, 0.f);
      cmfma(cr, ci, av, bv);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
      lds[V_OFF + (16 * mb + 4 * (lane >> 4) + r) * a.n1 + col] = make_float2(cr[r], ci[r]);
  }
}

// P = U0 V for this wave's 16-row block (all n1 columns) into registers.
__device__ inline void compute_P(const PlaneArgs& a, const float2* lds, f32x4 (&pr)[8], f32x4 (&pi)[8]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nbl = a.n1 / 16;
#pragma unroll
  for (int nb = 0; nb < 8; ++nb) { pr[nb] = z4(); pi[nb] = z4(); }
  if (wave >= a.n0 / 16) return;
  const int row = 16 * wave + (lane & 15);
  for (int k = 0; k < a.r0p; k += 4) {
    const int kk = k + (lane >> 4);
    const float2 av = kk < a.r0 ? a.U0[(size_t)row * a.r0 + kk] : make_float2(0.f, 0.f);
#pragma unroll
    for (int nb = 0; nb < 8; ++nb) {
      if (nb < nbl) {
        const float2 bv = lds[V_OFF + kk * a.n1 + 16 * nb + (lane & 15)];
        cmfma(pr[nb], pi[nb], av, bv);
      }
    }
  }
}

__device__ inline void plane_fft(const PlaneArgs& a, float2* lds, int dir) {
  const int PS = a.n1 + 1;
  LdsLines rows{a.n0, PS, 1};
  LdsLines cols{a.n1, 1, PS};
  if (dir < 0) {
    lds_fft_lines<PT, PMAX * PMAX / 2>(lds, rows, a.n1, a.rad1, a.nrad1, a.tw1, dir);
    lds_fft_lines<PT, PMAX * PMAX / 2>(lds, cols, a.n0, a.rad0, a.nrad0, a.tw0, dir);
  } else {
    lds_fft_lines<PT, PMAX * PMAX / 2>(lds, cols, a.n0, a.rad0, a.nrad0, a.tw0, dir);
    lds_fft_lines<PT, PMAX * PMAX / 2>(lds, rows, a.n1, a.rad1, a.nrad1, a.tw1, dir);
  }
}

__global__ __launch_bounds__(PT) void plane_fwd_kernel(PlaneArgs a) {
  __shared__ float2 lds[PLANE_ELEMS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ngrp = (a.J + a.G - 1) / a.G;
  const int i2 = blockIdx.x / ngrp, grp = blockIdx.x % ngrp;
  const int PS = a.n1 + 1;
  const int nbl = a.n1 / 16;
  const float2* xp = a.xt + (size_t)i2 * a.n0 * a.n1;
  for (int j = grp * a.G; j < a.J && j < (grp + 1) * a.G; ++j) {
    load_W(a, j, i2, lds);
    __syncthreads();
    compute_V(a, lds);
    __syncthreads();
    f32x4 pr[8], pi[8];
    compute_P(a, lds, pr, pi);
    __syncthreads();
    // m = x (.) P with the input chessboard sign, into the padded plane
    if (wave < a.n0 / 16) {
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) {
        if (nb < nbl) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i0 = 16 * wave + 4 * (lane >> 4) + r, i1 = 16 * nb + (lane & 15);
            float2 v = cmul(make_float2(pr[nb][r], pi[nb][r]), xp[i0 * a.n1 + i1]);
            if ((i0 + i1) & 1) v = make_float2(-v.x, -v.y);
            lds[i0 * PS + i1] = v;
          }
        }
      }
    }
    __syncthreads();
    plane_fft(a, lds, -1);
    float2* zo = a.Z + ((size_t)j * a.n2 + i2) * a.L;
    for (int l = threadIdx.x; l < a.L; l += PT) {
      const int q = a.pos[l];
      const int k0 = q / a.n1, k1 = q - k0 * a.n1;
      float2 v = lds[k0 * PS + k1];
      if ((k0 + k1) & 1) v = make_float2(-v.x, -v.y);
      zo[l] = v;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(PT) void plane_adj_kernel(PlaneArgs a) {
  __shared__ float2 lds[PLANE_ELEMS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ngrp = (a.J + a.G - 1) / a.G;
  const int i2 = blockIdx.x / ngrp, grp = blockIdx.x % ngrp;
  const int PS = a.n1 + 1;
  const int nbl = a.n1 / 16;
  const float2* xp = a.xt + (size_t)i2 * a.n0 * a.n1;
  float2* gxp = a.gxpart ? a.gxpart + ((size_t)grp * a.n2 + i2) * a.n0 * a.n1 : nullptr;
  const int jbeg = grp * a.G;
  for (int j = jbeg; j < a.J && j < (grp + 1) * a.G; ++j) {
    f32x4 pr[8], pi[8];
    if (gxp) {
      // recompute the coil map plane P = U0 W U1^T (B c recomputed)
      load_W(a, j, i2, lds);
      __syncthreads();
      compute_V(a, lds);
      __syncthreads();
      compute_P(a, lds, pr, pi);
      __syncthreads();
    }
    // zero-filled scatter of this plane's samples (with the chessboard sign)
    for (int e = threadIdx.x; e < a.n0 * PS; e += PT) lds[e] = make_float2(0.f, 0.f);
    __syncthreads();
    const float2* zi = a.Z + ((size_t)j * a.n2 + i2) * a.L;
    for (int l = threadIdx.x; l < a.L; l += PT) {
      const int q = a.pos[l];
      const int k0 = q / a.n1, k1 = q - k0 * a.n1;
      float2 v = zi[l];
      if ((k0 + k1) & 1) v = make_float2(-v.x, -v.y);
      lds[k0 * PS + k1] = v;
    }
    __syncthreads();
    plane_fft(a, lds, +1);
    // g (output chessboard sign), gx partial, h = conj(x) (.) g back into the plane
    if (wave < a.n0 / 16) {
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) {
        if (nb < nbl) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i0 = 16 * wave + 4 * (lane >> 4) + r, i1 = 16 * nb + (lane & 15);
            float2 g = lds[i0 * PS + i1];
            if ((i0 + i1) & 1) g = make_float2(-g.x, -g.y);
            if (gxp) {
              const float2 c = cmulc(make_float2(pr[nb][r], pi[nb][r]), g);
              float2* o = gxp + i0 * a.n1 + i1;
              *o = (j == jbeg) ? c : cadd(*o, c);
            }
            lds[i0 * PS + i1] = cmulc(xp[i0 * a.n1 + i1], g);
          }
        }
      }
    }
    __syncthreads();
    if (a.T3b) {
      // Y = h conj(U1)  ([n0][r1p]) -- this wave's 16-row block, into registers
      f32x4 yr[4], yi[4];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) { yr[nb] = z4(); yi[nb] = z4(); }
      const int nbr = a.r1p / 16;
      if (wave < a.n0 / 16) {
        const int row = 16 * wave + (lane & 15);
        for (int k = 0; k < a.n1; k += 4) {
          const int kk = k + (lane >> 4);
          const float2 av = lds[row * PS + kk];
#pragma unroll
          for (int nb = 0; nb < 4; ++nb) {
            if (nb < nbr) {
              const int col = 16 * nb + (lane & 15);
              const float2 bv = col < a.r1 ? cconj(a.U1[(size_t)kk * a.r1 + col]) : make_float2(0.f, 0.f);
              cmfma(yr[nb], yi[nb], av, bv);
            }
          }
        }
      }
      __syncthreads();
      if (wave < a.n0 / 16) {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          if (nb < nbr) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              lds[(16 * wave + 4 * (lane >> 4) + r) * a.r1p + 16 * nb + (lane & 15)] =
                  make_float2(yr[nb][r], yi[nb][r]);
          }
        }
      }
      __syncthreads();
      // Wb = U0^H Y  ([r0][r1]) -> T3b[j][i2]
      const int mbl = a.r0p / 16;
      float2* wo = a.T3b + ((size_t)j * a.n2 + i2) * a.r0 * a.r1;
      for (int blk = wave; blk < mbl * nbr; blk += NWAVE) {
        const int mb = blk / nbr, nb = blk % nbr;
        f32x4 cr = z4(), ci = z4();
        const int p0 = 16 * mb + (lane & 15);
        for (int k = 0; k < a.n0; k += 4) {
          const int kk = k + (lane >> 4);
          const float2 av = p0 < a.r0 ? cconj(a.U0[(size_t)kk * a.r0 + p0]) : make_float2(0.f, 0.f);
          const float2 bv = lds[kk * a.r1p + 16 * nb + (lane & 15)];
          cmfma(cr, ci, av, bv);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q0 = 16 * mb + 4 * (lane >> 4) + r, q1 = 16 * nb + (lane & 15);
          if (q0 < a.r0 && q1 < a.r1) wo[q0 * a.r1 + q1] = make_float2(cr[r], ci[r]);
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- line kernels
constexpr int LT = 32;     // lines per workgroup
constexpr int LNT = 256;   // threads
constexpr int LMAXN = 256; // max n2 on this path

__global__ __launch_bounds__(LNT) void line_fwd_kernel(LineArgs a) {
  __shared__ float2 tile[LMAXN * (LT + 1)];
  __shared__ double red[LNT];
  const int lblocks = (a.L + LT - 1) / LT;
  const int j = blockIdx.x / lblocks, l0 = (blockIdx.x % lblocks) * LT;
  const int n = a.n2, ES = LT + 1;
  for (int e = threadIdx.x; e < n * LT; e += LNT) {
    const int i2 = e / LT, l = e % LT;
    float2 v = make_float2(0.f, 0.f);
    if (l0 + l < a.L) v = a.Z[((size_t)j * n + i2) * a.L + l0 + l];
    if (i2 & 1) v = make_float2(-v.x, -v.y);
    tile[i2 * ES + l] = v;
  }
  __syncthreads();
  LdsLines tg{LT, 1, ES};
  lds_fft_lines<LNT, LMAXN * LT / 2>(tile, tg, n, a.rad2, a.nrad2, a.tw2, -1);
  double acc = 0.0;
  for (int e = threadIdx.x; e < n * LT; e += LNT) {
    const int l = e / n, k2 = e % n;
    if (l0 + l >= a.L) continue;
    float2 v = tile[k2 * ES + l];
    const float s = (k2 & 1) ? -a.gscale : a.gscale;
    v = cscale(v, s);
    const size_t m = (size_t)(l0 + l) * n + k2;
    const size_t o = (size_t)j * a.M + m;
    if (a.y) {
      const float2 d = csub(v, a.y[o]);
      const float wm = a.w ? a.w[m] : 1.0f;
      acc += (double)wm * ((double)d.x * d.x + (double)d.y * d.y);
      if (a.out) a.out[o] = cscale(d, wm);
    } else {
      a.out[o] = v;
    }
  }
  if (a.part) {
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = LNT / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) a.part[blockIdx.x] = red[0];
  }
}

__global__ __launch_bounds__(LNT) void line_adj_kernel(LineArgs a) {
  __shared__ float2 tile[LMAXN * (LT + 1)];
  const int lblocks = (a.L + LT - 1) / LT;
  const int j = blockIdx.x / lblocks, l0 = (blockIdx.x % lblocks) * LT;
  const int n = a.n2, ES = LT + 1;
  for (int e = threadIdx.x; e < n * LT; e += LNT) {
    const int l = e / n, k2 = e % n;
    float2 v = make_float2(0.f, 0.f);
    if (l0 + l < a.L) v = a.yin[(size_t)j * a.M + (size_t)(l0 + l) * n + k2];
    if (k2 & 1) v = make_float2(-v.x, -v.y);
    tile[k2 * ES + l] = v;
  }
  __syncthreads();
  LdsLines tg{LT, 1, ES};
  lds_fft_lines<LNT, LMAXN * LT / 2>(tile, tg, n, a.rad2, a.nrad2, a.tw2, +1);
  float s = a.gscale * a.alpha;
  if (a.scale_dev) s *= *a.scale_dev;
  for (int e = threadIdx.x; e < n * LT; e += LNT) {
    const int i2 = e / LT, l = e % LT;
    if (l0 + l >= a.L) continue;
    const float2 v = tile[i2 * ES + l];
    a.Zw[((size_t)j * n + i2) * a.L + l0 + l] = cscale(v, (i2 & 1) ? -s : s);
  }
}

// ---------------------------------------------------------------- transposes
constexpr int TT = 32;

// xt[c][r] = x[r][c] for an R x C matrix (complex)
__global__ void transpose_kernel(const float2* __restrict__ x, int64_t R, int64_t C, float2* __restrict__ xt) {
  __shared__ float2 t[TT][TT + 1];
  const int64_t tr = (int64_t)blockIdx.y * TT, tc = (int64_t)blockIdx.x * TT;
  const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
  for (int k = ty; k < TT; k += 256 / TT) {
    const int64_t r = tr + k, c = tc + tx;
    if (r < R && c < C) t[k][tx] = x[r * C + c];
  }
  __syncthreads();
  for (int k = ty; k < TT; k += 256 / TT) {
    const int64_t c = tc + k, r = tr + tx;
    if (r < R && c < C) xt[c * R + r] = t[tx][k];
  }
}

// gx[r][c] = sum_g part[g][c][r] : part is ngrp x (C x R), gx is R x C
__global__ void reduce_transpose_kernel(const float2* __restrict__ part, int ngrp, int64_t R, int64_t C,
                                        float2* __restrict__ gx) {
  __shared__ float2 t[TT][TT + 1];
  const int64_t tr = (int64_t)blockIdx.x * TT, tc = (int64_t)blockIdx.y * TT;
  const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
  for (int k = ty; k < TT; k += 256 / TT) {
    const int64_t c = tc + k, r = tr + tx;
    float2 s = make_float2(0.f, 0.f);
    if (r < R && c < C)
      for (int g = 0; g < ngrp; ++g) s = cadd(s, part[((size_t)g * C + c) * R + r]);
    t[k][tx] = s;
  }
  __syncthreads();
  for (int k = ty; k < TT; k += 256 / TT) {
    const int64_t r = tr + k, c = tc + tx;
    if (r < R && c < C) gx[r * C + c] = t[tx][k];
  }
}

}  // namespace

hipError_t plane_fwd_launch(const PlaneArgs& a, hipStream_t st) {
  const int ngrp = (a.J + a.G - 1) / a.G;
  hipLaunchKernelGGL(plane_fwd_kernel, dim3((unsigned)(a.n2 * ngrp)), dim3(PT), 0, st, a);
  return hipGetLastError();
}

hipError_t plane_adj_launch(const PlaneArgs& a, hipStream_t st) {
  const int ngrp = (a.J + a.G - 1) / a.G;
  hipLaunchKernelGGL(plane_adj_kernel, dim3((unsigned)(a.n2 * ngrp)), dim3(PT), 0, st, a);
  return hipGetLastError();
}

int line_blocks(int J, int64_t L) { return (int)(J * ((L + LT - 1) / LT)); }

hipError_t line_fwd_launch(const LineArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(line_fwd_kernel, dim3((unsigned)line_blocks(a.J, a.L)), dim3(LNT), 0, st, a);
  return hipGetLastError();
}

hipError_t line_adj_launch(const LineArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(line_adj_kernel, dim3((unsigned)line_blocks(a.J, a.L)), dim3(LNT), 0, st, a);
  return hipGetLastError();
}

hipError_t transpose_launch(const float2* x, int64_t R, int64_t C, float2* xt, hipStream_t st) {
  dim3 grid((unsigned)((C + TT - 1) / TT), (unsigned)((R + TT - 1) / TT));
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, st, x, R, C, xt);
  return hipGetLastError();
}

hipError_t reduce_transpose_launch(const float2* part, int ngrp, int64_t R, int64_t C, float2* gx,
                                   hipStream_t st) {
  dim3 grid((unsigned)((R + TT - 1) / TT), (unsigned)((C + TT - 1) / TT));
  hipLaunchKernelGGL(reduce_transpose_kernel, grid, dim3(256), 0, st, part, ngrp, R, C, gx);
  return hipGetLastError();
}

bool fused_supported(int64_t n0, int64_t n1, int64_t n2, int64_t r0, int64_t r1) {
  return n0 % 16 == 0 && n1 % 16 == 0 && n0 <= PMAX && n1 <= PMAX && n2 <= LMAXN && r0 <= 64 && r1 <= 64;
}

}  // namespace mx
