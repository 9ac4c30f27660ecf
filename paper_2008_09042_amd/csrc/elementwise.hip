// Sampling, residual, loss and coil-combination kernels.
//
//  gather   y_j = P k_j           Cartesian mask gather (paper Sec. II-A, F_s = P F)
//  scatter  k_j = P^T y_j         zero-filled adjoint of the gather (one pass, no memset)
//  residual r = w (.) (E - y) and FP64 partial sums of w |E - y|^2 (Sec. II-B, Eq. (6) data term)
//  combine  gx = s sum_j conj(s_j) (.) g_j and h_j = s conj(x) (.) g_j  (Sec. II-B, J_G^H)
#include "common.h"

namespace mx {

namespace {

constexpr int NT = 256;

inline unsigned grid_for(int64_t total, int64_t cap = 16384) {
  int64_t b = (total + NT - 1) / NT;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (unsigned)b;
}

__global__ void gather_kernel(const float2* __restrict__ ks, int64_t N, const int32_t* __restrict__ idx,
                              int64_t M, int J, float2* __restrict__ y) {
  const int64_t total = M * J;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t j = e / M, m = e % M;
    y[e] = ks[j * N + idx[m]];
  }
}

__global__ void scatter_kernel(const float2* __restrict__ y, int64_t M, const int32_t* __restrict__ inv,
                               int64_t N, int J, float2* __restrict__ ks) {
  const int64_t total = N * J;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t j = e / N, n = e % N;
    const int32_t m = inv[n];
    ks[e] = m >= 0 ? y[j * M + m] : make_float2(0.f, 0.f);
  }
}

__global__ void residual_kernel(const float2* __restrict__ E, const float2* __restrict__ y,
                                const float* __restrict__ w, int64_t M, int J, float2* __restrict__ r,
                                double* __restrict__ part) {
  __shared__ double red[NT];
  const int64_t total = M * J;
  double acc = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t m = e % M;
    const float2 d = csub(E[e], y[e]);
    const float wm = w ? w[m] : 1.0f;
    acc += (double)wm * ((double)d.x * d.x + (double)d.y * d.y);
    if (r) r[e] = cscale(d, wm);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void reduce_loss_kernel(const double* __restrict__ part, int nblocks, double* loss) {
  __shared__ double red[NT];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += NT) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0];
}

// GX: gx wanted (S read), H: h written in place of g.  Eight coils' loads are issued
// together (clamped coil index; the coils past J are neither added nor written), and the
// sum over j keeps its order, so gx is the same bits as one coil at a time.
template <bool GX, bool H>
__global__ void adjoint_combine_kernel(const float2* __restrict__ S, float2* __restrict__ g,
                                       const float2* __restrict__ x, int64_t N, int J, float alpha,
                                       const float* __restrict__ scale_dev, float2* __restrict__ gx) {
  float s = alpha;
  if (scale_dev) s *= *scale_dev;
  for (int64_t n = blockIdx.x * (int64_t)NT + threadIdx.x; n < N; n += (int64_t)gridDim.x * NT) {
    const float2 xn = H ? x[n] : make_float2(0.f, 0.f);
    float2 acc = make_float2(0.f, 0.f);
    for (int j0 = 0; j0 < J; j0 += 8) {
      float2 gv[8], sv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t j = min(j0 + u, J - 1);
        gv[u] = g[j * N + n];
        if (GX) sv[u] = S[j * N + n];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (j0 + u >= J) continue;
        if (GX) acc = cadd(acc, cmulc(sv[u], gv[u]));
        if (H) g[(int64_t)(j0 + u) * N + n] = cscale(cmulc(xn, gv[u]), s);
      }
    }
    if (GX) gx[n] = cscale(acc, s);
  }
}

__global__ void scale_copy_kernel(const float2* __restrict__ src, float2* __restrict__ dst, int64_t count,
                                  float alpha, const float* __restrict__ scale_dev) {
  float s = alpha;
  if (scale_dev) s *= *scale_dev;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < count; e += (int64_t)gridDim.x * NT)
    dst[e] = cscale(src[e], s);
}

// The residual of residual_kernel written in a sample order: r[inv[m] J + j].  The work is
// dealt in chunks of NT samples of one group of eight coils (blocks take chunks in grid-stride
// order, so every block has work however many coils there are): a thread reads its sample's
// eight coils down the columns of E and y (coalesced over m across a wave), all sixteen loads
// in flight together, and writes them as one contiguous run at the sample's position, 16
// bytes at a time when J is even.  The loss partials are per-thread sums in (chunk, coil)
// order, added per block as in residual_kernel.
__global__ void residual_ordered_kernel(const float2* __restrict__ E, const float2* __restrict__ y,
                                        const float* __restrict__ w, int64_t M, int J,
                                        const int32_t* __restrict__ inv, float2* __restrict__ r,
                                        double* __restrict__ part) {
  __shared__ double red[NT];
  double acc = 0.0;
  const int64_t cpg = (M + NT - 1) / NT;  // chunks per coil group
  const int64_t nchunks = cpg * ((J + 7) / 8);
  for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const int64_t g = c / cpg, m = (c - g * cpg) * NT + threadIdx.x;
    if (m >= M) continue;  // no barrier inside the loop
    const int j0 = 8 * (int)g;
    const float wm = w ? w[m] : 1.0f;
    float2* dst = r + (int64_t)inv[m] * J;
    float2 e[8], v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = min(j0 + u, J - 1);
      e[u] = E[(int64_t)j * M + m];
      v[u] = y[(int64_t)j * M + m];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float2 d = csub(e[u], v[u]);
      if (j0 + u < J) acc += (double)wm * ((double)d.x * d.x + (double)d.y * d.y);
      e[u] = cscale(d, wm);
    }
    if ((J & 1) == 0) {
#pragma unroll
      for (int u = 0; u < 8; u += 2)
        if (j0 + u < J) reinterpret_cast<float4*>(dst + j0)[u / 2] = make_float4(e[u].x, e[u].y, e[u + 1].x, e[u + 1].y);
    } else {
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (j0 + u < J) dst[j0 + u] = e[u];
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

}  // namespace

hipError_t gather_launch(const float2* kspace, int64_t N, const int32_t* idx, int64_t M, int J,
                         float2* y, hipStream_t st) {
  if (M * J == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel, dim3(grid_for(M * J)), dim3(NT), 0, st, kspace, N, idx, M, J, y);
  return hipGetLastError();
}

hipError_t scatter_launch(const float2* y, int64_t M, const int32_t* inv_mask, int64_t N, int J,
                          float2* kspace, hipStream_t st) {
  hipLaunchKernelGGL(scatter_kernel, dim3(grid_for(N * J)), dim3(NT), 0, st, y, M, inv_mask, N, J, kspace);
  return hipGetLastError();
}

int residual_blocks(int64_t total) { return (int)grid_for(total, 2048); }

hipError_t residual_launch(const float2* E, const float2* y, const float* w, int64_t M, int J,
                           float2* r, double* part, hipStream_t st) {
  hipLaunchKernelGGL(residual_kernel, dim3(residual_blocks(M * J)), dim3(NT), 0, st, E, y, w, M, J, r, part);
  return hipGetLastError();
}

hipError_t residual_ordered_launch(const float2* E, const float2* y, const float* w, int64_t M, int J,
                                   const int32_t* inv, float2* r, double* part, hipStream_t st) {
  hipLaunchKernelGGL(residual_ordered_kernel, dim3(residual_blocks(M * J)), dim3(NT), 0, st, E, y, w, M, J, inv, r,
                     part);
  return hipGetLastError();
}

hipError_t reduce_loss_launch(const double* part, int nblocks, double* loss, hipStream_t st) {
  hipLaunchKernelGGL(reduce_loss_kernel, dim3(1), dim3(NT), 0, st, part, nblocks, loss);
  return hipGetLastError();
}

hipError_t adjoint_combine_launch(const float2* S, float2* g, const float2* x, int64_t N, int J,
                                  float alpha, const float* scale_dev, float2* gx, int want_h,
                                  hipStream_t st) {
  if (N <= 0 || J <= 0) return hipSuccess;
  const dim3 gr(grid_for(N)), bl(NT);
  if (gx && want_h)
    hipLaunchKernelGGL((adjoint_combine_kernel<true, true>), gr, bl, 0, st, S, g, x, N, J, alpha, scale_dev, gx);
  else if (gx)
    hipLaunchKernelGGL((adjoint_combine_kernel<true, false>), gr, bl, 0, st, S, g, x, N, J, alpha, scale_dev, gx);
  else if (want_h)
    hipLaunchKernelGGL((adjoint_combine_kernel<false, true>), gr, bl, 0, st, S, g, x, N, J, alpha, scale_dev, gx);
  return hipGetLastError();
}

hipError_t scale_copy_launch(const float2* src, float2* dst, int64_t count, float alpha,
                             const float* scale_dev, hipStream_t st) {
  hipLaunchKernelGGL(scale_copy_kernel, dim3(grid_for(count)), dim3(NT), 0, st, src, dst, count, alpha,
                     scale_dev);
  return hipGetLastError();
}

// One device timestamp (the constant-rate wall clock) written by one lane.
__global__ void stamp_kernel(uint64_t* __restrict__ dst) {
  if (threadIdx.x == 0) *dst = wall_clock64();
}

hipError_t stamp_launch(uint64_t* dst, hipStream_t st) {
  hipLaunchKernelGGL(stamp_kernel, dim3(1), dim3(64), 0, st, dst);
  return hipGetLastError();
}

}  // namespace mx
