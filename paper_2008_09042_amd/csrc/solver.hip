// Vector kernels of the Gauss-Newton step (paper Sec. II-B, Eq. (6)): the normal operator
// J^H W J + diag(lambda) is applied with the operator kernels; conjugate gradients around it
// need complex axpy, a row weighting, and inner products.
//
// A CG vector v = (v_x, v_c) is an image block of N complex values and a coefficient block
// of J K values.  The work vectors live contiguously in the workspace ([N | J K]); the
// caller's solution blocks are two pointers.  Every kernel takes the two blocks as one
// virtual vector of N + J K entries.
//
// Inner products Re <a, b> = Re sum conj(a) b are accumulated in FP64: every thread sums its
// grid-stride entries in order, the workgroup reduces its 256 sums by a fixed tree, and one
// more workgroup reduces the DOT_BLOCKS partials by the same tree.  No atomics: the result
// does not depend on timing.  The CG scalars (rho = <r, r>, <d, q>, the step and the
// direction factor) stay in device memory in FP64 and are read by the update kernels, so a
// CG solve runs with no host synchronisation and can be captured into a graph.
#include "solver.h"

namespace mx {

namespace {

constexpr int NT = 256;

inline unsigned grid_for(int64_t total, int64_t cap = 16384) {
  int64_t b = (total + NT - 1) / NT;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (unsigned)b;
}

struct Split {
  float2* p0;  // entries [0, n0)
  float2* p1;  // entries [n0, n0 + n1)
  int64_t n0, n1;
  __device__ float2& at(int64_t e) const { return e < n0 ? p0[e] : p1[e - n0]; }
};

struct CSplit {
  const float2* p0;
  const float2* p1;
  int64_t n0, n1;
  __device__ float2 at(int64_t e) const { return e < n0 ? p0[e] : p1[e - n0]; }
};

__global__ void caxpy_kernel(float2* __restrict__ y, const float2* __restrict__ x, float a, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) {
    const float2 v = x[e];
    float2 o = y[e];
    o.x += a * v.x;
    o.y += a * v.y;
    y[e] = o;
  }
}

__global__ void weight_rows_kernel(float2* __restrict__ u, const float* __restrict__ w, int64_t M, int J) {
  const int64_t total = M * J;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const float s = w[e % M];
    float2 v = u[e];
    u[e] = make_float2(v.x * s, v.y * s);
  }
}

__global__ void copy_split_kernel(Split dst, CSplit src) {
  const int64_t n = dst.n0 + dst.n1;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT)
    dst.at(e) = src.at(e);
}

__global__ void zero_split_kernel(Split dst) {
  const int64_t n = dst.n0 + dst.n1;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT)
    dst.at(e) = make_float2(0.f, 0.f);
}

// 256 FP64 values in LDS -> s[0], by a fixed tree
__device__ __forceinline__ void tree256(double* s) {
  for (int h = NT / 2; h > 0; h >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
  }
  __syncthreads();
}

__global__ __launch_bounds__(NT) void dot_partial_kernel(CSplit a, CSplit b, double* __restrict__ part) {
  __shared__ double s[NT];
  const int64_t n = a.n0 + a.n1;
  double acc = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) {
    const float2 u = a.at(e), v = b.at(e);
    acc += (double)u.x * (double)v.x + (double)u.y * (double)v.y;
  }
  s[threadIdx.x] = acc;
  tree256(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(NT) void dot_final_kernel(const double* __restrict__ part, int nparts,
                                                       double* __restrict__ out) {
  __shared__ double s[NT];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += NT) acc += part[i];
  s[threadIdx.x] = acc;
  tree256(s);
  if (threadIdx.x == 0) *out = s[0];
}

// alpha = rho / <d, q> (0 when <d, q> = 0)
__global__ void cg_alpha_kernel(const double* __restrict__ rho, const double* __restrict__ dq,
                                double* __restrict__ alpha) {
  if (threadIdx.x == 0) *alpha = *dq != 0.0 ? *rho / *dq : 0.0;
}

// x += alpha d, r -= alpha q
__global__ void cg_xr_kernel(Split x, float2* __restrict__ r, const float2* __restrict__ d,
                             const float2* __restrict__ q, const double* __restrict__ alpha) {
  const float a = (float)*alpha;
  const int64_t n = x.n0 + x.n1;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) {
    const float2 dv = d[e], qv = q[e];
    float2& xv = x.at(e);
    xv.x += a * dv.x;
    xv.y += a * dv.y;
    float2 rv = r[e];
    rv.x -= a * qv.x;
    rv.y -= a * qv.y;
    r[e] = rv;
  }
}

// beta = rho_new / rho (0 when rho = 0); rho = rho_new; rr = rho_new
__global__ void cg_beta_kernel(double* __restrict__ rho, const double* __restrict__ rho_new,
                               double* __restrict__ beta, double* __restrict__ rr) {
  if (threadIdx.x != 0) return;
  *beta = *rho != 0.0 ? *rho_new / *rho : 0.0;
  *rho = *rho_new;
  if (rr) *rr = *rho_new;
}

// d = r + beta d
__global__ void cg_d_kernel(float2* __restrict__ d, const float2* __restrict__ r, int64_t n,
                            const double* __restrict__ beta) {
  const float b = (float)*beta;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) {
    const float2 rv = r[e];
    float2 dv = d[e];
    d[e] = make_float2(rv.x + b * dv.x, rv.y + b * dv.y);
  }
}

__global__ void copy_scalar_kernel(const double* __restrict__ src, double* __restrict__ dst) {
  if (threadIdx.x == 0) *dst = *src;
}

// out[e] = sum_i part[i * stride + e] in index order (plain FP32 adds)
__global__ void sum_rows_kernel(float2* __restrict__ out, const float2* __restrict__ part, int n, int64_t stride,
                                int64_t len) {
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < len; e += (int64_t)gridDim.x * NT) {
    float2 s = part[e];
    for (int i = 1; i < n; ++i) {
      const float2 v = part[(int64_t)i * stride + e];
      s.x = s.x + v.x;
      s.y = s.y + v.y;
    }
    out[e] = s;
  }
}

__global__ void sum_doubles_kernel(double* __restrict__ out, const double* __restrict__ part, int n, int64_t stride) {
  if (threadIdx.x != 0) return;
  double s = part[0];
  for (int i = 1; i < n; ++i) s += part[(int64_t)i * stride];
  *out = s;
}

}  // namespace

hipError_t caxpy_launch(float2* y, const float2* x, float a, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(caxpy_kernel, dim3(grid_for(n)), dim3(NT), 0, st, y, x, a, n);
  return hipGetLastError();
}

hipError_t weight_rows_launch(float2* u, const float* w, int64_t M, int J, hipStream_t st) {
  if (M * J <= 0) return hipSuccess;
  hipLaunchKernelGGL(weight_rows_kernel, dim3(grid_for(M * J)), dim3(NT), 0, st, u, w, M, J);
  return hipGetLastError();
}

hipError_t copy_split_launch(float2* d0, float2* d1, const float2* s0, const float2* s1, int64_t n0, int64_t n1,
                             hipStream_t st) {
  if (n0 + n1 <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_split_kernel, dim3(grid_for(n0 + n1)), dim3(NT), 0, st, Split{d0, d1, n0, n1},
                     CSplit{s0, s1, n0, n1});
  return hipGetLastError();
}

hipError_t zero_split_launch(float2* d0, float2* d1, int64_t n0, int64_t n1, hipStream_t st) {
  if (n0 + n1 <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_split_kernel, dim3(grid_for(n0 + n1)), dim3(NT), 0, st, Split{d0, d1, n0, n1});
  return hipGetLastError();
}

hipError_t dot_launch(const float2* a, const float2* b, int64_t n, double* part, double* out, hipStream_t st) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(DOT_BLOCKS), dim3(NT), 0, st, CSplit{a, nullptr, n, 0},
                     CSplit{b, nullptr, n, 0}, part);
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(NT), 0, st, part, DOT_BLOCKS, out);
  return hipGetLastError();
}

hipError_t dot2_launch(const float2* a0, const float2* a1, int64_t n0, int64_t n1, double* part, double* out,
                       hipStream_t st) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(DOT_BLOCKS), dim3(NT), 0, st, CSplit{a0, a1, n0, n1},
                     CSplit{a0, a1, n0, n1}, part);
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(NT), 0, st, part, DOT_BLOCKS, out);
  return hipGetLastError();
}

hipError_t cg_alpha_launch(const double* rho, const double* dq, double* alpha, hipStream_t st) {
  hipLaunchKernelGGL(cg_alpha_kernel, dim3(1), dim3(64), 0, st, rho, dq, alpha);
  return hipGetLastError();
}

hipError_t cg_xr_launch(float2* x0, float2* x1, int64_t n0, int64_t n1, float2* r, const float2* d, const float2* q,
                        const double* alpha, hipStream_t st) {
  if (n0 + n1 <= 0) return hipSuccess;
  hipLaunchKernelGGL(cg_xr_kernel, dim3(grid_for(n0 + n1)), dim3(NT), 0, st, Split{x0, x1, n0, n1}, r, d, q, alpha);
  return hipGetLastError();
}

hipError_t cg_beta_launch(double* rho, const double* rho_new, double* beta, double* rr, hipStream_t st) {
  hipLaunchKernelGGL(cg_beta_kernel, dim3(1), dim3(64), 0, st, rho, rho_new, beta, rr);
  return hipGetLastError();
}

hipError_t cg_d_launch(float2* d, const float2* r, int64_t n, const double* beta, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(cg_d_kernel, dim3(grid_for(n)), dim3(NT), 0, st, d, r, n, beta);
  return hipGetLastError();
}

hipError_t sum_rows_launch(float2* out, const float2* part, int n, int64_t stride, int64_t len, hipStream_t st) {
  if (len <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sum_rows_kernel, dim3(grid_for(len)), dim3(NT), 0, st, out, part, n, stride, len);
  return hipGetLastError();
}

hipError_t sum_doubles_launch(double* out, const double* part, int n, int64_t stride, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sum_doubles_kernel, dim3(1), dim3(64), 0, st, out, part, n, stride);
  return hipGetLastError();
}

hipError_t copy_scalar_launch(const double* src, double* dst, hipStream_t st) {
  hipLaunchKernelGGL(copy_scalar_kernel, dim3(1), dim3(64), 0, st, src, dst);
  return hipGetLastError();
}

}  // namespace mx
