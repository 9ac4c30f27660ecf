// Kernels of the constrained density reconstruction (paper Sec. II-C): total-variation prox,
// per-coil projection on the data-consistency balls, and the ADMM bookkeeping.
//
// TV(x) = sum_i sqrt(sum_d |x[i + e_d] - x[i]|^2) over the image (forward differences, zero at
// the last index of each axis; complex values with the real and imaginary parts coupled).
// Its prox, argmin 1/2 ||x - z||^2 + lam TV(x), runs Chambolle's dual projection steps
// (J. Math. Imaging Vis. 20, 2004) from a zero dual field P (ndim components per pixel):
//     d = div P - z / lam;   g = grad d;   P <- (P + tau g) / (1 + tau |g|),   tau = 1/(4 ndim)
// and returns x = z - lam div P, with div = -grad^H.  lam = 1 / rho is read from device memory
// (rho adapts inside the ADMM loop).  One launch per step: each thread recomputes d at its
// pixel and at its forward neighbours from the previous dual field (double-buffered), so the
// divergence and the gradient need no barrier between them.
//
// Ball projection (the closed form of the paper): z_k = y_k + eps_k (w_k - y_k) /
// max(||w_k - y_k||, eps_k), with the per-coil distance accumulated in FP64 by a fixed-order
// two-stage reduction.
#include "solver.h"
#include "admm.h"

#include <utility>

namespace mx {

namespace {

constexpr int NT = 256;

inline unsigned grid_for(int64_t total, int64_t cap = 16384) {
  int64_t b = (total + NT - 1) / NT;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (unsigned)b;
}

struct Dims {
  int nd;
  int64_t n[3], stride[3], N;
};

__device__ __forceinline__ void coords(const Dims& g, int64_t i, int64_t (&c)[3]) {
  int64_t r = i;
  for (int d = g.nd - 1; d >= 0; --d) {
    c[d] = r % g.n[d];
    r /= g.n[d];
  }
}

// mode 0: out = div P - z / lam;  mode 1: out = z - lam div P
__global__ void tv_div_kernel(Dims g, const float2* __restrict__ P, const float2* __restrict__ z,
                              const double* __restrict__ rho, float lam_fixed, int mode, float2* __restrict__ out) {
  const float lam = rho ? (float)(1.0 / *rho) : lam_fixed;
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < g.N; i += (int64_t)gridDim.x * NT) {
    int64_t c[3];
    coords(g, i, c);
    float2 dv = make_float2(0.f, 0.f);
    for (int d = 0; d < g.nd; ++d) {
      const float2* Pd = P + d * g.N;
      if (c[d] < g.n[d] - 1) dv = cadd(dv, Pd[i]);
      if (c[d] > 0) dv = csub(dv, Pd[i - g.stride[d]]);
    }
    const float2 zi = z[i];
    out[i] = mode == 0 ? make_float2(dv.x - zi.x / lam, dv.y - zi.y / lam)
                       : make_float2(zi.x - lam * dv.x, zi.y - lam * dv.y);
  }
}

// One Chambolle step in one pass: Pout = (Pin + tau grad d) / (1 + tau |grad d|) with
// d = div Pin - z / lam recomputed at the pixel and at its forward neighbours (Pin is only
// read, so the step needs no grid-wide barrier between the divergence and the gradient).
__device__ __forceinline__ float2 tv_d_at(const Dims& g, const float2* __restrict__ P, const float2* __restrict__ z,
                                          float inv_lam, int64_t i, const int64_t (&c)[3]) {
  float2 dv = make_float2(0.f, 0.f);
  for (int d = 0; d < g.nd; ++d) {
    const float2* Pd = P + d * g.N;
    if (c[d] < g.n[d] - 1) dv = cadd(dv, Pd[i]);
    if (c[d] > 0) dv = csub(dv, Pd[i - g.stride[d]]);
  }
  const float2 zi = z[i];
  return make_float2(dv.x - zi.x * inv_lam, dv.y - zi.y * inv_lam);
}

__global__ void tv_step_kernel(Dims g, const float2* __restrict__ Pin, float2* __restrict__ Pout,
                               const float2* __restrict__ z, const double* __restrict__ rho, float lam_fixed,
                               float tau) {
  const float inv_lam = rho ? (float)*rho : 1.f / lam_fixed;
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < g.N; i += (int64_t)gridDim.x * NT) {
    int64_t c[3];
    coords(g, i, c);
    const float2 di = tv_d_at(g, Pin, z, inv_lam, i, c);
    float2 gr[3];
    float m2 = 0.f;
    for (int d = 0; d < g.nd; ++d) {
      if (c[d] < g.n[d] - 1) {
        int64_t cn[3] = {c[0], c[1], c[2]};
        cn[d] += 1;
        gr[d] = csub(tv_d_at(g, Pin, z, inv_lam, i + g.stride[d], cn), di);
      } else {
        gr[d] = make_float2(0.f, 0.f);
      }
      m2 += gr[d].x * gr[d].x + gr[d].y * gr[d].y;
    }
    const float inv = 1.f / (1.f + tau * sqrtf(m2));
    for (int d = 0; d < g.nd; ++d) {
      const float2 pv = Pin[d * g.N + i];
      Pout[d * g.N + i] = make_float2((pv.x + tau * gr[d].x) * inv, (pv.y + tau * gr[d].y) * inv);
    }
  }
}

// part[j * PB + b] = sum over block b's share of coil j of |w - y|^2 (FP64)
constexpr int PB = 64;
__global__ __launch_bounds__(NT) void coil_dist_kernel(const float2* __restrict__ w, const float2* __restrict__ y,
                                                       int64_t M, double* __restrict__ part) {
  __shared__ double s[NT];
  const int j = blockIdx.y;
  const float2* wj = w + (int64_t)j * M;
  const float2* yj = y + (int64_t)j * M;
  double acc = 0.0;
  for (int64_t m = blockIdx.x * (int64_t)NT + threadIdx.x; m < M; m += (int64_t)PB * NT) {
    const double dx = (double)wj[m].x - (double)yj[m].x, dy = (double)wj[m].y - (double)yj[m].y;
    acc += dx * dx + dy * dy;
  }
  s[threadIdx.x] = acc;
  for (int h = NT / 2; h > 0; h >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
  }
  if (threadIdx.x == 0) part[(int64_t)j * PB + blockIdx.x] = s[0];
}

__global__ void coil_dist_final_kernel(const double* __restrict__ part, double* __restrict__ dist) {
  __shared__ double s[PB];
  const int j = blockIdx.x;
  s[threadIdx.x] = part[(int64_t)j * PB + threadIdx.x];
  for (int h = PB / 2; h > 0; h >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
  }
  if (threadIdx.x == 0) dist[j] = sqrt(s[0]);
}

__global__ void ball_kernel(const float2* __restrict__ w, const float2* __restrict__ y, const float* __restrict__ eps,
                            const double* __restrict__ dist, int64_t M, int J, float2* __restrict__ z) {
  const int64_t total = M * J;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int j = (int)(e / M);
    const double ej = (double)eps[j];
    const double den = dist[j] > ej ? dist[j] : ej;
    const float f = den > 0.0 ? (float)(ej / den) : 0.f;
    const float2 yv = y[e], wv = w[e];
    z[e] = make_float2(yv.x + f * (wv.x - yv.x), yv.y + f * (wv.y - yv.y));
  }
}

// out = a * u + b * v
__global__ void lincomb_kernel(float2* __restrict__ out, const float2* __restrict__ u, float a,
                               const float2* __restrict__ v, float b, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) {
    const float2 uv = u[e], vv = v[e];
    out[e] = make_float2(a * uv.x + b * vv.x, a * uv.y + b * vv.y);
  }
}

// hist = (rho, r, s) with r = sqrt(r2), s = rho sqrt(s2); residual balancing of rho
__global__ void admm_rho_kernel(const double* __restrict__ r2, const double* __restrict__ s2, double* __restrict__ rho,
                                double* __restrict__ ufac, double* __restrict__ hist) {
  if (threadIdx.x != 0) return;
  const double r = sqrt(*r2), s = *rho * sqrt(*s2);
  if (hist) {
    hist[0] = *rho;
    hist[1] = r;
    hist[2] = s;
  }
  if (r > 10.0 * s) {
    *rho *= 2.0;
    *ufac = 0.5;
  } else if (s > 10.0 * r) {
    *rho *= 0.5;
    *ufac = 2.0;
  } else {
    *ufac = 1.0;
  }
}

__global__ void scale_dev_kernel(float2* __restrict__ v, int64_t n, const double* __restrict__ f) {
  const float s = (float)*f;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) {
    const float2 a = v[e];
    v[e] = make_float2(a.x * s, a.y * s);
  }
}

__global__ void set_scalar_kernel(double* __restrict__ dst, double v) {
  if (threadIdx.x == 0) *dst = v;
}

Dims make_dims(int nd, const int64_t* n) {
  Dims g;
  g.nd = nd;
  g.N = 1;
  for (int d = 0; d < 3; ++d) g.n[d] = d < nd ? n[d] : 1;
  for (int d = nd - 1; d >= 0; --d) {
    g.stride[d] = g.N;
    g.N *= g.n[d];
  }
  for (int d = nd; d < 3; ++d) g.stride[d] = 0;
  return g;
}

}  // namespace

hipError_t tv_prox_launch(int nd, const int64_t* n, const float2* z, const double* rho_dev, float lam, int iters,
                          float2* P, float2* P2, float2* x, hipStream_t st) {
  const Dims g = make_dims(nd, n);
  const unsigned gr = grid_for(g.N);
  const float tau = 1.f / (4.f * (float)nd);
  if (!rho_dev && !(lam > 0.f)) return copy_split_launch(x, nullptr, z, nullptr, g.N, 0, st);  // prox of 0
  hipError_t e = zero_split_launch(P, nullptr, (int64_t)nd * g.N, 0, st);
  if (e != hipSuccess) return e;
  float2 *pin = P, *pout = P2;
  for (int k = 0; k < iters; ++k) {
    hipLaunchKernelGGL(tv_step_kernel, dim3(gr), dim3(NT), 0, st, g, pin, pout, z, rho_dev, lam, tau);
    std::swap(pin, pout);
  }
  hipLaunchKernelGGL(tv_div_kernel, dim3(gr), dim3(NT), 0, st, g, pin, z, rho_dev, lam, 1, x);
  return hipGetLastError();
}

hipError_t ball_project_launch(const float2* w, const float2* y, const float* eps, int64_t M, int J, double* part,
                               double* dist, float2* z, hipStream_t st) {
  if (M * J == 0) return hipSuccess;
  hipLaunchKernelGGL(coil_dist_kernel, dim3(PB, J), dim3(NT), 0, st, w, y, M, part);
  hipLaunchKernelGGL(coil_dist_final_kernel, dim3(J), dim3(PB), 0, st, part, dist);
  hipLaunchKernelGGL(ball_kernel, dim3(grid_for(M * J)), dim3(NT), 0, st, w, y, eps, dist, M, J, z);
  return hipGetLastError();
}

int ball_part_doubles(int J) { return J * PB + J; }

hipError_t lincomb_launch(float2* out, const float2* u, float a, const float2* v, float b, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(lincomb_kernel, dim3(grid_for(n)), dim3(NT), 0, st, out, u, a, v, b, n);
  return hipGetLastError();
}

hipError_t admm_rho_launch(const double* r2, const double* s2, double* rho, double* ufac, double* hist,
                           hipStream_t st) {
  hipLaunchKernelGGL(admm_rho_kernel, dim3(1), dim3(64), 0, st, r2, s2, rho, ufac, hist);
  return hipGetLastError();
}

hipError_t scale_dev_launch(float2* v, int64_t n, const double* f, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scale_dev_kernel, dim3(grid_for(n)), dim3(NT), 0, st, v, n, f);
  return hipGetLastError();
}

hipError_t set_scalar_launch(double* dst, double v, hipStream_t st) {
  hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(64), 0, st, dst, v);
  return hipGetLastError();
}

}  // namespace mx
