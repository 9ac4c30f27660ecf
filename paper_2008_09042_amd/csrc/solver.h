// Launchers of the Gauss-Newton / conjugate-gradient vector kernels (solver.hip).
#pragma once

#include "common.h"

namespace mx {

constexpr int DOT_BLOCKS = 512;  // FP64 partial sums per inner product

// y += a x over n complex entries
hipError_t caxpy_launch(float2* y, const float2* x, float a, int64_t n, hipStream_t st);
// u[j][m] *= w[m]
hipError_t weight_rows_launch(float2* u, const float* w, int64_t M, int J, hipStream_t st);
// (d0 | d1) = (s0 | s1), blocks of n0 and n1 entries
hipError_t copy_split_launch(float2* d0, float2* d1, const float2* s0, const float2* s1, int64_t n0, int64_t n1,
                             hipStream_t st);
hipError_t zero_split_launch(float2* d0, float2* d1, int64_t n0, int64_t n1, hipStream_t st);
// *out = Re <a, b> over n entries in FP64; part holds DOT_BLOCKS doubles
hipError_t dot_launch(const float2* a, const float2* b, int64_t n, double* part, double* out, hipStream_t st);
// *out = ||(a0 | a1)||^2 in FP64 over the two blocks
hipError_t dot2_launch(const float2* a0, const float2* a1, int64_t n0, int64_t n1, double* part, double* out,
                       hipStream_t st);
// *alpha = *rho / *dq (0 if *dq == 0)
hipError_t cg_alpha_launch(const double* rho, const double* dq, double* alpha, hipStream_t st);
// (x0 | x1) += alpha d, r -= alpha q
hipError_t cg_xr_launch(float2* x0, float2* x1, int64_t n0, int64_t n1, float2* r, const float2* d, const float2* q,
                        const double* alpha, hipStream_t st);
// *beta = *rho_new / *rho (0 if *rho == 0); *rho = *rho_new; *rr = *rho_new if rr
hipError_t cg_beta_launch(double* rho, const double* rho_new, double* beta, double* rr, hipStream_t st);
// d = r + beta d
hipError_t cg_d_launch(float2* d, const float2* r, int64_t n, const double* beta, hipStream_t st);
hipError_t copy_scalar_launch(const double* src, double* dst, hipStream_t st);
// out = sum over i < n of part[i * stride .. + len) in index order; the same for FP64 scalars
hipError_t sum_rows_launch(float2* out, const float2* part, int n, int64_t stride, int64_t len, hipStream_t st);
hipError_t sum_doubles_launch(double* out, const double* part, int n, int64_t stride, hipStream_t st);

}  // namespace mx
