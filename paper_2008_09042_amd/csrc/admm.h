// Launchers of the constrained-reconstruction kernels (admm.hip).
#pragma once

#include "common.h"

namespace mx {

// x = prox of lam TV at z (lam = 1 / *rho_dev when rho_dev is given, else lam); P and P2 hold
// nd * N complex values each (the dual field, double-buffered); iters Chambolle steps from
// P = 0, one launch per step.
hipError_t tv_prox_launch(int nd, const int64_t* n, const float2* z, const double* rho_dev, float lam, int iters,
                          float2* P, float2* P2, float2* x, hipStream_t st);
// z_j = y_j + eps_j (w_j - y_j) / max(||w_j - y_j||, eps_j); part holds ball_part_doubles(J)
// doubles (per-coil partial sums, then the distances)
hipError_t ball_project_launch(const float2* w, const float2* y, const float* eps, int64_t M, int J, double* part,
                               double* dist, float2* z, hipStream_t st);
int ball_part_doubles(int J);
// out = a u + b v
hipError_t lincomb_launch(float2* out, const float2* u, float a, const float2* v, float b, int64_t n, hipStream_t st);
// residual balancing: hist = (rho, r, s); rho and the dual scaling factor ufac updated
hipError_t admm_rho_launch(const double* r2, const double* s2, double* rho, double* ufac, double* hist,
                           hipStream_t st);
// v *= *f
hipError_t scale_dev_launch(float2* v, int64_t n, const double* f, hipStream_t st);
hipError_t set_scalar_launch(double* dst, double v, hipStream_t st);

}  // namespace mx
