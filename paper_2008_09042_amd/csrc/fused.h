// Arguments and launchers of the fused 3D Tucker / line-sampling path.
#pragma once

#include "common.h"

namespace mx {

struct PlaneArgs {
  int n0, n1, n2, r0, r1, r0p, r1p;  // r0p, r1p: ranks rounded up to 16
  int J, L, G;                       // coils, sampled lines, coils per workgroup
  const float2* T3;                  // [J][n2][r0][r1]  (core x_4 c x_3 U2)
  const float2* xt;                  // [n2][n0][n1]     image, readout axis first, times the
                                     //                  chessboard sign (-1)^(i0 + i1)
  const int32_t* pos;                // [L]  k0 * n1 + k1 of each sampled line
  float2* Z;                         // [J][n2][L]  plane-DFT samples (fwd out / adj in)
  float2* T3b;                       // [J][n2][r0][r1] adjoint out (or null)
  float2* gxpart;                    // [ngroups][n2][n0][n1] adjoint out (or null)
  const float2* tw0;                 // twiddles for n0, n1
  const float2* tw1;
  int nrad0, nrad1;
  int rad0[12], rad1[12];
  int precision;
  // Factor operands in matrix-core fragment order, built at plan time (frag_operand_launch):
  const void* U0F;                   // A of P = U0 V:        A(i0, p0) = U0[i0][p0]
  const void* U1TF;                  // B of V = W U1^T:      B(p1, i1) = U1[i1][p1]
  const void* U1CF;                  // B of Y = h conj(U1):  B(i1, p1) = conj(U1[i1][p1])
  const void* U0HF;                  // A of Wb = U0^H Y:     A(p0, i0) = conj(U0[i0][p0])
  const void* U0SF;                  // U0F and U1TF with row i0 / column i1 times (-1)^i: the
  const void* U1TSF;                 //   adjoint's coil map P' = s P carries the output sign s
};

struct LineArgs {
  int J, n2;
  int64_t L, M;                      // M = L * n2
  const float2* Z;                   // fwd in  [J][n2][L]
  float2* out;                       // fwd out [J][M]: E (y == null) or w (.) (E - y), or null
  const float2* y;                   // measured data or null
  const float* w;                    // weights or null
  double* part;                      // per-block loss partials or null
  const float2* yin;                 // adj in [J][M]
  float2* Zw;                        // adj out [J][n2][L]; in the forward (with y), the weighted
                                     // residual taken back along the readout (transfer layout), or null
  float gscale;                      // prod_d (-1)^(n_d/2) / sqrt(n0 n1 n2)
  float alpha;                       // adjoint scale alpha * (*scale_dev)
  const float* scale_dev;
  const float2* tw2;
  int nrad2;
  int rad2[12];
};

bool fused_supported(int64_t n0, int64_t n1, int64_t n2, int64_t r0, int64_t r1, int precision);
// Fragment-ordered copy (see tucker_fused.hip) of O(o, k) = src[o * so + k * sk], conjugated
// if bit 0 of conj, times (-1)^o if bit 1, zero for o >= no or k >= nk, as an A (is_b = 0) or
// B (is_b = 1) operand; bit 2 stores k in the FP32 rank order of a K16 block (position
// 4 g + t holds k = g + 4 t of the block; FP32 only).
size_t frag_operand_bytes(int no, int nk, int is_b, int precision);
hipError_t frag_operand_launch(const float2* src, int no, int nk, int64_t so, int64_t sk, int conj, int is_b,
                               int precision, void* dst, hipStream_t st);
hipError_t plane_fwd_launch(const PlaneArgs& a, hipStream_t st);
hipError_t plane_adj_launch(const PlaneArgs& a, hipStream_t st);
int line_blocks(int J, int64_t L);
hipError_t line_fwd_launch(const LineArgs& a, hipStream_t st);
hipError_t line_adj_launch(const LineArgs& a, hipStream_t st);
// xt = x^T (R x C -> C x R); with n1_sign > 0 each row r = i0 n1_sign + i1 of x is multiplied
// by (-1)^(i0 + i1), the plane kernels' input chessboard sign (n1_sign even).
hipError_t transpose_launch(const float2* x, int64_t R, int64_t C, int n1_sign, float2* xt, hipStream_t st);
hipError_t reduce_transpose_launch(const float2* part, int ngrp, int64_t R, int64_t C, float alpha,
                                   const float* scale_dev, float2* gx, hipStream_t st);

}  // namespace mx
