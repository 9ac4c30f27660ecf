// Dense basis apply and adjoint for few coils (skinny.hip).
#pragma once

#include "common.h"

namespace mx {

// Shapes the streaming kernel takes: K a multiple of 4 (32-byte row runs), 1 <= J <= 64.
bool skinny_apply_supported(int64_t N, int64_t K, int J);
// Bytes of the fragment-ordered c operand the call builds.
size_t skinny_frag_bytes(int64_t K, int J);
// S [J][N] = B [N][K] c^T for c [J][K]; B 16-byte aligned; frag holds skinny_frag_bytes.
// c [J][K] = alpha (* alpha_dev) B^H h for h [J][N]; ws holds skinny_adjoint_bytes (the
// row-chunk partials, summed in a fixed order).  Same shapes as the apply (the plan uses it
// for J <= 16, where it beats the tiled GEMM).
size_t skinny_adjoint_bytes(int64_t N, int64_t K, int J);
hipError_t skinny_adjoint_launch(const float2* B, int64_t N, int64_t K, const float2* h, int J, int precision,
                                 float alpha, const float* alpha_dev, void* ws, float2* c, hipStream_t st);
hipError_t skinny_apply_launch(const float2* B, int64_t N, int64_t K, const float2* c, int J, int precision,
                               void* frag, float2* S, hipStream_t st);

}  // namespace mx
