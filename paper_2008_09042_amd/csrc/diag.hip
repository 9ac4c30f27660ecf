// Diagnostic access to the device BF16 split routines of the BF16-split products
// (hi = bf16(a), lo = bf16(a - hi), round to nearest even), so that the split itself can
// be checked value by value against a host rounding rule.
//
//  variant 0: the packed hardware converts of the matrix-core tiles (split8 in
//             mfma_frag.h), which split W, V, h and Y in the plane kernels and build the
//             fragment-ordered factor operands;
//  variant 1: the software rounding of the tiled GEMM's operand split (split_bf16_launch);
//  variant 2: the software rounding of mfma_frag.h (bf16_rne), used by the core planes.
#include <algorithm>

#include "common.h"
#include "mfma_frag.h"

namespace mx {

namespace {

__global__ void split8_kernel(const float* __restrict__ x, int64_t n, uint16_t* __restrict__ hi,
                              uint16_t* __restrict__ lo) {
  const int64_t groups = (n + 7) / 8;
  for (int64_t gi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; gi < groups;
       gi += (int64_t)gridDim.x * blockDim.x) {
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = 8 * gi + e < n ? x[8 * gi + e] : 0.f;
    u16x8 h, l;
    split8(v, h, l);
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if (8 * gi + e < n) {
        hi[8 * gi + e] = h[e];
        lo[8 * gi + e] = l[e];
      }
  }
}

__global__ void rne_split_kernel(const float* __restrict__ x, int64_t n, uint16_t* __restrict__ hi,
                                 uint16_t* __restrict__ lo) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const float f = x[e];
    const unsigned short h = bf16_rne(f);
    hi[e] = h;
    lo[e] = bf16_rne(f - bf16_f32(h));
  }
}

}  // namespace

hipError_t bf16_split_diag_launch(const float* x, int64_t n, int variant, uint16_t* hi, uint16_t* lo,
                                  hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  if (variant == 0) {
    hipLaunchKernelGGL(split8_kernel, dim3(blocks), dim3(256), 0, st, x, n, hi, lo);
    return hipGetLastError();
  }
  if (variant == 1) {  // complex pairs (n is even, checked by the caller)
    return split_bf16_launch(reinterpret_cast<const float2*>(x), n / 2, hi, lo, st);
  }
  hipLaunchKernelGGL(rne_split_kernel, dim3(blocks), dim3(256), 0, st, x, n, hi, lo);
  return hipGetLastError();
}

}  // namespace mx
