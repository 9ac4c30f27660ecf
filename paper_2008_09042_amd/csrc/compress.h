// Accuracy-controlled Tucker compression (compress.hip).
#pragma once

#include "common.h"

namespace mx {

// B [N][K] (device, N = dims[0] dims[1] dims[2]) -> U_out[m] [dims[m]][ranks[m]] (device,
// capacity dims[m]^2), core_out [r0][r1][r2][K] (device, capacity N K), ranks and the
// discarded squared norm per mode (host).  Allocates and synchronises.
hipError_t tucker_compress_run(const int64_t* dims, int64_t K, const float2* B, double eps, float2* const* U_out,
                               float2* core_out, int64_t* ranks, double* dropped, hipStream_t st);

}  // namespace mx
