// Arguments and launchers of the third-mode products of the fused path.
#pragma once

#include "common.h"

namespace mx {

struct Mode3Args {
  int J, Q, n2, r2;        // coils, r0 r1, readout length, readout rank
  const float2* T1;        // forward in  [J][Q][r2]
  float2* T3;              // forward out [J][n2][Q]
  const float2* T3b;       // adjoint in  [J][n2][Q]
  float2* T1b;             // adjoint out [J][Q][r2]
  const void* U2F;         // A operand U2 (i2, p2), fragment order (frag_operand_launch)
  const void* U2CF;        // B operand conj(U2) (i2, p2), fragment order
};

bool mode3_supported(int r2);
hipError_t mode3_fwd_launch(const Mode3Args& a, int precision, hipStream_t st);
hipError_t mode3_adj_launch(const Mode3Args& a, int precision, hipStream_t st);

}  // namespace mx
