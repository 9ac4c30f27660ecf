// Arguments and launchers of the Tucker core contractions (core x_4 c and its adjoint).
#pragma once

#include "common.h"

namespace mx {

// Geometry of the BF16-split core planes built once per plan.  Both are stored in
// matrix-core fragment order: [row block of 16][k' step of 32][64 lanes][8 bf16], so
// each wave's operand load for one step is one contiguous 1 KiB run.
struct CoreGeom {
  int64_t R;        // rho = (p0, p1, p2) rows of the core
  int K;            // basis size
  int64_t Rp;       // R rounded up to the adjoint chunk
  int KP;           // 2K rounded up to 32 (forward reduction length, real-block)
  int Kp;           // K rounded up to 16 (adjoint output rows)
  size_t fwd_elems() const { return (size_t)((R + 15) / 16 * 16) * KP; }  // per plane (hi or lo)
  size_t adj_elems() const { return (size_t)Kp * 2 * Rp; }
  size_t total_elems() const { return 2 * fwd_elems() + 2 * adj_elems(); }
  // FP32 copies in fragment order (complex entries): forward [R16][Kp], adjoint [Kp][Rp]
  size_t fwd32_elems() const { return (size_t)((R + 15) / 16 * 16) * Kp; }
  size_t adj32_elems() const { return (size_t)Kp * Rp; }
};

CoreGeom core_geom(int64_t R, int K);
bool core_supported(int J);
int core_adj_chunks(int64_t R);

struct CoreArgs {
  CoreGeom g;
  int J;
  const float2* core;          // [R][K] (FP32 kernels)
  const uint16_t* fwd_hi;      // forward planes (BF16-split kernels), fragment order over [R][KP], step-major
  const uint16_t* fwd_lo;
  const uint16_t* adj_hi;      // adjoint planes: conj(core)^T, fragment order over [Kp][2 Rp], chunk-step-major
  const uint16_t* adj_lo;
  const float2* fwd_f32;       // FP32 copies in fragment order (FP32 kernels; null: read `core`)
  const float2* adj_f32;
  const float2* in;            // forward: c [J][K];  adjoint: T1b [J][R]
  float2* out;                 // forward: T1 [J][R]; adjoint: gc [J][K]
  float2* part;                // adjoint chunk partials [chunks][Kp][Jp]
};

// Builds the four BF16 planes of `core` into dst (core_geom(R, K).total_elems() entries).
hipError_t core_split_launch(const float2* core, const CoreGeom& g, uint16_t* dst, hipStream_t st);
// Builds the FP32 fragment-order copies (forward then adjoint) into dst
// (fwd32_elems() + adj32_elems() complex entries).
hipError_t core_frag32_launch(const float2* core, const CoreGeom& g, float2* dst, hipStream_t st);
hipError_t core_fwd_launch(const CoreArgs& a, int precision, hipStream_t st);
// gc = alpha * (*scale_dev if given) * core^H T1b
hipError_t core_adj_launch(const CoreArgs& a, int precision, float alpha, const float* scale_dev, hipStream_t st);
size_t core_adj_part_bytes(int64_t R, int K, int J);

}  // namespace mx
