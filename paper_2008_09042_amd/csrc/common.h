// Internal declarations shared by the HIP translation units of libmaxwell.
// Nothing here crosses the C ABI (see include/maxwell.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <vector>

namespace mx {

// ---------------------------------------------------------------- complex helpers
struct cf { float x, y; };  // interleaved complex64, same bytes as maxwell_complex64

__host__ __device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline float2 cmulc(float2 a, float2 b) {  // conj(a) * b
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__host__ __device__ inline float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// ---------------------------------------------------------------- GEMM
// C[b][m][n] = alpha * sum_k opA(b, m, k) * opB(b, k, n)  (+ C when accumulate)
// All strides in complex elements.  conjA / conjB conjugate the operand.
struct GemmArgs {
  int64_t M, N, K, batch;
  const float2* A; int64_t a_bs, a_ms, a_ks; int conjA;
  const float2* B; int64_t b_bs, b_ks, b_ns; int conjB;
  float2* C; int64_t c_bs, c_ms, c_ns;
  float alpha;
  const float* alpha_dev;  // optional device scalar multiplying alpha
  int accumulate;
  int splits;  // reduction split over workgroups: 0 = heuristic, otherwise as given (tuned)
};

// Split-K factor for g picked by timing candidates on the device (g's operand pointers must
// be valid; ws must hold max_ws bytes).  The choice is cached per shape for the process; with
// MAXWELL_GEMM_AUTOTUNE=0 in the environment the heuristic (0) is returned.  Synchronous: for
// plan creation only.
int gemm_autotune(const GemmArgs& g, int precision, void* ws, size_t max_ws, hipStream_t st,
                  float* best_ms = nullptr);  // best_ms: the chosen split's time per launch
// Bytes of workspace the GEMM needs for split-K partials for these sizes.
size_t gemm_workspace_bytes(const GemmArgs& g);
// Enqueue.  `ws` must hold gemm_workspace_bytes(g) bytes (may be null if 0).
hipError_t gemm_launch(const GemmArgs& g, int precision, void* ws, hipStream_t st);

// BF16 split of an FP32 complex array into hi/lo planes (used for constant bases).
hipError_t split_bf16_launch(const float2* src, int64_t count, uint16_t* hi, uint16_t* lo,
                             hipStream_t st);
// The device splits (hardware converts, GEMM operand split, core split) on n FP32 values.
hipError_t bf16_split_diag_launch(const float* x, int64_t n, int variant, uint16_t* hi, uint16_t* lo,
                                  hipStream_t st);

// ---------------------------------------------------------------- FFT
// Transform along one axis of data laid out [outer][n][inner] (complex elements).
// centred unitary DFT; dir = -1 forward (exp(-2 pi i ...)), +1 inverse.
struct FftAxisArgs {
  float2* data;           // in/out (in place)
  const float2* src;      // input (may equal data)
  int64_t n, inner, outer;
  int dir;
  const float2* twiddle;  // n entries, exp(-2 pi i t / n)
  int nrad; int radix[12];
  // optional image premultiply (forward, first axis pass): m = x[img_index] * src
  const float2* premul; int64_t outer_per_coil;
  // optional Cartesian sampling fused into the pass (index p within a coil of N elements,
  // coil j): the first inverse pass reads samples[j][inv[p]] (zero where inv[p] < 0) in
  // place of src; the last forward pass writes samples[j][inv[p]] for inv[p] >= 0 in place
  // of data.  Needs J N < 2^32 and M > 0.
  const int32_t* in_inv; const float2* in_samples;
  // optional for the reading pass: the sorted mask [M] and, per line of the last axis within
  // a coil, the first sample at or after it [N / n + 1]; with them a tile of whole lines of
  // one coil places its samples directly (no inverse-mask lookup per point)
  const int32_t* in_mask; const int32_t* in_lptr;
  const int32_t* out_inv; float2* out_samples;
  int64_t coil_elems, nsamples;  // N, M
  uint32_t coil_magic, coil_shift;  // multiply-high division by N (set by fft_axis_launch)
  int lines;              // lines per workgroup (set by fft_axis_launch)
  // optional gridding window (the NUFFT's zero-pad and crop with deapodisation, 2D grids of
  // g0 x g1 with the centred wn0 x wn1 window at (woff0, woff1)); grid rows and columns
  // outside the window that no later pass reads are neither computed nor written:
  //   win = WIN_PAD (first forward pass, along rows): reads, in place of src,
  //        src[j][r0][r1] premul[r0][r1] iphi[r0] iphi[wn0 + r1] (src the coil maps
  //        [J][wn0][wn1], premul the image); writes only the window's rows
  //   win = WIN_ROWS_IN (second forward pass, along columns): rows outside the window are
  //        taken as zero, not read
  //   win = WIN_COLS_OUT (first inverse pass, along rows): writes only the window's columns
  //   crop (last inverse pass, along columns, with crop_out set): writes only the window,
  //        crop_out[j][r0][r1] = v iphi[r0] iphi[wn0 + r1], and skips columns outside it
  const float* iphi; float2* crop_out;
  int woff0, woff1, wn0, wn1;
  int win;
};
constexpr int WIN_PAD = 1, WIN_ROWS_IN = 2, WIN_COLS_OUT = 3;
hipError_t fft_axis_launch(const FftAxisArgs& a, hipStream_t st);
// A pass prepared for launch (lines per workgroup, magic numbers, kernel variant, grid, LDS).
struct FftLaunch {
  FftAxisArgs a;
  int smp;
  bool twl;
  int64_t blocks;
  size_t lds;
};
hipError_t fft_axis_prepare(const FftAxisArgs& a, FftLaunch& out);
// Several passes per launch: descriptors in the kernel arguments.
constexpr int FFT_MULTI = 16;
struct FftMulti {
  FftAxisArgs d[FFT_MULTI];
  int start[FFT_MULTI + 1];
  int n;
};
// While a sink is set on the calling thread (non-null), fft_axis_launch appends the prepared
// pass to it instead of launching; fft_collect(nullptr) ends collection.
void fft_collect(std::vector<FftLaunch>* sink);
// Launches prepared passes of independent arrays, several per launch.
hipError_t fft_multi_launch(const std::vector<FftLaunch>& ls, hipStream_t st);
int fft_factorise(int64_t n, int* radix);  // returns number of passes, 0 if unsupported

// ---------------------------------------------------------------- elementwise / sampling
hipError_t gather_launch(const float2* kspace, int64_t N, const int32_t* idx, int64_t M, int J,
                         float2* y, hipStream_t st);
hipError_t scatter_launch(const float2* y, int64_t M, const int32_t* inv_mask, int64_t N, int J,
                          float2* kspace, hipStream_t st);
// r = w (.) (E - y); partial FP64 sums of w |E - y|^2 into part[nblocks]; returns nblocks.
int residual_blocks(int64_t total);
hipError_t residual_launch(const float2* E, const float2* y, const float* w, int64_t M, int J,
                           float2* r, double* part, hipStream_t st);
// The same residual at r[inv[m] J + j] (r must not alias E or y), with the same loss partials
// (residual_blocks(M J) of them).
hipError_t residual_ordered_launch(const float2* E, const float2* y, const float* w, int64_t M, int J,
                                   const int32_t* inv, float2* r, double* part, hipStream_t st);
hipError_t reduce_loss_launch(const double* part, int nblocks, double* loss, hipStream_t st);
// gx[n] = s sum_j conj(S[j][n]) g[j][n] ; g[j][n] <- s conj(x[n]) g[j][n] (when h_inplace)
hipError_t adjoint_combine_launch(const float2* S, float2* g, const float2* x, int64_t N, int J,
                                  float alpha, const float* scale_dev, float2* gx, int want_h,
                                  hipStream_t st);
// Writes the device's constant-rate wall clock (hipDeviceAttributeWallClockRate) to *dst.
hipError_t stamp_launch(uint64_t* dst, hipStream_t st);
hipError_t scale_copy_launch(const float2* src, float2* dst, int64_t count, float alpha,
                             const float* scale_dev, hipStream_t st);

}  // namespace mx
