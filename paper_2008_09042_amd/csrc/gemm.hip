// Strided-batched complex GEMM on CDNA4 matrix cores.
//
// C[b][m][n] = alpha * sum_k opA(b,m,k) opB(b,k,n) (+ C)
//
// This is the contraction behind the basis apply s_j = B c_j (paper Sec. II-B,
// Eq. (5)), its adjoint B^H (the basis block of J_G^H, Sec. II-B), and every
// k-mode product of the Tucker form (Sec. II-E).  A complex product is formed
// from four real products on the FP32 matrix-core instruction
// v_mfma_f32_16x16x4_f32:  Cr += Ar Br - Ai Bi,  Ci += Ar Bi + Ai Br.
// The BF16_SPLIT variant forms each real product from the split operands
// (hi*hi + hi*lo + lo*hi) on v_mfma_f32_16x16x32_bf16 with FP32 accumulation.
//
// Tiling: 256 threads (4 waves of 64) per 64x64 complex output tile, each
// wave owning a 32x32 quadrant as 2x2 blocks of 16x16.  Operand tiles are
// staged in LDS as split real/imaginary planes; the global loads walk the
// unit-stride dimension of each operand so they coalesce for any layout.
// Long reductions (basis adjoints: K up to N) are split over workgroups;
// partial tiles go to the workspace and are summed in a fixed order, so the
// result is deterministic.
#include "common.h"

#include <array>
#include <cstdlib>
#include <map>
#include <mutex>
#include <vector>

namespace mx {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int BM = 64, BN = 64, NT = 256;
constexpr int BK32 = 16;   // complex k per LDS stage, FP32 path
constexpr int BKS = 32;    // complex k per LDS stage, BF16-split path
constexpr int PAD = 4;

struct TileCtx {
  int64_t m0, n0, kbeg, kend;
  const float2* A; const float2* B;
};

__device__ inline void tile_coords(const GemmArgs& g, int splits, int64_t kchunk, TileCtx& t,
                                   int64_t& b, int& sp) {
  const int64_t ntn = (g.N + BN - 1) / BN;
  const int64_t tiles = ((g.M + BM - 1) / BM) * ntn;
  const int64_t tile = blockIdx.x % tiles;
  t.m0 = (tile / ntn) * BM;
  t.n0 = (tile % ntn) * BN;
  const int64_t bz = blockIdx.x / tiles;
  b = bz / splits;
  sp = (int)(bz % splits);
  t.kbeg = (int64_t)sp * kchunk;
  t.kend = t.kbeg + kchunk < g.K ? t.kbeg + kchunk : g.K;
  t.A = g.A + b * g.a_bs;
  t.B = g.B + b * g.b_bs;
}

// One operand stage held in registers between its global load and its LDS store, so the
// loads of the next stage are in flight while the current one is multiplied.  Element e of
// a ROWS x BK stage walks the operand's unit-stride dimension (k when ks == 1, else the
// row); an element outside the operand reads the operand's first element and is zeroed.
template <int ROWS, int BK>
struct Stage {
  static constexpr int CNT = ROWS * BK / NT;
  float2 v[CNT];
  __device__ static void coords(int u, bool kfast, int& ri, int& ki) {
    const int e = threadIdx.x + u * NT;
    if (kfast) { ri = e / BK; ki = e % BK; } else { ki = e / ROWS; ri = e % ROWS; }
  }
  __device__ void fetch(const float2* P, int64_t r0, int64_t rows, int64_t rs, int64_t ks, int64_t k0,
                        int64_t kend) {
    const bool kfast = ks == 1;
#pragma unroll
    for (int u = 0; u < CNT; ++u) {
      int ri, ki;
      coords(u, kfast, ri, ki);
      const int64_t r = r0 + ri, k = k0 + ki;
      const bool ok = r < rows && k < kend;
      const float2 x = P[ok ? r * rs + k * ks : 0];
      const uint32_t m = ok ? 0xffffffffu : 0u;
      v[u] = make_float2(__uint_as_float(__float_as_uint(x.x) & m), __uint_as_float(__float_as_uint(x.y) & m));
    }
  }
};

__device__ inline void store_tile(const GemmArgs& g, const TileCtx& t, int64_t b, int sp, int splits,
                                  float2* partial, f32x4 (&accR)[2][2], f32x4 (&accI)[2][2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  float alpha = g.alpha;
  if (g.alpha_dev) alpha *= *g.alpha_dev;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) {
        const int64_t m = t.m0 + wm + i * 16 + 4 * (lane >> 4) + r;
        const int64_t n = t.n0 + wn + j * 16 + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        float2 v = make_float2(accR[i][j][r], accI[i][j][r]);
        if (splits > 1) {
          partial[(((int64_t)sp * g.batch + b) * g.M + m) * g.N + n] = v;
        } else {
          float2* c = g.C + b * g.c_bs + m * g.c_ms + n * g.c_ns;
          v = cscale(v, alpha);
          if (g.accumulate) v = cadd(v, *c);
          *c = v;
        }
      }
}

__global__ __launch_bounds__(NT) void cgemm_f32_kernel(GemmArgs g, int splits, int64_t kchunk,
                                                       float2* partial) {
  __shared__ float AR[BK32][BM + PAD], AI[BK32][BM + PAD], BR[BK32][BN + PAD], BI[BK32][BN + PAD];
  TileCtx t;
  int64_t b;
  int sp;
  tile_coords(g, splits, kchunk, t, b, sp);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4 accR[2][2], accI[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) { accR[i][j] = f32x4{0, 0, 0, 0}; accI[i][j] = f32x4{0, 0, 0, 0}; }

  Stage<BM, BK32> sa;
  Stage<BN, BK32> sb;
  const bool akf = g.a_ks == 1, bkf = g.b_ks == 1;
  if (t.kbeg < t.kend) {
    sa.fetch(t.A, t.m0, g.M, g.a_ms, g.a_ks, t.kbeg, t.kend);
    sb.fetch(t.B, t.n0, g.N, g.b_ns, g.b_ks, t.kbeg, t.kend);
  }
  for (int64_t k0 = t.kbeg; k0 < t.kend; k0 += BK32) {
#pragma unroll
    for (int u = 0; u < Stage<BM, BK32>::CNT; ++u) {
      int mi, ki;
      Stage<BM, BK32>::coords(u, akf, mi, ki);
      AR[ki][mi] = sa.v[u].x;
      AI[ki][mi] = g.conjA ? -sa.v[u].y : sa.v[u].y;
    }
#pragma unroll
    for (int u = 0; u < Stage<BN, BK32>::CNT; ++u) {
      int ni, ki;
      Stage<BN, BK32>::coords(u, bkf, ni, ki);
      BR[ki][ni] = sb.v[u].x;
      BI[ki][ni] = g.conjB ? -sb.v[u].y : sb.v[u].y;
    }
    __syncthreads();
    if (k0 + BK32 < t.kend) {
      sa.fetch(t.A, t.m0, g.M, g.a_ms, g.a_ks, k0 + BK32, t.kend);
      sb.fetch(t.B, t.n0, g.N, g.b_ns, g.b_ks, k0 + BK32, t.kend);
    }
#pragma unroll
    for (int kk = 0; kk < BK32; kk += 4) {
      const int kr = kk + (lane >> 4), c = lane & 15;
      float aR[2], aI[2], bR[2], bI[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) { aR[i] = AR[kr][wm + i * 16 + c]; aI[i] = AI[kr][wm + i * 16 + c]; }
#pragma unroll
      for (int j = 0; j < 2; ++j) { bR[j] = BR[kr][wn + j * 16 + c]; bI[j] = BI[kr][wn + j * 16 + c]; }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          accR[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(aR[i], bR[j], accR[i][j], 0, 0, 0);
          accR[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(-aI[i], bI[j], accR[i][j], 0, 0, 0);
          accI[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(aR[i], bI[j], accI[i][j], 0, 0, 0);
          accI[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(aI[i], bR[j], accI[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  store_tile(g, t, b, sp, splits, partial, accR, accI);
}

// Round-to-nearest-even FP32 -> BF16 (bit pattern), finite inputs.
__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ inline void split_pair(float a, uint16_t& hi, uint16_t& lo) {
  hi = bf16_rne(a);
  lo = bf16_rne(a - bf16_to_f32(hi));
}

// BF16-split: operand planes hold hi and lo parts of real and imaginary planes.
// LDS layout per operand: [plane(4): Rhi,Rlo,Ihi,Ilo][row 16 lanes-dim][k BKS] with k fastest so
// a lane reads its 8 consecutive k values as one 16-byte vector.
constexpr int KP = BKS + 8;  // padded k extent (bf16 elements)

__global__ __launch_bounds__(NT) void cgemm_bf16s_kernel(GemmArgs g, int splits, int64_t kchunk,
                                                         float2* partial) {
  __shared__ __attribute__((aligned(16))) uint16_t As[4][BM][KP];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[4][BN][KP];
  TileCtx t;
  int64_t b;
  int sp;
  tile_coords(g, splits, kchunk, t, b, sp);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4 accR[2][2], accI[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) { accR[i][j] = f32x4{0, 0, 0, 0}; accI[i][j] = f32x4{0, 0, 0, 0}; }

  const bool akfast = (g.a_ks == 1), bkfast = (g.b_ks == 1);
  Stage<BM, BKS> sa;
  Stage<BN, BKS> sb;
  if (t.kbeg < t.kend) {
    sa.fetch(t.A, t.m0, g.M, g.a_ms, g.a_ks, t.kbeg, t.kend);
    sb.fetch(t.B, t.n0, g.N, g.b_ns, g.b_ks, t.kbeg, t.kend);
  }
  for (int64_t k0 = t.kbeg; k0 < t.kend; k0 += BKS) {
#pragma unroll
    for (int u = 0; u < Stage<BM, BKS>::CNT; ++u) {
      int mi, ki;
      Stage<BM, BKS>::coords(u, akfast, mi, ki);
      float2 v = sa.v[u];
      if (g.conjA) v.y = -v.y;
      uint16_t h, l;
      split_pair(v.x, h, l); As[0][mi][ki] = h; As[1][mi][ki] = l;
      split_pair(v.y, h, l); As[2][mi][ki] = h; As[3][mi][ki] = l;
    }
#pragma unroll
    for (int u = 0; u < Stage<BN, BKS>::CNT; ++u) {
      int ni, ki;
      Stage<BN, BKS>::coords(u, bkfast, ni, ki);
      float2 v = sb.v[u];
      if (g.conjB) v.y = -v.y;
      uint16_t h, l;
      split_pair(v.x, h, l); Bs[0][ni][ki] = h; Bs[1][ni][ki] = l;
      split_pair(v.y, h, l); Bs[2][ni][ki] = h; Bs[3][ni][ki] = l;
    }
    __syncthreads();
    if (k0 + BKS < t.kend) {
      sa.fetch(t.A, t.m0, g.M, g.a_ms, g.a_ks, k0 + BKS, t.kend);
      sb.fetch(t.B, t.n0, g.N, g.b_ns, g.b_ks, k0 + BKS, t.kend);
    }
    // one 16x16x32 step covers the whole BKS = 32 stage
    const int c = lane & 15, kq = (lane >> 4) * 8;
    bf16x8 a[2][4], bb[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        a[i][p] = *reinterpret_cast<const bf16x8*>(&As[p][wm + i * 16 + c][kq]);
        bb[i][p] = *reinterpret_cast<const bf16x8*>(&Bs[p][wn + i * 16 + c][kq]);
      }
    // negated imaginary A parts for the Ar*Br - Ai*Bi term
    bf16x8 na[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int p = 0; p < 2; ++p) na[i][p] = -a[i][2 + p];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        // real part: Ar*Br - Ai*Bi, each as hi*hi + hi*lo + lo*hi
        accR[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], bb[j][0], accR[i][j], 0, 0, 0);
        accR[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], bb[j][1], accR[i][j], 0, 0, 0);
        accR[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1], bb[j][0], accR[i][j], 0, 0, 0);
        accR[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(na[i][0], bb[j][2], accR[i][j], 0, 0, 0);
        accR[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(na[i][0], bb[j][3], accR[i][j], 0, 0, 0);
        accR[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(na[i][1], bb[j][2], accR[i][j], 0, 0, 0);
        // imaginary part: Ar*Bi + Ai*Br
        accI[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], bb[j][2], accI[i][j], 0, 0, 0);
        accI[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], bb[j][3], accI[i][j], 0, 0, 0);
        accI[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1], bb[j][2], accI[i][j], 0, 0, 0);
        accI[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][2], bb[j][0], accI[i][j], 0, 0, 0);
        accI[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][2], bb[j][1], accI[i][j], 0, 0, 0);
        accI[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][3], bb[j][0], accI[i][j], 0, 0, 0);
      }
    __syncthreads();
  }
  store_tile(g, t, b, sp, splits, partial, accR, accI);
}

// C = alpha * sum_p partial[p] (+ C).  G threads per output element, each summing every G-th
// split in four interleaved chains (independent loads), combined through LDS in a fixed
// order: the result does not depend on timing.
template <int G>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(GemmArgs g, int splits, const float2* partial) {
  constexpr int OPB = 256 / G;  // output elements per workgroup
  __shared__ float2 red[G][OPB];
  const int64_t total = g.batch * g.M * g.N;
  const int lo = threadIdx.x % OPB, grp = threadIdx.x / OPB;
  const int64_t e = blockIdx.x * (int64_t)OPB + lo;
  float2 s0 = make_float2(0.f, 0.f), s1 = s0, s2 = s0, s3 = s0;
  if (e < total) {
    const float2* pe = partial + e;
    int p = grp;
    for (; p + 3 * G < splits; p += 4 * G) {
      s0 = cadd(s0, pe[(int64_t)p * total]);
      s1 = cadd(s1, pe[(int64_t)(p + G) * total]);
      s2 = cadd(s2, pe[(int64_t)(p + 2 * G) * total]);
      s3 = cadd(s3, pe[(int64_t)(p + 3 * G) * total]);
    }
    for (; p < splits; p += G) s0 = cadd(s0, pe[(int64_t)p * total]);
  }
  red[grp][lo] = cadd(cadd(s0, s1), cadd(s2, s3));
  __syncthreads();
  if (grp != 0 || e >= total) return;
  float2 s = red[0][lo];
  for (int q = 1; q < G; ++q) s = cadd(s, red[q][lo]);
  const int64_t n = e % g.N, m = (e / g.N) % g.M, b = e / (g.N * g.M);
  float alpha = g.alpha;
  if (g.alpha_dev) alpha *= *g.alpha_dev;
  float2* c = g.C + b * g.c_bs + m * g.c_ms + n * g.c_ns;
  s = cscale(s, alpha);
  if (g.accumulate) s = cadd(s, *c);
  *c = s;
}

__global__ void split_bf16_kernel(const float2* src, int64_t count, uint16_t* hi, uint16_t* lo) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    float2 v = src[e];
    uint16_t h, l;
    split_pair(v.x, h, l); hi[2 * e] = h; lo[2 * e] = l;
    split_pair(v.y, h, l); hi[2 * e + 1] = h; lo[2 * e + 1] = l;
  }
}

void choose_split(const GemmArgs& g, int bk, int& splits, int64_t& kchunk) {
  const int64_t tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN) * g.batch;
  splits = 1;
  const int64_t kblocks = (g.K + bk - 1) / bk;
  if (g.splits > 0) {
    splits = (int)std::min<int64_t>(g.splits, std::max<int64_t>(kblocks, 1));
  } else if (tiles < 512 && kblocks >= 8) {
    int64_t want = (1024 + tiles - 1) / tiles;
    int64_t maxs = kblocks / 4;
    if (want > maxs) want = maxs;
    if (want > 1024) want = 1024;
    if (want < 1) want = 1;
    splits = (int)want;
  }
  const int64_t kb_per = (kblocks + splits - 1) / splits;
  kchunk = kb_per * bk;
  splits = (int)((g.K + kchunk - 1) / kchunk);
}

}  // namespace

size_t gemm_workspace_bytes(const GemmArgs& g) {
  int splits;
  int64_t kchunk;
  choose_split(g, BK32, splits, kchunk);
  int s2;
  int64_t kc2;
  choose_split(g, BKS, s2, kc2);
  if (s2 > splits) splits = s2;
  if (splits <= 1) return 0;
  return (size_t)splits * (size_t)(g.batch * g.M * g.N) * sizeof(float2);
}

hipError_t gemm_launch(const GemmArgs& g, int precision, void* ws, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  const int bk = precision == 1 ? BKS : BK32;
  int splits;
  int64_t kchunk;
  choose_split(g, bk, splits, kchunk);
  if (g.K <= 0) { splits = 1; kchunk = 0; }
  const int64_t tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  const int64_t nblocks = tiles * g.batch * splits;
  if (nblocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  dim3 grid((unsigned)nblocks, 1, 1);
  float2* partial = splits > 1 ? reinterpret_cast<float2*>(ws) : nullptr;
  if (precision == 1)
    hipLaunchKernelGGL(cgemm_bf16s_kernel, grid, dim3(NT), 0, st, g, splits, kchunk, partial);
  else
    hipLaunchKernelGGL(cgemm_f32_kernel, grid, dim3(NT), 0, st, g, splits, kchunk, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splits <= 1) return e;
  // threads per output: enough workgroups (about 512) when there are few outputs
  const int64_t total = g.batch * g.M * g.N;
  int G = 1;
  while (G < 16 && 2 * G <= splits && total * G < 512 * 256) G *= 2;
  const unsigned blocks = (unsigned)((total + 256 / G - 1) / (256 / G));
  switch (G) {
    case 1: hipLaunchKernelGGL(splitk_reduce_kernel<1>, dim3(blocks), dim3(256), 0, st, g, splits, partial); break;
    case 2: hipLaunchKernelGGL(splitk_reduce_kernel<2>, dim3(blocks), dim3(256), 0, st, g, splits, partial); break;
    case 4: hipLaunchKernelGGL(splitk_reduce_kernel<4>, dim3(blocks), dim3(256), 0, st, g, splits, partial); break;
    case 8: hipLaunchKernelGGL(splitk_reduce_kernel<8>, dim3(blocks), dim3(256), 0, st, g, splits, partial); break;
    default: hipLaunchKernelGGL(splitk_reduce_kernel<16>, dim3(blocks), dim3(256), 0, st, g, splits, partial); break;
  }
  return hipGetLastError();
}

int gemm_autotune(const GemmArgs& g0, int precision, void* ws, size_t max_ws, hipStream_t st, float* best_ms_out) {
  const char* env = std::getenv("MAXWELL_GEMM_AUTOTUNE");
  if (env && env[0] == '0') return 0;
  if (g0.M <= 0 || g0.N <= 0 || g0.K <= 0 || g0.batch <= 0) return 0;
  // the shape, strides and flags decide the timing; operand pointers do not
  const std::array<int64_t, 16> key = {g0.M, g0.N, g0.K, g0.batch, g0.a_ms, g0.a_ks, g0.b_ks, g0.b_ns,
                                       g0.c_ms, g0.c_ns, g0.conjA, g0.conjB, g0.accumulate, precision,
                                       g0.alpha_dev != nullptr, 0};
  static std::mutex mu;
  static std::map<std::array<int64_t, 16>, std::pair<int, float>> cache;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
      if (best_ms_out) *best_ms_out = it->second.second;
      return it->second.first;
    }
  }
  const int bk = precision == 1 ? BKS : BK32;
  const int64_t kblocks = (g0.K + bk - 1) / bk;
  std::vector<int> cands = {0, 1};
  for (int s = 2; s <= 1024 && s <= kblocks; s *= 2) cands.push_back(s);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return 0;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return 0; }
  int best = 0;
  float best_ms = 0.f;
  for (int c : cands) {
    GemmArgs g = g0;
    g.splits = c;
    if (gemm_workspace_bytes(g) > max_ws) continue;
    bool ok = gemm_launch(g, precision, ws, st) == hipSuccess;  // warm-up
    ok = ok && hipEventRecord(e0, st) == hipSuccess;
    for (int r = 0; ok && r < 3; ++r) ok = gemm_launch(g, precision, ws, st) == hipSuccess;
    ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float ms = 0.f;
    if (!ok || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) break;
    if (best_ms == 0.f || ms < best_ms) { best_ms = ms; best = c; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipGetLastError();
  best_ms /= 3.0f;  // per launch
  if (best_ms_out) *best_ms_out = best_ms;
  std::lock_guard<std::mutex> lk(mu);
  cache[key] = {best, best_ms};
  return best;
}

hipError_t split_bf16_launch(const float2* src, int64_t count, uint16_t* hi, uint16_t* lo,
                             hipStream_t st) {
  int64_t blocks = (count + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(split_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src, count, hi, lo);
  return hipGetLastError();
}

}  // namespace mx
