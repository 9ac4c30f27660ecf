// Batched centred unitary DFT along one axis, staged in LDS.
//
// The operator F inside F_s (paper Sec. II-A, Eq. (1)) is read as the centred
// unitary DFT: pixel r and frequency k both run over [-n/2, n/2) on each
// axis, forward kernel exp(-2 pi i k r / n), scale n^{-1/2} per axis.  With
// array indices r' = r + n/2 and k' = k + n/2,
//   exp(-2 pi i k r / n) = exp(-2 pi i k' r' / n) (-1)^{r'} (-1)^{k'} (-1)^{n/2},
// so the centred transform is a plain DFT with a chessboard sign on input
// and output and a global sign: no index shifts are needed.  The inverse is
// the same with the conjugate kernel.
//
// Data are [outer][n][inner] complex; a workgroup stages a tile of lines in
// LDS (coalesced along whichever dimension is contiguous in memory), runs
// self-sorting Stockham passes of radix 8, 4, 2, 3 or 5 (each thread
// holding its butterflies in registers between two barriers, so the tile is
// transformed in place), and writes back.  Twiddles come from a table
// exp(-2 pi i t / n) built on the host in FP64.
#include "fft_device.h"

namespace mx {

namespace {

constexpr int NT = 256;
constexpr int TILE = 8192;          // complex elements per LDS tile at most (before padding)
constexpr int TW_LDS_MAX = 1024;    // twiddle tables up to this length are staged in LDS

// complex elements of the LDS tile for T lines of length n
__host__ __device__ inline int tile_elems(int n, int T, bool contiguous) { return contiguous ? T * (n + 1) : T * n; }

// TWL: the twiddle table is copied into LDS behind the tile.
template <bool TWL>
__global__ __launch_bounds__(NT) void fft_axis_kernel(FftAxisArgs a) {
  extern __shared__ float2 lds[];
  const int n = (int)a.n;
  const float2* tw = a.twiddle;
  if constexpr (TWL) {
    float2* twl = lds + tile_elems(n, a.lines, a.inner == 1);
    for (int i = threadIdx.x; i < n; i += NT) twl[i] = a.twiddle[i];
    tw = twl;
  }
  LdsLines tg;
  int64_t o0, t0;
  int Tvalid;
  if (a.inner == 1) {
    tg.T = a.lines;
    tg.LS = n + 1;
    tg.ES = 1;
    o0 = (int64_t)blockIdx.x * tg.T;
    t0 = 0;
    Tvalid = (int)((a.outer - o0) < tg.T ? (a.outer - o0) : tg.T);
  } else {
    tg.T = a.lines;
    tg.LS = 1;
    tg.ES = tg.T;
    const int64_t chunks = (a.inner + tg.T - 1) / tg.T;
    o0 = blockIdx.x / chunks;
    t0 = (blockIdx.x % chunks) * tg.T;
    Tvalid = (int)((a.inner - t0) < tg.T ? (a.inner - t0) : tg.T);
  }
  const int total = tg.T * n;
  // ---- load (with optional image premultiply and the input chessboard sign)
  for (int e = threadIdx.x; e < total; e += NT) {
    int l, i;
    if (a.inner == 1) { l = e / n; i = e % n; } else { i = e / tg.T; l = e % tg.T; }
    float2 v = make_float2(0.f, 0.f);
    if (l < Tvalid) {
      int64_t gidx, o, t;
      if (a.inner == 1) { o = o0 + l; t = 0; } else { o = o0; t = t0 + l; }
      gidx = (o * a.n + i) * a.inner + t;
      v = a.src[gidx];
      if (a.premul) {
        const int64_t img = ((o % a.outer_per_coil) * a.n + i) * a.inner + t;
        v = cmul(v, a.premul[img]);
      }
      if (i & 1) v = make_float2(-v.x, -v.y);
    }
    lds[l * tg.LS + i * tg.ES] = v;
  }
  __syncthreads();
  lds_fft_lines<NT, TILE>(lds, tg, n, a.radix, a.nrad, tw, a.dir);
  // ---- store with the output chessboard sign, global sign and n^{-1/2}
  const float scale = (((n / 2) & 1) ? -1.f : 1.f) * rsqrtf((float)n);
  for (int e = threadIdx.x; e < total; e += NT) {
    int l, i;
    if (a.inner == 1) { l = e / n; i = e % n; } else { i = e / tg.T; l = e % tg.T; }
    if (l >= Tvalid) continue;
    int64_t o, t;
    if (a.inner == 1) { o = o0 + l; t = 0; } else { o = o0; t = t0 + l; }
    float2 v = lds[l * tg.LS + i * tg.ES];
    const float s = (i & 1) ? -scale : scale;
    a.data[(o * a.n + i) * a.inner + t] = cscale(v, s);
  }
}

}  // namespace

int fft_factorise(int64_t n, int* radix) {
  if (n < 2 || n > 4096 || (n & 1)) return 0;
  int64_t m = n;
  int twos = 0, threes = 0, fives = 0;
  while (m % 2 == 0) { m /= 2; ++twos; }
  while (m % 3 == 0) { m /= 3; ++threes; }
  while (m % 5 == 0) { m /= 5; ++fives; }
  if (m != 1) return 0;
  int np = 0;
  while (twos >= 3) { radix[np++] = 8; twos -= 3; }
  if (twos == 2) radix[np++] = 4;
  if (twos == 1) radix[np++] = 2;
  for (int i = 0; i < threes; ++i) radix[np++] = 3;
  for (int i = 0; i < fives; ++i) radix[np++] = 5;
  return np;
}

// Lines per workgroup: enough workgroups to spread a small transform over the whole
// chip (about 1024), at most 64 lines or TILE elements per tile, and for strided lines
// at least 8 adjacent ones (64-byte runs per load).
hipError_t fft_axis_launch(const FftAxisArgs& args, hipStream_t st) {
  FftAxisArgs a = args;
  const int n = (int)a.n;
  const bool contiguous = a.inner == 1;
  const bool twl = n <= TW_LDS_MAX;
  int Tmax = (TILE - (twl ? n : 0)) / (contiguous ? n + 1 : n);
  if (Tmax > 64) Tmax = 64;
  if (Tmax < 1) Tmax = 1;
  const int64_t lines = a.outer * a.inner;
  int64_t T = (lines + 1023) / 1024;
  if (!contiguous && T < 8) T = 8;
  if (T > Tmax) T = Tmax;
  if (!contiguous && T > a.inner) T = a.inner;
  if (T < 1) T = 1;
  a.lines = (int)T;
  const int64_t blocks = contiguous ? (a.outer + T - 1) / T : a.outer * ((a.inner + T - 1) / T);
  if (blocks <= 0) return hipSuccess;
  const size_t lds = (size_t)(tile_elems(n, a.lines, contiguous) + (twl ? n : 0)) * sizeof(float2);
  if (twl)
    hipLaunchKernelGGL(fft_axis_kernel<true>, dim3((unsigned)blocks), dim3(NT), lds, st, a);
  else
    hipLaunchKernelGGL(fft_axis_kernel<false>, dim3((unsigned)blocks), dim3(NT), lds, st, a);
  return hipGetLastError();
}

}  // namespace mx
