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
#include "common.h"

namespace mx {

namespace {

constexpr int NT = 256;
constexpr int TILE = 8192;          // complex elements per LDS tile (before padding)
constexpr int LDS_ELEMS = TILE + 256;

template <int R>
__device__ inline void dft_small(float2 (&v)[R], int dir);

template <>
__device__ inline void dft_small<2>(float2 (&v)[2], int) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

// multiply by -i*dir... helpers: rot(-i) for forward, rot(+i) for inverse
__device__ inline float2 mul_mi(float2 a, int dir) {  // a * (dir == -1 ? -i : +i)
  return dir < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

template <>
__device__ inline void dft_small<4>(float2 (&v)[4], int dir) {
  float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  float2 t2 = cadd(v[1], v[3]), t3 = mul_mi(csub(v[1], v[3]), dir);
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <>
__device__ inline void dft_small<8>(float2 (&v)[8], int dir) {
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  dft_small<4>(e, dir);
  dft_small<4>(o, dir);
  const float h = 0.70710678118654752440f;  // 1/sqrt(2)
  // w8^k, w8 = exp(dir * i pi / 4) (dir = -1 forward)
  float2 w1 = make_float2(h, dir * h);
  float2 o1 = cmul(o[1], w1);
  float2 o2 = mul_mi(o[2], dir);
  float2 o3 = cmul(o[3], make_float2(-h, dir * h));
  v[0] = cadd(e[0], o[0]); v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);   v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);   v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);   v[7] = csub(e[3], o3);
}

template <>
__device__ inline void dft_small<3>(float2 (&v)[3], int dir) {
  const float s = 0.86602540378443864676f;  // sin(2 pi / 3)
  float2 t1 = cadd(v[1], v[2]);
  float2 t2 = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
  float2 d = cscale(csub(v[1], v[2]), s);
  float2 rd = mul_mi(d, dir);  // forward: -i s (a1 - a2)
  v[0] = cadd(v[0], t1);
  v[1] = cadd(t2, rd);
  v[2] = csub(t2, rd);
}

template <>
__device__ inline void dft_small<5>(float2 (&v)[5], int dir) {
  const float c1 = 0.30901699437494742410f;   // cos(2 pi/5)
  const float c2 = -0.80901699437494742410f;  // cos(4 pi/5)
  const float s1 = 0.95105651629515357212f;   // sin(2 pi/5)
  const float s2 = 0.58778525229247312917f;   // sin(4 pi/5)
  float2 b1 = cadd(v[1], v[4]), b2 = cadd(v[2], v[3]);
  float2 d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
  float2 a0 = v[0];
  float2 t1 = make_float2(a0.x + c1 * b1.x + c2 * b2.x, a0.y + c1 * b1.y + c2 * b2.y);
  float2 t2 = make_float2(a0.x + c2 * b1.x + c1 * b2.x, a0.y + c2 * b1.y + c1 * b2.y);
  float2 u1 = make_float2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y);
  float2 u2 = make_float2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y);
  float2 ru1 = mul_mi(u1, dir), ru2 = mul_mi(u2, dir);
  v[0] = cadd(a0, cadd(b1, b2));
  v[1] = cadd(t1, ru1);
  v[4] = csub(t1, ru1);
  v[2] = cadd(t2, ru2);
  v[3] = csub(t2, ru2);
}

struct TileGeom {
  int T;          // lines in the tile
  int LS, ES;     // LDS strides of line and element
};

// One Stockham pass of radix R over `T` lines of length n held in LDS.
template <int R>
__device__ inline void stockham_pass(float2* lds, const TileGeom& tg, int n, int Ns,
                                     const float2* __restrict__ tw, int dir) {
  constexpr int MAXQ = (TILE / R + NT - 1) / NT;
  const int nR = n / R;
  const int nb = tg.T * nR;
  const int stride_tw = n / (Ns * R);
  float2 v[MAXQ][R];
#pragma unroll
  for (int q = 0; q < MAXQ; ++q) {
    const int bf = threadIdx.x + q * NT;
    if (bf < nb) {
      const int l = bf % tg.T, j = bf / tg.T;
      const int base = l * tg.LS;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = lds[base + (j + r * nR) * tg.ES];
      const int k = j % Ns;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 w = tw[k * r * stride_tw];
        if (dir > 0) w.y = -w.y;
        v[q][r] = cmul(v[q][r], w);
      }
      dft_small<R>(v[q], dir);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXQ; ++q) {
    const int bf = threadIdx.x + q * NT;
    if (bf < nb) {
      const int l = bf % tg.T, j = bf / tg.T;
      const int base = l * tg.LS;
      const int idxD = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
      for (int r = 0; r < R; ++r) lds[base + (idxD + r * Ns) * tg.ES] = v[q][r];
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(NT) void fft_axis_kernel(FftAxisArgs a) {
  __shared__ float2 lds[LDS_ELEMS];
  const int n = (int)a.n;
  TileGeom tg;
  int64_t o0, t0;
  int Tvalid;
  if (a.inner == 1) {
    tg.T = TILE / n;
    if (tg.T > 64) tg.T = 64;
    tg.LS = n + 1;
    tg.ES = 1;
    o0 = (int64_t)blockIdx.x * tg.T;
    t0 = 0;
    Tvalid = (int)((a.outer - o0) < tg.T ? (a.outer - o0) : tg.T);
  } else {
    tg.T = TILE / n;
    if (tg.T > 64) tg.T = 64;
    if (tg.T > a.inner) tg.T = (int)a.inner;
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
  int Ns = 1;
  for (int p = 0; p < a.nrad; ++p) {
    const int R = a.radix[p];
    switch (R) {
      case 8: stockham_pass<8>(lds, tg, n, Ns, a.twiddle, a.dir); break;
      case 4: stockham_pass<4>(lds, tg, n, Ns, a.twiddle, a.dir); break;
      case 2: stockham_pass<2>(lds, tg, n, Ns, a.twiddle, a.dir); break;
      case 3: stockham_pass<3>(lds, tg, n, Ns, a.twiddle, a.dir); break;
      default: stockham_pass<5>(lds, tg, n, Ns, a.twiddle, a.dir); break;
    }
    Ns *= R;
  }
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

hipError_t fft_axis_launch(const FftAxisArgs& a, hipStream_t st) {
  const int n = (int)a.n;
  int T = TILE / n;
  if (T > 64) T = 64;
  int64_t blocks;
  if (a.inner == 1) {
    blocks = (a.outer + T - 1) / T;
  } else {
    if (T > a.inner) T = (int)a.inner;
    blocks = a.outer * ((a.inner + T - 1) / T);
  }
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(fft_axis_kernel, dim3((unsigned)blocks), dim3(NT), 0, st, a);
  return hipGetLastError();
}

}  // namespace mx
