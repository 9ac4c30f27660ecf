// Fused path for a 3D Tucker basis with Cartesian sampling of full lines along
// the last axis (readout).  Paper: the bilinear operator of Sec. II-B, Eq. (5)
// with the Tucker-factored basis of Sec. II-E.
//
// Geometry: image (n0, n1, n2), ranks (r0, r1, r2), sampled lines L = {(k0, k1)}
// each with every k2, so y_j is [L][n2].  Because the mask is a product of a
// plane pattern and the full readout axis, the 3D centred DFT followed by the
// gather factors into (a) a 2D DFT of every (i0, i1) plane followed by a gather
// of the L sampled points, then (b) a 1D DFT along i2 of each sampled line.
// The coil map of plane i2 is
//     s_j[:, :, i2] = U0 W U1^T,   W = T3[j][i2] = (core x_4 c_j x_3 U2)[:, :, i2]
// (mode products of Sec. II-E), so no [J][N] array is ever written to memory:
//
//   forward   T1 = core x_4 c,  T3 = T1 x_3 U2                 (MFMA GEMM kernel)
//             plane kernel per (i2, coil): V = W U1^T, P = U0 V (MFMA, P kept in
//             registers), m = x (.) P, 2D DFT in LDS, gather L points -> Z[j][i2][L]
//             line kernel per (coil, 32 lines): DFT along i2, residual / loss -> y or r
//   adjoint   line kernel: inverse DFT along k2 (scaled) -> Zb[j][i2][L]
//             plane kernel per (i2, group of coils): recompute P, scatter Zb, inverse
//             2D DFT -> g;  gx += conj(P) (.) g (registers);  h = conj(x) (.) g;
//             Y = h conj(U1);  Wb = U0^H Y -> T3b[j][i2]
//             T1b = T3b x_3 U2^H,  gc = core^H T1b              (MFMA GEMM kernel)
//             gx = sum of the per-group partials (fixed order, no atomics)
//
// Matrix-core arithmetic.  FP32: each complex product is four real products on
// v_mfma_f32_16x16x4_f32.  BF16_SPLIT: the complex product over K is written as
// two real products over 2K (real-block form): with a' = (Re a_0, Im a_0, Re a_1,
// ...), Re c = a'.(Re b_0, -Im b_0, ...) and Im c = a'.(Im b_0, Re b_0, ...); every
// real operand is split into hi = bf16(v), lo = bf16(v - hi) and each real product
// is hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16 with FP32 accumulation.
// Constant factor operands are split once at plan time; W, V, h and Y are split
// in the kernel.
#include "fft_device.h"
#include "fused.h"

namespace mx {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int PT = 512;                          // threads per plane workgroup
constexpr int NWAVE = PT / 64;
constexpr int PMAX = 128;                        // max n0, n1 on this path
constexpr int PLANE_ELEMS = PMAX * (PMAX + 1);   // padded plane: 16,512 complex = 132 KB
constexpr int TW_ELEMS = 2 * PMAX;               // twiddles for n0 and n1
constexpr int SL = 40;                           // staged U1 row: 32 k' + 8 pad (bf16)
constexpr int SARR = 48 * SL;                    // one staged array (<= 48 columns)
constexpr int STAGE_ELEMS = 2 * 4 * SARR / 4;    // double-buffered chunk, in complex slots
// The twiddles and the adjoint's staging buffer share the region after the plane:
// they are never live at the same time (twiddles are reloaded for every coil).
constexpr int EXTRA_ELEMS = TW_ELEMS > STAGE_ELEMS ? TW_ELEMS : STAGE_ELEMS;
constexpr int LDS_ELEMS = PLANE_ELEMS + EXTRA_ELEMS;
constexpr int FFT_CHUNK = PMAX * PMAX / 2;       // elements per register chunk of a pass
// FP32 phase layout inside the plane region
constexpr int W_OFF = 0;                         // W  [r0p][r1p]  (<= 64 x 64)
constexpr int V_OFF = 64 * 64;                   // V  [r0p][n1]   (<= 64 x 128)

__device__ __forceinline__ f32x4 z4() { return f32x4{0.f, 0.f, 0.f, 0.f}; }

__device__ __forceinline__ void cmfma(f32x4& cr, f32x4& ci, float2 a, float2 b) {
  cr = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, cr, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, b.y, cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.y, ci, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.x, ci, 0, 0, 0);
}

// ---------------------------------------------------------------- BF16 split helpers
__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_f32(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

__device__ __forceinline__ void split8(const float (&v)[8], u16x8& hi, u16x8& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const unsigned short h = bf16_rne(v[e]);
    hi[e] = h;
    lo[e] = bf16_rne(v[e] - bf16_f32(h));
  }
}

__device__ __forceinline__ bf16x8 asbf(u16x8 v) { return __builtin_bit_cast(bf16x8, v); }

// c += a * b over one 32-wide k' step for both real-block halves (6 MFMAs).
__device__ __forceinline__ void mfma6(f32x4& cr, f32x4& ci, u16x8 ah, u16x8 al, u16x8 brh, u16x8 brl, u16x8 bih,
                             u16x8 bil) {
  cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(asbf(ah), asbf(brh), cr, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(asbf(ah), asbf(brl), cr, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(asbf(al), asbf(brh), cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(asbf(ah), asbf(bih), ci, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(asbf(ah), asbf(bil), ci, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(asbf(al), asbf(bih), ci, 0, 0, 0);
}

__device__ __forceinline__ u16x8 ld8(const unsigned short* p) { return *reinterpret_cast<const u16x8*>(p); }
__device__ __forceinline__ void st8(unsigned short* p, u16x8 v) { *reinterpret_cast<u16x8*>(p) = v; }

// Store one accumulator block as a B operand [n][k'] (k' = 2 * row + {0, 1}) in the
// real-block form: br = (Re, -Im), bi = (Im, Re), each split hi / lo.  The lane's four
// rows are consecutive, so its eight k' values are one 16-byte store per array.
__device__ __forceinline__ void store_bop(unsigned short* brh, unsigned short* brl, unsigned short* bih,
                                 unsigned short* bil, int ld, int n, int kp0, const f32x4& cr,
                                 const f32x4& ci) {
  float vr[8], vi[8];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    vr[2 * r] = cr[r];
    vr[2 * r + 1] = -ci[r];
    vi[2 * r] = ci[r];
    vi[2 * r + 1] = cr[r];
  }
  u16x8 h, l;
  split8(vr, h, l);
  st8(brh + n * ld + kp0, h);
  st8(brl + n * ld + kp0, l);
  split8(vi, h, l);
  st8(bih + n * ld + kp0, h);
  st8(bil + n * ld + kp0, l);
}

// ---------------------------------------------------------------- plane geometry
template <int N0, int N1>
struct Geo {
  int n0, n1, n2, r0, r1, r0p, r1p, PS;
  __device__ Geo(const PlaneArgs& a) {
    n0 = N0 ? N0 : a.n0;
    n1 = N1 ? N1 : a.n1;
    n2 = a.n2;
    r0 = a.r0;
    r1 = a.r1;
    r0p = a.r0p;
    r1p = a.r1p;
    PS = n1 + 1;
  }
};

template <int N0, int N1>
__device__ __forceinline__ void load_twiddles(const PlaneArgs& a, const Geo<N0, N1>& g, float2* lds) {
  float2* tw0 = lds + PLANE_ELEMS;
  float2* tw1 = tw0 + PMAX;
  for (int e = threadIdx.x; e < g.n0; e += PT) tw0[e] = a.tw0[e];
  for (int e = threadIdx.x; e < g.n1; e += PT) tw1[e] = a.tw1[e];
}

// 2D centred DFT of the plane (chessboard signs applied by the caller).
template <int N0, int N1>
__device__ __forceinline__ void plane_fft(const PlaneArgs& a, const Geo<N0, N1>& g, float2* lds, int dir) {
  const float2* tw0 = lds + PLANE_ELEMS;
  const float2* tw1 = tw0 + PMAX;
  auto rows = [&]() {
    if constexpr (N1 != 0) {
      lds_fft_ct<N1, PT, FFT_CHUNK>(lds, g.n0, g.PS, 1, tw1, dir);
    } else {
      LdsLines t{g.n0, g.PS, 1};
      lds_fft_lines<PT, FFT_CHUNK>(lds, t, g.n1, a.rad1, a.nrad1, tw1, dir);
    }
  };
  auto cols = [&]() {
    if constexpr (N0 != 0) {
      lds_fft_ct<N0, PT, FFT_CHUNK>(lds, g.n1, 1, g.PS, tw0, dir);
    } else {
      LdsLines t{g.n1, 1, g.PS};
      lds_fft_lines<PT, FFT_CHUNK>(lds, t, g.n0, a.rad0, a.nrad0, tw0, dir);
    }
  };
  if (dir < 0) { rows(); cols(); } else { cols(); rows(); }
}

// ---------------------------------------------------------------- FP32 contractions
// V = W U1^T ([r0p][n1] in LDS) from W = T3[j][i2] (zero-padded r0p x r1p in LDS).
template <int N0, int N1>
__device__ __forceinline__ void coilmap_V_f32(const PlaneArgs& a, const Geo<N0, N1>& g, int j, int i2, float2* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float2* src = a.T3 + ((size_t)j * g.n2 + i2) * g.r0 * g.r1;
  for (int e = threadIdx.x; e < g.r0p * g.r1p; e += PT) {
    const int p0 = e / g.r1p, p1 = e % g.r1p;
    lds[W_OFF + e] = (p0 < g.r0 && p1 < g.r1) ? src[p0 * g.r1 + p1] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  const int mbl = g.r0p / 16, nbl = g.n1 / 16;
  for (int blk = wave; blk < mbl * nbl; blk += NWAVE) {
    const int mb = blk / nbl, nb = blk % nbl;
    const int row = 16 * mb + (lane & 15), col = 16 * nb + (lane & 15);
    float2 bv[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int kk = 4 * s + (lane >> 4);
      bv[s] = (4 * s < g.r1p && kk < g.r1) ? a.U1[(size_t)col * g.r1 + kk] : make_float2(0.f, 0.f);
    }
    f32x4 cr = z4(), ci = z4();
#pragma unroll
    for (int s = 0; s < 16; ++s)
      if (4 * s < g.r1p) cmfma(cr, ci, lds[W_OFF + row * g.r1p + 4 * s + (lane >> 4)], bv[s]);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      lds[V_OFF + (16 * mb + 4 * (lane >> 4) + r) * g.n1 + col] = make_float2(cr[r], ci[r]);
  }
}

// P = U0 V, this wave's 16 rows, all n1 columns, into registers.
template <int N0, int N1>
__device__ __forceinline__ void coilmap_P_f32(const PlaneArgs& a, const Geo<N0, N1>& g, const float2* lds, f32x4 (&pr)[8],
                                     f32x4 (&pi)[8]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nbl = g.n1 / 16;
#pragma unroll
  for (int nb = 0; nb < 8; ++nb) { pr[nb] = z4(); pi[nb] = z4(); }
  if (wave >= g.n0 / 16) return;
  const int row = 16 * wave + (lane & 15);
  float2 av[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int kk = 4 * s + (lane >> 4);
    av[s] = (4 * s < g.r0p && kk < g.r0) ? a.U0[(size_t)row * g.r0 + kk] : make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    if (4 * s < g.r0p) {
      const int kk = 4 * s + (lane >> 4);
#pragma unroll
      for (int nb = 0; nb < 8; ++nb)
        if (nb < nbl) cmfma(pr[nb], pi[nb], av[s], lds[V_OFF + kk * g.n1 + 16 * nb + (lane & 15)]);
    }
  }
}

// Y = h conj(U1) (h in the plane) for this wave's rows; Wb = U0^H Y -> T3b.
template <int N0, int N1>
__device__ __forceinline__ void adjoint_W_f32(const PlaneArgs& a, const Geo<N0, N1>& g, int j, int i2, float2* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  f32x4 yr[4], yi[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) { yr[nb] = z4(); yi[nb] = z4(); }
  const int nbr = g.r1p / 16;
  if (wave < g.n0 / 16) {
    const int row = 16 * wave + (lane & 15);
    for (int k = 0; k < g.n1; k += 16) {
      float2 bv[4][4];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          const int kk = k + 4 * s + (lane >> 4), col = 16 * nb + (lane & 15);
          bv[s][nb] = (nb < nbr && col < g.r1) ? cconj(a.U1[(size_t)kk * g.r1 + col]) : make_float2(0.f, 0.f);
        }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const float2 av = lds[row * g.PS + k + 4 * s + (lane >> 4)];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
          if (nb < nbr) cmfma(yr[nb], yi[nb], av, bv[s][nb]);
      }
    }
  }
  __syncthreads();
  if (wave < g.n0 / 16) {
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
      if (nb < nbr)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          lds[(16 * wave + 4 * (lane >> 4) + r) * g.r1p + 16 * nb + (lane & 15)] = make_float2(yr[nb][r], yi[nb][r]);
  }
  __syncthreads();
  const int mbl = g.r0p / 16;
  float2* wo = a.T3b + ((size_t)j * g.n2 + i2) * g.r0 * g.r1;
  for (int blk = wave; blk < mbl * nbr; blk += NWAVE) {
    const int mb = blk / nbr, nb = blk % nbr;
    f32x4 cr = z4(), ci = z4();
    const int p0 = 16 * mb + (lane & 15);
    for (int k = 0; k < g.n0; k += 16) {
      float2 av[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int kk = k + 4 * s + (lane >> 4);
        av[s] = p0 < g.r0 ? cconj(a.U0[(size_t)kk * g.r0 + p0]) : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
        cmfma(cr, ci, av[s], lds[(k + 4 * s + (lane >> 4)) * g.r1p + 16 * nb + (lane & 15)]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int q0 = 16 * mb + 4 * (lane >> 4) + r, q1 = 16 * nb + (lane & 15);
      if (q0 < g.r0 && q1 < g.r1) wo[q0 * g.r1 + q1] = make_float2(cr[r], ci[r]);
    }
  }
}

// ---------------------------------------------------------------- BF16-split contractions
// LDS (unsigned short view of the plane region) during the coil-map phase:
//   WA hi/lo     [r0p][KS1]  A operand of V = W U1^T   (KS1 = KP1 + 8, padded row)
//   VB r/i hi/lo [n1][KS0]   B operand of P = U0 V     (KS0 = KP0 + 8)
__device__ __forceinline__ int kpad(int r) { return (2 * r + 31) / 32 * 32; }

template <int N0, int N1>
__device__ __forceinline__ void coilmap_V_bf(const PlaneArgs& a, const Geo<N0, N1>& g, int j, int i2, float2* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int KP1 = kpad(g.r1), KS1 = KP1 + 8, KP0 = kpad(g.r0), KS0 = KP0 + 8;
  unsigned short* u = reinterpret_cast<unsigned short*>(lds);
  unsigned short* wah = u;
  unsigned short* wal = wah + g.r0p * KS1;
  unsigned short* vbrh = wal + g.r0p * KS1;
  unsigned short* vbrl = vbrh + g.n1 * KS0;
  unsigned short* vbih = vbrl + g.n1 * KS0;
  unsigned short* vbil = vbih + g.n1 * KS0;
  // W rows as interleaved real pairs (the real-block A operand), split, zero-padded
  const float* src = reinterpret_cast<const float*>(a.T3 + ((size_t)j * g.n2 + i2) * g.r0 * g.r1);
  const int chunks = KP1 / 8;
  for (int e = threadIdx.x; e < g.r0p * chunks; e += PT) {
    const int p0 = e / chunks, c8 = (e % chunks) * 8;
    float v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = (p0 < g.r0 && c8 + t < 2 * g.r1) ? src[p0 * 2 * g.r1 + c8 + t] : 0.f;
    u16x8 h, l;
    split8(v, h, l);
    st8(wah + p0 * KS1 + c8, h);
    st8(wal + p0 * KS1 + c8, l);
  }
  // zero the padded k' tail of the V operand (k' from 2 r0p to KP0)
  const int tail = KP0 - 2 * g.r0p;
  for (int e = threadIdx.x; e < g.n1 * tail; e += PT) {
    const int n = e / tail, k = 2 * g.r0p + e % tail;
    vbrh[n * KS0 + k] = 0;
    vbrl[n * KS0 + k] = 0;
    vbih[n * KS0 + k] = 0;
    vbil[n * KS0 + k] = 0;
  }
  __syncthreads();
  // V blocks: B operand of U1^T from the plan's split copy [n1][KP1]
  const int mbl = g.r0p / 16, nbl = g.n1 / 16, ks = KP1 / 32;
  for (int nb = wave; nb < nbl; nb += NWAVE) {
    const int col = 16 * nb + (lane & 15);
    u16x8 brh[4], brl[4], bih[4], bil[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (s < ks) {
        const size_t o = (size_t)col * KP1 + 32 * s + 8 * (lane >> 4);
        brh[s] = ld8(a.U1B + 0 * (size_t)g.n1 * KP1 + o);
        brl[s] = ld8(a.U1B + 1 * (size_t)g.n1 * KP1 + o);
        bih[s] = ld8(a.U1B + 2 * (size_t)g.n1 * KP1 + o);
        bil[s] = ld8(a.U1B + 3 * (size_t)g.n1 * KP1 + o);
      }
    }
    for (int mb = 0; mb < mbl; ++mb) {
      f32x4 cr = z4(), ci = z4();
      const int row = 16 * mb + (lane & 15);
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if (s < ks) {
          const int ko = row * KS1 + 32 * s + 8 * (lane >> 4);
          mfma6(cr, ci, ld8(wah + ko), ld8(wal + ko), brh[s], brl[s], bih[s], bil[s]);
        }
      // V rows 16 mb + 4 (lane / 16) + r -> B operand of P at k' = 2 * row
      store_bop(vbrh, vbrl, vbih, vbil, KS0, col, 2 * (16 * mb + 4 * (lane >> 4)), cr, ci);
    }
  }
}

template <int N0, int N1>
__device__ __forceinline__ void coilmap_P_bf(const PlaneArgs& a, const Geo<N0, N1>& g, const float2* lds, f32x4 (&pr)[8],
                                    f32x4 (&pi)[8]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int KP1 = kpad(g.r1), KS1 = KP1 + 8, KP0 = kpad(g.r0), KS0 = KP0 + 8;
  const unsigned short* u = reinterpret_cast<const unsigned short*>(lds);
  const unsigned short* vbrh = u + 2 * g.r0p * KS1;
  const unsigned short* vbrl = vbrh + g.n1 * KS0;
  const unsigned short* vbih = vbrl + g.n1 * KS0;
  const unsigned short* vbil = vbih + g.n1 * KS0;
  const int nbl = g.n1 / 16, ks = KP0 / 32;
#pragma unroll
  for (int nb = 0; nb < 8; ++nb) { pr[nb] = z4(); pi[nb] = z4(); }
  if (wave >= g.n0 / 16) return;
  const int row = 16 * wave + (lane & 15);
  u16x8 ah[4], al[4];
#pragma unroll
  for (int s = 0; s < 4; ++s)
    if (s < ks) {
      const size_t o = (size_t)row * KP0 + 32 * s + 8 * (lane >> 4);
      ah[s] = ld8(a.U0A + o);
      al[s] = ld8(a.U0A + (size_t)g.n0 * KP0 + o);
    }
#pragma unroll
  for (int nb = 0; nb < 8; ++nb)
    if (nb < nbl) {
      const int col = 16 * nb + (lane & 15);
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if (s < ks) {
          const int ko = col * KS0 + 32 * s + 8 * (lane >> 4);
          mfma6(pr[nb], pi[nb], ah[s], al[s], ld8(vbrh + ko), ld8(vbrl + ko), ld8(vbih + ko), ld8(vbil + ko));
        }
    }
}

// Y = h conj(U1) with h (FP32 plane) split on the fly and U1's split copy staged through
// LDS one 32-wide k' chunk at a time; then Wb = U0^H Y -> T3b.
template <int N0, int N1>
__device__ __forceinline__ void adjoint_W_bf(const PlaneArgs& a, const Geo<N0, N1>& g, int j, int i2, float2* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nbr = g.r1p / 16, K2 = 2 * g.n1;
  unsigned short* stage = reinterpret_cast<unsigned short*>(lds + PLANE_ELEMS);
  f32x4 yr[4], yi[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) { yr[nb] = z4(); yi[nb] = z4(); }
  auto stage_chunk = [&](int s, int buf) {
    unsigned short* dst = stage + buf * 4 * SARR;
    for (int e = threadIdx.x; e < 4 * g.r1p * 4; e += PT) {
      const int arr = e / (g.r1p * 4), rem = e % (g.r1p * 4), p1 = rem / 4, c8 = (rem % 4) * 8;
      st8(dst + arr * SARR + p1 * SL + c8, ld8(a.U1C + (size_t)arr * g.r1p * K2 + (size_t)p1 * K2 + 32 * s + c8));
    }
  };
  const int ksteps = K2 / 32;
  stage_chunk(0, 0);
  __syncthreads();
  for (int s = 0; s < ksteps; ++s) {
    if (s + 1 < ksteps) stage_chunk(s + 1, (s + 1) & 1);
    if (wave < g.n0 / 16) {
      const int row = 16 * wave + (lane & 15);
      const int c0 = (32 * s + 8 * (lane >> 4)) / 2;  // first complex column of this lane's 8 k'
      float v[8];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float2 h = lds[row * g.PS + c0 + t];
        v[2 * t] = h.x;
        v[2 * t + 1] = h.y;
      }
      u16x8 ah, al;
      split8(v, ah, al);
      const unsigned short* src = stage + (s & 1) * 4 * SARR;
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
        if (nb < nbr) {
          const int ko = (16 * nb + (lane & 15)) * SL + 8 * (lane >> 4);
          mfma6(yr[nb], yi[nb], ah, al, ld8(src + ko), ld8(src + SARR + ko), ld8(src + 2 * SARR + ko),
                ld8(src + 3 * SARR + ko));
        }
    }
    __syncthreads();
  }
  // Y -> B operand of Wb, [r1p][KS] with k' = 2 i0 + {0, 1}
  const int KS = 2 * g.n0 + 8;
  unsigned short* u = reinterpret_cast<unsigned short*>(lds);
  unsigned short* ybrh = u;
  unsigned short* ybrl = ybrh + g.r1p * KS;
  unsigned short* ybih = ybrl + g.r1p * KS;
  unsigned short* ybil = ybih + g.r1p * KS;
  if (wave < g.n0 / 16) {
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
      if (nb < nbr)
        store_bop(ybrh, ybrl, ybih, ybil, KS, 16 * nb + (lane & 15), 2 * (16 * wave + 4 * (lane >> 4)), yr[nb],
                  yi[nb]);
  }
  __syncthreads();
  const int mbl = g.r0p / 16, K0 = 2 * g.n0;
  float2* wo = a.T3b + ((size_t)j * g.n2 + i2) * g.r0 * g.r1;
  for (int blk = wave; blk < mbl * nbr; blk += NWAVE) {
    const int mb = blk / nbr, nb = blk % nbr;
    f32x4 cr = z4(), ci = z4();
    const int p0 = 16 * mb + (lane & 15), p1 = 16 * nb + (lane & 15);
    for (int s = 0; s < K0 / 32; ++s) {
      const size_t ao = (size_t)p0 * K0 + 32 * s + 8 * (lane >> 4);
      const int ko = p1 * KS + 32 * s + 8 * (lane >> 4);
      mfma6(cr, ci, ld8(a.U0H + ao), ld8(a.U0H + (size_t)g.r0p * K0 + ao), ld8(ybrh + ko), ld8(ybrl + ko),
            ld8(ybih + ko), ld8(ybil + ko));
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int q0 = 16 * mb + 4 * (lane >> 4) + r;
      if (q0 < g.r0 && p1 < g.r1) wo[q0 * g.r1 + p1] = make_float2(cr[r], ci[r]);
    }
  }
}

// ---------------------------------------------------------------- plane kernels
template <int PREC, int N0, int N1>
__device__ __forceinline__ void coil_map(const PlaneArgs& a, const Geo<N0, N1>& g, int j, int i2, float2* lds,
                                f32x4 (&pr)[8], f32x4 (&pi)[8]) {
  if constexpr (PREC == 1) {
    coilmap_V_bf(a, g, j, i2, lds);
    __syncthreads();
    coilmap_P_bf(a, g, lds, pr, pi);
  } else {
    coilmap_V_f32(a, g, j, i2, lds);
    __syncthreads();
    coilmap_P_f32(a, g, lds, pr, pi);
  }
  __syncthreads();
}

template <int PREC, int N0, int N1>
__global__ __launch_bounds__(PT) void plane_fwd_kernel(PlaneArgs a) {
  __shared__ float2 lds[LDS_ELEMS];
  const Geo<N0, N1> g(a);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ngrp = (a.J + a.G - 1) / a.G;
  const int i2 = blockIdx.x / ngrp, grp = blockIdx.x % ngrp;
  const int nbl = g.n1 / 16;
  const float2* xp = a.xt + (size_t)i2 * g.n0 * g.n1;
  load_twiddles(a, g, lds);
  for (int j = grp * a.G; j < a.J && j < (grp + 1) * a.G; ++j) {
    f32x4 pr[8], pi[8];
    coil_map<PREC>(a, g, j, i2, lds, pr, pi);
    // m = x (.) P with the input chessboard sign, into the padded plane
    if (wave < g.n0 / 16) {
#pragma unroll
      for (int nb = 0; nb < 8; ++nb)
        if (nb < nbl)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i0 = 16 * wave + 4 * (lane >> 4) + r, i1 = 16 * nb + (lane & 15);
            float2 v = cmul(make_float2(pr[nb][r], pi[nb][r]), xp[i0 * g.n1 + i1]);
            if ((i0 + i1) & 1) v = make_float2(-v.x, -v.y);
            lds[i0 * g.PS + i1] = v;
          }
    }
    __syncthreads();
    plane_fft(a, g, lds, -1);
    float2* zo = a.Z + ((size_t)j * g.n2 + i2) * a.L;
    for (int l = threadIdx.x; l < a.L; l += PT) {
      const int q = a.pos[l];
      const int k0 = q / g.n1, k1 = q - k0 * g.n1;
      float2 v = lds[k0 * g.PS + k1];
      if ((k0 + k1) & 1) v = make_float2(-v.x, -v.y);
      zo[l] = v;
    }
    __syncthreads();
  }
}

template <int PREC, int N0, int N1>
__global__ __launch_bounds__(PT) void plane_adj_kernel(PlaneArgs a) {
  __shared__ float2 lds[LDS_ELEMS];
  const Geo<N0, N1> g(a);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ngrp = (a.J + a.G - 1) / a.G;
  const int i2 = blockIdx.x / ngrp, grp = blockIdx.x % ngrp;
  const int nbl = g.n1 / 16;
  const float2* xp = a.xt + (size_t)i2 * g.n0 * g.n1;
  const bool want_gx = a.gxpart != nullptr;
  f32x4 gr[8], gi[8];
#pragma unroll
  for (int nb = 0; nb < 8; ++nb) { gr[nb] = z4(); gi[nb] = z4(); }
  for (int j = grp * a.G; j < a.J && j < (grp + 1) * a.G; ++j) {
    f32x4 pr[8], pi[8];
    if (want_gx) coil_map<PREC>(a, g, j, i2, lds, pr, pi);  // B c recomputed
    // zero-filled scatter of this plane's samples (with the chessboard sign)
    load_twiddles(a, g, lds);
    for (int e = threadIdx.x; e < g.n0 * g.PS; e += PT) lds[e] = make_float2(0.f, 0.f);
    __syncthreads();
    const float2* zi = a.Z + ((size_t)j * g.n2 + i2) * a.L;
    for (int l = threadIdx.x; l < a.L; l += PT) {
      const int q = a.pos[l];
      const int k0 = q / g.n1, k1 = q - k0 * g.n1;
      float2 v = zi[l];
      if ((k0 + k1) & 1) v = make_float2(-v.x, -v.y);
      lds[k0 * g.PS + k1] = v;
    }
    __syncthreads();
    plane_fft(a, g, lds, +1);
    // g (output chessboard sign); gx += conj(P) g; h = conj(x) g back into the plane
    if (wave < g.n0 / 16) {
#pragma unroll
      for (int nb = 0; nb < 8; ++nb)
        if (nb < nbl)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i0 = 16 * wave + 4 * (lane >> 4) + r, i1 = 16 * nb + (lane & 15);
            float2 gv = lds[i0 * g.PS + i1];
            if ((i0 + i1) & 1) gv = make_float2(-gv.x, -gv.y);
            if (want_gx) {
              const float2 c = cmulc(make_float2(pr[nb][r], pi[nb][r]), gv);
              gr[nb][r] += c.x;
              gi[nb][r] += c.y;
            }
            lds[i0 * g.PS + i1] = cmulc(xp[i0 * g.n1 + i1], gv);
          }
    }
    __syncthreads();
    if (a.T3b) {
      if constexpr (PREC == 1)
        adjoint_W_bf(a, g, j, i2, lds);
      else
        adjoint_W_f32(a, g, j, i2, lds);
    }
    __syncthreads();
  }
  if (want_gx && wave < g.n0 / 16) {
    float2* gxp = a.gxpart + ((size_t)grp * g.n2 + i2) * g.n0 * g.n1;
#pragma unroll
    for (int nb = 0; nb < 8; ++nb)
      if (nb < nbl)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i0 = 16 * wave + 4 * (lane >> 4) + r, i1 = 16 * nb + (lane & 15);
          gxp[i0 * g.n1 + i1] = make_float2(gr[nb][r], gi[nb][r]);
        }
  }
}

// ---------------------------------------------------------------- line kernels
constexpr int LT = 32;     // lines per workgroup
constexpr int LNT = 256;   // threads
constexpr int LMAXN = 256; // max n2 on this path

template <int N2>
__device__ __forceinline__ void line_fft(const LineArgs& a, float2* tile, const float2* tw, int n, int dir) {
  if constexpr (N2 != 0) {
    lds_fft_ct<N2, LNT, LMAXN * LT / 2>(tile, LT, 1, LT + 1, tw, dir);
  } else {
    LdsLines tg{LT, 1, LT + 1};
    lds_fft_lines<LNT, LMAXN * LT / 2>(tile, tg, n, a.rad2, a.nrad2, tw, dir);
  }
}

template <int N2>
__global__ __launch_bounds__(LNT) void line_fwd_kernel(LineArgs a) {
  __shared__ float2 tile[LMAXN * (LT + 1)];
  __shared__ float2 tw[LMAXN];
  __shared__ double red[LNT];
  const int lblocks = (a.L + LT - 1) / LT;
  const int j = blockIdx.x / lblocks, l0 = (blockIdx.x % lblocks) * LT;
  const int n = N2 ? N2 : a.n2, ES = LT + 1;
  for (int e = threadIdx.x; e < n; e += LNT) tw[e] = a.tw2[e];
  for (int e = threadIdx.x; e < n * LT; e += LNT) {
    const int i2 = e / LT, l = e % LT;
    float2 v = make_float2(0.f, 0.f);
    if (l0 + l < a.L) v = a.Z[((size_t)j * n + i2) * a.L + l0 + l];
    if (i2 & 1) v = make_float2(-v.x, -v.y);
    tile[i2 * ES + l] = v;
  }
  __syncthreads();
  line_fft<N2>(a, tile, tw, n, -1);
  double acc = 0.0;
  for (int e = threadIdx.x; e < n * LT; e += LNT) {
    const int l = e / n, k2 = e % n;
    if (l0 + l >= a.L) continue;
    float2 v = tile[k2 * ES + l];
    const float s = (k2 & 1) ? -a.gscale : a.gscale;
    v = cscale(v, s);
    const size_t m = (size_t)(l0 + l) * n + k2;
    const size_t o = (size_t)j * a.M + m;
    if (a.y) {
      const float2 d = csub(v, a.y[o]);
      const float wm = a.w ? a.w[m] : 1.0f;
      acc += (double)wm * ((double)d.x * d.x + (double)d.y * d.y);
      if (a.out) a.out[o] = cscale(d, wm);
    } else {
      a.out[o] = v;
    }
  }
  if (a.part) {
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = LNT / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) a.part[blockIdx.x] = red[0];
  }
}

template <int N2>
__global__ __launch_bounds__(LNT) void line_adj_kernel(LineArgs a) {
  __shared__ float2 tile[LMAXN * (LT + 1)];
  __shared__ float2 tw[LMAXN];
  const int lblocks = (a.L + LT - 1) / LT;
  const int j = blockIdx.x / lblocks, l0 = (blockIdx.x % lblocks) * LT;
  const int n = N2 ? N2 : a.n2, ES = LT + 1;
  for (int e = threadIdx.x; e < n; e += LNT) tw[e] = a.tw2[e];
  for (int e = threadIdx.x; e < n * LT; e += LNT) {
    const int l = e / n, k2 = e % n;
    float2 v = make_float2(0.f, 0.f);
    if (l0 + l < a.L) v = a.yin[(size_t)j * a.M + (size_t)(l0 + l) * n + k2];
    if (k2 & 1) v = make_float2(-v.x, -v.y);
    tile[k2 * ES + l] = v;
  }
  __syncthreads();
  line_fft<N2>(a, tile, tw, n, +1);
  float s = a.gscale * a.alpha;
  if (a.scale_dev) s *= *a.scale_dev;
  for (int e = threadIdx.x; e < n * LT; e += LNT) {
    const int i2 = e / LT, l = e % LT;
    if (l0 + l >= a.L) continue;
    const float2 v = tile[i2 * ES + l];
    a.Zw[((size_t)j * n + i2) * a.L + l0 + l] = cscale(v, (i2 & 1) ? -s : s);
  }
}

// ---------------------------------------------------------------- transposes
constexpr int TT = 32;

// xt[c][r] = x[r][c] for an R x C matrix (complex)
__global__ void transpose_kernel(const float2* __restrict__ x, int64_t R, int64_t C, float2* __restrict__ xt) {
  __shared__ float2 t[TT][TT + 1];
  const int64_t tr = (int64_t)blockIdx.y * TT, tc = (int64_t)blockIdx.x * TT;
  const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
  for (int k = ty; k < TT; k += 256 / TT) {
    const int64_t r = tr + k, c = tc + tx;
    if (r < R && c < C) t[k][tx] = x[r * C + c];
  }
  __syncthreads();
  for (int k = ty; k < TT; k += 256 / TT) {
    const int64_t c = tc + k, r = tr + tx;
    if (r < R && c < C) xt[c * R + r] = t[tx][k];
  }
}

// gx[r][c] = sum_g part[g][c][r] : part is ngrp x (C x R), gx is R x C
__global__ void reduce_transpose_kernel(const float2* __restrict__ part, int ngrp, int64_t R, int64_t C,
                                        float2* __restrict__ gx) {
  __shared__ float2 t[TT][TT + 1];
  const int64_t tr = (int64_t)blockIdx.x * TT, tc = (int64_t)blockIdx.y * TT;
  const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
  for (int k = ty; k < TT; k += 256 / TT) {
    const int64_t c = tc + k, r = tr + tx;
    float2 s = make_float2(0.f, 0.f);
    if (r < R && c < C)
      for (int g = 0; g < ngrp; ++g) s = cadd(s, part[((size_t)g * C + c) * R + r]);
    t[k][tx] = s;
  }
  __syncthreads();
  for (int k = ty; k < TT; k += 256 / TT) {
    const int64_t r = tr + k, c = tc + tx;
    if (r < R && c < C) gx[r * C + c] = t[tx][k];
  }
}

// Plan-time split of a complex matrix into the real-block operand planes.
//   mode 0 (A operand): dst[m][k'] = (Re, Im) of src(m, k) at k' = 2k, 2k+1; planes hi, lo
//   mode 1 (B operand): br[n][k'] = (Re, -Im), bi[n][k'] = (Im, Re) of src(n, k); planes
//                       br hi, br lo, bi hi, bi lo
// src(m, k) = src[m * sm + k * sk], optionally conjugated; zero beyond (rows, cols).
__global__ void split_operand_kernel(const float2* __restrict__ src, int rows, int cols, int64_t sm, int64_t sk,
                                     int conj, int mode, int rows_pad, int kp, unsigned short* __restrict__ dst) {
  const int64_t total = (int64_t)rows_pad * kp;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int m = (int)(e / kp), kq = (int)(e % kp), k = kq / 2, c = kq & 1;
    float2 v = make_float2(0.f, 0.f);
    if (m < rows && k < cols) v = src[(int64_t)m * sm + (int64_t)k * sk];
    if (conj) v.y = -v.y;
    if (mode == 0) {
      const float f = c ? v.y : v.x;
      const unsigned short h = bf16_rne(f);
      dst[e] = h;
      dst[total + e] = bf16_rne(f - bf16_f32(h));
    } else {
      const float fr = c ? -v.y : v.x, fi = c ? v.x : v.y;
      const unsigned short hr = bf16_rne(fr), hi = bf16_rne(fi);
      dst[e] = hr;
      dst[total + e] = bf16_rne(fr - bf16_f32(hr));
      dst[2 * total + e] = hi;
      dst[3 * total + e] = bf16_rne(fi - bf16_f32(hi));
    }
  }
}

template <int PREC>
hipError_t plane_launch_prec(const PlaneArgs& a, bool adj, hipStream_t st) {
  const int ngrp = (a.J + a.G - 1) / a.G;
  const dim3 grid((unsigned)(a.n2 * ngrp)), block(PT);
  if (a.n0 == 128 && a.n1 == 128) {
    if (adj) hipLaunchKernelGGL((plane_adj_kernel<PREC, 128, 128>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((plane_fwd_kernel<PREC, 128, 128>), grid, block, 0, st, a);
  } else if (a.n0 == 64 && a.n1 == 64) {
    if (adj) hipLaunchKernelGGL((plane_adj_kernel<PREC, 64, 64>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((plane_fwd_kernel<PREC, 64, 64>), grid, block, 0, st, a);
  } else {
    if (adj) hipLaunchKernelGGL((plane_adj_kernel<PREC, 0, 0>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((plane_fwd_kernel<PREC, 0, 0>), grid, block, 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t plane_fwd_launch(const PlaneArgs& a, hipStream_t st) {
  return a.precision == 1 ? plane_launch_prec<1>(a, false, st) : plane_launch_prec<0>(a, false, st);
}

hipError_t plane_adj_launch(const PlaneArgs& a, hipStream_t st) {
  return a.precision == 1 ? plane_launch_prec<1>(a, true, st) : plane_launch_prec<0>(a, true, st);
}

int line_blocks(int J, int64_t L) { return (int)(J * ((L + LT - 1) / LT)); }

hipError_t line_fwd_launch(const LineArgs& a, hipStream_t st) {
  const dim3 grid((unsigned)line_blocks(a.J, a.L)), block(LNT);
  if (a.n2 == 128) hipLaunchKernelGGL(line_fwd_kernel<128>, grid, block, 0, st, a);
  else hipLaunchKernelGGL(line_fwd_kernel<0>, grid, block, 0, st, a);
  return hipGetLastError();
}

hipError_t line_adj_launch(const LineArgs& a, hipStream_t st) {
  const dim3 grid((unsigned)line_blocks(a.J, a.L)), block(LNT);
  if (a.n2 == 128) hipLaunchKernelGGL(line_adj_kernel<128>, grid, block, 0, st, a);
  else hipLaunchKernelGGL(line_adj_kernel<0>, grid, block, 0, st, a);
  return hipGetLastError();
}

hipError_t transpose_launch(const float2* x, int64_t R, int64_t C, float2* xt, hipStream_t st) {
  dim3 grid((unsigned)((C + TT - 1) / TT), (unsigned)((R + TT - 1) / TT));
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, st, x, R, C, xt);
  return hipGetLastError();
}

hipError_t reduce_transpose_launch(const float2* part, int ngrp, int64_t R, int64_t C, float2* gx,
                                   hipStream_t st) {
  dim3 grid((unsigned)((R + TT - 1) / TT), (unsigned)((C + TT - 1) / TT));
  hipLaunchKernelGGL(reduce_transpose_kernel, grid, dim3(256), 0, st, part, ngrp, R, C, gx);
  return hipGetLastError();
}

hipError_t split_operand_launch(const float2* src, int rows, int cols, int64_t sm, int64_t sk, int conj, int mode,
                                int rows_pad, int kp, uint16_t* dst, hipStream_t st) {
  int64_t total = (int64_t)rows_pad * kp;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(split_operand_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src, rows, cols, sm, sk, conj,
                     mode, rows_pad, kp, reinterpret_cast<unsigned short*>(dst));
  return hipGetLastError();
}

bool fused_supported(int64_t n0, int64_t n1, int64_t n2, int64_t r0, int64_t r1, int precision) {
  if (!(n0 % 16 == 0 && n1 % 16 == 0 && n0 <= PMAX && n1 <= PMAX && n2 <= LMAXN)) return false;
  if (precision == 1) return r0 <= 48 && r1 <= 48;  // split operands must fit the plane region
  return r0 <= 64 && r1 <= 64;
}

}  // namespace mx
