// Tucker core contractions of the fused path.  The core is the fourth-mode factor of
// the basis (Sec. II-E), so B c_j starts with core x_4 c_j, and the coefficient block
// of the adjoint Jacobian (Sec. II-B) ends with the adjoint of that product:
//
//   forward  T1[j][rho] = sum_k core[rho][k] c[j][k]              rho = (p0, p1, p2)
//   adjoint  gc[j][k]   = s * sum_rho conj(core[rho][k]) T1b[j][rho]
//
// Both stream the core (R x K complex) from HBM once per call, as the matrix-core A
// operand; the small per-call operand (c or T1b) is staged through double-buffered LDS
// shared by the workgroup's four waves.
//
// FP32 kernels: v_mfma_f32_16x16x4_f32, four real products per complex product.
// BF16-split kernels: real-block form over 2K on v_mfma_f32_16x16x32_bf16, six products
// per complex tile (hi*hi, hi*lo, lo*hi for the real and imaginary parts).  The core's
// hi / lo planes are built once per plan in fragment order (row-major for the forward,
// conjugate-transposed for the adjoint); the per-call operand is split while staged.
// The adjoint reduces over rho in chunks whose partials are summed in a fixed order.
#include "../../include/maxwell.h"
#include "core.h"

namespace mx {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int NT = 256;     // four waves
constexpr int MAXNB = 4;    // coil blocks of 16: J <= 64
constexpr int RB = 2;       // row blocks of 16 per wave
constexpr int RC = 512;     // adjoint: rho per workgroup chunk
constexpr int SLB = 40;     // staged bf16 row: 32 k' + 8 pad

__device__ __forceinline__ f32x4 z4() { return f32x4{0.f, 0.f, 0.f, 0.f}; }

__device__ __forceinline__ void cmfma(f32x4& cr, f32x4& ci, float2 a, float2 b) {
  cr = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, cr, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, b.y, cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.y, ci, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.x, ci, 0, 0, 0);
}

__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_f32(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }
__device__ __forceinline__ bf16x8 asbf(u16x8 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ __forceinline__ u16x8 ld8(const unsigned short* p) { return *reinterpret_cast<const u16x8*>(p); }
__device__ __forceinline__ void st8(unsigned short* p, u16x8 v) { *reinterpret_cast<u16x8*>(p) = v; }
__device__ __forceinline__ u16x8 zero8() { return u16x8{0, 0, 0, 0, 0, 0, 0, 0}; }

__device__ __forceinline__ void mfma6(f32x4& cr, f32x4& ci, u16x8 ah, u16x8 al, u16x8 brh, u16x8 brl, u16x8 bih,
                                      u16x8 bil) {
  cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(asbf(ah), asbf(brh), cr, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(asbf(ah), asbf(brl), cr, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(asbf(al), asbf(brh), cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(asbf(ah), asbf(bih), ci, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(asbf(ah), asbf(bil), ci, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(asbf(al), asbf(bih), ci, 0, 0, 0);
}

// Real-block B operand of four consecutive complex reduction entries b[t]:
// br = (Re b, -Im b), bi = (Im b, Re b), each split into hi / lo.
__device__ __forceinline__ void split_b4(const float2 (&v)[4], u16x8& brh, u16x8& brl, u16x8& bih, u16x8& bil) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const float q[4] = {v[t].x, -v[t].y, v[t].y, v[t].x};
    unsigned short h[4], l[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      h[u] = bf16_rne(q[u]);
      l[u] = bf16_rne(q[u] - bf16_f32(h[u]));
    }
    brh[2 * t] = h[0]; brh[2 * t + 1] = h[1];
    brl[2 * t] = l[0]; brl[2 * t + 1] = l[1];
    bih[2 * t] = h[2]; bih[2 * t + 1] = h[3];
    bil[2 * t] = l[2]; bil[2 * t + 1] = l[3];
  }
}

// Stages 16 complex reduction entries (one 32-wide k' step) of the J rows of `src`
// (row stride ld, entries [e0, e0 + 16) clipped at len) into the four planes of sb.
__device__ __forceinline__ void stage_split(unsigned short (*sb)[MAXNB * 16][SLB], const float2* __restrict__ src,
                                            int J, int Jp, int64_t ld, int64_t e0, int64_t len) {
  for (int e = threadIdx.x; e < Jp * 4; e += NT) {
    const int j = e >> 2, q = e & 3;
    float2 v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t k = e0 + 4 * q + t;
      v[t] = (j < J && k < len) ? src[(int64_t)j * ld + k] : make_float2(0.f, 0.f);
    }
    u16x8 brh, brl, bih, bil;
    split_b4(v, brh, brl, bih, bil);
    st8(&sb[0][j][8 * q], brh);
    st8(&sb[1][j][8 * q], brl);
    st8(&sb[2][j][8 * q], bih);
    st8(&sb[3][j][8 * q], bil);
  }
}

// ---------------------------------------------------------------- forward, BF16-split
// Workgroup: 8 row blocks (128 rho), all coils.
__global__ __launch_bounds__(NT) void core_fwd_bf16_kernel(CoreArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned short sb[2][4][MAXNB * 16][SLB];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nb = (a.J + 15) / 16, Jp = nb * 16;
  const int steps = a.g.KP / 32;
  const int64_t rbs = (a.g.R + 15) / 16;
  const int64_t rb0 = (int64_t)blockIdx.x * (4 * RB) + wave * RB;
  auto loadA = [&](int s, u16x8 (&ah)[RB], u16x8 (&al)[RB]) {
#pragma unroll
    for (int m = 0; m < RB; ++m) {
      if (rb0 + m < rbs) {
        const int64_t o = ((rb0 + m) * steps + s) * 512 + lane * 8;
        ah[m] = ld8(a.fwd_hi + o);
        al[m] = ld8(a.fwd_lo + o);
      } else {
        ah[m] = zero8();
        al[m] = zero8();
      }
    }
  };
  f32x4 cr[RB][MAXNB], ci[RB][MAXNB];
#pragma unroll
  for (int m = 0; m < RB; ++m)
#pragma unroll
    for (int c = 0; c < MAXNB; ++c) { cr[m][c] = z4(); ci[m][c] = z4(); }
  u16x8 ah[RB], al[RB], nh[RB], nl[RB];
  stage_split(sb[0], a.in, a.J, Jp, a.g.K, 0, a.g.K);
  loadA(0, ah, al);
  __syncthreads();
  for (int s = 0; s < steps; ++s) {
    if (s + 1 < steps) {
      stage_split(sb[(s + 1) & 1], a.in, a.J, Jp, a.g.K, 16 * (int64_t)(s + 1), a.g.K);
      loadA(s + 1, nh, nl);
    }
    const int buf = s & 1;
#pragma unroll
    for (int c = 0; c < MAXNB; ++c) {
      if (c < nb) {
        const int n = 16 * c + (lane & 15), ko = 8 * (lane >> 4);
        const u16x8 b0 = ld8(&sb[buf][0][n][ko]), b1 = ld8(&sb[buf][1][n][ko]);
        const u16x8 b2 = ld8(&sb[buf][2][n][ko]), b3 = ld8(&sb[buf][3][n][ko]);
#pragma unroll
        for (int m = 0; m < RB; ++m) mfma6(cr[m][c], ci[m][c], ah[m], al[m], b0, b1, b2, b3);
      }
    }
    __syncthreads();
    if (s + 1 < steps) {
#pragma unroll
      for (int m = 0; m < RB; ++m) { ah[m] = nh[m]; al[m] = nl[m]; }
    }
  }
  // D rows are rho, columns coils: T1[j][rho]
#pragma unroll
  for (int m = 0; m < RB; ++m)
#pragma unroll
    for (int c = 0; c < MAXNB; ++c)
      if (c < nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = 16 * (rb0 + m) + 4 * (lane >> 4) + r;
          const int j = 16 * c + (lane & 15);
          if (row < a.g.R && j < a.J) a.out[(int64_t)j * a.g.R + row] = make_float2(cr[m][c][r], ci[m][c][r]);
        }
}

// ---------------------------------------------------------------- forward, FP32
constexpr int KC = 64;  // complex k per staged chunk

__global__ __launch_bounds__(NT) void core_fwd_f32_kernel(CoreArgs a) {
  __shared__ float2 sc[2][MAXNB * 16][KC + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nb = (a.J + 15) / 16, Jp = nb * 16;
  const int K = a.g.K;
  const int64_t R = a.g.R;
  const int64_t row0 = (int64_t)blockIdx.x * (64 * RB) + wave * (16 * RB);
  const int chunks = (K + KC - 1) / KC;
  auto stage = [&](int ch, int buf) {
    for (int e = threadIdx.x; e < Jp * KC; e += NT) {
      const int j = e / KC, k = e % KC, kk = ch * KC + k;
      sc[buf][j][k] = (j < a.J && kk < K) ? a.in[(int64_t)j * K + kk] : make_float2(0.f, 0.f);
    }
  };
  f32x4 cr[RB][MAXNB], ci[RB][MAXNB];
#pragma unroll
  for (int m = 0; m < RB; ++m)
#pragma unroll
    for (int c = 0; c < MAXNB; ++c) { cr[m][c] = z4(); ci[m][c] = z4(); }
  stage(0, 0);
  __syncthreads();
  for (int ch = 0; ch < chunks; ++ch) {
    if (ch + 1 < chunks) stage(ch + 1, (ch + 1) & 1);
    const int buf = ch & 1;
    for (int k4 = 0; k4 < KC; k4 += 4) {
      const int kl = k4 + (lane >> 4), kg = ch * KC + kl;
      float2 av[RB];
#pragma unroll
      for (int m = 0; m < RB; ++m) {
        const int64_t row = row0 + 16 * m + (lane & 15);
        av[m] = (row < R && kg < K) ? a.core[row * K + kg] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int c = 0; c < MAXNB; ++c)
        if (c < nb) {
          const float2 bv = sc[buf][16 * c + (lane & 15)][kl];
#pragma unroll
          for (int m = 0; m < RB; ++m) cmfma(cr[m][c], ci[m][c], av[m], bv);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < RB; ++m)
#pragma unroll
    for (int c = 0; c < MAXNB; ++c)
      if (c < nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = row0 + 16 * m + 4 * (lane >> 4) + r;
          const int j = 16 * c + (lane & 15);
          if (row < R && j < a.J) a.out[(int64_t)j * R + row] = make_float2(cr[m][c][r], ci[m][c][r]);
        }
}

// ---------------------------------------------------------------- adjoint, BF16-split
// Grid (rho chunks, k groups of 8 row blocks).  D rows are k, columns coils.
__global__ __launch_bounds__(NT) void core_adj_bf16_kernel(CoreArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned short sb[2][4][MAXNB * 16][SLB];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nb = (a.J + 15) / 16, Jp = nb * 16;
  const int mbl = a.g.Kp / 16;
  const int mb0 = blockIdx.y * (4 * RB) + wave * RB;
  const int64_t rho0 = (int64_t)blockIdx.x * RC;
  const int64_t steps_total = a.g.Rp / 16;
  const int64_t sg0 = rho0 / 16;
  constexpr int steps = RC / 16;
  auto loadA = [&](int s, u16x8 (&ah)[RB], u16x8 (&al)[RB]) {
#pragma unroll
    for (int m = 0; m < RB; ++m) {
      if (mb0 + m < mbl) {
        const int64_t o = ((int64_t)(mb0 + m) * steps_total + sg0 + s) * 512 + lane * 8;
        ah[m] = ld8(a.adj_hi + o);
        al[m] = ld8(a.adj_lo + o);
      } else {
        ah[m] = zero8();
        al[m] = zero8();
      }
    }
  };
  f32x4 cr[RB][MAXNB], ci[RB][MAXNB];
#pragma unroll
  for (int m = 0; m < RB; ++m)
#pragma unroll
    for (int c = 0; c < MAXNB; ++c) { cr[m][c] = z4(); ci[m][c] = z4(); }
  u16x8 ah[RB], al[RB], nh[RB], nl[RB];
  stage_split(sb[0], a.in, a.J, Jp, a.g.R, rho0, a.g.R);
  loadA(0, ah, al);
  __syncthreads();
  for (int s = 0; s < steps; ++s) {
    if (s + 1 < steps) {
      stage_split(sb[(s + 1) & 1], a.in, a.J, Jp, a.g.R, rho0 + 16 * (s + 1), a.g.R);
      loadA(s + 1, nh, nl);
    }
    const int buf = s & 1;
#pragma unroll
    for (int c = 0; c < MAXNB; ++c) {
      if (c < nb) {
        const int n = 16 * c + (lane & 15), ko = 8 * (lane >> 4);
        const u16x8 b0 = ld8(&sb[buf][0][n][ko]), b1 = ld8(&sb[buf][1][n][ko]);
        const u16x8 b2 = ld8(&sb[buf][2][n][ko]), b3 = ld8(&sb[buf][3][n][ko]);
#pragma unroll
        for (int m = 0; m < RB; ++m) mfma6(cr[m][c], ci[m][c], ah[m], al[m], b0, b1, b2, b3);
      }
    }
    __syncthreads();
    if (s + 1 < steps) {
#pragma unroll
      for (int m = 0; m < RB; ++m) { ah[m] = nh[m]; al[m] = nl[m]; }
    }
  }
  float2* part = a.part + (int64_t)blockIdx.x * a.g.Kp * Jp;
#pragma unroll
  for (int m = 0; m < RB; ++m)
    if (mb0 + m < mbl)
#pragma unroll
      for (int c = 0; c < MAXNB; ++c)
        if (c < nb)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            part[(int64_t)(16 * (mb0 + m) + 4 * (lane >> 4) + r) * Jp + 16 * c + (lane & 15)] =
                make_float2(cr[m][c][r], ci[m][c][r]);
}

// ---------------------------------------------------------------- adjoint, FP32
constexpr int RCH = 64;  // rho per staged chunk

__global__ __launch_bounds__(NT) void core_adj_f32_kernel(CoreArgs a) {
  __shared__ float2 sc[2][MAXNB * 16][RCH + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nb = (a.J + 15) / 16, Jp = nb * 16;
  const int K = a.g.K;
  const int64_t R = a.g.R;
  const int mbl = a.g.Kp / 16;
  const int mb0 = blockIdx.y * (4 * RB) + wave * RB;
  const int64_t rho0 = (int64_t)blockIdx.x * RC;
  auto stage = [&](int ch, int buf) {
    for (int e = threadIdx.x; e < Jp * RCH; e += NT) {
      const int j = e / RCH, t = e % RCH;
      const int64_t rho = rho0 + ch * RCH + t;
      sc[buf][j][t] = (j < a.J && rho < R) ? a.in[(int64_t)j * R + rho] : make_float2(0.f, 0.f);
    }
  };
  f32x4 cr[RB][MAXNB], ci[RB][MAXNB];
#pragma unroll
  for (int m = 0; m < RB; ++m)
#pragma unroll
    for (int c = 0; c < MAXNB; ++c) { cr[m][c] = z4(); ci[m][c] = z4(); }
  stage(0, 0);
  __syncthreads();
  constexpr int chunks = RC / RCH;
  for (int ch = 0; ch < chunks; ++ch) {
    if (ch + 1 < chunks) stage(ch + 1, (ch + 1) & 1);
    const int buf = ch & 1;
    for (int k4 = 0; k4 < RCH; k4 += 4) {
      const int tl = k4 + (lane >> 4);
      const int64_t rho = rho0 + ch * RCH + tl;
      float2 bv[MAXNB];
#pragma unroll
      for (int c = 0; c < MAXNB; ++c) bv[c] = c < nb ? sc[buf][16 * c + (lane & 15)][tl] : make_float2(0.f, 0.f);
#pragma unroll
      for (int m = 0; m < RB; ++m) {
        const int k = 16 * (mb0 + m) + (lane & 15);
        const float2 av = (rho < R && k < K) ? cconj(a.core[rho * K + k]) : make_float2(0.f, 0.f);
#pragma unroll
        for (int c = 0; c < MAXNB; ++c)
          if (c < nb) cmfma(cr[m][c], ci[m][c], av, bv[c]);
      }
    }
    __syncthreads();
  }
  float2* part = a.part + (int64_t)blockIdx.x * a.g.Kp * Jp;
#pragma unroll
  for (int m = 0; m < RB; ++m)
    if (mb0 + m < mbl)
#pragma unroll
      for (int c = 0; c < MAXNB; ++c)
        if (c < nb)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            part[(int64_t)(16 * (mb0 + m) + 4 * (lane >> 4) + r) * Jp + 16 * c + (lane & 15)] =
                make_float2(cr[m][c][r], ci[m][c][r]);
}

// gc[j][k] = s * sum over chunks of part[chunk][k][j], in a fixed order: each workgroup
// owns 32 consecutive (k, j) entries; its 8 slices sum interleaved chunks, then slice
// sums are added in slice order.
constexpr int RED_OUT = 32, RED_SL = 8;

__global__ __launch_bounds__(RED_OUT * RED_SL) void core_adj_reduce_kernel(CoreArgs a, int nch, float alpha,
                                                                           const float* __restrict__ scale_dev) {
  __shared__ float2 acc_s[RED_SL][RED_OUT];
  const int Jp = (a.J + 15) / 16 * 16;
  const int o = threadIdx.x % RED_OUT, sl = threadIdx.x / RED_OUT;
  const int64_t e = (int64_t)blockIdx.x * RED_OUT + o;      // over Kp * Jp
  const int64_t plane = (int64_t)a.g.Kp * Jp;
  float2 acc = make_float2(0.f, 0.f);
  if (e < plane)
    for (int c = sl; c < nch; c += RED_SL) acc = cadd(acc, a.part[(int64_t)c * plane + e]);
  acc_s[sl][o] = acc;
  __syncthreads();
  if (sl == 0 && e < plane) {
    float2 t = acc_s[0][o];
#pragma unroll
    for (int q = 1; q < RED_SL; ++q) t = cadd(t, acc_s[q][o]);
    const int k = (int)(e / Jp), j = (int)(e % Jp);
    float s = alpha;
    if (scale_dev) s *= *scale_dev;
    if (k < a.g.K && j < a.J) a.out[(int64_t)j * a.g.K + k] = cscale(t, s);
  }
}

// Fragment-order planes: entry e of a plane with `steps` k' steps per row block holds
// A(16 rb + lane % 16, 32 s + 8 (lane / 16) + el) for e = ((rb steps + s) 64 + lane) 8 + el.
// mode 0: A(rho, 2k + c) = (Re, Im) core[rho][k];  mode 1: A(k, 2 rho + c) = (Re, -Im) core[rho][k].
__global__ void core_split_kernel(const float2* __restrict__ core, int64_t R, int K, int mode, int64_t nrb,
                                  int64_t steps, unsigned short* __restrict__ hi, unsigned short* __restrict__ lo) {
  const int64_t total = nrb * steps * 512;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t rb = e / (steps * 512), s = (e / 512) % steps;
    const int lane = (int)((e / 8) % 64), el = (int)(e % 8);
    const int64_t row = 16 * rb + lane % 16, kq = 32 * s + 8 * (lane / 16) + el;
    float f = 0.f;
    if (mode == 0) {
      const int64_t k = kq / 2;
      if (row < R && k < K) {
        const float2 v = core[row * K + k];
        f = (kq & 1) ? v.y : v.x;
      }
    } else {
      const int64_t rho = kq / 2;
      if (row < K && rho < R) {
        const float2 v = core[rho * K + row];
        f = (kq & 1) ? -v.y : v.x;
      }
    }
    const unsigned short h = bf16_rne(f);
    hi[e] = h;
    lo[e] = bf16_rne(f - bf16_f32(h));
  }
}

}  // namespace

CoreGeom core_geom(int64_t R, int K) {
  CoreGeom g;
  g.R = R;
  g.K = K;
  g.Rp = (R + RC - 1) / RC * RC;
  g.KP = (2 * K + 31) / 32 * 32;
  g.Kp = (K + 15) / 16 * 16;
  return g;
}

bool core_supported(int J) { return J >= 1 && J <= MAXNB * 16; }

int core_adj_chunks(int64_t R) { return (int)((R + RC - 1) / RC); }

size_t core_adj_part_bytes(int64_t R, int K, int J) {
  const CoreGeom g = core_geom(R, K);
  return (size_t)core_adj_chunks(R) * g.Kp * ((J + 15) / 16 * 16) * sizeof(float2);
}

hipError_t core_split_launch(const float2* core, const CoreGeom& g, uint16_t* dst, hipStream_t st) {
  unsigned short* p = reinterpret_cast<unsigned short*>(dst);
  const size_t nf = g.fwd_elems(), na = g.adj_elems();
  hipLaunchKernelGGL(core_split_kernel, dim3(4096), dim3(256), 0, st, core, g.R, g.K, 0, (g.R + 15) / 16,
                     (int64_t)g.KP / 32, p, p + nf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(core_split_kernel, dim3(4096), dim3(256), 0, st, core, g.R, g.K, 1, (int64_t)g.Kp / 16,
                     g.Rp / 16, p + 2 * nf, p + 2 * nf + na);
  return hipGetLastError();
}

hipError_t core_fwd_launch(const CoreArgs& a, int precision, hipStream_t st) {
  const dim3 grid((unsigned)((a.g.R + 64 * RB - 1) / (64 * RB))), block(NT);
  if (precision == MAXWELL_BF16_SPLIT) hipLaunchKernelGGL(core_fwd_bf16_kernel, grid, block, 0, st, a);
  else hipLaunchKernelGGL(core_fwd_f32_kernel, grid, block, 0, st, a);
  return hipGetLastError();
}

hipError_t core_adj_launch(const CoreArgs& a, int precision, float alpha, const float* scale_dev, hipStream_t st) {
  const int nch = core_adj_chunks(a.g.R);
  const int kgroups = (a.g.Kp / 16 + 4 * RB - 1) / (4 * RB);
  const dim3 grid((unsigned)nch, (unsigned)kgroups), block(NT);
  if (precision == MAXWELL_BF16_SPLIT) hipLaunchKernelGGL(core_adj_bf16_kernel, grid, block, 0, st, a);
  else hipLaunchKernelGGL(core_adj_f32_kernel, grid, block, 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t plane = (int64_t)a.g.Kp * ((a.J + 15) / 16 * 16);
  hipLaunchKernelGGL(core_adj_reduce_kernel, dim3((unsigned)((plane + RED_OUT - 1) / RED_OUT)),
                     dim3(RED_OUT * RED_SL), 0, st, a, nch, alpha, scale_dev);
  return hipGetLastError();
}

}  // namespace mx
