// Device-side building blocks of the LDS-staged FFT (radix 2, 3, 4, 5, 8
// butterflies and one self-sorting Stockham pass), shared by the per-axis FFT
// kernel and the fused plane kernels.
//
// Each pass of radix R over `T` lines of length n held in LDS: every thread
// loads its butterflies' R inputs (stride n/R), applies the twiddles
// w^(k r) with w = exp(-+2 pi i / (Ns R)) and k = j mod Ns, runs the R-point DFT
// and, after a barrier, stores the outputs at (j div Ns) Ns R + (j mod Ns) + r Ns.
// After all passes the line holds its DFT in natural order (Stockham autosort).
#pragma once

#include "common.h"

namespace mx {

template <int R>
__device__ __forceinline__ void dft_small(float2 (&v)[R], int dir);

template <>
__device__ __forceinline__ void dft_small<2>(float2 (&v)[2], int) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

// a * (-i) for the forward direction (dir = -1), a * (+i) for the inverse.
__device__ __forceinline__ float2 mul_mi(float2 a, int dir) {
  return dir < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

template <>
__device__ __forceinline__ void dft_small<4>(float2 (&v)[4], int dir) {
  float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  float2 t2 = cadd(v[1], v[3]), t3 = mul_mi(csub(v[1], v[3]), dir);
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <>
__device__ __forceinline__ void dft_small<8>(float2 (&v)[8], int dir) {
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  dft_small<4>(e, dir);
  dft_small<4>(o, dir);
  const float h = 0.70710678118654752440f;  // 1/sqrt(2)
  const float hd = dir < 0 ? -h : h;
  // o[k] * exp(dir i pi k / 4)
  float2 o1 = cmul(o[1], make_float2(h, hd));
  float2 o2 = mul_mi(o[2], dir);
  float2 o3 = cmul(o[3], make_float2(-h, hd));
  v[0] = cadd(e[0], o[0]); v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);   v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);   v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);   v[7] = csub(e[3], o3);
}

// 16-point DFT as 4 x 4: DFT4 over n1 for each n2 (n = 4 n1 + n2), twiddle
// w16^(n2 k1), DFT4 over n2 for each k1; output index k = k1 + 4 k2.
template <>
__device__ __forceinline__ void dft_small<16>(float2 (&v)[16], int dir) {
  float2 a[4][4];  // a[n2][k1]
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    float2 t[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
    dft_small<4>(t, dir);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) a[n2][k1] = t[k1];
  }
  const float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;  // cos, sin of pi/8
  const float h = 0.70710678118654752440f;
  const float sg = dir < 0 ? -1.f : 1.f;
  // w16^m = (cos(2 pi m/16), sg * sin(2 pi m/16)) for m = n2 * k1
  a[1][1] = cmul(a[1][1], make_float2(c1, sg * s1));
  a[1][2] = cmul(a[1][2], make_float2(h, sg * h));
  a[1][3] = cmul(a[1][3], make_float2(s1, sg * c1));
  a[2][1] = cmul(a[2][1], make_float2(h, sg * h));
  a[2][2] = mul_mi(a[2][2], dir);
  a[2][3] = cmul(a[2][3], make_float2(-h, sg * h));
  a[3][1] = cmul(a[3][1], make_float2(s1, sg * c1));
  a[3][2] = cmul(a[3][2], make_float2(-h, sg * h));
  a[3][3] = cmul(a[3][3], make_float2(-c1, -sg * s1));
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 t[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
    dft_small<4>(t, dir);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
  }
}

template <>
__device__ __forceinline__ void dft_small<3>(float2 (&v)[3], int dir) {
  const float s = 0.86602540378443864676f;  // sin(2 pi / 3)
  float2 t1 = cadd(v[1], v[2]);
  float2 t2 = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
  float2 rd = mul_mi(cscale(csub(v[1], v[2]), s), dir);
  v[0] = cadd(v[0], t1);
  v[1] = cadd(t2, rd);
  v[2] = csub(t2, rd);
}

template <>
__device__ __forceinline__ void dft_small<5>(float2 (&v)[5], int dir) {
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

// Division of x < 2^31 by a divisor 1 <= d < 2^20 known only at run time, as a
// multiply-high, an add and a shift (Granlund and Montgomery, "Division by invariant
// integers using multiplication", 1994): with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1, x / d = (umulhi(x, m) + x) >> l.  The quotient
// for m is taken in FP64, exact here: the numerator is below 2^53 and a fractional
// part, at least 1/d, stays clear of the rounding error.
struct FastDiv {
  uint32_t d, m, l;
};
__host__ __device__ inline FastDiv fast_div(uint32_t d) {
  const uint32_t l = d > 1 ? 32u - (uint32_t)__builtin_clz(d - 1) : 0u;
  const double q = 4294967296.0 * (double)((1ull << l) - d) / (double)d;
  return {d, (uint32_t)q + 1u, l};
}
__device__ __forceinline__ uint32_t fdiv(uint32_t x, const FastDiv& f) { return (__umulhi(x, f.m) + x) >> f.l; }

// Line geometry of a tile held in LDS: element i of line l sits at l*LS + i*ES.
struct LdsLines {
  int T;       // number of lines
  int LS, ES;  // strides of line and element (complex elements)
};

// One Stockham pass of radix R over lines [l0, l0 + Tc) of the tile.  NTHREADS
// threads cooperate; CHUNK bounds Tc*n, so each thread holds at most
// ceil(CHUNK / (R NTHREADS)) butterflies in registers between the two barriers.
// Consecutive threads take consecutive lines.
template <int R, int NTHREADS, int CHUNK>
__device__ __forceinline__ void stockham_pass(float2* lds, const LdsLines& tg, int l0, const FastDiv& fTc, int n,
                                              const FastDiv& fNs, const float2* __restrict__ tw, int dir) {
  constexpr int MAXQ = (CHUNK / R + NTHREADS - 1) / NTHREADS;
  const int Tc = (int)fTc.d, Ns = (int)fNs.d;
  const int nR = n / R;
  const int nb = Tc * nR;
  const int stride_tw = n / (Ns * R);
  float2 v[MAXQ][R];
#pragma unroll
  for (int q = 0; q < MAXQ; ++q) {
    const int bf = threadIdx.x + q * NTHREADS;
    if (bf < nb) {
      const int j = (int)fdiv(bf, fTc);
      const int l = l0 + bf - j * Tc;
      const int base = l * tg.LS;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = lds[base + (j + r * nR) * tg.ES];
      const int k = j - (int)fdiv(j, fNs) * Ns;
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
    const int bf = threadIdx.x + q * NTHREADS;
    if (bf < nb) {
      const int j = (int)fdiv(bf, fTc);
      const int l = l0 + bf - j * Tc;
      const int base = l * tg.LS;
      const int jq = (int)fdiv(j, fNs);
      const int idxD = jq * Ns * R + (j - jq * Ns);
#pragma unroll
      for (int r = 0; r < R; ++r) lds[base + (idxD + r * Ns) * tg.ES] = v[q][r];
    }
  }
  __syncthreads();
}

// All passes of one transform over every line of `tg`, CHUNK elements of lines at
// a time (lines are independent, so a pass may finish one group of lines before
// the next starts).  The caller has synchronised after filling the tile; on
// return the tile is synchronised again.
template <int NTHREADS, int CHUNK>
__device__ __forceinline__ void lds_fft_lines(float2* lds, const LdsLines& tg, int n, const int* radix, int nrad,
                                     const float2* __restrict__ tw, int dir) {
  int Tc = CHUNK / n;
  if (Tc < 1) Tc = 1;
  if (Tc > tg.T) Tc = tg.T;
  const FastDiv fTc = fast_div((uint32_t)Tc);
  const int tail = tg.T % Tc;
  const FastDiv fTail = fast_div((uint32_t)(tail ? tail : 1));
  int Ns = 1;
  for (int p = 0; p < nrad; ++p) {
    const int R = radix[p];
    const FastDiv fNs = fast_div((uint32_t)Ns);
    for (int l0 = 0; l0 < tg.T; l0 += Tc) {
      const FastDiv& ft = (tg.T - l0) < Tc ? fTail : fTc;
      switch (R) {
        case 8: stockham_pass<8, NTHREADS, CHUNK>(lds, tg, l0, ft, n, fNs, tw, dir); break;
        case 4: stockham_pass<4, NTHREADS, CHUNK>(lds, tg, l0, ft, n, fNs, tw, dir); break;
        case 2: stockham_pass<2, NTHREADS, CHUNK>(lds, tg, l0, ft, n, fNs, tw, dir); break;
        case 3: stockham_pass<3, NTHREADS, CHUNK>(lds, tg, l0, ft, n, fNs, tw, dir); break;
        default: stockham_pass<5, NTHREADS, CHUNK>(lds, tg, l0, ft, n, fNs, tw, dir); break;
      }
    }
    Ns *= R;
  }
}


// ---------------------------------------------------------------- compile-time sizes
// Radix plan for the sizes the fused kernels specialise on.
template <int N> struct CtPlan;
template <> struct CtPlan<256> { static constexpr int P = 2, R0 = 16, R1 = 16; };
template <> struct CtPlan<128> { static constexpr int P = 2, R0 = 16, R1 = 8; };
template <> struct CtPlan<64> { static constexpr int P = 2, R0 = 8, R1 = 8; };
template <> struct CtPlan<32> { static constexpr int P = 2, R0 = 8, R1 = 4; };
template <> struct CtPlan<16> { static constexpr int P = 1, R0 = 16, R1 = 1; };

// One Stockham pass with compile-time size, radix and stride.  `tw` holds
// exp(-2 pi i t / N), t < N (in LDS).  T lines, CH elements per register chunk.
// tid is the thread's index in the workgroup (callers may pass it through an opaque
// copy so that the pass's addresses are recomputed where used, not held in registers).
template <int N, int R, int Ns, int NTHREADS, int CH>
__device__ __forceinline__ void stockham_pass_ct(float2* lds, int T, int LS, int ES, const float2* tw, int dir,
                                                 int tid) {
  constexpr int nR = N / R;
  constexpr int Tc = CH / N;
  constexpr int MAXQ = (Tc * nR + NTHREADS - 1) / NTHREADS;
  constexpr int STW = N / (Ns * R);
  for (int l0 = 0; l0 < T; l0 += Tc) {
    float2 v[MAXQ][R];
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int bf = tid + q * NTHREADS;
      const int l = l0 + bf % Tc, j = bf / Tc;
      if (bf < Tc * nR && l < T) {
        const int base = l * LS;
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = lds[base + (j + r * nR) * ES];
        if (Ns > 1) {
          // twiddles w^(k r), r < R, from the table entries for r = 1, 2, 4, 8: each is a
          // product of at most three of them (a few ulp), which saves LDS reads
          const int k = j % Ns;
          float2 wp[4];
#pragma unroll
          for (int b = 0; b < 4; ++b)
            if ((1 << b) < R) {
              wp[b] = tw[k * (1 << b) * STW];
              if (dir > 0) wp[b].y = -wp[b].y;
            }
#pragma unroll
          for (int r = 1; r < R; ++r) {
            float2 w = make_float2(1.f, 0.f);
            bool first = true;
#pragma unroll
            for (int b = 0; b < 4; ++b)
              if (r & (1 << b)) {
                w = first ? wp[b] : cmul(w, wp[b]);
                first = false;
              }
            v[q][r] = cmul(v[q][r], w);
          }
        }
        dft_small<R>(v[q], dir);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int bf = tid + q * NTHREADS;
      const int l = l0 + bf % Tc, j = bf / Tc;
      if (bf < Tc * nR && l < T) {
        const int base = l * LS;
        const int idxD = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
        for (int r = 0; r < R; ++r) lds[base + (idxD + r * Ns) * ES] = v[q][r];
      }
    }
    __syncthreads();
  }
}

// The same pass over the lines one wave owns: in each chunk of Tc = min(CH / N, TL) lines
// (TL: the number of lines, known at compile time here), wave w
// takes lines [w LPW, (w + 1) LPW), LPW = Tc / (NTHREADS / 64), lane -> (line lane % LPW,
// butterfly column lane / LPW + (64 / LPW) q).  A wave's LDS accesses are performed in
// program order, so the pass needs no workgroup barrier; the empty asm statements keep the
// compiler from moving LDS accesses across the read / write phases.  The caller
// synchronises the workgroup before the first pass (other waves' data) and after the last.
template <int N, int R, int Ns, int NTHREADS, int CH, int TL>
__device__ __forceinline__ void stockham_pass_wave(float2* lds, int LS, int ES, const float2* tw, int dir, int tid) {
  constexpr int nR = N / R;
  constexpr int NW = NTHREADS / 64;
  constexpr int T = TL;
  constexpr int Tc = CH / N < TL ? CH / N : TL;
  constexpr int LPW = Tc / NW;
  static_assert(Tc % NW == 0 && T % Tc == 0, "chunks split evenly over the waves");
  static_assert(LPW >= 1 && LPW <= 64 && 64 % LPW == 0, "lines per wave must divide 64");
  constexpr int JG = 64 / LPW;
  constexpr int MAXQ = (nR + JG - 1) / JG;
  constexpr int STW = N / (Ns * R);
  const int wave = tid >> 6, lane = tid & 63;
  const int lo = lane % LPW, jg = lane / LPW;
  for (int l0 = 0; l0 < T; l0 += Tc) {
    const int l = l0 + wave * LPW + lo;
    const int base = l * LS;
    float2 v[MAXQ][R];
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int j = jg + JG * q;
      if (j < nR && l < T) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = lds[base + (j + r * nR) * ES];
        if (Ns > 1) {
          const int k = j % Ns;
          float2 wp[4];
#pragma unroll
          for (int b = 0; b < 4; ++b)
            if ((1 << b) < R) {
              wp[b] = tw[k * (1 << b) * STW];
              if (dir > 0) wp[b].y = -wp[b].y;
            }
#pragma unroll
          for (int r = 1; r < R; ++r) {
            float2 w = make_float2(1.f, 0.f);
            bool first = true;
#pragma unroll
            for (int b = 0; b < 4; ++b)
              if (r & (1 << b)) {
                w = first ? wp[b] : cmul(w, wp[b]);
                first = false;
              }
            v[q][r] = cmul(v[q][r], w);
          }
        }
        dft_small<R>(v[q], dir);
      }
    }
    asm volatile("" ::: "memory");
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int j = jg + JG * q;
      if (j < nR && l < T) {
        const int idxD = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
        for (int r = 0; r < R; ++r) lds[base + (idxD + r * Ns) * ES] = v[q][r];
      }
    }
    asm volatile("" ::: "memory");
  }
}

// The last pass (Ns R = N, so butterfly column j has twiddle index k = j) over wave-owned
// lines, with each lane keeping one column and stepping over lines: lane -> (column
// lane % nR, line lane / nR + (64 / nR) q).  The lane's R - 1 twiddles are read once and serve
// every butterfly it computes, where the general mapping reads or forms them per butterfly.
// A quarter wave touches 16 consecutive columns of one line: conflict-free for unit and for
// odd element strides.
template <int N, int R, int NTHREADS, int CH, int TL, int QB = 0>
__device__ __forceinline__ void stockham_last_pass_wave(float2* lds, int LS, int ES, const float2* tw, int dir,
                                                        int tid) {
  constexpr int nR = N / R;
  constexpr int NW = NTHREADS / 64;
  constexpr int Tc = CH / N < TL ? CH / N : TL;
  constexpr int LPW = Tc / NW;
  constexpr int LG = 64 / nR;  // lines of one q step
  constexpr int MAXQ = LPW / LG;
  static_assert(Tc % NW == 0 && TL % Tc == 0 && 64 % nR == 0 && LPW % LG == 0, "lane mapping");
  const int wave = tid >> 6, lane = tid & 63;
  const int j = lane % nR, lsub = lane / nR;
  float2 w[R];
#pragma unroll
  for (int r = 1; r < R; ++r) {
    w[r] = tw[j * r];  // w^(j r), j r < N
    if (dir > 0) w[r].y = -w[r].y;
  }
  // a butterfly's outputs j + r Ns go where its inputs j + r nR were: each batch of QB line
  // steps is read, transformed and written back before the next (fewer live registers)
  constexpr int B = QB > 0 && QB < MAXQ ? QB : MAXQ;
  static_assert(MAXQ % B == 0, "batches split the line steps evenly");
  for (int l0 = 0; l0 < TL; l0 += Tc) {
#pragma unroll
    for (int q0 = 0; q0 < MAXQ; q0 += B) {
      const int base = (l0 + wave * LPW + lsub + q0 * LG) * LS + j * ES;
      float2 v[B][R];
#pragma unroll
      for (int q = 0; q < B; ++q) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = lds[base + q * LG * LS + r * nR * ES];
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], w[r]);
        dft_small<R>(v[q], dir);
      }
      asm volatile("" ::: "memory");
#pragma unroll
      for (int q = 0; q < B; ++q) {
#pragma unroll
        for (int r = 0; r < R; ++r) lds[base + q * LG * LS + r * nR * ES] = v[q][r];
      }
      asm volatile("" ::: "memory");
    }
  }
}

// Whether wave-owned passes are free of LDS bank conflicts for an odd line stride: a
// quarter wave (16 lanes) then reads 16 different lines at one butterfly column.
template <int N, int NTHREADS, int CH, int TL>
constexpr bool wave_lines_fit() {
  constexpr int n = N > 0 ? N : 1;  // N = 0: a run-time size, never wave-owned
  return N > 0 && (CH / n < TL ? CH / n : TL) / (NTHREADS / 64) >= 16;
}

// All passes of one transform over wave-owned lines (stockham_pass_wave): no workgroup
// barrier inside; the caller synchronises before and after.
template <int N, int NTHREADS, int CH, int TL, int QB = 0>
__device__ __forceinline__ void lds_fft_ct_wave(float2* lds, int LS, int ES, const float2* tw, int dir, int tid) {
  using P = CtPlan<N>;
  stockham_pass_wave<N, P::R0, 1, NTHREADS, CH, TL>(lds, LS, ES, tw, dir, tid);
  if constexpr (P::P > 1) {
    static_assert(P::R0 * P::R1 == N, "two passes: the second is the last");
    stockham_last_pass_wave<N, P::R1, NTHREADS, CH, TL, QB>(lds, LS, ES, tw, dir, tid);
  }
}

template <int N, int NTHREADS, int CH>
__device__ __forceinline__ void lds_fft_ct(float2* lds, int T, int LS, int ES, const float2* tw, int dir,
                                           int tid = -1) {
  using P = CtPlan<N>;
  if (tid < 0) tid = threadIdx.x;
  stockham_pass_ct<N, P::R0, 1, NTHREADS, CH>(lds, T, LS, ES, tw, dir, tid);
  if constexpr (P::P > 1) stockham_pass_ct<N, P::R1, P::R0, NTHREADS, CH>(lds, T, LS, ES, tw, dir, tid);
}

}  // namespace mx
