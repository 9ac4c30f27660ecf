// Matrix-core tiles and fragment-ordered operands shared by the HIP kernels.
//
// Complex products on the matrix cores.  FP32: each complex product is four real
// products on v_mfma_f32_16x16x4_f32 (cmfma), or three in the accumulator form Tile<0>::Acc
// (Re = sum ar br - sum ai bi, Im = sum (ar + ai)(br + bi) - sum ar br - sum ai bi, the
// three-multiplication complex product).  BF16_SPLIT: the complex product over K is
// written as two real products over 2K (real-block form): with a' = (Re a_0, Im a_0,
// Re a_1, ...), Re c = a'.(Re b_0, -Im b_0, ...) and Im c = a'.(Im b_0, Re b_0, ...);
// every real operand is split into hi = bf16(v), lo = bf16(v - hi) and each real
// product is hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16 with FP32 accumulation.
#pragma once

#include "common.h"

namespace mx {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

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

// hi = bf16(v), lo = bf16(v - hi), both rounded to nearest even.  The conversions are the
// hardware's packed FP32 -> BF16 converts (same rounding as bf16_rne for finite values).
__device__ __forceinline__ void split8(const float (&v)[8], u16x8& hi, u16x8& lo) {
  typedef float f32x8 __attribute__((ext_vector_type(8)));
  f32x8 x;
#pragma unroll
  for (int e = 0; e < 8; ++e) x[e] = v[e];
  const bf16x8 h = __builtin_convertvector(x, bf16x8);
  const f32x8 r = x - __builtin_convertvector(h, f32x8);
  hi = __builtin_bit_cast(u16x8, h);
  lo = __builtin_bit_cast(u16x8, __builtin_convertvector(r, bf16x8));
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

// ---------------------------------------------------------------- matrix-core tiles
// A K16 block spans 16 complex reduction indices.  In both precisions lane l (tile row
// or column l % 16, group g = l / 16) holds the operand values of k = 4 g + t, t < 4,
// and an accumulator tile holds D[4 g + r][l % 16].  A result tile is therefore, as it
// stands, the lane's B operand of one K16 block of a following product whose reduction
// runs over the result's rows.
template <int PREC>
struct Tile;

template <>
struct Tile<1> {  // BF16 split in the real-block form
  struct A { u16x8 h, l; };
  struct B { u16x8 rh, rl, ih, il; };
  static __device__ __forceinline__ A make_a(const float2 (&v)[4]) {
    float f[8];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f[2 * t] = v[t].x;
      f[2 * t + 1] = v[t].y;
    }
    A a;
    split8(f, a.h, a.l);
    return a;
  }
  static __device__ __forceinline__ B make_b(const float2 (&v)[4]) {
    float fr[8], fi[8];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      fr[2 * t] = v[t].x;
      fr[2 * t + 1] = -v[t].y;
      fi[2 * t] = v[t].y;
      fi[2 * t + 1] = v[t].x;
    }
    B b;
    split8(fr, b.rh, b.rl);
    split8(fi, b.ih, b.il);
    return b;
  }
  static __device__ __forceinline__ void mma(f32x4& cr, f32x4& ci, const A& a, const B& b) {
    mfma6(cr, ci, a.h, a.l, b.rh, b.rl, b.ih, b.il);
  }
  // accumulator form (the same products here)
  struct Acc { f32x4 r, i; };
  static __device__ __forceinline__ Acc zero() { return Acc{z4(), z4()}; }
  static __device__ __forceinline__ void mma(Acc& c, const A& a, const B& b) { mma(c.r, c.i, a, b); }
  static __device__ __forceinline__ void finish(const Acc& c, f32x4& cr, f32x4& ci) { cr = c.r; ci = c.i; }
};

template <>
struct Tile<0> {  // FP32; sub-step t uses k = 4 g + t (mma: four real products, Acc form: three)
  struct A { float2 v[4]; };
  struct B { float2 v[4]; };
  static __device__ __forceinline__ A make_a(const float2 (&v)[4]) { return A{{v[0], v[1], v[2], v[3]}}; }
  static __device__ __forceinline__ B make_b(const float2 (&v)[4]) { return B{{v[0], v[1], v[2], v[3]}}; }
  static __device__ __forceinline__ void mma(f32x4& cr, f32x4& ci, const A& a, const B& b) {
#pragma unroll
    for (int t = 0; t < 4; ++t) cmfma(cr, ci, a.v[t], b.v[t]);
  }
  // accumulator form: three real products per complex product (p1 = sum ar br,
  // p2 = sum ai bi, p3 = sum (ar + ai)(br + bi)); finish forms Re = p1 - p2, Im = p3 - p1 - p2
  struct Acc { f32x4 p1, p2, p3; };
  static __device__ __forceinline__ Acc zero() { return Acc{z4(), z4(), z4()}; }
  static __device__ __forceinline__ void mma(Acc& c, const A& a, const B& b) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      c.p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[t].x, b.v[t].x, c.p1, 0, 0, 0);
      c.p2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[t].y, b.v[t].y, c.p2, 0, 0, 0);
      c.p3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[t].x + a.v[t].y, b.v[t].x + b.v[t].y, c.p3, 0, 0, 0);
    }
  }
  // sub-steps 0 and 1 only (the caller knows the others hold zeros)
  static __device__ __forceinline__ void mma_half(Acc& c, const A& a, const B& b) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      c.p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[t].x, b.v[t].x, c.p1, 0, 0, 0);
      c.p2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[t].y, b.v[t].y, c.p2, 0, 0, 0);
      c.p3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[t].x + a.v[t].y, b.v[t].x + b.v[t].y, c.p3, 0, 0, 0);
    }
  }
  static __device__ __forceinline__ void finish(const Acc& c, f32x4& cr, f32x4& ci) {
    cr = c.p1 - c.p2;
    ci = c.p3 - c.p1 - c.p2;
  }
};

// ---------------------------------------------------------------- fragment order
// An operand O(o, k) (o: tile row of an A operand or tile column of a B operand, k: the
// reduction index) is kept in fragment order: one (o block, K16 step) fragment is the 64
// lanes' operand registers, stored lane-contiguously, so a wave loads it as one contiguous
// 1 KiB run per array and a fragment store from registers is conflict-free in LDS.
//   A type: [o block][step][hi, lo][lane][8 bf16]             FP32: [o block][step][lane][4 complex]
//   B type: [step][br hi, br lo, bi hi, bi lo][o block][lane][8 bf16]
//                                                             FP32: [step][o block][lane][4 complex]
// One K16 step of a B operand is one contiguous block (it is staged through LDS whole).
constexpr int FRAG_U16 = 512;  // bf16 entries of one array of one fragment

template <int PREC>
__device__ __forceinline__ typename Tile<PREC>::A frag_a(const void* base, int ks, int ob, int s, int lane) {
  const size_t f = (size_t)ob * ks + s;
  if constexpr (PREC == 1) {
    const unsigned short* p = reinterpret_cast<const unsigned short*>(base) + f * 2 * FRAG_U16 + lane * 8;
    return typename Tile<1>::A{ld8(p), ld8(p + FRAG_U16)};
  } else {
    const float4* p = reinterpret_cast<const float4*>(base) + (f * 64 + lane) * 2;
    const float4 u = p[0], w = p[1];
    return typename Tile<0>::A{{make_float2(u.x, u.y), make_float2(u.z, u.w), make_float2(w.x, w.y),
                                make_float2(w.z, w.w)}};
  }
}

template <int PREC>
__device__ __forceinline__ typename Tile<PREC>::B frag_b(const void* base, int obs, int ob, int s, int lane) {
  if constexpr (PREC == 1) {
    const size_t arr = (size_t)obs * FRAG_U16;
    const unsigned short* p =
        reinterpret_cast<const unsigned short*>(base) + (size_t)s * 4 * arr + (size_t)ob * FRAG_U16 + lane * 8;
    return typename Tile<1>::B{ld8(p), ld8(p + arr), ld8(p + 2 * arr), ld8(p + 3 * arr)};
  } else {
    const float4* p = reinterpret_cast<const float4*>(base) + (((size_t)s * obs + ob) * 64 + lane) * 2;
    const float4 u = p[0], w = p[1];
    return typename Tile<0>::B{{make_float2(u.x, u.y), make_float2(u.z, u.w), make_float2(w.x, w.y),
                                make_float2(w.z, w.w)}};
  }
}

// Store a fragment built from four complex values per lane.
template <int PREC>
__device__ __forceinline__ void put_frag_a(void* base, int ks, int ob, int s, int lane, const float2 (&v)[4]) {
  const size_t f = (size_t)ob * ks + s;
  if constexpr (PREC == 1) {
    const typename Tile<1>::A a = Tile<1>::make_a(v);
    unsigned short* p = reinterpret_cast<unsigned short*>(base) + f * 2 * FRAG_U16 + lane * 8;
    st8(p, a.h);
    st8(p + FRAG_U16, a.l);
  } else {
    float4* p = reinterpret_cast<float4*>(base) + (f * 64 + lane) * 2;
    p[0] = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
    p[1] = make_float4(v[2].x, v[2].y, v[3].x, v[3].y);
  }
}

template <int PREC>
__device__ __forceinline__ void put_frag_b(void* base, int obs, int ob, int s, int lane, const float2 (&v)[4]) {
  if constexpr (PREC == 1) {
    const typename Tile<1>::B b = Tile<1>::make_b(v);
    const size_t arr = (size_t)obs * FRAG_U16;
    unsigned short* p = reinterpret_cast<unsigned short*>(base) + (size_t)s * 4 * arr + (size_t)ob * FRAG_U16 + lane * 8;
    st8(p, b.rh);
    st8(p + arr, b.rl);
    st8(p + 2 * arr, b.ih);
    st8(p + 3 * arr, b.il);
  } else {
    float4* p = reinterpret_cast<float4*>(base) + (((size_t)s * obs + ob) * 64 + lane) * 2;
    p[0] = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
    p[1] = make_float4(v[2].x, v[2].y, v[3].x, v[3].y);
  }
}

// An accumulator tile as the lane's B fragment of one K16 step (its rows become k).
template <int PREC>
__device__ __forceinline__ typename Tile<PREC>::B tile_as_b(const f32x4& cr, const f32x4& ci) {
  float2 v[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) v[t] = make_float2(cr[t], ci[t]);
  return Tile<PREC>::make_b(v);
}

// An accumulator tile as the B fragment of step s (its rows become the reduction index).
template <int PREC>
__device__ __forceinline__ void put_tile_b(void* base, int obs, int ob, int s, int lane, const f32x4& cr,
                                           const f32x4& ci) {
  float2 v[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) v[t] = make_float2(cr[t], ci[t]);
  put_frag_b<PREC>(base, obs, ob, s, lane, v);
}

// Bytes of one K16 step of a B-type operand with obs o blocks.
template <int PREC>
__host__ __device__ constexpr int frag_b_step_bytes(int obs) { return obs * (PREC == 1 ? 4 * 1024 : 2048); }

}  // namespace mx
