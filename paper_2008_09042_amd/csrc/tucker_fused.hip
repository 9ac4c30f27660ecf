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
// Matrix-core arithmetic as in mfma_frag.h.  Constant factor operands are put in
// fragment order (and split, in BF16_SPLIT plans) once at plan time; W, V, h and Y
// are split in the kernel.
#include "fft_device.h"
#include "fused.h"
#include "mfma_frag.h"

namespace mx {

namespace {

constexpr int PT = 512;                          // threads per plane workgroup
constexpr int NWAVE = PT / 64;
constexpr int PMAX = 128;                        // max n0, n1 on this path
constexpr int RMAX = 48;                         // max r0, r1 on this path (three K16 blocks)
constexpr int PLANE_ELEMS = PMAX * (PMAX + 1);   // padded plane: 16,512 complex = 132 KB
constexpr int STAGE_OFF = PLANE_ELEMS;           // W of the current coil, or two K16 steps of conj(U1)
constexpr int STAGE_ELEMS = 3072;                // 24 KB
constexpr int TW_OFF = STAGE_OFF + STAGE_ELEMS;  // twiddles of n0 and n1 (2 x PMAX), kept for the workgroup
constexpr int LDS_ELEMS = TW_OFF + 2 * PMAX;
// the adjoint's Wb partials (8 waves x 9 tiles x 256) overwrite the plane and staging regions
static_assert(NWAVE * 9 * 256 <= PLANE_ELEMS + STAGE_ELEMS, "Wb partials must fit");
constexpr int FFT_CHUNK_FWD = PMAX * PMAX;       // elements per register chunk of a transform pass
constexpr int FFT_CHUNK_ADJ = PMAX * PMAX / 2;   // run-time plane sizes in plane_adj_kernel (P and gx held)
constexpr int SCAT = 4;                          // samples per thread loaded ahead of the scatter

// ---------------------------------------------------------------- plane geometry
template <int N0, int N1, int RB>
struct Geo {
  int n0, n1, n2, r0, r1, PS;
  int n0b, n1b, r0b, r1b;  // 16-blocks of each extent
  __device__ Geo(const PlaneArgs& a) {
    n0 = N0 ? N0 : a.n0;
    n1 = N1 ? N1 : a.n1;
    n2 = a.n2;
    r0 = a.r0;
    r1 = a.r1;
    PS = n1 + 1;
    n0b = n0 / 16;
    n1b = n1 / 16;
    r0b = RB ? RB : a.r0p / 16;
    r1b = RB ? RB : a.r1p / 16;
  }
};

// Rank order inside a K16 block of the FP32 rank reductions (V = W U1^T over r1, P = U0 V
// over r0): position 4 g + t (lane group g, sub-step t) holds rank g + 4 t of the block, in
// W, in the U0 / U1^T fragments and, through W's rows, in V.  A last block holding at most
// 8 ranks then has its padding in sub-steps 2 and 3, which rank_mma skips when the kernel is
// built for it (HALF: compile-time rank blocks, both ranks in (32, 40]).  The sum runs over
// the same products; BF16-split plans keep the natural order (one K16 block is one MFMA).
__host__ __device__ constexpr int kperm(int q) { return (q >> 2) | ((q & 3) << 2); }

template <int PREC>
__device__ __forceinline__ void rank_mma(typename Tile<PREC>::Acc& c, const typename Tile<PREC>::A& a,
                                         const typename Tile<PREC>::B& b, bool half) {
  if constexpr (PREC == 0) {
    if (half)
      Tile<0>::mma_half(c, a, b);
    else
      Tile<0>::mma(c, a, b);
  } else {
    Tile<PREC>::mma(c, a, b);
  }
}

// The wave's share of the plane: column block cb and row blocks part, part + q, ...
// (every (row block, column block) tile has exactly one owner).  A whole column block per
// wave lets the wave form its P tiles from its own V tiles (V = W U1^T for that column
// block) held in registers.
struct Share {
  int cb, part, q;
  bool on;
};

template <int N0, int N1, int RB>
__device__ __forceinline__ Share plane_share(const Geo<N0, N1, RB>& g) {
  const int wave = threadIdx.x >> 6;
  Share s;
  s.q = NWAVE / g.n1b;
  s.cb = wave % g.n1b;
  s.part = wave / g.n1b;
  s.on = s.part < s.q;
  return s;
}

// Workgroup -> (plane i2, coil group).  Consecutive workgroups are dispatched to the 8
// XCDs in turn, each with its own L2; the mapping gives every XCD a contiguous range of
// planes, so the groups of one plane share an L2 (and its x plane) while they run.
constexpr int NXCD = 8;

__device__ __forceinline__ void plane_block(int ngrp, int n2, int& i2, int& grp) {
  const int nb = ngrp * n2;
  int l = blockIdx.x;
  if (nb % NXCD == 0) l = (blockIdx.x % NXCD) * (nb / NXCD) + blockIdx.x / NXCD;
  i2 = l / ngrp;
  grp = l % ngrp;
}

template <int N0, int N1, int RB>
__device__ __forceinline__ void load_twiddles(const PlaneArgs& a, const Geo<N0, N1, RB>& g, float2* lds) {
  float2* tw0 = lds + TW_OFF;
  float2* tw1 = tw0 + PMAX;
  for (int e = threadIdx.x; e < g.n0; e += PT) tw0[e] = a.tw0[e];
  for (int e = threadIdx.x; e < g.n1; e += PT) tw1[e] = a.tw1[e];
}

// 2D centred DFT of the plane (chessboard signs applied by the caller); ends synchronised.
// CH elements of a pass are held in registers at a time.
template <int CH, int N0, int N1, int RB, int QB = 0>
__device__ __forceinline__ void plane_fft(const PlaneArgs& a, const Geo<N0, N1, RB>& g, float2* lds, int dir) {
  const float2* tw0 = lds + TW_OFF;
  const float2* tw1 = tw0 + PMAX;
  int tid = threadIdx.x;  // opaque: the passes' addresses are not hoisted out of the coil loop
  asm volatile("" : "+v"(tid));
  // wave-owned lines (no barrier inside the transform of one axis) where a chunk holds at
  // least 16 lines per wave; otherwise every pass synchronises the workgroup
  auto rows = [&]() {
    if constexpr (N1 != 0 && wave_lines_fit<N1, PT, CH, N0>()) {
      lds_fft_ct_wave<N1, PT, CH, N0, QB>(lds, g.PS, 1, tw1, dir, tid);
      __syncthreads();
    } else if constexpr (N1 != 0) {
      lds_fft_ct<N1, PT, CH>(lds, g.n0, g.PS, 1, tw1, dir, tid);
    } else {
      LdsLines t{g.n0, g.PS, 1};
      lds_fft_lines<PT, CH>(lds, t, g.n1, a.rad1, a.nrad1, tw1, dir);
    }
  };
  auto cols = [&]() {
    if constexpr (N0 != 0 && wave_lines_fit<N0, PT, CH, N1>()) {
      lds_fft_ct_wave<N0, PT, CH, N1, QB>(lds, 1, g.PS, tw0, dir, tid);
      __syncthreads();
    } else if constexpr (N0 != 0) {
      lds_fft_ct<N0, PT, CH>(lds, g.n1, 1, g.PS, tw0, dir, tid);
    } else {
      LdsLines t{g.n1, 1, g.PS};
      lds_fft_lines<PT, CH>(lds, t, g.n0, a.rad0, a.nrad0, tw0, dir);
    }
  };
  if (dir < 0) { rows(); cols(); } else { cols(); rows(); }
}

// ---------------------------------------------------------------- coil map
// W = T3[j][i2] (r0 x r1) as the A operand of V = W U1^T: each thread gathers the values
// of at most two fragment lanes into registers (issued early), then stores them split.
// The thread's element offsets in a W slab are the same for every coil: computed once per
// workgroup (-1 for padding entries).
struct WPrefetch {
  float2 v[2][4];
};
struct WSlots {
  unsigned p[4];  // entry (q, t) in bits 16 (t & 1) of p[2 q + t / 2]; 0xffff for padding
};

template <int PREC, int N0, int N1, int RB>
__device__ __forceinline__ WSlots w_slots(const Geo<N0, N1, RB>& g, int tid) {
  WSlots w;
  const int nfl = g.r0b * g.r1b * 64;  // (o block, step, lane) entries
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = tid + q * PT;
    const int f = e / 64, lane = e % 64;
    const int mb = f / g.r1b, s = f % g.r1b;
    const int p0 = 16 * mb + (PREC == 0 ? kperm(lane & 15) : (lane & 15));
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      unsigned pk = 0;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int q1 = 4 * (lane >> 4) + 2 * h + b;
        const int p1 = 16 * s + (PREC == 0 ? kperm(q1) : q1);
        const unsigned o = (e < nfl && p0 < g.r0 && p1 < g.r1) ? (unsigned)(p0 * g.r1 + p1) : 0xffffu;
        pk |= o << (16 * b);
      }
      w.p[2 * q + h] = pk;
    }
  }
  return w;
}

template <int N0, int N1, int RB>
__device__ __forceinline__ void w_load(const PlaneArgs& a, const Geo<N0, N1, RB>& g, int j, int i2, const WSlots& sl,
                                       WPrefetch& w) {
  const float2* src = a.T3 + ((size_t)j * g.n2 + i2) * g.r0 * g.r1;
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      // unconditional loads (an in-range address for the padding entries, zeroed by a
      // multiply, which keeps the compiler from moving the load under a branch): a load
      // under a branch would make every later wait a full drain
      const unsigned o = (sl.p[2 * q + t / 2] >> (16 * (t & 1))) & 0xffffu;
      const bool pad = o == 0xffffu;
      const float2 v = src[pad ? 0u : o];
      const float m = pad ? 0.f : 1.f;
      w.v[q][t] = make_float2(v.x * m, v.y * m);
    }
}

template <int PREC, int N0, int N1, int RB>
__device__ __forceinline__ void w_store(const Geo<N0, N1, RB>& g, float2* lds, int tid, const WPrefetch& w) {
  const int nfl = g.r0b * g.r1b * 64;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = tid + q * PT;
    if (e < nfl) {
      const int f = e / 64, lane = e % 64;
      put_frag_a<PREC>(lds + STAGE_OFF, g.r1b, f / g.r1b, f % g.r1b, lane, w.v[q]);
    }
  }
}

// V[:, cb] = W U1^T[:, cb] (W staged) for the wave's column block, as the B operands (one
// per K16 step over p0) of P = U0 V.  u1: this column block's U1^T fragments.
template <int PREC, bool HALF, int N0, int N1, int RB>
__device__ __forceinline__ void coil_v(const Geo<N0, N1, RB>& g, const float2* lds, int lane,
                                       const typename Tile<PREC>::B (&u1)[3], typename Tile<PREC>::B (&vb)[3]) {
  typename Tile<PREC>::Acc c[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) c[m] = Tile<PREC>::zero();
#pragma unroll
  for (int s = 0; s < 3; ++s)
    if (s < g.r1b) {
#pragma unroll
      for (int m = 0; m < 3; ++m)
        if (m < g.r0b)
          rank_mma<PREC>(c[m], frag_a<PREC>(lds + STAGE_OFF, g.r1b, m, s, lane), u1[s], HALF && s == g.r1b - 1);
    }
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    f32x4 cr, ci;
    Tile<PREC>::finish(c[m], cr, ci);
    vb[m] = tile_as_b<PREC>(cr, ci);
  }
}

// P tiles of the wave's share: P[rb][cb] = sum_s U0[rb][s] V[s][cb], U0 staged in the
// plane region, V in registers.
template <int PREC, bool HALF, int N0, int N1, int RB>
__device__ __forceinline__ void coil_p(const Geo<N0, N1, RB>& g, const float2* lds, const Share& sh, int lane,
                                       const typename Tile<PREC>::B (&vb)[3], f32x4 (&pr)[8], f32x4 (&pi)[8]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    typename Tile<PREC>::Acc c = Tile<PREC>::zero();
    const int rb = sh.part + i * sh.q;
    if (sh.on && rb < g.n0b) {
#pragma unroll
      for (int s = 0; s < 3; ++s)
        if (s < g.r0b) rank_mma<PREC>(c, frag_a<PREC>(lds, g.r0b, rb, s, lane), vb[s], HALF && s == g.r0b - 1);
    }
    Tile<PREC>::finish(c, pr[i], pi[i]);
  }
}

// ---------------------------------------------------------------- adjoint contraction
// Y = h conj(U1) with h in the plane, then Wb = U0^H Y -> T3b[j][i2].  Wave w takes Y row
// block w % n0b over a 1 / q share of the K16 steps over i1.  conj(U1) is staged through
// two LDS step buffers, each thread carrying the pieces of the next two steps in
// registers (loads issued two steps ahead).  Ends synchronised.
template <int PREC, int N0, int N1, int RB>
__device__ __forceinline__ void adjoint_w(const PlaneArgs& a, const Geo<N0, N1, RB>& g, int j, int i2, float2* lds,
                                          int lane, int tid) {
  const int wave = threadIdx.x >> 6, grp = lane >> 4;
  const int qy = NWAVE / g.n0b, yb = wave % g.n0b, kq = wave / g.n0b;
  const bool on = kq < qy;
  const int sp = frag_b_step_bytes<PREC>(g.r1b) / 16;  // 16-byte pieces of one step (<= 2 PT)
  const bool two = tid + PT < sp;
  const float4* src = reinterpret_cast<const float4*>(a.U1CF);
  float4* stage = reinterpret_cast<float4*>(lds + STAGE_OFF);
  auto fetch = [&](float4& p0, float4& p1, int s) {
    if (s < g.n1b) {
      const float4* q = src + (size_t)s * sp;
      if (tid < sp) p0 = q[tid];
      if (two) p1 = q[tid + PT];
    }
  };
  auto put = [&](const float4& p0, const float4& p1, int s) {
    if (s < g.n1b) {
      float4* q = stage + (s & 1) * sp;
      if (tid < sp) q[tid] = p0;
      if (two) q[tid + PT] = p1;
    }
  };
  typename Tile<PREC>::Acc yc[3];
#pragma unroll
  for (int nb = 0; nb < 3; ++nb) yc[nb] = Tile<PREC>::zero();
  const int i0 = 16 * yb + (lane & 15);
  auto compute = [&](int s) {
    if (on && (s % qy) == kq) {
      float2 hv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) hv[t] = lds[i0 * g.PS + 16 * s + 4 * grp + t];
      const float4* buf = stage + (s & 1) * sp;
      if constexpr (RB != 0) {
        // compile-time rank blocks: the step's B fragments read together, so that their LDS
        // latencies overlap
        typename Tile<PREC>::B bf[RB];
#pragma unroll
        for (int nb = 0; nb < RB; ++nb) bf[nb] = frag_b<PREC>(buf, RB, nb, 0, lane);
        const typename Tile<PREC>::A av = Tile<PREC>::make_a(hv);
#pragma unroll
        for (int nb = 0; nb < RB; ++nb) Tile<PREC>::mma(yc[nb], av, bf[nb]);
      } else {
        const typename Tile<PREC>::A av = Tile<PREC>::make_a(hv);
#pragma unroll
        for (int nb = 0; nb < 3; ++nb)
          if (nb < g.r1b) {
            Tile<PREC>::mma(yc[nb], av, frag_b<PREC>(buf, g.r1b, nb, 0, lane));
            __builtin_amdgcn_sched_barrier(0);  // one B fragment live at a time
          }
      }
    }
  };
  float4 o0, o1, e0, e1;  // pieces of the next odd and even steps
  fetch(e0, e1, 0);
  put(e0, e1, 0);
  fetch(o0, o1, 1);
  fetch(e0, e1, 2);
  __syncthreads();
  for (int s = 0; s < g.n1b; s += 2) {
    put(o0, o1, s + 1);
    fetch(o0, o1, s + 3);
    compute(s);
    __syncthreads();
    if (s + 1 < g.n1b) {
      put(e0, e1, s + 2);
      fetch(e0, e1, s + 4);
      compute(s + 1);
      __syncthreads();
    }
  }
  // Wb = U0^H Y.  The wave's Y tiles (rows = Y row block yb) are one K16 step of Wb: every
  // wave forms Wb's partial over its rows and its share of i1, and the partials are summed
  // in wave order through the plane and staging regions (free after the loop's last barrier).
  if (on) {
    typename Tile<PREC>::B yf[3];
#pragma unroll
    for (int nb = 0; nb < 3; ++nb)
      if (nb < g.r1b) {
        f32x4 yr, yi;
        Tile<PREC>::finish(yc[nb], yr, yi);
        yf[nb] = tile_as_b<PREC>(yr, yi);
      }
#pragma unroll
    for (int mb = 0; mb < 3; ++mb)
      if (mb < g.r0b) {
        const typename Tile<PREC>::A ua = frag_a<PREC>(a.U0HF, g.n0b, mb, yb, lane);
#pragma unroll
        for (int nb = 0; nb < 3; ++nb)
          if (nb < g.r1b) {
            typename Tile<PREC>::Acc wc = Tile<PREC>::zero();
            Tile<PREC>::mma(wc, ua, yf[nb]);
            f32x4 wr, wi;
            Tile<PREC>::finish(wc, wr, wi);
#pragma unroll
            for (int r = 0; r < 4; ++r)
              lds[((wave * 3 + mb) * 3 + nb) * 256 + (4 * grp + r) * 16 + (lane & 15)] = make_float2(wr[r], wi[r]);
          }
      }
  }
  __syncthreads();
  const int nw = qy * g.n0b;  // waves with a share (the first nw)
  const int c1 = 16 * g.r1b, nout = 16 * g.r0b * c1;
  float2* wo = a.T3b + ((size_t)j * g.n2 + i2) * g.r0 * g.r1;
  for (int e = tid; e < nout; e += PT) {
    const int q0 = e / c1, q1 = e % c1;
    const int o = ((q0 >> 4) * 3 + (q1 >> 4)) * 256 + (q0 & 15) * 16 + (q1 & 15);
    float2 acc = make_float2(0.f, 0.f);
    for (int w = 0; w < nw; ++w) acc = cadd(acc, lds[w * 9 * 256 + o]);
    if (q0 < g.r0 && q1 < g.r1) wo[q0 * g.r1 + q1] = acc;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- plane kernels
// Per coil: W (and in the adjoint the coil's samples) loaded early; U0 (fragment order,
// the whole factor) staged in the plane region and W in the stage region; V = W U1^T for
// the wave's column block into registers, then the wave's P tiles.
template <int PREC, bool HALF, int N0, int N1, int RB>
__device__ __forceinline__ void coil_map(const void* u0f, const void* u1tf, const Geo<N0, N1, RB>& g, float2* lds,
                                         const Share& sh, int lane, int tid, const WPrefetch& w, f32x4 (&pr)[8],
                                         f32x4 (&pi)[8]) {
  // the column block's U1^T fragments, in flight across the stores
  typename Tile<PREC>::B u1[3];
#pragma unroll
  for (int s = 0; s < 3; ++s)
    if (s < g.r1b) u1[s] = frag_b<PREC>(u1tf, g.n1b, sh.cb, s, lane);
  {
    const int n = g.n0b * g.r0b * 128;  // 16-byte pieces of U0 in fragment order (2 KiB a fragment)
    const uint4* src = reinterpret_cast<const uint4*>(u0f);
    uint4* dst = reinterpret_cast<uint4*>(lds);
    for (int e = tid; e < n; e += PT) dst[e] = src[e];
  }
  w_store<PREC>(g, lds, tid, w);
  __syncthreads();
  typename Tile<PREC>::B vb[3];
  coil_v<PREC, HALF>(g, lds, lane, u1, vb);
  coil_p<PREC, HALF>(g, lds, sh, lane, vb, pr, pi);
  __syncthreads();  // U0 is consumed; the plane region is free
}

template <int PREC, int N0, int N1, int RB, bool HALF = false>
__global__ __launch_bounds__(PT) void plane_fwd_kernel(PlaneArgs a) {
  __shared__ float2 lds[LDS_ELEMS];
  const Geo<N0, N1, RB> g(a);
  const int ngrp = (a.J + a.G - 1) / a.G;
  int i2, gi;
  plane_block(ngrp, g.n2, i2, gi);
  const float2* xp = a.xt + (size_t)i2 * g.n0 * g.n1;
  const Share sh = plane_share(g);
  int pq[SCAT];  // sampled plane positions, the same for every coil
#pragma unroll
  for (int k = 0; k < SCAT; ++k) pq[k] = (int)threadIdx.x + k * PT < a.L ? a.pos[threadIdx.x + k * PT] : -1;
  load_twiddles(a, g, lds);
  const int j0 = gi * a.G, j1 = min(a.J, (gi + 1) * a.G);
  const WSlots wsl = w_slots<PREC>(g, (int)threadIdx.x);
  WPrefetch w;  // W of the next coil, loaded one coil ahead
  if (j0 < j1) w_load(a, g, j0, i2, wsl, w);
  // the x values of the wave's share, the same for every coil: loaded once
  float2 xr[8][4];
  {
    const int lane = threadIdx.x & 63, grp = lane >> 4;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int rb = min(sh.part + i * sh.q, g.n0b - 1);
#pragma unroll
      for (int r = 0; r < 4; ++r) xr[i][r] = xp[(16 * rb + 4 * grp + r) * g.n1 + 16 * sh.cb + (lane & 15)];
    }
  }
  for (int j = j0; j < j1; ++j) {
    // lane and thread index through an empty asm: per-coil addresses are recomputed
    // here rather than hoisted out of the coil loop and held across the transform
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, grp = lane >> 4;
    f32x4 pr[8], pi[8];
    coil_map<PREC, HALF>(a.U0F, a.U1TF, g, lds, sh, lane, tid, w, pr, pi);
    if (j + 1 < j1) w_load(a, g, j + 1, i2, wsl, w);
    // m = x (.) P; the input chessboard sign of the centred DFT is carried by xt
    if (sh.on) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int rb = sh.part + i * sh.q;
        if (rb < g.n0b) {
          const int i1 = 16 * sh.cb + (lane & 15);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i0 = 16 * rb + 4 * grp + r;
            lds[i0 * g.PS + i1] = cmul(make_float2(pr[i][r], pi[i][r]), xr[i][r]);
          }
        }
      }
    }
    __syncthreads();
    plane_fft<FFT_CHUNK_FWD>(a, g, lds, -1);
    float2* zo = a.Z + ((size_t)j * g.n2 + i2) * a.L;
#pragma unroll
    for (int k = 0; k < SCAT; ++k)
      if (pq[k] >= 0) {
        const int k0 = pq[k] / g.n1, k1 = pq[k] - k0 * g.n1;
        float2 v = lds[k0 * g.PS + k1];
        if ((k0 + k1) & 1) v = make_float2(-v.x, -v.y);
        zo[tid + k * PT] = v;
      }
    for (int l = tid + SCAT * PT; l < a.L; l += PT) {  // beyond the preloaded positions
      const int q = a.pos[l];
      const int k0 = q / g.n1, k1 = q - k0 * g.n1;
      float2 v = lds[k0 * g.PS + k1];
      if ((k0 + k1) & 1) v = make_float2(-v.x, -v.y);
      zo[l] = v;
    }
    __syncthreads();  // the gather is done with the plane
  }
}

// The adjoint's coil map, formed after the transform one P tile at a time where gx uses
// it (nothing of P is held across the transform): V = W U1^T for the wave's column block
// (W staged), then per row block P = U0 V with U0's fragments read from memory three
// steps ahead.
template <int PREC, int N0, int N1, int RB>
struct AdjMap {
  typename Tile<PREC>::B vb[3];
  typename Tile<PREC>::A ring[4];
  int k;  // next (row block index, step) to load, 3 i + s over the wave's row blocks
};

template <int PREC, int N0, int N1, int RB>
__device__ __forceinline__ void adj_map_load(const PlaneArgs& a, const Geo<N0, N1, RB>& g, const Share& sh, int lane,
                                             AdjMap<PREC, N0, N1, RB>& m, int k) {
  const int i = k / 3, s = k % 3, rb = sh.part + i * sh.q;
  if (i < 8 && rb < g.n0b && s < g.r0b) m.ring[k & 3] = frag_a<PREC>(a.U0SF, g.r0b, rb, s, lane);
}

// Adjoint plane kernel, two forms.  plane_adj_kernel (BF16-split plans) forms the coil map
// before the transform, with U0 staged in the plane region, and holds P across it (the
// transform then works in half-plane chunks).  plane_adj_late_kernel (FP32 plans) forms
// each P tile after the transform where gx uses it, with U0 read from memory; its
// transform holds whole passes.  Measured at 128 x 128 planes, the first is faster in
// BF16-split (its matrix-core steps are short, so U0 read latency from memory shows) and
// the second in FP32.
template <int PREC, int N0, int N1, int RB, bool FULL = false>
__global__ __launch_bounds__(PT) void plane_adj_kernel(PlaneArgs a) {
  __shared__ __align__(16) float2 lds[LDS_ELEMS];
  const Geo<N0, N1, RB> g(a);
  const int ngrp = (a.J + a.G - 1) / a.G;
  int i2, gi;
  plane_block(ngrp, g.n2, i2, gi);
  const float2* xp = a.xt + (size_t)i2 * g.n0 * g.n1;
  const bool want_gx = FULL || a.gxpart != nullptr;  // FULL: gx and T3b both wanted, known at compile time
  const Share sh = plane_share(g);
  int zq[SCAT];  // sampled plane positions, the same for every coil
#pragma unroll
  for (int k = 0; k < SCAT; ++k) zq[k] = (int)threadIdx.x + k * PT < a.L ? a.pos[threadIdx.x + k * PT] : -1;
  f32x4 gr[8], gim[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) { gr[i] = z4(); gim[i] = z4(); }
  load_twiddles(a, g, lds);
  for (int j = gi * a.G; j < a.J && j < (gi + 1) * a.G; ++j) {
    int tid = threadIdx.x;  // opaque per coil, as in the forward kernel
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, grp = lane >> 4;
    // this plane's samples (at most SCAT per thread) and W, loaded early
    const float2* zi = a.Z + ((size_t)j * g.n2 + i2) * a.L;
    float2 zv[SCAT];
#pragma unroll
    for (int k = 0; k < SCAT; ++k) {  // unconditional loads (L >= 1 on this path), as in w_load
      const float2 v = zi[min(tid + k * PT, (int)a.L - 1)];
      const float m = zq[k] >= 0 ? 1.f : 0.f;
      zv[k] = make_float2(v.x * m, v.y * m);
    }
    f32x4 pr[8], pi[8];
    if (want_gx) {
      WPrefetch w;
      w_load(a, g, j, i2, w_slots<PREC>(g, tid), w);  // offsets recomputed: no registers held across coils
      // B c recomputed, with U0 and U1 carrying the output chessboard sign: P' = s P
      coil_map<PREC, false>(a.U0SF, a.U1TSF, g, lds, sh, lane, tid, w, pr, pi);
    }
    // zero-filled scatter (with the chessboard sign)
    {  // 16-byte stores (the plane region starts the 16-byte aligned LDS array); n0 PS is even
      float4* z4p = reinterpret_cast<float4*>(lds);
      for (int e = tid; e < g.n0 * g.PS / 2; e += PT) z4p[e] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SCAT; ++k)
      if (zq[k] >= 0) {
        const int k0 = zq[k] / g.n1, k1 = zq[k] - k0 * g.n1;
        float2 v = zv[k];
        if ((k0 + k1) & 1) v = make_float2(-v.x, -v.y);
        lds[k0 * g.PS + k1] = v;
      }
    for (int l = tid + SCAT * PT; l < a.L; l += PT) {  // beyond the prefetched samples
      const int q = a.pos[l];
      const int k0 = q / g.n1, k1 = q - k0 * g.n1;
      float2 v = zi[l];
      if ((k0 + k1) & 1) v = make_float2(-v.x, -v.y);
      lds[k0 * g.PS + k1] = v;
    }
    __syncthreads();
    // compile-time plane sizes: whole passes over wave-owned lines (fewer barriers)
    // last pass two line steps at a time: the map and gx stay in registers across it
    plane_fft<(N0 != 0 ? FFT_CHUNK_FWD : FFT_CHUNK_ADJ), N0, N1, RB, 2>(a, g, lds, +1);
    // g = s g' (g' the plane after the transform, s the output chessboard sign):
    // gx += conj(P) s g' = conj(P') g' in registers (P' = s P from the signed factors);
    // h = conj(x) s g' = conj(s x) g' into the plane, s x being what xt holds.  x in two
    // batches of four tiles, each batch's loads issued together.
    if (sh.on) {
#pragma unroll
      for (int hb = 0; hb < 2; ++hb) {
        float2 xv[4][4];
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const int rb = sh.part + (4 * hb + ii) * sh.q;
          if (rb < g.n0b)
#pragma unroll
            for (int r = 0; r < 4; ++r) xv[ii][r] = xp[(16 * rb + 4 * grp + r) * g.n1 + 16 * sh.cb + (lane & 15)];
        }
        float2 gvs[4][4];  // all of the batch's plane values read before any is rewritten
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const int rb = sh.part + (4 * hb + ii) * sh.q;
          if (rb < g.n0b)
#pragma unroll
            for (int r = 0; r < 4; ++r) gvs[ii][r] = lds[(16 * rb + 4 * grp + r) * g.PS + 16 * sh.cb + (lane & 15)];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const int i = 4 * hb + ii;
          const int rb = sh.part + i * sh.q;
          if (rb < g.n0b) {
            const int i1 = 16 * sh.cb + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i0 = 16 * rb + 4 * grp + r;
              const float2 gv = gvs[ii][r];
              if (want_gx) {  // conj(P') g' = s conj(P) g'
                const float2 c = cmulc(make_float2(pr[i][r], pi[i][r]), gv);
                gr[i][r] += c.x;
                gim[i][r] += c.y;
              }
              lds[i0 * g.PS + i1] = cmulc(xv[ii][r], gv);
            }
          }
        }
      }
    }
    __syncthreads();
    if (FULL || a.T3b) adjoint_w<PREC>(a, g, j, i2, lds, lane, tid);
  }
  if (want_gx && sh.on) {
    const int lane = threadIdx.x & 63, grp = lane >> 4;
    float2* gxp = a.gxpart + ((size_t)gi * g.n2 + i2) * g.n0 * g.n1;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int rb = sh.part + i * sh.q;
      if (rb < g.n0b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i0 = 16 * rb + 4 * grp + r, i1 = 16 * sh.cb + (lane & 15);
          gxp[i0 * g.n1 + i1] = make_float2(gr[i][r], gim[i][r]);
        }
    }
  }
}

template <int PREC, int N0, int N1, int RB, bool FULL = false, bool HALF = false>
__global__ __launch_bounds__(PT) void plane_adj_late_kernel(PlaneArgs a) {
  __shared__ __align__(16) float2 lds[LDS_ELEMS];
  const Geo<N0, N1, RB> g(a);
  const int ngrp = (a.J + a.G - 1) / a.G;
  int i2, gi;
  plane_block(ngrp, g.n2, i2, gi);
  const float2* xp = a.xt + (size_t)i2 * g.n0 * g.n1;
  const bool want_gx = FULL || a.gxpart != nullptr;  // FULL: gx and T3b both wanted, known at compile time
  const Share sh = plane_share(g);
  int zq[SCAT];  // sampled plane positions, the same for every coil
#pragma unroll
  for (int k = 0; k < SCAT; ++k) zq[k] = (int)threadIdx.x + k * PT < a.L ? a.pos[threadIdx.x + k * PT] : -1;
  f32x4 gr[8], gim[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) { gr[i] = z4(); gim[i] = z4(); }
  load_twiddles(a, g, lds);
  for (int j = gi * a.G; j < a.J && j < (gi + 1) * a.G; ++j) {
    int tid = threadIdx.x;  // opaque per coil, as in the forward kernel
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, grp = lane >> 4;
    // this plane's samples (at most SCAT per thread) and W, loaded early
    const float2* zi = a.Z + ((size_t)j * g.n2 + i2) * a.L;
    float2 zv[SCAT];
#pragma unroll
    for (int k = 0; k < SCAT; ++k) {  // unconditional loads (L >= 1 on this path), as in w_load
      const float2 v = zi[min(tid + k * PT, (int)a.L - 1)];
      const float m = zq[k] >= 0 ? 1.f : 0.f;
      zv[k] = make_float2(v.x * m, v.y * m);
    }
    if (want_gx) {
      WPrefetch w;
      w_load(a, g, j, i2, w_slots<PREC>(g, tid), w);  // offsets recomputed: no registers held across coils
      w_store<PREC>(g, lds, tid, w);              // the stage region is free (previous coil done)
    }
    // zero-filled scatter (with the chessboard sign)
    {  // 16-byte stores (the plane region starts the 16-byte aligned LDS array); n0 PS is even
      float4* z4p = reinterpret_cast<float4*>(lds);
      for (int e = tid; e < g.n0 * g.PS / 2; e += PT) z4p[e] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SCAT; ++k)
      if (zq[k] >= 0) {
        const int k0 = zq[k] / g.n1, k1 = zq[k] - k0 * g.n1;
        float2 v = zv[k];
        if ((k0 + k1) & 1) v = make_float2(-v.x, -v.y);
        lds[k0 * g.PS + k1] = v;
      }
    for (int l = tid + SCAT * PT; l < a.L; l += PT) {  // beyond the prefetched samples
      const int q = a.pos[l];
      const int k0 = q / g.n1, k1 = q - k0 * g.n1;
      float2 v = zi[l];
      if ((k0 + k1) & 1) v = make_float2(-v.x, -v.y);
      lds[k0 * g.PS + k1] = v;
    }
    __syncthreads();
    plane_fft<FFT_CHUNK_FWD>(a, g, lds, +1);  // nothing held across it but gx: whole passes
    // g = s g' (g' the plane after the transform, s the output chessboard sign):
    // gx += conj(P) s g' in registers; h = conj(x) s g' = conj(s x) g' into the plane, s x
    // being what xt holds.  Each P tile is formed just before its use.
    if (sh.on) {
      AdjMap<PREC, N0, N1, RB> m;
      if (want_gx) {
        // V = W U1^T[:, cb], the U1^T fragment of the next step loaded during this one
        typename Tile<PREC>::Acc cv[3];
#pragma unroll
        for (int mb = 0; mb < 3; ++mb) cv[mb] = Tile<PREC>::zero();
        typename Tile<PREC>::B u1[2];
        u1[0] = frag_b<PREC>(a.U1TSF, g.n1b, sh.cb, 0, lane);
#pragma unroll
        for (int s = 0; s < 3; ++s)
          if (s < g.r1b) {
            if (s + 1 < g.r1b) u1[(s + 1) & 1] = frag_b<PREC>(a.U1TSF, g.n1b, sh.cb, s + 1, lane);
            if (s == 1)
#pragma unroll
              for (int k = 0; k < 3; ++k) adj_map_load(a, g, sh, lane, m, k);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int mb = 0; mb < 3; ++mb)
              if (mb < g.r0b)
                rank_mma<PREC>(cv[mb], frag_a<PREC>(lds + STAGE_OFF, g.r1b, mb, s, lane), u1[s & 1],
                               HALF && s == g.r1b - 1);
          }
        if (g.r1b < 2)
#pragma unroll
          for (int k = 0; k < 3; ++k) adj_map_load(a, g, sh, lane, m, k);
#pragma unroll
        for (int mb = 0; mb < 3; ++mb) {
          f32x4 cr, ci;
          Tile<PREC>::finish(cv[mb], cr, ci);
          m.vb[mb] = tile_as_b<PREC>(cr, ci);
        }
      }
      const int i1 = 16 * sh.cb + (lane & 15);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int rb = sh.part + i * sh.q;
        if (rb < g.n0b) {
          float2 xv[4], gv[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            xv[r] = xp[(16 * rb + 4 * grp + r) * g.n1 + i1];
            gv[r] = lds[(16 * rb + 4 * grp + r) * g.PS + i1];
          }
          if (want_gx) {
            typename Tile<PREC>::Acc c = Tile<PREC>::zero();
#pragma unroll
            for (int s = 0; s < 3; ++s) {
              adj_map_load(a, g, sh, lane, m, 3 * i + s + 3);
              __builtin_amdgcn_sched_barrier(0);
              if (s < g.r0b) rank_mma<PREC>(c, m.ring[(3 * i + s) & 3], m.vb[s], HALF && s == g.r0b - 1);
            }
            f32x4 pr, pi;
            Tile<PREC>::finish(c, pr, pi);
#pragma unroll
            for (int r = 0; r < 4; ++r) {  // conj(P') g' = s conj(P) g' (signed factors)
              const float2 cg = cmulc(make_float2(pr[r], pi[r]), gv[r]);
              gr[i][r] += cg.x;
              gim[i][r] += cg.y;
            }
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) lds[(16 * rb + 4 * grp + r) * g.PS + i1] = cmulc(xv[r], gv[r]);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    __syncthreads();
    if (FULL || a.T3b) adjoint_w<PREC>(a, g, j, i2, lds, lane, tid);
  }
  if (want_gx && sh.on) {
    const int lane = threadIdx.x & 63, grp = lane >> 4;
    float2* gxp = a.gxpart + ((size_t)gi * g.n2 + i2) * g.n0 * g.n1;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int rb = sh.part + i * sh.q;
      if (rb < g.n0b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i0 = 16 * rb + 4 * grp + r, i1 = 16 * sh.cb + (lane & 15);
          gxp[i0 * g.n1 + i1] = make_float2(gr[i][r], gim[i][r]);
        }
    }
  }
}

// Plan-time fragment-ordered copy of O(o, k) = src[o * so + k * sk] (conjugated if bit 0 of
// conj, times (-1)^o if bit 1), zero for o >= no or k >= nk.  One thread per (o block, step, lane).
template <int PREC>
__global__ void frag_operand_kernel(const float2* __restrict__ src, int no, int nk, int64_t so, int64_t sk, int conj,
                                    int is_b, void* dst) {
  const int obs = (no + 15) / 16, ks = (nk + 15) / 16;
  const int total = obs * ks * 64;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int lane = e % 64, f = e / 64, ob = f / ks, s = f % ks;
    const int o = 16 * ob + (lane & 15);
    float2 v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = 16 * s + ((conj & 4) ? kperm(4 * (lane >> 4) + t) : 4 * (lane >> 4) + t);
      v[t] = (o < no && k < nk) ? src[(int64_t)o * so + (int64_t)k * sk] : make_float2(0.f, 0.f);
      if (conj & 1) v[t].y = -v[t].y;
      if ((conj & 2) && (o & 1)) v[t] = make_float2(-v[t].x, -v[t].y);
    }
    if (is_b) put_frag_b<PREC>(dst, obs, ob, s, lane, v);
    else put_frag_a<PREC>(dst, ks, ob, s, lane, v);
  }
}

// ---------------------------------------------------------------- line kernels
constexpr int LT = 32;     // lines per workgroup
constexpr int LNT = 256;   // threads
constexpr int LMAXN = 256; // max n2 on this path

template <int N2>
__device__ __forceinline__ void line_fft(const LineArgs& a, float2* tile, const float2* tw, int n, int dir) {
  if constexpr (N2 != 0) {
    lds_fft_ct<N2, LNT, N2 * LT>(tile, LT, 1, LT + 1, tw, dir);
  } else {
    LdsLines tg{LT, 1, LT + 1};
    lds_fft_lines<LNT, LMAXN * LT / 2>(tile, tg, n, a.rad2, a.nrad2, tw, dir);
  }
}

template <int N2>
__global__ __launch_bounds__(LNT) void line_fwd_kernel(LineArgs a) {
  __shared__ float2 tile[(N2 ? N2 : LMAXN) * (LT + 1)];  // sized to the readout: more workgroups per CU
  __shared__ float2 tw[N2 ? N2 : LMAXN];
  __shared__ double red[LNT];
  const int lblocks = (a.L + LT - 1) / LT;
  const int j = blockIdx.x / lblocks, l0 = (blockIdx.x % lblocks) * LT;
  const int n = N2 ? N2 : a.n2, ES = LT + 1;
  for (int e = threadIdx.x; e < n; e += LNT) tw[e] = a.tw2[e];
  // With the compile-time readout, the thread's Z values are loaded together, unguarded (lines
  // past L read line L - 1 and are zeroed), before any is stored; then the measured samples of
  // its outputs, ahead of the transform.
  constexpr int YQ = N2 ? N2 * LT / LNT : 1;
  if constexpr (N2 != 0) {
    float2 zv[YQ];
#pragma unroll
    for (int q = 0; q < YQ; ++q) {
      const int e = threadIdx.x + q * LNT, i2 = e / LT, l = e % LT;
      zv[q] = a.Z[((size_t)j * n + i2) * a.L + min(l0 + l, (int)a.L - 1)];
    }
#pragma unroll
    for (int q = 0; q < YQ; ++q) {
      const int e = threadIdx.x + q * LNT, i2 = e / LT, l = e % LT;
      const float m = l0 + l < a.L ? ((i2 & 1) ? -1.f : 1.f) : 0.f;
      tile[i2 * ES + l] = make_float2(zv[q].x * m, zv[q].y * m);
    }
  } else {
    for (int e = threadIdx.x; e < n * LT; e += LNT) {
      const int i2 = e / LT, l = e % LT;
      float2 v = make_float2(0.f, 0.f);
      if (l0 + l < a.L) v = a.Z[((size_t)j * n + i2) * a.L + l0 + l];
      if (i2 & 1) v = make_float2(-v.x, -v.y);
      tile[i2 * ES + l] = v;
    }
  }
  float2 yv[YQ];
  if constexpr (N2 != 0) {
    if (a.y) {
#pragma unroll
      for (int q = 0; q < YQ; ++q) {
        const int e = threadIdx.x + q * LNT, l = e / N2, k2 = e % N2;
        yv[q] = a.y[(size_t)j * a.M + (size_t)min(l0 + l, (int)a.L - 1) * N2 + k2];
      }
    }
  }
  __syncthreads();
  line_fft<N2>(a, tile, tw, n, -1);
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < (N2 ? YQ : 1); ++q)
  for (int e = threadIdx.x + q * LNT; e < n * LT; e += (N2 ? n * LT : LNT)) {
    const int l = e / n, k2 = e % n;
    if (l0 + l >= a.L) continue;
    float2 v = tile[k2 * ES + l];
    const float s = (k2 & 1) ? -a.gscale : a.gscale;
    v = cscale(v, s);
    const size_t m = (size_t)(l0 + l) * n + k2;
    const size_t o = (size_t)j * a.M + m;
    if (a.y) {
      const float2 d = csub(v, N2 ? yv[q] : a.y[o]);
      const float wm = a.w ? a.w[m] : 1.0f;
      acc += (double)wm * ((double)d.x * d.x + (double)d.y * d.y);
      const float2 r = cscale(d, wm);
      if (a.out) a.out[o] = r;
      if (a.Zw) tile[k2 * ES + l] = (k2 & 1) ? make_float2(-r.x, -r.y) : r;  // each entry is this thread's
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
  if (a.Zw) {
    // transfer layout: the weighted residual taken back along the readout while the lines
    // are on chip (the adjoint's first step, as the adjoint line kernel computes it, without
    // the adjoint's scale, which the adjoint applies at its ends)
    if (!a.part) __syncthreads();
    line_fft<N2>(a, tile, tw, n, +1);
    for (int e = threadIdx.x; e < n * LT; e += LNT) {
      const int i2 = e / LT, l = e % LT;
      if (l0 + l >= a.L) continue;
      const float2 v = tile[i2 * ES + l];
      a.Zw[((size_t)j * n + i2) * a.L + l0 + l] = cscale(v, (i2 & 1) ? -a.gscale : a.gscale);
    }
  }
}

template <int N2>
__global__ __launch_bounds__(LNT) void line_adj_kernel(LineArgs a) {
  __shared__ float2 tile[(N2 ? N2 : LMAXN) * (LT + 1)];
  __shared__ float2 tw[N2 ? N2 : LMAXN];
  const int lblocks = (a.L + LT - 1) / LT;
  const int j = blockIdx.x / lblocks, l0 = (blockIdx.x % lblocks) * LT;
  const int n = N2 ? N2 : a.n2, ES = LT + 1;
  for (int e = threadIdx.x; e < n; e += LNT) tw[e] = a.tw2[e];
  if constexpr (N2 != 0) {
    // the thread's samples loaded together and unguarded (lines past L read line L - 1 and
    // are zeroed), as in the forward line kernel
    constexpr int YQ = N2 * LT / LNT;
    float2 yv[YQ];
#pragma unroll
    for (int q = 0; q < YQ; ++q) {
      const int e = threadIdx.x + q * LNT, l = e / N2, k2 = e % N2;
      yv[q] = a.yin[(size_t)j * a.M + (size_t)min(l0 + l, (int)a.L - 1) * N2 + k2];
    }
#pragma unroll
    for (int q = 0; q < YQ; ++q) {
      const int e = threadIdx.x + q * LNT, l = e / N2, k2 = e % N2;
      const float m = l0 + l < a.L ? ((k2 & 1) ? -1.f : 1.f) : 0.f;
      tile[k2 * ES + l] = make_float2(yv[q].x * m, yv[q].y * m);
    }
  } else {
    for (int e = threadIdx.x; e < n * LT; e += LNT) {
      const int l = e / n, k2 = e % n;
      float2 v = make_float2(0.f, 0.f);
      if (l0 + l < a.L) v = a.yin[(size_t)j * a.M + (size_t)(l0 + l) * n + k2];
      if (k2 & 1) v = make_float2(-v.x, -v.y);
      tile[k2 * ES + l] = v;
    }
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

// xt[c][r] = s(r) x[r][c] for an R x C matrix (complex).  With n1 > 0 (even), r = i0 n1 + i1
// and s(r) = (-1)^(i0 + i1), the input chessboard sign of the centred plane DFT; else s = 1.
__global__ void transpose_kernel(const float2* __restrict__ x, int64_t R, int64_t C, int n1, float2* __restrict__ xt) {
  __shared__ float2 t[TT][TT + 1];
  const int64_t tr = (int64_t)blockIdx.y * TT, tc = (int64_t)blockIdx.x * TT;
  const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
  for (int k = ty; k < TT; k += 256 / TT) {
    const int64_t r = tr + k, c = tc + tx;
    if (r < R && c < C) {
      float2 v = x[r * C + c];
      // n1 even: i0 + i1 = r - i0 (n1 - 1) has the parity of r + i0
      if (n1 > 0 && ((r + r / n1) & 1)) v = make_float2(-v.x, -v.y);
      t[k][tx] = v;
    }
  }
  __syncthreads();
  for (int k = ty; k < TT; k += 256 / TT) {
    const int64_t c = tc + k, r = tr + tx;
    if (r < R && c < C) xt[c * R + r] = t[tx][k];
  }
}

// gx[r][c] = sum_g part[g][c][r] : part is ngrp x (C x R), gx is R x C
__global__ void reduce_transpose_kernel(const float2* __restrict__ part, int ngrp, int64_t R, int64_t C,
                                        float alpha, const float* __restrict__ scale_dev, float2* __restrict__ gx) {
  float sc = alpha;
  if (scale_dev) sc *= *scale_dev;
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
    if (r < R && c < C) gx[r * C + c] = cscale(t[tx][k], sc);
  }
}

// The adjoint form by precision (see plane_adj_kernel); at 128 x 128 planes ranks in (32, 48]
// take compile-time rank blocks (fewer register moves and SGPR spills; at 128^3, 32 coils:
// BF16-split 442 -> 420 us, FP32 675 -> 637 us).
template <int PREC, int N0, int N1>
void adj_launch(dim3 grid, dim3 block, const PlaneArgs& a, hipStream_t st) {
  constexpr int RB3 = N0 == 128 && N1 == 128 ? 3 : 0;
  const bool rb3 = RB3 == 3 && a.r0p == 48 && a.r1p == 48;
  // with both outputs wanted (the gradient step) the output checks are compile-time too
  const bool full = a.gxpart != nullptr && a.T3b != nullptr;
  if constexpr (PREC == 0) {
    // ranks in (32, 40]: the last rank block's padding skipped at compile time
    const bool half = a.r0 <= 40 && a.r1 <= 40;
    if (rb3 && full && half)
      hipLaunchKernelGGL((plane_adj_late_kernel<PREC, N0, N1, RB3, true, true>), grid, block, 0, st, a);
    else if (rb3 && full) hipLaunchKernelGGL((plane_adj_late_kernel<PREC, N0, N1, RB3, true>), grid, block, 0, st, a);
    else if (rb3) hipLaunchKernelGGL((plane_adj_late_kernel<PREC, N0, N1, RB3>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((plane_adj_late_kernel<PREC, N0, N1, 0>), grid, block, 0, st, a);
  } else {
    if (rb3 && full) hipLaunchKernelGGL((plane_adj_kernel<PREC, N0, N1, RB3, true>), grid, block, 0, st, a);
    else if (rb3) hipLaunchKernelGGL((plane_adj_kernel<PREC, N0, N1, RB3>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((plane_adj_kernel<PREC, N0, N1, 0>), grid, block, 0, st, a);
  }
}

template <int PREC>
hipError_t plane_launch_prec(const PlaneArgs& a, bool adj, hipStream_t st) {
  const int ngrp = (a.J + a.G - 1) / a.G;
  const dim3 grid((unsigned)(a.n2 * ngrp)), block(PT);
  // ranks in (32, 48] (three K16 blocks each) take compile-time rank blocks at 128 x 128
  const bool rb3 = a.r0p == 48 && a.r1p == 48;
  if (a.n0 == 128 && a.n1 == 128 && rb3 && !adj) {
    if (PREC == 0 && a.r0 <= 40 && a.r1 <= 40)  // FP32 ranks in (32, 40]: padding skipped
      hipLaunchKernelGGL((plane_fwd_kernel<PREC, 128, 128, 3, PREC == 0>), grid, block, 0, st, a);
    else
      hipLaunchKernelGGL((plane_fwd_kernel<PREC, 128, 128, 3>), grid, block, 0, st, a);
  } else if (a.n0 == 128 && a.n1 == 128) {
    if (adj) adj_launch<PREC, 128, 128>(grid, block, a, st);
    else hipLaunchKernelGGL((plane_fwd_kernel<PREC, 128, 128, 0>), grid, block, 0, st, a);
  } else if (a.n0 == 64 && a.n1 == 64) {
    if (adj) adj_launch<PREC, 64, 64>(grid, block, a, st);
    else hipLaunchKernelGGL((plane_fwd_kernel<PREC, 64, 64, 0>), grid, block, 0, st, a);
  } else {
    if (adj) adj_launch<PREC, 0, 0>(grid, block, a, st);
    else hipLaunchKernelGGL((plane_fwd_kernel<PREC, 0, 0, 0>), grid, block, 0, st, a);
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

hipError_t transpose_launch(const float2* x, int64_t R, int64_t C, int n1_sign, float2* xt, hipStream_t st) {
  dim3 grid((unsigned)((C + TT - 1) / TT), (unsigned)((R + TT - 1) / TT));
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, st, x, R, C, n1_sign, xt);
  return hipGetLastError();
}

hipError_t reduce_transpose_launch(const float2* part, int ngrp, int64_t R, int64_t C, float alpha,
                                   const float* scale_dev, float2* gx, hipStream_t st) {
  dim3 grid((unsigned)((R + TT - 1) / TT), (unsigned)((C + TT - 1) / TT));
  hipLaunchKernelGGL(reduce_transpose_kernel, grid, dim3(256), 0, st, part, ngrp, R, C, alpha, scale_dev, gx);
  return hipGetLastError();
}

size_t frag_operand_bytes(int no, int nk, int is_b, int precision) {
  const size_t blocks = (size_t)((no + 15) / 16) * ((nk + 15) / 16);
  return blocks * ((precision == 1 && is_b) ? 4096 : 2048);
}

hipError_t frag_operand_launch(const float2* src, int no, int nk, int64_t so, int64_t sk, int conj, int is_b,
                               int precision, void* dst, hipStream_t st) {
  const int total = ((no + 15) / 16) * ((nk + 15) / 16) * 64;
  const dim3 grid((unsigned)((total + 255) / 256)), block(256);
  if (precision == 1) hipLaunchKernelGGL(frag_operand_kernel<1>, grid, block, 0, st, src, no, nk, so, sk, conj, is_b, dst);
  else hipLaunchKernelGGL(frag_operand_kernel<0>, grid, block, 0, st, src, no, nk, so, sk, conj, is_b, dst);
  return hipGetLastError();
}

bool fused_supported(int64_t n0, int64_t n1, int64_t n2, int64_t r0, int64_t r1, int) {
  return n0 % 16 == 0 && n1 % 16 == 0 && n0 <= PMAX && n1 <= PMAX && n2 <= LMAXN && r0 <= RMAX && r1 <= RMAX;
}

}  // namespace mx
