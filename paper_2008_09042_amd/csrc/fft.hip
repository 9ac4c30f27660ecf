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
#include <cstring>
#include <vector>

#include "fft_device.h"

namespace mx {

namespace {

constexpr int NT = 256;
constexpr int TILE = 4096;          // complex elements per LDS tile at most (before padding):
                                    // with the twiddles, about 40 KB, four workgroups per CU
constexpr int TW_LDS_MAX = 1024;    // twiddle tables up to this length are staged in LDS

// complex elements of the LDS tile for T lines of length n
__host__ __device__ inline int tile_elems(int n, int T, bool contiguous) { return contiguous ? T * (n + 1) : T * n; }

// Row ga of the grid of the line l of a pad-mode tile (contiguous lines of g0 rows per coil):
// the tile starts at row pga0 of its coil; `tall` tiles span more than a coil.
__device__ __forceinline__ int64_t pad_row(const FftAxisArgs& a, int64_t o0, int64_t pga0, bool tall, int l) {
  if (tall) return (o0 + l) % a.outer_per_coil;
  const int64_t ga = pga0 + l;
  return ga >= a.outer_per_coil ? ga - a.outer_per_coil : ga;
}

// TWL: the twiddle table is copied into LDS behind the tile.  SMP: 4 the input is the gridding
// window (zero-pad), 6 rows outside it are zero, 7 only its columns are written, 5 the output
// is cropped to it (see FftAxisArgs); 1 the input comes from
// the samples through the inverse mask, 2 the output goes to them.  bid / nbl: this
// workgroup's index among the nbl workgroups of the pass.
template <bool TWL, int SMP>
__device__ __forceinline__ void fft_axis_body(const FftAxisArgs& a, int64_t bid_in, int64_t nbl) {
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
    o0 = bid_in * tg.T;
    t0 = 0;
    Tvalid = (int)((a.outer - o0) < tg.T ? (a.outer - o0) : tg.T);
  } else {
    tg.T = a.lines;
    tg.LS = 1;
    tg.ES = tg.T;
    const int64_t chunks = (a.inner + tg.T - 1) / tg.T;
    // consecutive chunks (adjacent columns, which share cache lines) go to one XCD: the
    // hardware deals workgroups round-robin over the 8 XCDs, each with its own L2
    int64_t bid = bid_in;
    if ((nbl & 7) == 0) bid = (bid_in & 7) * (nbl >> 3) + (bid_in >> 3);
    o0 = bid / chunks;
    t0 = (bid % chunks) * tg.T;
    Tvalid = (int)((a.inner - t0) < tg.T ? (a.inner - t0) : tg.T);
  }
  if constexpr (SMP == 5) {
    // cropping pass (strided lines = grid columns t0 .. t0 + Tvalid - 1): a tile wholly
    // outside the window's columns has nothing to write (uniform per workgroup, before any
    // barrier)
    if (t0 + Tvalid <= a.woff1 || t0 >= a.woff1 + a.wn1) return;
  }
  const int total = tg.T * n;
  // element e of the tile: (line, index) = (e / n, e % n) for contiguous lines, else
  // (e % T, e / T), so that consecutive threads touch consecutive addresses
  const FastDiv fd = fast_div((uint32_t)(a.inner == 1 ? n : tg.T));
  const FastDiv fN = {(uint32_t)a.coil_elems, a.coil_magic, a.coil_shift};
  // ---- load (with optional image premultiply and the input chessboard sign); LU
  // elements per thread are loaded before any is stored, so their latencies overlap
  // (an element past the tile reads the tile's first element and is masked to zero)
  constexpr int LU = 8;
  const int64_t gbase = a.inner == 1 ? o0 * a.n * a.inner : o0 * a.n * a.inner + t0;
  // pad mode: coil and row of the tile's first line, once per workgroup (a tile no taller
  // than a coil's grid spans at most two coils)
  int64_t pj0 = 0, pga0 = 0;
  bool ptall = false;
  if constexpr (SMP == 4) {
    pj0 = o0 / a.outer_per_coil;
    pga0 = o0 - pj0 * a.outer_per_coil;
    ptall = tg.T > a.outer_per_coil;
    // a tile of rows wholly outside the window has nothing to write: the next pass takes
    // them as zero (uniform per workgroup, before any barrier).  Its rows are [pga0, end) of
    // one coil, continued at row 0 of the next past the coil's last row.
    if (!ptall) {
      const int64_t end = pga0 + Tvalid, opc = a.outer_per_coil, w0 = a.woff0, w1 = a.woff0 + a.wn0;
      bool any = pga0 < w1 && (end < opc ? end : opc) > w0;
      if (end > opc) any = any || end - opc > w0;
      if (!any) return;
    }
  }
  if constexpr (SMP == 3) {
    // whole lines l0 .. l0 + T - 1 of coil j (contiguous axis): zero the tile, then put the
    // tile's samples, one contiguous range of the sorted mask, at their points
    for (int e = threadIdx.x; e < tg.T * tg.LS; e += NT) lds[e] = make_float2(0.f, 0.f);
    __syncthreads();
    const int64_t j = o0 / a.outer_per_coil, l0 = o0 % a.outer_per_coil;
    const int lo = a.in_lptr[l0], hi = a.in_lptr[l0 + Tvalid];
    const int64_t first = l0 * a.n;
    for (int sm = lo + threadIdx.x; sm < hi; sm += NT) {
      const uint32_t pp = (uint32_t)(a.in_mask[sm] - first);
      const int l = (int)fdiv(pp, fd), i = (int)pp - l * n;
      float2 x = a.in_samples[j * a.nsamples + sm];
      if (i & 1) {
        x.x = -x.x;
        x.y = -x.y;
      }
      lds[l * tg.LS + i] = x;
    }
  }
  for (int e0 = threadIdx.x; SMP != 3 && e0 < total; e0 += NT * LU) {
    float2 v[LU], pm[LU];
    uint32_t keep[LU];
    int li[LU];
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const int e = e0 + u * NT;
      const int ec = e < total ? e : 0;
      const int qd = (int)fdiv(ec, fd), rm = ec - qd * (int)fd.d;
      const int l = a.inner == 1 ? qd : rm, i = a.inner == 1 ? rm : qd;
      const bool ok = e < total && l < Tvalid;
      keep[u] = ok ? ((i & 1) ? 0xffffffffu : 0x7fffffffu) : 0u;  // sign bit kept only for odd i
      li[u] = e < total ? l * tg.LS + i * tg.ES : -1;
      const int64_t gidx = ok ? gbase + (int64_t)l * (a.inner == 1 ? a.n : 1) + (int64_t)i * a.inner : gbase;
      if constexpr (SMP == 1) {
        // the sample of this k-space point, or zero: both loads unconditional (index 0 when
        // unsampled), the zero applied by the mask below
        const uint32_t f = (uint32_t)gidx, j = fdiv(f, fN), pp = f - j * (uint32_t)fN.d;
        const int m = a.in_inv[pp];
        v[u] = a.in_samples[(int64_t)j * a.nsamples + (m >= 0 ? m : 0)];
        if (m < 0) keep[u] = 0u;
      } else if constexpr (SMP == 4) {
        // zero-padded, deapodised grid row ga of coil j (contiguous lines): the window's
        // points read S x / (Phi0 Phi1), the rest are zero (loads clamped into the window)
        const int lc = ok ? l : 0;  // the tile's lines are consecutive
        const int64_t ga = pad_row(a, o0, pga0, ptall, lc);
        const int64_t j = ptall ? (o0 + lc) / a.outer_per_coil : pj0 + (pga0 + lc >= a.outer_per_coil ? 1 : 0);
        const int r0 = (int)ga - a.woff0, r1 = i - a.woff1;
        const bool in = r0 >= 0 && r0 < a.wn0 && r1 >= 0 && r1 < a.wn1;
        const int c0 = min(max(r0, 0), a.wn0 - 1), c1 = min(max(r1, 0), a.wn1 - 1);
        const int64_t r = (int64_t)c0 * a.wn1 + c1;
        const float2 sv = a.src[j * (int64_t)a.wn0 * a.wn1 + r], xv = a.premul[r];
        const float w = a.iphi[c0] * a.iphi[a.wn0 + c1];
        v[u] = cscale(cmul(sv, xv), w);
        if (!in) keep[u] = 0u;
      } else if constexpr (SMP == 6) {
        // strided lines (grid columns), i the row: rows outside the window are zero and not
        // read (their loads clamped to the window's edge rows of the same columns)
        const bool in = i >= a.woff0 && i < a.woff0 + a.wn0;
        const int ic = min(max(i, a.woff0), a.woff0 + a.wn0 - 1);
        v[u] = a.src[gbase + (ok ? (int64_t)l + (int64_t)ic * a.inner : (int64_t)a.woff0 * a.inner)];
        if (!in) keep[u] = 0u;
      } else {
        v[u] = a.src[gidx];
      }
      if (SMP != 4 && a.premul) {
        const int64_t o = a.inner == 1 ? o0 + (ok ? l : 0) : o0;
        const int64_t oc = a.outer < 0x7fffffffLL ? (int64_t)((uint32_t)o % (uint32_t)a.outer_per_coil)
                                                  : o % a.outer_per_coil;
        const int64_t t = a.inner == 1 ? 0 : t0 + (ok ? l : 0);
        pm[u] = a.premul[(oc * a.n + (ok ? i : 0)) * a.inner + t];
      }
    }
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      if (li[u] < 0) continue;
      float2 x = v[u];
      if (SMP != 4 && a.premul) x = cmul(x, pm[u]);
      // odd i: negate (flip the sign bit); invalid: zero (clear every bit)
      const uint32_t flip = keep[u] == 0xffffffffu ? 0x80000000u : 0u;
      const uint32_t mask = keep[u] ? 0xffffffffu : 0u;
      x.x = __uint_as_float((__float_as_uint(x.x) ^ flip) & mask);
      x.y = __uint_as_float((__float_as_uint(x.y) ^ flip) & mask);
      lds[li[u]] = x;
    }
  }
  __syncthreads();
  lds_fft_lines<NT, TILE>(lds, tg, n, a.radix, a.nrad, tw, a.dir);
  // ---- store with the output chessboard sign, global sign and n^{-1/2}
  const float scale = (((n / 2) & 1) ? -1.f : 1.f) * rsqrtf((float)n);
  for (int e0 = threadIdx.x; e0 < total; e0 += NT * LU) {
    float2 v[LU];
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const int e = e0 + u * NT;
      const int ec = e < total ? e : 0;
      const int qd = (int)fdiv(ec, fd), rm = ec - qd * (int)fd.d;
      const int l = a.inner == 1 ? qd : rm, i = a.inner == 1 ? rm : qd;
      v[u] = lds[l * tg.LS + i * tg.ES];
    }
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const int e = e0 + u * NT;
      const int ec = e < total ? e : 0;
      const int qd = (int)fdiv(ec, fd), rm = ec - qd * (int)fd.d;
      const int l = a.inner == 1 ? qd : rm, i = a.inner == 1 ? rm : qd;
      if (e >= total || l >= Tvalid) continue;
      const float s = (i & 1) ? -scale : scale;
      const int64_t gidx = gbase + (int64_t)l * (a.inner == 1 ? a.n : 1) + (int64_t)i * a.inner;
      if constexpr (SMP == 2) {
        const uint32_t f = (uint32_t)gidx, j = fdiv(f, fN), pp = f - j * (uint32_t)fN.d;
        const int m = a.out_inv[pp];
        if (m >= 0) a.out_samples[(int64_t)j * a.nsamples + m] = cscale(v[u], s);
      } else if constexpr (SMP == 4) {
        // only the window's rows
        const int64_t ga = pad_row(a, o0, pga0, ptall, l);
        if (ga >= a.woff0 && ga < a.woff0 + a.wn0) a.data[gidx] = cscale(v[u], s);
      } else if constexpr (SMP == 7) {
        // contiguous lines (grid rows), i the column: only the window's columns
        if (i >= a.woff1 && i < a.woff1 + a.wn1) a.data[gidx] = cscale(v[u], s);
      } else if constexpr (SMP == 5) {
        // only the window: row i, column t0 + l of coil o0, deapodised
        const int r0 = i - a.woff0, r1 = (int)(t0 + l) - a.woff1;
        if (r0 >= 0 && r0 < a.wn0 && r1 >= 0 && r1 < a.wn1)
          a.crop_out[(o0 * a.wn0 + r0) * (int64_t)a.wn1 + r1] = cscale(v[u], s * a.iphi[r0] * a.iphi[a.wn0 + r1]);
      } else {
        a.data[gidx] = cscale(v[u], s);
      }
    }
  }
}

template <bool TWL, int SMP>
__global__ __launch_bounds__(NT) void fft_axis_kernel(FftAxisArgs a) {
  fft_axis_body<TWL, SMP>(a, blockIdx.x, gridDim.x);
}

// Several passes (of different slices) in one launch: descriptor i takes workgroups
// [start[i], start[i + 1]).  The descriptors travel in the kernel arguments.
template <bool TWL, int SMP>
__global__ __launch_bounds__(NT) void fft_axis_multi_kernel(FftMulti m) {
  int i = 0;
  while (i + 1 < m.n && (int)blockIdx.x >= m.start[i + 1]) ++i;
  fft_axis_body<TWL, SMP>(m.d[i], (int64_t)blockIdx.x - m.start[i], (int64_t)m.start[i + 1] - m.start[i]);
}

thread_local std::vector<FftLaunch>* g_fft_collect = nullptr;

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
// chip (about 1024), at most 64 lines or TILE elements per tile (small tiles keep
// several workgroups resident per CU), and for strided lines at least 8 adjacent ones
// (64-byte runs per load) where the tile allows.
hipError_t fft_axis_prepare(const FftAxisArgs& args, FftLaunch& out) {
  FftAxisArgs a = args;
  const int n = (int)a.n;
  const bool contiguous = a.inner == 1;
  const bool twl = n <= TW_LDS_MAX;
  int Tmax = TILE / n;
  if (Tmax > 64) Tmax = 64;
  if (Tmax < 1) Tmax = 1;
  // lines that carry work: the pad pass transforms only the window's rows (the other tiles
  // exit at once)
  int64_t lines = a.outer * a.inner;
  if (a.win == WIN_PAD && contiguous && a.outer_per_coil > 0 && a.wn0 > 0 && a.wn0 < a.outer_per_coil)
    lines = a.outer / a.outer_per_coil * a.wn0;
  int64_t T = (lines + 1023) / 1024;
  if (!contiguous && T < 8) T = 8;
  if (T > Tmax) T = Tmax;
  if (!contiguous && T > a.inner) T = a.inner;
  if (T < 1) T = 1;
  a.lines = (int)T;
  const int64_t blocks = contiguous ? (a.outer + T - 1) / T : a.outer * ((a.inner + T - 1) / T);
  const size_t lds = (size_t)(tile_elems(n, a.lines, contiguous) + (twl ? n : 0)) * sizeof(float2);
  int smp = a.in_inv ? 1 : a.out_inv ? 2 : 0;
  if (a.win || a.crop_out) {
    // the gridding window: pad on the first forward pass (rows), zero rows on the second
    // (columns), window columns out of the first inverse pass (rows), crop on the last (columns)
    if (smp || (a.win && a.crop_out) || a.win < 0 || a.win > WIN_COLS_OUT) return hipErrorInvalidValue;
    const int64_t g0 = contiguous ? a.outer_per_coil : a.n, g1 = contiguous ? a.n : a.inner;
    if (a.wn0 < 1 || a.wn1 < 1 || a.woff0 < 0 || a.woff1 < 0 || a.woff0 + a.wn0 > g0 || a.woff1 + a.wn1 > g1)
      return hipErrorInvalidValue;
    if (a.win == WIN_PAD && (!contiguous || !a.src || !a.premul || !a.iphi)) return hipErrorInvalidValue;
    if (a.win == WIN_ROWS_IN && (contiguous || a.premul || a.outer_per_coil != 1)) return hipErrorInvalidValue;
    if (a.win == WIN_COLS_OUT && (!contiguous || a.premul)) return hipErrorInvalidValue;
    if (a.crop_out && (contiguous || !a.iphi || a.outer_per_coil != 1)) return hipErrorInvalidValue;
    smp = a.crop_out ? 5 : a.win == WIN_PAD ? 4 : a.win == WIN_ROWS_IN ? 6 : 7;
  }
  // the reading pass places whole lines' samples directly when every tile holds lines of
  // one coil only
  if (smp == 1 && contiguous && a.in_mask && a.in_lptr && a.outer_per_coil % T == 0) smp = 3;
  if (smp && (a.in_inv && a.out_inv)) return hipErrorInvalidValue;
  // element indices j N + p below 2^31, so the multiply-high division of the flat index by
  // N is exact; its magic number in integer arithmetic (Granlund and Montgomery)
  if (smp && (a.nsamples <= 0 || a.coil_elems <= 0 || a.outer / a.outer_per_coil * a.coil_elems > 0x7fffffffLL))
    return hipErrorInvalidValue;
  if (smp) {
    const uint64_t d = (uint64_t)a.coil_elems;
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    a.coil_shift = l;
    a.coil_magic = (uint32_t)((((1ull << l) - d) << 32) / d + 1);
  }
  out.a = a;
  out.smp = smp;
  out.twl = twl;
  out.blocks = blocks;
  out.lds = lds;
  return hipSuccess;
}

void fft_collect(std::vector<FftLaunch>* sink) { g_fft_collect = sink; }

// Lines per workgroup: enough workgroups to spread a small transform over the whole
// chip (about 1024), at most 64 lines or TILE elements per tile (small tiles keep
// several workgroups resident per CU), and for strided lines at least 8 adjacent ones
// (64-byte runs per load) where the tile allows.  With a collector set on the calling
// thread (fft_collect) the prepared pass is appended to it instead of launched.
hipError_t fft_axis_launch(const FftAxisArgs& args, hipStream_t st) {
  FftLaunch l;
  hipError_t e = fft_axis_prepare(args, l);
  if (e != hipSuccess) return e;
  if (l.blocks <= 0) return hipSuccess;
  if (g_fft_collect) {
    g_fft_collect->push_back(l);
    return hipSuccess;
  }
  const dim3 gr((unsigned)l.blocks), bl(NT);
  const FftAxisArgs& a = l.a;
  switch (l.smp * 2 + (l.twl ? 1 : 0)) {
    case 15: hipLaunchKernelGGL((fft_axis_kernel<true, 7>), gr, bl, l.lds, st, a); break;
    case 14: hipLaunchKernelGGL((fft_axis_kernel<false, 7>), gr, bl, l.lds, st, a); break;
    case 13: hipLaunchKernelGGL((fft_axis_kernel<true, 6>), gr, bl, l.lds, st, a); break;
    case 12: hipLaunchKernelGGL((fft_axis_kernel<false, 6>), gr, bl, l.lds, st, a); break;
    case 11: hipLaunchKernelGGL((fft_axis_kernel<true, 5>), gr, bl, l.lds, st, a); break;
    case 10: hipLaunchKernelGGL((fft_axis_kernel<false, 5>), gr, bl, l.lds, st, a); break;
    case 9: hipLaunchKernelGGL((fft_axis_kernel<true, 4>), gr, bl, l.lds, st, a); break;
    case 8: hipLaunchKernelGGL((fft_axis_kernel<false, 4>), gr, bl, l.lds, st, a); break;
    case 7: hipLaunchKernelGGL((fft_axis_kernel<true, 3>), gr, bl, l.lds, st, a); break;
    case 6: hipLaunchKernelGGL((fft_axis_kernel<false, 3>), gr, bl, l.lds, st, a); break;
    case 1: hipLaunchKernelGGL((fft_axis_kernel<true, 0>), gr, bl, l.lds, st, a); break;
    case 0: hipLaunchKernelGGL((fft_axis_kernel<false, 0>), gr, bl, l.lds, st, a); break;
    case 3: hipLaunchKernelGGL((fft_axis_kernel<true, 1>), gr, bl, l.lds, st, a); break;
    case 2: hipLaunchKernelGGL((fft_axis_kernel<false, 1>), gr, bl, l.lds, st, a); break;
    case 5: hipLaunchKernelGGL((fft_axis_kernel<true, 2>), gr, bl, l.lds, st, a); break;
    default: hipLaunchKernelGGL((fft_axis_kernel<false, 2>), gr, bl, l.lds, st, a); break;
  }
  return hipGetLastError();
}

// Prepared passes of several slices, grouped by kernel variant, FFT_MULTI per launch.
hipError_t fft_multi_launch(const std::vector<FftLaunch>& ls, hipStream_t st) {
  for (int variant = 0; variant < 16; ++variant) {
    FftMulti m;
    std::memset(&m, 0, sizeof(m));
    size_t lds = 0;
    auto flush = [&]() -> hipError_t {
      if (m.n == 0) return hipSuccess;
      const dim3 gr((unsigned)m.start[m.n]), bl(NT);
      switch (variant) {
        case 15: hipLaunchKernelGGL((fft_axis_multi_kernel<true, 7>), gr, bl, lds, st, m); break;
        case 14: hipLaunchKernelGGL((fft_axis_multi_kernel<false, 7>), gr, bl, lds, st, m); break;
        case 13: hipLaunchKernelGGL((fft_axis_multi_kernel<true, 6>), gr, bl, lds, st, m); break;
        case 12: hipLaunchKernelGGL((fft_axis_multi_kernel<false, 6>), gr, bl, lds, st, m); break;
        case 11: hipLaunchKernelGGL((fft_axis_multi_kernel<true, 5>), gr, bl, lds, st, m); break;
        case 10: hipLaunchKernelGGL((fft_axis_multi_kernel<false, 5>), gr, bl, lds, st, m); break;
        case 9: hipLaunchKernelGGL((fft_axis_multi_kernel<true, 4>), gr, bl, lds, st, m); break;
        case 8: hipLaunchKernelGGL((fft_axis_multi_kernel<false, 4>), gr, bl, lds, st, m); break;
        case 7: hipLaunchKernelGGL((fft_axis_multi_kernel<true, 3>), gr, bl, lds, st, m); break;
        case 6: hipLaunchKernelGGL((fft_axis_multi_kernel<false, 3>), gr, bl, lds, st, m); break;
        case 1: hipLaunchKernelGGL((fft_axis_multi_kernel<true, 0>), gr, bl, lds, st, m); break;
        case 0: hipLaunchKernelGGL((fft_axis_multi_kernel<false, 0>), gr, bl, lds, st, m); break;
        case 3: hipLaunchKernelGGL((fft_axis_multi_kernel<true, 1>), gr, bl, lds, st, m); break;
        case 2: hipLaunchKernelGGL((fft_axis_multi_kernel<false, 1>), gr, bl, lds, st, m); break;
        case 5: hipLaunchKernelGGL((fft_axis_multi_kernel<true, 2>), gr, bl, lds, st, m); break;
        default: hipLaunchKernelGGL((fft_axis_multi_kernel<false, 2>), gr, bl, lds, st, m); break;
      }
      hipError_t e = hipGetLastError();
      std::memset(&m, 0, sizeof(m));
      lds = 0;
      return e;
    };
    for (const FftLaunch& l : ls) {
      if (l.smp * 2 + (l.twl ? 1 : 0) != variant || l.blocks <= 0) continue;
      if (m.n == FFT_MULTI || (int64_t)m.start[m.n] + l.blocks > 0x7fffffff) {
        hipError_t e = flush();
        if (e != hipSuccess) return e;
      }
      m.d[m.n] = l.a;
      m.start[m.n + 1] = m.start[m.n] + (int)l.blocks;
      ++m.n;
      if (l.lds > lds) lds = l.lds;
    }
    hipError_t e = flush();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mx
