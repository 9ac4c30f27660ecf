// Dense basis apply and adjoint for few coils: S_j = B c_j (paper Sec. II-B, Eq. (5)) and
// c_j = B^H h_j (the basis block of J_G^H) with B [N][K] row-major, J <= 64 for the apply
// and J <= 16 for the adjoint (the plan chooses; larger J takes the tiled GEMM).  Each
// product streams B once from HBM (J flops per byte, far below the matrix cores' ridge
// point), so the kernels are built for the stream: no LDS staging of B.
//
// Written as S^T = B c^T on 16 x 16 complex tiles (mfma_frag.h): the A operand of a K16 step
// is 16 rows of B, and lane l (row l % 16, group g = l / 16) holds B[n][k0 + 4g .. +3], 32
// contiguous bytes loaded straight into registers; the B operand is c^T, whose fragments are
// built once per call in fragment order (tiny, L2-resident, shared by every wave).  An
// accumulator tile holds S^T[n0 + 4g + r][j0 + l % 16]: each lane writes 4 consecutive n of
// one coil.  Each wave owns RB row blocks (16 RB rows of B) and all coils, and loads the next
// step's B rows before multiplying the current ones.
//
// The adjoint, gc^T[k][j] = sum_n conj(B[n][k]) h[j][n], reduces over the long dimension: the
// A operand (rows k, reduction n) is conj(B) read down four rows per lane (each load of a
// wave covers 128 contiguous bytes of four rows), the B operand is h, 32 contiguous bytes per
// lane.  A workgroup's four waves take four consecutive row chunks of one 64-column group of
// B and add their tiles through LDS; a second kernel sums the workgroup partials over the
// chunks in a fixed order (no atomics).  Workgroups of one row chunk and different
// column groups are dealt to one XCD, so the rows they share are fetched into one L2.
#include "mfma_frag.h"
#include "skinny.h"

#include <algorithm>

namespace mx {

namespace {

constexpr int NT = 256;  // 4 waves per workgroup, independent

// fragment-order B operand of c^T: [step][..][jb][lane], zero beyond J and K
template <int PREC>
__global__ void skinny_cfrag_kernel(const float2* __restrict__ c, int J, int K, int JB, int steps,
                                    void* __restrict__ frag) {
  const int w = blockIdx.x * (NT / 64) + threadIdx.x / 64, lane = threadIdx.x % 64;
  if (w >= steps * JB) return;
  const int s = w / JB, jb = w % JB;
  const int j = jb * 16 + lane % 16, k0 = s * 16 + 4 * (lane / 16);
  float2 v[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) v[t] = (j < J && k0 + t < K) ? c[(int64_t)j * K + k0 + t] : make_float2(0.f, 0.f);
  put_frag_b<PREC>(frag, JB, jb, s, lane, v);
}

template <int PREC, int JB, int RB>
__global__ __launch_bounds__(NT) void skinny_apply_kernel(const float2* __restrict__ B, int64_t N, int K,
                                                          const void* __restrict__ cfrag, int steps, int J,
                                                          float2* __restrict__ S) {
  const int lane = threadIdx.x % 64, g = lane / 16, c16 = lane % 16;
  const int64_t n0 = ((int64_t)blockIdx.x * (NT / 64) + threadIdx.x / 64) * (16 * RB);
  if (n0 >= N) return;
  // this lane's rows (clamped: rows past N are computed and not stored)
  const float2* rowp[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int64_t n = n0 + rb * 16 + c16;
    rowp[rb] = B + (n < N ? n : N - 1) * K;
  }
  f32x4 cr[RB][JB], ci[RB][JB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) { cr[rb][jb] = z4(); ci[rb][jb] = z4(); }
  // raw[rb] = B[row][k0 .. k0 + 4) of step s (zero past K; K is a multiple of 4)
  auto fetch = [&](float4 (&raw)[RB][2], int s) {
    const int k = s * 16 + 4 * g;
    const bool ok = k < K;
    const uint32_t m = ok ? 0xffffffffu : 0u;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const float4* p = reinterpret_cast<const float4*>(rowp[rb] + (ok ? k : 0));
      float4 a = p[0], b = p[1];
      a = make_float4(__uint_as_float(__float_as_uint(a.x) & m), __uint_as_float(__float_as_uint(a.y) & m),
                      __uint_as_float(__float_as_uint(a.z) & m), __uint_as_float(__float_as_uint(a.w) & m));
      b = make_float4(__uint_as_float(__float_as_uint(b.x) & m), __uint_as_float(__float_as_uint(b.y) & m),
                      __uint_as_float(__float_as_uint(b.z) & m), __uint_as_float(__float_as_uint(b.w) & m));
      raw[rb][0] = a;
      raw[rb][1] = b;
    }
  };
  auto compute = [&](const float4 (&raw)[RB][2], int s) {
    typename Tile<PREC>::B bf[JB];
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) bf[jb] = frag_b<PREC>(cfrag, JB, jb, s, lane);
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const float2 v[4] = {make_float2(raw[rb][0].x, raw[rb][0].y), make_float2(raw[rb][0].z, raw[rb][0].w),
                           make_float2(raw[rb][1].x, raw[rb][1].y), make_float2(raw[rb][1].z, raw[rb][1].w)};
      const typename Tile<PREC>::A a = Tile<PREC>::make_a(v);
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) Tile<PREC>::mma(cr[rb][jb], ci[rb][jb], a, bf[jb]);
    }
  };
  float4 r0[RB][2], r1[RB][2];
  fetch(r0, 0);
  int s = 0;
  for (; s + 2 <= steps; s += 2) {
    fetch(r1, s + 1);
    compute(r0, s);
    if (s + 2 < steps) fetch(r0, s + 2);
    compute(r1, s + 1);
  }
  if (s < steps) compute(r0, s);
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) {
      const int j = jb * 16 + c16;
      if (j >= J) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t n = n0 + rb * 16 + 4 * g + r;
        if (n < N) S[(int64_t)j * N + n] = make_float2(cr[rb][jb][r], ci[rb][jb][r]);
      }
    }
}

template <int PREC, int JB>
hipError_t launch_jb(const float2* B, int64_t N, int K, const void* frag, int steps, int J, float2* S, hipStream_t st) {
  constexpr int RB = 4;
  const int64_t waves = (N + 16 * RB - 1) / (16 * RB);
  const unsigned blocks = (unsigned)((waves + NT / 64 - 1) / (NT / 64));
  hipLaunchKernelGGL((skinny_apply_kernel<PREC, JB, RB>), dim3(blocks), dim3(NT), 0, st, B, N, K, frag, steps, J, S);
  return hipGetLastError();
}

// ---- adjoint
constexpr int AKB = 4;  // 16-column blocks of B per wave (a 64-column group)

template <int PREC, int JB>
__global__ __launch_bounds__(NT) void skinny_adjoint_kernel(const float2* __restrict__ B, int64_t N, int K,
                                                            const float2* __restrict__ h, int J, int64_t chunk,
                                                            int nchunk, int kgroups, float2* __restrict__ part) {
  __shared__ f32x4 red[3][AKB][JB][2][64];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64, g = lane / 16, c16 = lane % 16;
  // XCD-aware order: the column groups of one row chunk on one XCD
  const int xcd = blockIdx.x % 8, i = blockIdx.x / 8;
  const int kg = i % kgroups, ch = 8 * (i / kgroups) + xcd;
  if (ch >= nchunk) return;  // the whole workgroup leaves together (no barrier reached)
  const int k0 = kg * 16 * AKB;
  // this wave's rows: the quarter `wave` of the chunk, in 16-row steps
  const int64_t q = (chunk / 4 + 15) / 16 * 16;
  const int64_t r0 = (int64_t)ch * chunk + wave * q;
  const int64_t r1 = min(min(r0 + q, (int64_t)ch * chunk + chunk), N);
  f32x4 cr[AKB][JB], ci[AKB][JB];
#pragma unroll
  for (int kb = 0; kb < AKB; ++kb)
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) { cr[kb][jb] = z4(); ci[kb][jb] = z4(); }
  for (int64_t n = r0; n < r1; n += 16) {
    // B operand: h[j][n + 4g .. +3] (zero past N or J)
    typename Tile<PREC>::B hb[JB];
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) {
      const int j = jb * 16 + c16;
      float2 v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t nn = n + 4 * g + t;
        const bool ok = j < J && nn < r1;
        const float2 x = h[(ok ? (int64_t)j * N + nn : 0)];
        v[t] = ok ? x : make_float2(0.f, 0.f);
      }
      hb[jb] = Tile<PREC>::make_b(v);
    }
    // A operand: conj(B[n + 4g + t][k]) for the lane's column k = k0 + 16 kb + c16
#pragma unroll
    for (int kb = 0; kb < AKB; ++kb) {
      const int k = k0 + 16 * kb + c16;
      float2 v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t nn = n + 4 * g + t;
        const bool ok = k < K && nn < r1;
        const float2 x = B[(ok ? nn * K + k : 0)];
        v[t] = ok ? make_float2(x.x, -x.y) : make_float2(0.f, 0.f);
      }
      const typename Tile<PREC>::A a = Tile<PREC>::make_a(v);
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) Tile<PREC>::mma(cr[kb][jb], ci[kb][jb], a, hb[jb]);
    }
  }
  // waves 1..3 hand their tiles to wave 0, which adds them in wave order
  if (wave > 0) {
#pragma unroll
    for (int kb = 0; kb < AKB; ++kb)
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) {
        red[wave - 1][kb][jb][0][lane] = cr[kb][jb];
        red[wave - 1][kb][jb][1][lane] = ci[kb][jb];
      }
  }
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int kb = 0; kb < AKB; ++kb)
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) {
      f32x4 sr = cr[kb][jb], si = ci[kb][jb];
      for (int w = 0; w < 3; ++w) {
        sr += red[w][kb][jb][0][lane];
        si += red[w][kb][jb][1][lane];
      }
      const int j = jb * 16 + c16;
      if (j >= J) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = k0 + 16 * kb + 4 * g + r;
        if (k < K) part[((int64_t)ch * J + j) * K + k] = make_float2(sr[r], si[r]);
      }
    }
}

// out[j][k] = s * sum over chunks of part[chunk][j][k], s = alpha (* alpha_dev).  RG threads
// per output each sum every RG-th chunk in four interleaved chains, and the RG sums are added
// through LDS in a fixed order: the result does not depend on timing.
constexpr int RG = 16;
__global__ __launch_bounds__(NT) void skinny_reduce_kernel(const float2* __restrict__ part, int nchunk, int64_t JK,
                                                           float alpha, const float* __restrict__ alpha_dev,
                                                           float2* __restrict__ out) {
  constexpr int OPB = NT / RG;
  __shared__ float2 red[RG][OPB];
  const int lo = threadIdx.x % OPB, grp = threadIdx.x / OPB;
  const int64_t e = (int64_t)blockIdx.x * OPB + lo;
  float2 a0 = make_float2(0.f, 0.f), a1 = a0, a2 = a0, a3 = a0;
  if (e < JK) {
    int c = grp;
    for (; c + 3 * RG < nchunk; c += 4 * RG) {
      a0 = cadd(a0, part[(int64_t)c * JK + e]);
      a1 = cadd(a1, part[(int64_t)(c + RG) * JK + e]);
      a2 = cadd(a2, part[(int64_t)(c + 2 * RG) * JK + e]);
      a3 = cadd(a3, part[(int64_t)(c + 3 * RG) * JK + e]);
    }
    for (; c < nchunk; c += RG) a0 = cadd(a0, part[(int64_t)c * JK + e]);
  }
  red[grp][lo] = cadd(cadd(a0, a1), cadd(a2, a3));
  __syncthreads();
  if (grp != 0 || e >= JK) return;
  float2 v = red[0][lo];
  for (int q = 1; q < RG; ++q) v = cadd(v, red[q][lo]);
  float sc = alpha;
  if (alpha_dev) sc *= *alpha_dev;
  out[e] = cscale(v, sc);
}

template <int PREC, int JB>
hipError_t launch_adj(const float2* B, int64_t N, int K, const float2* h, int J, int64_t chunk, int nchunk,
                      int kgroups, float2* part, hipStream_t st) {
  const int64_t wg = (int64_t)((nchunk + 7) / 8) * 8 * kgroups;
  hipLaunchKernelGGL((skinny_adjoint_kernel<PREC, JB>), dim3((unsigned)wg), dim3(NT), 0, st, B, N, K, h, J, chunk,
                     nchunk, kgroups, part);
  return hipGetLastError();
}

// row chunks: about 1024 workgroups in all, each chunk a multiple of 64 rows
void adjoint_geometry(int64_t N, int64_t K, int64_t& chunk, int& nchunk, int& kgroups) {
  kgroups = (int)((K + 16 * AKB - 1) / (16 * AKB));
  int64_t want = 1024 / kgroups;
  if (want < 8) want = 8;
  chunk = (N + want - 1) / want;
  chunk = (chunk + 63) / 64 * 64;
  nchunk = (int)((N + chunk - 1) / chunk);
}

}  // namespace

size_t skinny_adjoint_bytes(int64_t N, int64_t K, int J) {
  int64_t chunk;
  int nchunk, kgroups;
  adjoint_geometry(N, K, chunk, nchunk, kgroups);
  return (size_t)nchunk * (size_t)J * (size_t)K * sizeof(float2);
}

hipError_t skinny_adjoint_launch(const float2* B, int64_t N, int64_t K, const float2* h, int J, int precision,
                                 float alpha, const float* alpha_dev, void* ws, float2* c, hipStream_t st) {
  int64_t chunk;
  int nchunk, kgroups;
  adjoint_geometry(N, K, chunk, nchunk, kgroups);
  float2* part = reinterpret_cast<float2*>(ws);
  const int JB = (J + 15) / 16;
  hipError_t e;
  switch (JB * 2 + (precision == 1 ? 1 : 0)) {
    case 3: e = launch_adj<1, 1>(B, N, (int)K, h, J, chunk, nchunk, kgroups, part, st); break;
    case 2: e = launch_adj<0, 1>(B, N, (int)K, h, J, chunk, nchunk, kgroups, part, st); break;
    case 5: e = launch_adj<1, 2>(B, N, (int)K, h, J, chunk, nchunk, kgroups, part, st); break;
    case 4: e = launch_adj<0, 2>(B, N, (int)K, h, J, chunk, nchunk, kgroups, part, st); break;
    case 7: e = launch_adj<1, 3>(B, N, (int)K, h, J, chunk, nchunk, kgroups, part, st); break;
    case 6: e = launch_adj<0, 3>(B, N, (int)K, h, J, chunk, nchunk, kgroups, part, st); break;
    case 9: e = launch_adj<1, 4>(B, N, (int)K, h, J, chunk, nchunk, kgroups, part, st); break;
    default: e = launch_adj<0, 4>(B, N, (int)K, h, J, chunk, nchunk, kgroups, part, st); break;
  }
  if (e != hipSuccess) return e;
  const int64_t JK = (int64_t)J * K;
  const unsigned rb = (unsigned)((JK + NT / RG - 1) / (NT / RG));
  hipLaunchKernelGGL(skinny_reduce_kernel, dim3(rb), dim3(NT), 0, st, part, nchunk, JK, alpha, alpha_dev, c);
  return hipGetLastError();
}

bool skinny_apply_supported(int64_t N, int64_t K, int J) { return N > 0 && K > 0 && K % 4 == 0 && J >= 1 && J <= 64; }

size_t skinny_frag_bytes(int64_t K, int J) {
  const int64_t steps = (K + 15) / 16, JB = (J + 15) / 16;
  return (size_t)(steps * JB) * 4 * 1024;  // BF16: 4 arrays of 1 KiB per fragment; FP32: 2 KiB
}

hipError_t skinny_apply_launch(const float2* B, int64_t N, int64_t K, const float2* c, int J, int precision,
                               void* frag, float2* S, hipStream_t st) {
  const int steps = (int)((K + 15) / 16), JB = (J + 15) / 16;
  const unsigned fb = (unsigned)((steps * JB + NT / 64 - 1) / (NT / 64));
  if (precision == 1)
    hipLaunchKernelGGL(skinny_cfrag_kernel<1>, dim3(fb), dim3(NT), 0, st, c, J, (int)K, JB, steps, frag);
  else
    hipLaunchKernelGGL(skinny_cfrag_kernel<0>, dim3(fb), dim3(NT), 0, st, c, J, (int)K, JB, steps, frag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (JB * 2 + (precision == 1 ? 1 : 0)) {
    case 3: return launch_jb<1, 1>(B, N, (int)K, frag, steps, J, S, st);
    case 2: return launch_jb<0, 1>(B, N, (int)K, frag, steps, J, S, st);
    case 5: return launch_jb<1, 2>(B, N, (int)K, frag, steps, J, S, st);
    case 4: return launch_jb<0, 2>(B, N, (int)K, frag, steps, J, S, st);
    case 7: return launch_jb<1, 3>(B, N, (int)K, frag, steps, J, S, st);
    case 6: return launch_jb<0, 3>(B, N, (int)K, frag, steps, J, S, st);
    case 9: return launch_jb<1, 4>(B, N, (int)K, frag, steps, J, S, st);
    default: return launch_jb<0, 4>(B, N, (int)K, frag, steps, J, S, st);
  }
}

}  // namespace mx
