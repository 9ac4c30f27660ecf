// Third-mode products of the fused path (Sec. II-E, the k-mode product along the readout
// factor U2):
//
//   forward  T3[j][i2][q] = sum_p2 T1[j][q][p2] U2[i2][p2]          q = (p0, p1)
//   adjoint  T1b[j][q][p2] = sum_i2 T3b[j][i2][q] conj(U2[i2][p2])
//
// Per coil both are a skinny product with reduction r2 (forward) or n2 (adjoint) over the
// Q = r0 r1 rows of the coil's slab.  Each wave owns 16 consecutive q of one coil and runs
// all of the small dimension, so the coil's slab is read once and the result written
// once; U2 (fragment order, built per plan) is read from L2.  No LDS: many light waves
// per CU hide the load latency.
#include "mfma_frag.h"
#include "mode3.h"

namespace mx {

namespace {

constexpr int MT = 256;       // four independent waves per workgroup
constexpr int MAX_R2B = 4;    // r2 <= 64

// B fragment of T1_j^T for K16 step s: B(p2, q) = T1[j][q][p2].
template <int PREC>
__device__ __forceinline__ typename Tile<PREC>::B t1_frag(const float2* __restrict__ t1, int Q, int r2, int q, int s,
                                                          int lane) {
  float2 v[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int p2 = 16 * s + 4 * (lane >> 4) + t;
    v[t] = (q < Q && p2 < r2) ? t1[(size_t)q * r2 + p2] : make_float2(0.f, 0.f);
  }
  return Tile<PREC>::make_b(v);
}

template <int PREC>
__global__ __launch_bounds__(MT) void mode3_fwd_kernel(Mode3Args a) {
  const int lane = threadIdx.x & 63;
  const int qbs = (a.Q + 15) / 16;
  const int64_t w = (int64_t)blockIdx.x * (MT / 64) + (threadIdx.x >> 6);
  if (w >= (int64_t)a.J * qbs) return;
  const int j = (int)(w / qbs), qb = (int)(w % qbs);
  const int r2b = (a.r2 + 15) / 16, n2b = (a.n2 + 15) / 16;
  const float2* t1 = a.T1 + (size_t)j * a.Q * a.r2;
  const int qc = 16 * qb + (lane & 15);
  typename Tile<PREC>::B b[MAX_R2B];
#pragma unroll
  for (int s = 0; s < MAX_R2B; ++s)
    if (s < r2b) b[s] = t1_frag<PREC>(t1, a.Q, a.r2, qc, s, lane);
  float2* t3 = a.T3 + (size_t)j * a.n2 * a.Q;
  for (int ib = 0; ib < n2b; ++ib) {
    f32x4 cr = z4(), ci = z4();
#pragma unroll
    for (int s = 0; s < MAX_R2B; ++s)
      if (s < r2b) Tile<PREC>::mma(cr, ci, frag_a<PREC>(a.U2F, r2b, ib, s, lane), b[s]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i2 = 16 * ib + 4 * (lane >> 4) + r;
      if (i2 < a.n2 && qc < a.Q) t3[(size_t)i2 * a.Q + qc] = make_float2(cr[r], ci[r]);
    }
  }
}

template <int PREC>
__global__ __launch_bounds__(MT) void mode3_adj_kernel(Mode3Args a) {
  const int lane = threadIdx.x & 63, grp = lane >> 4;
  const int qbs = (a.Q + 15) / 16;
  const int64_t w = (int64_t)blockIdx.x * (MT / 64) + (threadIdx.x >> 6);
  if (w >= (int64_t)a.J * qbs) return;
  const int j = (int)(w / qbs), qb = (int)(w % qbs);
  const int r2b = (a.r2 + 15) / 16, n2b = (a.n2 + 15) / 16;
  const float2* t3 = a.T3b + (size_t)j * a.n2 * a.Q;
  const int qa = 16 * qb + (lane & 15);
  f32x4 cr[MAX_R2B], ci[MAX_R2B];
#pragma unroll
  for (int nb = 0; nb < MAX_R2B; ++nb) { cr[nb] = z4(); ci[nb] = z4(); }
  for (int s = 0; s < n2b; ++s) {
    // A fragment of T3b_j^T: A(q, i2) = T3b[j][i2][q]
    float2 v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i2 = 16 * s + 4 * grp + t;
      v[t] = (qa < a.Q && i2 < a.n2) ? t3[(size_t)i2 * a.Q + qa] : make_float2(0.f, 0.f);
    }
    const typename Tile<PREC>::A av = Tile<PREC>::make_a(v);
#pragma unroll
    for (int nb = 0; nb < MAX_R2B; ++nb)
      if (nb < r2b) Tile<PREC>::mma(cr[nb], ci[nb], av, frag_b<PREC>(a.U2CF, r2b, nb, s, lane));
  }
  float2* t1 = a.T1b + (size_t)j * a.Q * a.r2;
#pragma unroll
  for (int nb = 0; nb < MAX_R2B; ++nb)
    if (nb < r2b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = 16 * qb + 4 * grp + r, p2 = 16 * nb + (lane & 15);
        if (q < a.Q && p2 < a.r2) t1[(size_t)q * a.r2 + p2] = make_float2(cr[nb][r], ci[nb][r]);
      }
}

}  // namespace

bool mode3_supported(int r2) { return r2 >= 1 && r2 <= 16 * MAX_R2B; }

static dim3 mode3_grid(const Mode3Args& a) {
  const int64_t waves = (int64_t)a.J * ((a.Q + 15) / 16);
  return dim3((unsigned)((waves + MT / 64 - 1) / (MT / 64)));
}

hipError_t mode3_fwd_launch(const Mode3Args& a, int precision, hipStream_t st) {
  if (precision == 1) hipLaunchKernelGGL(mode3_fwd_kernel<1>, mode3_grid(a), dim3(MT), 0, st, a);
  else hipLaunchKernelGGL(mode3_fwd_kernel<0>, mode3_grid(a), dim3(MT), 0, st, a);
  return hipGetLastError();
}

hipError_t mode3_adj_launch(const Mode3Args& a, int precision, hipStream_t st) {
  if (precision == 1) hipLaunchKernelGGL(mode3_adj_kernel<1>, mode3_grid(a), dim3(MT), 0, st, a);
  else hipLaunchKernelGGL(mode3_adj_kernel<0>, mode3_grid(a), dim3(MT), 0, st, a);
  return hipGetLastError();
}

}  // namespace mx
