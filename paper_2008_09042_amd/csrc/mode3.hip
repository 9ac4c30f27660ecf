// Third-mode products of the fused path (Sec. II-E, the k-mode product along the readout
// factor U2):
//
//   forward  T3[j][i2][q] = sum_p2 T1[j][q][p2] U2[i2][p2]          q = (p0, p1)
//   adjoint  T1b[j][q][p2] = sum_i2 T3b[j][i2][q] conj(U2[i2][p2])
//
// Per coil both are a skinny product with reduction r2 (forward) or n2 (adjoint) over the
// Q = r0 r1 rows of the coil's slab.  Each wave owns QB blocks of 16 consecutive q of one
// coil and runs all of the small dimension, so the coil's slab is read once and the result
// written once; U2 (fragment order, built per plan) is read from L2, one step ahead of its
// use.  No LDS: many light waves per CU hide the load latency.
#include "mfma_frag.h"
#include "mode3.h"

namespace mx {

namespace {

constexpr int MT = 256;       // four independent waves per workgroup
constexpr int MAX_R2B = 4;    // r2 <= 64

// Loads are unconditional (clamped into the operand, the value zeroed past its end): a load
// under a branch makes the compiler wait for every load in flight before the next one.

// B fragment of T1_j^T for K16 step s: B(p2, q) = T1[j][q][p2].
template <int PREC>
__device__ __forceinline__ typename Tile<PREC>::B t1_frag(const float2* __restrict__ t1, int Q, int r2, int q, int s,
                                                          int lane) {
  float2 v[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int p2 = 16 * s + 4 * (lane >> 4) + t;
    const float m = (q < Q && p2 < r2) ? 1.f : 0.f;
    const float2 x = t1[(size_t)min(q, Q - 1) * r2 + min(p2, r2 - 1)];
    v[t] = make_float2(x.x * m, x.y * m);
  }
  return Tile<PREC>::make_b(v);
}

// U2 fragments of output block ib (clamped to the last block)
template <int PREC, int R2B>
__device__ __forceinline__ void u2_frags(const void* u2f, int n2b, int ib, int lane,
                                         typename Tile<PREC>::A (&u)[R2B]) {
  ib = min(ib, n2b - 1);
#pragma unroll
  for (int s = 0; s < R2B; ++s) u[s] = frag_a<PREC>(u2f, R2B, ib, s, lane);
}

// Each wave takes QB blocks of 16 q, so every U2 fragment it loads (from L2) serves QB
// products: the fragments, not the slabs, dominate the kernels' cache traffic.

// T3[j][16 ib + i][q] for the wave's QB x 16 q: a block past the last is computed, not stored
template <int PREC, int R2B, int QB>
__device__ __forceinline__ void fwd_block(const Mode3Args& a, float2* t3, int ib, const int (&qc)[QB], int lane,
                                          const typename Tile<PREC>::A (&u)[R2B],
                                          const typename Tile<PREC>::B (&b)[QB][R2B]) {
#pragma unroll
  for (int h = 0; h < QB; ++h) {
    // accumulator form: three real products per complex product in FP32
    typename Tile<PREC>::Acc c = Tile<PREC>::zero();
#pragma unroll
    for (int s = 0; s < R2B; ++s) Tile<PREC>::mma(c, u[s], b[h][s]);
    f32x4 cr, ci;
    Tile<PREC>::finish(c, cr, ci);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i2 = 16 * ib + 4 * (lane >> 4) + r;
      if (i2 < a.n2 && qc[h] < a.Q) t3[(size_t)i2 * a.Q + qc[h]] = make_float2(cr[r], ci[r]);
    }
  }
}

template <int PREC, int R2B, int QB>
__global__ __launch_bounds__(MT) void mode3_fwd_kernel(Mode3Args a) {
  const int lane = threadIdx.x & 63;
  const int qws = ((a.Q + 15) / 16 + QB - 1) / QB;  // q groups of QB blocks
  const int64_t w = (int64_t)blockIdx.x * (MT / 64) + (threadIdx.x >> 6);
  if (w >= (int64_t)a.J * qws) return;
  const int j = (int)(w / qws), qg = (int)(w % qws);
  const int n2b = (a.n2 + 15) / 16;
  const float2* t1 = a.T1 + (size_t)j * a.Q * a.r2;
  int qc[QB];
  typename Tile<PREC>::B b[QB][R2B];
#pragma unroll
  for (int h = 0; h < QB; ++h) {
    qc[h] = 16 * (QB * qg + h) + (lane & 15);
#pragma unroll
    for (int s = 0; s < R2B; ++s) b[h][s] = t1_frag<PREC>(t1, a.Q, a.r2, qc[h], s, lane);
  }
  float2* t3 = a.T3 + (size_t)j * a.n2 * a.Q;
  // the next block's U2 fragments load during this block's products: two buffers, the loop
  // unrolled by two so that each keeps its own registers
  typename Tile<PREC>::A u0[R2B], u1[R2B];
  u2_frags<PREC, R2B>(a.U2F, n2b, 0, lane, u0);
  for (int ib = 0; ib < n2b; ib += 2) {
    u2_frags<PREC, R2B>(a.U2F, n2b, ib + 1, lane, u1);
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
    fwd_block<PREC, R2B, QB>(a, t3, ib, qc, lane, u0, b);
    u2_frags<PREC, R2B>(a.U2F, n2b, ib + 2, lane, u0);
    __builtin_amdgcn_sched_barrier(0);
    fwd_block<PREC, R2B, QB>(a, t3, ib + 1, qc, lane, u1, b);
  }
}

// One reduction step of the adjoint: the lane's values of the A fragments of T3b_j^T,
// A(q, i2) = T3b[j][i2][q], for the wave's QB q blocks, zero past n2 or Q (a step past the
// last adds nothing), and the conj(U2) fragments of the step (clamped to the last step).
template <int PREC, int R2B, int QB>
struct AdjStep {
  float2 v[QB][4];
  typename Tile<PREC>::B u[R2B];
};

template <int PREC, int R2B, int QB>
__device__ __forceinline__ void adj_step_load(const Mode3Args& a, const float2* t3, int n2b, int s,
                                              const int (&qa)[QB], int lane, AdjStep<PREC, R2B, QB>& st) {
  const int grp = lane >> 4;
#pragma unroll
  for (int h = 0; h < QB; ++h)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i2 = 16 * s + 4 * grp + t;
      const float m = (qa[h] < a.Q && i2 < a.n2) ? 1.f : 0.f;
      const float2 x = t3[(size_t)min(i2, a.n2 - 1) * a.Q + min(qa[h], a.Q - 1)];
      st.v[h][t] = make_float2(x.x * m, x.y * m);
    }
  const int sc = min(s, n2b - 1);
#pragma unroll
  for (int nb = 0; nb < R2B; ++nb) st.u[nb] = frag_b<PREC>(a.U2CF, R2B, nb, sc, lane);
}

template <int PREC, int R2B, int QB>
__device__ __forceinline__ void adj_step_mma(const AdjStep<PREC, R2B, QB>& st,
                                             typename Tile<PREC>::Acc (&c)[QB][R2B]) {
#pragma unroll
  for (int h = 0; h < QB; ++h) {
    const typename Tile<PREC>::A av = Tile<PREC>::make_a(st.v[h]);
#pragma unroll
    for (int nb = 0; nb < R2B; ++nb) Tile<PREC>::mma(c[h][nb], av, st.u[nb]);
  }
}

template <int PREC, int R2B, int QB>
__global__ __launch_bounds__(MT) void mode3_adj_kernel(Mode3Args a) {
  const int lane = threadIdx.x & 63, grp = lane >> 4;
  const int qws = ((a.Q + 15) / 16 + QB - 1) / QB;
  const int64_t w = (int64_t)blockIdx.x * (MT / 64) + (threadIdx.x >> 6);
  if (w >= (int64_t)a.J * qws) return;
  const int j = (int)(w / qws), qg = (int)(w % qws);
  const int n2b = (a.n2 + 15) / 16;
  const float2* t3 = a.T3b + (size_t)j * a.n2 * a.Q;
  int qa[QB];
#pragma unroll
  for (int h = 0; h < QB; ++h) qa[h] = 16 * (QB * qg + h) + (lane & 15);
  typename Tile<PREC>::Acc c[QB][R2B];  // accumulator form (three real products in FP32)
#pragma unroll
  for (int h = 0; h < QB; ++h)
#pragma unroll
    for (int nb = 0; nb < R2B; ++nb) c[h][nb] = Tile<PREC>::zero();
  // the next step's loads are in flight during this step's products (two buffers, the loop
  // unrolled by two)
  AdjStep<PREC, R2B, QB> s0, s1;
  adj_step_load<PREC, R2B, QB>(a, t3, n2b, 0, qa, lane, s0);
  for (int s = 0; s < n2b; s += 2) {
    adj_step_load<PREC, R2B, QB>(a, t3, n2b, s + 1, qa, lane, s1);
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
    adj_step_mma<PREC, R2B, QB>(s0, c);
    adj_step_load<PREC, R2B, QB>(a, t3, n2b, s + 2, qa, lane, s0);
    __builtin_amdgcn_sched_barrier(0);
    adj_step_mma<PREC, R2B, QB>(s1, c);
  }
  float2* t1 = a.T1b + (size_t)j * a.Q * a.r2;
#pragma unroll
  for (int h = 0; h < QB; ++h)
#pragma unroll
    for (int nb = 0; nb < R2B; ++nb) {
      f32x4 cr, ci;
      Tile<PREC>::finish(c[h][nb], cr, ci);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = 16 * (QB * qg + h) + 4 * grp + r, p2 = 16 * nb + (lane & 15);
        if (q < a.Q && p2 < a.r2) t1[(size_t)q * a.r2 + p2] = make_float2(cr[r], ci[r]);
      }
    }
}

}  // namespace

bool mode3_supported(int r2) { return r2 >= 1 && r2 <= 16 * MAX_R2B; }

static dim3 mode3_grid(const Mode3Args& a, int QB) {
  const int64_t waves = (int64_t)a.J * (((a.Q + 15) / 16 + QB - 1) / QB);
  return dim3((unsigned)((waves + MT / 64 - 1) / (MT / 64)));
}

// q blocks per wave, measured at Q = 1600, r2 = 40, n2 = 128, 32 coils (BF16-split / FP32,
// us per launch): forward 18.5 with two / 21.9 with one, FP32 35.1 / 31.6 (its products,
// at 32 cycles per FP32 MFMA, outweigh the fragment traffic); adjoint 25.7 / 25.6 and FP32
// 32.4 / 31.6.
template <int PREC, int R2B>
static void mode3_launch_r(const Mode3Args& a, bool adj, hipStream_t st) {
  constexpr int QF = PREC == 1 ? 2 : 1;
  const dim3 b(MT);
  if (adj) hipLaunchKernelGGL((mode3_adj_kernel<PREC, R2B, 1>), mode3_grid(a, 1), b, 0, st, a);
  else hipLaunchKernelGGL((mode3_fwd_kernel<PREC, R2B, QF>), mode3_grid(a, QF), b, 0, st, a);
}

template <int PREC>
static void mode3_launch_prec(const Mode3Args& a, bool adj, hipStream_t st) {
  switch ((a.r2 + 15) / 16) {  // rank blocks of 16, known at compile time
    case 1: mode3_launch_r<PREC, 1>(a, adj, st); break;
    case 2: mode3_launch_r<PREC, 2>(a, adj, st); break;
    case 3: mode3_launch_r<PREC, 3>(a, adj, st); break;
    default: mode3_launch_r<PREC, 4>(a, adj, st); break;
  }
}

hipError_t mode3_fwd_launch(const Mode3Args& a, int precision, hipStream_t st) {
  if (!mode3_supported(a.r2) || a.Q < 1 || a.n2 < 1) return hipErrorInvalidValue;
  if (precision == 1) mode3_launch_prec<1>(a, false, st);
  else mode3_launch_prec<0>(a, false, st);
  return hipGetLastError();
}

hipError_t mode3_adj_launch(const Mode3Args& a, int precision, hipStream_t st) {
  if (!mode3_supported(a.r2) || a.Q < 1 || a.n2 < 1) return hipErrorInvalidValue;
  if (precision == 1) mode3_launch_prec<1>(a, true, st);
  else mode3_launch_prec<0>(a, true, st);
  return hipGetLastError();
}

}  // namespace mx
