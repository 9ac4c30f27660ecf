// Tucker core contractions of the fused path.  The core is the fourth-mode factor of
// the basis (Sec. II-E), so B c_j starts with core x_4 c_j, and the coefficient block
// of the adjoint Jacobian (Sec. II-B) ends with the adjoint of that product:
//
//   forward  T1[j][rho] = sum_k core[rho][k] c[j][k]              rho = (p0, p1, p2)
//   adjoint  gc[j][k]   = s * sum_rho conj(core[rho][k]) T1b[j][rho]
//
// Both stream the core (R x K complex) from HBM once per call, as the matrix-core A
// operand.
//
// BF16-split kernels: real-block form over 2K on v_mfma_f32_16x16x32_bf16, six products
// per complex tile (hi*hi, hi*lo, lo*hi for the real and imaginary parts).  The core's
// hi / lo planes are built once per plan in fragment order (row-major for the forward,
// conjugate-transposed for the adjoint).  Waves are independent: each loads its core
// fragments and its lanes' entries of the small per-call operand (c or T1b, L2-resident)
// itself, FD reduction steps ahead, and splits the latter in registers.  No LDS and no
// barriers, so the loads of several steps stay in flight.
// FP32 kernels: v_mfma_f32_16x16x4_f32 in the same independent-wave form, over FP32 core
// copies in fragment order built once per plan, with three real products per complex
// product (Tile<0>::Acc).  (The kernels that read the caller's core directly, four real
// products per complex product with the per-call operand staged through LDS, remain for
// plans built without the copies.)  The adjoint reduces over rho in chunks whose partials
// are summed in a fixed order.
#include "../../include/maxwell.h"
#include "core.h"
#include "mfma_frag.h"

namespace mx {

namespace {

constexpr int NT = 256;     // four waves
constexpr int MAXNB = 4;    // coil blocks of 16: J <= 64
constexpr int RB = 2;       // FP32 kernels: row blocks of 16 per wave
constexpr int RC = 512;     // adjoint: rho per workgroup chunk
// BF16-split kernels: reduction steps whose loads are in flight, and row blocks per wave
// (more rows per load of the per-call operand where the accumulators of NB coil blocks
// leave room).  Measured at R = 64000, K = 300, J = 32.
constexpr int FWD_FD = 2, ADJ_FD = 3;
constexpr int FWD_RB_FEW = 4, FWD_RB_MANY = 2;  // NB <= 2, NB > 2
constexpr int ADJ_RB_FEW = 3, ADJ_RB_MANY = 2;

// Lane operand of the per-call matrix src [rows][len] for one K16 step starting at e0:
// src[j][e0 + 4 g + t], t < 4, j = 16 cb + lane % 16.  Rows past the last and entries
// past len are clamped into the matrix; they meet zero core entries or are not stored.
template <int NB>
__device__ __forceinline__ void call_operand(const float2* const (&row)[NB], int64_t e0, int64_t len, int grp,
                                             float2 (&v)[NB][4]) {
#pragma unroll
  for (int cb = 0; cb < NB; ++cb)
#pragma unroll
    for (int t = 0; t < 4; ++t) v[cb][t] = row[cb][min(e0 + 4 * grp + t, len - 1)];
}

// ---------------------------------------------------------------- forward, BF16-split
// One wave: RB row blocks (16 RB rho) against all NB coil blocks.
template <int NB, int RB, int FD = FWD_FD>
__global__ __launch_bounds__(NT) void core_fwd_bf16_kernel(CoreArgs a) {
  const int lane = threadIdx.x & 63, grp = lane >> 4;
  const int steps = a.g.KP / 32;
  const int64_t rbs = (a.g.R + 15) / 16;
  const int64_t rb0 = ((int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6)) * RB;
  if (rb0 >= rbs) return;
  int64_t oa[RB];
#pragma unroll
  for (int m = 0; m < RB; ++m) oa[m] = min(rb0 + m, rbs - 1) * 512 + lane * 8;
  const float2* row[NB];
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) row[cb] = a.in + (int64_t)min(16 * cb + (lane & 15), a.J - 1) * a.g.K;
  u16x8 ah[FD][RB], al[FD][RB];
  float2 bv[FD][NB][4];
  auto load = [&](int d, int s) {
    s = min(s, steps - 1);
#pragma unroll
    for (int m = 0; m < RB; ++m) {
      ah[d][m] = ld8(a.fwd_hi + oa[m] + (int64_t)s * rbs * 512);
      al[d][m] = ld8(a.fwd_lo + oa[m] + (int64_t)s * rbs * 512);
    }
    call_operand<NB>(row, 16 * (int64_t)s, a.g.K, grp, bv[d]);
  };
  f32x4 cr[RB][NB], ci[RB][NB];
#pragma unroll
  for (int m = 0; m < RB; ++m)
#pragma unroll
    for (int c = 0; c < NB; ++c) { cr[m][c] = z4(); ci[m][c] = z4(); }
  auto compute = [&](int d) {
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const Tile<1>::B b = Tile<1>::make_b(bv[d][c]);
#pragma unroll
      for (int m = 0; m < RB; ++m) mfma6(cr[m][c], ci[m][c], ah[d][m], al[d][m], b.rh, b.rl, b.ih, b.il);
    }
  };
  // FD stages in flight; the issue order of the stages' loads is kept, so the wait before
  // a stage's products only covers that stage's loads.
#pragma unroll
  for (int d = 0; d < FD; ++d) load(d, d);
  int s0 = 0;
  for (; s0 + FD <= steps; s0 += FD) {
#pragma unroll
    for (int d = 0; d < FD; ++d) {
      compute(d);
      load(d, s0 + d + FD);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int d = 0; d + 1 < FD; ++d)
    if (s0 + d < steps) compute(d);
  // D rows are rho, columns coils: T1[j][rho]
#pragma unroll
  for (int m = 0; m < RB; ++m)
#pragma unroll
    for (int c = 0; c < NB; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t rw = 16 * (rb0 + m) + 4 * grp + r;
        const int j = 16 * c + (lane & 15);
        if (rw < a.g.R && j < a.J) a.out[(int64_t)j * a.g.R + rw] = make_float2(cr[m][c][r], ci[m][c][r]);
      }
}

// ---------------------------------------------------------------- FP32, fragment order
// The FP32 core copies: A operands in fragment order, [K16 step][row block][lane][4 complex]
// (frag_a<0> with the step as its outer index; the adjoint's steps grouped by rho chunk as in
// the BF16 planes).  Forward: A(rho, k) = core[rho][k], (R + 15) / 16 row blocks x Kp / 16 steps.
// Adjoint: A(k, rho) = conj(core[rho][k]), Kp / 16 row blocks x Rp / 16 steps.  Zero past R
// and K.
__global__ void core_frag32_kernel(const float2* __restrict__ core, int64_t R, int K, int adj, int64_t nrb,
                                   int64_t steps, float4* __restrict__ dst) {
  const int64_t total = nrb * steps * 64;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    // step-major, as the BF16 planes: forward [step][row block], adjoint [step within a rho
    // chunk of RC][chunk][k row block]
    const int64_t idx = e / 64, rb = idx % nrb, t = idx / nrb;
    const int64_t st = !adj ? t : (t % (steps / (RC / 16))) * (RC / 16) + t / (steps / (RC / 16));
    const int lane = (int)(e % 64);
    const int64_t row = 16 * rb + lane % 16;
    float2 v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t kk = 16 * st + 4 * (lane / 16) + t;
      v[t] = make_float2(0.f, 0.f);
      if (!adj) {
        if (row < R && kk < K) v[t] = core[row * K + kk];
      } else if (row < K && kk < R) {
        v[t] = cconj(core[kk * K + row]);
      }
    }
    dst[2 * e] = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
    dst[2 * e + 1] = make_float4(v[2].x, v[2].y, v[3].x, v[3].y);
  }
}

// One wave: RB row blocks (16 RB rho) against all NB coil blocks, FD steps of loads in flight.
template <int NB, int RB, int FD = FWD_FD>
__global__ __launch_bounds__(NT) void core_fwd_f32f_kernel(CoreArgs a) {
  const int lane = threadIdx.x & 63, grp = lane >> 4;
  const int steps = a.g.Kp / 16;
  const int64_t rbs = (a.g.R + 15) / 16;
  const int64_t rb0 = ((int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6)) * RB;
  if (rb0 >= rbs) return;
  int64_t rbm[RB];
#pragma unroll
  for (int m = 0; m < RB; ++m) rbm[m] = min(rb0 + m, rbs - 1);
  const float2* row[NB];
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) row[cb] = a.in + (int64_t)min(16 * cb + (lane & 15), a.J - 1) * a.g.K;
  Tile<0>::A av[FD][RB];
  float2 bv[FD][NB][4];
  auto load = [&](int d, int s) {
    s = min(s, steps - 1);
#pragma unroll
    for (int m = 0; m < RB; ++m) av[d][m] = frag_a<0>(a.fwd_f32, (int)rbs, s, (int)rbm[m], lane);  // step-major
    call_operand<NB>(row, 16 * (int64_t)s, a.g.K, grp, bv[d]);
  };
  Tile<0>::Acc acc[RB][NB];
#pragma unroll
  for (int m = 0; m < RB; ++m)
#pragma unroll
    for (int c = 0; c < NB; ++c) acc[m][c] = Tile<0>::zero();
  auto compute = [&](int d) {
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const Tile<0>::B b = Tile<0>::make_b(bv[d][c]);
#pragma unroll
      for (int m = 0; m < RB; ++m) Tile<0>::mma(acc[m][c], av[d][m], b);
    }
  };
#pragma unroll
  for (int d = 0; d < FD; ++d) load(d, d);
  int s0 = 0;
  for (; s0 + FD <= steps; s0 += FD) {
#pragma unroll
    for (int d = 0; d < FD; ++d) {
      compute(d);
      load(d, s0 + d + FD);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int d = 0; d + 1 < FD; ++d)
    if (s0 + d < steps) compute(d);
#pragma unroll
  for (int m = 0; m < RB; ++m)
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      f32x4 cr, ci;
      Tile<0>::finish(acc[m][c], cr, ci);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t rw = 16 * (rb0 + m) + 4 * grp + r;
        const int j = 16 * c + (lane & 15);
        if (rw < a.g.R && j < a.J) a.out[(int64_t)j * a.g.R + rw] = make_float2(cr[r], ci[r]);
      }
    }
}

// Adjoint: one rho chunk of RC per workgroup and RB k row blocks per wave (workgroups of one
// chunk on one XCD, as in the BF16-split kernel); partials per chunk, summed afterwards.
// Launched with two steps in flight (the three-product accumulators take the registers of
// the third).
template <int NB, int RB, int FD = ADJ_FD>
__global__ __launch_bounds__(NT) void core_adj_f32f_kernel(CoreArgs a, int nch, int kgroups) {
  const int xcd = blockIdx.x % 8, i = blockIdx.x / 8;
  const int ky = i % kgroups, ch = 8 * (i / kgroups) + xcd;
  const int lane = threadIdx.x & 63, grp = lane >> 4, wave = threadIdx.x >> 6;
  const int mbl = a.g.Kp / 16;
  const int mb0 = ky * (4 * RB) + wave * RB;
  if (ch >= nch || mb0 >= mbl) return;
  const int64_t rho0 = (int64_t)ch * RC;
  const int steps_total = (int)(a.g.Rp / 16);
  constexpr int steps = RC / 16;
  int mbm[RB];
#pragma unroll
  for (int m = 0; m < RB; ++m) mbm[m] = min(mb0 + m, mbl - 1);
  const float2* row[NB];
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) row[cb] = a.in + (int64_t)min(16 * cb + (lane & 15), a.J - 1) * a.g.R;
  Tile<0>::A av[FD][RB];
  float2 bv[FD][NB][4];
  auto load = [&](int d, int s) {
    s = min(s, steps - 1);
#pragma unroll
    // chunk-step-major: fragment (step s of chunk ch, k row block mb) at (s nch + ch) mbl + mb
    for (int m = 0; m < RB; ++m) av[d][m] = frag_a<0>(a.adj_f32, mbl, s * (steps_total / steps) + ch, mbm[m], lane);
    call_operand<NB>(row, rho0 + 16 * s, a.g.R, grp, bv[d]);
  };
  Tile<0>::Acc acc[RB][NB];
#pragma unroll
  for (int m = 0; m < RB; ++m)
#pragma unroll
    for (int c = 0; c < NB; ++c) acc[m][c] = Tile<0>::zero();
  auto compute = [&](int d) {
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const Tile<0>::B b = Tile<0>::make_b(bv[d][c]);
#pragma unroll
      for (int m = 0; m < RB; ++m) Tile<0>::mma(acc[m][c], av[d][m], b);
    }
  };
#pragma unroll
  for (int d = 0; d < FD; ++d) load(d, d);
  int s0 = 0;
  for (; s0 + FD <= steps; s0 += FD) {
#pragma unroll
    for (int d = 0; d < FD; ++d) {
      compute(d);
      load(d, s0 + d + FD);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int d = 0; d + 1 < FD; ++d)
    if (s0 + d < steps) compute(d);
  const int Jp = 16 * ((a.J + 15) / 16);
  float2* part = a.part + (int64_t)ch * a.g.Kp * Jp;
#pragma unroll
  for (int m = 0; m < RB; ++m)
    if (mb0 + m < mbl)
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        f32x4 cr, ci;
        Tile<0>::finish(acc[m][c], cr, ci);
#pragma unroll
        for (int r = 0; r < 4; ++r)
          part[(int64_t)(16 * (mb0 + m) + 4 * grp + r) * Jp + 16 * c + (lane & 15)] = make_float2(cr[r], ci[r]);
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
// Workgroup: one rho chunk of RC, one group of 4 RB k row blocks (RB per wave); D rows
// are k, columns coils.  The k groups of one chunk are placed on one XCD (workgroups are
// dispatched round-robin over the 8 XCDs), so the chunk's T1b is fetched into one L2.
template <int NB, int RB, int FD = ADJ_FD>
__global__ __launch_bounds__(NT) void core_adj_bf16_kernel(CoreArgs a, int nch, int kgroups) {
  const int xcd = blockIdx.x % 8, i = blockIdx.x / 8;
  const int ky = i % kgroups, ch = 8 * (i / kgroups) + xcd;
  const int lane = threadIdx.x & 63, grp = lane >> 4, wave = threadIdx.x >> 6;
  const int mbl = a.g.Kp / 16;
  const int mb0 = ky * (4 * RB) + wave * RB;
  if (ch >= nch || mb0 >= mbl) return;
  const int64_t rho0 = (int64_t)ch * RC;
  const int64_t steps_total = a.g.Rp / 16;
  constexpr int steps = RC / 16;
  const int64_t nchp = steps_total / steps;  // chunks in the planes' order (Rp / RC)
  int64_t oa[RB];
#pragma unroll
  for (int m = 0; m < RB; ++m) oa[m] = ((int64_t)ch * mbl + min(mb0 + m, mbl - 1)) * 512 + lane * 8;
  const float2* row[NB];
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) row[cb] = a.in + (int64_t)min(16 * cb + (lane & 15), a.J - 1) * a.g.R;
  u16x8 ah[FD][RB], al[FD][RB];
  float2 bv[FD][NB][4];
  auto load = [&](int d, int s) {
    s = min(s, steps - 1);
#pragma unroll
    for (int m = 0; m < RB; ++m) {
      ah[d][m] = ld8(a.adj_hi + oa[m] + (int64_t)s * nchp * mbl * 512);
      al[d][m] = ld8(a.adj_lo + oa[m] + (int64_t)s * nchp * mbl * 512);
    }
    call_operand<NB>(row, rho0 + 16 * s, a.g.R, grp, bv[d]);
  };
  f32x4 cr[RB][NB], ci[RB][NB];
#pragma unroll
  for (int m = 0; m < RB; ++m)
#pragma unroll
    for (int c = 0; c < NB; ++c) { cr[m][c] = z4(); ci[m][c] = z4(); }
  auto compute = [&](int d) {
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const Tile<1>::B b = Tile<1>::make_b(bv[d][c]);
#pragma unroll
      for (int m = 0; m < RB; ++m) mfma6(cr[m][c], ci[m][c], ah[d][m], al[d][m], b.rh, b.rl, b.ih, b.il);
    }
  };
  // FD stages in flight; the issue order of the stages' loads is kept, so the wait before
  // a stage's products only covers that stage's loads.
#pragma unroll
  for (int d = 0; d < FD; ++d) load(d, d);
  int s0 = 0;
  for (; s0 + FD <= steps; s0 += FD) {
#pragma unroll
    for (int d = 0; d < FD; ++d) {
      compute(d);
      load(d, s0 + d + FD);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int d = 0; d + 1 < FD; ++d)
    if (s0 + d < steps) compute(d);
  const int Jp = 16 * ((a.J + 15) / 16);
  float2* part = a.part + (int64_t)ch * a.g.Kp * Jp;
#pragma unroll
  for (int m = 0; m < RB; ++m)
    if (mb0 + m < mbl)
#pragma unroll
      for (int c = 0; c < NB; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          part[(int64_t)(16 * (mb0 + m) + 4 * grp + r) * Jp + 16 * c + (lane & 15)] =
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
    // step-major, so that the waves of a contraction read one contiguous region per step:
    // forward (mode 0) [step][row block][lane][8]; adjoint [step within a rho chunk of RC]
    // [chunk][k row block][lane][8] (its waves each take RB k row blocks of one chunk)
    const int64_t idx = e / 512, rb = idx % nrb, t = idx / nrb;
    const int64_t s = mode == 0 ? t : (t % (steps / (RC / 16))) * (RC / 16) + t / (steps / (RC / 16));
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

hipError_t core_frag32_launch(const float2* core, const CoreGeom& g, float2* dst, hipStream_t st) {
  float4* p = reinterpret_cast<float4*>(dst);
  hipLaunchKernelGGL(core_frag32_kernel, dim3(4096), dim3(256), 0, st, core, g.R, g.K, 0, (g.R + 15) / 16,
                     (int64_t)g.Kp / 16, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(core_frag32_kernel, dim3(4096), dim3(256), 0, st, core, g.R, g.K, 1, (int64_t)g.Kp / 16,
                     g.Rp / 16, p + g.fwd32_elems() / 2);
  return hipGetLastError();
}

hipError_t core_fwd_launch(const CoreArgs& a, int precision, hipStream_t st) {
  const dim3 block(NT);
  auto grid = [&](int rb) { return dim3((unsigned)((a.g.R + 64 * rb - 1) / (64 * rb))); };
  if (precision == MAXWELL_BF16_SPLIT) {
    constexpr int F = FWD_RB_FEW, M = FWD_RB_MANY;
    switch ((a.J + 15) / 16) {
      case 1: hipLaunchKernelGGL((core_fwd_bf16_kernel<1, F>), grid(F), block, 0, st, a); break;
      case 2: hipLaunchKernelGGL((core_fwd_bf16_kernel<2, F>), grid(F), block, 0, st, a); break;
      case 3: hipLaunchKernelGGL((core_fwd_bf16_kernel<3, M>), grid(M), block, 0, st, a); break;
      default: hipLaunchKernelGGL((core_fwd_bf16_kernel<4, M>), grid(M), block, 0, st, a); break;
    }
  } else if (a.fwd_f32) {
    constexpr int F = FWD_RB_FEW, M = FWD_RB_MANY;
    switch ((a.J + 15) / 16) {
      case 1: hipLaunchKernelGGL((core_fwd_f32f_kernel<1, F>), grid(F), block, 0, st, a); break;
      case 2: hipLaunchKernelGGL((core_fwd_f32f_kernel<2, F>), grid(F), block, 0, st, a); break;
      case 3: hipLaunchKernelGGL((core_fwd_f32f_kernel<3, M>), grid(M), block, 0, st, a); break;
      default: hipLaunchKernelGGL((core_fwd_f32f_kernel<4, M>), grid(M), block, 0, st, a); break;
    }
  } else {
    hipLaunchKernelGGL(core_fwd_f32_kernel, grid(RB), block, 0, st, a);
  }
  return hipGetLastError();
}

hipError_t core_adj_launch(const CoreArgs& a, int precision, float alpha, const float* scale_dev, hipStream_t st) {
  const int nch = core_adj_chunks(a.g.R);
  const int nb = (a.J + 15) / 16;
  const dim3 block(NT);
  auto kgroups = [&](int rb) { return (a.g.Kp / 16 + 4 * rb - 1) / (4 * rb); };
  if (precision == MAXWELL_BF16_SPLIT) {
    const int rb = nb <= 2 ? ADJ_RB_FEW : ADJ_RB_MANY, kg = kgroups(rb);
    const dim3 grid((unsigned)(8 * kg * ((nch + 7) / 8)));
    constexpr int F = ADJ_RB_FEW, M = ADJ_RB_MANY;
    switch (nb) {
      case 1: hipLaunchKernelGGL((core_adj_bf16_kernel<1, F>), grid, block, 0, st, a, nch, kg); break;
      case 2: hipLaunchKernelGGL((core_adj_bf16_kernel<2, F>), grid, block, 0, st, a, nch, kg); break;
      case 3: hipLaunchKernelGGL((core_adj_bf16_kernel<3, M>), grid, block, 0, st, a, nch, kg); break;
      default: hipLaunchKernelGGL((core_adj_bf16_kernel<4, M>), grid, block, 0, st, a, nch, kg); break;
    }
  } else if (a.adj_f32) {
    const int rb = nb <= 2 ? ADJ_RB_FEW : ADJ_RB_MANY, kg = kgroups(rb);
    const dim3 grid((unsigned)(8 * kg * ((nch + 7) / 8)));
    constexpr int F = ADJ_RB_FEW, M = ADJ_RB_MANY;
    switch (nb) {
      case 1: hipLaunchKernelGGL((core_adj_f32f_kernel<1, F, 2>), grid, block, 0, st, a, nch, kg); break;
      case 2: hipLaunchKernelGGL((core_adj_f32f_kernel<2, F, 2>), grid, block, 0, st, a, nch, kg); break;
      case 3: hipLaunchKernelGGL((core_adj_f32f_kernel<3, M, 2>), grid, block, 0, st, a, nch, kg); break;
      default: hipLaunchKernelGGL((core_adj_f32f_kernel<4, M, 2>), grid, block, 0, st, a, nch, kg); break;
    }
  } else {
    hipLaunchKernelGGL(core_adj_f32_kernel, dim3((unsigned)nch, (unsigned)kgroups(RB)), block, 0, st, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t plane = (int64_t)a.g.Kp * ((a.J + 15) / 16 * 16);
  hipLaunchKernelGGL(core_adj_reduce_kernel, dim3((unsigned)((plane + RED_OUT - 1) / RED_OUT)),
                     dim3(RED_OUT * RED_SL), 0, st, a, nch, alpha, scale_dev);
  return hipGetLastError();
}

}  // namespace mx
