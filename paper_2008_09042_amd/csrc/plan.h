// Plan object and the enqueue sequences behind the C ABI.
#pragma once

#include <functional>
#include <string>
#include <vector>

#include "../../include/maxwell.h"
#include "common.h"
#include "core.h"

namespace mx {

// Optional per-kernel timing (HIP events on the launch stream).
struct Timing {
  bool on = false;
  struct Rec { int name; int ev; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> ev_start, ev_stop;   // pool, reused across sessions
  std::vector<const char*> names;
};

struct Plan {
  mutable Timing timing;
  int device = -1;  // the device current at plan creation
  // geometry
  int ndim = 0;
  int64_t n[3] = {1, 1, 1};
  int64_t N = 0;
  int J = 0;
  int64_t K = 0, M = 0;
  int precision = 0, sampling = 0;
  // basis (caller-owned device pointers)
  int basis_kind = 0;
  const float2* dense = nullptr;
  int64_t r[3] = {0, 0, 0};
  const float2* U[3] = {nullptr, nullptr, nullptr};
  const float2* core = nullptr;
  // device tables owned by the plan
  int32_t* d_mask = nullptr;   // [M] linear k-space index of each sample
  int32_t* d_inv = nullptr;    // [N] sample position of each grid point, -1 if unsampled
  int32_t* d_lptr = nullptr;   // [N / n_last + 1] first sample at or after each last-axis line
  float* d_w = nullptr;        // [M] data weights or null (w = 1)
  float2* d_tw[3] = {nullptr, nullptr, nullptr};  // twiddle tables per axis
  int nrad[3] = {0, 0, 0};
  int radix[3][12];
  // fused 3D Tucker path (Cartesian mask made of full lines along the last axis)
  bool fused = false;
  int64_t L = 0;               // sampled lines
  int32_t* d_pos = nullptr;    // [L] plane index k0 * n1 + k1 of each line
  void* d_frag = nullptr;      // fragment-ordered factor operands (one allocation)
  const void *U0F = nullptr, *U1TF = nullptr, *U1CF = nullptr, *U0HF = nullptr;
  const void *U0SF = nullptr, *U1TSF = nullptr;  // with the adjoint's chessboard sign
  bool mode3_direct = false;   // dedicated third-mode product kernels (r2 <= 64)
  const void *U2F = nullptr, *U2CF = nullptr;
  // dedicated core contraction kernels (Tucker basis, J <= 64)
  bool core_direct = false;
  CoreGeom cg{};
  uint16_t* d_core_split = nullptr;  // BF16-split core planes (BF16_SPLIT plans only)
  float2* d_core_f32 = nullptr;      // FP32 core copies in fragment order (FP32 plans only)
  int G_fwd = 2, G_adj = 8;    // coils per plane workgroup (set at plan creation)
  int split_apply = 0, split_adj = 0;  // dense basis GEMMs: split-K factors tuned at plan creation
  bool skinny_apply = false, skinny_adj = false;  // dense basis: streaming kernels chosen at plan creation
  float gscale = 1.0f;         // prod_d (-1)^(n_d/2) / sqrt(N)
  // non-Cartesian sampling (Kaiser-Bessel NUFFT, 2D)
  int g[2] = {0, 0};             // oversampled grid
  int W = 0;                     // kernel width
  float kscale = 1.0f;           // sqrt(g0 g1 / N)
  float* d_iphi = nullptr;       // [n0 + n1] inverse deapodisation per axis
  int32_t* d_cptr = nullptr;     // [g0 g1 + 1] samples sorted by first-tap cell (CSR)
  int32_t* d_sperm = nullptr;    // [M] original index of each sorted sample
  int32_t* d_sinv = nullptr;     // [M] sorted position of each sample
  int32_t* d_scol = nullptr;     // [M] first-tap column of each sorted sample
  float* d_swts = nullptr;       // [M][16] tap weights in sorted order (axis 1 from slot 8)
  int2* d_sbase = nullptr;       // [M] first-tap (row, column) in sorted order
  uint8_t* d_sheavy = nullptr;   // [g0 ceil(g1 / 64)] spread blocks taken by the split kernel
  int32_t* d_shlist = nullptr;   // [n_heavy] their indices
  int n_heavy = 0, n_med = 0;
  int split_pm = 4, split_ph = 16;  // column parts of the split spread rows
  bool spread_lds = true;     // plain spread blocks through LDS ($MAXWELL_SPREAD_LDS=0: from memory)
  bool ordered_transfer = false;  // gridding path: the transfer residual in the spread's sample order
  float2* d_twg[2] = {nullptr, nullptr};  // grid twiddles
  int nradg[2] = {0, 0};
  int radixg[2][12];
  // workspace layout (byte offsets into the caller's workspace)
  size_t ws_bytes = 0;
  size_t off_S = 0, off_K = 0, off_tA = 0, off_tB = 0, off_E = 0, off_gemm = 0, off_part = 0;
  size_t off_T1 = 0, off_T3 = 0, off_xt = 0, off_Z = 0, off_gxp = 0, off_T3b = 0, off_T1b = 0, off_G = 0, off_Ys = 0, off_cpart = 0;
  size_t off_U = 0, off_cg = 0;  // Gauss-Newton / CG: JVP result; r, d, q, FP64 scalars
  size_t off_admm = 0;           // SENSE / ADMM state (general path only)
  size_t off_cfrag = 0;          // dense apply: fragment-ordered coefficients (0: generic GEMM)
  size_t off_adjp = 0;           // dense adjoint: row-chunk partials of the streaming kernel
  int part_blocks = 0;

  size_t bytes_x() const { return (size_t)N * 8; }
  size_t bytes_c() const { return (size_t)J * (size_t)K * 8; }
  size_t bytes_S() const { return (size_t)J * (size_t)N * 8; }
  size_t bytes_y() const { return (size_t)J * (size_t)M * 8; }
};

// Records the thread-local message returned by maxwell_last_error().
void set_last_error(const std::string& msg);

// Launch recording for batched execution: while a recorder is set on the calling thread,
// each launch step of the run_* calls (one TIMED expression: one kernel or one short fixed
// sequence) is kept as an op, a closure that enqueues it on a given stream, instead of being
// enqueued.  The closures hold copies of their arguments; the plan is referenced.
struct Op {
  const char* name;
  std::function<hipError_t(hipStream_t)> run;
};
struct OpRecorder {
  std::vector<Op> ops;
  hipError_t add(const char* name, std::function<hipError_t(hipStream_t)> f) {
    ops.push_back(Op{name, std::move(f)});
    return hipSuccess;
  }
};
void set_recorder(OpRecorder* r);  // nullptr: launch again
OpRecorder* recorder();

// Brackets one kernel launch with timing events when timing is on.
struct Span {
  const Plan& p;
  hipStream_t st;
  int ev = -1;
  Span(const Plan& plan, const char* name, hipStream_t stream);
  ~Span();
};

maxwell_status plan_build(Plan& p, const maxwell_plan_desc& d, const maxwell_basis_desc& b);
void plan_release(Plan& p);

hipError_t run_basis_apply(const Plan& p, const float2* c, float2* S, void* ws, hipStream_t st);
hipError_t run_basis_adjoint(const Plan& p, const float2* S, float2* c, float alpha, const float* alpha_dev,
                             void* ws, hipStream_t st);
hipError_t run_encode(const Plan& p, const float2* x, const float2* c, float2* y, void* ws, hipStream_t st);
// transfer: the residual is (forward: written / adjoint: read) in the plan's transfer
// layout, the weighted residual taken back along the readout on the fused path and the
// residual itself elsewhere.
hipError_t run_adjoint(const Plan& p, const float2* x, const float2* c, const float2* y, float alpha,
                       const float* scale_dev, float2* gx, float2* gc, void* ws, hipStream_t st,
                       bool maps_ready, bool transfer = false);
hipError_t run_forward_loss(const Plan& p, const float2* x, const float2* c, const float2* y, float2* r,
                            double* loss, void* ws, hipStream_t st, bool transfer = false);
hipError_t run_grad(const Plan& p, const float2* x, const float2* c, const float2* y, float2* gx, float2* gc,
                    double* loss, void* ws, hipStream_t st);
// Gauss-Newton step: Jacobian-vector product, normal operator, conjugate gradients
constexpr int CG_SCALARS = 8;
hipError_t run_jvp(const Plan& p, const float2* x, const float2* c, const float2* dx, const float2* dc, float2* y,
                   void* ws, hipStream_t st);
hipError_t run_normal(const Plan& p, const float2* x, const float2* c, const float2* dx, const float2* dc,
                      float lam_x, float lam_c, float2* ox, float2* oc, void* ws, hipStream_t st);
hipError_t run_cg(const Plan& p, const float2* x, const float2* c, const float2* bx, const float2* bc, float lam_x,
                  float lam_c, int iters, float2* dx, float2* dc, double* rr, void* ws, hipStream_t st);
// extra bilinear terms: n map sets, x n x [N], c n x [J][K]
hipError_t run_multi_encode(const Plan& p, int n, const float2* x, const float2* c, float2* y, void* ws,
                            hipStream_t st);
hipError_t run_multi_grad(const Plan& p, int n, const float2* x, const float2* c, const float2* y, float2* gx,
                          float2* gc, double* loss, void* ws, hipStream_t st);
// SENSE with fixed maps S [J][N] and the constrained reconstruction (general path only)
constexpr int ADMM_SCALARS = 8;
hipError_t run_sense_encode(const Plan& p, const float2* S, const float2* x, float2* y, void* ws, hipStream_t st);
hipError_t run_sense_adjoint(const Plan& p, const float2* S, const float2* y, float2* gx, void* ws, hipStream_t st);
hipError_t run_sense_normal(const Plan& p, const float2* S, const float2* x, float2* out, void* ws, hipStream_t st);
hipError_t run_tv_prox(const Plan& p, const float2* z, float lam, int iters, float2* x, void* ws, hipStream_t st);
hipError_t run_ball_project(const Plan& p, const float2* w, const float2* y, const float* eps, float2* z, void* ws,
                            hipStream_t st);
hipError_t run_admm(const Plan& p, const float2* S, const float2* y, const float* eps, float rho0, int iters,
                    int cg_iters, int tv_iters, float2* pimg, double* hist, void* ws, hipStream_t st);

}  // namespace mx
