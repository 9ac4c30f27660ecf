// Plan construction and the enqueue sequences of the general path.
//
// General path (any geometry the plan accepts):
//   encode   S = B c (MFMA GEMM chain)  ->  m = x (.) S fused into the first
//            FFT pass  ->  centred unitary DFT, one LDS-staged pass per axis
//            ->  mask gather  ->  y                         (Sec. II-B, Eq. (5))
//   adjoint  zero-filled scatter  ->  inverse DFT per axis  ->
//            gx = s sum_j conj(S_j) (.) g_j,  h_j = s conj(x) (.) g_j  ->
//            gc = B^H h                                      (Sec. II-B, J_G^H)
// The per-coil maps S live only in the caller's workspace for the duration
// of one call.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <sstream>
#include <vector>

#include "fused.h"
#include "mode3.h"
#include "nufft.h"
#include "solver.h"
#include "admm.h"
#include "skinny.h"
#include "plan.h"
#include "tune.h"

namespace mx {

Span::Span(const Plan& plan, const char* name, hipStream_t stream) : p(plan), st(stream) {
  Timing& t = p.timing;
  if (!t.on) return;
  int id = -1;
  for (size_t i = 0; i < t.names.size(); ++i)
    if (std::strcmp(t.names[i], name) == 0) id = (int)i;
  if (id < 0) { t.names.push_back(name); id = (int)t.names.size() - 1; }
  const size_t k = t.recs.size();
  if (k >= t.ev_start.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
    t.ev_start.push_back(a);
    t.ev_stop.push_back(b);
  }
  if (hipEventRecord(t.ev_start[k], st) != hipSuccess) return;
  t.recs.push_back({id, (int)k});
  ev = (int)k;
}

Span::~Span() {
  if (ev >= 0) (void)hipEventRecord(p.timing.ev_stop[ev], st);
}

namespace {
thread_local OpRecorder* g_rec = nullptr;
}  // namespace

void set_recorder(OpRecorder* r) { g_rec = r; }
OpRecorder* recorder() { return g_rec; }

// One launch step: enqueued on st (bracketed by timing events when timing is on), or, with a
// recorder set, kept as an op that enqueues the same launch on the stream it is given.
#define TIMED(name, expr)                                                                        \
  (g_rec ? g_rec->add(name, [=, &p](hipStream_t st) -> hipError_t { return (expr); })         \
         : [&]() { Span _span(p, name, st); return (expr); }())

namespace {

size_t al(size_t v) { return (v + 255) & ~size_t(255); }

GemmArgs gemm0() {
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.batch = 1;
  g.alpha = 1.0f;
  return g;
}

// ---- dense basis
GemmArgs dense_apply_args(const Plan& p, const float2* c, float2* S) {
  GemmArgs g = gemm0();
  g.M = p.J; g.N = p.N; g.K = p.K;
  g.A = c; g.a_ms = p.K; g.a_ks = 1;
  g.B = p.dense; g.b_ks = 1; g.b_ns = p.K;
  g.C = S; g.c_ms = p.N; g.c_ns = 1;
  g.splits = p.split_apply;
  return g;
}

GemmArgs dense_adjoint_args(const Plan& p, const float2* h, float2* c) {
  GemmArgs g = gemm0();
  g.M = p.J; g.N = p.K; g.K = p.N;
  g.A = h; g.a_ms = p.N; g.a_ks = 1;
  g.B = p.dense; g.b_ks = p.K; g.b_ns = 1; g.conjB = 1;
  g.C = c; g.c_ms = p.K; g.c_ns = 1;
  g.splits = p.split_adj;
  return g;
}

// ---- Tucker basis: the chain of k-mode products (Sec. II-E)
void tucker_apply_args(const Plan& p, const float2* c, float2* tA, float2* tB, float2* S, GemmArgs* g) {
  const int64_t r0 = p.r[0], r1 = p.r[1], r2 = p.r[2], n0 = p.n[0], n1 = p.n[1], n2 = p.n[2];
  const int64_t R = r0 * r1 * r2, Q = r1 * r2, J = p.J;
  // (1) T1[j][rho] = sum_k c[j][k] core[rho][k]
  g[0] = gemm0();
  g[0].M = J; g[0].N = R; g[0].K = p.K;
  g[0].A = c; g[0].a_ms = p.K; g[0].a_ks = 1;
  g[0].B = p.core; g[0].b_ks = 1; g[0].b_ns = p.K;
  g[0].C = tA; g[0].c_ms = R; g[0].c_ns = 1;
  // (2) T2[j][i0][q] = sum_p0 U0[i0][p0] T1[j][p0][q]
  g[1] = gemm0();
  g[1].batch = J; g[1].M = n0; g[1].N = Q; g[1].K = r0;
  g[1].A = p.U[0]; g[1].a_ms = r0; g[1].a_ks = 1;
  g[1].B = tA; g[1].b_bs = R; g[1].b_ks = Q; g[1].b_ns = 1;
  g[1].C = tB; g[1].c_bs = n0 * Q; g[1].c_ms = Q; g[1].c_ns = 1;
  // (3) T3[j i0][i1][p2] = sum_p1 U1[i1][p1] T2[j i0][p1][p2]
  g[2] = gemm0();
  g[2].batch = J * n0; g[2].M = n1; g[2].N = r2; g[2].K = r1;
  g[2].A = p.U[1]; g[2].a_ms = r1; g[2].a_ks = 1;
  g[2].B = tB; g[2].b_bs = Q; g[2].b_ks = r2; g[2].b_ns = 1;
  g[2].C = tA; g[2].c_bs = n1 * r2; g[2].c_ms = r2; g[2].c_ns = 1;
  // (4) S[j i0 i1][i2] = sum_p2 T3[j i0 i1][p2] U2[i2][p2]
  g[3] = gemm0();
  g[3].M = J * n0 * n1; g[3].N = n2; g[3].K = r2;
  g[3].A = tA; g[3].a_ms = r2; g[3].a_ks = 1;
  g[3].B = p.U[2]; g[3].b_ks = 1; g[3].b_ns = r2;
  g[3].C = S; g[3].c_ms = n2; g[3].c_ns = 1;
}

void tucker_adjoint_args(const Plan& p, const float2* h, float2* tA, float2* tB, float2* c, GemmArgs* g) {
  const int64_t r0 = p.r[0], r1 = p.r[1], r2 = p.r[2], n0 = p.n[0], n1 = p.n[1], n2 = p.n[2];
  const int64_t R = r0 * r1 * r2, Q = r1 * r2, J = p.J;
  // (4') Q3[j i0 i1][p2] = sum_i2 h[j i0 i1][i2] conj(U2[i2][p2])
  g[0] = gemm0();
  g[0].M = J * n0 * n1; g[0].N = r2; g[0].K = n2;
  g[0].A = h; g[0].a_ms = n2; g[0].a_ks = 1;
  g[0].B = p.U[2]; g[0].b_ks = r2; g[0].b_ns = 1; g[0].conjB = 1;
  g[0].C = tA; g[0].c_ms = r2; g[0].c_ns = 1;
  // (3') Q2[j i0][p1][p2] = sum_i1 conj(U1[i1][p1]) Q3[j i0][i1][p2]
  g[1] = gemm0();
  g[1].batch = J * n0; g[1].M = r1; g[1].N = r2; g[1].K = n1;
  g[1].A = p.U[1]; g[1].a_ms = 1; g[1].a_ks = r1; g[1].conjA = 1;
  g[1].B = tA; g[1].b_bs = n1 * r2; g[1].b_ks = r2; g[1].b_ns = 1;
  g[1].C = tB; g[1].c_bs = Q; g[1].c_ms = r2; g[1].c_ns = 1;
  // (2') Q1[j][p0][q] = sum_i0 conj(U0[i0][p0]) Q2[j][i0][q]
  g[2] = gemm0();
  g[2].batch = J; g[2].M = r0; g[2].N = Q; g[2].K = n0;
  g[2].A = p.U[0]; g[2].a_ms = 1; g[2].a_ks = r0; g[2].conjA = 1;
  g[2].B = tB; g[2].b_bs = n0 * Q; g[2].b_ks = Q; g[2].b_ns = 1;
  g[2].C = tA; g[2].c_bs = R; g[2].c_ms = Q; g[2].c_ns = 1;
  // (1') c[j][k] = sum_rho conj(core[rho][k]) Q1[j][rho]
  g[3] = gemm0();
  g[3].M = J; g[3].N = p.K; g[3].K = R;
  g[3].A = tA; g[3].a_ms = R; g[3].a_ks = 1;
  g[3].B = p.core; g[3].b_ks = p.K; g[3].b_ns = 1; g[3].conjB = 1;
  g[3].C = c; g[3].c_ms = p.K; g[3].c_ns = 1;
}

template <typename T>
T* wsp(void* ws, size_t off) { return reinterpret_cast<T*>(reinterpret_cast<char*>(ws) + off); }

// Centred unitary DFT over every axis of J stacked arrays of shape dims[0..nd).
// Axis passes over [J][dims]; optionally the first pass reads the samples through the inverse
// mask (in_samples [J][M]) and the last writes them (out_samples).
hipError_t fft_dims(const Plan& p, const float2* src, float2* dst, int dir, const float2* premul, int nd,
                    const int64_t* dims, float2* const* tw, const int* nrad, const int (*radix)[12], hipStream_t st,
                    const float2* in_samples = nullptr, float2* out_samples = nullptr) {
  const float2* cur = src;
  for (int t = 0; t < nd; ++t) {
    const int d = nd - 1 - t;
    int64_t inner = 1, opc = 1;
    for (int e = d + 1; e < nd; ++e) inner *= dims[e];
    for (int e = 0; e < d; ++e) opc *= dims[e];
    FftAxisArgs a;
    std::memset(&a, 0, sizeof(a));
    a.data = dst;
    a.src = cur;
    a.n = dims[d];
    a.inner = inner;
    a.outer = (int64_t)p.J * opc;
    a.outer_per_coil = opc;
    a.dir = dir;
    a.twiddle = tw[d];
    a.nrad = nrad[d];
    for (int q = 0; q < nrad[d]; ++q) a.radix[q] = radix[d][q];
    a.premul = (t == 0) ? premul : nullptr;
    if (t == 0 && in_samples) {
      a.in_inv = p.d_inv;
      a.in_samples = in_samples;
      a.in_mask = p.d_mask;
      a.in_lptr = p.d_lptr;
    }
    if (t == nd - 1 && out_samples) {
      a.out_inv = p.d_inv;
      a.out_samples = out_samples;
    }
    a.coil_elems = p.N;
    a.nsamples = p.M;
    hipError_t e = TIMED("fft_axis", fft_axis_launch(a, st));
    if (e != hipSuccess) return e;
    cur = dst;
  }
  return hipSuccess;
}

hipError_t fft_image(const Plan& p, const float2* src, float2* dst, int dir, const float2* premul,
                     hipStream_t st) {
  return fft_dims(p, src, dst, dir, premul, p.ndim, p.n, p.d_tw, p.nrad, p.radix, st);
}

// The NUFFT's transform over the oversampled grid G [J][g0][g1], with its zero-pad and crop
// folded into the passes: forward (dir < 0), the first pass (along rows) reads S x / (Phi0
// Phi1) inside the centred n0 x n1 window in place of a padded grid and transforms and writes
// only the window's rows, which are all the second pass (along columns) reads; inverse
// (dir > 0), the first pass (along rows) writes only the window's columns, and the last (along
// them) writes only the window, deapodised, to out [J][n0][n1].  Between the passes the rows
// (columns) of G outside the window hold stale values that no pass reads.
hipError_t fft_grid_window(const Plan& p, const float2* S, const float2* x, float2* G, float2* out, int dir,
                           hipStream_t st) {
  const int64_t dims[2] = {p.g[0], p.g[1]};
  for (int t = 0; t < 2; ++t) {
    const int d = 1 - t;  // rows first, then columns
    FftAxisArgs a;
    std::memset(&a, 0, sizeof(a));
    a.data = G;
    a.src = G;
    a.n = dims[d];
    a.inner = d == 1 ? 1 : dims[1];
    a.outer_per_coil = d == 1 ? dims[0] : 1;
    a.outer = (int64_t)p.J * a.outer_per_coil;
    a.dir = dir;
    a.twiddle = p.d_twg[d];
    a.nrad = p.nradg[d];
    for (int q = 0; q < p.nradg[d]; ++q) a.radix[q] = p.radixg[d][q];
    a.coil_elems = dims[0] * dims[1];
    a.nsamples = p.M;
    a.iphi = p.d_iphi;
    a.woff0 = (int)(dims[0] / 2 - p.n[0] / 2);
    a.woff1 = (int)(dims[1] / 2 - p.n[1] / 2);
    a.wn0 = (int)p.n[0];
    a.wn1 = (int)p.n[1];
    if (dir < 0) {
      if (t == 0) {
        a.src = S;
        a.premul = x;
        a.win = WIN_PAD;
      } else {
        a.win = WIN_ROWS_IN;
      }
    } else {
      if (t == 0) a.win = WIN_COLS_OUT;
      else a.crop_out = out;
    }
    hipError_t e = TIMED("fft_axis", fft_axis_launch(a, st));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

NufftArgs nufft_args(const Plan& p) {
  NufftArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n0 = (int)p.n[0]; a.n1 = (int)p.n[1];
  a.g0 = p.g[0]; a.g1 = p.g[1];
  a.J = p.J; a.W = p.W; a.M = p.M;
  a.iphi0 = p.d_iphi; a.iphi1 = p.d_iphi + p.n[0];
  a.cell_ptr = p.d_cptr; a.s_perm = p.d_sperm; a.s_inv = p.d_sinv; a.s_col = p.d_scol; a.s_wts = p.d_swts; a.s_base = p.d_sbase;
  a.s_heavy = p.n_heavy ? p.d_sheavy : nullptr; a.s_hlist = p.d_shlist; a.n_heavy = p.n_heavy;
  a.n_med = p.n_med;
  a.split_pm = p.split_pm;
  a.split_ph = p.split_ph;
  a.spread_lds = p.spread_lds ? 1 : 0;
  a.cscale = p.kscale;
  return a;
}

// Modified Bessel function I0 from its power series sum_k ((x/2)^(2k)) / (k!)^2.
double bessel_i0(double x) {
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 200; ++k) {
    term *= q / ((double)k * (double)k);
    sum += term;
    if (term < 1e-17 * sum) break;
  }
  return sum;
}

// ---- fused path GEMMs
// T3[j][i2][p0 p1] = sum_p2 U2[i2][p2] T1[j][p0 p1][p2]
GemmArgs fused_T3_args(const Plan& p, const float2* T1, float2* T3) {
  const int64_t R01 = p.r[0] * p.r[1], R = R01 * p.r[2];
  GemmArgs g = gemm0();
  g.batch = p.J; g.M = p.n[2]; g.N = R01; g.K = p.r[2];
  g.A = p.U[2]; g.a_ms = p.r[2]; g.a_ks = 1;
  g.B = T1; g.b_bs = R; g.b_ks = 1; g.b_ns = p.r[2];
  g.C = T3; g.c_bs = p.n[2] * R01; g.c_ms = R01; g.c_ns = 1;
  return g;
}

// T1b[j][p0 p1][p2] = sum_i2 T3b[j][i2][p0 p1] conj(U2[i2][p2])
GemmArgs fused_T1b_args(const Plan& p, const float2* T3b, float2* T1b) {
  const int64_t R01 = p.r[0] * p.r[1], R = R01 * p.r[2];
  GemmArgs g = gemm0();
  g.batch = p.J; g.M = R01; g.N = p.r[2]; g.K = p.n[2];
  g.A = T3b; g.a_bs = p.n[2] * R01; g.a_ms = 1; g.a_ks = R01;
  g.B = p.U[2]; g.b_ks = p.r[2]; g.b_ns = 1; g.conjB = 1;
  g.C = T1b; g.c_bs = R; g.c_ms = p.r[2]; g.c_ns = 1;
  return g;
}

Mode3Args mode3_args(const Plan& p) {
  Mode3Args m;
  std::memset(&m, 0, sizeof(m));
  m.J = p.J;
  m.Q = (int)(p.r[0] * p.r[1]);
  m.n2 = (int)p.n[2];
  m.r2 = (int)p.r[2];
  m.U2F = p.U2F;
  m.U2CF = p.U2CF;
  return m;
}

bool detect_lines(const maxwell_plan_desc& d, std::vector<int32_t>& pos) {
  const int64_t n2 = d.n[2];
  if (d.M <= 0 || d.M % n2) return false;
  const int64_t L = d.M / n2;
  pos.resize(L);
  for (int64_t l = 0; l < L; ++l) {
    const int64_t base = d.mask_idx[l * n2];
    if (base % n2) return false;
    for (int64_t t = 1; t < n2; ++t)
      if (d.mask_idx[l * n2 + t] != base + t) return false;
    pos[l] = (int32_t)(base / n2);
  }
  return true;
}

PlaneArgs plane_args(const Plan& p, void* ws, int G) {
  PlaneArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n0 = (int)p.n[0]; a.n1 = (int)p.n[1]; a.n2 = (int)p.n[2];
  a.r0 = (int)p.r[0]; a.r1 = (int)p.r[1];
  a.r0p = (a.r0 + 15) / 16 * 16; a.r1p = (a.r1 + 15) / 16 * 16;
  a.J = p.J; a.L = (int)p.L; a.G = G;
  a.T3 = wsp<float2>(ws, p.off_T3);
  a.xt = wsp<float2>(ws, p.off_xt);
  a.pos = p.d_pos;
  a.Z = wsp<float2>(ws, p.off_Z);
  a.tw0 = p.d_tw[0]; a.tw1 = p.d_tw[1];
  a.nrad0 = p.nrad[0]; a.nrad1 = p.nrad[1];
  for (int q = 0; q < 12; ++q) { a.rad0[q] = p.radix[0][q]; a.rad1[q] = p.radix[1][q]; }
  a.precision = p.precision;
  a.U0F = p.U0F;
  a.U1TF = p.U1TF;
  a.U1CF = p.U1CF;
  a.U0HF = p.U0HF;
  a.U0SF = p.U0SF;
  a.U1TSF = p.U1TSF;
  return a;
}

LineArgs line_args(const Plan& p) {
  LineArgs a;
  std::memset(&a, 0, sizeof(a));
  a.J = p.J; a.n2 = (int)p.n[2]; a.L = p.L; a.M = p.M;
  a.gscale = p.gscale;
  a.alpha = 1.0f;
  a.tw2 = p.d_tw[2];
  a.nrad2 = p.nrad[2];
  for (int q = 0; q < 12; ++q) a.rad2[q] = p.radix[2][q];
  return a;
}

}  // namespace

// Kaiser-Bessel NUFFT tables (host, FP64): oversampled grid, twiddles, inverse
// deapodisation per axis, per-sample first tap and weights, and the samples
// sorted by first-tap cell for the spread.  Kernel phi(t) = I0(beta sqrt(1 - (2t/W)^2)) / W on |t| <= W/2,
// its Fourier transform Phi(nu) = sinh(sqrt(beta^2 - (pi W nu)^2)) / sqrt(...)
// (sin form when the radicand is negative); beta defaults to Beatty, Nishimura
// and Pauly: pi sqrt((W/sigma)^2 (sigma - 1/2)^2 - 0.8).
static maxwell_status nufft_build(Plan& p, const maxwell_plan_desc& d) {
  auto hip_err = [&](hipError_t e) {
    set_last_error(std::string("HIP error during plan creation: ") + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? MAXWELL_ERR_OUT_OF_MEMORY : MAXWELL_ERR_HIP;
  };
  const int W = d.kb_width;
  const double sigma = d.oversamp;
  double beta = d.kb_beta;
  if (beta <= 0.0) beta = M_PI * std::sqrt((W / sigma) * (W / sigma) * (sigma - 0.5) * (sigma - 0.5) - 0.8);
  p.W = W;
  for (int ax = 0; ax < 2; ++ax) p.g[ax] = (int)std::llround(sigma * (double)p.n[ax]);
  p.kscale = (float)std::sqrt((double)p.g[0] * p.g[1] / ((double)p.n[0] * p.n[1]));
  hipError_t e;
  for (int ax = 0; ax < 2; ++ax) {
    const int G = p.g[ax];
    p.nradg[ax] = fft_factorise(G, p.radixg[ax]);
    std::vector<float2> tw(G);
    for (int t = 0; t < G; ++t) {
      const double ang = -2.0 * M_PI * (double)t / (double)G;
      tw[t] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    if ((e = hipMalloc(&p.d_twg[ax], G * sizeof(float2))) != hipSuccess) return hip_err(e);
    if ((e = hipMemcpy(p.d_twg[ax], tw.data(), G * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_err(e);
  }
  auto Phi = [&](double nu) {
    const double z2 = beta * beta - (M_PI * W * nu) * (M_PI * W * nu);
    if (z2 > 0) { const double z = std::sqrt(z2); return std::sinh(z) / z; }
    if (z2 < 0) { const double z = std::sqrt(-z2); return std::sin(z) / z; }
    return 1.0;
  };
  auto phi = [&](double t) {
    const double a = 1.0 - (2.0 * t / W) * (2.0 * t / W);
    return a >= 0 ? bessel_i0(beta * std::sqrt(a)) / W : 0.0;
  };
  std::vector<float> iphi(p.n[0] + p.n[1]);
  for (int ax = 0, o = 0; ax < 2; o += (int)p.n[ax], ++ax)
    for (int r = 0; r < p.n[ax]; ++r) iphi[o + r] = (float)(1.0 / Phi((double)(r - p.n[ax] / 2) / (double)p.g[ax]));
  const int64_t M = p.M;
  std::vector<int2> base(M);
  std::vector<float> wts((size_t)M * 2 * W);
  std::vector<int32_t> cell((size_t)M);
  for (int64_t m = 0; m < M; ++m) {
    int b[2];
    for (int ax = 0; ax < 2; ++ax) {
      const double u = sigma * (double)d.traj[m * 2 + ax];
      const double g0 = std::ceil(u - 0.5 * W);
      for (int t = 0; t < W; ++t) wts[(size_t)m * 2 * W + ax * W + t] = (float)phi(u - (g0 + t));
      const int G = p.g[ax];
      b[ax] = (int)((((int64_t)g0 + G / 2) % G + G) % G);
    }
    base[m] = make_int2(b[0], b[1]);
    cell[m] = b[0] * p.g[1] + b[1];
  }
  // counting sort of the samples by first-tap cell (stable: equal cells keep sample order)
  const size_t ncell = (size_t)p.g[0] * p.g[1];
  std::vector<int32_t> cptr(ncell + 1, 0), sperm((size_t)M), scol((size_t)M);
  std::vector<int2> sbase((size_t)M);
  std::vector<float> swts((size_t)M * 16, 0.f);  // per sorted sample: w0 in [0, 8), w1 in [8, 16)
  for (int64_t m = 0; m < M; ++m) ++cptr[(size_t)cell[m] + 1];
  for (size_t q = 0; q < ncell; ++q) cptr[q + 1] += cptr[q];
  {
    std::vector<int32_t> fill(cptr.begin(), cptr.end() - 1);
    for (int64_t m = 0; m < M; ++m) {
      const int32_t s = fill[cell[m]]++;
      sperm[s] = (int32_t)m;
      scol[s] = base[m].y;
      sbase[s] = base[m];
      for (int t = 0; t < W; ++t) {
        swts[(size_t)s * 16 + t] = wts[(size_t)m * 2 * W + t];
        swts[(size_t)s * 16 + 8 + t] = wts[(size_t)m * 2 * W + W + t];
      }
    }
  }
  // Longest sample sequence of each plain spread block (SPREAD_ROWS grid rows from r0,
  // SPREAD_COLS columns): a lane of column c walks the W + R - 1 cell rows r0 + R - 1 - t and
  // in each the W cells c - W + 1 .. c.  Blocks above the threshold go, row by row, to the
  // split kernel.
  int split_min = SPREAD_SPLIT_DEFAULT;
  if (const char* env = std::getenv("MAXWELL_SPREAD_SPLIT")) split_min = std::max(0, std::atoi(env));
  if (const char* env = std::getenv("MAXWELL_SPREAD_LDS")) p.spread_lds = std::atoi(env) != 0;
  p.split_pm = SPREAD_SPLIT_PM;
  p.split_ph = SPREAD_SPLIT_PH;
  // coil groups that fill J: the spread reads a residual written in its sample order as is
  p.ordered_transfer = p.J % spread_group(p.J) == 0;
  if (const char* env = std::getenv("MAXWELL_SPREAD_SPLIT_PARTS")) {
    int pm = 0, ph = 0;
    auto pow2 = [](int v) { return v >= 1 && v <= 64 && (v & (v - 1)) == 0; };
    if (std::sscanf(env, "%d,%d", &pm, &ph) == 2 && pow2(pm) && pow2(ph)) {
      p.split_pm = pm;
      p.split_ph = ph;
    }
  }
  constexpr int R = SPREAD_ROWS;
  const int bc = (p.g[1] + SPREAD_COLS - 1) / SPREAD_COLS;
  const int nrg = (p.g[0] + R - 1) / R;
  std::vector<uint8_t> heavy((size_t)nrg * bc, 0);
  std::vector<int32_t> hlist, hot;  // split rows of moderately long and of the longest blocks
  {
    std::vector<int32_t> win(ncell);  // samples in the W cells ending at (row, c)
    for (int r = 0; r < p.g[0]; ++r)
      for (int c = 0; c < p.g[1]; ++c) {
        int32_t n = 0;
        for (int t = 0; t < W; ++t) {
          const int cc = ((c - t) % p.g[1] + p.g[1]) % p.g[1];
          const size_t q = (size_t)r * p.g[1] + cc;
          n += cptr[q + 1] - cptr[q];
        }
        win[(size_t)r * p.g[1] + c] = n;
      }
    for (int rg = 0; rg < nrg; ++rg)
      for (int b = 0; b < bc; ++b) {
        int32_t longest = 0;
        for (int c = b * SPREAD_COLS; c < std::min(p.g[1], (b + 1) * SPREAD_COLS); ++c) {
          int32_t n = 0;
          for (int t = 0; t < W + R - 1; ++t)
            n += win[(size_t)(((rg * R + R - 1 - t) % p.g[0] + p.g[0]) % p.g[0]) * p.g[1] + c];
          longest = std::max(longest, n);
        }
        if (longest > split_min) {
          heavy[(size_t)rg * bc + b] = 1;
          std::vector<int32_t>& dst = longest > 4 * std::max(split_min, 1) ? hot : hlist;
          for (int r = rg * R; r < std::min(p.g[0], rg * R + R); ++r) dst.push_back(r * bc + b);
        }
      }
  }
  p.n_med = (int)hlist.size();
  hlist.insert(hlist.end(), hot.begin(), hot.end());
  p.n_heavy = (int)hlist.size();
  auto up = [&](void** dst, const void* src, size_t bytes) -> hipError_t {
    hipError_t r = hipMalloc(dst, bytes ? bytes : 8);
    if (r != hipSuccess || !bytes) return r;
    return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  };
  if ((e = up((void**)&p.d_iphi, iphi.data(), iphi.size() * sizeof(float))) != hipSuccess) return hip_err(e);
  if ((e = up((void**)&p.d_cptr, cptr.data(), cptr.size() * sizeof(int32_t))) != hipSuccess) return hip_err(e);
  if ((e = up((void**)&p.d_sperm, sperm.data(), sperm.size() * sizeof(int32_t))) != hipSuccess) return hip_err(e);
  {
    std::vector<int32_t> sinv((size_t)M);
    for (int64_t s = 0; s < M; ++s) sinv[(size_t)sperm[(size_t)s]] = (int32_t)s;
    if ((e = up((void**)&p.d_sinv, sinv.data(), sinv.size() * sizeof(int32_t))) != hipSuccess) return hip_err(e);
  }
  if ((e = up((void**)&p.d_scol, scol.data(), scol.size() * sizeof(int32_t))) != hipSuccess) return hip_err(e);
  if ((e = up((void**)&p.d_swts, swts.data(), swts.size() * sizeof(float))) != hipSuccess) return hip_err(e);
  if ((e = up((void**)&p.d_sbase, sbase.data(), sbase.size() * sizeof(int2))) != hipSuccess) return hip_err(e);
  if ((e = up((void**)&p.d_sheavy, heavy.data(), heavy.size())) != hipSuccess) return hip_err(e);
  if ((e = up((void**)&p.d_shlist, hlist.data(), hlist.size() * sizeof(int32_t))) != hipSuccess) return hip_err(e);
  return MAXWELL_OK;
}

maxwell_status plan_build(Plan& p, const maxwell_plan_desc& d, const maxwell_basis_desc& b) {
  p.ndim = d.ndim;
  p.N = 1;
  for (int i = 0; i < 3; ++i) p.n[i] = i < d.ndim ? d.n[i] : 1;
  for (int i = 0; i < d.ndim; ++i) p.N *= d.n[i];
  p.J = d.J;
  p.K = b.K;
  p.M = d.M;
  p.precision = d.precision;
  p.sampling = d.sampling;
  p.basis_kind = b.kind;
  p.dense = reinterpret_cast<const float2*>(b.dense);
  for (int m = 0; m < 3; ++m) {
    p.r[m] = b.r[m];
    p.U[m] = reinterpret_cast<const float2*>(b.U[m]);
  }
  p.core = reinterpret_cast<const float2*>(b.core);


  auto hip_err = [&](hipError_t e) {
    set_last_error(std::string("HIP error during plan creation: ") + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? MAXWELL_ERR_OUT_OF_MEMORY : MAXWELL_ERR_HIP;
  };
  hipError_t e;
  // twiddle tables, exp(-2 pi i t / n), computed in FP64 and rounded
  double gs = 1.0;
  for (int ax = 0; ax < p.ndim; ++ax) {
    p.nrad[ax] = fft_factorise(p.n[ax], p.radix[ax]);
    std::vector<float2> tw(p.n[ax]);
    for (int64_t t = 0; t < p.n[ax]; ++t) {
      const double ang = -2.0 * M_PI * (double)t / (double)p.n[ax];
      tw[t] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    if ((e = hipMalloc(&p.d_tw[ax], tw.size() * sizeof(float2))) != hipSuccess) return hip_err(e);
    if ((e = hipMemcpy(p.d_tw[ax], tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_err(e);
    gs *= (((p.n[ax] / 2) & 1) ? -1.0 : 1.0) / std::sqrt((double)p.n[ax]);
  }
  p.gscale = (float)gs;
  // fused 3D Tucker path?
  std::vector<int32_t> pos;
  if (p.basis_kind == MAXWELL_BASIS_TUCKER && p.ndim == 3 &&
      fused_supported(p.n[0], p.n[1], p.n[2], p.r[0], p.r[1], p.precision) && detect_lines(d, pos)) {
    p.fused = true;
    p.L = (int64_t)pos.size();
    {
      // coils per plane workgroup: the largest group (up to 16) that still gives every
      // compute unit a workgroup; larger groups amortise the per-workgroup set-up (the
      // forward's x share, held in registers across the group's coils) and, in the adjoint,
      // mean fewer gx partials to sum
      int dev = 0, cus = 256;
      if (hipGetDevice(&dev) == hipSuccess &&
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
      auto pick = [&](int gmax) {
        int G = gmax;
        while (G > 1 && p.n[2] * ((p.J + G - 1) / G) < cus) G /= 2;
        return G;
      };
      p.G_fwd = pick(16);
      p.G_adj = pick(16);
    }
    if ((e = hipMalloc(&p.d_pos, pos.size() * sizeof(int32_t))) != hipSuccess) return hip_err(e);
    if ((e = hipMemcpy(p.d_pos, pos.data(), pos.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_err(e);
    // factor operands of the plane kernels in fragment order
    const int n0 = (int)p.n[0], n1 = (int)p.n[1], r0 = (int)p.r[0], r1 = (int)p.r[1], pr = p.precision;
    const size_t bU0F = frag_operand_bytes(n0, r0, 0, pr), bU1TF = frag_operand_bytes(n1, r1, 1, pr);
    const size_t bU1CF = frag_operand_bytes(r1, n1, 1, pr), bU0HF = frag_operand_bytes(r0, n0, 0, pr);
    const int n2 = (int)p.n[2], r2 = (int)p.r[2];
    p.mode3_direct = mode3_supported(r2);
    const size_t bU2F = p.mode3_direct ? frag_operand_bytes(n2, r2, 0, pr) : 0;
    const size_t bU2CF = p.mode3_direct ? frag_operand_bytes(r2, n2, 1, pr) : 0;
    if ((e = hipMalloc(&p.d_frag, 2 * (bU0F + bU1TF) + bU1CF + bU0HF + bU2F + bU2CF)) != hipSuccess) return hip_err(e);
    char* q = reinterpret_cast<char*>(p.d_frag);
    p.U0F = q; q += bU0F;
    p.U1TF = q; q += bU1TF;
    p.U0SF = q; q += bU0F;
    p.U1TSF = q; q += bU1TF;
    p.U1CF = q; q += bU1CF;
    p.U0HF = q; q += bU0HF;
    p.U2F = q; q += bU2F;
    p.U2CF = q;
    const int kp = pr == 0 ? 4 : 0;  // FP32: the rank order of the plane kernels' rank reductions
    if ((e = frag_operand_launch(p.U[0], n0, r0, r0, 1, kp, 0, pr, const_cast<void*>(p.U0F), 0)) ||
        (e = frag_operand_launch(p.U[1], n1, r1, r1, 1, kp, 1, pr, const_cast<void*>(p.U1TF), 0)) ||
        (e = frag_operand_launch(p.U[0], n0, r0, r0, 1, 2 | kp, 0, pr, const_cast<void*>(p.U0SF), 0)) ||
        (e = frag_operand_launch(p.U[1], n1, r1, r1, 1, 2 | kp, 1, pr, const_cast<void*>(p.U1TSF), 0)) ||
        (e = frag_operand_launch(p.U[1], r1, n1, 1, r1, 1, 1, pr, const_cast<void*>(p.U1CF), 0)) ||
        (e = frag_operand_launch(p.U[0], r0, n0, 1, r0, 1, 0, pr, const_cast<void*>(p.U0HF), 0)))
      return hip_err(e);
    if (p.mode3_direct &&
        ((e = frag_operand_launch(p.U[2], n2, r2, r2, 1, 0, 0, pr, const_cast<void*>(p.U2F), 0)) ||
         (e = frag_operand_launch(p.U[2], r2, n2, 1, r2, 1, 1, pr, const_cast<void*>(p.U2CF), 0))))
      return hip_err(e);
    if ((e = hipStreamSynchronize(0)) != hipSuccess) return hip_err(e);
  }
  if (p.basis_kind == MAXWELL_BASIS_TUCKER && core_supported(p.J)) {
    p.core_direct = true;
    p.cg = core_geom(p.r[0] * p.r[1] * p.r[2], (int)p.K);
    if (p.precision == MAXWELL_BF16_SPLIT) {
      if ((e = hipMalloc(&p.d_core_split, p.cg.total_elems() * sizeof(uint16_t))) != hipSuccess) return hip_err(e);
      if ((e = core_split_launch(p.core, p.cg, p.d_core_split, 0)) != hipSuccess) return hip_err(e);
      if ((e = hipStreamSynchronize(0)) != hipSuccess) return hip_err(e);
    } else {
      const size_t n32 = p.cg.fwd32_elems() + p.cg.adj32_elems();
      if ((e = hipMalloc(&p.d_core_f32, n32 * sizeof(float2))) != hipSuccess) return hip_err(e);
      if ((e = core_frag32_launch(p.core, p.cg, p.d_core_f32, 0)) != hipSuccess) return hip_err(e);
      if ((e = hipStreamSynchronize(0)) != hipSuccess) return hip_err(e);
    }
  }
  if (p.sampling == MAXWELL_NONCARTESIAN) {
    maxwell_status ns = nufft_build(p, d);
    if (ns != MAXWELL_OK) return ns;
  }
  // mask tables (general Cartesian path)
  if (!p.fused && p.sampling == MAXWELL_CARTESIAN) {
    std::vector<int32_t> idx(p.M), inv(p.N, -1);
    for (int64_t m = 0; m < p.M; ++m) {
      idx[m] = (int32_t)d.mask_idx[m];
      inv[d.mask_idx[m]] = (int32_t)m;
    }
    if (p.M > 0) {
      if ((e = hipMalloc(&p.d_mask, p.M * sizeof(int32_t))) != hipSuccess) return hip_err(e);
      if ((e = hipMemcpy(p.d_mask, idx.data(), p.M * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_err(e);
    }
    if ((e = hipMalloc(&p.d_inv, p.N * sizeof(int32_t))) != hipSuccess) return hip_err(e);
    if ((e = hipMemcpy(p.d_inv, inv.data(), p.N * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_err(e);
    // samples before each line of the last axis (the mask is strictly ascending)
    const int64_t nl = p.n[p.ndim - 1], lines = p.N / nl;
    std::vector<int32_t> lptr(lines + 1, 0);
    for (int64_t m = 0; m < p.M; ++m) ++lptr[d.mask_idx[m] / nl + 1];
    for (int64_t l = 0; l < lines; ++l) lptr[l + 1] += lptr[l];
    if ((e = hipMalloc(&p.d_lptr, lptr.size() * sizeof(int32_t))) != hipSuccess) return hip_err(e);
    if ((e = hipMemcpy(p.d_lptr, lptr.data(), lptr.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_err(e);
  }
  if (d.weights && p.M > 0) {
    if ((e = hipMalloc(&p.d_w, p.M * sizeof(float))) != hipSuccess) return hip_err(e);
    if ((e = hipMemcpy(p.d_w, d.weights, p.M * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_err(e);
  }

  // dense basis: for each of the two basis products, the streaming kernel (few coils) or the
  // tiled GEMM at one split-K factor, picked by timing the candidates on scratch operands of
  // the plan's shapes; the choices persist in the tuning cache (tune.h), keyed by the GPU
  // architecture and the shape.  MAXWELL_GEMM_AUTOTUNE=0: the rule (streaming apply where
  // supported, streaming adjoint up to 16 coils, no split) without timing.
  if (p.basis_kind == MAXWELL_BASIS_DENSE && !p.fused && p.J > 0 && p.K > 0 && p.N > 0) {
    const bool stream_ok = skinny_apply_supported(p.N, p.K, p.J) && (reinterpret_cast<uintptr_t>(p.dense) & 15u) == 0;
    const char* env = std::getenv("MAXWELL_GEMM_AUTOTUNE");
    if (env && env[0] == '0') {
      p.skinny_apply = stream_ok;
      p.skinny_adj = stream_ok && p.J <= 16;
    } else {
      const size_t nbuf = (size_t)p.J * std::max<int64_t>(p.N, p.K) * 8;  // c, S, h and gc all fit
      const size_t max_ws = (size_t)256 << 20;
      void *bufA = nullptr, *bufC = nullptr, *bufW = nullptr;
      bool ok = hipMalloc(&bufA, nbuf) == hipSuccess && hipMalloc(&bufC, nbuf) == hipSuccess &&
                hipMalloc(&bufW, max_ws) == hipSuccess && hipMemset(bufA, 0, nbuf) == hipSuccess &&
                hipMemset(bufC, 0, nbuf) == hipSuccess;
      if (ok) {
        const float2* A = reinterpret_cast<const float2*>(bufA);
        float2* C = reinterpret_cast<float2*>(bufC);
        // time per launch of one candidate (a warm-up, then three launches)
        auto time_ms = [&](const std::function<hipError_t()>& launch) -> float {
          hipEvent_t e0, e1;
          if (hipEventCreate(&e0) != hipSuccess) return -1.f;
          if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return -1.f; }
          bool good = launch() == hipSuccess && hipEventRecord(e0, 0) == hipSuccess;
          for (int r = 0; good && r < 3; ++r) good = launch() == hipSuccess;
          float ms = -1.f;
          if (good && hipEventRecord(e1, 0) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
              hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
            ms /= 3.f;
          else
            ms = -1.f;
          (void)hipEventDestroy(e0);
          (void)hipEventDestroy(e1);
          (void)hipGetLastError();
          return ms;
        };
        std::ostringstream shape;
        shape << device_arch() << " N=" << p.N << " K=" << p.K << " J=" << p.J << " prec=" << p.precision
              << " stream=" << (stream_ok ? 1 : 0);
        const int ca = tuned_choice("dense_apply " + shape.str(), [&]() -> int {
          float gemm_ms = -1.f;
          const int split = gemm_autotune(dense_apply_args(p, A, C), p.precision, bufW, max_ws, 0, &gemm_ms);
          if (!stream_ok || skinny_frag_bytes(p.K, p.J) > max_ws) return split;
          const float sk = time_ms([&]() { return skinny_apply_launch(p.dense, p.N, p.K, A, p.J, p.precision, bufW, C, 0); });
          return (sk > 0.f && (gemm_ms <= 0.f || sk < gemm_ms)) ? -1 : split;
        });
        const int cd = tuned_choice("dense_adjoint " + shape.str(), [&]() -> int {
          float gemm_ms = -1.f;
          const int split = gemm_autotune(dense_adjoint_args(p, A, C), p.precision, bufW, max_ws, 0, &gemm_ms);
          if (!stream_ok || skinny_adjoint_bytes(p.N, p.K, p.J) > max_ws) return split;
          const float sk = time_ms([&]() {
            return skinny_adjoint_launch(p.dense, p.N, p.K, A, p.J, p.precision, 1.0f, nullptr, bufW, C, 0);
          });
          return (sk > 0.f && (gemm_ms <= 0.f || sk < gemm_ms)) ? -1 : split;
        });
        p.skinny_apply = ca < 0;
        p.skinny_adj = cd < 0;
        p.split_apply = ca < 0 ? 0 : ca;
        p.split_adj = cd < 0 ? 0 : cd;
      } else {
        p.skinny_apply = stream_ok;
        p.skinny_adj = stream_ok && p.J <= 16;
      }
      (void)hipStreamSynchronize(0);
      if (bufA) (void)hipFree(bufA);
      if (bufC) (void)hipFree(bufC);
      if (bufW) (void)hipFree(bufW);
      (void)hipGetLastError();
    }
  }

  // workspace layout
  const size_t JN = (size_t)p.J * (size_t)p.N * 8, JM = (size_t)p.J * (size_t)p.M * 8;
  size_t off = 0;
  size_t gemm_ws = 0;
  if (!p.fused) {
    p.off_S = off; off += al(JN);
    p.off_K = off; off += al(JN);
  }
  if (p.basis_kind == MAXWELL_BASIS_TUCKER) {
    const size_t R = (size_t)(p.r[0] * p.r[1] * p.r[2]);
    size_t tA = std::max((size_t)p.J * R, (size_t)p.J * p.n[0] * p.n[1] * p.r[2]) * 8;
    size_t tB = (size_t)p.J * p.n[0] * p.r[1] * p.r[2] * 8;
    p.off_tA = off; off += al(tA);
    p.off_tB = off; off += al(tB);
    GemmArgs g[4];
    tucker_apply_args(p, nullptr, nullptr, nullptr, nullptr, g);
    for (int i = 0; i < 4; ++i) gemm_ws = std::max(gemm_ws, gemm_workspace_bytes(g[i]));
    tucker_adjoint_args(p, nullptr, nullptr, nullptr, nullptr, g);
    for (int i = 0; i < 4; ++i) gemm_ws = std::max(gemm_ws, gemm_workspace_bytes(g[i]));
  } else {
    gemm_ws = std::max(gemm_workspace_bytes(dense_apply_args(p, nullptr, nullptr)),
                       gemm_workspace_bytes(dense_adjoint_args(p, nullptr, nullptr)));
  }
  if (p.fused) {
    const size_t R = (size_t)(p.r[0] * p.r[1] * p.r[2]);
    const size_t T3 = (size_t)p.J * p.n[2] * p.r[0] * p.r[1] * 8;
    const int ngrp = (p.J + p.G_adj - 1) / p.G_adj;
    p.off_T1 = off; off += al((size_t)p.J * R * 8);
    p.off_T3 = off; off += al(T3);
    p.off_xt = off; off += al((size_t)p.N * 8);
    p.off_Z = off; off += al(JM);
    p.off_gxp = off; off += al((size_t)ngrp * p.N * 8);
    p.off_T3b = off; off += al(T3);
    p.off_T1b = off; off += al((size_t)p.J * R * 8);
    gemm_ws = std::max(gemm_ws, gemm_workspace_bytes(fused_T3_args(p, nullptr, nullptr)));
    gemm_ws = std::max(gemm_ws, gemm_workspace_bytes(fused_T1b_args(p, nullptr, nullptr)));
  }
  if (p.sampling == MAXWELL_NONCARTESIAN) {
    p.off_G = off;
    off += al((size_t)p.J * p.g[0] * p.g[1] * 8);
    p.off_Ys = off;
    off += al(spread_stage_bytes(p.J, p.M));
  }
  if (p.core_direct) {
    p.off_cpart = off;
    off += al(core_adj_part_bytes(p.cg.R, p.cg.K, p.J));
  }
  if (p.skinny_apply) {
    p.off_cfrag = off;
    off += al(skinny_frag_bytes(p.K, p.J));
  }
  if (p.skinny_adj) {
    p.off_adjp = off;
    off += al(skinny_adjoint_bytes(p.N, p.K, p.J));
  }
  p.off_E = off; off += al(JM);
  p.off_gemm = off; off += al(gemm_ws);
  p.part_blocks = residual_blocks((int64_t)p.J * p.M);
  if (p.fused) p.part_blocks = std::max(p.part_blocks, line_blocks(p.J, p.L));
  p.off_part = off; off += al((size_t)p.part_blocks * sizeof(double));
  // Gauss-Newton / CG: the JVP result, the work vectors r, d, q ([N | J K] each), and the
  // FP64 scalars and inner-product partials
  const size_t V = ((size_t)p.N + (size_t)p.J * (size_t)p.K) * 8;
  p.off_U = off; off += al(JM);
  p.off_cg = off; off += 3 * al(V) + al(CG_SCALARS * sizeof(double)) + al(DOT_BLOCKS * sizeof(double));
  if (!p.fused) {
    // SENSE / ADMM (general path): 5 + 2 ndim image-sized buffers (z0 twice, u0, two
    // temporaries, the TV dual field twice), 5 sample-sized ones (F S p, z_k
    // twice, u_k, a temporary), the ball-projection partials and the ADMM scalars
    const size_t NB = al((size_t)p.N * 8);
    p.off_admm = off;
    off += (5 + 2 * p.ndim) * NB + 5 * al(JM) + al((size_t)ball_part_doubles(p.J) * sizeof(double)) +
           al(ADMM_SCALARS * sizeof(double));
  }
  p.ws_bytes = off;
  return MAXWELL_OK;
}

void plan_release(Plan& p) {
  for (int ax = 0; ax < 2; ++ax) {
    if (p.d_twg[ax]) (void)hipFree(p.d_twg[ax]);
    p.d_twg[ax] = nullptr;
  }
  if (p.d_iphi) (void)hipFree(p.d_iphi);
  if (p.d_cptr) (void)hipFree(p.d_cptr);
  if (p.d_sperm) (void)hipFree(p.d_sperm);
  if (p.d_sinv) (void)hipFree(p.d_sinv);
  if (p.d_scol) (void)hipFree(p.d_scol);
  if (p.d_swts) (void)hipFree(p.d_swts);
  if (p.d_sbase) (void)hipFree(p.d_sbase);
  if (p.d_sheavy) (void)hipFree(p.d_sheavy);
  if (p.d_shlist) (void)hipFree(p.d_shlist);
  p.d_iphi = nullptr;
  p.d_cptr = nullptr;
  p.d_sperm = nullptr;
  p.d_sinv = nullptr;
  p.d_scol = nullptr;
  p.d_swts = nullptr;
  p.d_sbase = nullptr;
  p.d_sheavy = nullptr;
  p.d_shlist = nullptr;
  p.n_heavy = 0;
  p.n_med = 0;
  for (auto e : p.timing.ev_start) (void)hipEventDestroy(e);
  for (auto e : p.timing.ev_stop) (void)hipEventDestroy(e);
  p.timing = Timing();
  for (int ax = 0; ax < 3; ++ax) {
    if (p.d_tw[ax]) (void)hipFree(p.d_tw[ax]);
    p.d_tw[ax] = nullptr;
  }
  if (p.d_mask) (void)hipFree(p.d_mask);
  if (p.d_inv) (void)hipFree(p.d_inv);
  if (p.d_lptr) (void)hipFree(p.d_lptr);
  if (p.d_w) (void)hipFree(p.d_w);
  if (p.d_pos) (void)hipFree(p.d_pos);
  if (p.d_frag) (void)hipFree(p.d_frag);
  p.d_frag = nullptr;
  if (p.d_core_split) (void)hipFree(p.d_core_split);
  p.d_core_split = nullptr;
  if (p.d_core_f32) (void)hipFree(p.d_core_f32);
  p.d_core_f32 = nullptr;
  p.d_mask = nullptr;
  p.d_inv = nullptr;
  p.d_lptr = nullptr;
  p.d_w = nullptr;
  p.d_pos = nullptr;
}

static CoreArgs core_args(const Plan& p, const float2* in, float2* out, void* ws) {
  CoreArgs a{};
  a.g = p.cg;
  a.J = p.J;
  a.core = p.core;
  if (p.d_core_split) {
    const size_t nf = p.cg.fwd_elems(), na = p.cg.adj_elems();
    a.fwd_hi = p.d_core_split;
    a.fwd_lo = p.d_core_split + nf;
    a.adj_hi = p.d_core_split + 2 * nf;
    a.adj_lo = p.d_core_split + 2 * nf + na;
  }
  if (p.d_core_f32) {
    a.fwd_f32 = p.d_core_f32;
    a.adj_f32 = p.d_core_f32 + p.cg.fwd32_elems();
  }
  a.in = in;
  a.out = out;
  a.part = wsp<float2>(ws, p.off_cpart);
  return a;
}

// T1 = core x_4 c  (first product of the Tucker chain)
static hipError_t core_forward(const Plan& p, const float2* c, float2* T1, void* ws, hipStream_t st) {
  if (p.core_direct) return TIMED("core_fwd", core_fwd_launch(core_args(p, c, T1, ws), p.precision, st));
  GemmArgs g[4];
  tucker_apply_args(p, c, T1, nullptr, nullptr, g);
  return TIMED("gemm_core_coef", gemm_launch(g[0], p.precision, wsp<void>(ws, p.off_gemm), st));
}

// gc = alpha (*alpha_dev) core^H T1b  (last product of the adjoint chain)
static hipError_t core_adjoint(const Plan& p, const float2* T1b, float2* gc, float alpha, const float* alpha_dev,
                               void* ws, hipStream_t st) {
  if (p.core_direct)
    return TIMED("core_adj", core_adj_launch(core_args(p, T1b, gc, ws), p.precision, alpha, alpha_dev, st));
  GemmArgs g[4];
  tucker_adjoint_args(p, nullptr, const_cast<float2*>(T1b), nullptr, gc, g);
  g[3].alpha = alpha;
  g[3].alpha_dev = alpha_dev;
  return TIMED("gemm_core_adjoint", gemm_launch(g[3], p.precision, wsp<void>(ws, p.off_gemm), st));
}

hipError_t run_basis_apply(const Plan& p, const float2* c, float2* S, void* ws, hipStream_t st) {
  void* gws = wsp<void>(ws, p.off_gemm);
  if (p.basis_kind == MAXWELL_BASIS_DENSE) {
    if (p.off_cfrag)  // streaming kernel for few coils
      return TIMED("gemm_dense_apply", skinny_apply_launch(p.dense, p.N, p.K, c, p.J, p.precision,
                                                           wsp<void>(ws, p.off_cfrag), S, st));
    return TIMED("gemm_dense_apply", gemm_launch(dense_apply_args(p, c, S), p.precision, gws, st));
  }
  GemmArgs g[4];
  tucker_apply_args(p, c, wsp<float2>(ws, p.off_tA), wsp<float2>(ws, p.off_tB), S, g);
  hipError_t e0 = core_forward(p, c, wsp<float2>(ws, p.off_tA), ws, st);
  if (e0 != hipSuccess) return e0;
  for (int i = 1; i < 4; ++i) {
    hipError_t e = TIMED("gemm_tucker_chain", gemm_launch(g[i], p.precision, gws, st));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t run_basis_adjoint(const Plan& p, const float2* S, float2* c, float alpha, const float* alpha_dev,
                             void* ws, hipStream_t st) {
  void* gws = wsp<void>(ws, p.off_gemm);
  if (p.basis_kind == MAXWELL_BASIS_DENSE && p.off_adjp)  // streaming kernel for up to 16 coils
    return TIMED("gemm_dense_adjoint", skinny_adjoint_launch(p.dense, p.N, p.K, S, p.J, p.precision, alpha,
                                                             alpha_dev, wsp<void>(ws, p.off_adjp), c, st));
  if (p.basis_kind == MAXWELL_BASIS_DENSE) {
    GemmArgs g = dense_adjoint_args(p, S, c);
    g.alpha = alpha;
    g.alpha_dev = alpha_dev;
    return TIMED("gemm_dense_adjoint", gemm_launch(g, p.precision, gws, st));
  }
  GemmArgs g[4];
  tucker_adjoint_args(p, S, wsp<float2>(ws, p.off_tA), wsp<float2>(ws, p.off_tB), c, g);
  for (int i = 0; i < 3; ++i) {
    hipError_t e = TIMED("gemm_tucker_adjoint_chain", gemm_launch(g[i], p.precision, gws, st));
    if (e != hipSuccess) return e;
  }
  return core_adjoint(p, wsp<float2>(ws, p.off_tA), c, alpha, alpha_dev, ws, st);
}

// ---- fused path pieces
static hipError_t fused_prepare(const Plan& p, const float2* x, const float2* c, void* ws, hipStream_t st) {
  void* gws = wsp<void>(ws, p.off_gemm);
  hipError_t e = core_forward(p, c, wsp<float2>(ws, p.off_T1), ws, st);
  if (e != hipSuccess) return e;
  if (p.mode3_direct) {
    Mode3Args m = mode3_args(p);
    m.T1 = wsp<float2>(ws, p.off_T1);
    m.T3 = wsp<float2>(ws, p.off_T3);
    e = TIMED("mode3_fwd", mode3_fwd_launch(m, p.precision, st));
  } else {
    e = TIMED("gemm_mode3", gemm_launch(fused_T3_args(p, wsp<float2>(ws, p.off_T1), wsp<float2>(ws, p.off_T3)),
                                        p.precision, gws, st));
  }
  if (e != hipSuccess) return e;
  return TIMED("transpose_x", transpose_launch(x, p.n[0] * p.n[1], p.n[2], (int)p.n[1], wsp<float2>(ws, p.off_xt), st));
}

// out: E (y null) or the weighted residual; with `transfer` (y given) the residual goes out
// in the transfer layout: taken back along the readout by the line kernel itself.
static hipError_t fused_forward(const Plan& p, const float2* x, const float2* c, const float2* y, float2* out,
                                double* part, void* ws, hipStream_t st, bool transfer) {
  hipError_t e = fused_prepare(p, x, c, ws, st);
  if (e != hipSuccess) return e;
  PlaneArgs pa = plane_args(p, ws, p.G_fwd);
  if ((e = TIMED("plane_fwd", plane_fwd_launch(pa, st))) != hipSuccess) return e;
  LineArgs la = line_args(p);
  la.Z = wsp<float2>(ws, p.off_Z);
  la.out = transfer ? nullptr : out;
  la.Zw = transfer ? out : nullptr;
  la.y = y;
  la.w = y ? p.d_w : nullptr;
  la.part = part;
  return TIMED("line_fwd", line_fwd_launch(la, st));
}

// y: samples [J][M], or (transfer) a residual already in the transfer layout, in which
// case the line kernel is skipped and the scale is applied where gx and gc are written.
static hipError_t fused_adjoint(const Plan& p, const float2* x, const float2* c, const float2* y, float alpha,
                                const float* scale_dev, float2* gx, float2* gc, void* ws, hipStream_t st,
                                bool prepared, bool transfer) {
  hipError_t e;
  if (!prepared) {
    if (gx) {
      if ((e = fused_prepare(p, x, c, ws, st)) != hipSuccess) return e;
    } else {
      e = TIMED("transpose_x", transpose_launch(x, p.n[0] * p.n[1], p.n[2], (int)p.n[1], wsp<float2>(ws, p.off_xt), st));
      if (e != hipSuccess) return e;
    }
  }
  // the scale: in the line kernel, or (transfer) where the outputs are written
  const float end_alpha = transfer ? alpha : 1.0f;
  const float* end_scale = transfer ? scale_dev : nullptr;
  PlaneArgs pa = plane_args(p, ws, p.G_adj);
  if (transfer) {
    pa.Z = const_cast<float2*>(y);  // read only by the adjoint plane kernel
  } else {
    LineArgs la = line_args(p);
    la.yin = y;
    la.Zw = wsp<float2>(ws, p.off_Z);
    la.alpha = alpha;
    la.scale_dev = scale_dev;
    if ((e = TIMED("line_adj", line_adj_launch(la, st))) != hipSuccess) return e;
  }
  pa.gxpart = gx ? wsp<float2>(ws, p.off_gxp) : nullptr;
  pa.T3b = gc ? wsp<float2>(ws, p.off_T3b) : nullptr;
  if ((e = TIMED("plane_adj", plane_adj_launch(pa, st))) != hipSuccess) return e;
  if (gx) {
    const int ngrp = (p.J + p.G_adj - 1) / p.G_adj;
    e = TIMED("gx_reduce", reduce_transpose_launch(pa.gxpart, ngrp, p.n[0] * p.n[1], p.n[2], end_alpha, end_scale,
                                                   gx, st));
    if (e != hipSuccess) return e;
  }
  if (gc) {
    if (p.mode3_direct) {
      Mode3Args m = mode3_args(p);
      m.T3b = pa.T3b;
      m.T1b = wsp<float2>(ws, p.off_T1b);
      e = TIMED("mode3_adj", mode3_adj_launch(m, p.precision, st));
    } else {
      void* gws = wsp<void>(ws, p.off_gemm);
      e = TIMED("gemm_mode3_adjoint",
                gemm_launch(fused_T1b_args(p, pa.T3b, wsp<float2>(ws, p.off_T1b)), p.precision, gws, st));
    }
    if (e != hipSuccess) return e;
    if ((e = core_adjoint(p, wsp<float2>(ws, p.off_T1b), gc, end_alpha, end_scale, ws, st)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

// The Cartesian mask is applied inside the first inverse and the last forward FFT pass
// (no separate gather or scatter) when there are samples and J N < 2^31.
static bool fuse_sampling(const Plan& p) {
  return p.sampling == MAXWELL_CARTESIAN && p.M > 0 && p.ndim >= 2 && p.d_inv && (int64_t)p.J * p.N < 0x7fffffffLL;
}

// y = F_s(S (.) x) for coil maps S [J][N] already in memory (general path)
static hipError_t encode_maps(const Plan& p, const float2* S, const float2* x, float2* y, void* ws, hipStream_t st) {
  hipError_t e;
  if (p.sampling == MAXWELL_NONCARTESIAN) {
    const NufftArgs na = nufft_args(p);
    float2* G = wsp<float2>(ws, p.off_G);
    if ((e = fft_grid_window(p, S, x, G, nullptr, -1, st)) != hipSuccess) return e;  // zero-pad in the first pass
    return TIMED("nufft_degrid", degrid_launch(na, G, y, st));
  }
  float2* Kb = wsp<float2>(ws, p.off_K);
  if (fuse_sampling(p))  // the last pass writes the sampled points straight to y
    return fft_dims(p, S, Kb, -1, x, p.ndim, p.n, p.d_tw, p.nrad, p.radix, st, nullptr, y);
  if ((e = fft_image(p, S, Kb, -1, x, st)) != hipSuccess) return e;
  return TIMED("gather", gather_launch(Kb, p.N, p.d_mask, p.M, p.J, y, st));
}

hipError_t run_encode(const Plan& p, const float2* x, const float2* c, float2* y, void* ws, hipStream_t st) {
  if (p.fused) return fused_forward(p, x, c, nullptr, y, nullptr, ws, st, false);
  float2* S = wsp<float2>(ws, p.off_S);
  hipError_t e = run_basis_apply(p, c, S, ws, st);
  if (e != hipSuccess) return e;
  return encode_maps(p, S, x, y, ws, st);
}

hipError_t run_forward_loss(const Plan& p, const float2* x, const float2* c, const float2* y, float2* r,
                            double* loss, void* ws, hipStream_t st, bool transfer) {
  double* part = wsp<double>(ws, p.off_part);
  hipError_t e;
  if (p.fused) {
    if ((e = fused_forward(p, x, c, y, r, part, ws, st, transfer && r)) != hipSuccess) return e;
    if (loss) return TIMED("reduce_loss", reduce_loss_launch(part, line_blocks(p.J, p.L), loss, st));
    return hipSuccess;
  }
  float2* E = wsp<float2>(ws, p.off_E);
  if ((e = run_encode(p, x, c, E, ws, st)) != hipSuccess) return e;
  if (transfer && r && p.sampling == MAXWELL_NONCARTESIAN && p.ordered_transfer) {
    // the transfer layout of the gridding path: the residual in the spread's sample order
    const int32_t* inv = p.d_sinv;
    if ((e = TIMED("residual", residual_ordered_launch(E, y, p.d_w, p.M, p.J, inv, r, part, st))) != hipSuccess)
      return e;
  } else if ((e = TIMED("residual", residual_launch(E, y, p.d_w, p.M, p.J, r, part, st))) != hipSuccess) {
    return e;
  }
  if (loss) return TIMED("reduce_loss", reduce_loss_launch(part, residual_blocks((int64_t)p.J * p.M), loss, st));
  return hipSuccess;
}

// gx = s sum_j conj(S_j) (.) F_s^H y_j for coil maps S [J][N] (general path), s = alpha *
// (*scale_dev); with want_h the K region of the workspace is left holding
// h_j = s conj(x) (.) F_s^H y_j, the input of the basis adjoint.
static hipError_t adjoint_maps(const Plan& p, const float2* S, const float2* x, const float2* y, float alpha,
                               const float* scale_dev, float2* gx, bool want_h, void* ws, hipStream_t st,
                               bool ordered = false) {
  float2* Kb = wsp<float2>(ws, p.off_K);
  hipError_t e;
  if (p.sampling == MAXWELL_NONCARTESIAN) {
    const NufftArgs na = nufft_args(p);
    float2* G = wsp<float2>(ws, p.off_G);
    // `ordered`: y is a residual written in the spread's sample order (no staging pass)
    if ((e = TIMED("nufft_spread", spread_launch(na, y, alpha, scale_dev, wsp<float2>(ws, p.off_Ys), G, st,
                                                 ordered))) !=
        hipSuccess)
      return e;
    if ((e = fft_grid_window(p, nullptr, nullptr, G, Kb, +1, st)) != hipSuccess) return e;  // crop in the last pass
    alpha = 1.0f;  // the scale was applied by the spread
    scale_dev = nullptr;
  } else {
    if (fuse_sampling(p)) {  // the first pass reads the samples through the inverse mask
      if ((e = fft_dims(p, Kb, Kb, +1, nullptr, p.ndim, p.n, p.d_tw, p.nrad, p.radix, st, y, nullptr)) !=
          hipSuccess)
        return e;
    } else {
      if ((e = TIMED("scatter", scatter_launch(y, p.M, p.d_inv, p.N, p.J, Kb, st))) != hipSuccess) return e;
      if ((e = fft_image(p, Kb, Kb, +1, nullptr, st)) != hipSuccess) return e;
    }
  }
  return TIMED("adjoint_combine", adjoint_combine_launch(S, Kb, x, p.N, p.J, alpha, scale_dev, gx, want_h ? 1 : 0, st));
}

hipError_t run_adjoint(const Plan& p, const float2* x, const float2* c, const float2* y, float alpha,
                       const float* scale_dev, float2* gx, float2* gc, void* ws, hipStream_t st,
                       bool maps_ready, bool transfer) {
  if (p.fused) return fused_adjoint(p, x, c, y, alpha, scale_dev, gx, gc, ws, st, maps_ready, transfer);
  float2* S = wsp<float2>(ws, p.off_S);
  float2* Kb = wsp<float2>(ws, p.off_K);
  hipError_t e;
  if (gx && !maps_ready) {
    if ((e = run_basis_apply(p, c, S, ws, st)) != hipSuccess) return e;
  }
  const bool ordered = transfer && p.sampling == MAXWELL_NONCARTESIAN && p.ordered_transfer;
  if ((e = adjoint_maps(p, S, x, y, alpha, scale_dev, gx, gc != nullptr, ws, st, ordered)) != hipSuccess) return e;
  if (gc) return run_basis_adjoint(p, Kb, gc, 1.0f, nullptr, ws, st);
  return hipSuccess;
}

hipError_t run_grad(const Plan& p, const float2* x, const float2* c, const float2* y, float2* gx, float2* gc,
                    double* loss, void* ws, hipStream_t st) {
  const bool want = gx || gc;
  // the residual in the transfer layout; on the fused path in place of the plane output
  // (each line workgroup reads its lines before writing them); on the gridding path in the
  // spread's sample order, in its staging region (a permuted write cannot be in place)
  float2* r = !want                ? nullptr
              : p.fused            ? wsp<float2>(ws, p.off_Z)
              : p.sampling == MAXWELL_NONCARTESIAN && p.ordered_transfer ? wsp<float2>(ws, p.off_Ys)
                                   : wsp<float2>(ws, p.off_E);
  hipError_t e = run_forward_loss(p, x, c, y, r, loss, ws, st, true);
  if (e != hipSuccess) return e;
  if (!want) return hipSuccess;
  return run_adjoint(p, x, c, r, 2.0f, nullptr, gx, gc, ws, st, true, true);
}

// ---- Gauss-Newton step (Sec. II-B, Eq. (6) and Eq. (7))

// J[dx, dc] = E(dx, c) + E(x, dc): E is bilinear, so the Jacobian-vector product of Eq. (7)
// is two encodes; the second goes through the E region of the workspace.
hipError_t run_jvp(const Plan& p, const float2* x, const float2* c, const float2* dx, const float2* dc, float2* y,
                   void* ws, hipStream_t st) {
  hipError_t e = run_encode(p, dx, c, y, ws, st);
  if (e != hipSuccess) return e;
  float2* E = wsp<float2>(ws, p.off_E);
  if ((e = run_encode(p, x, dc, E, ws, st)) != hipSuccess) return e;
  return TIMED("jvp_sum", caxpy_launch(y, E, 1.0f, (int64_t)p.J * p.M, st));
}

// (ox, oc) = J^H (w (.) J[dx, dc]) + (lam_x dx, lam_c dc)
hipError_t run_normal(const Plan& p, const float2* x, const float2* c, const float2* dx, const float2* dc,
                      float lam_x, float lam_c, float2* ox, float2* oc, void* ws, hipStream_t st) {
  float2* u = wsp<float2>(ws, p.off_U);
  hipError_t e = run_jvp(p, x, c, dx, dc, u, ws, st);
  if (e != hipSuccess) return e;
  if (p.d_w && (e = TIMED("weights", weight_rows_launch(u, p.d_w, p.M, p.J, st))) != hipSuccess) return e;
  if ((e = run_adjoint(p, x, c, u, 1.0f, nullptr, ox, oc, ws, st, false, false)) != hipSuccess) return e;
  if ((e = TIMED("normal_axpy", caxpy_launch(ox, dx, lam_x, p.N, st))) != hipSuccess) return e;
  return TIMED("normal_axpy", caxpy_launch(oc, dc, lam_c, (int64_t)p.J * p.K, st));
}

// iters steps of conjugate gradients from zero on apply(dv) = b for a vector of two blocks
// (n0 and n1 entries: the caller's x0 / x1, b0 / b1); rr (optional, device, iters + 1
// doubles) receives <r_k, r_k>.  The work vectors r, d, q ([n0 | n1] each) and the FP64
// scalars sit in the CG region of the workspace; nothing synchronises with the host.
// apply(d0, d1, q0, q1) must not touch that region.
template <class Apply>
static hipError_t cg_loop(const Plan& p, Apply apply, int64_t n0, int64_t n1, const float2* b0, const float2* b1,
                          int iters, float2* x0, float2* x1, double* rr, void* ws, hipStream_t st) {
  const int64_t n = n0 + n1;
  const size_t V = al(((size_t)p.N + (size_t)p.J * (size_t)p.K) * 8);
  char* base = wsp<char>(ws, p.off_cg);
  float2* r = reinterpret_cast<float2*>(base);
  float2* d = reinterpret_cast<float2*>(base + V);
  float2* q = reinterpret_cast<float2*>(base + 2 * V);
  double* sc = reinterpret_cast<double*>(base + 3 * V);
  double *rho = sc, *rho_new = sc + 1, *dq = sc + 2, *alpha = sc + 3, *beta = sc + 4;
  double* part = reinterpret_cast<double*>(base + 3 * V + al(CG_SCALARS * sizeof(double)));
  hipError_t e;
  if ((e = zero_split_launch(x0, x1, n0, n1, st)) != hipSuccess) return e;
  if ((e = copy_split_launch(r, r + n0, b0, b1, n0, n1, st)) != hipSuccess) return e;
  if ((e = copy_split_launch(d, d + n0, b0, b1, n0, n1, st)) != hipSuccess) return e;
  if ((e = TIMED("cg_dot", dot_launch(r, r, n, part, rho, st))) != hipSuccess) return e;
  if (rr && (e = copy_scalar_launch(rho, rr, st)) != hipSuccess) return e;
  for (int k = 0; k < iters; ++k) {
    if ((e = apply(d, d + n0, q, q + n0)) != hipSuccess) return e;
    if ((e = TIMED("cg_dot", dot_launch(d, q, n, part, dq, st))) != hipSuccess) return e;
    if ((e = cg_alpha_launch(rho, dq, alpha, st)) != hipSuccess) return e;
    if ((e = TIMED("cg_update", cg_xr_launch(x0, x1, n0, n1, r, d, q, alpha, st))) != hipSuccess) return e;
    if ((e = TIMED("cg_dot", dot_launch(r, r, n, part, rho_new, st))) != hipSuccess) return e;
    if ((e = cg_beta_launch(rho, rho_new, beta, rr ? rr + k + 1 : nullptr, st)) != hipSuccess) return e;
    if ((e = TIMED("cg_update", cg_d_launch(d, r, n, beta, st))) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t run_cg(const Plan& p, const float2* x, const float2* c, const float2* bx, const float2* bc, float lam_x,
                  float lam_c, int iters, float2* dx, float2* dc, double* rr, void* ws, hipStream_t st) {
  auto apply = [&](const float2* d0, const float2* d1, float2* q0, float2* q1) {
    return run_normal(p, x, c, d0, d1, lam_x, lam_c, q0, q1, ws, st);
  };
  return cg_loop(p, apply, p.N, (int64_t)p.J * p.K, bx, bc, iters, dx, dc, rr, ws, st);
}

// ---- SENSE with fixed maps and the constrained reconstruction (Sec. II-C)

hipError_t run_sense_encode(const Plan& p, const float2* S, const float2* x, float2* y, void* ws, hipStream_t st) {
  return encode_maps(p, S, x, y, ws, st);
}

hipError_t run_sense_adjoint(const Plan& p, const float2* S, const float2* y, float2* gx, void* ws, hipStream_t st) {
  return adjoint_maps(p, S, nullptr, y, 1.0f, nullptr, gx, false, ws, st);
}

// out = x + sum_j conj(S_j) (.) F_s^H F_s (S_j (.) x), the p-update operator of the ADMM
hipError_t run_sense_normal(const Plan& p, const float2* S, const float2* x, float2* out, void* ws, hipStream_t st) {
  float2* u = wsp<float2>(ws, p.off_U);
  hipError_t e = encode_maps(p, S, x, u, ws, st);
  if (e != hipSuccess) return e;
  if ((e = adjoint_maps(p, S, nullptr, u, 1.0f, nullptr, out, false, ws, st)) != hipSuccess) return e;
  return TIMED("sense_axpy", caxpy_launch(out, x, 1.0f, p.N, st));
}

namespace {
struct AdmmWs {
  float2 *z0a, *z0b, *u0, *tN, *tN2, *P, *P2;
  float2 *Fp, *zka, *zkb, *uk, *tM;
  double *part, *dist, *r2, *s2, *rho, *ufac;
};
AdmmWs admm_ws(const Plan& p, void* ws) {
  AdmmWs a;
  const size_t NB = al((size_t)p.N * 8), MB = al((size_t)p.J * (size_t)p.M * 8);
  char* b = wsp<char>(ws, p.off_admm);
  float2** nb[] = {&a.z0a, &a.z0b, &a.u0, &a.tN, &a.tN2};
  for (auto q : nb) { *q = reinterpret_cast<float2*>(b); b += NB; }
  a.P = reinterpret_cast<float2*>(b);
  b += p.ndim * NB;
  a.P2 = reinterpret_cast<float2*>(b);
  b += p.ndim * NB;
  float2** mb[] = {&a.Fp, &a.zka, &a.zkb, &a.uk, &a.tM};
  for (auto q : mb) { *q = reinterpret_cast<float2*>(b); b += MB; }
  a.part = reinterpret_cast<double*>(b);
  a.dist = a.part + (size_t)ball_part_doubles(p.J) - p.J;
  b += al((size_t)ball_part_doubles(p.J) * sizeof(double));
  double* sc = reinterpret_cast<double*>(b);
  a.r2 = sc; a.s2 = sc + 1; a.rho = sc + 2; a.ufac = sc + 3;
  return a;
}
}  // namespace

hipError_t run_tv_prox(const Plan& p, const float2* z, float lam, int iters, float2* x, void* ws, hipStream_t st) {
  const AdmmWs a = admm_ws(p, ws);
  return TIMED("tv_prox", tv_prox_launch(p.ndim, p.n, z, nullptr, lam, iters, a.P, a.P2, x, st));
}

hipError_t run_ball_project(const Plan& p, const float2* w, const float2* y, const float* eps, float2* z, void* ws,
                            hipStream_t st) {
  const AdmmWs a = admm_ws(p, ws);
  return TIMED("ball", ball_project_launch(w, y, eps, p.M, p.J, a.part, a.dist, z, st));
}

// The scaled ADMM iteration of Sec. II-C (z_0 prox, z_k ball projections, p-update by CG
// on I + S^H F^H F S from the current p, dual update, residual-balanced rho).  p starts at
// the SENSE combination S^H F^H y; z and u at zero.
hipError_t run_admm(const Plan& p, const float2* S, const float2* y, const float* eps, float rho0, int iters,
                    int cg_iters, int tv_iters, float2* pimg, double* hist, void* ws, hipStream_t st) {
  AdmmWs a = admm_ws(p, ws);
  const int64_t N = p.N, JM = (int64_t)p.J * p.M;
  double* part = wsp<double>(ws, p.off_cg + 3 * al(((size_t)p.N + (size_t)p.J * (size_t)p.K) * 8) +
                                     al(CG_SCALARS * sizeof(double)));
  hipError_t e;
  if ((e = run_sense_adjoint(p, S, y, pimg, ws, st)) != hipSuccess) return e;
  if ((e = zero_split_launch(a.z0a, a.u0, N, N, st)) != hipSuccess) return e;
  if ((e = zero_split_launch(a.zka, a.uk, JM, JM, st)) != hipSuccess) return e;
  if ((e = set_scalar_launch(a.rho, (double)rho0, st)) != hipSuccess) return e;
  if ((e = run_sense_encode(p, S, pimg, a.Fp, ws, st)) != hipSuccess) return e;
  float2 *z0 = a.z0a, *z0p = a.z0b, *zk = a.zka, *zkp = a.zkb;
  auto sense_op = [&](const float2* d0, const float2*, float2* q0, float2*) {
    return run_sense_normal(p, S, d0, q0, ws, st);
  };
  for (int it = 0; it < iters; ++it) {
    std::swap(z0, z0p);  // z0p, zkp: the previous iterates
    std::swap(zk, zkp);
    // z0 = prox_{TV / rho}(p + u0)
    if ((e = lincomb_launch(a.tN, pimg, 1.f, a.u0, 1.f, N, st)) != hipSuccess) return e;
    if ((e = TIMED("tv_prox", tv_prox_launch(p.ndim, p.n, a.tN, a.rho, 0.f, tv_iters, a.P, a.P2, z0, st))) !=
        hipSuccess)
      return e;
    // z_k = ball projection of F S p + u_k
    if ((e = lincomb_launch(a.tM, a.Fp, 1.f, a.uk, 1.f, JM, st)) != hipSuccess) return e;
    if ((e = TIMED("ball", ball_project_launch(a.tM, y, eps, p.M, p.J, a.part, a.dist, zk, st))) != hipSuccess)
      return e;
    // rhs = z0 - u0 + S^H F^H (z_k - u_k);  res = rhs - (I + S^H F^H F S) p
    if ((e = lincomb_launch(a.tM, zk, 1.f, a.uk, -1.f, JM, st)) != hipSuccess) return e;
    if ((e = run_sense_adjoint(p, S, a.tM, a.tN, ws, st)) != hipSuccess) return e;
    if ((e = caxpy_launch(a.tN, z0, 1.f, N, st)) != hipSuccess) return e;
    if ((e = caxpy_launch(a.tN, a.u0, -1.f, N, st)) != hipSuccess) return e;
    if ((e = run_sense_normal(p, S, pimg, a.tN2, ws, st)) != hipSuccess) return e;
    if ((e = caxpy_launch(a.tN, a.tN2, -1.f, N, st)) != hipSuccess) return e;
    // p += CG(res)
    if ((e = cg_loop(p, sense_op, N, 0, a.tN, nullptr, cg_iters, a.tN2, nullptr, nullptr, ws, st)) != hipSuccess)
      return e;
    if ((e = caxpy_launch(pimg, a.tN2, 1.f, N, st)) != hipSuccess) return e;
    if ((e = run_sense_encode(p, S, pimg, a.Fp, ws, st)) != hipSuccess) return e;
    // u += A p - z
    if ((e = caxpy_launch(a.u0, pimg, 1.f, N, st)) != hipSuccess) return e;
    if ((e = caxpy_launch(a.u0, z0, -1.f, N, st)) != hipSuccess) return e;
    if ((e = caxpy_launch(a.uk, a.Fp, 1.f, JM, st)) != hipSuccess) return e;
    if ((e = caxpy_launch(a.uk, zk, -1.f, JM, st)) != hipSuccess) return e;
    // primal residual ||A p - z||^2 and dual residual ||A^H (z - z_prev)||^2 (before rho)
    if ((e = lincomb_launch(a.tN, pimg, 1.f, z0, -1.f, N, st)) != hipSuccess) return e;
    if ((e = lincomb_launch(a.tM, a.Fp, 1.f, zk, -1.f, JM, st)) != hipSuccess) return e;
    if ((e = dot2_launch(a.tN, a.tM, N, JM, part, a.r2, st)) != hipSuccess) return e;
    if ((e = lincomb_launch(a.tM, zk, 1.f, zkp, -1.f, JM, st)) != hipSuccess) return e;
    if ((e = run_sense_adjoint(p, S, a.tM, a.tN, ws, st)) != hipSuccess) return e;
    if ((e = caxpy_launch(a.tN, z0, 1.f, N, st)) != hipSuccess) return e;
    if ((e = caxpy_launch(a.tN, z0p, -1.f, N, st)) != hipSuccess) return e;
    if ((e = dot_launch(a.tN, a.tN, N, part, a.s2, st)) != hipSuccess) return e;
    if ((e = admm_rho_launch(a.r2, a.s2, a.rho, a.ufac, hist ? hist + 3 * it : nullptr, st)) != hipSuccess) return e;
    if ((e = scale_dev_launch(a.u0, N, a.ufac, st)) != hipSuccess) return e;
    if ((e = scale_dev_launch(a.uk, JM, a.ufac, st)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---- extra bilinear terms (multi-map, Sec. IV-A): y = sum_i E(x_i, c_i)

// y = sum over the n map sets of E(x_i, c_i); x: n x [N], c: n x [J][K]
hipError_t run_multi_encode(const Plan& p, int n, const float2* x, const float2* c, float2* y, void* ws,
                            hipStream_t st) {
  const int64_t JK = (int64_t)p.J * p.K, JM = (int64_t)p.J * p.M;
  hipError_t e = run_encode(p, x, c, y, ws, st);
  float2* E = wsp<float2>(ws, p.off_E);
  for (int i = 1; i < n && e == hipSuccess; ++i) {
    if ((e = run_encode(p, x + (int64_t)i * p.N, c + (int64_t)i * JK, E, ws, st)) != hipSuccess) return e;
    e = TIMED("multi_sum", caxpy_launch(y, E, 1.0f, JM, st));
  }
  return e;
}

// f = sum w |sum_i E(x_i, c_i) - y|^2 and (gx_i, gc_i) = 2 J_i^H (w (.) r) for every map set
hipError_t run_multi_grad(const Plan& p, int n, const float2* x, const float2* c, const float2* y, float2* gx,
                          float2* gc, double* loss, void* ws, hipStream_t st) {
  const int64_t JK = (int64_t)p.J * p.K;
  float2* r = wsp<float2>(ws, p.off_U);
  double* part = wsp<double>(ws, p.off_part);
  hipError_t e = run_multi_encode(p, n, x, c, r, ws, st);
  if (e != hipSuccess) return e;
  if ((e = TIMED("residual", residual_launch(r, y, p.d_w, p.M, p.J, r, part, st))) != hipSuccess) return e;
  if (loss && (e = TIMED("reduce_loss", reduce_loss_launch(part, residual_blocks((int64_t)p.J * p.M), loss, st))) !=
                  hipSuccess)
    return e;
  if (!gx && !gc) return hipSuccess;
  for (int i = 0; i < n; ++i)
    if ((e = run_adjoint(p, x + (int64_t)i * p.N, c + (int64_t)i * JK, r, 2.0f, nullptr,
                         gx ? gx + (int64_t)i * p.N : nullptr, gc ? gc + (int64_t)i * JK : nullptr, ws, st, false,
                         false)) != hipSuccess)
      return e;
  return hipSuccess;
}

}  // namespace mx
