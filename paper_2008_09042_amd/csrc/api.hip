// Host side of the C ABI declared in include/maxwell.h: plan construction,
// argument validation, workspace layout, and the enqueue sequences of the
// encoding operator (paper Sec. II-B, Eq. (5)), its Jacobian adjoint
// (Sec. II-B, J_G^H), and the data-fidelity loss and gradient.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/maxwell.h"
#include "common.h"
#include "plan.h"
#include "compress.h"
#include "solver.h"
#include "tune.h"

using namespace mx;

namespace {

thread_local std::string g_last_error;

maxwell_status fail(maxwell_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

maxwell_status hip_fail(hipError_t e, const char* where) {
  g_last_error = std::string("HIP error in ") + where + ": " + hipGetErrorString(e);
  return MAXWELL_ERR_HIP;
}

// ---------------------------------------------------------------- library-held workspace
// The workspace of maxwell_grad_static: a file-scope device array of MAXWELL_STATIC_WS_BYTES,
// one copy per device (each device that loads the library holds it until the process ends).
// Host code never uses the array's name as an address (its host-side stand-in): the device
// address comes from hipGetSymbolAddress, fetched once per device with that device current
// (at plan creation) and kept per device.
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[MAXWELL_STATIC_WS_BYTES];

namespace {

// Device address of `scratch` on the current device `dev` (fetched and cached on first use).
hipError_t scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

#define HIP_TRY(expr, where)                      \
  do {                                            \
    hipError_t _e = (expr);                       \
    if (_e != hipSuccess) return hip_fail(_e, where); \
  } while (0)

bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

bool overlap(const void* a, size_t abytes, const void* b, size_t bbytes) {
  if (!a || !b || abytes == 0 || bbytes == 0) return false;
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
  return a0 < b0 + bbytes && b0 < a0 + abytes;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace

// ------------------------------------------------------------------ plan
namespace mx {

void set_last_error(const std::string& msg) { g_last_error = msg; }

static maxwell_status validate_desc(const maxwell_plan_desc* d, const maxwell_basis_desc* b) {
  if (!d || !b) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "null descriptor");
  if (d->ndim != 2 && d->ndim != 3) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "ndim must be 2 or 3");
  int64_t N = 1;
  for (int i = 0; i < d->ndim; ++i) {
    if (d->n[i] < 2 || d->n[i] > 4096)
      return fail(MAXWELL_ERR_INVALID_ARGUMENT, "image size must be in [2, 4096] on every axis");
    if (d->n[i] & 1) return fail(MAXWELL_ERR_UNSUPPORTED, "odd image sizes are not supported");
    int rad[12];
    if (!fft_factorise(d->n[i], rad))
      return fail(MAXWELL_ERR_UNSUPPORTED, "image sizes must factor into 2, 3 and 5");
    N *= d->n[i];
  }
  if (N > (int64_t(1) << 30)) return fail(MAXWELL_ERR_UNSUPPORTED, "image larger than 2^30 voxels");
  if (d->J < 1) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "J must be >= 1");
  if (d->precision != MAXWELL_FP32 && d->precision != MAXWELL_BF16_SPLIT)
    return fail(MAXWELL_ERR_INVALID_ARGUMENT, "unknown precision");
  if (b->K < 1) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "K must be >= 1");
  if (b->kind == MAXWELL_BASIS_DENSE) {
    if (!b->dense || !aligned8(b->dense)) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "dense basis pointer null or misaligned");
  } else if (b->kind == MAXWELL_BASIS_TUCKER) {
    if (d->ndim != 3) return fail(MAXWELL_ERR_UNSUPPORTED, "Tucker bases need a 3D image");
    for (int m = 0; m < 3; ++m) {
      if (b->r[m] < 1 || b->r[m] > d->n[m])
        return fail(MAXWELL_ERR_INVALID_ARGUMENT, "Tucker rank must be in [1, n_m]");
      if (!b->U[m] || !aligned8(b->U[m])) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "Tucker factor pointer null or misaligned");
    }
    if (!b->core || !aligned8(b->core)) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "Tucker core pointer null or misaligned");
  } else {
    return fail(MAXWELL_ERR_INVALID_ARGUMENT, "unknown basis kind");
  }
  if (d->M < 0) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "M must be >= 0");
  if (d->sampling == MAXWELL_CARTESIAN) {
    if (d->M > N) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "more mask samples than grid points");
    if (d->M > 0 && !d->mask_idx) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "mask_idx is null");
    for (int64_t m = 0; m < d->M; ++m) {
      const int64_t v = d->mask_idx[m];
      if (v < 0 || v >= N) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "mask index out of range");
      if (m > 0 && v <= d->mask_idx[m - 1])
        return fail(MAXWELL_ERR_INVALID_ARGUMENT, "mask indices must be strictly ascending (no duplicates)");
    }
  } else if (d->sampling == MAXWELL_NONCARTESIAN) {
    if (d->ndim != 2) return fail(MAXWELL_ERR_UNSUPPORTED, "non-Cartesian sampling is 2D only");
    if (d->M > 0 && !d->traj) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "traj is null");
    if (d->kb_width < 2 || d->kb_width > 8) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "kb_width must be in [2, 8]");
    if (!(d->oversamp >= 1.0f) || !std::isfinite(d->oversamp))
      return fail(MAXWELL_ERR_INVALID_ARGUMENT, "oversamp must be finite and >= 1");
    if (!std::isfinite(d->kb_beta)) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "kb_beta must be finite");
    for (int i = 0; i < 2; ++i) {
      const double g = (double)d->oversamp * (double)d->n[i];
      const int64_t gi = (int64_t)std::llround(g);
      if (std::fabs(g - (double)gi) > 1e-6 || (gi & 1))
        return fail(MAXWELL_ERR_INVALID_ARGUMENT, "oversamp * n must be an even integer");
      int rad[12];
      if (!fft_factorise(gi, rad)) return fail(MAXWELL_ERR_UNSUPPORTED, "oversampled grid must factor into 2, 3, 5 and be <= 4096");
      if (gi < d->kb_width) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "oversampled grid must be at least kb_width");
    }
    for (int64_t m = 0; m < d->M * d->ndim; ++m) {
      const float v = d->traj[m];
      const int ax = (int)(m % d->ndim);
      if (!std::isfinite(v) || v < -0.5f * (float)d->n[ax] || v >= 0.5f * (float)d->n[ax])
        return fail(MAXWELL_ERR_INVALID_ARGUMENT, "trajectory point outside [-n/2, n/2)");
    }
  } else {
    return fail(MAXWELL_ERR_INVALID_ARGUMENT, "unknown sampling kind");
  }
  if (d->weights) {
    for (int64_t m = 0; m < d->M; ++m)
      if (!std::isfinite(d->weights[m]) || d->weights[m] < 0.f)
        return fail(MAXWELL_ERR_INVALID_ARGUMENT, "weights must be finite and >= 0");
  }
  return MAXWELL_OK;
}

}  // namespace mx

extern "C" {

const char* maxwell_last_error(void) { return g_last_error.c_str(); }

const char* maxwell_version(void) { return "maxwell-gfx950 0.1"; }

maxwell_status maxwell_tune_counts(int64_t* measured, int64_t* reused) {
  long long m = 0, r = 0;
  tune_counts(&m, &r);
  if (measured) *measured = m;
  if (reused) *reused = r;
  return MAXWELL_OK;
}

maxwell_status maxwell_bf16_split(const float* x, int64_t n, int32_t variant, uint16_t* hi, uint16_t* lo,
                                  void* stream) {
  if (n < 0 || n > ((int64_t)1 << 40)) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "n out of range");
  if (variant < 0 || variant > 2) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "variant must be 0, 1 or 2");
  if (variant == 1 && (n & 1)) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "variant 1 splits complex pairs: n must be even");
  if (n == 0) return MAXWELL_OK;
  if (!x || !hi || !lo) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "null pointer");
  if ((reinterpret_cast<uintptr_t>(x) & (variant == 1 ? 7u : 3u)) || (reinterpret_cast<uintptr_t>(hi) & 1u) ||
      (reinterpret_cast<uintptr_t>(lo) & 1u))
    return fail(MAXWELL_ERR_INVALID_ARGUMENT, "misaligned pointer");
  const uintptr_t xs = reinterpret_cast<uintptr_t>(x), xe = xs + (uintptr_t)n * 4;
  const uintptr_t hs = reinterpret_cast<uintptr_t>(hi), he = hs + (uintptr_t)n * 2;
  const uintptr_t ls = reinterpret_cast<uintptr_t>(lo), le = ls + (uintptr_t)n * 2;
  if ((xs < he && hs < xe) || (xs < le && ls < xe) || (hs < le && ls < he))
    return fail(MAXWELL_ERR_INVALID_ARGUMENT, "x, hi and lo must not overlap");
  HIP_TRY(bf16_split_diag_launch(x, n, variant, hi, lo, (hipStream_t)stream), "bf16_split");
  return MAXWELL_OK;
}

maxwell_status maxwell_plan_create(const maxwell_plan_desc* desc, const maxwell_basis_desc* basis,
                                   maxwell_plan_t* plan_out) {
  if (!plan_out) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan_out is null");
  *plan_out = nullptr;
  maxwell_status s = validate_desc(desc, basis);
  if (s != MAXWELL_OK) return s;
  Plan* p = new (std::nothrow) Plan();
  if (!p) return fail(MAXWELL_ERR_OUT_OF_MEMORY, "host allocation failed");
  s = plan_build(*p, *desc, *basis);
  if (s == MAXWELL_OK) {
    // the plan's device and its copy of the library-held workspace (maxwell_grad_static)
    void* unused = nullptr;
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = scratch_address(p->device, &unused);
    if (e != hipSuccess) s = hip_fail(e, "plan_create (static workspace address)");
  }
  if (s != MAXWELL_OK) {
    plan_release(*p);
    delete p;
    return s;
  }
  *plan_out = reinterpret_cast<maxwell_plan_t>(p);
  return MAXWELL_OK;
}

void maxwell_plan_destroy(maxwell_plan_t plan) {
  if (!plan) return;
  Plan* p = reinterpret_cast<Plan*>(plan);
  plan_release(*p);
  delete p;
}

maxwell_status maxwell_plan_set_timing(maxwell_plan_t plan, int enable) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  Timing& t = reinterpret_cast<Plan*>(plan)->timing;
  if (enable) {
    t.recs.clear();
    t.names.clear();
  }
  t.on = enable != 0;
  return MAXWELL_OK;
}

maxwell_status maxwell_plan_timing(maxwell_plan_t plan, int i, int* count, const char** name, int64_t* launches,
                                   double* total_ms) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  Timing& t = reinterpret_cast<Plan*>(plan)->timing;
  if (count) *count = (int)t.names.size();
  if (!name && !launches && !total_ms) return MAXWELL_OK;
  if (i < 0 || i >= (int)t.names.size()) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "timing index out of range");
  if (!t.recs.empty()) {
    hipError_t e = hipEventSynchronize(t.ev_stop[t.recs.back().ev]);
    if (e != hipSuccess) return hip_fail(e, "plan_timing");
  }
  int64_t n = 0;
  double ms = 0.0;
  for (const auto& r : t.recs) {
    if (r.name != i) continue;
    float f = 0.f;
    hipError_t e = hipEventElapsedTime(&f, t.ev_start[r.ev], t.ev_stop[r.ev]);
    if (e != hipSuccess) return hip_fail(e, "plan_timing");
    ms += f;
    ++n;
  }
  if (name) *name = t.names[i];
  if (launches) *launches = n;
  if (total_ms) *total_ms = ms;
  return MAXWELL_OK;
}

const char* maxwell_plan_path(maxwell_plan_t plan) {
  if (!plan) return nullptr;
  return reinterpret_cast<Plan*>(plan)->fused ? "fused-tucker-lines" : "general";
}

maxwell_status maxwell_plan_workspace_size(maxwell_plan_t plan, size_t* bytes) {
  if (!plan || !bytes) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "null plan or bytes pointer");
  *bytes = reinterpret_cast<Plan*>(plan)->ws_bytes;
  return MAXWELL_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ compute calls
namespace {

struct Check {
  const Plan* p;
  maxwell_status st = MAXWELL_OK;
  std::vector<std::pair<const void*, size_t>> ins, outs;
  explicit Check(const Plan* pp) : p(pp) {}
  bool in(const void* ptr, size_t bytes, const char* name, bool required = true) {
    if (st != MAXWELL_OK) return false;
    if (!ptr) {
      if (required && bytes) { st = fail(MAXWELL_ERR_INVALID_ARGUMENT, std::string(name) + " is null"); return false; }
      return true;
    }
    if (!aligned8(ptr)) { st = fail(MAXWELL_ERR_INVALID_ARGUMENT, std::string(name) + " is not 8-byte aligned"); return false; }
    ins.push_back({ptr, bytes});
    return true;
  }
  bool out(const void* ptr, size_t bytes, const char* name, bool required = true) {
    if (st != MAXWELL_OK) return false;
    if (!ptr) {
      if (required && bytes) { st = fail(MAXWELL_ERR_INVALID_ARGUMENT, std::string(name) + " is null"); return false; }
      return true;
    }
    if (!aligned8(ptr)) { st = fail(MAXWELL_ERR_INVALID_ARGUMENT, std::string(name) + " is not 8-byte aligned"); return false; }
    outs.push_back({ptr, bytes});
    return true;
  }
  bool ws(const void* w, size_t bytes) {
    if (st != MAXWELL_OK) return false;
    if (bytes < p->ws_bytes) {
      st = fail(MAXWELL_ERR_WORKSPACE_TOO_SMALL, "workspace smaller than maxwell_plan_workspace_size");
      return false;
    }
    if (p->ws_bytes && !w) { st = fail(MAXWELL_ERR_INVALID_ARGUMENT, "workspace is null"); return false; }
    if (w && (reinterpret_cast<uintptr_t>(w) & 255u)) {
      st = fail(MAXWELL_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
      return false;
    }
    outs.push_back({w, p->ws_bytes});
    return true;
  }
  maxwell_status finish() {
    if (st != MAXWELL_OK) return st;
    for (size_t i = 0; i < outs.size(); ++i) {
      for (auto& in : ins)
        if (overlap(outs[i].first, outs[i].second, in.first, in.second))
          return fail(MAXWELL_ERR_INVALID_ARGUMENT, "an output overlaps an input");
      for (size_t k = i + 1; k < outs.size(); ++k)
        if (overlap(outs[i].first, outs[i].second, outs[k].first, outs[k].second))
          return fail(MAXWELL_ERR_INVALID_ARGUMENT, "two outputs overlap");
    }
    return MAXWELL_OK;
  }
};

}  // namespace

extern "C" {

maxwell_status maxwell_basis_apply(maxwell_plan_t plan, const maxwell_complex64* c, maxwell_complex64* S,
                                   void* ws, size_t ws_bytes, void* stream) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  Check ck(p);
  ck.in(c, p->bytes_c(), "c");
  ck.out(S, p->bytes_S(), "S");
  ck.ws(ws, ws_bytes);
  maxwell_status s = ck.finish();
  if (s != MAXWELL_OK) return s;
  HIP_TRY(run_basis_apply(*p, reinterpret_cast<const float2*>(c), reinterpret_cast<float2*>(S), ws,
                          (hipStream_t)stream),
          "basis_apply");
  return MAXWELL_OK;
}

maxwell_status maxwell_basis_apply_adjoint(maxwell_plan_t plan, const maxwell_complex64* S,
                                           maxwell_complex64* c, void* ws, size_t ws_bytes, void* stream) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  Check ck(p);
  ck.in(S, p->bytes_S(), "S");
  ck.out(c, p->bytes_c(), "c");
  ck.ws(ws, ws_bytes);
  maxwell_status s = ck.finish();
  if (s != MAXWELL_OK) return s;
  HIP_TRY(run_basis_adjoint(*p, reinterpret_cast<const float2*>(S), reinterpret_cast<float2*>(c), 1.0f,
                            nullptr, ws, (hipStream_t)stream),
          "basis_apply_adjoint");
  return MAXWELL_OK;
}

maxwell_status maxwell_encode(maxwell_plan_t plan, const maxwell_complex64* x, const maxwell_complex64* c,
                              maxwell_complex64* y, void* ws, size_t ws_bytes, void* stream) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  Check ck(p);
  ck.in(x, p->bytes_x(), "x");
  ck.in(c, p->bytes_c(), "c");
  ck.out(y, p->bytes_y(), "y");
  ck.ws(ws, ws_bytes);
  maxwell_status s = ck.finish();
  if (s != MAXWELL_OK) return s;
  HIP_TRY(run_encode(*p, reinterpret_cast<const float2*>(x), reinterpret_cast<const float2*>(c),
                     reinterpret_cast<float2*>(y), ws, (hipStream_t)stream),
          "encode");
  return MAXWELL_OK;
}

maxwell_status maxwell_adjoint(maxwell_plan_t plan, const maxwell_complex64* x, const maxwell_complex64* c,
                               const maxwell_complex64* y, float alpha, const float* scale_dev,
                               maxwell_complex64* gx, maxwell_complex64* gc, void* ws, size_t ws_bytes,
                               void* stream) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  if (!std::isfinite(alpha)) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "alpha must be finite");
  Check ck(p);
  ck.in(x, p->bytes_x(), "x");
  ck.in(c, p->bytes_c(), "c");
  ck.in(y, p->bytes_y(), "y");
  if (scale_dev && (reinterpret_cast<uintptr_t>(scale_dev) & 3u))
    return fail(MAXWELL_ERR_INVALID_ARGUMENT, "scale_dev must be 4-byte aligned");
  if (scale_dev) ck.ins.push_back({scale_dev, sizeof(float)});
  ck.out(gx, p->bytes_x(), "gx", false);
  ck.out(gc, p->bytes_c(), "gc", false);
  ck.ws(ws, ws_bytes);
  maxwell_status s = ck.finish();
  if (s != MAXWELL_OK) return s;
  if (!gx && !gc) return MAXWELL_OK;
  HIP_TRY(run_adjoint(*p, reinterpret_cast<const float2*>(x), reinterpret_cast<const float2*>(c),
                      reinterpret_cast<const float2*>(y), alpha, scale_dev, reinterpret_cast<float2*>(gx),
                      reinterpret_cast<float2*>(gc), ws, (hipStream_t)stream, false),
          "adjoint");
  return MAXWELL_OK;
}

maxwell_status maxwell_forward_loss(maxwell_plan_t plan, const maxwell_complex64* x, const maxwell_complex64* c,
                                    const maxwell_complex64* y, maxwell_complex64* r, double* loss_dev, void* ws,
                                    size_t ws_bytes, void* stream) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  Check ck(p);
  ck.in(x, p->bytes_x(), "x");
  ck.in(c, p->bytes_c(), "c");
  ck.in(y, p->bytes_y(), "y");
  ck.out(r, p->bytes_y(), "r", false);
  ck.out(loss_dev, sizeof(double), "loss_dev", false);
  ck.ws(ws, ws_bytes);
  maxwell_status s = ck.finish();
  if (s != MAXWELL_OK) return s;
  if (!r && !loss_dev) return MAXWELL_OK;
  HIP_TRY(run_forward_loss(*p, reinterpret_cast<const float2*>(x), reinterpret_cast<const float2*>(c),
                           reinterpret_cast<const float2*>(y), reinterpret_cast<float2*>(r), loss_dev, ws,
                           (hipStream_t)stream),
          "forward_loss");
  return MAXWELL_OK;
}

maxwell_status maxwell_forward_transfer(maxwell_plan_t plan, const maxwell_complex64* x, const maxwell_complex64* c,
                                        const maxwell_complex64* y, maxwell_complex64* t, double* loss_dev, void* ws,
                                        size_t ws_bytes, void* stream) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  Check ck(p);
  ck.in(x, p->bytes_x(), "x");
  ck.in(c, p->bytes_c(), "c");
  ck.in(y, p->bytes_y(), "y");
  ck.out(t, p->bytes_y(), "t", true);
  ck.out(loss_dev, sizeof(double), "loss_dev", false);
  ck.ws(ws, ws_bytes);
  maxwell_status s = ck.finish();
  if (s != MAXWELL_OK) return s;
  HIP_TRY(run_forward_loss(*p, reinterpret_cast<const float2*>(x), reinterpret_cast<const float2*>(c),
                           reinterpret_cast<const float2*>(y), reinterpret_cast<float2*>(t), loss_dev, ws,
                           (hipStream_t)stream, true),
          "forward_transfer");
  return MAXWELL_OK;
}

maxwell_status maxwell_adjoint_transfer(maxwell_plan_t plan, const maxwell_complex64* x, const maxwell_complex64* c,
                                        const maxwell_complex64* t, float alpha, const float* scale_dev,
                                        maxwell_complex64* gx, maxwell_complex64* gc, void* ws, size_t ws_bytes,
                                        void* stream) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  if (!std::isfinite(alpha)) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "alpha must be finite");
  Check ck(p);
  ck.in(x, p->bytes_x(), "x");
  ck.in(c, p->bytes_c(), "c");
  ck.in(t, p->bytes_y(), "t");
  if (scale_dev && (reinterpret_cast<uintptr_t>(scale_dev) & 3u))
    return fail(MAXWELL_ERR_INVALID_ARGUMENT, "scale_dev must be 4-byte aligned");
  if (scale_dev) ck.ins.push_back({scale_dev, sizeof(float)});
  ck.out(gx, p->bytes_x(), "gx", false);
  ck.out(gc, p->bytes_c(), "gc", false);
  ck.ws(ws, ws_bytes);
  maxwell_status s = ck.finish();
  if (s != MAXWELL_OK) return s;
  if (!gx && !gc) return MAXWELL_OK;
  HIP_TRY(run_adjoint(*p, reinterpret_cast<const float2*>(x), reinterpret_cast<const float2*>(c),
                      reinterpret_cast<const float2*>(t), alpha, scale_dev, reinterpret_cast<float2*>(gx),
                      reinterpret_cast<float2*>(gc), ws, (hipStream_t)stream, false, true),
          "adjoint_transfer");
  return MAXWELL_OK;
}

maxwell_status maxwell_grad(maxwell_plan_t plan, const maxwell_complex64* x, const maxwell_complex64* c,
                            const maxwell_complex64* y, maxwell_complex64* gx, maxwell_complex64* gc,
                            double* loss_dev, void* ws, size_t ws_bytes, void* stream) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  Check ck(p);
  ck.in(x, p->bytes_x(), "x");
  ck.in(c, p->bytes_c(), "c");
  ck.in(y, p->bytes_y(), "y");
  ck.out(gx, p->bytes_x(), "gx", false);
  ck.out(gc, p->bytes_c(), "gc", false);
  ck.out(loss_dev, sizeof(double), "loss_dev", false);
  ck.ws(ws, ws_bytes);
  maxwell_status s = ck.finish();
  if (s != MAXWELL_OK) return s;
  HIP_TRY(run_grad(*p, reinterpret_cast<const float2*>(x), reinterpret_cast<const float2*>(c),
                   reinterpret_cast<const float2*>(y), reinterpret_cast<float2*>(gx), reinterpret_cast<float2*>(gc),
                   loss_dev, ws, (hipStream_t)stream),
          "grad");
  return MAXWELL_OK;
}

maxwell_status maxwell_grad_static(maxwell_plan_t plan, const maxwell_complex64* x, const maxwell_complex64* c,
                                   const maxwell_complex64* y, maxwell_complex64* gx, maxwell_complex64* gc,
                                   double* loss_dev, void* stream) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  if (p->ws_bytes > MAXWELL_STATIC_WS_BYTES)
    return fail(MAXWELL_ERR_WORKSPACE_TOO_SMALL,
                "plan workspace (" + std::to_string(p->ws_bytes) + " bytes) exceeds the library-held workspace (" +
                    std::to_string((size_t)MAXWELL_STATIC_WS_BYTES) + " bytes); use maxwell_grad with a workspace");
  if (p->timing.on)
    return fail(MAXWELL_ERR_UNSUPPORTED, "maxwell_grad_static: per-kernel timing must be off (it creates events)");
  void* ws = nullptr;
  if (p->device < 0 || p->device >= MAX_DEVICES || !(ws = g_scratch_ptr[p->device]))
    return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan has no library-held workspace on its device");
  Check ck(p);
  ck.in(x, p->bytes_x(), "x");
  ck.in(c, p->bytes_c(), "c");
  ck.in(y, p->bytes_y(), "y");
  ck.out(gx, p->bytes_x(), "gx", false);
  ck.out(gc, p->bytes_c(), "gc", false);
  ck.out(loss_dev, sizeof(double), "loss_dev", false);
  ck.ws(ws, MAXWELL_STATIC_WS_BYTES);
  maxwell_status s = ck.finish();
  if (s != MAXWELL_OK) return s;
  HIP_TRY(run_grad(*p, reinterpret_cast<const float2*>(x), reinterpret_cast<const float2*>(c),
                   reinterpret_cast<const float2*>(y), reinterpret_cast<float2*>(gx), reinterpret_cast<float2*>(gc),
                   loss_dev, ws, (hipStream_t)stream),
          "grad_static");
  return MAXWELL_OK;
}

maxwell_status maxwell_jvp(maxwell_plan_t plan, const maxwell_complex64* x, const maxwell_complex64* c,
                           const maxwell_complex64* dx, const maxwell_complex64* dc, maxwell_complex64* y, void* ws,
                           size_t ws_bytes, void* stream) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  Check ck(p);
  ck.in(x, p->bytes_x(), "x");
  ck.in(c, p->bytes_c(), "c");
  ck.in(dx, p->bytes_x(), "dx");
  ck.in(dc, p->bytes_c(), "dc");
  ck.out(y, p->bytes_y(), "y");
  ck.ws(ws, ws_bytes);
  maxwell_status s = ck.finish();
  if (s != MAXWELL_OK) return s;
  HIP_TRY(run_jvp(*p, reinterpret_cast<const float2*>(x), reinterpret_cast<const float2*>(c),
                  reinterpret_cast<const float2*>(dx), reinterpret_cast<const float2*>(dc), reinterpret_cast<float2*>(y),
                  ws, (hipStream_t)stream),
          "jvp");
  return MAXWELL_OK;
}

maxwell_status maxwell_normal(maxwell_plan_t plan, const maxwell_complex64* x, const maxwell_complex64* c,
                              const maxwell_complex64* dx, const maxwell_complex64* dc, float lambda_x, float lambda_c,
                              maxwell_complex64* ox, maxwell_complex64* oc, void* ws, size_t ws_bytes, void* stream) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  if (!std::isfinite(lambda_x) || !std::isfinite(lambda_c))
    return fail(MAXWELL_ERR_INVALID_ARGUMENT, "lambda_x and lambda_c must be finite");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  Check ck(p);
  ck.in(x, p->bytes_x(), "x");
  ck.in(c, p->bytes_c(), "c");
  ck.in(dx, p->bytes_x(), "dx");
  ck.in(dc, p->bytes_c(), "dc");
  ck.out(ox, p->bytes_x(), "ox");
  ck.out(oc, p->bytes_c(), "oc");
  ck.ws(ws, ws_bytes);
  maxwell_status s = ck.finish();
  if (s != MAXWELL_OK) return s;
  HIP_TRY(run_normal(*p, reinterpret_cast<const float2*>(x), reinterpret_cast<const float2*>(c),
                     reinterpret_cast<const float2*>(dx), reinterpret_cast<const float2*>(dc), lambda_x, lambda_c,
                     reinterpret_cast<float2*>(ox), reinterpret_cast<float2*>(oc), ws, (hipStream_t)stream),
          "normal");
  return MAXWELL_OK;
}

maxwell_status maxwell_cg(maxwell_plan_t plan, const maxwell_complex64* x, const maxwell_complex64* c,
                          const maxwell_complex64* bx, const maxwell_complex64* bc, float lambda_x, float lambda_c,
                          int32_t iters, maxwell_complex64* dx, maxwell_complex64* dc, double* rr_dev, void* ws,
                          size_t ws_bytes, void* stream) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  if (!std::isfinite(lambda_x) || !std::isfinite(lambda_c))
    return fail(MAXWELL_ERR_INVALID_ARGUMENT, "lambda_x and lambda_c must be finite");
  if (iters < 0 || iters > 100000) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "iters must be in [0, 100000]");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  Check ck(p);
  ck.in(x, p->bytes_x(), "x");
  ck.in(c, p->bytes_c(), "c");
  ck.in(bx, p->bytes_x(), "bx");
  ck.in(bc, p->bytes_c(), "bc");
  ck.out(dx, p->bytes_x(), "dx");
  ck.out(dc, p->bytes_c(), "dc");
  ck.out(rr_dev, (size_t)(iters + 1) * sizeof(double), "rr_dev", false);
  ck.ws(ws, ws_bytes);
  maxwell_status s = ck.finish();
  if (s != MAXWELL_OK) return s;
  HIP_TRY(run_cg(*p, reinterpret_cast<const float2*>(x), reinterpret_cast<const float2*>(c),
                 reinterpret_cast<const float2*>(bx), reinterpret_cast<const float2*>(bc), lambda_x, lambda_c, iters,
                 reinterpret_cast<float2*>(dx), reinterpret_cast<float2*>(dc), rr_dev, ws, (hipStream_t)stream),
          "cg");
  return MAXWELL_OK;
}

// ---- accuracy-controlled Tucker compression of a dense basis

maxwell_status maxwell_tucker_compress(const int64_t* dims, int64_t K, const maxwell_complex64* B, float eps,
                                       maxwell_complex64* U0, maxwell_complex64* U1, maxwell_complex64* U2,
                                       maxwell_complex64* core, int64_t* ranks, double* dropped, void* stream) {
  if (!dims || !B || !U0 || !U1 || !U2 || !core || !ranks)
    return fail(MAXWELL_ERR_INVALID_ARGUMENT, "null argument (dims, B, U0..U2, core and ranks are required)");
  for (int m = 0; m < 3; ++m)
    if (dims[m] < 1 || dims[m] > 4096) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "dims must be in [1, 4096]");
  if (K < 1) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "K must be >= 1");
  if (!std::isfinite(eps) || eps < 0.f || eps >= 1.f) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "eps must be in [0, 1)");
  const void* ptrs[] = {B, U0, U1, U2, core};
  for (const void* q : ptrs)
    if (!aligned8(q)) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "device buffers must be 8-byte aligned");
  float2* U[3] = {reinterpret_cast<float2*>(U0), reinterpret_cast<float2*>(U1), reinterpret_cast<float2*>(U2)};
  double drop[3] = {0.0, 0.0, 0.0};
  HIP_TRY(tucker_compress_run(dims, K, reinterpret_cast<const float2*>(B), (double)eps, U,
                              reinterpret_cast<float2*>(core), ranks, drop, (hipStream_t)stream),
          "tucker_compress");
  if (dropped)
    for (int m = 0; m < 3; ++m) dropped[m] = drop[m];
  return MAXWELL_OK;
}

// ---- extra bilinear terms (multi-map)

maxwell_status maxwell_multi_encode(maxwell_plan_t plan, int32_t nmaps, const maxwell_complex64* x,
                                    const maxwell_complex64* c, maxwell_complex64* y, void* ws, size_t ws_bytes,
                                    void* stream) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  if (nmaps < 1 || nmaps > 64) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "nmaps must be in [1, 64]");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  Check ck(p);
  ck.in(x, nmaps * p->bytes_x(), "x");
  ck.in(c, nmaps * p->bytes_c(), "c");
  ck.out(y, p->bytes_y(), "y");
  ck.ws(ws, ws_bytes);
  maxwell_status s = ck.finish();
  if (s != MAXWELL_OK) return s;
  HIP_TRY(run_multi_encode(*p, nmaps, reinterpret_cast<const float2*>(x), reinterpret_cast<const float2*>(c),
                           reinterpret_cast<float2*>(y), ws, (hipStream_t)stream),
          "multi_encode");
  return MAXWELL_OK;
}

maxwell_status maxwell_multi_grad(maxwell_plan_t plan, int32_t nmaps, const maxwell_complex64* x,
                                  const maxwell_complex64* c, const maxwell_complex64* y, maxwell_complex64* gx,
                                  maxwell_complex64* gc, double* loss_dev, void* ws, size_t ws_bytes, void* stream) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  if (nmaps < 1 || nmaps > 64) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "nmaps must be in [1, 64]");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  Check ck(p);
  ck.in(x, nmaps * p->bytes_x(), "x");
  ck.in(c, nmaps * p->bytes_c(), "c");
  ck.in(y, p->bytes_y(), "y");
  ck.out(gx, nmaps * p->bytes_x(), "gx", false);
  ck.out(gc, nmaps * p->bytes_c(), "gc", false);
  ck.out(loss_dev, sizeof(double), "loss_dev", false);
  ck.ws(ws, ws_bytes);
  maxwell_status s = ck.finish();
  if (s != MAXWELL_OK) return s;
  HIP_TRY(run_multi_grad(*p, nmaps, reinterpret_cast<const float2*>(x), reinterpret_cast<const float2*>(c),
                         reinterpret_cast<const float2*>(y), reinterpret_cast<float2*>(gx),
                         reinterpret_cast<float2*>(gc), loss_dev, ws, (hipStream_t)stream),
          "multi_grad");
  return MAXWELL_OK;
}

// ---- SENSE with fixed maps and the constrained reconstruction (general path)

static maxwell_status need_general(const Plan* p) {
  if (p->fused)
    return fail(MAXWELL_ERR_UNSUPPORTED, "SENSE / ADMM calls need a plan on the general path (maxwell_plan_path)");
  return MAXWELL_OK;
}

maxwell_status maxwell_sense_encode(maxwell_plan_t plan, const maxwell_complex64* S, const maxwell_complex64* x,
                                    maxwell_complex64* y, void* ws, size_t ws_bytes, void* stream) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  if (maxwell_status g = need_general(p)) return g;
  Check ck(p);
  ck.in(S, p->bytes_S(), "S");
  ck.in(x, p->bytes_x(), "x");
  ck.out(y, p->bytes_y(), "y");
  ck.ws(ws, ws_bytes);
  maxwell_status s = ck.finish();
  if (s != MAXWELL_OK) return s;
  HIP_TRY(run_sense_encode(*p, reinterpret_cast<const float2*>(S), reinterpret_cast<const float2*>(x),
                           reinterpret_cast<float2*>(y), ws, (hipStream_t)stream),
          "sense_encode");
  return MAXWELL_OK;
}

maxwell_status maxwell_sense_adjoint(maxwell_plan_t plan, const maxwell_complex64* S, const maxwell_complex64* y,
                                     maxwell_complex64* gx, void* ws, size_t ws_bytes, void* stream) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  if (maxwell_status g = need_general(p)) return g;
  Check ck(p);
  ck.in(S, p->bytes_S(), "S");
  ck.in(y, p->bytes_y(), "y");
  ck.out(gx, p->bytes_x(), "gx");
  ck.ws(ws, ws_bytes);
  maxwell_status s = ck.finish();
  if (s != MAXWELL_OK) return s;
  HIP_TRY(run_sense_adjoint(*p, reinterpret_cast<const float2*>(S), reinterpret_cast<const float2*>(y),
                            reinterpret_cast<float2*>(gx), ws, (hipStream_t)stream),
          "sense_adjoint");
  return MAXWELL_OK;
}

maxwell_status maxwell_sense_normal(maxwell_plan_t plan, const maxwell_complex64* S, const maxwell_complex64* x,
                                    maxwell_complex64* out, void* ws, size_t ws_bytes, void* stream) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  if (maxwell_status g = need_general(p)) return g;
  Check ck(p);
  ck.in(S, p->bytes_S(), "S");
  ck.in(x, p->bytes_x(), "x");
  ck.out(out, p->bytes_x(), "out");
  ck.ws(ws, ws_bytes);
  maxwell_status s = ck.finish();
  if (s != MAXWELL_OK) return s;
  HIP_TRY(run_sense_normal(*p, reinterpret_cast<const float2*>(S), reinterpret_cast<const float2*>(x),
                           reinterpret_cast<float2*>(out), ws, (hipStream_t)stream),
          "sense_normal");
  return MAXWELL_OK;
}

maxwell_status maxwell_tv_prox(maxwell_plan_t plan, const maxwell_complex64* z, float lambda, int32_t iters,
                               maxwell_complex64* x, void* ws, size_t ws_bytes, void* stream) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  if (!std::isfinite(lambda) || lambda < 0.f) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "lambda must be finite and >= 0");
  if (iters < 0 || iters > 100000) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "iters must be in [0, 100000]");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  if (maxwell_status g = need_general(p)) return g;
  Check ck(p);
  ck.in(z, p->bytes_x(), "z");
  ck.out(x, p->bytes_x(), "x");
  ck.ws(ws, ws_bytes);
  maxwell_status s = ck.finish();
  if (s != MAXWELL_OK) return s;
  HIP_TRY(run_tv_prox(*p, reinterpret_cast<const float2*>(z), lambda, iters, reinterpret_cast<float2*>(x), ws,
                      (hipStream_t)stream),
          "tv_prox");
  return MAXWELL_OK;
}

maxwell_status maxwell_ball_project(maxwell_plan_t plan, const maxwell_complex64* w, const maxwell_complex64* y,
                                    const float* eps_dev, maxwell_complex64* z, void* ws, size_t ws_bytes,
                                    void* stream) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  if (maxwell_status g = need_general(p)) return g;
  Check ck(p);
  ck.in(w, p->bytes_y(), "w");
  ck.in(y, p->bytes_y(), "y");
  ck.in(eps_dev, (size_t)p->J * sizeof(float), "eps_dev");
  ck.out(z, p->bytes_y(), "z");
  ck.ws(ws, ws_bytes);
  maxwell_status s = ck.finish();
  if (s != MAXWELL_OK) return s;
  HIP_TRY(run_ball_project(*p, reinterpret_cast<const float2*>(w), reinterpret_cast<const float2*>(y), eps_dev,
                           reinterpret_cast<float2*>(z), ws, (hipStream_t)stream),
          "ball_project");
  return MAXWELL_OK;
}

maxwell_status maxwell_sense_admm(maxwell_plan_t plan, const maxwell_complex64* S, const maxwell_complex64* y,
                                  const float* eps_dev, float rho0, int32_t iters, int32_t cg_iters, int32_t tv_iters,
                                  maxwell_complex64* p_out, double* hist_dev, void* ws, size_t ws_bytes,
                                  void* stream) {
  if (!plan) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plan is null");
  if (!std::isfinite(rho0) || !(rho0 > 0.f)) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "rho0 must be finite and > 0");
  if (iters < 0 || iters > 100000 || cg_iters < 0 || cg_iters > 100000 || tv_iters < 0 || tv_iters > 100000)
    return fail(MAXWELL_ERR_INVALID_ARGUMENT, "iteration counts must be in [0, 100000]");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  if (maxwell_status g = need_general(p)) return g;
  Check ck(p);
  ck.in(S, p->bytes_S(), "S");
  ck.in(y, p->bytes_y(), "y");
  ck.in(eps_dev, (size_t)p->J * sizeof(float), "eps_dev");
  ck.out(p_out, p->bytes_x(), "p_out");
  ck.out(hist_dev, (size_t)iters * 3 * sizeof(double), "hist_dev", false);
  ck.ws(ws, ws_bytes);
  maxwell_status s = ck.finish();
  if (s != MAXWELL_OK) return s;
  HIP_TRY(run_admm(*p, reinterpret_cast<const float2*>(S), reinterpret_cast<const float2*>(y), eps_dev, rho0, iters,
                   cg_iters, tv_iters, reinterpret_cast<float2*>(p_out), hist_dev, ws, (hipStream_t)stream),
          "sense_admm");
  return MAXWELL_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches of slices
// A batch runs the gradient of many independent problems (slices, each with its own plan,
// basis and sampling) in one call: the slices are spread over `branches` internal streams
// forked from and joined back into the caller's stream with events, so the call can be
// captured into one hipGraph and replayed as a single launch.  Slices are assigned to
// branches longest-first by an estimate of their work (basis GEMMs + transforms).
namespace {

struct Batch {
  std::vector<const Plan*> plans;
  std::vector<size_t> off;   // workspace offset of each slice (256-aligned)
  size_t ws_total = 0;
  // shared-coefficient form (frames of one J x K): per-frame gc and loss after the slices
  bool same_jk = false;
  size_t off_gc = 0, off_loss = 0, gc_stride = 0;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  std::vector<std::vector<int>> branch;  // slice indices of each branch, in issue order
  bool staged = true;                    // phases over the slices' steps (else whole chains per branch)
  uint64_t* stamps = nullptr;            // device [2 n]: each slice's first and last step (or null)
};

// The slices' gradient steps (recorded launches) issued in phases, per branch.  A slice's
// steps form blocks: each FFT pass is a block of its own, and each run of consecutive other
// steps is one block (a segment).  Each branch takes its slices (given at creation, longest
// first) through the phases on its own stream: in phase r the segments of its slices whose
// r-th block is one run in turn, and the FFT passes of those whose r-th block is one are
// launched together, several slices per launch.  Stream order keeps each slice's blocks in
// order; the branches run side by side, forked from and joined back into the caller's
// stream by events.
hipError_t run_batch_phases(Batch& b, const std::vector<OpRecorder>& rec, hipStream_t st) {
  const int n = (int)rec.size(), nb = (int)b.streams.size();
  std::vector<std::vector<size_t>> blk(n);  // first op of each block, then a sentinel
  auto is_fft = [](const Op& op) { return std::strcmp(op.name, "fft_axis") == 0; };
  for (int i = 0; i < n; ++i) {
    const auto& ops = rec[i].ops;
    for (size_t k = 0; k < ops.size(); ++k)
      if (k == 0 || is_fft(ops[k]) || is_fft(ops[k - 1])) blk[i].push_back(k);
    blk[i].push_back(ops.size());
  }
  hipError_t e = hipEventRecord(b.fork, st);
  if (e != hipSuccess) return e;
  std::vector<FftLaunch> fft;
  for (int q = 0; q < nb; ++q) {
    hipStream_t bs = b.streams[q];
    if ((e = hipStreamWaitEvent(bs, b.fork, 0)) != hipSuccess) return e;
    size_t nphase = 0;
    for (int i : b.branch[q]) nphase = std::max(nphase, blk[i].size() - 1);
    for (size_t r = 0; r < nphase; ++r) {
      fft.clear();
      for (int i : b.branch[q]) {
        if (r + 1 >= blk[i].size()) continue;
        const auto& ops = rec[i].ops;
        const size_t k0 = blk[i][r], k1 = blk[i][r + 1];
        const bool first = k0 == 0, last = k1 == ops.size();
        if (is_fft(ops[k0]) && !first && !last) {
          fft_collect(&fft);
          e = ops[k0].run(bs);
          fft_collect(nullptr);
          if (e != hipSuccess) return e;
          continue;
        }
        if (first && b.stamps && (e = stamp_launch(b.stamps + 2 * i, bs)) != hipSuccess) return e;
        for (size_t k = k0; k < k1; ++k)
          if ((e = ops[k].run(bs)) != hipSuccess) return e;
        if (last && b.stamps && (e = stamp_launch(b.stamps + 2 * i + 1, bs)) != hipSuccess) return e;
      }
      if (!fft.empty() && (e = fft_multi_launch(fft, bs)) != hipSuccess) return e;
    }
    if ((e = hipEventRecord(b.join[q], bs)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(st, b.join[q], 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

double slice_work(const Plan& p) {
  const double N = (double)p.N, J = (double)p.J, K = (double)p.K, M = (double)p.M;
  return 3.0 * N * J * K + 2.0 * 5.0 * N * J * std::log2(N > 2 ? N : 2) + 16.0 * J * M;
}

void batch_free(Batch* b) {
  for (hipStream_t s : b->streams)
    if (s) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b->join)
    if (e) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  delete b;
}

}  // namespace

extern "C" {

maxwell_status maxwell_batch_create(const maxwell_plan_t* plans, int32_t n, int32_t branches,
                                    maxwell_batch_t* out) {
  if (!out) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "out is null");
  *out = nullptr;
  if (!plans || n < 1) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "plans must hold n >= 1 handles");
  if (branches < 0 || branches > 16) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "branches must be in [0, 16]");
  if (branches == 0) branches = 4;
  if (branches > n) branches = n;
  Batch* b = new Batch;
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    if (!plans[i]) {
      delete b;
      return fail(MAXWELL_ERR_INVALID_ARGUMENT, "a plan handle is null");
    }
    const Plan* p = reinterpret_cast<const Plan*>(plans[i]);
    b->plans.push_back(p);
    b->off.push_back(off);
    off += align256(p->ws_bytes);
  }
  b->same_jk = true;
  for (int i = 1; i < n; ++i)
    b->same_jk = b->same_jk && b->plans[i]->J == b->plans[0]->J && b->plans[i]->K == b->plans[0]->K;
  if (b->same_jk) {
    b->gc_stride = (size_t)b->plans[0]->J * (size_t)b->plans[0]->K;
    b->off_gc = off;
    off += align256(b->gc_stride * (size_t)n * 8);
    b->off_loss = off;
    off += align256((size_t)n * sizeof(double));
  }
  b->ws_total = off;
  // longest-processing-time assignment of slices to branches
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int u, int v) { return slice_work(*b->plans[u]) > slice_work(*b->plans[v]); });
  std::vector<double> load(branches, 0.0);
  b->branch.assign(branches, {});
  for (int i : idx) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b->branch[k].push_back(i);
    load[k] += slice_work(*b->plans[i]);
  }
  hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  for (int k = 0; e == hipSuccess && k < branches; ++k) {
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);  // default priority
    if (e == hipSuccess) b->streams.push_back(s);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) b->join.push_back(ev);
  }
  if (e != hipSuccess) {
    batch_free(b);
    return hip_fail(e, "batch_create");
  }
  *out = reinterpret_cast<maxwell_batch_t>(b);
  return MAXWELL_OK;
}

void maxwell_batch_destroy(maxwell_batch_t batch) {
  if (batch) batch_free(reinterpret_cast<Batch*>(batch));
}

maxwell_status maxwell_batch_workspace_size(maxwell_batch_t batch, size_t* bytes) {
  if (!batch || !bytes) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "batch or bytes is null");
  *bytes = reinterpret_cast<Batch*>(batch)->ws_total;
  return MAXWELL_OK;
}

maxwell_status maxwell_batch_grad(maxwell_batch_t batch, const maxwell_complex64* const* x,
                                  const maxwell_complex64* const* c, const maxwell_complex64* const* y,
                                  maxwell_complex64* const* gx, maxwell_complex64* const* gc,
                                  double* const* loss_dev, void* ws, size_t ws_bytes, void* stream) {
  if (!batch) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "batch is null");
  Batch* b = reinterpret_cast<Batch*>(batch);
  if (!x || !c || !y) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "x, c and y must be arrays of n pointers");
  if (ws_bytes < b->ws_total) return fail(MAXWELL_ERR_WORKSPACE_TOO_SMALL, "workspace smaller than maxwell_batch_workspace_size");
  if (b->ws_total && !ws) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "workspace is null");
  if (ws && (reinterpret_cast<uintptr_t>(ws) & 255u)) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
  const int n = (int)b->plans.size();
  // every slice validated before anything is enqueued
  for (int i = 0; i < n; ++i) {
    const Plan* p = b->plans[i];
    Check ck(p);
    ck.in(x[i], p->bytes_x(), "x");
    ck.in(c[i], p->bytes_c(), "c");
    ck.in(y[i], p->bytes_y(), "y");
    ck.out(gx ? gx[i] : nullptr, p->bytes_x(), "gx", false);
    ck.out(gc ? gc[i] : nullptr, p->bytes_c(), "gc", false);
    ck.out(loss_dev ? loss_dev[i] : nullptr, sizeof(double), "loss_dev", false);
    ck.ws(static_cast<char*>(ws) + b->off[i], ws_bytes - b->off[i]);
    const maxwell_status s = ck.finish();
    if (s != MAXWELL_OK) return fail(s, "slice " + std::to_string(i) + ": " + g_last_error);
  }
  hipStream_t st = (hipStream_t)stream;
  if (b->staged) {
    // record every slice's steps (nothing is enqueued), then issue them in rounds
    std::vector<OpRecorder> rec(n);
    for (int i = 0; i < n; ++i) {
      const Plan* p = b->plans[i];
      if (p->timing.on) return fail(MAXWELL_ERR_UNSUPPORTED, "batch_grad: per-kernel timing must be off on its plans");
      set_recorder(&rec[i]);
      const hipError_t e = run_grad(*p, reinterpret_cast<const float2*>(x[i]), reinterpret_cast<const float2*>(c[i]),
                                    reinterpret_cast<const float2*>(y[i]), gx ? reinterpret_cast<float2*>(gx[i]) : nullptr,
                                    gc ? reinterpret_cast<float2*>(gc[i]) : nullptr, loss_dev ? loss_dev[i] : nullptr,
                                    static_cast<char*>(ws) + b->off[i], st);
      set_recorder(nullptr);
      if (e != hipSuccess) return hip_fail(e, "batch_grad (record)");
    }
    HIP_TRY(run_batch_phases(*b, rec, st), "batch_grad");
    return MAXWELL_OK;
  }
  HIP_TRY(hipEventRecord(b->fork, st), "batch_grad fork");
  for (size_t k = 0; k < b->streams.size(); ++k) {
    hipStream_t bs = b->streams[k];
    HIP_TRY(hipStreamWaitEvent(bs, b->fork, 0), "batch_grad fork");
    for (int i : b->branch[k]) {
      if (b->stamps) HIP_TRY(stamp_launch(b->stamps + 2 * i, bs), "batch_grad stamp");
      HIP_TRY(run_grad(*b->plans[i], reinterpret_cast<const float2*>(x[i]), reinterpret_cast<const float2*>(c[i]),
                       reinterpret_cast<const float2*>(y[i]), gx ? reinterpret_cast<float2*>(gx[i]) : nullptr,
                       gc ? reinterpret_cast<float2*>(gc[i]) : nullptr, loss_dev ? loss_dev[i] : nullptr,
                       static_cast<char*>(ws) + b->off[i], bs),
              "batch_grad");
      if (b->stamps) HIP_TRY(stamp_launch(b->stamps + 2 * i + 1, bs), "batch_grad stamp");
    }
    HIP_TRY(hipEventRecord(b->join[k], bs), "batch_grad join");
    HIP_TRY(hipStreamWaitEvent(st, b->join[k], 0), "batch_grad join");
  }
  return MAXWELL_OK;
}

maxwell_status maxwell_batch_set_options(maxwell_batch_t batch, int32_t staged, uint64_t* stamps_dev,
                                         double* ticks_per_second) {
  if (!batch) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "batch is null");
  if (staged != 0 && staged != 1) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "staged must be 0 or 1");
  if (stamps_dev && (reinterpret_cast<uintptr_t>(stamps_dev) & 7u))
    return fail(MAXWELL_ERR_INVALID_ARGUMENT, "stamps_dev must be 8-byte aligned");
  Batch* b = reinterpret_cast<Batch*>(batch);
  if (ticks_per_second) {
    int dev = 0, khz = 0;
    HIP_TRY(hipGetDevice(&dev), "batch_set_options");
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev), "batch_set_options");
    *ticks_per_second = 1e3 * (double)khz;
  }
  b->staged = staged != 0;
  b->stamps = stamps_dev;
  return MAXWELL_OK;
}

maxwell_status maxwell_batch_grad_shared(maxwell_batch_t batch, const maxwell_complex64* const* x,
                                         const maxwell_complex64* c, const maxwell_complex64* const* y,
                                         maxwell_complex64* const* gx, maxwell_complex64* gc, double* loss_dev,
                                         void* ws, size_t ws_bytes, void* stream) {
  if (!batch) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "batch is null");
  Batch* b = reinterpret_cast<Batch*>(batch);
  if (!b->same_jk) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "shared coefficients need plans with one J and one K");
  if (!x || !c || !y) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "x, c and y are required");
  if (ws_bytes < b->ws_total) return fail(MAXWELL_ERR_WORKSPACE_TOO_SMALL, "workspace smaller than maxwell_batch_workspace_size");
  if (!ws) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "workspace is null");
  if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(MAXWELL_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
  const int n = (int)b->plans.size();
  char* w = static_cast<char*>(ws);
  float2* gcp = reinterpret_cast<float2*>(w + b->off_gc);
  double* lp = reinterpret_cast<double*>(w + b->off_loss);
  for (int i = 0; i < n; ++i) {
    const Plan* p = b->plans[i];
    Check ck(p);
    ck.in(x[i], p->bytes_x(), "x");
    ck.in(c, p->bytes_c(), "c");
    ck.in(y[i], p->bytes_y(), "y");
    ck.out(gx ? gx[i] : nullptr, p->bytes_x(), "gx", false);
    ck.out(gc, p->bytes_c(), "gc", false);
    ck.out(loss_dev, sizeof(double), "loss_dev", false);
    ck.ws(w + b->off[i], ws_bytes - b->off[i]);
    const maxwell_status s = ck.finish();
    if (s != MAXWELL_OK) return fail(s, "frame " + std::to_string(i) + ": " + g_last_error);
  }
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipEventRecord(b->fork, st), "batch_grad_shared fork");
  for (size_t k = 0; k < b->streams.size(); ++k) {
    hipStream_t bs = b->streams[k];
    HIP_TRY(hipStreamWaitEvent(bs, b->fork, 0), "batch_grad_shared fork");
    for (int i : b->branch[k])
      HIP_TRY(run_grad(*b->plans[i], reinterpret_cast<const float2*>(x[i]), reinterpret_cast<const float2*>(c),
                       reinterpret_cast<const float2*>(y[i]), gx ? reinterpret_cast<float2*>(gx[i]) : nullptr,
                       gc ? gcp + (size_t)i * b->gc_stride : nullptr, loss_dev ? lp + i : nullptr, w + b->off[i], bs),
              "batch_grad_shared");
    HIP_TRY(hipEventRecord(b->join[k], bs), "batch_grad_shared join");
    HIP_TRY(hipStreamWaitEvent(st, b->join[k], 0), "batch_grad_shared join");
  }
  if (gc) HIP_TRY(sum_rows_launch(reinterpret_cast<float2*>(gc), gcp, n, (int64_t)b->gc_stride, (int64_t)b->gc_stride, st),
                  "batch_grad_shared sum");
  if (loss_dev) HIP_TRY(sum_doubles_launch(loss_dev, lp, n, 1, st), "batch_grad_shared sum");
  return MAXWELL_OK;
}

}  // extern "C"
