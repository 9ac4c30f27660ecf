// Accuracy-controlled Tucker compression of a dense basis (paper Sec. II-E, Eqs.
// (truncated_tucker) and (tucker_error)) by the sequentially truncated higher-order SVD.
//
// The basis B [N][K] is the tensor T [n0][n1][n2][K]; for modes m = 0, 1, 2 in turn:
//   G = Y_(m) Y_(m)^H            the Gram matrix of the mode-m unfolding of the current tensor,
//                                accumulated in FP64 (gram kernels below)
//   G = V diag(lambda) V^H       cyclic Jacobi in FP64 (one workgroup, round-robin pairs)
//   r_m = fewest leading eigenvalues whose discarded sum is <= eps^2 ||T||^2 / 3
//   U_m = those eigenvectors;  Y <- Y x_m U_m^H   (a batched complex GEMM, FP32)
// The core is the final Y [r0][r1][r2][K].  The squared error is the sum of the discarded
// eigenvalues, so ||T - core x U|| <= eps ||T||.
//
// FP64 Gram: the truncation threshold sits at eps^2 / 3 of the energy (3e-9 at eps = 1e-4),
// far below FP32 resolution of a Gram entry, so the products are accumulated in FP64.
//
// Jacobi (Golub and Van Loan, Matrix Computations, Sec. 8.5, the symmetric Schur step, made
// complex by a phase): for a pair (p, q) with a = G_pp, b = G_qq, c = G_pq = |c| e^{i phi},
// tau = (b - a) / (2|c|), t = sign(tau) / (|tau| + sqrt(1 + tau^2)), cs = 1 / sqrt(1 + t^2),
// sn = t cs, and R = [[cs, sn], [-sn e^{-i phi}, cs e^{-i phi}]] zeroes G_pq in R^H G R.
// n/2 disjoint pairs per round (the circle schedule); all pairs' rotations are formed from
// the matrix at the start of the round, then applied to the columns (and V), then to the rows.
// This call is preprocessing: it allocates, synchronises with the host to choose the ranks,
// and frees before returning.
#include "common.h"
#include "compress.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

namespace mx {

namespace {

struct z64 {
  double x, y;
};
__device__ __forceinline__ z64 zmul(z64 a, z64 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ z64 zconj(z64 a) { return {a.x, -a.y}; }
__device__ __forceinline__ z64 zadd(z64 a, z64 b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ z64 zscale(z64 a, double s) { return {a.x * s, a.y * s}; }

constexpr int GT = 16;  // Gram tile edge
constexpr int GL = 32;  // unfolding columns per LDS stage

// part[c][a][b] (upper-triangle tiles only) = sum over the chunk's columns l of
// Y(l, a) conj(Y(l, b)),  Y(l, a) = Y[alpha][a][beta] with l = alpha * Bq + beta.
__global__ __launch_bounds__(GT* GT) void gram_partial_kernel(const float2* __restrict__ Y, int64_t A, int n,
                                                              int64_t Bq, int64_t chunk, int ntile,
                                                              z64* __restrict__ part) {
  __shared__ z64 sa[GT][GL + 1], sb[GT][GL + 1];
  // tile pair (ta <= tb) from blockIdx.x, chunk from blockIdx.y
  int ta = 0, rem = blockIdx.x;
  while (rem >= ntile - ta) { rem -= ntile - ta; ++ta; }
  const int tb = ta + rem;
  const int64_t L = A * Bq;
  const int64_t l0 = (int64_t)blockIdx.y * chunk, l1 = l0 + chunk < L ? l0 + chunk : L;
  const int ai = threadIdx.x / GT, bi = threadIdx.x % GT;
  z64 acc = {0.0, 0.0};
  for (int64_t lb = l0; lb < l1; lb += GL) {
    __syncthreads();
    for (int e = threadIdx.x; e < GT * GL; e += GT * GT) {
      const int r = e / GL, t = e % GL;
      const int64_t l = lb + t;
      z64 va = {0.0, 0.0}, vb = {0.0, 0.0};
      if (l < l1) {
        const int64_t al = l / Bq, be = l % Bq;
        const int a = ta * GT + r, b = tb * GT + r;
        if (a < n) { const float2 v = Y[(al * n + a) * Bq + be]; va = {(double)v.x, (double)v.y}; }
        if (b < n) { const float2 v = Y[(al * n + b) * Bq + be]; vb = {(double)v.x, (double)v.y}; }
      }
      sa[r][t] = va;
      sb[r][t] = vb;
    }
    __syncthreads();
#pragma unroll 8
    for (int t = 0; t < GL; ++t) acc = zadd(acc, zmul(sa[ai][t], zconj(sb[bi][t])));
  }
  const int a = ta * GT + ai, b = tb * GT + bi;
  if (a < n && b < n) part[((int64_t)blockIdx.y * n + a) * n + b] = acc;
}

// G[a][b] = sum_c part[c][a][b] in chunk order for a <= b (tile-wise), mirrored Hermitian
__global__ void gram_reduce_kernel(const z64* __restrict__ part, int n, int nchunk, z64* __restrict__ G) {
  const int64_t total = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e / n), b = (int)(e % n);
    const bool upper = (a / GT) <= (b / GT);
    const int ra = upper ? a : b, rb = upper ? b : a;
    z64 s = {0.0, 0.0};
    for (int c = 0; c < nchunk; ++c) s = zadd(s, part[((int64_t)c * n + ra) * n + rb]);
    G[e] = upper ? s : zconj(s);
  }
}

constexpr int JT = 1024;  // threads of the Jacobi workgroup

__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  for (int h = JT / 2; h > 0; h >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
  }
  __syncthreads();
  const double s = red[0];
  __syncthreads();
  return s;
}

// G (n x n, Hermitian, FP64) -> diag(G) = eigenvalues, V = eigenvectors (columns).
// MAXP bounds the pairs per round (n <= 2 MAXP); LDS_RESIDENT: G and V are copied into
// dynamic LDS (2 n^2 complex doubles) for the sweeps and back at the end.
template <int MAXP, bool LDS_RESIDENT>
__global__ __launch_bounds__(JT) void jacobi_kernel(z64* __restrict__ Gg, z64* __restrict__ Vg, int n, int max_sweeps,
                                                   int* __restrict__ sweeps_done) {
  extern __shared__ z64 dyn[];
  __shared__ double red[JT];
  __shared__ int pp[MAXP], pq[MAXP];
  __shared__ double pc[MAXP], ps[MAXP];
  __shared__ z64 pe[MAXP];
  const int n2 = n + (n & 1);
  const int npair = n2 / 2;
  // leading dimension: rows padded by one entry in LDS, so that a column walk spreads over banks
  const int ld = LDS_RESIDENT ? n + 1 : n;
  z64* G = LDS_RESIDENT ? dyn : Gg;
  z64* V = LDS_RESIDENT ? dyn + (int64_t)n * ld : Vg;
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += JT) {
    const int a = (int)(e / n), b = (int)(e % n);
    V[(int64_t)a * ld + b] = {a == b ? 1.0 : 0.0, 0.0};
    if (LDS_RESIDENT) G[(int64_t)a * ld + b] = Gg[e];
  }
  __syncthreads();
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += JT) {
      const int a = (int)(e / n), b = (int)(e % n);
      const z64 g = G[(int64_t)a * ld + b];
      const double m2 = g.x * g.x + g.y * g.y;
      if (a == b) dia += m2; else off += m2;
    }
    off = block_sum(off, red);
    dia = block_sum(dia, red);
    if (off <= 1e-30 * dia || dia == 0.0) break;
    for (int round = 0; round < n2 - 1; ++round) {
      for (int k = threadIdx.x; k < npair; k += JT) {
        int p, q;
        if (k == 0) { p = round; q = n2 - 1; }
        else { p = (round + k) % (n2 - 1); q = (round - k + n2 - 1) % (n2 - 1); }
        if (p > q) { const int t = p; p = q; q = t; }
        double cs = 1.0, sn = 0.0;
        z64 ph = {1.0, 0.0};
        if (q < n) {
          const double a = G[(int64_t)p * ld + p].x, b = G[(int64_t)q * ld + q].x;
          const z64 c = G[(int64_t)p * ld + q];
          const double ac = sqrt(c.x * c.x + c.y * c.y);
          if (ac > 1e-300 && ac > 1e-18 * sqrt(fabs(a * b))) {
            const double tau = (b - a) / (2.0 * ac);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            cs = 1.0 / sqrt(1.0 + t * t);
            sn = t * cs;
            ph = {c.x / ac, c.y / ac};
          }
        }
        pp[k] = p; pq[k] = q < n ? q : -1; pc[k] = cs; ps[k] = sn; pe[k] = ph;
      }
      __syncthreads();
      // columns p, q of G and V:  col_p <- cs col_p - sn conj(e) col_q;  col_q <- sn col_p + cs conj(e) col_q
      // (consecutive threads take different pairs of one row)
      for (int64_t w = threadIdx.x; w < (int64_t)npair * n; w += JT) {
        const int i = (int)(w / npair), k = (int)(w % npair);
        const int q = pq[k];
        if (q < 0 || ps[k] == 0.0) continue;
        const int p = pp[k];
        const double cs = pc[k], sn = ps[k];
        const z64 ec = zconj(pe[k]);
        for (int mat = 0; mat < 2; ++mat) {
          z64* M = mat == 0 ? G : V;
          const z64 gp = M[(int64_t)i * ld + p], gq = zmul(ec, M[(int64_t)i * ld + q]);
          M[(int64_t)i * ld + p] = zadd(zscale(gp, cs), zscale(gq, -sn));
          M[(int64_t)i * ld + q] = zadd(zscale(gp, sn), zscale(gq, cs));
        }
      }
      __syncthreads();
      // rows p, q of G:  row_p <- cs row_p - sn e row_q;  row_q <- sn row_p + cs e row_q
      for (int64_t w = threadIdx.x; w < (int64_t)npair * n; w += JT) {
        const int k = (int)(w / n), j = (int)(w % n);
        const int q = pq[k];
        if (q < 0 || ps[k] == 0.0) continue;
        const int p = pp[k];
        const double cs = pc[k], sn = ps[k];
        const z64 gp = G[(int64_t)p * ld + j], gq = zmul(pe[k], G[(int64_t)q * ld + j]);
        G[(int64_t)p * ld + j] = zadd(zscale(gp, cs), zscale(gq, -sn));
        G[(int64_t)q * ld + j] = zadd(zscale(gp, sn), zscale(gq, cs));
      }
      __syncthreads();
    }
  }
  if (LDS_RESIDENT) {
    __syncthreads();
    for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += JT) {
      const int a = (int)(e / n), b = (int)(e % n);
      Gg[e] = G[(int64_t)a * ld + b];
      Vg[e] = V[(int64_t)a * ld + b];
    }
  }
  if (threadIdx.x == 0) *sweeps_done = sweep;
}

__global__ void sumsq_kernel(const float2* __restrict__ v, int64_t n, double* __restrict__ part) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    acc += (double)v[e].x * v[e].x + (double)v[e].y * v[e].y;
  s[threadIdx.x] = acc;
  for (int h = 128; h > 0; h >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() { if (p) (void)hipFree(p); }
  hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes ? bytes : 8); }
  template <typename T> T* as() { return reinterpret_cast<T*>(p); }
};

}  // namespace

hipError_t tucker_compress_run(const int64_t* dims, int64_t K, const float2* B, double eps, float2* const* U_out,
                               float2* core_out, int64_t* ranks, double* dropped, hipStream_t st) {
  const int64_t N = dims[0] * dims[1] * dims[2];
  hipError_t e;
  // ||T||^2 in FP64
  DevBuf sq;
  if ((e = sq.alloc(1024 * sizeof(double))) != hipSuccess) return e;
  hipLaunchKernelGGL(sumsq_kernel, dim3(1024), dim3(256), 0, st, B, N * K, sq.as<double>());
  std::vector<double> hs(1024);
  if ((e = hipMemcpyAsync(hs.data(), sq.p, 1024 * sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  double total = 0.0;
  for (double v : hs) total += v;
  const double budget = eps * eps * total / 3.0;
  DevBuf ping, pong;
  if ((e = ping.alloc((size_t)N * K * sizeof(float2))) != hipSuccess) return e;
  if ((e = pong.alloc((size_t)N * K * sizeof(float2))) != hipSuccess) return e;
  const float2* Y = B;
  float2* out = ping.as<float2>();
  int64_t cur[3] = {dims[0], dims[1], dims[2]};
  for (int m = 0; m < 3; ++m) {
    const int n = (int)cur[m];
    int64_t A = 1, Bq = K;
    for (int d = 0; d < m; ++d) A *= cur[d];
    for (int d = m + 1; d < 3; ++d) Bq *= cur[d];
    const int ntile = (n + GT - 1) / GT;
    const int npairs = ntile * (ntile + 1) / 2;
    const int64_t L = A * Bq;
    int nchunk = (int)std::max<int64_t>(1, std::min<int64_t>(2048 / std::max(npairs, 1), (L + 4095) / 4096));
    const int64_t chunk = ((L + nchunk - 1) / nchunk + GL - 1) / GL * GL;
    nchunk = (int)((L + chunk - 1) / chunk);
    DevBuf part, G, V, sw;
    if ((e = part.alloc((size_t)nchunk * n * n * sizeof(z64))) != hipSuccess) return e;
    if ((e = G.alloc((size_t)n * n * sizeof(z64))) != hipSuccess) return e;
    if ((e = V.alloc((size_t)n * n * sizeof(z64))) != hipSuccess) return e;
    if ((e = sw.alloc(sizeof(int))) != hipSuccess) return e;
    hipLaunchKernelGGL(gram_partial_kernel, dim3(npairs, nchunk), dim3(GT * GT), 0, st, Y, A, n, Bq, chunk, ntile,
                       part.as<z64>());
    hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)std::min<int64_t>(((int64_t)n * n + 255) / 256, 4096)),
                       dim3(256), 0, st, part.as<z64>(), n, nchunk, G.as<z64>());
    if (n <= 64)  // both matrices, rows padded by one, fit in LDS (about 130 KiB)
      hipLaunchKernelGGL((jacobi_kernel<32, true>), dim3(1), dim3(JT), 2 * (size_t)n * (n + 1) * sizeof(z64), st,
                         G.as<z64>(), V.as<z64>(), n, 60, sw.as<int>());
    else
      hipLaunchKernelGGL((jacobi_kernel<2048, false>), dim3(1), dim3(JT), 0, st, G.as<z64>(), V.as<z64>(), n, 60,
                         sw.as<int>());
    if ((e = hipGetLastError()) != hipSuccess) return e;
    std::vector<z64> hG((size_t)n * n), hV((size_t)n * n);
    if ((e = hipMemcpyAsync(hG.data(), G.p, hG.size() * sizeof(z64), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(hV.data(), V.p, hV.size() * sizeof(z64), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    // eigenvalues in descending order; fewest kept with discarded sum <= budget
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return hG[(size_t)a * n + a].x > hG[(size_t)b * n + b].x; });
    std::vector<double> tail(n + 1, 0.0);
    for (int i = n - 1; i >= 0; --i) tail[i] = tail[i + 1] + std::max(0.0, hG[(size_t)order[i] * n + order[i]].x);
    int r = 0;
    while (r < n && tail[r] > budget) ++r;
    if (r < 1) r = 1;
    ranks[m] = r;
    dropped[m] = tail[r];
    std::vector<float2> hU((size_t)n * r);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < r; ++k) {
        const z64 v = hV[(size_t)i * n + order[k]];
        hU[(size_t)i * r + k] = make_float2((float)v.x, (float)v.y);
      }
    if ((e = hipMemcpyAsync(U_out[m], hU.data(), hU.size() * sizeof(float2), hipMemcpyHostToDevice, st)) != hipSuccess)
      return e;
    // Y' [A][r][Bq] = U^H applied along mode m, one GEMM per leading index
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    g.alpha = 1.0f;
    g.batch = A;
    g.M = r; g.N = Bq; g.K = n;
    g.A = U_out[m]; g.a_ms = 1; g.a_ks = r; g.a_bs = 0; g.conjA = 1;
    g.B = Y; g.b_ks = Bq; g.b_ns = 1; g.b_bs = (int64_t)n * Bq;
    g.C = m == 2 ? core_out : out; g.c_ms = Bq; g.c_ns = 1; g.c_bs = (int64_t)r * Bq;
    DevBuf gws;
    if ((e = gws.alloc(gemm_workspace_bytes(g))) != hipSuccess) return e;
    if ((e = gemm_launch(g, 0, gws.p, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    cur[m] = r;
    Y = out;
    out = (out == ping.as<float2>()) ? pong.as<float2>() : ping.as<float2>();
  }
  return hipSuccess;
}

}  // namespace mx
