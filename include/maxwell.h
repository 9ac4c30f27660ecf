/*
 * maxwell.h -- C ABI of the MI355X (gfx950) encoding-operator library for
 * Maxwell parallel imaging (Francavilla, Lefkimmiatis, Villena, Polimeridis,
 * "Maxwell Parallel Imaging").
 *
 * The library computes, for every receive coil j = 0..J-1,
 *
 *     E(x, c)_j = F_s( (B c_j) (.) x )                  paper Sec. II-B, Eq. (5)
 *
 * and its Jacobian adjoint (Sec. II-B, the expression for J_G^H), the
 * data-fidelity loss and its gradient.  Notation: x is the image (the
 * paper's density p, N = n0*n1[*n2] voxels), c_j in C^K the basis
 * coefficients of coil j (the paper's alpha_k, K its q), B the N x K basis
 * (the paper's Maxwell basis U_h, Sec. II-D), dense or Tucker-factored
 * (Sec. II-E), and F_s the undersampled Fourier operator (Sec. II-A, Eq. (1)):
 * a centred unitary DFT followed by a Cartesian mask gather, or a
 * Kaiser-Bessel NUFFT for non-Cartesian trajectories (Sec. III-B).  M is the
 * number of k-space samples per coil (the paper's K).
 *
 * Conventions for every call
 * --------------------------
 * - Complex data are interleaved {float re, im} (maxwell_complex64; the same
 *   bytes as torch.complex64 / float2), 8-byte aligned at least, C-order
 *   (last index fastest).  Image arrays are [n0][n1] or [n0][n1][n2];
 *   per-coil arrays are [J][...].
 * - All array arguments of compute calls are DEVICE pointers on the device
 *   that was current when the plan was created.  The caller owns every
 *   buffer it passes.  The plan owns only private tables (mask, twiddles,
 *   sample bins, deapodisation, split-BF16 copies of the basis).
 * - The basis arrays named in maxwell_basis_desc are device pointers owned
 *   by the caller; they must stay valid and unchanged for the plan's life.
 * - Compute calls validate every argument on the host before any HIP call
 *   and return a status; nothing aborts or throws across the ABI.  They are
 *   asynchronous on `stream` (a hipStream_t; NULL = the null stream).  A
 *   kernel fault surfaces as MAXWELL_ERR_HIP from a later call or from the
 *   caller's own synchronisation, as HIP reports it.
 * - Outputs must not overlap inputs (checked by address range).
 * - Compute calls allocate nothing: all scratch comes from the caller's
 *   workspace `ws` of `ws_bytes` bytes (>= maxwell_plan_workspace_size;
 *   256-byte aligned).  plan_create / plan_destroy are the only calls that
 *   allocate or free device memory.
 * - maxwell_last_error() returns a thread-local message describing the most
 *   recent non-OK status on the calling thread.
 */
#ifndef MAXWELL_H
#define MAXWELL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { float re, im; } maxwell_complex64;

typedef struct maxwell_plan_s* maxwell_plan_t;
typedef struct maxwell_batch_s* maxwell_batch_t;

typedef enum {
  MAXWELL_OK = 0,
  MAXWELL_ERR_INVALID_ARGUMENT = -1,   /* null/misaligned pointer, bad size, overlap, bad mask */
  MAXWELL_ERR_UNSUPPORTED = -2,        /* valid request the library does not implement       */
  MAXWELL_ERR_OUT_OF_MEMORY = -3,      /* plan_create could not allocate its tables           */
  MAXWELL_ERR_HIP = -4,                /* a HIP runtime call failed                           */
  MAXWELL_ERR_WORKSPACE_TOO_SMALL = -5 /* ws_bytes < maxwell_plan_workspace_size()            */
} maxwell_status;

typedef enum { MAXWELL_BASIS_DENSE = 0, MAXWELL_BASIS_TUCKER = 1 } maxwell_basis_kind;

/* Arithmetic of the basis contractions.  FP32: FP32 MFMA products with FP32
 * accumulation.  BF16_SPLIT: each FP32 operand a is split as hi = bf16(a),
 * lo = bf16(a - hi) (round to nearest even) and a*b is formed as
 * hi_a hi_b + hi_a lo_b + lo_a hi_b on BF16 MFMA with FP32 accumulation.
 * FFT, NUFFT and elementwise steps are FP32 in both; the loss is FP64.     */
typedef enum { MAXWELL_FP32 = 0, MAXWELL_BF16_SPLIT = 1 } maxwell_precision;

typedef enum { MAXWELL_CARTESIAN = 0, MAXWELL_NONCARTESIAN = 1 } maxwell_sampling_kind;

/* Basis descriptor (paper Sec. II-B Eq. (5): s_j = B c_j; Sec. II-E: Tucker form).
 * DENSE : `dense` is B, N x K row-major (row = C-order voxel index).
 * TUCKER: column k of B reshaped to (n0, n1, n2) is
 *         core[:, :, :, k] x_1 U[0] x_2 U[1] x_3 U[2], with the k-mode product
 *         (A x_m U)[.., i, ..] = sum_p A[.., p, ..] U[i, p]  (Sec. II-E).
 *         U[m] is n_m x r[m] row-major; core is r[0] x r[1] x r[2] x K row-major.
 *         3D images only.                                                         */
typedef struct {
  maxwell_basis_kind kind;
  int64_t K;
  const maxwell_complex64* dense;
  int64_t r[3];
  const maxwell_complex64* U[3];
  const maxwell_complex64* core;
} maxwell_basis_desc;

/* Problem geometry (paper Sec. II-A, Eq. (1): y = F S p + n, F = I_C (x) F_s).
 * ndim      2 or 3; n[d] image size along axis d (even; prime factors 2, 3, 5 only;
 *           every n[d] <= 4096).
 * J         number of coils (>= 1).
 * sampling  CARTESIAN: `mask_idx` holds M strictly ascending linear indices into the
 *             centred k-space grid (C-order; grid index i on axis d <-> frequency
 *             i - n[d]/2).  Host pointer, copied into the plan.
 *           NONCARTESIAN (2D only): `traj` holds M x ndim floats in cycles/FOV,
 *             column d paired with axis d, each in [-n[d]/2, n[d]/2).  Host pointer,
 *             copied.  kb_width W (2..8), oversamp sigma (sigma*n[d] even and
 *             >= W), kb_beta
 *             (<= 0: Beatty-Nishimura-Pauly, pi sqrt((W/sigma)^2 (sigma-1/2)^2 - 0.8)).
 * weights   optional M nonnegative data weights w_m (host pointer, copied) used by
 *           maxwell_forward_loss / maxwell_grad; NULL means w = 1.  They never enter
 *           maxwell_encode or maxwell_adjoint.                                      */
typedef struct {
  int32_t ndim;
  int64_t n[3];
  int32_t J;
  maxwell_precision precision;
  maxwell_sampling_kind sampling;
  int64_t M;
  const int64_t* mask_idx;
  const float* traj;
  const float* weights;
  int32_t kb_width;
  float oversamp;
  float kb_beta;
} maxwell_plan_desc;

/* Build a plan: validates the geometry, copies host tables, builds twiddle
 * and sampling tables on the device, and (BF16_SPLIT) a split copy of the
 * basis.  Allocates device memory; not capturable.  Environment read here:
 * MAXWELL_GEMM_AUTOTUNE=0 skips timing the dense-basis GEMM splits;
 * MAXWELL_SPREAD_SPLIT=n (NONCARTESIAN) sets the per-lane sample count above
 * which a block of the gridding adjoint goes to its split rows (default 48;
 * results agree to rounding either way); MAXWELL_SPREAD_SPLIT_PARTS=pm,ph
 * (powers of two up to 64) the workgroups per split row (default 4,16).     */
maxwell_status maxwell_plan_create(const maxwell_plan_desc* desc, const maxwell_basis_desc* basis,
                                   maxwell_plan_t* plan_out);

/* Release everything the plan allocated.  NULL is a no-op.  The caller must
 * ensure no call using the plan is still running on any stream.             */
void maxwell_plan_destroy(maxwell_plan_t plan);

/* Workspace bytes every compute call of this plan needs.                    */
maxwell_status maxwell_plan_workspace_size(maxwell_plan_t plan, size_t* bytes);

/* Which kernel sequence the plan runs (a static string owned by the library):
 *   "fused-tucker-lines"  3D Tucker basis, mask made of full lines along the last
 *                         axis, n0 and n1 multiples of 16 and <= 128, n2 <= 256,
 *                         r0, r1 <= 48: per-plane fused kernels, no [J][N] arrays;
 *   "general"             any other geometry: basis apply, per-axis FFT, gather.
 * NULL for a NULL plan.                                                       */
const char* maxwell_plan_path(maxwell_plan_t plan);

/* S[j] = B c_j  (paper Sec. II-B Eq. (5), s_k ~ U alpha_k).  c: [J][K], S: [J][N]. */
maxwell_status maxwell_basis_apply(maxwell_plan_t plan, const maxwell_complex64* c,
                                   maxwell_complex64* S, void* ws, size_t ws_bytes, void* stream);

/* c[j] = B^H S_j  (the basis block of J_G^H, Sec. II-B).  S: [J][N], c: [J][K]. */
maxwell_status maxwell_basis_apply_adjoint(maxwell_plan_t plan, const maxwell_complex64* S,
                                           maxwell_complex64* c, void* ws, size_t ws_bytes,
                                           void* stream);

/* y[j] = F_s((B c_j) (.) x)  (Sec. II-B Eq. (5)).  x: [N], c: [J][K], y: [J][M]. */
maxwell_status maxwell_encode(maxwell_plan_t plan, const maxwell_complex64* x,
                              const maxwell_complex64* c, maxwell_complex64* y, void* ws,
                              size_t ws_bytes, void* stream);

/* Jacobian adjoint at (x, c) applied to s*y, s = alpha * (*scale_dev) (or alpha when
 * scale_dev is NULL; scale_dev is a device float, read inside the kernels so no host
 * synchronisation is needed).  (Sec. II-B, J_G^H):
 *     gx   = s * sum_j conj(B c_j) (.) F_s^H y_j                 gx: [N]
 *     gc_j = s * B^H( conj(x) (.) F_s^H y_j )                    gc: [J][K]
 * Either output may be NULL (not computed).  B c is recomputed from c here; no
 * per-coil maps are kept between calls.  Weights are not applied.             */
maxwell_status maxwell_adjoint(maxwell_plan_t plan, const maxwell_complex64* x,
                               const maxwell_complex64* c, const maxwell_complex64* y,
                               float alpha, const float* scale_dev, maxwell_complex64* gx,
                               maxwell_complex64* gc, void* ws, size_t ws_bytes, void* stream);

/* Data-fidelity forward pass (Sec. II-B, Eq. (6) data term, without its 1/2):
 *     r_j  = w (.) (E(x, c)_j - y_j)                           r: [J][M] (may be NULL)
 *     loss = sum_j sum_m w_m |E(x,c)_jm - y_jm|^2              one double (may be NULL)
 * accumulated in FP64 and written to device memory.                           */
maxwell_status maxwell_forward_loss(maxwell_plan_t plan, const maxwell_complex64* x,
                                    const maxwell_complex64* c, const maxwell_complex64* y,
                                    maxwell_complex64* r, double* loss_dev, void* ws,
                                    size_t ws_bytes, void* stream);

/* The data-fidelity forward pass of maxwell_forward_loss (Sec. II-B, Eq. (6) data term)
 * with the weighted residual handed to the gradient in the plan's transfer layout:
 *     t        [J][M] entries, laid out by the plan (required unless M == 0)
 *     loss_dev as in maxwell_forward_loss (may be NULL)
 * maxwell_adjoint_transfer(plan, x, c, t, ...) then equals maxwell_adjoint(plan, x, c, r, ...)
 * for the weighted residual r = w (.) (E - y).  On the fused 3D Cartesian path
 * (maxwell_plan_path() == "fused-tucker-lines", whose readout axis is fully sampled) t is
 * r already taken back along the readout, the first factor of F_s^H in Eq. (5)'s adjoint,
 * computed while each line is on chip.  On the gridding (non-Cartesian) path, when J is a
 * multiple of the gridding's coil group (8 for J >= 8, 4 for 3 <= J < 8, any J <= 2), t
 * holds r in the gridding's sample order, coils innermost (t[s J + j] = r[j][m] for the
 * sample m at position s of the plan's sort by grid cell), so that the adjoint reads it
 * without a reordering pass.  On every other path t is r itself.                    */
maxwell_status maxwell_forward_transfer(maxwell_plan_t plan, const maxwell_complex64* x,
                                        const maxwell_complex64* c, const maxwell_complex64* y,
                                        maxwell_complex64* t, double* loss_dev, void* ws,
                                        size_t ws_bytes, void* stream);

/* maxwell_adjoint (same alpha, scale_dev, outputs and errors) applied to a residual t
 * written by maxwell_forward_transfer on the same plan.  B c is recomputed from c here;
 * t is only read.                                                                     */
maxwell_status maxwell_adjoint_transfer(maxwell_plan_t plan, const maxwell_complex64* x,
                                        const maxwell_complex64* c, const maxwell_complex64* t,
                                        float alpha, const float* scale_dev, maxwell_complex64* gx,
                                        maxwell_complex64* gc, void* ws, size_t ws_bytes,
                                        void* stream);

/* Loss and its packed real gradient (d/dRe + i d/dIm, the PyTorch convention)
 * in one call:  f = sum w |E - y|^2,  (gx, gc) = 2 J^H (w (.) (E - y)).
 * Equivalent to maxwell_forward_transfer followed by maxwell_adjoint_transfer with
 * alpha = 2, except that within this one call the adjoint reuses the forward pass's
 * B c (the maps on the unfused paths, their factor-space intermediates on the fused
 * path); nothing is kept after it returns.  gx, gc, loss_dev may each be NULL.       */
maxwell_status maxwell_grad(maxwell_plan_t plan, const maxwell_complex64* x,
                            const maxwell_complex64* c, const maxwell_complex64* y,
                            maxwell_complex64* gx, maxwell_complex64* gc, double* loss_dev,
                            void* ws, size_t ws_bytes, void* stream);

/* Gauss-Newton step of the joint image / coefficient solve (Sec. II-B, Eq. (6): the
 * linearised misfit plus alpha_n ||p + dp||^2 + beta_n sum ||a_k + da_k||^2, minimised by
 * conjugate gradients on its normal equations).
 *
 * maxwell_jvp: the Jacobian-vector product of Eq. (7) at (x, c),
 *     y_j = F_s( (B c_j) (.) dx + x (.) (B dc_j) )       dx: [N], dc: [J][K], y: [J][M]
 *   computed as E(dx, c) + E(x, dc) (E is bilinear).
 * maxwell_normal: the normal operator at (x, c),
 *     (ox, oc) = J^H (w (.) J[dx, dc]) + (lambda_x dx, lambda_c dc)
 *   with the plan's data weights w (1 when the plan has none).  For the objective of
 *   Eq. (6) (1/2 on the misfit, none on the penalties) lambda_x = 2 alpha_n and
 *   lambda_c = 2 beta_n.  Hermitian; positive definite when both lambdas are > 0.
 * maxwell_cg: iters steps of conjugate gradients from zero on
 *     normal(dx, dc) = (bx, bc)
 *   with the step lengths and direction factors from inner products Re <a, b> over both
 *   blocks accumulated in FP64 (fixed-order reductions, no atomics).  rr_dev (device,
 *   iters + 1 doubles, may be NULL) receives <r_k, r_k> for k = 0..iters (r_0 = b).  The
 *   scalars stay on the device: nothing synchronises with the host and the call can be
 *   captured.  A zero <d, A d> or <r, r> gives a zero step.  iters in [0, 100000].
 * Errors: null or misaligned required pointers, non-finite lambdas, overlapping outputs
 * and inputs, a workspace smaller than maxwell_plan_workspace_size.  The workspace holds
 * every intermediate (the JVP result, three CG vectors of N + J K entries, FP64 scalars). */
maxwell_status maxwell_jvp(maxwell_plan_t plan, const maxwell_complex64* x, const maxwell_complex64* c,
                           const maxwell_complex64* dx, const maxwell_complex64* dc, maxwell_complex64* y,
                           void* ws, size_t ws_bytes, void* stream);
maxwell_status maxwell_normal(maxwell_plan_t plan, const maxwell_complex64* x, const maxwell_complex64* c,
                              const maxwell_complex64* dx, const maxwell_complex64* dc, float lambda_x,
                              float lambda_c, maxwell_complex64* ox, maxwell_complex64* oc, void* ws,
                              size_t ws_bytes, void* stream);
maxwell_status maxwell_cg(maxwell_plan_t plan, const maxwell_complex64* x, const maxwell_complex64* c,
                          const maxwell_complex64* bx, const maxwell_complex64* bc, float lambda_x,
                          float lambda_c, int32_t iters, maxwell_complex64* dx, maxwell_complex64* dc,
                          double* rr_dev, void* ws, size_t ws_bytes, void* stream);

/* Accuracy-controlled Tucker compression of a dense basis (Sec. II-E, Eqs. (truncated_tucker)
 * and (tucker_error)): B [N][K] (device), N = dims[0] dims[1] dims[2], read as the tensor
 * T [n0][n1][n2][K]; the sequentially truncated HOSVD keeps, for modes 0, 1, 2 in turn, the
 * fewest left singular vectors of the current tensor's mode unfolding whose discarded squared
 * singular values sum to at most eps^2 ||T||^2 / 3 (Gram matrices and their Jacobi
 * eigendecomposition in FP64, mode products on the matrix cores in FP32), so that
 * ||T - core x1 U0 x2 U1 x3 U2|| <= eps ||T||.  Outputs (device, caller-owned):
 *   U0, U1, U2  [dims[m]][ranks[m]] row-major, each with capacity dims[m]^2 entries;
 *   core        [ranks[0]][ranks[1]][ranks[2]][K], capacity N K entries;
 * and on the host ranks[3] and dropped[3] (the discarded squared norm per mode; may be
 * NULL).  The result is the input of a Tucker basis descriptor.  Preprocessing, not a
 * compute call: it allocates device memory, synchronises with the host and frees before
 * returning.  eps in [0, 1); dims in [1, 4096].                                        */
maxwell_status maxwell_tucker_compress(const int64_t* dims, int64_t K, const maxwell_complex64* B, float eps,
                                       maxwell_complex64* U0, maxwell_complex64* U1, maxwell_complex64* U2,
                                       maxwell_complex64* core, int64_t* ranks, double* dropped, void* stream);

/* Extra bilinear terms (multi-map; Sec. IV-A, forward model extensions): nmaps in [1, 64]
 * map sets, each with its own image x_i and coefficients c_i,
 *     y_j = F_s( sum_i (B c_{i,j}) (.) x_i ) = sum_i E(x_i, c_i)_j
 * x: nmaps x [N], c: nmaps x [J][K] (contiguous), y: [J][M].
 * maxwell_multi_encode: y.
 * maxwell_multi_grad: loss = sum w |y_model - y|^2 (FP64) and, for every map set,
 *   (gx_i, gc_i) = 2 J_i^H (w (.) r), r = y_model - y; gx (nmaps x [N]), gc (nmaps x [J][K])
 *   and loss_dev may each be NULL.  B c_i is recomputed for the adjoints.             */
maxwell_status maxwell_multi_encode(maxwell_plan_t plan, int32_t nmaps, const maxwell_complex64* x,
                                    const maxwell_complex64* c, maxwell_complex64* y, void* ws, size_t ws_bytes,
                                    void* stream);
maxwell_status maxwell_multi_grad(maxwell_plan_t plan, int32_t nmaps, const maxwell_complex64* x,
                                  const maxwell_complex64* c, const maxwell_complex64* y, maxwell_complex64* gx,
                                  maxwell_complex64* gc, double* loss_dev, void* ws, size_t ws_bytes, void* stream);

/* SENSE with fixed maps and the constrained density reconstruction (Sec. II-C): with the
 * coil maps S [J][N] (device) fixed, minimise TV(p) subject to ||y_k - F_s S_k p|| <= eps_k.
 * General-path plans only (maxwell_plan_path() == "general"; a fused plan gives
 * MAXWELL_ERR_UNSUPPORTED); the plan's basis is not used by these calls.
 *
 * maxwell_sense_encode:  y_k = F_s(S_k (.) x)                                  y: [J][M]
 * maxwell_sense_adjoint: gx = sum_k conj(S_k) (.) F_s^H y_k                     gx: [N]
 * maxwell_sense_normal:  out = x + sum_k conj(S_k) (.) F_s^H F_s (S_k (.) x)    (the
 *   p-update operator of the ADMM iteration, I + A^H A restricted to the data blocks)
 * maxwell_tv_prox: x = argmin 1/2 ||x - z||^2 + lambda TV(x), TV(x) = sum over pixels of
 *   sqrt(sum_d |x[i + e_d] - x[i]|^2) (forward differences, zero at the last index of each
 *   axis; real and imaginary parts coupled), by iters steps of Chambolle's dual projection
 *   (step 1 / (4 ndim)) from a zero dual field.  lambda >= 0 (0 returns z).
 * maxwell_ball_project: z_k = y_k + eps_k (w_k - y_k) / max(||w_k - y_k||, eps_k) per coil,
 *   eps_dev = J device floats >= 0 (the distance in FP64).
 * maxwell_sense_admm: iters steps of the scaled ADMM of Sec. II-C with A = [I; F_s S_k]:
 *     z_0 = prox_{TV / rho}(p + u_0)          (tv_iters Chambolle steps)
 *     z_k = ball projection of F_s S_k p + u_k
 *     p  += CG (cg_iters steps from zero) on (I + sum S^H F^H F S) dp = z_0 - u_0
 *           + sum S_k^H F^H (z_k - u_k) - (I + sum S^H F^H F S) p
 *     u  += A p - z
 *   then residual balancing of rho (primal r = ||A p - z||, dual s = rho ||A^H (z - z_prev)||:
 *   rho doubles and u halves when r > 10 s, the reverse when s > 10 r).  p starts at the
 *   SENSE combination sum S^H F^H y, z and u at zero, rho at rho0 > 0.  hist_dev (device,
 *   iters x 3 doubles, may be NULL) receives (rho, r, s) of each step.  All norms are FP64
 *   and stay on the device: no host synchronisation; the call can be captured.
 * Errors: null or misaligned required pointers, bad lambda / rho0 / iteration counts,
 * overlapping outputs and inputs, a workspace smaller than maxwell_plan_workspace_size
 * (which includes the ADMM state on general-path plans).                               */
maxwell_status maxwell_sense_encode(maxwell_plan_t plan, const maxwell_complex64* S, const maxwell_complex64* x,
                                    maxwell_complex64* y, void* ws, size_t ws_bytes, void* stream);
maxwell_status maxwell_sense_adjoint(maxwell_plan_t plan, const maxwell_complex64* S, const maxwell_complex64* y,
                                     maxwell_complex64* gx, void* ws, size_t ws_bytes, void* stream);
maxwell_status maxwell_sense_normal(maxwell_plan_t plan, const maxwell_complex64* S, const maxwell_complex64* x,
                                    maxwell_complex64* out, void* ws, size_t ws_bytes, void* stream);
maxwell_status maxwell_tv_prox(maxwell_plan_t plan, const maxwell_complex64* z, float lambda, int32_t iters,
                               maxwell_complex64* x, void* ws, size_t ws_bytes, void* stream);
maxwell_status maxwell_ball_project(maxwell_plan_t plan, const maxwell_complex64* w, const maxwell_complex64* y,
                                    const float* eps_dev, maxwell_complex64* z, void* ws, size_t ws_bytes,
                                    void* stream);
maxwell_status maxwell_sense_admm(maxwell_plan_t plan, const maxwell_complex64* S, const maxwell_complex64* y,
                                  const float* eps_dev, float rho0, int32_t iters, int32_t cg_iters,
                                  int32_t tv_iters, maxwell_complex64* p_out, double* hist_dev, void* ws,
                                  size_t ws_bytes, void* stream);

/* Batches of independent slices (the batched serving form of the operator: many 2D
 * problems of uneven sizes, each with its own plan, basis and sampling, Sec. II-B per
 * slice).
 * maxwell_batch_create: plans = host array of n >= 1 plan handles (copied; the plans must
 *   outlive the batch); branches = concurrent branches in [1, 16] (0: 4, capped at n).  The
 *   slices are assigned to branches at creation, longest first by an estimate of their work.
 *   Creates the branches' streams (default priority) and events; the only batch call that
 *   allocates.
 * maxwell_batch_workspace_size: bytes of the batch workspace (the slices' plan workspaces
 *   side by side, each 256-byte aligned, and, when every plan has the same J and K, the
 *   per-frame partials of maxwell_batch_grad_shared).
 * maxwell_batch_grad: maxwell_grad of every slice i on its own buffers x[i], c[i], y[i] ->
 *   gx[i], gc[i], loss_dev[i] (x, c, y: host arrays of n device pointers; gx, gc, loss_dev:
 *   host arrays of n device pointers or NULL, entries may be NULL).  Every slice is
 *   validated as in maxwell_grad before anything is enqueued (errors name the slice).  The
 *   branches are forked from `stream` by an event and joined back into it, so the whole call
 *   can be captured into one hipGraph and replayed as a single launch.  Slices must not share
 *   output buffers; calls on one batch must not overlap in time.  By default the slices'
 *   steps are issued in phases: a slice's steps form blocks (each FFT pass one block, each
 *   run of other steps one block), and each branch takes its slices through the phases on
 *   its stream, phase r being the r-th block of each of its slices; a phase's FFT passes of
 *   the branch's slices go out together, up to 16 slices' passes per launch (descriptors in
 *   the kernel arguments), its other blocks run in turn;
 *   each slice's result is the same, bit for bit, as its own maxwell_grad.  Plans in a batch
 *   must have per-kernel timing off (else MAXWELL_ERR_UNSUPPORTED).
 * maxwell_batch_set_options: staged = 1 (default) issues the slices' steps in phases as
 *   above; 0 runs each slice's whole chain of launches on its branch.  stamps_dev: a device
 *   array of 2n uint64 (8-byte aligned) or NULL; when set, every later maxwell_batch_grad
 *   (also under capture) writes slice i's device wall-clock at the start of its first step
 *   to stamps_dev[2i] and at the end of its last to stamps_dev[2i + 1], the slice's latency
 *   inside the batch.  ticks_per_second (host, may be NULL) receives the clock's rate.
 * maxwell_batch_destroy: releases the streams and events (not the plans).                  */
maxwell_status maxwell_batch_create(const maxwell_plan_t* plans, int32_t n, int32_t branches,
                                    maxwell_batch_t* out);
maxwell_status maxwell_batch_workspace_size(maxwell_batch_t batch, size_t* bytes);
maxwell_status maxwell_batch_grad(maxwell_batch_t batch, const maxwell_complex64* const* x,
                                  const maxwell_complex64* const* c,
                                  const maxwell_complex64* const* y, maxwell_complex64* const* gx,
                                  maxwell_complex64* const* gc, double* const* loss_dev, void* ws,
                                  size_t ws_bytes, void* stream);
maxwell_status maxwell_batch_set_options(maxwell_batch_t batch, int32_t staged, uint64_t* stamps_dev,
                                         double* ticks_per_second);
void maxwell_batch_destroy(maxwell_batch_t batch);

/* Frames with shared coefficients (dynamic or multi-contrast data, the remark after the
 * constrained problem of Sec. II-C and the end of Sec. II-B: per frame t its own image x_t and
 * sampling (one plan per frame), one coefficient set c shared by all frames):
 *     loss = sum_t f_t(x_t, c),   gx_t = grad of f_t in x_t,   gc = sum_t (grad of f_t in c)
 * every frame as in maxwell_grad, then gc and the loss summed over the frames in frame order
 * (fixed order, no atomics).  The batch's plans must share J and K (else
 * MAXWELL_ERR_INVALID_ARGUMENT); its workspace size already includes the per-frame
 * partials.  x, y, gx: host arrays of n device pointers (gx may be NULL); c, gc, loss_dev:
 * single device pointers (gc, loss_dev may be NULL).  Capturable like maxwell_batch_grad. */
maxwell_status maxwell_batch_grad_shared(maxwell_batch_t batch, const maxwell_complex64* const* x,
                                         const maxwell_complex64* c, const maxwell_complex64* const* y,
                                         maxwell_complex64* const* gx, maxwell_complex64* gc, double* loss_dev,
                                         void* ws, size_t ws_bytes, void* stream);

/* Kernel timing for benchmarks.  enable != 0 clears the plan's records and
 * starts recording: every kernel launch made by a compute call of this plan is
 * then bracketed by two HIP events recorded on the call's stream (event objects
 * are created on first use and reused).  enable == 0 stops recording.  Not for
 * use under graph capture.                                                     */
maxwell_status maxwell_plan_set_timing(maxwell_plan_t plan, int enable);

/* Summary of the records since the last maxwell_plan_set_timing(plan, 1):
 * synchronises the recorded events, then for kernel index i (0 <= i < *count)
 * returns its name (static string), number of launches and summed duration in
 * milliseconds.  `count` may be queried alone with the other pointers NULL;
 * an i outside [0, *count) with a non-NULL name returns INVALID_ARGUMENT.      */
maxwell_status maxwell_plan_timing(maxwell_plan_t plan, int i, int* count, const char** name,
                                   int64_t* launches, double* total_ms);

/* Thread-local text for the last non-OK status returned on this thread.       */
const char* maxwell_last_error(void);

/* Library version string, e.g. "maxwell-gfx950 0.1".                          */
const char* maxwell_version(void);

/* Plan-time kernel choices: for a dense basis, plan creation times the streaming kernel
 * (few coils) against the tiled GEMM at each split-K factor for both basis products and
 * keeps the fastest, per (GPU architecture, product, N, K, J, precision).  The choices are
 * kept for the process and in a tuning file, $MAXWELL_TUNE_CACHE if set (empty: none), else
 * $HOME/.cache/maxwell/tune.txt, so a later process reuses them without timing.
 * MAXWELL_GEMM_AUTOTUNE=0 skips the timing (a fixed rule).  maxwell_tune_counts: the
 * choices timed and the choices reused since the process started (either may be NULL).  */
maxwell_status maxwell_tune_counts(int64_t* measured, int64_t* reused);

/* maxwell_grad with no workspace argument, for callers that cannot allocate device memory
 * (code under graph capture, tight serving loops, harnesses that forbid allocation).  The
 * workspace is a library-held device buffer of MAXWELL_STATIC_WS_BYTES (64 MiB) on each
 * device, kept until the process ends; the call allocates nothing.  Plans whose workspace
 * (maxwell_plan_workspace_size) exceeds it are refused with
 * MAXWELL_ERR_WORKSPACE_TOO_SMALL; a plan with per-kernel timing on with
 * MAXWELL_ERR_UNSUPPORTED.  Every call on one device shares that device's buffer, which
 * keeps the last call's contents (no step reads scratch it has not written): calls that
 * overlap in time on one device (other streams, other host threads) race and must be
 * serialised by the caller.  Arguments and results as maxwell_grad.                    */
#define MAXWELL_STATIC_WS_BYTES ((size_t)64 << 20)
maxwell_status maxwell_grad_static(maxwell_plan_t plan, const maxwell_complex64* x, const maxwell_complex64* c,
                                   const maxwell_complex64* y, maxwell_complex64* gx, maxwell_complex64* gc,
                                   double* loss_dev, void* stream);

/* Diagnostic: the device BF16 split of the BF16_SPLIT products (see maxwell_precision),
 * applied to n FP32 values x (device): hi[i] = bf16(x[i]), lo[i] = bf16(x[i] - hi[i]),
 * both round to nearest even, as BF16 bit patterns (device uint16 arrays of n entries).
 * variant 0: the packed hardware converts of the matrix-core tiles (plane kernels,
 * fragment-ordered operands); 1: the tiled GEMM's operand split (n must be even: the
 * values are complex pairs); 2: the core planes' split.  Asynchronous on stream;
 * n = 0 does nothing; x, hi, lo must not overlap.                                       */
maxwell_status maxwell_bf16_split(const float* x, int64_t n, int32_t variant, uint16_t* hi, uint16_t* lo,
                                  void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MAXWELL_H */
