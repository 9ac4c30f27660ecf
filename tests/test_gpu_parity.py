"""GPU parity: every C-ABI entry point against the FP64 oracle on the same seeded inputs.

Sizes span several 64-wide GEMM tiles and FFT tiles with ragged tails, radix
2/3/5 axes, 2D dense and 3D Tucker bases, random-point and full-line masks.
Bar (relative L2 over the whole output, FP64): FP32 <= 1e-5, BF16-split <= 1e-4.
"""
import math

import numpy as np
import pytest
import torch

from _common import TOL, Case, assert_close, c64, rel

pytestmark = pytest.mark.gpu

DEV = "cuda:0"

CASES = {
    "dense2d_48x40_J5_K37": dict(seed=101, dims=(48, 40), J=5, K=37, basis="dense", weights=True),
    "dense2d_64x64_J8_K32": dict(seed=102, dims=(64, 64), J=8, K=32, basis="dense"),
    "dense2d_30x20_radix35": dict(seed=103, dims=(30, 20), J=3, K=9, basis="dense"),
    # dense apply streaming kernel: three and four coil blocks, a ragged K16 step, N not a
    # multiple of its 64-row wave share
    "dense2d_40x36_J40_K24": dict(seed=120, dims=(40, 36), J=40, K=24, basis="dense", weights=True),
    "dense2d_30x30_J64_K20": dict(seed=121, dims=(30, 30), J=64, K=20, basis="dense"),
    "tucker3d_24x20x18_r7x5x6_K13": dict(seed=104, dims=(24, 20, 18), ranks=(7, 5, 6), J=3, K=13,
                                         basis="tucker", mask="lines3d", frac=0.3, weights=True),
    "tucker3d_12x10x6_radix35": dict(seed=105, dims=(12, 10, 6), ranks=(4, 3, 5), J=2, K=7,
                                     basis="tucker", mask="random"),
    "tucker3d_32x32x32_r12_K70_J4": dict(seed=106, dims=(32, 32, 32), ranks=(12, 12, 12), J=4, K=70,
                                         basis="tucker", mask="lines3d", frac=0.25),
    # fused plane path: n0, n1 multiples of 16; ragged coil groups, radix-5 plane axis, rank padding
    "fused_48x32x20_r9x13x5_K23_J5": dict(seed=109, dims=(48, 32, 20), ranks=(9, 13, 5), J=5, K=23,
                                          basis="tucker", mask="lines3d", frac=0.3, weights=True),
    "fused_16x80x12_r3x17x4_K11_J3": dict(seed=110, dims=(16, 80, 12), ranks=(3, 17, 4), J=3, K=11,
                                          basis="tucker", mask="lines3d", frac=0.2),
    "fused_128x128x64_r40_K60_J5": dict(seed=111, dims=(128, 128, 64), ranks=(40, 40, 40), J=5, K=60,
                                        basis="tucker", mask="lines3d", frac=0.125),
    "fused_64x64x32_r20_K30_J3": dict(seed=112, dims=(64, 64, 32), ranks=(20, 20, 7), J=3, K=30,
                                      basis="tucker", mask="lines3d", frac=0.2, weights=True),
    # 128 x 128 planes with ranks below 33 (run-time rank blocks in both plane kernels)
    "fused_128x128x32_r20x14x9_K30_J3": dict(seed=122, dims=(128, 128, 32), ranks=(20, 14, 9), J=3, K=30,
                                             basis="tucker", mask="lines3d", frac=0.15, weights=True),
    # core contraction kernels: several rho chunks with a ragged tail, two k groups, 3 and 4
    # coil blocks; J = 65 takes the GEMM fallback
    "tucker3d_16x16x12_r9x10x11_K150_J37": dict(seed=116, dims=(16, 16, 12), ranks=(9, 10, 11), J=37, K=150,
                                                basis="tucker", mask="random", frac=0.3, weights=True),
    "fused_32x32x16_r9x10x11_K150_J64": dict(seed=117, dims=(32, 32, 16), ranks=(9, 10, 11), J=64, K=150,
                                             basis="tucker", mask="lines3d", frac=0.3),
    "tucker3d_12x10x8_r5x4x3_K20_J65": dict(seed=118, dims=(12, 10, 8), ranks=(5, 4, 3), J=65, K=20,
                                            basis="tucker", mask="lines3d", frac=0.3),
    # fused path with a readout rank above the third-mode kernels' limit (GEMM fallback)
    "fused_32x16x80_r5x6x70_K9_J2": dict(seed=119, dims=(32, 16, 80), ranks=(5, 6, 70), J=2, K=9,
                                         basis="tucker", mask="lines3d", frac=0.3),
    # radial sampling (KB NUFFT, W = 6, sigma = 2, ramp density compensation in the loss)
    "radial_32x24_J3_K9_7spokes": dict(seed=113, dims=(32, 24), J=3, K=9, mask="radial", spokes=7, weights=True),
    "radial_40x30_J2_K6_5spokes": dict(seed=114, dims=(40, 30), J=2, K=6, mask="radial", spokes=5, n_read=48),
    "radial_256_J2_K20_64spokes": dict(seed=115, dims=(256, 256), J=2, K=20, mask="radial", spokes=64,
                                       n_read=512, weights=True),
    # N = 1,105,920 (not a power of two, above 2^20): the FFT passes that carry the mask divide
    # flat indices by N with a multiply-high
    "dense3d_96x96x120_J2_K4": dict(seed=117, dims=(96, 96, 120), J=2, K=4, basis="dense", mask="random",
                                    frac=0.3),
    # 12 coils: one full and one padded group of 8 in the spread
    "radial_64x48_J12_K7_16spokes": dict(seed=116, dims=(64, 48), J=12, K=7, mask="radial", spokes=16,
                                         n_read=128, weights=True),
    # coil groups that fill J: the gradient's residual is handed to the spread in its sample
    # order (J = 1: scalar writes, one coil per lane; J = 8: one full group, 16-byte writes)
    "radial_48x40_J1_K5_9spokes": dict(seed=123, dims=(48, 40), J=1, K=5, mask="radial", spokes=9,
                                       n_read=96, weights=True),
    "radial_64x64_J8_K6_12spokes": dict(seed=124, dims=(64, 64), J=8, K=6, mask="radial", spokes=12,
                                        n_read=128),
    # other oversampling factors and kernel widths: the image window sits at other offsets of
    # the grid (60 x 54 with the window at rows 10.., columns 9..; 80 x 60 at 8.., 6..), which
    # the grid transform's pad, pruned and crop passes must honour; grid sizes with radices 3
    # and 5
    "radial_40x36_J3_K6_sigma1.5_W4": dict(seed=125, dims=(40, 36), J=3, K=6, mask="radial", spokes=10,
                                           n_read=80, weights=True, oversamp=1.5, kb_width=4),
    "radial_64x48_J9_K5_sigma1.25_W5": dict(seed=126, dims=(64, 48), J=9, K=5, mask="radial", spokes=14,
                                            n_read=128, oversamp=1.25, kb_width=5),
}
FUSED = {"tucker3d_32x32x32_r12_K70_J4", "fused_48x32x20_r9x13x5_K23_J5", "fused_16x80x12_r3x17x4_K11_J3",
         "fused_128x128x64_r40_K60_J5", "fused_64x64x32_r20_K30_J3", "fused_32x32x16_r9x10x11_K150_J64",
         "fused_32x16x80_r5x6x70_K9_J2", "fused_128x128x32_r20x14x9_K30_J3"}

_cache = {}


def get_case(name):
    if name not in _cache:
        _cache[name] = Case(**CASES[name])
    return _cache[name]


def T(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(np.complex64))).to(DEV)


def H(t):
    return t.detach().cpu().numpy().astype(np.complex128)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible ROCm GPU"
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["fp32", "bf16_split"])
@pytest.mark.parametrize("name", list(CASES))
def test_basis_apply_and_adjoint(name, prec):
    cs = get_case(name)
    print(f"[case] {name} {prec}", flush=True)
    plan = cs.plan(prec)
    S = H(plan.basis_apply(T(cs.c0)))
    S_ref = cs.op.coil_maps(cs.c0)
    assert_close(S, S_ref, TOL[prec], coils=True, what="S")
    h = c64(np.random.default_rng(7).normal(size=S_ref.shape) + 1j * np.random.default_rng(8).normal(size=S_ref.shape))
    c_back = H(plan.basis_adjoint(T(h)))
    assert_close(c_back, cs.op.basis_adjoint(h), TOL[prec], coils=True, what="B^H h")


@pytest.mark.parametrize("prec", ["fp32", "bf16_split"])
@pytest.mark.parametrize("name", list(CASES))
def test_encode_adjoint_grad(name, prec):
    cs = get_case(name)
    print(f"[case] {name} {prec}", flush=True)
    plan = cs.plan(prec)
    assert plan.path == ("fused-tucker-lines" if name in FUSED else "general")
    tol = TOL[prec]
    x, c, y = T(cs.x0), T(cs.c0), T(cs.y)
    # encode
    E = H(plan.encode(x, c))
    E_ref = cs.op.encode(cs.x0, cs.c0)
    assert_close(E, E_ref, tol, coils=True, what="E")
    # exact adjoint (unweighted) on the measured data
    gx, gc = plan.adjoint(x, c, y)
    gx_ref, gc_ref = cs.op.adjoint(cs.x0, cs.c0, cs.y)
    assert_close(H(gx), gx_ref, tol, what="gx")
    assert_close(H(gc), gc_ref, tol, coils=True, what="gc")
    # loss and gradient in one call
    loss, gx, gc = plan.grad(x, c, y)
    f_ref, gx_ref, gc_ref = cs.op.loss_and_grad(cs.x0, cs.c0, cs.y, cs.w)
    assert abs(float(loss.item()) - f_ref) / f_ref <= tol
    assert_close(H(gx), gx_ref, tol, what="gx")
    assert_close(H(gc), gc_ref, tol, coils=True, what="gc")
    # the transfer pair (residual in the plan's layout), with a device scale, one output each
    t, loss_t = plan.forward_transfer(x, c, y)
    assert abs(float(loss_t.item()) - f_ref) / f_ref <= tol
    s = torch.full((1,), 0.5, dtype=torch.float32, device=DEV)
    gx, _ = plan.adjoint_transfer(x, c, t, alpha=2.0, scale=s, want_gc=False)
    _, gc = plan.adjoint_transfer(x, c, t, alpha=2.0, scale=s, want_gx=False)
    assert_close(H(gx), 0.5 * gx_ref, tol, what="gx transfer")
    assert_close(H(gc), 0.5 * gc_ref, tol, coils=True, what="gc transfer")
    # the sample-order residual and the plain adjoint give the same gradient
    r, _ = plan.forward_loss(x, c, y)
    gx, gc = plan.adjoint(x, c, r, alpha=2.0)
    assert_close(H(gx), gx_ref, tol, what="gx")
    assert_close(H(gc), gc_ref, tol, coils=True, what="gc")


@pytest.mark.parametrize("prec", ["fp32", "bf16_split"])
@pytest.mark.parametrize("name", ["dense2d_48x40_J5_K37", "tucker3d_24x20x18_r7x5x6_K13",
                                  "fused_48x32x20_r9x13x5_K23_J5"])
def test_autograd_data_fidelity(name, prec):
    """torch.autograd.Function: forward = loss (+ residual in the transfer layout), backward =
    adjoint with B c recomputed; without a wanted gradient forward gives the same loss."""
    from paper_2008_09042_amd.encoding import MaxwellDataFidelity, MaxwellEncode
    cs = get_case(name)
    plan = cs.plan(prec)
    tol = TOL[prec]
    x = T(cs.x0).requires_grad_(True)
    c = T(cs.c0).requires_grad_(True)
    f = MaxwellDataFidelity.apply(x, c, T(cs.y), plan)
    (3.0 * f).backward()
    f_ref, gx_ref, gc_ref = cs.op.loss_and_grad(cs.x0, cs.c0, cs.y, cs.w)
    assert abs(float(f.item()) - f_ref) / f_ref <= tol
    assert_close(H(x.grad), 3.0 * gx_ref, tol, what="x.grad")
    assert_close(H(c.grad), 3.0 * gc_ref, tol, coils=True, what="c.grad")
    with torch.no_grad():
        f0 = MaxwellDataFidelity.apply(T(cs.x0), T(cs.c0), T(cs.y), plan)
    assert abs(float(f0.item()) - f_ref) / f_ref <= tol
    # MaxwellEncode's VJP is J^H gy
    x2 = T(cs.x0).requires_grad_(True)
    c2 = T(cs.c0).requires_grad_(True)
    yhat = MaxwellEncode.apply(x2, c2, plan)
    gy = c64(np.random.default_rng(3).normal(size=yhat.shape) + 1j * np.random.default_rng(4).normal(size=yhat.shape))
    yhat.backward(T(gy))
    gx_ref, gc_ref = cs.op.adjoint(cs.x0, cs.c0, gy)
    assert_close(H(x2.grad), gx_ref, tol, what="x.grad")
    assert_close(H(c2.grad), gc_ref, tol, coils=True, what="c.grad")


def test_edge_single_coil_single_column():
    """J = 1, K = 1 with B = 1/sqrt(N): E = P F x exactly (up to FP32 rounding)."""
    from paper_2008_09042_amd.encoding import MaxwellPlan
    dims = (20, 12)
    N = 240
    B = np.full((N, 1), 1 / math.sqrt(N), dtype=complex)
    mask = np.sort(np.random.default_rng(1).choice(N, 77, replace=False))
    plan = MaxwellPlan(dims, 1, B=B, mask_idx=mask)
    x = c64(np.random.default_rng(2).normal(size=dims) + 1j)
    c = c64(np.array([[math.sqrt(N)]]))
    from oracle import Oracle
    ref = Oracle(dims, B=c64(B), mask_idx=mask).encode(x, c)
    assert_close(H(plan.encode(T(x), T(c))), ref, 1e-5, coils=True, what="E")


def test_edge_full_and_empty_mask():
    cs = Case(seed=107, dims=(16, 24), J=2, K=5, mask="full")
    plan = cs.plan()
    E = H(plan.encode(T(cs.x0), T(cs.c0)))
    assert_close(E, cs.op.encode(cs.x0, cs.c0), 1e-5, coils=True, what="E")
    ce = Case(seed=108, dims=(16, 24), J=2, K=5, mask="empty")
    plan = ce.plan()
    x, c = T(ce.x0), T(ce.c0)
    assert plan.encode(x, c).numel() == 0
    loss, gx, gc = plan.grad(x, c, T(np.zeros((2, 0))))
    assert float(loss.item()) == 0.0
    assert float(gx.abs().max().item()) == 0.0 and float(gc.abs().max().item()) == 0.0


@pytest.mark.parametrize("split", ["1000000", None])
@pytest.mark.parametrize("name", ["radial_32x24_J3_K9_7spokes", "radial_40x30_J2_K6_5spokes",
                                  "radial_256_J2_K20_64spokes", "radial_64x48_J12_K7_16spokes",
                                  "radial_40x36_J3_K6_sigma1.5_W4", "radial_64x48_J9_K5_sigma1.25_W5"])
def test_radial_spread_through_lds(name, split, monkeypatch):
    """The plain spread blocks stage their samples through LDS (MAXWELL_SPREAD_LDS, default 1)
    or walk them from memory (0).  Both add the same products in the same order per grid
    point, so the gradients agree bit for bit; the LDS form meets the oracle.  A split
    threshold of 1000000 sends the dense centre to the plain kernel too (long ranges over
    many staged chunks)."""
    if split is not None:
        monkeypatch.setenv("MAXWELL_SPREAD_SPLIT", split)
    cs = get_case(name)
    x, c, y = T(cs.x0), T(cs.c0), T(cs.y)
    out = {}
    for lds in ("1", "0"):
        monkeypatch.setenv("MAXWELL_SPREAD_LDS", lds)
        print(f"[case] {name} spread through LDS {lds}, split {split}", flush=True)
        out[lds] = cs.plan("fp32").adjoint(x, c, y)
    gx_ref, gc_ref = cs.op.adjoint(cs.x0, cs.c0, cs.y)
    assert_close(H(out["1"][0]), gx_ref, TOL["fp32"], what="gx")
    assert_close(H(out["1"][1]), gc_ref, TOL["fp32"], coils=True, what="gc")
    assert torch.equal(out["1"][0], out["0"][0]) and torch.equal(out["1"][1], out["0"][1])


@pytest.mark.parametrize("name", ["tucker3d_24x20x18_r7x5x6_K13", "fused_48x32x20_r9x13x5_K23_J5"])
def test_repeatable_bitwise(name):
    """No atomics anywhere: two runs give identical bits."""
    cs = get_case(name)
    plan = cs.plan()
    x, c, y = T(cs.x0), T(cs.c0), T(cs.y)
    a = plan.grad(x, c, y)
    b = plan.grad(x, c, y)
    for u, v in zip(a, b):
        assert torch.equal(u, v)


def test_radial_encode_close_to_exact_ndft():
    """With J = 1, K = 1 and B = 1/sqrt(N), c = sqrt(N), E is the KB NUFFT of x; it must
    match the plain non-uniform DFT within the NUFFT's approximation error (W = 6, sigma = 2)."""
    from paper_2008_09042_amd.encoding import MaxwellPlan
    from oracle import ndft
    from synth import golden_angle_radial
    dims = (48, 40)
    N = 48 * 40
    traj = golden_angle_radial(dims, 9, 96).astype(np.float32).astype(np.float64)
    B = np.full((N, 1), 1 / math.sqrt(N), dtype=complex)
    plan = MaxwellPlan(dims, 1, B=B, traj=traj)
    x = c64(np.random.default_rng(5).normal(size=dims) + 1j * np.random.default_rng(6).normal(size=dims))
    y = H(plan.encode(T(x), T(np.array([[math.sqrt(N)]]))))[0]
    assert rel(y, ndft(x, traj)) <= 1e-4


def test_radial_adjoint_identity_on_gpu():
    """<E_c z, y> = <z, E_c^H y> for the GPU operator itself (FP32 consistency)."""
    cs = get_case("radial_32x24_J3_K9_7spokes")
    plan = cs.plan()
    rng = np.random.default_rng(9)
    z = c64(rng.normal(size=cs.dims) + 1j * rng.normal(size=cs.dims))
    y = c64(rng.normal(size=(cs.J, cs.M)) + 1j * rng.normal(size=(cs.J, cs.M)))
    Ez = H(plan.encode(T(z), T(cs.c0)))
    gx, _ = plan.adjoint(T(cs.x0), T(cs.c0), T(y), want_gc=False)
    lhs = np.vdot(Ez.reshape(-1), y.reshape(-1))
    rhs = np.vdot(z.reshape(-1), H(gx).reshape(-1))
    assert abs(lhs - rhs) / abs(lhs) < 1e-5


@pytest.mark.parametrize("split", ["0", "1000000"])
@pytest.mark.parametrize("name", ["radial_32x24_J3_K9_7spokes", "radial_40x30_J2_K6_5spokes",
                                  "radial_256_J2_K20_64spokes", "radial_64x48_J12_K7_16spokes",
                                  "radial_40x36_J3_K6_sigma1.5_W4", "radial_64x48_J9_K5_sigma1.25_W5"])
def test_radial_spread_split_and_plain(name, split, monkeypatch):
    """The spread has a plain kernel and a split kernel for the blocks whose longest sample
    chain exceeds MAXWELL_SPREAD_SPLIT (read at plan creation; by default the dense centre of
    a radial trajectory).  Each alone must meet the oracle: "0" sends every block holding a
    sample to the split kernel, a large value sends none.  Both runs must also be repeatable
    bit for bit (fixed summation order)."""
    monkeypatch.setenv("MAXWELL_SPREAD_SPLIT", split)
    cs = get_case(name)
    print(f"[case] {name} spread split threshold {split}", flush=True)
    plan = cs.plan("fp32")
    x, c, y = T(cs.x0), T(cs.c0), T(cs.y)
    gx, gc = plan.adjoint(x, c, y)
    gx_ref, gc_ref = cs.op.adjoint(cs.x0, cs.c0, cs.y)
    assert_close(H(gx), gx_ref, TOL["fp32"], what="gx")
    assert_close(H(gc), gc_ref, TOL["fp32"], coils=True, what="gc")
    gx2, gc2 = plan.adjoint(x, c, y)
    assert torch.equal(gx, gx2) and torch.equal(gc, gc2)
