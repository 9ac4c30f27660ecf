"""GPU parity of the Gauss-Newton step (maxwell_jvp, maxwell_normal, maxwell_cg) and of the
multi-map operator (maxwell_multi_encode, maxwell_multi_grad) against the FP64 oracle
(oracle.solver, oracle.encoding) on the same seeded, complex64-rounded inputs.

* JVP and normal operator: one operator application each, so the operator bar applies
  (relative L2, FP32 <= 1e-5, BF16-split <= 1e-4).
* CG: five steps.  Each step applies the normal operator once and feeds two FP64 inner
  products into the next step's coefficients, so an operator error delta perturbs the
  iterate by about (steps x condition) delta; with the shift lambda set to a fifth of the
  operator's Rayleigh quotient the bar is ten times the operator bar (FP32 1e-4,
  BF16-split 1e-3) for the iterate and for every <r_k, r_k> relative to <r_0, r_0>.
* <r_0, r_0> = <b, b> is an FP64 sum of the same FP32 values: 1e-12.
* Determinism (two calls, bit for bit) and a captured graph replayed twice, each replay equal
  to the eager call bit for bit.
Cases: dense 2D with weights, Tucker 3D general path, the fused 3D path, radial with ramp
weights.
"""
import ctypes

import numpy as np
import pytest
import torch

from _common import TOL, Case, assert_close, c64, maxrel, rel
from oracle.solver import gn_cg, inner, normal

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
CASES = {
    "dense2d_48x40_J5_K37_w": dict(seed=201, dims=(48, 40), J=5, K=37, basis="dense", weights=True),
    "tucker3d_24x20x18_J3_K13": dict(seed=202, dims=(24, 20, 18), ranks=(7, 5, 6), J=3, K=13, basis="tucker",
                                     mask="lines3d", frac=0.3),
    "fused_48x32x20_J5_K23_w": dict(seed=203, dims=(48, 32, 20), ranks=(9, 13, 5), J=5, K=23, basis="tucker",
                                    mask="lines3d", frac=0.3, weights=True),
    "radial_32x24_J3_K9_w": dict(seed=204, dims=(32, 24), J=3, K=9, mask="radial", spokes=7, weights=True),
}
ITERS = 5
_cache = {}


def get_case(name):
    if name not in _cache:
        cs = Case(**CASES[name])
        rng = np.random.default_rng(99)
        cs.dx = c64(0.3 * (rng.normal(size=cs.dims) + 1j * rng.normal(size=cs.dims)))
        cs.dc = c64(rng.normal(size=(cs.J, cs.K)) + 1j * rng.normal(size=(cs.J, cs.K)))
        # shift: a fifth of the Rayleigh quotient of J^H W J on the (dx, dc) direction
        gx, gc = normal(cs.op, cs.x0, cs.c0, cs.dx, cs.dc, 0.0, 0.0, cs.w)
        q = inner((gx, gc), (cs.dx.reshape(-1), cs.dc)) / inner((cs.dx.reshape(-1), cs.dc), (cs.dx.reshape(-1), cs.dc))
        cs.lam = (float(np.float32(0.2 * q)), float(np.float32(0.3 * q)))
        cs.bx = c64(rng.normal(size=cs.dims) + 1j * rng.normal(size=cs.dims))
        cs.bc = c64(rng.normal(size=(cs.J, cs.K)) + 1j * rng.normal(size=(cs.J, cs.K)))
        _cache[name] = cs
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
def test_jvp_and_normal(name, prec):
    cs = get_case(name)
    print(f"[case] {name} {prec} jvp/normal", flush=True)
    plan = cs.plan(prec)
    x, c, dx, dc = T(cs.x0), T(cs.c0), T(cs.dx), T(cs.dc)
    y = H(plan.jvp(x, c, dx, dc))
    assert_close(y, cs.op.jvp(cs.x0, cs.c0, cs.dx, cs.dc), TOL[prec], coils=True, what="jvp")
    ox, oc = plan.normal(x, c, dx, dc, *cs.lam)
    rx, rc = normal(cs.op, cs.x0, cs.c0, cs.dx, cs.dc, cs.lam[0], cs.lam[1], cs.w)
    assert_close(H(ox), rx, TOL[prec], what="normal x")
    assert_close(H(oc), rc, TOL[prec], coils=True, what="normal c")


@pytest.mark.parametrize("prec", ["fp32", "bf16_split"])
@pytest.mark.parametrize("name", list(CASES))
def test_cg(name, prec):
    cs = get_case(name)
    print(f"[case] {name} {prec} cg x{ITERS}", flush=True)
    plan = cs.plan(prec)
    x, c, bx, bc = T(cs.x0), T(cs.c0), T(cs.bx), T(cs.bc)
    dx, dc, rr = plan.cg(x, c, bx, bc, *cs.lam, ITERS)
    torch.cuda.synchronize()
    rx, rc, rr_ref = gn_cg(cs.op, cs.x0, cs.c0, cs.bx, cs.bc, cs.lam[0], cs.lam[1], ITERS, cs.w)
    bar = 10 * TOL[prec]
    errs = (rel(H(dx), rx), rel(H(dc), rc), maxrel(H(dx), rx), maxrel(H(dc), rc, coils=True))
    rr = rr.cpu().numpy()
    print(f"[case] iterate errors {errs}, rr {rr}, rr_ref {rr_ref}", flush=True)
    assert max(errs) <= bar
    assert abs(rr[0] - rr_ref[0]) <= 1e-12 * rr_ref[0]
    assert np.max(np.abs(rr - rr_ref)) <= bar * rr_ref[0]
    # bitwise repeatable
    dx2, dc2, rr2 = plan.cg(x, c, bx, bc, *cs.lam, ITERS)
    assert torch.equal(dx, dx2) and torch.equal(dc, dc2) and torch.equal(rr2, torch.from_numpy(rr).to(DEV))


def test_cg_graph_replays():
    from paper_2008_09042_amd import _lib as L
    from paper_2008_09042_amd.encoding import _ptr
    cs = get_case("dense2d_48x40_J5_K37_w")
    print("[case] cg graph capture and replays", flush=True)
    plan = cs.plan("bf16_split")
    x, c, bx, bc = T(cs.x0), T(cs.c0), T(cs.bx), T(cs.bc)
    ref = plan.cg(x, c, bx, bc, *cs.lam, ITERS)
    dx = torch.empty_like(ref[0])
    dc = torch.empty_like(ref[1])
    rr = torch.empty_like(ref[2])
    ws, nb = plan._wsargs()

    def call():
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        L.check(plan.lib.maxwell_cg(plan.handle, _ptr(x), _ptr(c), _ptr(bx), _ptr(bc), cs.lam[0], cs.lam[1],
                                    ITERS, _ptr(dx), _ptr(dc), _ptr(rr), ws, nb, stream))

    side = torch.cuda.Stream(device=DEV)
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        call()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    for k in range(2):
        dx.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(dx, ref[0]) and torch.equal(dc, ref[1]) and torch.equal(rr, ref[2]), f"replay {k}"
        again = plan.cg(x, c, bx, bc, *cs.lam, ITERS)  # eager work between replays
        assert torch.equal(again[0], ref[0])


@pytest.mark.parametrize("prec", ["fp32", "bf16_split"])
@pytest.mark.parametrize("name", list(CASES))
def test_multi_map(name, prec):
    """Two map sets (extra bilinear terms): encode, loss and every map set's gradient at the
    operator bar; one map set equals maxwell_grad bit for bit."""
    from oracle.encoding import multi_encode, multi_loss_and_grad
    cs = get_case(name)
    print(f"[case] {name} {prec} multi-map", flush=True)
    plan = cs.plan(prec)
    rng = np.random.default_rng(17)
    x2 = c64(0.5 * (rng.normal(size=cs.dims) + 1j * rng.normal(size=cs.dims)))
    c2 = c64(rng.normal(size=(cs.J, cs.K)) + 1j * rng.normal(size=(cs.J, cs.K)))
    xs = T(np.stack([cs.x0, x2]))
    cc = T(np.stack([cs.c0, c2]))
    y = T(cs.y)
    E = H(plan.multi_encode(xs, cc))
    assert_close(E, multi_encode(cs.op, [cs.x0, x2], [cs.c0, c2]), TOL[prec], coils=True, what="multi E")
    loss, gx, gc = plan.multi_grad(xs, cc, y)
    f_ref, gx_ref, gc_ref = multi_loss_and_grad(cs.op, [cs.x0, x2], [cs.c0, c2], cs.y, cs.w)
    assert abs(float(loss.item()) - f_ref) / f_ref <= TOL[prec]
    for i in range(2):
        assert_close(H(gx[i]), gx_ref[i], TOL[prec], what=f"gx[{i}]")
        assert_close(H(gc[i]), gc_ref[i], TOL[prec], coils=True, what=f"gc[{i}]")
    # a single map set: the same loss and gradient as the plain call (to the operator bar;
    # the multi-map residual goes through the sample-order path)
    l1, gx1, gc1 = plan.multi_grad(xs[:1].contiguous(), cc[:1].contiguous(), y)
    l0, gx0, gc0 = plan.grad(T(cs.x0), T(cs.c0), y)
    assert abs(float(l1.item()) - float(l0.item())) <= TOL[prec] * float(l0.item())
    assert rel(H(gx1[0]), H(gx0)) <= TOL[prec] and rel(H(gc1[0]), H(gc0)) <= TOL[prec]
