"""GPU parity at the batched-slices workload's own shapes (the bilinear operator of Sec. II-B,
Eq. (5), per slice), both precisions, against the FP64 oracle:

* Cartesian 192 x 320 (radix 3 and 5 axes), 32 coils, K = 256, variable-density Poisson-disc
  mask (R = 5, 32 x 32 centre);
* radial 320 x 192 on the 640 x 384 oversampled grid, 128 golden-angle spokes x 640 readout
  samples, 16 coils, K = 128, ramp weights;
* a batch of three slices (320 x 320 Cartesian, 32 coils, K = 256; the radial slice above;
  128 x 256 Cartesian, 8 coils, K = 64) through maxwell_batch_grad: each slice against the
  oracle and, bit for bit, against its own maxwell_grad call.

Bar on every output: relative L2 and per-coil max-abs / max|ref| <= 1e-5 (FP32), 1e-4
(BF16-split).
"""
import numpy as np
import pytest
import torch

from _common import TOL, Case, assert_close
from synth import plane_mask_to_indices, poisson_disc_plane, rng_for

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
_cache = {}


def pd_mask(seed, dims, R, centre):
    return plane_mask_to_indices(poisson_disc_plane(rng_for(seed, 4), dims, R, centre))


def case(name):
    if name not in _cache:
        if name == "cart_192x320_J32_K256":
            cs = Case(seed=301, dims=(192, 320), J=32, K=256, degree=10, kmax=5.0,
                      mask=pd_mask(301, (192, 320), 5.0, 32))
        elif name == "radial_320x192_J16_K128_128spokes":
            cs = Case(seed=302, dims=(320, 192), J=16, K=128, degree=10, kmax=5.0, mask="radial",
                      spokes=128, n_read=640, weights=True)
        elif name == "cart_320x320_J32_K256":
            cs = Case(seed=303, dims=(320, 320), J=32, K=256, degree=10, kmax=5.0,
                      mask=pd_mask(303, (320, 320), 4.0, 32))
        elif name == "cart_128x256_J8_K64":
            cs = Case(seed=304, dims=(128, 256), J=8, K=64, degree=10, kmax=5.0,
                      mask=pd_mask(304, (128, 256), 7.0, 25), weights=True)
        else:
            raise KeyError(name)
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


def ref(cs):
    key = ("ref", id(cs))
    if key not in _cache:
        E = cs.op.encode(cs.x0, cs.c0)
        ad = cs.op.adjoint(cs.x0, cs.c0, cs.y)
        lg = cs.op.loss_and_grad(cs.x0, cs.c0, cs.y, cs.w)
        _cache[key] = (E, ad, lg)
    return _cache[key]


@pytest.mark.parametrize("prec", ["fp32", "bf16_split"])
@pytest.mark.parametrize("name", ["cart_192x320_J32_K256", "radial_320x192_J16_K128_128spokes"])
def test_slice_shapes_against_oracle(name, prec):
    print(f"[case] {name} {prec}", flush=True)
    cs = case(name)
    plan = cs.plan(prec)
    tol = TOL[prec]
    E_ref, (gxa_ref, gca_ref), (f_ref, gx_ref, gc_ref) = ref(cs)
    x, c, y = T(cs.x0), T(cs.c0), T(cs.y)
    assert_close(H(plan.encode(x, c)), E_ref, tol, coils=True, what="E")
    gx, gc = plan.adjoint(x, c, y)
    assert_close(H(gx), gxa_ref, tol, what="adjoint gx")
    assert_close(H(gc), gca_ref, tol, coils=True, what="adjoint gc")
    loss, gx, gc = plan.grad(x, c, y)
    assert abs(float(loss.item()) - f_ref) / f_ref <= tol
    assert_close(H(gx), gx_ref, tol, what="gx")
    assert_close(H(gc), gc_ref, tol, coils=True, what="gc")


@pytest.mark.parametrize("prec", ["fp32", "bf16_split"])
def test_batch_with_320_slice(prec):
    from paper_2008_09042_amd.encoding import MaxwellBatch
    print(f"[case] batch 320x320 / radial 320x192 / 128x256 {prec}", flush=True)
    names = ["cart_320x320_J32_K256", "radial_320x192_J16_K128_128spokes", "cart_128x256_J8_K64"]
    css = [case(n) for n in names]
    plans = [cs.plan(prec) for cs in css]
    batch = MaxwellBatch(plans, branches=2)
    xs = [T(cs.x0) for cs in css]
    cs_ = [T(cs.c0) for cs in css]
    ys = [T(cs.y) for cs in css]
    loss, gx, gc = batch.grad(xs, cs_, ys)
    torch.cuda.synchronize()
    tol = TOL[prec]
    for i, (n, cs, plan) in enumerate(zip(names, css, plans)):
        _, _, (f_ref, gx_ref, gc_ref) = ref(cs)
        print(f"[case]   slice {n}", flush=True)
        assert abs(float(loss[i]) - f_ref) / f_ref <= tol
        assert_close(H(gx[i]), gx_ref, tol, what=f"{n} gx")
        assert_close(H(gc[i]), gc_ref, tol, coils=True, what=f"{n} gc")
        l1, gx1, gc1 = plan.grad(xs[i], cs_[i], ys[i])
        assert torch.equal(l1, loss[i]) and torch.equal(gx1, gx[i]) and torch.equal(gc1, gc[i]), n
