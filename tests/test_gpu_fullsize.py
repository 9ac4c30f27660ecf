"""GPU parity at the full sizes of the four single-GPU workloads (2D Cartesian 64^2 and
256^2 with dense bases, 2D radial 256^2, 3D Cartesian 128^3 with a Tucker basis), in the
launch configuration the benchmark times: the autograd data-fidelity function, forward
loss then backward (B c recomputed), against the FP64 oracle on the same complex64 inputs.

Bar: FP32 <= 1e-5 and BF16-split <= 1e-4 relative (L2 over the whole gradient; loss
relative).  The 256^2 Cartesian case also checks the GPU gradient against a central finite
difference of the GPU loss along a random direction (h = 1e-3).
"""
import numpy as np
import pytest
import torch

from _common import TOL, assert_close, c64, maxrel, rel
from oracle import Oracle
from synth import problem as make

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
_cache = {}


def T(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(np.complex64))).to(DEV)


def H(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def problem(name):
    """Seeded full-size problem, complex64-rounded, with its oracle and measured data."""
    if name not in _cache:
        p = make(name)
        kw = dict(mask_idx=p.mask_idx)
        if p.sampling == "radial":
            p.traj = p.traj.astype(np.float32).astype(np.float64)
            kw = dict(traj=p.traj)
        w = None if p.weights is None else p.weights.astype(np.float32).astype(np.float64)
        if p.basis_kind == "dense":
            basis = dict(B=c64(p.B))
        else:
            basis = dict(U=[c64(u) for u in p.U], core=c64(p.core))
        op = Oracle(p.dims, **basis, **kw)
        y = op.encode(c64(p.x_true), c64(p.c_true))
        y = c64(y + 10 ** (-p.snr_db / 20) * np.linalg.norm(y) / np.linalg.norm(p.noise) * p.noise)
        _cache[name] = (p, basis, kw, w, op, y)
    return _cache[name]


def gpu_grad(name, prec):
    from paper_2008_09042_amd.encoding import MaxwellDataFidelity, MaxwellPlan
    p, basis, kw, w, op, y = problem(name)
    gbasis = {k: ([T(u) for u in v] if isinstance(v, list) else T(v)) for k, v in basis.items()}
    plan = MaxwellPlan(p.dims, p.J, **gbasis, **kw, weights=w, precision=prec, device=DEV)
    x = T(p.x0).requires_grad_(True)
    c = T(p.c0).requires_grad_(True)
    f = MaxwellDataFidelity.apply(x, c, T(y), plan)
    f.backward()
    torch.cuda.synchronize()
    return plan, float(f.item()), H(x.grad), H(c.grad)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible ROCm GPU"
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["fp32", "bf16_split"])
@pytest.mark.parametrize("name", ["cart2d_64_dense32_j8", "cart2d_256_dense200_j32", "radial2d_256_dense128_j16",
                                  "cart3d_128_tucker40x300_j32"])
def test_fullsize_gradient(name, prec):
    print(f"[case] {name} {prec}", flush=True)
    p, basis, kw, w, op, y = problem(name)
    plan, f, gx, gc = gpu_grad(name, prec)
    if p.basis_kind == "tucker":
        assert plan.path == "fused-tucker-lines"
    key = ("ref", name)
    if key not in _cache:
        _cache[key] = op.loss_and_grad(c64(p.x0), c64(p.c0), y, w)
    f_ref, gx_ref, gc_ref = _cache[key]
    errs = (abs(f - f_ref) / f_ref, rel(gx, gx_ref), rel(gc, gc_ref), maxrel(gx, gx_ref), maxrel(gc, gc_ref, coils=True))
    print(f"[case] {name} {prec}: loss {errs[0]:.2e} gx {errs[1]:.2e} gc {errs[2]:.2e} "
          f"max-abs gx {errs[3]:.2e} gc (per coil) {errs[4]:.2e}", flush=True)
    assert max(errs) <= TOL[prec], errs


def test_fullsize_directional_derivative():
    """GPU gradient vs a central difference of the GPU loss (256^2 Cartesian, FP32)."""
    from paper_2008_09042_amd.encoding import MaxwellDataFidelity
    name = "cart2d_256_dense200_j32"
    p, basis, kw, w, op, y = problem(name)
    plan, f0, gx, gc = gpu_grad(name, "fp32")
    rng = np.random.default_rng(11)
    dx = rng.normal(size=p.x0.shape) + 1j * rng.normal(size=p.x0.shape)
    dc = rng.normal(size=p.c0.shape) + 1j * rng.normal(size=p.c0.shape)
    dx *= np.linalg.norm(p.x0) / np.linalg.norm(dx)
    dc *= np.linalg.norm(p.c0) / np.linalg.norm(dc)
    h = 1e-3

    def loss(s):
        with torch.no_grad():
            return float(MaxwellDataFidelity.apply(T(p.x0 + s * dx), T(p.c0 + s * dc), T(y), plan).item())

    fd = (loss(h) - loss(-h)) / (2 * h)
    # the gradient is the conjugate (Wirtinger) gradient scaled by 2: df = Re<g, d>
    an = float(np.real(np.vdot(gx, dx) + np.vdot(gc, dc)))
    print(f"[case] directional derivative: fd {fd:.6e} analytic {an:.6e}", flush=True)
    assert abs(fd - an) / abs(an) <= 1e-3
