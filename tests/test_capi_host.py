"""Host-side tests of the C ABI (no GPU needed).

The library must load on a GPU-less host, export every entry point the public
header declares, and reject invalid requests with a status and a message
before touching the HIP runtime.  Only invalid descriptors are passed here, so
no device memory is ever touched.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2008_09042_amd._lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "maxwell.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_2008_09042_amd.build import build
        build()
    return L.load()


def header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(maxwell_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_function(lib):
    declared = header_functions()
    assert len(declared) >= 12
    missing = [f for f in declared if not hasattr(lib, f)]
    assert not missing, missing
    assert sorted(L.EXPORTS) == declared


def test_version_string(lib):
    assert lib.maxwell_version().decode().startswith("maxwell-gfx950")


FAKE = 0x10000  # aligned, never dereferenced: every descriptor below fails validation first


def dense_basis(K=4):
    b = L.BasisDesc()
    b.kind = L.MAXWELL_BASIS_DENSE
    b.K = K
    b.dense = FAKE
    return b


def tucker_basis(r=(2, 2, 2), K=3):
    b = L.BasisDesc()
    b.kind = L.MAXWELL_BASIS_TUCKER
    b.K = K
    for m in range(3):
        b.r[m] = r[m]
        b.U[m] = FAKE
    b.core = FAKE
    return b


def cart_desc(dims=(8, 6), J=2, mask=None, weights=None):
    d = L.PlanDesc()
    d.ndim = len(dims)
    for i, n in enumerate(dims):
        d.n[i] = n
    d.J = J
    d.precision = L.MAXWELL_FP32
    d.sampling = L.MAXWELL_CARTESIAN
    m = np.arange(5, dtype=np.int64) if mask is None else np.asarray(mask, dtype=np.int64)
    d._keep = [m]
    d.M = m.size
    d.mask_idx = m.ctypes.data if m.size else None
    if weights is not None:
        w = np.asarray(weights, dtype=np.float32)
        d._keep.append(w)
        d.weights = w.ctypes.data
    return d


def radial_desc(dims=(8, 8), traj=None, width=6, oversamp=2.0):
    d = L.PlanDesc()
    d.ndim = len(dims)
    for i, n in enumerate(dims):
        d.n[i] = n
    d.J = 1
    d.sampling = L.MAXWELL_NONCARTESIAN
    t = np.zeros((3, len(dims)), dtype=np.float32) if traj is None else np.asarray(traj, dtype=np.float32)
    d._keep = [t]
    d.M = t.shape[0]
    d.traj = t.ctypes.data
    d.kb_width = width
    d.oversamp = oversamp
    d.kb_beta = 0.0
    return d


def create(lib, desc, basis):
    h = ctypes.c_void_p()
    st = lib.maxwell_plan_create(ctypes.byref(desc) if desc is not None else None,
                                 ctypes.byref(basis) if basis is not None else None, ctypes.byref(h))
    return st, h, lib.maxwell_last_error().decode()


@pytest.mark.parametrize("mutate,status,needle", [
    (lambda d, b: setattr(d, "ndim", 4), L.MAXWELL_ERR_INVALID_ARGUMENT, "ndim"),
    (lambda d, b: d.n.__setitem__(0, 7), L.MAXWELL_ERR_UNSUPPORTED, "odd"),
    (lambda d, b: d.n.__setitem__(0, 14), L.MAXWELL_ERR_UNSUPPORTED, "factor"),
    (lambda d, b: d.n.__setitem__(1, 8192), L.MAXWELL_ERR_INVALID_ARGUMENT, "4096"),
    (lambda d, b: setattr(d, "J", 0), L.MAXWELL_ERR_INVALID_ARGUMENT, "J must"),
    (lambda d, b: setattr(b, "K", 0), L.MAXWELL_ERR_INVALID_ARGUMENT, "K must"),
    (lambda d, b: setattr(b, "dense", None), L.MAXWELL_ERR_INVALID_ARGUMENT, "dense basis"),
    (lambda d, b: setattr(b, "dense", FAKE + 4), L.MAXWELL_ERR_INVALID_ARGUMENT, "misaligned"),
    (lambda d, b: setattr(d, "precision", 7), L.MAXWELL_ERR_INVALID_ARGUMENT, "precision"),
    (lambda d, b: setattr(b, "kind", 5), L.MAXWELL_ERR_INVALID_ARGUMENT, "basis kind"),
    (lambda d, b: setattr(d, "sampling", 9), L.MAXWELL_ERR_INVALID_ARGUMENT, "sampling"),
])
def test_plan_create_rejects(lib, mutate, status, needle):
    d, b = cart_desc(), dense_basis()
    mutate(d, b)
    st, h, msg = create(lib, d, b)
    assert st == status and not h.value
    assert needle in msg


@pytest.mark.parametrize("mask,needle", [
    ([3, 1, 2], "ascending"),
    ([1, 1, 2], "ascending"),
    ([0, 5, 48], "out of range"),
    ([-1, 2], "out of range"),
    (list(range(49)), "more mask samples"),
])
def test_bad_masks(lib, mask, needle):
    st, h, msg = create(lib, cart_desc(mask=mask), dense_basis())
    assert st == L.MAXWELL_ERR_INVALID_ARGUMENT and needle in msg


def test_bad_weights(lib):
    for w in ([1, -1, 0, 0, 0], [1, float("nan"), 0, 0, 0]):
        st, h, msg = create(lib, cart_desc(weights=w), dense_basis())
        assert st == L.MAXWELL_ERR_INVALID_ARGUMENT and "weights" in msg


def test_tucker_validation(lib):
    st, _, msg = create(lib, cart_desc(dims=(8, 6)), tucker_basis())
    assert st == L.MAXWELL_ERR_UNSUPPORTED and "3D" in msg
    st, _, msg = create(lib, cart_desc(dims=(8, 6, 4)), tucker_basis(r=(2, 9, 2)))
    assert st == L.MAXWELL_ERR_INVALID_ARGUMENT and "rank" in msg
    b = tucker_basis()
    b.core = None
    st, _, msg = create(lib, cart_desc(dims=(8, 6, 4)), b)
    assert st == L.MAXWELL_ERR_INVALID_ARGUMENT and "core" in msg


def test_radial_validation(lib):
    st, _, msg = create(lib, radial_desc(dims=(8, 8, 8)), dense_basis())
    assert st == L.MAXWELL_ERR_UNSUPPORTED and "2D" in msg
    st, _, msg = create(lib, radial_desc(traj=[[0.0, 4.0]]), dense_basis())  # k = n/2 is outside [-n/2, n/2)
    assert st == L.MAXWELL_ERR_INVALID_ARGUMENT and "trajectory" in msg
    st, _, msg = create(lib, radial_desc(traj=[[0.0, float("nan")]]), dense_basis())
    assert st == L.MAXWELL_ERR_INVALID_ARGUMENT and "trajectory" in msg
    st, _, msg = create(lib, radial_desc(width=9), dense_basis())
    assert st == L.MAXWELL_ERR_INVALID_ARGUMENT and "kb_width" in msg
    st, _, msg = create(lib, radial_desc(oversamp=1.3), dense_basis())  # 1.3 * 8 is not an even integer
    assert st == L.MAXWELL_ERR_INVALID_ARGUMENT and "oversamp" in msg


def test_null_arguments(lib):
    st, _, _ = create(lib, None, dense_basis())
    assert st == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert lib.maxwell_plan_create(None, None, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    sz = ctypes.c_size_t()
    assert lib.maxwell_plan_workspace_size(None, ctypes.byref(sz)) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert lib.maxwell_plan_path(None) is None
    lib.maxwell_plan_destroy(None)  # no-op
    z = ctypes.c_void_p(FAKE)
    assert lib.maxwell_encode(None, z, z, z, None, 0, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert lib.maxwell_grad(None, z, z, z, z, z, None, None, 0, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert lib.maxwell_adjoint(None, z, z, z, 1.0, None, z, z, None, 0, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert lib.maxwell_forward_loss(None, z, z, z, z, None, None, 0, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert lib.maxwell_forward_transfer(None, z, z, z, z, None, None, 0, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    out = ctypes.c_void_p()
    assert lib.maxwell_batch_create(None, 1, 0, ctypes.byref(out)) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert lib.maxwell_batch_create(None, 1, 0, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    arr = (ctypes.c_void_p * 1)(None)
    assert lib.maxwell_batch_create(arr, 1, 0, ctypes.byref(out)) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert "null" in lib.maxwell_last_error().decode()
    assert lib.maxwell_batch_create(arr, 1, 17, ctypes.byref(out)) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert lib.maxwell_batch_workspace_size(None, ctypes.byref(sz)) == L.MAXWELL_ERR_INVALID_ARGUMENT
    pz = (ctypes.c_void_p * 1)(FAKE)
    assert (lib.maxwell_batch_grad(None, pz, pz, pz, None, None, None, None, 0, None)
            == L.MAXWELL_ERR_INVALID_ARGUMENT)
    assert (lib.maxwell_batch_grad_shared(None, pz, z, pz, None, None, None, None, 0, None)
            == L.MAXWELL_ERR_INVALID_ARGUMENT)
    lib.maxwell_batch_destroy(None)  # no-op
    assert (lib.maxwell_adjoint_transfer(None, z, z, z, 1.0, None, z, z, None, 0, None)
            == L.MAXWELL_ERR_INVALID_ARGUMENT)
    assert lib.maxwell_basis_apply(None, z, z, None, 0, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert lib.maxwell_basis_apply_adjoint(None, z, z, None, 0, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert lib.maxwell_jvp(None, z, z, z, z, z, None, 0, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert lib.maxwell_normal(None, z, z, z, z, 0.1, 0.1, z, z, None, 0, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert (lib.maxwell_cg(None, z, z, z, z, 0.1, 0.1, 3, z, z, None, None, 0, None)
            == L.MAXWELL_ERR_INVALID_ARGUMENT)
    for f in ("maxwell_sense_encode", "maxwell_sense_adjoint", "maxwell_sense_normal"):
        assert getattr(lib, f)(None, z, z, z, None, 0, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert lib.maxwell_tv_prox(None, z, 0.1, 5, z, None, 0, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert lib.maxwell_ball_project(None, z, z, z, z, None, 0, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert (lib.maxwell_sense_admm(None, z, z, z, 1.0, 3, 3, 3, z, None, None, 0, None)
            == L.MAXWELL_ERR_INVALID_ARGUMENT)
    assert lib.maxwell_multi_encode(None, 2, z, z, z, None, 0, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert lib.maxwell_multi_grad(None, 2, z, z, z, z, z, None, None, 0, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    r3 = (ctypes.c_int64 * 3)()
    d3 = (ctypes.c_int64 * 3)(4, 4, 4)
    assert lib.maxwell_tucker_compress(None, 2, z, 0.1, z, z, z, z, r3, None, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert lib.maxwell_tucker_compress(d3, 2, z, 1.5, z, z, z, z, r3, None, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert "eps" in lib.maxwell_last_error().decode()
    assert lib.maxwell_tucker_compress(d3, 0, z, 0.1, z, z, z, z, r3, None, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert lib.maxwell_plan_set_timing(None, 1) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert "plan is null" in lib.maxwell_last_error().decode()


def test_missing_library_fails_loudly():
    saved = L._lib
    try:
        L._lib = None
        with pytest.raises(RuntimeError, match="missing"):
            L.load("/nonexistent/libmaxwell.so")
    finally:
        L._lib = saved


def test_plan_needs_a_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_2008_09042_amd.encoding import MaxwellPlan
    with pytest.raises(RuntimeError, match="GPU"):
        MaxwellPlan((8, 8), 1, B=np.ones((64, 1)), mask_idx=np.arange(4))


def test_bf16_split_validation(lib):
    """maxwell_bf16_split checks its arguments on the host before any HIP call."""
    import ctypes
    fake = ctypes.c_void_p(0x10000)
    other = ctypes.c_void_p(0x20000)
    third = ctypes.c_void_p(0x30000)
    assert lib.maxwell_bf16_split(None, 0, 0, None, None, None) == L.MAXWELL_OK
    assert lib.maxwell_bf16_split(None, 8, 0, other, third, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert lib.maxwell_bf16_split(fake, 7, 1, other, third, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert "even" in lib.maxwell_last_error().decode()
    assert lib.maxwell_bf16_split(fake, 8, 3, other, third, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert lib.maxwell_bf16_split(fake, -1, 0, other, third, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    # hi overlapping x
    assert lib.maxwell_bf16_split(fake, 1 << 20, 0, ctypes.c_void_p(0x10000 + 64), third, None) == \
        L.MAXWELL_ERR_INVALID_ARGUMENT
    assert "overlap" in lib.maxwell_last_error().decode()


def test_grad_static_validation(lib):
    """maxwell_grad_static refuses a null plan before any HIP call."""
    assert lib.maxwell_grad_static(None, None, None, None, None, None, None, None) == L.MAXWELL_ERR_INVALID_ARGUMENT
    assert "plan is null" in lib.maxwell_last_error().decode()
