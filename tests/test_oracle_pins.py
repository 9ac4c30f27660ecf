"""Pins for the FP64 oracle: brute force, closed forms, invariants, special cases.

None of these re-types the oracle's own formula.  Each checks the oracle
against something fixed independently: a DFT matrix built from its
definition, a hand-written fixture, a different library route, a
mathematical identity of the paper's operator, or finite differences.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import quad

import oracle
from oracle import Oracle
from synth import (coefficients, complex_normal, golden_angle_radial, phantom, problem,
                   rng_for, smooth_dense_basis, tucker_basis, ramp_dcf)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def brute_dft_matrix(n):
    """Centred DFT matrix from the definition: F[k, r] = n^-1/2 exp(-2 pi i k r / n)."""
    k = np.arange(n) - n // 2
    return np.exp(-2j * math.pi * np.outer(k, k) / n) / math.sqrt(n)


def brute_dft(a):
    """Apply the brute-force matrix along every axis."""
    out = np.asarray(a, dtype=np.complex128)
    for ax, n in enumerate(out.shape):
        out = np.moveaxis(np.tensordot(brute_dft_matrix(n), out, axes=(1, ax)), 0, ax)
    return out


# ---------------------------------------------------------------- P1: the DFT
@pytest.mark.parametrize("shape", [(4, 6), (8, 8), (6, 10), (12, 20), (4, 4, 6), (2, 8)])
def test_dft_matches_brute_force(shape):
    rng = np.random.default_rng(1)
    a = complex_normal(rng, shape)
    axes = tuple(range(len(shape)))
    assert rel(oracle.centred_dft(a, axes), brute_dft(a)) < 1e-13
    # inverse is the conjugate-transposed matrix
    b = complex_normal(rng, shape)
    inv = np.asarray(b)
    for ax, n in enumerate(shape):
        inv = np.moveaxis(np.tensordot(brute_dft_matrix(n).conj().T, inv, axes=(1, ax)), 0, ax)
    assert rel(oracle.centred_idft(b, axes), inv) < 1e-13


def test_dft_golden_n4():
    g = json.load(open(os.path.join(GOLDEN, "dft_n4_centred.json")))
    F = np.array(g["re"]) + 1j * np.array(g["im"])
    cols = np.stack([oracle.centred_dft(np.eye(4)[:, r], (0,)) for r in range(4)], axis=1)
    assert np.max(np.abs(cols - F)) < 1e-15


def test_dft_closed_forms():
    n0, n1 = 8, 6
    # delta at centred pixel (r0, r1) -> N^-1/2 exp(-2 pi i (k0 r0/n0 + k1 r1/n1))
    r0, r1 = 3, -2
    a = np.zeros((n0, n1), dtype=complex)
    a[r0 + n0 // 2, r1 + n1 // 2] = 1.0
    k0 = (np.arange(n0) - n0 // 2)[:, None]
    k1 = (np.arange(n1) - n1 // 2)[None, :]
    expect = np.exp(-2j * math.pi * (k0 * r0 / n0 + k1 * r1 / n1)) / math.sqrt(n0 * n1)
    assert np.max(np.abs(oracle.centred_dft(a, (0, 1)) - expect)) < 1e-15
    # constant image -> sqrt(N) at k = 0 (array centre), zero elsewhere
    c = oracle.centred_dft(np.ones((n0, n1)), (0, 1))
    e = np.zeros((n0, n1), dtype=complex)
    e[n0 // 2, n1 // 2] = math.sqrt(n0 * n1)
    assert np.max(np.abs(c - e)) < 1e-13


@pytest.mark.parametrize("shape", [(64, 64), (16, 12, 10), (30, 20)])
def test_dft_parseval_and_modulation_route(shape):
    """Unitary: Parseval and inverse.  Also equal to scipy's FFT with the
    chessboard modulation (-1)^r on input and (-1)^k on output and the
    global sign prod_d (-1)^(n_d/2), which needs no shifts."""
    rng = np.random.default_rng(2)
    a = complex_normal(rng, shape)
    axes = tuple(range(len(shape)))
    fa = oracle.centred_dft(a, axes)
    assert abs(np.linalg.norm(fa) - np.linalg.norm(a)) / np.linalg.norm(a) < 1e-14
    assert rel(oracle.centred_idft(fa, axes), a) < 1e-14
    chess = np.ones(shape)
    for ax, n in enumerate(shape):
        s = [1] * len(shape)
        s[ax] = n
        chess = chess * ((-1.0) ** np.arange(n)).reshape(s)
    sign = np.prod([(-1.0) ** (n // 2) for n in shape])
    alt = sign * chess * np.fft.fftn(chess * a, norm="ortho")  # NumPy: a library the oracle does not use
    assert rel(fa, alt) < 1e-13


# ---------------------------------------------------------------- P3: Tucker
def test_mode_product_golden():
    g = json.load(open(os.path.join(GOLDEN, "mode_product_2x2.json")))
    A = np.array(g["A"]).reshape(2, 1, 1)
    U = np.array(g["U"])
    C = oracle.mode_product(A, U, 0).reshape(-1)
    assert np.array_equal(C, np.array(g["C"]))


def test_mode_product_matches_einsum_each_mode():
    rng = np.random.default_rng(3)
    A = complex_normal(rng, (3, 4, 5))
    U = [complex_normal(rng, (6, 3)), complex_normal(rng, (7, 4)), complex_normal(rng, (2, 5))]
    assert rel(oracle.mode_product(A, U[0], 0), np.einsum("pjk,ip->ijk", A, U[0])) < 1e-14
    assert rel(oracle.mode_product(A, U[1], 1), np.einsum("ipk,jp->ijk", A, U[1])) < 1e-14
    assert rel(oracle.mode_product(A, U[2], 2), np.einsum("ijp,kp->ijk", A, U[2])) < 1e-14


def test_tucker_equals_dense():
    """Materialise B from (core, U) by a direct 4-index sum and compare the
    coil maps and the adjoint, on a non-cubic shape."""
    rng = rng_for(99, 2)
    dims, ranks, K, J = (12, 10, 8), (4, 5, 3), 7, 3
    U, core = tucker_basis(rng, dims, ranks, K)
    Bfull = np.einsum("abck,ia,jb,lc->ijlk", core, U[0], U[1], U[2]).reshape(-1, K)
    c = coefficients(rng, J, K)
    assert rel(oracle.tucker_apply(U, core, c), (Bfull @ c.T).T) < 1e-13
    S = complex_normal(rng, (J, int(np.prod(dims))))
    assert rel(oracle.tucker_adjoint(U, core, S), (Bfull.conj().T @ S.T).T) < 1e-13
    assert rel(oracle.tucker_materialise(U, core), Bfull) < 1e-13


def test_tucker_identity_factors_is_reshaped_core():
    rng = np.random.default_rng(4)
    dims, K = (3, 4, 5), 6
    core = complex_normal(rng, dims + (K,))
    U = [np.eye(n) for n in dims]
    B = oracle.tucker_materialise(U, core)
    assert np.array_equal(B, core.reshape(-1, K))


# ---------------------------------------------------------------- P4: orthonormal basis
def test_orthonormal_tucker_basis_roundtrip():
    rng = rng_for(98, 2)
    dims, ranks, K, J = (16, 12, 10), (6, 5, 4), 20, 4
    U, core = tucker_basis(rng, dims, ranks, K)
    c = coefficients(rng, J, K)
    S = oracle.tucker_apply(U, core, c)
    assert rel(np.linalg.norm(S, axis=1), np.linalg.norm(c, axis=1)) < 1e-13
    assert rel(oracle.tucker_adjoint(U, core, S), c) < 1e-13
    B = oracle.tucker_materialise(U, core)
    assert np.max(np.abs(B.conj().T @ B - np.eye(K))) < 1e-13


def test_orthonormal_dense_basis():
    rng = rng_for(97, 2)
    B = smooth_dense_basis(rng, (16, 16), 12, 6, 3.0)
    assert np.max(np.abs(B.conj().T @ B - np.eye(12))) < 1e-13
    c = coefficients(rng, 3, 12)
    assert rel(oracle.dense_adjoint(B, oracle.dense_apply(B, c)), c) < 1e-13


# ---------------------------------------------------------------- helpers for small problems
def small_cartesian_dense(seed=11, dims=(16, 12), J=3, K=5, full=False):
    rng = rng_for(seed, 2)
    B = smooth_dense_basis(rng, dims, K, 4, 2.0)
    N = int(np.prod(dims))
    if full:
        mask = np.arange(N)
    else:
        mask = np.sort(rng.choice(N, size=N // 3, replace=False))
    x = phantom(rng_for(seed, 1), dims)
    c = coefficients(rng_for(seed, 3), J, K)
    return Oracle(dims, B=B, mask_idx=mask), x, c


def small_cartesian_tucker(seed=12, dims=(10, 8, 12), ranks=(3, 4, 5), J=3, K=6):
    rng = rng_for(seed, 2)
    U, core = tucker_basis(rng, dims, ranks, K)
    N = int(np.prod(dims))
    mask = np.sort(rng.choice(N, size=N // 4, replace=False))
    x = phantom(rng_for(seed, 1), dims)
    c = coefficients(rng_for(seed, 3), J, K)
    return Oracle(dims, U=U, core=core, mask_idx=mask), x, c


def small_radial(seed=13, dims=(16, 16), J=2, K=4, exact=False, spokes=6):
    rng = rng_for(seed, 2)
    B = smooth_dense_basis(rng, dims, K, 4, 2.0)
    traj = golden_angle_radial(dims, spokes, 2 * max(dims))
    x = phantom(rng_for(seed, 1), dims)
    c = coefficients(rng_for(seed, 3), J, K)
    return Oracle(dims, B=B, traj=traj, exact_ndft=exact), x, c


def cdot(a, b):
    return np.vdot(np.asarray(a).reshape(-1), np.asarray(b).reshape(-1))


# ---------------------------------------------------------------- P2: adjoint identity
@pytest.mark.parametrize("maker", [small_cartesian_dense, small_cartesian_tucker, small_radial,
                                   lambda: small_radial(exact=True)])
def test_adjoint_identity_both_partial_maps(maker):
    op, x, c = maker()
    rng = np.random.default_rng(5)
    J = c.shape[0]
    y = complex_normal(rng, (J, op.encode(x, c).shape[1]))
    # partial map in x (c fixed): E_c z = E(z, c)
    z = complex_normal(rng, op.dims)
    gx, _ = op.adjoint(x, c, y)
    lhs = cdot(op.encode(z, c), y)
    rhs = cdot(z, gx)
    assert abs(lhs - rhs) / abs(lhs) < 1e-12
    # partial map in c (x fixed): E_x v = E(x, v)
    v = complex_normal(rng, c.shape)
    _, gc = op.adjoint(x, c, y)
    lhs = cdot(op.encode(x, v), y)
    rhs = cdot(v, gc)
    assert abs(lhs - rhs) / abs(lhs) < 1e-12


# ---------------------------------------------------------------- P5: special cases
def test_single_coil_constant_basis_is_plain_fft():
    """J = 1, K = 1, B = 1/sqrt(N), c = sqrt(N): E = P (centred FFT of x), with the
    FFT taken through scipy and explicit index rolls."""
    dims = (12, 10)
    N = 120
    B = np.full((N, 1), 1.0 / math.sqrt(N), dtype=complex)
    mask = np.sort(np.random.default_rng(6).choice(N, 50, replace=False))
    op = Oracle(dims, B=B, mask_idx=mask)
    x = phantom(rng_for(7, 1), dims)
    y = op.encode(x, np.array([[math.sqrt(N)]]))
    k = np.roll(np.fft.fft2(np.roll(x, (-6, -5), axis=(0, 1)), norm="ortho"), (6, 5), axis=(0, 1))
    assert rel(y[0], k.reshape(-1)[mask]) < 1e-13


def test_full_mask_normal_operator_closed_form():
    """With every k-space sample taken, F is unitary, so E_c^H E_c x = sum_j |s_j|^2 x."""
    op, x, c = small_cartesian_dense(full=True)
    gx, _ = op.adjoint(x, c, op.encode(x, c))
    S = op.coil_maps(c)
    expect = (np.sum(np.abs(S) ** 2, axis=0) * x.reshape(-1))
    assert rel(gx, expect) < 1e-13


def test_identity_basis_is_sense():
    """B = I_N: the coefficients are the maps themselves (plain SENSE)."""
    dims = (6, 8)
    N = 48
    rng = np.random.default_rng(8)
    mask = np.sort(rng.choice(N, 20, replace=False))
    op = Oracle(dims, B=np.eye(N, dtype=complex), mask_idx=mask)
    x = complex_normal(rng, dims)
    s = complex_normal(rng, (2, N))
    y = op.encode(x, s)
    for j in range(2):
        expect = brute_dft(s[j].reshape(dims) * x).reshape(-1)[mask]
        assert rel(y[j], expect) < 1e-13


# ---------------------------------------------------------------- P6: bilinearity
def test_bilinearity_and_coil_permutation():
    op, x, c = small_cartesian_tucker()
    a = 0.7 - 1.3j
    y = op.encode(x, c)
    assert rel(op.encode(a * x, c), a * y) < 1e-13
    assert rel(op.encode(x, a * c), a * y) < 1e-13
    rng = np.random.default_rng(9)
    x2 = complex_normal(rng, op.dims)
    c2 = complex_normal(rng, c.shape)
    assert rel(op.encode(x + x2, c), y + op.encode(x2, c)) < 1e-13
    assert rel(op.encode(x, c + c2), y + op.encode(x, c2)) < 1e-13
    perm = np.array([2, 0, 1])
    assert rel(op.encode(x, c[perm]), y[perm]) < 1e-14


# ---------------------------------------------------------------- P7/P9: gradient
def _problem_with_data(maker, weighted=False):
    op, x, c = maker()
    rng = np.random.default_rng(10)
    y = op.encode(x, c) + 0.1 * complex_normal(rng, (c.shape[0], op.encode(x, c).shape[1]))
    x0 = complex_normal(rng, op.dims)
    c0 = complex_normal(rng, c.shape) / math.sqrt(c.shape[1])
    w = rng.uniform(0.2, 1.0, size=y.shape[1]) if weighted else None
    return op, x0, c0, y, w


@pytest.mark.parametrize("maker,weighted", [(small_cartesian_dense, False),
                                            (small_cartesian_tucker, True),
                                            (small_radial, True)])
def test_gradient_finite_differences(maker, weighted):
    op, x, c, y, w = _problem_with_data(maker, weighted)
    f0, gx, gc = op.loss_and_grad(x, c, y, w)
    rng = np.random.default_rng(11)
    dx = complex_normal(rng, x.shape)
    dc = complex_normal(rng, c.shape)
    # x-only direction: f is quadratic along it, central FD with h = 1e-3 is exact
    h = 1e-3
    fd = (op.loss(x + h * dx, c, y, w) - op.loss(x - h * dx, c, y, w)) / (2 * h)
    an = np.real(cdot(gx, dx))
    assert abs(fd - an) / abs(an) < 1e-9
    fd = (op.loss(x, c + h * dc, y, w) - op.loss(x, c - h * dc, y, w)) / (2 * h)
    an = np.real(cdot(gc, dc))
    assert abs(fd - an) / abs(an) < 1e-9
    # joint direction: f is quartic along it; Richardson removes the h^2 term exactly

    def D(hh):
        return (op.loss(x + hh * dx, c + hh * dc, y, w) - op.loss(x - hh * dx, c - hh * dc, y, w)) / (2 * hh)
    rich = (4 * D(h / 2) - D(h)) / 3
    an = np.real(cdot(gx, dx) + cdot(gc, dc))
    assert abs(rich - an) / abs(an) < 1e-8


def test_euler_identity():
    op, x, c, y, w = _problem_with_data(small_cartesian_tucker, True)
    f0, gx, gc = op.loss_and_grad(x, c, y, w)
    E = op.encode(x, c)
    t = 2 * np.real(np.sum(w[None, :] * np.conj(E - y) * E))
    assert abs(np.real(cdot(gx, x)) - t) / abs(t) < 1e-12
    assert abs(np.real(cdot(gc, c)) - t) / abs(t) < 1e-12


def test_loss_and_gradient_at_truth():
    """Zero noise at the truth: f = 0 and the gradient vanishes; with noise n,
    f = ||n||^2 exactly."""
    op, x, c = small_cartesian_dense()
    y = op.encode(x, c)
    f, gx, gc = op.loss_and_grad(x, c, y)
    assert f < 1e-25
    assert np.linalg.norm(gx) < 1e-12 * np.linalg.norm(y) and np.linalg.norm(gc) < 1e-12 * np.linalg.norm(y)
    n = 0.01 * complex_normal(np.random.default_rng(12), y.shape)
    assert abs(op.loss(x, c, y + n) - np.sum(np.abs(n) ** 2)) / np.sum(np.abs(n) ** 2) < 1e-12


def test_jvp_is_exact_central_difference():
    """E is quadratic along any joint line, so the central difference is exact."""
    op, x, c = small_cartesian_tucker()
    rng = np.random.default_rng(13)
    dx = complex_normal(rng, x.shape)
    dc = complex_normal(rng, c.shape)
    h = 0.37
    fd = (op.encode(x + h * dx, c + h * dc) - op.encode(x - h * dx, c - h * dc)) / (2 * h)
    assert rel(op.jvp(x, c, dx, dc), fd) < 1e-13
    # and J is the transpose of J^H
    w = complex_normal(rng, fd.shape)
    gx, gc = op.adjoint(x, c, w)
    lhs = cdot(op.jvp(x, c, dx, dc), w)
    rhs = cdot(dx, gx) + cdot(dc, gc)
    assert abs(lhs - rhs) / abs(lhs) < 1e-12


# ---------------------------------------------------------------- P10: NUFFT
def test_kb_beta_value():
    # W = 6, sigma = 2: pi sqrt(9 * 2.25 - 0.8) = pi sqrt(19.45)
    assert abs(oracle.kb_beta(6, 2.0) - 13.8551003) < 1e-6


@pytest.mark.parametrize("nu", [0.0, 0.05, 0.13, 0.25, 0.4])
def test_kb_deapod_is_fourier_transform_of_kernel(nu):
    W, beta = 6, oracle.kb_beta(6, 2.0)
    val, _ = quad(lambda t: oracle.kb_kernel(np.array([t]), W, beta)[0] * math.cos(2 * math.pi * t * nu),
                  -W / 2, W / 2, epsabs=0, epsrel=1e-13, limit=200)
    ref = oracle.kb_deapod(np.array([nu]), W, beta)[0]
    assert abs(val - ref) / abs(ref) < 1e-12


def test_kb_deapod_sin_branch():
    W, beta = 6, 2.0  # small beta so pi W nu exceeds beta
    nu = 0.3
    val, _ = quad(lambda t: oracle.kb_kernel(np.array([t]), W, beta)[0] * math.cos(2 * math.pi * t * nu),
                  -W / 2, W / 2, epsabs=0, epsrel=1e-13, limit=200)
    assert abs(val - oracle.kb_deapod(np.array([nu]), W, beta)[0]) < 1e-12


def test_nufft_approximates_ndft():
    rng = np.random.default_rng(14)
    dims = (32, 24)
    img = phantom(rng_for(14, 1), dims)
    traj = np.stack([rng.uniform(-16, 16, 400), rng.uniform(-12, 12, 400)], axis=1)
    y = oracle.nufft_type2(img, traj)
    yref = oracle.ndft(img, traj)
    assert rel(y, yref) < 1e-4
    yy = complex_normal(rng, 400)
    assert rel(oracle.nufft_type1(yy, traj, dims), oracle.ndft_adjoint(yy, traj, dims)) < 1e-4


def test_ndft_on_grid_equals_dft():
    """NDFT at integer k on the full grid is the centred DFT (brute force)."""
    dims = (6, 8)
    kk = np.stack(np.meshgrid(np.arange(6) - 3, np.arange(8) - 4, indexing="ij"), -1).reshape(-1, 2)
    img = complex_normal(np.random.default_rng(15), dims)
    assert rel(oracle.ndft(img, kk.astype(float)), brute_dft(img).reshape(-1)) < 1e-13


def test_nufft_type1_is_transpose_of_type2():
    rng = np.random.default_rng(16)
    dims = (20, 16)
    traj = golden_angle_radial(dims, 5, 40)
    a = complex_normal(rng, dims)
    b = complex_normal(rng, traj.shape[0])
    lhs = cdot(oracle.nufft_type2(a, traj), b)
    rhs = cdot(a, oracle.nufft_type1(b, traj, dims))
    assert abs(lhs - rhs) / abs(lhs) < 1e-13


def test_nufft_kernel_tie_break():
    """At |u - g| = W/2 the first tap weight is I0(0)/W (not zero): a sample at
    u - W/2 integral puts weight 1/W on the first tap."""
    W, beta = 6, oracle.kb_beta(6, 2.0)
    assert abs(oracle.kb_kernel(np.array([3.0]), W, beta)[0] - 1.0 / W) < 1e-15


# ---------------------------------------------------------------- input generators
def test_config_generators_shapes():
    p = problem("cart2d_64_dense32_j8")
    assert p.M == 28 * 64 and p.B.shape == (4096, 32)
    traj = golden_angle_radial((256, 256), 64, 512)
    assert traj.shape == (32768, 2) and np.max(np.abs(traj)) <= 128
    w = ramp_dcf(traj, (256, 256), 512)
    assert abs(w.max() - 1.0) < 1e-15 and w.min() > 0


# ---------------------------------------------------------------- multi-map (extra bilinear terms)
def test_multi_map_reduces_and_matches_finite_differences():
    from oracle.encoding import multi_encode, multi_loss_and_grad
    op, x, c = small_cartesian_dense()
    rng = np.random.default_rng(21)
    x2 = complex_normal(rng, x.shape)
    c2 = coefficients(rng, *c.shape)
    y = complex_normal(rng, (c.shape[0], op.mask_idx.size))
    # one map set is the plain operator; a zero second image changes nothing
    assert rel(multi_encode(op, [x], [c]), op.encode(x, c)) < 1e-14
    assert rel(multi_encode(op, [x, 0 * x2], [c, c2]), op.encode(x, c)) < 1e-14
    # the loss is quadratic along a direction in (x, x2) with c, c2 fixed: exact central difference
    f, gxs, gcs = multi_loss_and_grad(op, [x, x2], [c, c2], y)
    d1, d2 = complex_normal(rng, x.shape), complex_normal(rng, x.shape)
    h = 0.3
    fp = multi_loss_and_grad(op, [x + h * d1, x2 + h * d2], [c, c2], y)[0]
    fm = multi_loss_and_grad(op, [x - h * d1, x2 - h * d2], [c, c2], y)[0]
    dd = np.real(np.vdot(gxs[0], d1) + np.vdot(gxs[1], d2))
    assert abs((fp - fm) / (2 * h) - dd) < 1e-10 * abs(dd)
    # and along the coefficients of the second map set
    e2 = complex_normal(rng, c.shape)
    fp = multi_loss_and_grad(op, [x, x2], [c, c2 + h * e2], y)[0]
    fm = multi_loss_and_grad(op, [x, x2], [c, c2 - h * e2], y)[0]
    dd = np.real(np.vdot(gcs[1], e2))
    assert abs((fp - fm) / (2 * h) - dd) < 1e-10 * abs(dd)


def test_poisson_disc_helper_matches_the_loop():
    """Input generation: the C dart-throwing helper gives the same masks as the Python loop."""
    from synth import poisson_disc_plane, rng_for
    import synth.inputs as si
    if si._pd_native() is None:
        import pytest
        pytest.skip("libpdisc.so not built")
    for shape, R, c in [((40, 56), 4.0, 8), ((64, 48), 6.0, 12), ((30, 30), 2.5, 4)]:
        a = poisson_disc_plane(rng_for(9, 4), shape, R, c, native=False)
        b = poisson_disc_plane(rng_for(9, 4), shape, R, c, native=True)
        assert np.array_equal(a, b)
        assert int(b.sum()) == int(round(shape[0] * shape[1] / R))
