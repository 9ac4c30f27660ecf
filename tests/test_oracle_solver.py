"""Pins for the oracle's Gauss-Newton normal operator and conjugate gradients.

* The normal operator equals J^H W J + diag(lambda) with J the explicit matrix of the JVP,
  assembled column by column from unit vectors and conjugate-transposed as a matrix (so the
  adjoint inside the operator is checked against the JVP, not against itself).
* It is Hermitian and positive definite for lambda > 0.
* CG run to the problem's dimension reproduces a dense linear solve of that matrix.
* On a diagonal operator with k distinct eigenvalues CG is exact after k steps; its recursive
  residuals equal the true residuals b - A x_k.
* A zero right-hand side stays at zero (the guarded step).
"""
import numpy as np
import pytest

from oracle import Oracle
from oracle.solver import cg, gn_cg, inner, normal
from synth import coefficients, complex_normal, golden_angle_radial, phantom, ramp_dcf, rng_for, smooth_dense_basis


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def tiny_cartesian(seed=21, dims=(4, 6), J=2, K=3):
    rng = rng_for(seed, 2)
    B = smooth_dense_basis(rng, dims, K, 2, 1.0)
    N = int(np.prod(dims))
    mask = np.sort(rng.choice(N, size=N // 2, replace=False))
    x = phantom(rng_for(seed, 1), dims).reshape(-1)
    c = coefficients(rng_for(seed, 3), J, K)
    w = rng_for(seed, 4).uniform(0.2, 1.0, size=mask.size)
    return Oracle(dims, B=B, mask_idx=mask), x, c, w


def tiny_radial(seed=22, dims=(6, 6), J=2, K=3):
    rng = rng_for(seed, 2)
    B = smooth_dense_basis(rng, dims, K, 2, 1.0)
    traj = golden_angle_radial(dims, 3, 8)
    x = phantom(rng_for(seed, 1), dims).reshape(-1)
    c = coefficients(rng_for(seed, 3), J, K)
    return Oracle(dims, B=B, traj=traj), x, c, ramp_dcf(traj, dims, 8)


def jacobian_matrix(op, x, c):
    """Columns J e_i for the unit vectors of (dx, dc): complex (J*M) x (N + J*K)."""
    N, (J, K) = x.size, c.shape
    cols = []
    for i in range(N + J * K):
        e = np.zeros(N + J * K, dtype=np.complex128)
        e[i] = 1.0
        cols.append(op.jvp(x, c, e[:N], e[N:].reshape(J, K)).reshape(-1))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("maker", [tiny_cartesian, tiny_radial])
def test_normal_operator_matches_explicit_matrix(maker):
    op, x, c, w = maker()
    N, (J, K) = x.size, c.shape
    Jm = jacobian_matrix(op, x, c)
    W = np.tile(w, J)
    lam_x, lam_c = 0.3, 0.05
    A = Jm.conj().T @ (W[:, None] * Jm) + np.diag(np.r_[np.full(N, lam_x), np.full(J * K, lam_c)])
    rng = np.random.default_rng(7)
    v = complex_normal(rng, N + J * K)
    gx, gc = normal(op, x, c, v[:N], v[N:].reshape(J, K), lam_x, lam_c, w)
    assert rel(np.r_[gx, gc.reshape(-1)], A @ v) < 1e-12
    # Hermitian, positive definite
    assert np.max(np.abs(A - A.conj().T)) < 1e-12 * np.max(np.abs(A))
    assert np.min(np.linalg.eigvalsh(A)) >= min(lam_x, lam_c) * (1 - 1e-9)


def test_normal_operator_is_hermitian_on_vectors():
    op, x, c, w = tiny_cartesian(seed=23, dims=(6, 4))
    N, (J, K) = x.size, c.shape
    rng = np.random.default_rng(8)
    u = (complex_normal(rng, N), complex_normal(rng, (J, K)))
    v = (complex_normal(rng, N), complex_normal(rng, (J, K)))
    Au = normal(op, x, c, *u, 0.1, 0.2, w)
    Av = normal(op, x, c, *v, 0.1, 0.2, w)
    lhs = np.vdot(u[0], Av[0]) + np.vdot(u[1], Av[1])
    rhs = np.conj(np.vdot(v[0], Au[0]) + np.vdot(v[1], Au[1]))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    assert inner(v, Av) > 0


@pytest.mark.parametrize("maker", [tiny_cartesian, tiny_radial])
def test_cg_reaches_the_dense_solve(maker):
    op, x, c, w = maker()
    N, (J, K) = x.size, c.shape
    Jm = jacobian_matrix(op, x, c)
    W = np.tile(w, J)
    lam_x, lam_c = 0.3, 0.05
    A = Jm.conj().T @ (W[:, None] * Jm) + np.diag(np.r_[np.full(N, lam_x), np.full(J * K, lam_c)])
    rng = np.random.default_rng(9)
    b = complex_normal(rng, N + J * K)
    ref = np.linalg.solve(A, b)
    dx, dc, rr = gn_cg(op, x, c, b[:N], b[N:].reshape(J, K), lam_x, lam_c, 3 * (N + J * K), w)
    assert rel(np.r_[dx, dc.reshape(-1)], ref) < 1e-7
    assert rr[0] == pytest.approx(float(np.vdot(b, b).real))
    assert rr[-1] < 1e-12 * rr[0]


def test_cg_on_diagonal_operator():
    """k distinct eigenvalues: exact after k steps; recursive residual = true residual."""
    rng = np.random.default_rng(10)
    dx_diag = np.repeat([1.0, 2.5, 7.0], 4)     # 12 image entries, 3 distinct values
    dc_diag = np.full((2, 3), 4.0)              # a fourth value
    A = lambda a, b: (dx_diag * a, dc_diag * b)  # noqa: E731
    bx, bc = complex_normal(rng, 12), complex_normal(rng, (2, 3))
    for k in range(1, 5):
        dx, dc, rr = cg(A, bx, bc, k)
        true_r = (bx - dx_diag * dx, bc - dc_diag * dc)
        assert abs(inner(true_r, true_r) - rr[-1]) <= 1e-10 * rr[0]
    assert rel(dx, bx / dx_diag) < 1e-12 and rel(dc, bc / dc_diag) < 1e-12
    # residual norms after 3 steps are not yet zero (four distinct eigenvalues)
    _, _, rr3 = cg(A, bx, bc, 3)
    assert rr3[-1] > 1e-8 * rr3[0]


def test_cg_zero_rhs_stays_zero():
    A = lambda a, b: (2.0 * a, 3.0 * b)  # noqa: E731
    dx, dc, rr = cg(A, np.zeros(5, complex), np.zeros((1, 2), complex), 3)
    assert not np.any(dx) and not np.any(dc) and not np.any(rr)
