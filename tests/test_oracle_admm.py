"""Pins for the oracle's SENSE operators and the ADMM pieces of the constrained reconstruction.

* SENSE with maps S_k = B c_k equals the pinned bilinear encode; its adjoint passes the adjoint
  identity; the p-update operator I + sum S^H F^H F S is Hermitian with eigenvalues >= 1.
* Ball projection: points inside are kept, points outside land on the sphere along the ray
  from the centre, and the projection is idempotent.
* grad / div: <grad x, p> = -<x, div p> on random complex fields (2D and 3D).
* TV prox: a constant image is its own prox; the two-pixel problem has a closed form
  (the difference shrinks by 2 lam, or the pair merges to its mean); the prox objective at the
  result is below that of random perturbations of it.
* ADMM (maps scaled to order-one sensitivities, eps_k = least-squares misfit + 10 % of ||y_k||):
  the result is feasible (every coil's misfit within eps_k, to 1 %), its TV is below that of
  the least-squares solution, which is feasible by the choice of eps, and the primal residual
  has fallen a hundredfold.
"""
import numpy as np
import pytest

from oracle import Oracle
from oracle.admm import admm, ball_project, div, grad, sense_adjoint, sense_encode, sense_normal, tv, tv_prox
from synth import coefficients, complex_normal, phantom, rng_for, smooth_dense_basis


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def small(seed=31, dims=(12, 10), J=3, K=4, frac=0.5):
    rng = rng_for(seed, 2)
    B = smooth_dense_basis(rng, dims, K, 3, 1.5)
    N = int(np.prod(dims))
    mask = np.sort(rng.choice(N, size=int(frac * N), replace=False))
    c = coefficients(rng_for(seed, 3), J, K)
    op = Oracle(dims, B=B, mask_idx=mask)
    S = op.coil_maps(c)
    x = phantom(rng_for(seed, 1), dims).reshape(-1)
    return op, S, c, x


def test_sense_equals_bilinear_encode_and_adjoint_identity():
    op, S, c, x = small()
    assert rel(sense_encode(op, S, x), op.encode(x, c)) < 1e-13
    rng = np.random.default_rng(3)
    y = complex_normal(rng, (S.shape[0], op.mask_idx.size))
    v = complex_normal(rng, op.N)
    lhs = np.vdot(sense_encode(op, S, v).reshape(-1), y.reshape(-1))
    rhs = np.vdot(v, sense_adjoint(op, S, y))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_sense_normal_is_hermitian_and_at_least_identity():
    op, S, c, x = small(dims=(6, 5), J=2, K=3)
    A = np.stack([sense_normal(op, S, e) for e in np.eye(op.N)], axis=1)
    assert np.max(np.abs(A - A.conj().T)) < 1e-12 * np.max(np.abs(A))
    assert np.min(np.linalg.eigvalsh(A)) > 1 - 1e-10


def test_ball_projection():
    rng = np.random.default_rng(4)
    y = complex_normal(rng, (3, 20))
    z = y + np.stack([0.1, 1.0, 5.0])[:, None] * complex_normal(rng, (3, 20))
    eps = np.array([10.0, 1.0, 2.0])
    pz = ball_project(z, y, eps)
    d = np.linalg.norm(z - y, axis=1)
    assert np.max(np.abs(pz[0] - z[0])) < 1e-14              # inside: unchanged
    for k in (1, 2):                                        # outside: on the sphere, same ray
        assert abs(np.linalg.norm(pz[k] - y[k]) - eps[k]) < 1e-12
        assert rel(pz[k] - y[k], (z[k] - y[k]) * eps[k] / d[k]) < 1e-13
    assert np.allclose(ball_project(pz, y, eps), pz, rtol=0, atol=1e-13)


@pytest.mark.parametrize("shape", [(7, 5), (4, 6, 5)])
def test_grad_div_adjoint(shape):
    rng = np.random.default_rng(5)
    x = complex_normal(rng, shape)
    p = complex_normal(rng, (len(shape),) + shape)
    lhs = np.vdot(grad(x).reshape(-1), p.reshape(-1))
    rhs = -np.vdot(x.reshape(-1), div(p).reshape(-1))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_tv_prox_constant_and_two_pixel_closed_form():
    const = np.full((5, 4), 0.3 - 0.7j)
    assert np.allclose(tv_prox(const, 0.5, 50), const, atol=1e-14)
    z = np.array([1.0 + 0.5j, -0.2 + 1.1j])
    d = z[1] - z[0]
    for lam in (0.1, 0.3, 2.0):
        x = tv_prox(z, lam, 4000)
        if abs(d) > 2 * lam:
            u = d / abs(d)
            ref = np.array([z[0] + lam * u, z[1] - lam * u])
        else:
            ref = np.full(2, z.mean())
        assert np.max(np.abs(x - ref)) < 1e-6, lam


def test_tv_prox_beats_perturbations():
    rng = np.random.default_rng(6)
    z = phantom(rng_for(7, 1), (10, 9)) + 0.1 * complex_normal(rng, (10, 9))
    lam = 0.05
    x = tv_prox(z, lam, 500)
    obj = lambda v: 0.5 * np.linalg.norm(v - z) ** 2 + lam * tv(v)  # noqa: E731
    f = obj(x)
    for _ in range(20):
        assert f <= obj(x + 1e-3 * complex_normal(rng, z.shape)) + 1e-9


def test_admm_is_feasible_and_not_rougher_than_least_squares():
    op, S, c, x = small(seed=33, dims=(12, 12), J=3, K=4, frac=0.6)
    S = S / np.sqrt(np.mean(np.sum(np.abs(S) ** 2, axis=0)))  # sensitivities of order one
    rng = np.random.default_rng(8)
    y = sense_encode(op, S, x)
    y = y + 0.02 * np.linalg.norm(y) / np.sqrt(y.size) * complex_normal(rng, y.shape)
    # least-squares solution (dense normal equations on this small problem)
    Amat = np.stack([sense_normal(op, S, e) - e for e in np.eye(op.N)], axis=1)
    p_ls = np.linalg.lstsq(Amat, sense_adjoint(op, S, y), rcond=None)[0]
    eps = np.linalg.norm(y - sense_encode(op, S, p_ls), axis=1) + 0.1 * np.linalg.norm(y, axis=1)
    p, hist = admm(op, S, y, eps, rho0=1.0, iters=200, cg_iters=20, tv_iters=30)
    mis = np.linalg.norm(y - sense_encode(op, S, p), axis=1)
    assert np.all(mis <= eps * 1.01), (mis, eps)
    assert tv(p.reshape(op.dims)) < 0.9 * tv(p_ls.reshape(op.dims))
    assert hist.shape == (200, 3) and hist[-1, 1] < 1e-2 * hist[0, 1]
