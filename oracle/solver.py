"""Gauss-Newton normal operator and conjugate gradients (oracle; test infrastructure only).

Paper, Sec. II-B, Eq. (6): the modified IRGN step minimises half the squared misfit of the
model linearised at v_n = (p, a_1..a_C), plus alpha_n ||p + dp||^2 and
beta_n sum_k ||a_k + da_k||^2.  The objective is quadratic, so its minimiser solves the
normal equations, by conjugate gradients, using the Jacobian-vector product (Eq. (7)) and the
Jacobian adjoint (the J_G^H expression of Sec. II-B).

Setting the derivative with respect to conj(dv) to zero gives

    (J^H J + 2 diag(alpha_n, beta_n)) dv = J^H (y - G(v_n)) - 2 diag(alpha_n, beta_n) v_n

so the operator here is

    normal(dv) = J^H (w (.) J dv) + (lam_x dx, lam_c dc)

with optional data weights w (w = 1 gives the paper's operator) and lam_x = 2 alpha_n,
lam_c = 2 beta_n supplied by the caller together with the right-hand side.

cg() is the textbook method for a Hermitian positive definite operator, started from zero
(Shewchuk, "An introduction to the conjugate gradient method without the agonizing pain",
1994, the reference the paper gives): step length <r, r> / <d, A d>, residual update, new
direction r + (<r', r'> / <r, r>) d.  Inner products are the real part of the complex one
over both blocks (image and coefficients); for a Hermitian operator both ratios are real.
A zero denominator gives a zero step (the iteration then stands still).
"""
from typing import Callable, List, Tuple

import numpy as np

from .encoding import Oracle

Vec = Tuple[np.ndarray, np.ndarray]


def inner(a: Vec, b: Vec) -> float:
    """Re <a, b> = Re sum conj(a) b over the image block and the coefficient block."""
    return float(np.real(np.vdot(a[0], b[0]) + np.vdot(a[1], b[1])))


def normal(op: Oracle, x, c, dx, dc, lam_x: float, lam_c: float, w=None) -> Vec:
    """J^H (w (.) J[dx, dc]) + (lam_x dx, lam_c dc) at (x, c)."""
    u = op.jvp(x, c, dx, dc)
    if w is not None:
        u = np.asarray(w, dtype=np.float64)[None, :] * u
    gx, gc = op.adjoint(x, c, u)
    dx = np.asarray(dx, dtype=np.complex128).reshape(-1)
    dc = np.asarray(dc, dtype=np.complex128)
    return gx + lam_x * dx, gc + lam_c * dc


def cg(apply: Callable[[np.ndarray, np.ndarray], Vec], bx, bc, iters: int):
    """iters steps of CG from zero on apply(dx, dc) = (bx, bc).

    Returns (dx, dc, rr) with rr[k] = <r_k, r_k> for k = 0..iters (r_0 = b)."""
    xs = (np.zeros_like(np.asarray(bx, dtype=np.complex128).reshape(-1)),
          np.zeros_like(np.asarray(bc, dtype=np.complex128)))
    r = (np.asarray(bx, dtype=np.complex128).reshape(-1).copy(), np.asarray(bc, dtype=np.complex128).copy())
    d = (r[0].copy(), r[1].copy())
    rho = inner(r, r)
    rr: List[float] = [rho]
    for _ in range(iters):
        q = apply(d[0], d[1])
        dq = inner(d, q)
        alpha = rho / dq if dq != 0.0 else 0.0
        xs = (xs[0] + alpha * d[0], xs[1] + alpha * d[1])
        r = (r[0] - alpha * q[0], r[1] - alpha * q[1])
        rho_new = inner(r, r)
        beta = rho_new / rho if rho != 0.0 else 0.0
        d = (r[0] + beta * d[0], r[1] + beta * d[1])
        rho = rho_new
        rr.append(rho)
    return xs[0], xs[1], np.array(rr)


def gn_cg(op: Oracle, x, c, bx, bc, lam_x: float, lam_c: float, iters: int, w=None):
    """CG on the normal operator at (x, c)."""
    return cg(lambda dx, dc: normal(op, x, c, dx, dc, lam_x, lam_c, w), bx, bc, iters)
