"""SENSE with fixed maps and the constrained density reconstruction by ADMM (oracle; test
infrastructure only).

Paper, Sec. II-C ("Regularized density reconstruction via constrained optimization"): with
the coil maps S_k fixed, the density minimises R(p) subject to ||y_k - F_s S_k p|| <= eps_k for
every coil.  With A = [I; F_s S_1; ...; F_s S_C] and z = (z_0, z_1..z_C) the scaled ADMM
iteration of the paper's Eq. (algo) is

    z_0 <- prox_{R / rho}(p + u_0)
    z_k <- Pi_{C(y_k, eps_k)}(F_s S_k p + u_k)
    p   <- (I + sum_k S_k^H F_s^H F_s S_k)^{-1} (z_0 - u_0 + sum_k S_k^H F_s^H (z_k - u_k))
    u   <- u + A p - z

(the paper prints the argument of the first prox garbled; the scaled form it cites, Boyd
et al. 2011 Sec. 3.1.1, gives p + u_0).  The ball projection is the closed form
Pi(z) = y + eps (z - y) / max(||z - y||, eps).  R is isotropic total variation.  rho adapts
after every iteration by residual balancing (He, Yang and Wang 2000; Boyd et al. Sec. 3.4.1):
with the primal residual r = ||A p - z|| and the dual residual s = rho ||A^H (z - z_prev)||,
rho <- 2 rho and u <- u / 2 when r > 10 s, rho <- rho / 2 and u <- 2 u when s > 10 r.

Readings (not fixed by the paper): TV(x) = sum over pixels of sqrt(sum_d |x[i + e_d] - x[i]|^2)
with forward differences that are zero at the last index of each axis (complex values, the
real and imaginary parts coupled under the root); its prox is Chambolle's dual projection
algorithm (J. Math. Imaging Vis. 20, 2004) with step 1 / (4 ndim) and a fixed number of
steps from a zero dual field; the p-update runs a fixed number of CG steps on the residual
system from the current p; p starts at the adjoint A^H (0, y) scaled by nothing (the
zero-filled SENSE combination) and z, u at zero.
"""
import numpy as np

from .encoding import Oracle
from .solver import cg


# ---- SENSE with fixed maps (Sec. II-A, Eq. (1); Sec. II-C)
def sense_encode(op: Oracle, S, x) -> np.ndarray:
    """y_k = F_s(S_k (.) x) for maps S (J, N) -> (J, M)."""
    x = np.asarray(x, dtype=np.complex128).reshape(-1)
    return np.stack([op.fs((np.asarray(s, dtype=np.complex128) * x).reshape(op.dims)) for s in np.asarray(S)])


def sense_adjoint(op: Oracle, S, y) -> np.ndarray:
    """sum_k conj(S_k) (.) F_s^H y_k -> (N,)."""
    out = np.zeros(op.N, dtype=np.complex128)
    for s, yk in zip(np.asarray(S), np.asarray(y)):
        out += np.conj(np.asarray(s, dtype=np.complex128)) * op.fs_adjoint(yk).reshape(-1)
    return out


def sense_normal(op: Oracle, S, x) -> np.ndarray:
    """(I + sum_k S_k^H F_s^H F_s S_k) x, the p-update operator of the ADMM iteration."""
    x = np.asarray(x, dtype=np.complex128).reshape(-1)
    return x + sense_adjoint(op, S, sense_encode(op, S, x))


# ---- the proximal and projection steps
def ball_project(z, y, eps) -> np.ndarray:
    """Per coil k: y_k + eps_k (z_k - y_k) / max(||z_k - y_k||, eps_k)."""
    z = np.asarray(z, dtype=np.complex128)
    y = np.asarray(y, dtype=np.complex128)
    out = np.empty_like(z)
    for k in range(z.shape[0]):
        d = z[k] - y[k]
        out[k] = y[k] + eps[k] * d / max(float(np.linalg.norm(d)), float(eps[k]))
    return out


def grad(x: np.ndarray) -> np.ndarray:
    """Forward differences along every axis, zero at the last index: (ndim, *shape)."""
    g = np.zeros((x.ndim,) + x.shape, dtype=np.complex128)
    for d in range(x.ndim):
        sl_hi = [slice(None)] * x.ndim
        sl_lo = [slice(None)] * x.ndim
        sl_hi[d] = slice(1, None)
        sl_lo[d] = slice(0, -1)
        g[d][tuple(sl_lo)] = x[tuple(sl_hi)] - x[tuple(sl_lo)]
    return g


def div(p: np.ndarray) -> np.ndarray:
    """Minus the adjoint of grad: <grad x, p> = -<x, div p>.  Along axis d,
    (div p)_i = p_i - p_{i-1}, with p_{-1} = 0 and p_{n-1} taken as 0."""
    out = np.zeros(p.shape[1:], dtype=np.complex128)
    nd = p.shape[0]
    for d in range(nd):
        q = np.moveaxis(p[d], d, 0)
        t = np.zeros_like(q)
        t[:-1] += q[:-1]
        t[1:] -= q[:-1]
        out += np.moveaxis(t, 0, d)
    return out


def tv(x: np.ndarray) -> float:
    g = grad(np.asarray(x, dtype=np.complex128))
    return float(np.sum(np.sqrt(np.sum(np.abs(g) ** 2, axis=0))))


def tv_prox(z: np.ndarray, lam: float, iters: int) -> np.ndarray:
    """argmin_x 1/2 ||x - z||^2 + lam TV(x) by Chambolle's dual projection steps."""
    z = np.asarray(z, dtype=np.complex128)
    nd = z.ndim
    tau = 1.0 / (4.0 * nd)
    p = np.zeros((nd,) + z.shape, dtype=np.complex128)
    if lam <= 0:
        return z.copy()
    for _ in range(iters):
        g = grad(div(p) - z / lam)
        mag = np.sqrt(np.sum(np.abs(g) ** 2, axis=0))
        p = (p + tau * g) / (1.0 + tau * mag)[None]
    return z - lam * div(p)


# ---- the ADMM iteration
def admm(op: Oracle, S, y, eps, rho0: float, iters: int, cg_iters: int, tv_iters: int):
    """Constrained TV-SENSE reconstruction.  Returns (p, history) with history rows
    (rho used, primal residual, dual residual) per iteration."""
    S = np.asarray(S, dtype=np.complex128)
    y = np.asarray(y, dtype=np.complex128)
    J = S.shape[0]
    p = sense_adjoint(op, S, y)
    z0 = np.zeros(op.N, dtype=np.complex128)
    u0 = np.zeros(op.N, dtype=np.complex128)
    zk = np.zeros_like(y)
    uk = np.zeros_like(y)
    rho = float(rho0)
    hist = []
    for _ in range(iters):
        z0_prev, zk_prev = z0, zk
        Fp = sense_encode(op, S, p)
        z0 = tv_prox((p + u0).reshape(op.dims), 1.0 / rho, tv_iters).reshape(-1)
        zk = ball_project(Fp + uk, y, eps)
        rhs = (z0 - u0) + sense_adjoint(op, S, zk - uk)
        res = rhs - sense_normal(op, S, p)
        dp, _, _ = cg(lambda a, b: (sense_normal(op, S, a), np.zeros_like(b)), res, np.zeros((J, 0)), cg_iters)
        p = p + dp
        Fp = sense_encode(op, S, p)
        u0 = u0 + p - z0
        uk = uk + Fp - zk
        r = np.sqrt(np.linalg.norm(p - z0) ** 2 + np.linalg.norm(Fp - zk) ** 2)
        s = rho * np.linalg.norm((z0 - z0_prev) + sense_adjoint(op, S, zk - zk_prev))
        hist.append((rho, r, s))
        if r > 10.0 * s:
            rho *= 2.0
            u0, uk = u0 / 2.0, uk / 2.0
        elif s > 10.0 * r:
            rho /= 2.0
            u0, uk = u0 * 2.0, uk * 2.0
    return p, np.array(hist)
