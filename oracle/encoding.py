"""Encoding operator, Jacobian adjoint, loss and gradient (oracle; test infrastructure only).

Paper, Sec. II-B, Eq. (5): for every coil j the bilinear model is

    E(x, c)_j = F_s( (B c_j) (.) x )

with x the rasterised image (the paper's density p), c_j the basis
coefficients of coil j (the paper's alpha_k), B the basis (U / U_h) and (.)
the elementwise product.  F_s is the undersampled Fourier operator of
Sec. II-A, Eq. (1): here either P F with F the centred unitary DFT and P the
gather of a sorted Cartesian mask, or the KB NUFFT / exact NDFT for radial
sampling.

The Jacobian adjoint (Sec. II-B, the expression for J_G^H) at (x, c) is

    gx   = sum_j conj(B c_j) (.) F_s^H y_j
    gc_j = B^H ( conj(x) (.) F_s^H y_j )

and the Jacobian-vector product (Sec. II-B, Eq. (7)) is

    J[dx, dc]_j = F_s( (B c_j) (.) dx + x (.) (B dc_j) ).

The data-fidelity loss is f = sum_j sum_m w_m |E_jm - y_jm|^2 (the paper's
objective, Eq. (6), carries a factor 1/2; this loss does not).  Its packed
real gradient (d f / d Re + i d f / d Im, the PyTorch convention) is
2 J^H (w (.) r) with r = E - y.

Large problems are processed one coil at a time to bound memory.
"""
from typing import Optional, Sequence

import numpy as np

from . import basis as _basis
from .dft import centred_dft, centred_idft
from .nufft import kb_beta, ndft, ndft_adjoint, nufft_type1, nufft_type2


class Oracle:
    """FP64 operator for one problem geometry.

    Parameters
    ----------
    dims      image dimensions (2 or 3 axes, C-order)
    B         dense basis (N, K), or None
    U, core   Tucker factors (n_m, r_m) and core (r0, r1, r2, K), or None
    mask_idx  sorted unique linear indices into the centred k-space grid (Cartesian)
    traj      (M, ndim) trajectory in cycles/FOV (radial); ``exact_ndft`` selects the
              plain NDFT instead of the KB NUFFT
    """

    def __init__(self, dims: Sequence[int], B: Optional[np.ndarray] = None, U=None, core=None,
                 mask_idx: Optional[np.ndarray] = None, traj: Optional[np.ndarray] = None,
                 kb_width: int = 6, oversamp: float = 2.0, kb_beta_value: Optional[float] = None,
                 exact_ndft: bool = False):
        self.dims = tuple(int(n) for n in dims)
        self.N = int(np.prod(self.dims))
        self.B = None if B is None else np.asarray(B, dtype=np.complex128)
        self.U = None if U is None else [np.asarray(u, dtype=np.complex128) for u in U]
        self.core = None if core is None else np.asarray(core, dtype=np.complex128)
        if (self.B is None) == (self.core is None):
            raise ValueError("give exactly one of a dense basis or a Tucker basis")
        self.K = self.B.shape[1] if self.B is not None else self.core.shape[-1]
        self.mask_idx = None if mask_idx is None else np.asarray(mask_idx, dtype=np.int64)
        self.traj = None if traj is None else np.asarray(traj, dtype=np.float64)
        if (self.mask_idx is None) == (self.traj is None):
            raise ValueError("give exactly one of a Cartesian mask or a trajectory")
        self.W = int(kb_width)
        self.sigma = float(oversamp)
        self.beta = kb_beta(self.W, self.sigma) if kb_beta_value is None else float(kb_beta_value)
        self.exact_ndft = exact_ndft
        self.axes = tuple(range(len(self.dims)))

    @classmethod
    def from_problem(cls, p, exact_ndft: bool = False) -> "Oracle":
        return cls(p.dims, B=p.B, U=p.U, core=p.core, mask_idx=p.mask_idx, traj=p.traj,
                   kb_width=p.kb_width, oversamp=p.oversamp, exact_ndft=exact_ndft)

    # --- basis (Sec. II-B Eq. (5); Sec. II-E) -------------------------------------------
    def coil_map(self, cj: np.ndarray) -> np.ndarray:
        """s_j = B c_j as an image-shaped array."""
        if self.B is not None:
            return (self.B @ np.asarray(cj, dtype=np.complex128)).reshape(self.dims)
        return _basis.tucker_coil_map(self.U, self.core, cj)

    def coil_maps(self, c: np.ndarray) -> np.ndarray:
        """S (J, N)."""
        return np.stack([self.coil_map(cj).reshape(-1) for cj in np.asarray(c)])

    def basis_adjoint_one(self, v: np.ndarray) -> np.ndarray:
        """B^H v for one image-shaped v -> (K,)."""
        v = np.asarray(v, dtype=np.complex128).reshape(1, -1)
        if self.B is not None:
            return _basis.dense_adjoint(self.B, v)[0]
        return _basis.tucker_adjoint(self.U, self.core, v)[0]

    def basis_adjoint(self, S: np.ndarray) -> np.ndarray:
        """B^H S_j for every row of S (J, N) -> (J, K)."""
        return np.stack([self.basis_adjoint_one(s) for s in np.asarray(S)])

    # --- F_s and F_s^H (Sec. II-A Eq. (1)) ------------------------------------------------
    def fs(self, m: np.ndarray) -> np.ndarray:
        """Undersampled Fourier operator of one image -> (M,)."""
        m = np.asarray(m, dtype=np.complex128).reshape(self.dims)
        if self.mask_idx is not None:
            return centred_dft(m, self.axes).reshape(-1)[self.mask_idx]
        if self.exact_ndft:
            return ndft(m, self.traj)
        return nufft_type2(m, self.traj, self.W, self.sigma, self.beta)

    def fs_adjoint(self, yj: np.ndarray) -> np.ndarray:
        """F_s^H of one coil's samples -> image-shaped array."""
        yj = np.asarray(yj, dtype=np.complex128)
        if self.mask_idx is not None:
            k = np.zeros(self.N, dtype=np.complex128)
            k[self.mask_idx] = yj
            return centred_idft(k.reshape(self.dims), self.axes)
        if self.exact_ndft:
            return ndft_adjoint(yj, self.traj, self.dims)
        return nufft_type1(yj, self.traj, self.dims, self.W, self.sigma, self.beta)

    # --- the operator (Sec. II-B Eq. (5)) --------------------------------------------------
    def encode(self, x: np.ndarray, c: np.ndarray) -> np.ndarray:
        """y (J, M) with y_j = F_s((B c_j) (.) x)."""
        x = np.asarray(x, dtype=np.complex128).reshape(self.dims)
        return np.stack([self.fs(self.coil_map(cj) * x) for cj in np.asarray(c)])

    def adjoint(self, x: np.ndarray, c: np.ndarray, y: np.ndarray):
        """Jacobian adjoint at (x, c) applied to y (J, M) -> (gx (N,), gc (J, K))."""
        x = np.asarray(x, dtype=np.complex128).reshape(self.dims)
        gx = np.zeros(self.dims, dtype=np.complex128)
        gc = []
        for cj, yj in zip(np.asarray(c), np.asarray(y)):
            g = self.fs_adjoint(yj)
            gx += np.conj(self.coil_map(cj)) * g
            gc.append(self.basis_adjoint_one(np.conj(x) * g))
        return gx.reshape(-1), np.stack(gc)

    def jvp(self, x: np.ndarray, c: np.ndarray, dx: np.ndarray, dc: np.ndarray) -> np.ndarray:
        """J[dx, dc] (Sec. II-B, Eq. (7)) -> (J, M)."""
        x = np.asarray(x, dtype=np.complex128).reshape(self.dims)
        dx = np.asarray(dx, dtype=np.complex128).reshape(self.dims)
        out = []
        for cj, dcj in zip(np.asarray(c), np.asarray(dc)):
            out.append(self.fs(self.coil_map(cj) * dx + x * self.coil_map(dcj)))
        return np.stack(out)

    def loss(self, x, c, y, w=None) -> float:
        """f = sum_j sum_m w_m |E_jm - y_jm|^2."""
        r = self.encode(x, c) - np.asarray(y, dtype=np.complex128)
        wr = np.ones(r.shape[1]) if w is None else np.asarray(w, dtype=np.float64)
        return float(np.sum(wr[None, :] * np.abs(r) ** 2))

    def loss_and_grad(self, x, c, y, w=None):
        """(f, gx, gc) with the packed real gradient 2 J^H (w (.) r)."""
        y = np.asarray(y, dtype=np.complex128)
        r = self.encode(x, c) - y
        wr = np.ones(r.shape[1]) if w is None else np.asarray(w, dtype=np.float64)
        f = float(np.sum(wr[None, :] * np.abs(r) ** 2))
        gx, gc = self.adjoint(x, c, 2.0 * wr[None, :] * r)
        return f, gx, gc


# ---- extra bilinear terms (multi-map), Sec. IV-A "Forward model extensions"
def multi_encode(op: Oracle, xs, cs) -> np.ndarray:
    """y_j = F_s( sum_m (B c_{m,j}) (.) x_m ) = sum_m E(x_m, c_m): one image and one set of
    coefficients per map set (F_s is linear)."""
    return sum(op.encode(x, c) for x, c in zip(xs, cs))


def multi_loss_and_grad(op: Oracle, xs, cs, y, w=None):
    """f = sum_j sum_m w_m |sum_maps E(x_i, c_i)_jm - y_jm|^2 and the packed real gradient
    2 J_i^H (w (.) r) with respect to every (x_i, c_i)."""
    y = np.asarray(y, dtype=np.complex128)
    r = multi_encode(op, xs, cs) - y
    wr = np.ones(r.shape[1]) if w is None else np.asarray(w, dtype=np.float64)
    f = float(np.sum(wr[None, :] * np.abs(r) ** 2))
    grads = [op.adjoint(x, c, 2.0 * wr[None, :] * r) for x, c in zip(xs, cs)]
    return f, [g[0] for g in grads], [g[1] for g in grads]
