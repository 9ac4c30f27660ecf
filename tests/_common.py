"""Shared helpers for the GPU parity tests (seeded problems, oracle references)."""
import math

import numpy as np

from oracle import Oracle
from synth import (coefficients, complex_normal, golden_angle_radial, phantom, ramp_dcf, rng_for,
                   smooth_dense_basis, tucker_basis, plane_mask_to_lines)

TOL = {"fp32": 1e-5, "bf16_split": 1e-4}


def c64(a):
    """Round to complex64 and back, so both sides see the same input values."""
    return np.asarray(a).astype(np.complex64).astype(np.complex128)


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128).reshape(-1)
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def maxrel(a, b, coils=False):
    """Largest max|a - b| / max|b|: per coil (rows of the leading axis) when coils, else over
    the whole tensor.  A coil whose reference is all zero is compared in absolute terms."""
    b = np.asarray(b, dtype=np.complex128)
    a = np.asarray(a, dtype=np.complex128).reshape(b.shape)
    if not coils or b.ndim == 0:
        a, b = a.reshape(1, -1), b.reshape(1, -1)
    else:
        a, b = a.reshape(b.shape[0], -1), b.reshape(b.shape[0], -1)
    if b.shape[1] == 0:
        return 0.0
    err = np.abs(a - b).max(axis=1)
    ref = np.abs(b).max(axis=1)
    return float(np.max(np.where(ref > 0, err / np.where(ref > 0, ref, 1.0), err)))


def assert_close(a, b, tol, coils=False, what=""):
    """Parity bar on an output: the relative L2 error over the whole tensor and the max-abs
    error relative to max|ref| (per coil for coil-indexed outputs) are both <= tol."""
    e2, em = rel(a, b), maxrel(a, b, coils)
    assert e2 <= tol and em <= tol, f"{what}: rel L2 {e2:.3e}, max-abs/max|ref| {em:.3e}, bar {tol:.0e}"
    return e2, em


class Case:
    """A seeded problem with complex64-rounded inputs and its FP64 oracle."""

    def __init__(self, seed, dims, J, K, basis="dense", ranks=None, mask="random", frac=0.35,
                 weights=False, degree=4, kmax=2.0, spokes=None, n_read=None, oversamp=2.0, kb_width=6):
        self.dims = tuple(dims)
        self.oversamp, self.kb_width = float(oversamp), int(kb_width)
        self.N = int(np.prod(dims))
        self.J, self.K = J, K
        rb = rng_for(seed, 2)
        if basis == "dense":
            self.B = c64(smooth_dense_basis(rb, dims, K, degree, kmax))
            self.U = self.core = None
        else:
            U, core = tucker_basis(rb, dims, ranks, K, degree, kmax)
            self.U = [c64(u) for u in U]
            self.core = c64(core)
            self.B = None
        rs = rng_for(seed, 4)
        self.traj = None
        if not isinstance(mask, str):
            self.mask = np.asarray(mask, dtype=np.int64)
        elif mask == "radial":
            nr = n_read if n_read is not None else 2 * max(dims)
            # both sides see the float32-rounded trajectory
            self.traj = golden_angle_radial(dims, spokes, nr).astype(np.float32).astype(np.float64)
            self.mask = None
            self.M = self.traj.shape[0]
            self.w = ramp_dcf(self.traj, dims, nr).astype(np.float32).astype(np.float64) if weights else None
        elif mask == "random":
            M = int(round(frac * self.N))
            self.mask = np.sort(rs.choice(self.N, size=M, replace=False)).astype(np.int64)
        elif mask == "lines3d":
            plane = rs.uniform(size=dims[:2]) < frac
            self.mask = plane_mask_to_lines(plane, dims[2])
        elif mask == "full":
            self.mask = np.arange(self.N, dtype=np.int64)
        elif mask == "empty":
            self.mask = np.zeros(0, dtype=np.int64)
        else:
            raise ValueError(mask)
        if self.traj is None:
            self.M = int(self.mask.size)
            self.w = rs.uniform(0.2, 1.0, size=self.M).astype(np.float32).astype(np.float64) if weights else None
        self.x_true = c64(phantom(rng_for(seed, 1), dims))
        self.c_true = c64(coefficients(rng_for(seed, 3), J, K))
        re = rng_for(seed, 6)
        self.x0 = c64(phantom(re, dims) + 0.1 * complex_normal(re, dims))
        self.c0 = c64(coefficients(re, J, K))
        self.op = Oracle(dims, B=self.B, U=self.U, core=self.core, mask_idx=self.mask, traj=self.traj,
                         kb_width=self.kb_width, oversamp=self.oversamp)
        y_clean = self.op.encode(self.x_true, self.c_true)
        noise = complex_normal(rng_for(seed, 5), (J, self.M))
        scale = 0.01 * np.linalg.norm(y_clean) / max(np.linalg.norm(noise), 1e-300)
        self.y = c64(y_clean + scale * noise)

    def plan(self, precision="fp32"):
        from paper_2008_09042_amd.encoding import MaxwellPlan
        kw = dict(mask_idx=self.mask, traj=self.traj, weights=self.w, precision=precision)
        if self.traj is not None:
            kw.update(kb_width=self.kb_width, oversamp=self.oversamp)
        if self.B is not None:
            return MaxwellPlan(self.dims, self.J, B=self.B, **kw)
        return MaxwellPlan(self.dims, self.J, U=self.U, core=self.core, **kw)
