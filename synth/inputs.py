"""Seeded input generators (NumPy, FP64).

Every random draw comes from ``rng_for(seed, role)``, a
``numpy.random.Generator`` seeded by ``SeedSequence([seed, role])``, so the
same (seed, role) pair always yields the same data on any machine; each
workload carries its own seed.

Roles: 1 phantom, 2 basis, 3 true coefficients, 4 mask / trajectory,
5 noise, 6 evaluation point (x0, c0), 7 finite-difference directions.

Conventions shared with both consumers (they are data conventions, not
arithmetic of the method):

* images are C-order arrays, the last axis fastest;
* pixel coordinate along an axis of length n is r = (i - n/2)/n in [-1/2, 1/2);
* a Cartesian mask is a sorted array of unique int64 linear indices into the
  centred k-space grid (k-space index i <-> frequency i - n/2);
* a non-Cartesian trajectory is an (M, ndim) float64 array in cycles/FOV,
  column d paired with image axis d;
* "complex N(0,1)" has E|z|^2 = 1 (real and imaginary parts each N(0, 1/2)).
"""
from __future__ import annotations

import ctypes
import dataclasses
import itertools
import math
import os
import subprocess
from typing import List, Optional, Sequence, Tuple

import numpy as np

ROLE_PHANTOM = 1
ROLE_BASIS = 2
ROLE_CTRUE = 3
ROLE_SAMPLING = 4
ROLE_NOISE = 5
ROLE_EVAL = 6
ROLE_DIRECTIONS = 7

__all__ = [
    "ROLE_PHANTOM", "ROLE_BASIS", "ROLE_CTRUE", "ROLE_SAMPLING", "ROLE_NOISE",
    "ROLE_EVAL", "ROLE_DIRECTIONS",
    "rng_for", "complex_normal", "pixel_coords", "phantom", "smooth_dense_basis",
    "smooth_factor", "tucker_basis", "coefficients", "line_mask", "poisson_disc_plane",
    "plane_mask_to_lines", "plane_mask_to_indices", "golden_angle_radial", "ramp_dcf",
    "unit_noise", "noise_scale_for_snr", "Problem", "make_problem", "problem", "WORKLOADS",
    "BATCH", "slice_rng", "slice_problems", "build_native", "smooth_params",
]


def rng_for(seed: int, role: int) -> np.random.Generator:
    """Generator for one (seed, role) pair."""
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(role)]))


def complex_normal(rng: np.random.Generator, shape) -> np.ndarray:
    """Complex Gaussian with E|z|^2 = 1."""
    s = math.sqrt(0.5)
    return rng.normal(0.0, s, size=shape) + 1j * rng.normal(0.0, s, size=shape)


def pixel_coords(dims: Sequence[int]) -> List[np.ndarray]:
    """Broadcastable per-axis coordinates r_d = (i - n_d/2)/n_d."""
    out = []
    nd = len(dims)
    for d, n in enumerate(dims):
        shape = [1] * nd
        shape[d] = n
        out.append(((np.arange(n) - n // 2) / n).reshape(shape))
    return out


def _rotation(rng: np.random.Generator, nd: int) -> np.ndarray:
    if nd == 1:
        return np.ones((1, 1))
    if nd == 2:
        t = rng.uniform(0.0, math.pi)
        c, s = math.cos(t), math.sin(t)
        return np.array([[c, -s], [s, c]])
    a, b, g = rng.uniform(0.0, math.pi, size=3)

    def rz(t):
        c, s = math.cos(t), math.sin(t)
        return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])

    def ry(t):
        c, s = math.cos(t), math.sin(t)
        return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])

    return rz(a) @ ry(b) @ rz(g)


def _monomial_exponents(nd: int, degree: int) -> List[Tuple[int, ...]]:
    exps = [e for e in itertools.product(range(degree + 1), repeat=nd) if sum(e) <= degree]
    exps.sort(key=lambda e: (sum(e), e))
    return exps


def phantom(rng: np.random.Generator, dims: Sequence[int], n_ellipses: int = 10) -> np.ndarray:
    """Sum of random ellipses (ellipsoids in 3D) with a smooth random phase.

    Centres U(-0.35, 0.35), semi-axes U(0.05, 0.35), random rotation, additive
    magnitudes U(0.1, 1).  The phase is exp(i*phi) with phi a random degree-2
    polynomial in the pixel coordinates scaled so that max|phi| = pi.
    """
    dims = tuple(int(n) for n in dims)
    nd = len(dims)
    coords = pixel_coords(dims)
    mag = np.zeros(dims)
    for _ in range(n_ellipses):
        centre = rng.uniform(-0.35, 0.35, size=nd)
        axes = rng.uniform(0.05, 0.35, size=nd)
        rot = _rotation(rng, nd)
        amp = rng.uniform(0.1, 1.0)
        rel = [coords[d] - centre[d] for d in range(nd)]
        q = np.zeros(dims)
        for a in range(nd):
            # component a of rot^T (r - centre)
            comp = sum(rot[b, a] * rel[b] for b in range(nd))
            q = q + (comp / axes[a]) ** 2
        mag = mag + amp * (q <= 1.0)
    phi = np.zeros(dims)
    for e in _monomial_exponents(nd, 2):
        term = rng.normal()
        for d in range(nd):
            term = term * (2.0 * coords[d]) ** e[d]
        phi = phi + term
    peak = np.max(np.abs(phi))
    if peak > 0:
        phi = phi * (math.pi / peak)
    return mag * np.exp(1j * phi)


def smooth_params(rng: np.random.Generator, nd: int, ncols: int, degree: int, kmax: float):
    """Random parameters of the smooth columns: (monomial exponents, complex coefficients
    (n_monomials, ncols), wave vectors (ncols, nd) uniform in the ball |k| <= kmax)."""
    exps = _monomial_exponents(nd, degree)
    coef = complex_normal(rng, (len(exps), ncols))
    dirs = rng.normal(size=(ncols, nd))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    rad = kmax * rng.uniform(0.0, 1.0, size=ncols) ** (1.0 / nd)
    return exps, coef, dirs * rad[:, None]


def _smooth_columns(rng: np.random.Generator, dims: Sequence[int], ncols: int,
                    degree: int, kmax: float) -> np.ndarray:
    """Columns poly_q(2r) * exp(2 pi i k_q . r), flattened C-order, shape (N, ncols).

    poly_q has every monomial of total degree <= degree with complex N(0,1)
    coefficients; k_q is uniform in the ball |k| <= kmax (cycles/FOV).
    """
    dims = tuple(int(n) for n in dims)
    nd = len(dims)
    N = int(np.prod(dims))
    coords = [c.reshape(-1) for c in np.meshgrid(*[(np.arange(n) - n // 2) / n for n in dims],
                                                 indexing="ij")]
    exps, coef, kvec = smooth_params(rng, nd, ncols, degree, kmax)
    mono = np.empty((N, len(exps)))
    for t, e in enumerate(exps):
        v = np.ones(N)
        for d in range(nd):
            if e[d]:
                v = v * (2.0 * coords[d]) ** e[d]
        mono[:, t] = v
    phase = np.zeros((N, ncols))
    for d in range(nd):
        phase += np.outer(coords[d], kvec[:, d])
    return (mono @ coef) * np.exp(2j * math.pi * phase)


def _orthonormalise(a: np.ndarray) -> np.ndarray:
    q, _ = np.linalg.qr(a, mode="reduced")
    return q


def smooth_dense_basis(rng: np.random.Generator, dims: Sequence[int], K: int,
                       degree: int, kmax: float) -> np.ndarray:
    """Orthonormal (N, K) complex128 basis of smooth fields (Householder QR)."""
    return _orthonormalise(_smooth_columns(rng, dims, K, degree, kmax))


def smooth_factor(rng: np.random.Generator, n: int, r: int, degree: int, kmax: float) -> np.ndarray:
    """Orthonormal (n, r) factor matrix built from 1D smooth fields."""
    return _orthonormalise(_smooth_columns(rng, (n,), r, degree, kmax))


def tucker_basis(rng: np.random.Generator, dims: Sequence[int], ranks: Sequence[int], K: int,
                 degree: int = 6, kmax: float = 3.0):
    """Tucker-factored orthonormal basis.

    Returns (U, core): U[m] is (n_m, r_m) with orthonormal columns; core is
    (r_0, r_1, r_2, K) whose mode-4 unfolding (r0 r1 r2, K) has orthonormal
    columns, so the materialised basis has orthonormal columns too.
    """
    U = [smooth_factor(rng, int(n), int(r), degree, kmax) for n, r in zip(dims, ranks)]
    R = int(np.prod(ranks))
    if K > R:
        raise ValueError("K must not exceed r0*r1*r2 for an orthonormal core")
    core = _orthonormalise(complex_normal(rng, (R, K))).reshape(*[int(r) for r in ranks], K)
    return U, core


def coefficients(rng: np.random.Generator, J: int, K: int) -> np.ndarray:
    """c_j ~ complex N(0,1)/sqrt(K), shape (J, K)."""
    return complex_normal(rng, (J, K)) / math.sqrt(K)


def line_mask(dims: Sequence[int], step: int, centre: int) -> np.ndarray:
    """Uniform lines along the last axis: rows i of axis 0 with (i - n0/2) % step == 0
    or |i - n0/2| within the centre band [n0/2 - centre/2, n0/2 + centre/2).  2D only."""
    n0, n1 = int(dims[0]), int(dims[1])
    rows = [i for i in range(n0)
            if (i - n0 // 2) % step == 0 or (n0 // 2 - centre // 2 <= i < n0 // 2 + centre // 2)]
    rows = np.array(rows, dtype=np.int64)
    return (rows[:, None] * n1 + np.arange(n1, dtype=np.int64)[None, :]).reshape(-1)


_PD_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpdisc.so")
_pd_lib = None


def build_native() -> str:
    """Compile the dart-throwing helper (pdisc.c) next to this file with the host compiler."""
    src = os.path.join(os.path.dirname(_PD_LIB), "pdisc.c")
    tmp = _PD_LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, src, "-lm"], check=True)
    os.replace(tmp, _PD_LIB)
    return _PD_LIB


def _pd_native():
    global _pd_lib
    if _pd_lib is None and os.path.exists(_PD_LIB):
        lib = ctypes.CDLL(_PD_LIB)
        lib.pd_throw.restype = ctypes.c_int64
        lib.pd_throw.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        _pd_lib = lib
    return _pd_lib


def _pd_throw_native(cen: np.ndarray, ii: np.ndarray, jj: np.ndarray, dmin: np.ndarray) -> List[int]:
    occ = np.ascontiguousarray(cen, dtype=np.uint8)
    i32 = np.ascontiguousarray(ii, dtype=np.int32)
    j32 = np.ascontiguousarray(jj, dtype=np.int32)
    d64 = np.ascontiguousarray(dmin, dtype=np.float64)
    acc = np.empty(i32.size, dtype=np.int64)
    n = _pd_native().pd_throw(cen.shape[0], cen.shape[1], occ.ctypes.data, i32.size, i32.ctypes.data,
                              j32.ctypes.data, d64.ctypes.data, acc.ctypes.data)
    if n < 0:
        raise MemoryError("pd_throw")
    return acc[:n].tolist()


def poisson_disc_plane(rng: np.random.Generator, shape: Sequence[int], R: float,
                       centre: int, native: Optional[bool] = None) -> np.ndarray:
    """Variable-density Poisson-disc mask over a 2D plane (boolean array).

    The centre ``centre x centre`` block is fully sampled.  Other points are
    accepted by dart throwing over a seeded random order of all grid points:
    a candidate at normalised radius rho in [0, 1] is accepted if no accepted
    point lies within s*(1 + 3*rho) grid cells.  The scale s is found by
    bisection so that at least round(n0*n1/R) points (centre included) are
    accepted; the first accepted points in acceptance order are kept to hit
    that count exactly.

    The acceptance pass runs in the C helper (pdisc.c) when it is built, else in the loop
    below; both give the same mask.  native=False forces the loop, native=True the helper.
    """
    use_native = (_pd_native() is not None) if native is None else bool(native)
    if use_native and _pd_native() is None:
        raise RuntimeError("libpdisc.so is not built (synth.build_native())")
    n0, n1 = int(shape[0]), int(shape[1])
    target = int(round(n0 * n1 / R))
    cen = np.zeros((n0, n1), dtype=bool)
    cen[n0 // 2 - centre // 2: n0 // 2 - centre // 2 + centre,
        n1 // 2 - centre // 2: n1 // 2 - centre // 2 + centre] = True
    ncen = int(cen.sum())
    if target <= ncen:
        return cen
    order = rng.permutation(n0 * n1)
    ii, jj = np.divmod(order, n1)
    keep = ~cen[ii, jj]
    ii, jj = ii[keep], jj[keep]
    rho = np.sqrt(((ii - n0 // 2) / (n0 / 2.0)) ** 2 + ((jj - n1 // 2) / (n1 / 2.0)) ** 2) / math.sqrt(2.0)

    def throw(s: float):
        dmin = s * (1.0 + 3.0 * rho)
        if use_native:
            return _pd_throw_native(cen, ii, jj, dmin)
        occ = cen.copy()
        acc = []
        for t in range(ii.size):
            i, j, d = int(ii[t]), int(jj[t]), float(dmin[t])
            w = int(math.ceil(d))
            i0, i1 = max(0, i - w), min(n0, i + w + 1)
            j0, j1 = max(0, j - w), min(n1, j + w + 1)
            win = occ[i0:i1, j0:j1]
            if win.any():
                pi, pj = np.nonzero(win)
                if np.any((pi + i0 - i) ** 2 + (pj + j0 - j) ** 2 < d * d):
                    continue
            occ[i, j] = True
            acc.append(t)
        return acc

    need = target - ncen
    lo, hi = 0.0, 8.0
    acc_lo = throw(lo)  # s = 0 accepts every candidate
    for _ in range(12):
        mid = 0.5 * (lo + hi)
        acc = throw(mid)
        if len(acc) >= need:
            lo, acc_lo = mid, acc
        else:
            hi = mid
    mask = cen.copy()
    sel = np.array(acc_lo[:need], dtype=np.int64)
    mask[ii[sel], jj[sel]] = True
    return mask


def plane_mask_to_lines(plane: np.ndarray, n_last: int) -> np.ndarray:
    """3D Cartesian mask: full lines along the last axis at every sampled (k0, k1)."""
    k0, k1 = np.nonzero(plane)
    base = (k0.astype(np.int64) * plane.shape[1] + k1) * n_last
    idx = base[:, None] + np.arange(n_last, dtype=np.int64)[None, :]
    return np.sort(idx.reshape(-1))


def plane_mask_to_indices(plane: np.ndarray) -> np.ndarray:
    """2D Cartesian mask over the whole plane: sorted linear indices."""
    return np.flatnonzero(plane.reshape(-1)).astype(np.int64)


def golden_angle_radial(dims: Sequence[int], n_spokes: int, n_read: Optional[int] = None) -> np.ndarray:
    """Golden-angle radial trajectory, layout [spoke][readout], (M, 2) cycles/FOV.

    k_{s,m} = (m - n_read/2) * (n_d / n_read) * (sin t_s, cos t_s) per axis (axis 0, axis 1),
    t_s = s * pi * (sqrt(5) - 1)/2 mod pi, so the readout spans [-n_d/2, n_d/2).
    Deterministic (no random draw).
    """
    n0, n1 = int(dims[0]), int(dims[1])
    if n_read is None:
        n_read = 2 * max(n0, n1)
    ga = math.pi * (math.sqrt(5.0) - 1.0) / 2.0
    theta = np.mod(np.arange(n_spokes) * ga, math.pi)
    m = np.arange(n_read) - n_read // 2
    k0 = (m[None, :] * (n0 / n_read)) * np.sin(theta)[:, None]
    k1 = (m[None, :] * (n1 / n_read)) * np.cos(theta)[:, None]
    return np.stack([k0.reshape(-1), k1.reshape(-1)], axis=1)


def ramp_dcf(traj: np.ndarray, dims: Sequence[int], n_read: int) -> np.ndarray:
    """Ramp density compensation |k| (k normalised per axis to cycles of the
    largest axis); the DC sample gets dk/4, its Voronoi share of the central
    disc.  Normalised to max 1."""
    scale = np.array([max(dims) / n for n in dims], dtype=np.float64)
    kk = np.linalg.norm(traj * scale[None, :], axis=1)
    dk = max(dims) / n_read
    w = kk.copy()
    w[kk == 0.0] = dk / 4.0
    return w / w.max()


def unit_noise(rng: np.random.Generator, J: int, M: int) -> np.ndarray:
    """White complex Gaussian noise, shape (J, M), E|n|^2 = 1."""
    return complex_normal(rng, (J, M))


def noise_scale_for_snr(y_clean: np.ndarray, noise: np.ndarray, snr_db: float) -> float:
    """Factor a such that ||a*noise|| = 10^(-snr/20) ||y_clean|| over all coils."""
    return float(10.0 ** (-snr_db / 20.0) * np.linalg.norm(y_clean) / np.linalg.norm(noise))


@dataclasses.dataclass
class Problem:
    """One seeded problem instance (FP64 / complex128 arrays)."""

    name: str
    dims: Tuple[int, ...]
    J: int
    K: int
    basis_kind: str                      # "dense" or "tucker"
    B: Optional[np.ndarray] = None       # (N, K) dense basis
    U: Optional[List[np.ndarray]] = None  # Tucker factors (n_m, r_m)
    core: Optional[np.ndarray] = None    # (r0, r1, r2, K)
    sampling: str = "cartesian"          # or "radial"
    mask_idx: Optional[np.ndarray] = None  # sorted int64 linear indices
    traj: Optional[np.ndarray] = None    # (M, ndim) cycles/FOV
    weights: Optional[np.ndarray] = None  # (M,) or None
    kb_width: int = 6
    oversamp: float = 2.0
    x_true: Optional[np.ndarray] = None
    c_true: Optional[np.ndarray] = None
    noise: Optional[np.ndarray] = None   # unit noise (J, M)
    snr_db: float = 40.0
    x0: Optional[np.ndarray] = None
    c0: Optional[np.ndarray] = None
    basis_params: Optional[tuple] = None  # (exponents, coef, kvec) when not materialised

    @property
    def N(self) -> int:
        return int(np.prod(self.dims))

    @property
    def M(self) -> int:
        if self.sampling == "cartesian":
            return int(self.mask_idx.size)
        return int(self.traj.shape[0])


def make_problem(seed: int, name: str, dims, J: int, K: int, basis_kind: str = "dense",
                 degree: int = 6, kmax: float = 3.0, ranks=None, sampling: str = "cartesian",
                 mask: str = "lines", R: float = 4.0, centre: int = 16, n_spokes: int = 64,
                 n_read: Optional[int] = None, snr_db: float = 40.0) -> Problem:
    """Draw every input of one problem from the seeded generators."""
    dims = tuple(int(n) for n in dims)
    p = Problem(name=name, dims=dims, J=J, K=K, basis_kind=basis_kind, sampling=sampling,
                snr_db=snr_db)
    rb = rng_for(seed, ROLE_BASIS)
    if basis_kind == "dense":
        p.B = smooth_dense_basis(rb, dims, K, degree, kmax)
    else:
        p.U, p.core = tucker_basis(rb, dims, ranks, K, degree, kmax)
    rs = rng_for(seed, ROLE_SAMPLING)
    if sampling == "cartesian":
        if mask == "lines":
            p.mask_idx = line_mask(dims, int(R), centre)
        elif mask == "pd2d":
            p.mask_idx = plane_mask_to_indices(poisson_disc_plane(rs, dims, R, centre))
        elif mask == "pd3d":
            plane = poisson_disc_plane(rs, dims[:2], R, centre)
            p.mask_idx = plane_mask_to_lines(plane, dims[2])
        elif mask == "full":
            p.mask_idx = np.arange(p.N, dtype=np.int64)
        else:
            raise ValueError(mask)
    else:
        nr = n_read if n_read is not None else 2 * max(dims)
        p.traj = golden_angle_radial(dims, n_spokes, nr)
        p.weights = ramp_dcf(p.traj, dims, nr)
    p.x_true = phantom(rng_for(seed, ROLE_PHANTOM), dims)
    p.c_true = coefficients(rng_for(seed, ROLE_CTRUE), J, K)
    p.noise = unit_noise(rng_for(seed, ROLE_NOISE), J, p.M)
    re = rng_for(seed, ROLE_EVAL)
    p.x0 = phantom(re, dims)
    p.c0 = coefficients(re, J, K)
    return p


# The single-problem workloads by name (image, basis, coils), each with its own seed; each
# entry is the keyword set for make_problem.
WORKLOADS = {w["name"]: w for w in (
    dict(seed=1, name="cart2d_64_dense32_j8", dims=(64, 64), J=8, K=32, basis_kind="dense",
         degree=6, kmax=3.0, sampling="cartesian", mask="lines", R=4, centre=16),
    dict(seed=2, name="cart2d_256_dense200_j32", dims=(256, 256), J=32, K=200, basis_kind="dense",
         degree=10, kmax=5.0, sampling="cartesian", mask="pd2d", R=6.0, centre=24),
    dict(seed=3, name="radial2d_256_dense128_j16", dims=(256, 256), J=16, K=128, basis_kind="dense",
         degree=10, kmax=5.0, sampling="radial", n_spokes=64, n_read=512),
    dict(seed=4, name="cart3d_128_tucker40x300_j32", dims=(128, 128, 128), J=32, K=300,
         basis_kind="tucker", ranks=(40, 40, 40), degree=6, kmax=3.0, sampling="cartesian",
         mask="pd3d", R=8.0, centre=20),
    # coil stacks of 268 MB (above the 256 MB last-level cache), for the bandwidth of the axis
    # FFT passes and the gridding when their arrays stream from HBM
    dict(seed=6, name="cart2d_512_dense16_j128", dims=(512, 512), J=128, K=16, basis_kind="dense",
         degree=10, kmax=5.0, sampling="cartesian", mask="pd2d", R=6.0, centre=48),
    dict(seed=7, name="radial2d_256_dense32_j128", dims=(256, 256), J=128, K=32, basis_kind="dense",
         degree=10, kmax=5.0, sampling="radial", n_spokes=64, n_read=512),
)}


def problem(name: str) -> Problem:
    """The named workload's seeded problem."""
    return make_problem(**WORKLOADS[name])


# ---------------------------------------------------------------- batched slices
# Many independent 2D problems of uneven sizes, each with its own dense basis, coils and
# sampling (the batched serving form).  Slice i draws everything from
# SeedSequence([seed, role, i]).  Bases follow the single-problem recipe (smooth columns of
# degree <= 10 and |k| <= 5, QR-orthonormalised); Cartesian slices take a variable-density
# Poisson-disc mask with a fully sampled centre of max(16, n/10)^2.  With
# materialise_basis=False only the basis parameters are drawn (p.basis_params), so that a
# caller can evaluate the columns and their QR elsewhere (64 bases of up to 102,400 x 256
# take minutes of host time).
BATCH = dict(name="batch64_slices_dense", n_slices=64, sizes=(128, 192, 256, 320), Js=(8, 16, 32),
             Ks=(64, 128, 256), degree=10, kmax=5.0)


def slice_rng(seed: int, role: int, i: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(role), int(i)]))


def slice_problems(seed: int = 5, n_slices: int = 64, sizes=BATCH["sizes"], Js=BATCH["Js"],
                   Ks=BATCH["Ks"], spokes=(32, 128), materialise_basis: bool = True) -> List[Problem]:
    """The batched-slices workload: n_slices seeded 2D problems (see the block comment)."""
    out = []
    for i in range(n_slices):
        rp = slice_rng(seed, ROLE_SAMPLING, i)
        dims = (int(rp.choice(sizes)), int(rp.choice(sizes)))
        J, K = int(rp.choice(Js)), int(rp.choice(Ks))
        cart = bool(rp.uniform() < 0.5)
        p = Problem(name=f"slice{i}", dims=dims, J=J, K=K, basis_kind="dense",
                    sampling="cartesian" if cart else "radial")
        rb = slice_rng(seed, ROLE_BASIS, i)
        if materialise_basis:
            p.B = smooth_dense_basis(rb, dims, K, BATCH["degree"], BATCH["kmax"])
        else:
            p.basis_params = smooth_params(rb, 2, K, BATCH["degree"], BATCH["kmax"])
        if cart:
            R = float(rp.uniform(3.0, 8.0))
            plane = poisson_disc_plane(rp, dims, R, max(16, max(dims) // 10))
            p.mask_idx = plane_mask_to_indices(plane)
        else:
            ns = int(rp.integers(spokes[0], spokes[1] + 1))
            nr = 2 * max(dims)
            p.traj = golden_angle_radial(dims, ns, nr)
            p.weights = ramp_dcf(p.traj, dims, nr)
        p.x_true = phantom(slice_rng(seed, ROLE_PHANTOM, i), dims)
        p.c_true = coefficients(slice_rng(seed, ROLE_CTRUE, i), J, K)
        p.noise = unit_noise(slice_rng(seed, ROLE_NOISE, i), J, p.M)
        re = slice_rng(seed, ROLE_EVAL, i)
        p.x0 = phantom(re, dims)
        p.c0 = coefficients(re, J, K)
        out.append(p)
    return out
