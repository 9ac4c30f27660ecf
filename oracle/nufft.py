"""Non-Cartesian Fourier operator (oracle; test infrastructure only).

The paper applies the same formulation to radial sampling once the
non-Cartesian operator F is available (Sec. III-B) but does not say how F is
computed.  Its plain definition is the non-uniform DFT (NDFT)

    y_m = N^{-1/2} sum_r x_r exp(-2 pi i k_m . r / n)      (k in cycles/FOV)

and the method approximates it with a Kaiser-Bessel (KB) NUFFT.  Both are
written out here; the NUFFT follows the standard gridding steps in FP64:

  type 2 (image -> samples)
    (i)   divide each pixel by the KB deapodisation Phi(r_d / (sigma n_d)) (product over axes)
    (ii)  zero-pad, centred, to the oversampled grid sigma*n
    (iii) centred DFT on that grid, unnormalised
    (iv)  per sample, u = sigma k; W taps per axis starting at ceil(u - W/2);
          weight prod_d phi(u_d - g_d); grid index (g + sigma n/2) mod sigma n
    (v)   multiply by N^{-1/2}
  type 1 is the exact transpose of (i)-(v).

Kernel phi(t) = I0(beta sqrt(1 - (2t/W)^2)) / W on |t| <= W/2, whose Fourier
transform is Phi(nu) = sinh(sqrt(beta^2 - (pi W nu)^2)) / sqrt(beta^2 - (pi W nu)^2)
(the sin form when the radicand is negative).  beta follows Beatty, Nishimura
and Pauly (2005): beta = pi sqrt((W/sigma)^2 (sigma - 1/2)^2 - 0.8).
"""
import math
from typing import Sequence

import numpy as np
import scipy.fft
from scipy.special import i0


def kb_beta(W: int, sigma: float) -> float:
    """Beatty-Nishimura-Pauly shape parameter."""
    return math.pi * math.sqrt((W / sigma) ** 2 * (sigma - 0.5) ** 2 - 0.8)


def kb_kernel(t: np.ndarray, W: int, beta: float) -> np.ndarray:
    """phi(t) = I0(beta sqrt(1 - (2t/W)^2)) / W, zero outside |t| <= W/2."""
    t = np.asarray(t, dtype=np.float64)
    arg = 1.0 - (2.0 * t / W) ** 2
    out = np.where(arg >= 0.0, i0(beta * np.sqrt(np.clip(arg, 0.0, None))) / W, 0.0)
    return out


def kb_deapod(nu: np.ndarray, W: int, beta: float) -> np.ndarray:
    """Phi(nu), the continuous Fourier transform of phi."""
    nu = np.asarray(nu, dtype=np.float64)
    z2 = beta ** 2 - (math.pi * W * nu) ** 2
    out = np.empty_like(nu)
    pos = z2 > 0
    zp = np.sqrt(z2[pos])
    out[pos] = np.sinh(zp) / zp
    neg = z2 < 0
    zn = np.sqrt(-z2[neg])
    out[neg] = np.sin(zn) / zn
    out[z2 == 0] = 1.0
    return out


def _deapod_image(dims: Sequence[int], W: int, sigma: float, beta: float) -> np.ndarray:
    phi = np.ones(tuple(dims))
    nd = len(dims)
    for d, n in enumerate(dims):
        r = np.arange(n) - n // 2
        shape = [1] * nd
        shape[d] = n
        phi = phi * kb_deapod(r / (sigma * n), W, beta).reshape(shape)
    return phi


def _grid_dims(dims, sigma):
    g = tuple(int(round(sigma * n)) for n in dims)
    for a, b in zip(g, dims):
        if a % 2 or abs(a - sigma * b) > 1e-9:
            raise ValueError("sigma * n must be an even integer")
    return g


def _taps(traj: np.ndarray, gdims, W: int, sigma: float, beta: float):
    """Per axis: (M, W) wrapped grid indices and (M, W) kernel weights."""
    idx, wts = [], []
    for d, G in enumerate(gdims):
        u = sigma * traj[:, d]
        g0 = np.ceil(u - W / 2.0)
        g = g0[:, None] + np.arange(W)[None, :]
        wts.append(kb_kernel(u[:, None] - g, W, beta))
        idx.append(np.mod(g.astype(np.int64) + G // 2, G))
    return idx, wts


def nufft_type2(img: np.ndarray, traj: np.ndarray, W: int = 6, sigma: float = 2.0,
                beta: float = None) -> np.ndarray:
    """KB NUFFT image -> samples, steps (i)-(v).  img (n0, n1[, n2]); traj (M, ndim)."""
    img = np.asarray(img, dtype=np.complex128)
    dims = img.shape
    nd = len(dims)
    if beta is None:
        beta = kb_beta(W, sigma)
    N = int(np.prod(dims))
    gdims = _grid_dims(dims, sigma)
    # (i) deapodise
    pre = img / _deapod_image(dims, W, sigma, beta)
    # (ii) centred zero-pad
    pad = np.zeros(gdims, dtype=np.complex128)
    sl = tuple(slice(G // 2 - n // 2, G // 2 - n // 2 + n) for G, n in zip(gdims, dims))
    pad[sl] = pre
    # (iii) centred DFT, unnormalised
    axes = tuple(range(nd))
    grid = scipy.fft.fftshift(scipy.fft.fftn(scipy.fft.ifftshift(pad, axes=axes), axes=axes), axes=axes)
    # (iv) interpolate
    idx, wts = _taps(np.asarray(traj, dtype=np.float64), gdims, W, sigma, beta)
    M = traj.shape[0]
    y = np.zeros(M, dtype=np.complex128)
    for t in np.ndindex(*([W] * nd)):
        lin = np.zeros(M, dtype=np.int64)
        w = np.ones(M)
        for d in range(nd):
            lin = lin * gdims[d] + idx[d][:, t[d]]
            w = w * wts[d][:, t[d]]
        y += w * grid.reshape(-1)[lin]
    # (v) scale
    return y / math.sqrt(N)


def nufft_type1(y: np.ndarray, traj: np.ndarray, dims: Sequence[int], W: int = 6,
                sigma: float = 2.0, beta: float = None) -> np.ndarray:
    """Exact transpose (adjoint) of nufft_type2: samples -> image."""
    y = np.asarray(y, dtype=np.complex128)
    dims = tuple(int(n) for n in dims)
    nd = len(dims)
    if beta is None:
        beta = kb_beta(W, sigma)
    N = int(np.prod(dims))
    gdims = _grid_dims(dims, sigma)
    Gtot = int(np.prod(gdims))
    # adjoint of (v) and (iv): spread
    idx, wts = _taps(np.asarray(traj, dtype=np.float64), gdims, W, sigma, beta)
    M = traj.shape[0]
    ys = y / math.sqrt(N)
    gre = np.zeros(Gtot)
    gim = np.zeros(Gtot)
    for t in np.ndindex(*([W] * nd)):
        lin = np.zeros(M, dtype=np.int64)
        w = np.ones(M)
        for d in range(nd):
            lin = lin * gdims[d] + idx[d][:, t[d]]
            w = w * wts[d][:, t[d]]
        gre += np.bincount(lin, weights=w * ys.real, minlength=Gtot)
        gim += np.bincount(lin, weights=w * ys.imag, minlength=Gtot)
    grid = (gre + 1j * gim).reshape(gdims)
    # adjoint of (iii): the conjugate-transposed unnormalised DFT = Gtot * inverse DFT
    axes = tuple(range(nd))
    pad = scipy.fft.fftshift(scipy.fft.ifftn(scipy.fft.ifftshift(grid, axes=axes), axes=axes),
                          axes=axes) * Gtot
    # adjoint of (ii): crop
    sl = tuple(slice(G // 2 - n // 2, G // 2 - n // 2 + n) for G, n in zip(gdims, dims))
    img = pad[sl]
    # adjoint of (i): divide by the (real) deapodisation
    return img / _deapod_image(dims, W, sigma, beta)


def _phase_matrix(traj: np.ndarray, dims: Sequence[int]) -> np.ndarray:
    dims = tuple(int(n) for n in dims)
    grids = np.meshgrid(*[np.arange(n) - n // 2 for n in dims], indexing="ij")
    arg = np.zeros((traj.shape[0], int(np.prod(dims))))
    for d, n in enumerate(dims):
        arg += np.outer(traj[:, d], grids[d].reshape(-1) / n)
    return np.exp(-2j * math.pi * arg)


def ndft(img: np.ndarray, traj: np.ndarray) -> np.ndarray:
    """Exact non-uniform DFT (the plain definition); small sizes only."""
    img = np.asarray(img, dtype=np.complex128)
    return _phase_matrix(np.asarray(traj, dtype=np.float64), img.shape) @ img.reshape(-1) \
        / math.sqrt(img.size)


def ndft_adjoint(y: np.ndarray, traj: np.ndarray, dims: Sequence[int]) -> np.ndarray:
    """Adjoint of the exact NDFT; small sizes only."""
    dims = tuple(int(n) for n in dims)
    A = _phase_matrix(np.asarray(traj, dtype=np.float64), dims)
    return (A.conj().T @ np.asarray(y, dtype=np.complex128)).reshape(dims) / math.sqrt(np.prod(dims))
