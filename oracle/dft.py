"""Centred unitary DFT (oracle; test infrastructure only).

The paper writes the undersampled Fourier operator F_s (Sec. II-A, Eq. (1))
and the DFT matrix (Sec. II-B, NLINV regulariser) without fixing the
normalisation or the index convention.  Readings used here:

* unitary normalisation N^{-1/2} in both directions;
* centred indices: for an axis of length n (even), pixel r and frequency k
  both run over [-n/2, n/2), stored at array index (value + n/2);
* forward kernel exp(-2 pi i k r / n), inverse exp(+2 pi i k r / n).

Written as SciPy's FFT wrapped in the shifts that move the centred index
ranges to and from the library's [0, n) ranges.  The transforms run on as many
threads as scipy.fft.set_workers allows (one by default).
"""
import numpy as np
import scipy.fft


def centred_dft(a: np.ndarray, axes) -> np.ndarray:
    """Forward centred unitary DFT over ``axes``."""
    a = np.asarray(a, dtype=np.complex128)
    return scipy.fft.fftshift(scipy.fft.fftn(scipy.fft.ifftshift(a, axes=axes), axes=axes, norm="ortho"),
                              axes=axes)


def centred_idft(a: np.ndarray, axes) -> np.ndarray:
    """Inverse (= adjoint) centred unitary DFT over ``axes``."""
    a = np.asarray(a, dtype=np.complex128)
    return scipy.fft.fftshift(scipy.fft.ifftn(scipy.fft.ifftshift(a, axes=axes), axes=axes, norm="ortho"),
                              axes=axes)
