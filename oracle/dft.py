"""Discrete Fourier transform as dense separable matrices (oracle).

Sec. 2.1 (text around Eqs. 6-8): fields are sampled at voxel centres and the
trapezoidal rule turns the convolution with the projection operator into a
product in discrete Fourier space.  The oracle writes the DFT out as its
definition, one axis at a time:

    Ahat[k] = sum_a A[a] exp(-2 pi i k a / n),
    A[a]    = (1/n) sum_k Ahat[k] exp(+2 pi i k a / n),

applied along each of the three spatial axes.  No FFT algorithm is used.

Pins: round trip, agreement with the definition summed voxel by voxel on tiny
grids, and with a library FFT (tests only).  Status: pinned.
"""

from __future__ import annotations

import numpy as np

_CACHE: dict = {}


def dft_matrix(n: int) -> np.ndarray:
    """W[k, a] = exp(-2 pi i k a / n), complex128 (n, n)."""
    W = _CACHE.get(n)
    if W is None:
        k = np.arange(n)
        # reduce k*a mod n before scaling so large products stay exact
        W = np.exp(-2j * np.pi * (np.outer(k, k) % n) / n)
        _CACHE[n] = W
    return W


def _apply_axis(A: np.ndarray, M: np.ndarray, axis: int) -> np.ndarray:
    A = np.moveaxis(A, axis, -1)
    B = A @ M.T
    return np.moveaxis(B, -1, axis)


def dft3(A: np.ndarray) -> np.ndarray:
    """Forward DFT over the last three axes (any leading component axes)."""
    B = A.astype(np.complex128)
    nd = A.ndim
    for ax in (nd - 3, nd - 2, nd - 1):
        B = _apply_axis(B, dft_matrix(A.shape[ax]), ax)
    return B


def idft3(B: np.ndarray) -> np.ndarray:
    """Inverse DFT over the last three axes, including the 1/N factor."""
    A = B.astype(np.complex128)
    nd = B.ndim
    for ax in (nd - 3, nd - 2, nd - 1):
        n = B.shape[ax]
        A = _apply_axis(A, np.conj(dft_matrix(n)) / n, ax)
    return A


def idft3_real(B: np.ndarray, check: bool = True,
               scale: float = 0.0) -> np.ndarray:
    """Inverse DFT, keeping the real part and checking the imaginary part.

    The projection of a real field is real when the operator is even in the
    frequency and zero on the unpaired (Nyquist) frequencies; a large
    imaginary part therefore flags a broken operator.  ``scale`` is the
    magnitude of the field the spectrum came from (rounding noise is
    relative to it, not to a small projected output).
    """
    A = idft3(B)
    if check:
        scale = max(float(np.max(np.abs(A.real))) if A.size else 0.0,
                    scale, 1e-300)
        im = float(np.max(np.abs(A.imag))) if A.size else 0.0
        if im > 1e-11 * scale + 1e-300:
            raise FloatingPointError(
                f"inverse DFT not real: max|imag| = {im:.3e}, scale {scale:.3e}")
    return A.real.copy()
