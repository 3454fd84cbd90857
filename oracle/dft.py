"""The oracle's own discrete Fourier transform (test infrastructure).

A dense N x N matrix exp(sign 2 pi i (j k mod N) / N) applied along each axis
in turn.  Forward is unnormalised; the inverse carries 1/N per axis, the
convention of Octave's fft/ifft that Algorithm 2 is written in.  No FFT
library is used here; tests compare this against numpy.fft.
"""
import numpy as np


def dft_matrix(N, sign):
    j = np.arange(N)
    jk = np.outer(j, j) % N  # reduce the integer product before scaling
    return np.exp(sign * 2j * np.pi * jk / N)


def _apply_axes(a, sign, scale):
    a = np.asarray(a, dtype=complex)
    out = a
    for ax in range(a.ndim):
        F = dft_matrix(a.shape[ax], sign)
        out = np.moveaxis(np.tensordot(F, out, axes=([1], [ax])), 0, ax)
        if scale:
            out = out / a.shape[ax]
    return out


def fft3(a):
    """Unnormalised forward transform sum_j a_j exp(-2 pi i j.k / N)."""
    return _apply_axes(a, -1.0, False)


def ifft3(a):
    """Inverse transform (1/N^3) sum_k a_k exp(+2 pi i j.k / N)."""
    return _apply_axes(a, +1.0, True)
