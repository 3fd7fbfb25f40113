"""The PSF convolution operator H (Sect. 3.2 defines H_L as convolution by the
low-resolution PSF; Sect. 3.3 does the same for H_H).

Discretisation (the paper does not fix it; this is the reading used
throughout): an N x N image x is zero-embedded into a P x P grid at offset
o = (P - N) // 2 (operator E), circularly convolved with the P x P PSF whose
phase centre sits at (P/2, P/2), and cropped back (E^T):

    (H x)[p] = sum_q PSF[(P/2 + p - q) mod P] x[q],    p, q in [0, N)^2.

With P = 2N every offset p - q lies in (-N, N), so nothing wraps: H is the
exact linear convolution.  With P = N (circular mode) the sum wraps.

Three interchangeable back-ends compute the same thing:
* ``conv_brute``  -- the spatial sum above, O(N^4); the definition.
* ``conv_direct`` -- separable DFT matrices, O(P^3).
* ``conv_fft``    -- real FFTs (scipy.fft), for large sizes and CPU timing.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

WORKERS = os.cpu_count() or 1


def embed(x: np.ndarray, P: int) -> np.ndarray:
    """E: zero-embed an N x N image into P x P at offset (P - N) // 2."""
    n = x.shape[0]
    o = (P - n) // 2
    out = np.zeros((P, P), dtype=x.dtype)
    out[o : o + n, o : o + n] = x
    return out


def crop(y: np.ndarray, n: int) -> np.ndarray:
    """E^T: the central N x N block of a P x P grid (same offset as ``embed``)."""
    P = y.shape[0]
    o = (P - n) // 2
    return y[o : o + n, o : o + n]


def psf_spectrum(psf: np.ndarray) -> np.ndarray:
    """h_hat = DFT(ifftshift(PSF)) as a complex array (real for a point-symmetric PSF)."""
    return np.fft.fft2(np.fft.ifftshift(psf))


# ---------------------------------------------------------------- brute force
def conv_brute(x: np.ndarray, psf: np.ndarray, adjoint: bool = False) -> np.ndarray:
    """The defining spatial sum.  ``adjoint`` gives H^T: (H^T y)[q] = sum_p PSF[P/2+p-q] y[p]."""
    n = x.shape[0]
    P = psf.shape[0]
    c = P // 2
    out = np.zeros((n, n), dtype=np.result_type(x, psf))
    for qi in range(n):
        for qj in range(n):
            xv = x[qi, qj]
            if xv == 0:
                continue
            for pi in range(n):
                di = (c + pi - qi) if not adjoint else (c + qi - pi)
                row = psf[di % P]
                for pj in range(n):
                    dj = (c + pj - qj) if not adjoint else (c + qj - pj)
                    out[pi, pj] += row[dj % P] * xv
    return out


def conv_brute_vec(x: np.ndarray, psf: np.ndarray, adjoint: bool = False) -> np.ndarray:
    """Same sum, vectorised over the output pixel (still O(N^4) work)."""
    n = x.shape[0]
    P = psf.shape[0]
    c = P // 2
    p = np.arange(n)
    out = np.zeros((n, n), dtype=np.result_type(x, psf))
    for qi in range(n):
        di = ((c + p - qi) if not adjoint else (c + qi - p)) % P
        for qj in range(n):
            xv = x[qi, qj]
            if xv == 0:
                continue
            dj = ((c + p - qj) if not adjoint else (c + qj - p)) % P
            out += xv * psf[np.ix_(di, dj)]
    return out


# ---------------------------------------------------------------- direct DFT
def dft_matrix(P: int, sign: int = -1) -> np.ndarray:
    k = np.arange(P)
    return np.exp(sign * 2j * np.pi * np.outer(k, k) / P)


def conv_direct(x: np.ndarray, psf: np.ndarray, adjoint: bool = False) -> np.ndarray:
    """E^T F^{-1} [h_hat * F(E x)] with explicit DFT matrices (adjoint: conj(h_hat))."""
    n = x.shape[0]
    P = psf.shape[0]
    F = dft_matrix(P, -1)
    Fi = dft_matrix(P, +1) / P
    h = F @ np.fft.ifftshift(psf) @ F.T
    if adjoint:
        h = np.conj(h)
    X = F @ embed(x.astype(np.complex128), P) @ F.T
    y = Fi @ (h * X) @ Fi.T
    return crop(y, n).real


# ---------------------------------------------------------------- FFT
def spectrum_apply(x: np.ndarray, mult: np.ndarray, P: int) -> np.ndarray:
    """E^T F^{-1}[mult * F(E x)] for a real multiplier on the rfft half plane (P x (P/2+1))."""
    n = x.shape[0]
    X = sfft.rfft2(embed(x, P), workers=WORKERS)
    y = sfft.irfft2(X * mult, s=(P, P), workers=WORKERS)
    return crop(y, n)


def half_plane(full: np.ndarray) -> np.ndarray:
    """The rfft half plane of a P x P spectrum."""
    P = full.shape[0]
    return full[:, : P // 2 + 1]


def conv_fft(x: np.ndarray, psf: np.ndarray, adjoint: bool = False, dtype=np.float64) -> np.ndarray:
    n = x.shape[0]
    P = psf.shape[0]
    h = psf_spectrum(psf)
    if adjoint:
        h = np.conj(h)
    X = sfft.fft2(embed(x.astype(dtype), P), workers=WORKERS)
    y = sfft.ifft2(X * h.astype(np.complex128 if dtype == np.float64 else np.complex64), workers=WORKERS)
    return crop(y, n).real


class Operator:
    """H for one PSF with the spectrum cached (FFT back-end).

    ``h`` is the complex spectrum of the PSF.  ``apply`` is H, ``adjoint`` is
    H^T.  ``dtype`` selects float64 (default) or float32 arithmetic.
    """

    def __init__(self, psf: np.ndarray, n: int, dtype=np.float64):
        self.P = psf.shape[0]
        self.n = n
        self.dtype = np.dtype(dtype)
        cdt = np.complex128 if self.dtype == np.float64 else np.complex64
        self.h = psf_spectrum(psf.astype(np.float64)).astype(cdt)

    def _apply(self, x, h):
        X = sfft.fft2(embed(np.asarray(x, dtype=self.dtype), self.P), workers=WORKERS)
        y = sfft.ifft2(X * h, workers=WORKERS)
        return crop(y, self.n).real.astype(self.dtype)

    def apply(self, x):
        return self._apply(x, self.h)

    def adjoint(self, y):
        return self._apply(y, np.conj(self.h))
