"""Filter responses g_L(r), g_H(r) of the full-resolution step (Eqs. 6-10).

Outside the overlap band the filters are flat (Eqs. 6, 7):
    r > ell + delta :  g_H = 1/sigma,  g_L = 0
    r < ell - delta :  g_H = 0,        g_L = 1/eta
Inside it (Eqs. 9, 10) they cross-fade with a sine,
    g_L(r) = a(r) (1 - s(r)),  g_H(r) = a(r) (1 + s(r)),  s(r) = sin(pi (r - ell) / (2 delta)),
with the normaliser a(r) (printed as alpha(r) in the paper) fixed by Eq. 8,
    sigma^2 g_H^2 + eta^2 g_L^2 = 1  =>  a(r) = [sigma^2 (1+s)^2 + eta^2 (1-s)^2]^(-1/2).

The radial coordinate r is the distance of a DFT cell from the origin in grid
cells, with signed frequency indices k in [-P/2, P/2) on each axis.
"""
from __future__ import annotations

import numpy as np


def radial_grid(P: int) -> np.ndarray:
    k = np.fft.fftfreq(P) * P  # signed integer indices in FFT order
    return np.sqrt(k[:, None] ** 2 + k[None, :] ** 2)


def responses(r, ell: float, delta: float, sigma2: float, eta2: float):
    """(g_L(r), g_H(r)) for an array of radii."""
    r = np.asarray(r, dtype=np.float64)
    sigma, eta = np.sqrt(sigma2), np.sqrt(eta2)
    gL = np.zeros_like(r)
    gH = np.zeros_like(r)
    hi = r > ell + delta
    lo = r < ell - delta
    band = ~(hi | lo)
    gH[hi] = 1.0 / sigma
    gL[lo] = 1.0 / eta
    s = np.sin(np.pi * (r[band] - ell) / (2.0 * delta))
    a = 1.0 / np.sqrt(sigma2 * (1.0 + s) ** 2 + eta2 * (1.0 - s) ** 2)
    gL[band] = a * (1.0 - s)
    gH[band] = a * (1.0 + s)
    return gL, gH


def squared_on_grid(P: int, ell: float, delta: float, sigma2: float, eta2: float):
    """(g_L^2, g_H^2) on the full P x P DFT grid in FFT order."""
    gL, gH = responses(radial_grid(P), ell, delta, sigma2, eta2)
    return gL * gL, gH * gH
