"""Objectives and gradients of the two steps, with the dictionary W = I.

Step 1, the low-resolution problem (Eq. 4):
    F1(x) = || i_L - H_L x ||_2^2 + lambda_L ||x||_1
    grad f1(x) = 2 H_L^T (H_L x - i_L)                                   (Eq. 11)

Step 2, the full-resolution problem (Eq. 5):
    F2(x) = || G_H (i_H - H_H x) ||_2^2 + || G_L (l - x) ||_2^2 + lambda_H ||x||_1
    grad f2(x) = 2 H_H^T G_H^T G_H (H_H x - i_H) + 2 G_L^T G_L (x - l)   (Eq. 12)

Reading of G (not fixed by the paper): G = C_g E, i.e. the filter acts on
the zero-embedded P x P image and its norm is taken over the whole grid, so

    || G r ||^2 = (1/P^2) sum_k g(k)^2 |DFT(E r)(k)|^2,   G^T G = E^T C_{g^2} E.

Positivity (x >= 0) is not in the paper; it is a switch handled by the prox.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .conv import Operator, embed, crop, WORKERS
from .filters import squared_on_grid


def _filter_apply(x, mult, P, dtype=np.float64):
    """E^T C_mult E x for a real multiplier on the full P x P grid."""
    n = x.shape[0]
    X = sfft.fft2(embed(np.asarray(x, dtype=dtype), P), workers=WORKERS)
    return crop(sfft.ifft2(X * mult, workers=WORKERS), n).real.astype(dtype)


def _filter_norm2(r, mult, P):
    """|| C_g E r ||^2 = (1/P^2) sum g^2 |DFT(E r)|^2 with mult = g^2."""
    X = sfft.fft2(embed(np.asarray(r, dtype=np.float64), P), workers=WORKERS)
    return float(np.sum(mult * (X.real ** 2 + X.imag ** 2)) / (P * P))


class Step1:
    """Eq. 4 with W = I."""

    def __init__(self, dirty, psf, dtype=np.float64):
        self.n = dirty.shape[0]
        self.P = psf.shape[0]
        self.dtype = np.dtype(dtype)
        self.H = Operator(psf, self.n, dtype)
        self.y = np.asarray(dirty, dtype=self.dtype)

    def residual(self, x):
        return self.H.apply(x) - self.y

    def data_term(self, x):
        r = self.residual(x).astype(np.float64)
        return float(np.sum(r * r))

    def objective(self, x, lam):
        d = self.data_term(x)
        l1 = float(np.sum(np.abs(np.asarray(x, dtype=np.float64))))
        return d + lam * l1, d, l1

    def grad(self, x):
        return 2.0 * self.H.adjoint(self.residual(x))

    def normal(self, v):
        """The linear part A1 v = H^T H v (grad f1 = 2 (A1 x - H^T y))."""
        return self.H.adjoint(self.H.apply(v))


class Step2:
    """Eq. 5 with W = I.  ``low_res`` is l (the low-resolution image constraint)."""

    def __init__(self, dirty, psf, low_res, ell, delta, sigma2, eta2, dtype=np.float64):
        self.n = dirty.shape[0]
        self.P = psf.shape[0]
        self.dtype = np.dtype(dtype)
        self.H = Operator(psf, self.n, dtype)
        self.y = np.asarray(dirty, dtype=self.dtype)
        self.l = np.asarray(low_res, dtype=self.dtype)
        gL2, gH2 = squared_on_grid(self.P, ell, delta, sigma2, eta2)
        self.gL2 = gL2
        self.gH2 = gH2

    def data_terms(self, x):
        r = self.y - self.H.apply(x)
        dH = _filter_norm2(r, self.gH2, self.P)
        dL = _filter_norm2(self.l - np.asarray(x, dtype=self.dtype), self.gL2, self.P)
        return dH, dL

    def objective(self, x, lam):
        dH, dL = self.data_terms(x)
        l1 = float(np.sum(np.abs(np.asarray(x, dtype=np.float64))))
        return dH + dL + lam * l1, dH + dL, l1

    def grad(self, x):
        r = self.H.apply(x) - self.y
        t1 = self.H.adjoint(_filter_apply(r, self.gH2, self.P, self.dtype))
        t2 = _filter_apply(np.asarray(x, dtype=self.dtype) - self.l, self.gL2, self.P, self.dtype)
        return 2.0 * (t1 + t2)

    def normal(self, v):
        """A2 v = H^T E^T C_{gH^2} E H v + E^T C_{gL^2} E v."""
        t1 = self.H.adjoint(_filter_apply(self.H.apply(v), self.gH2, self.P, self.dtype))
        return t1 + _filter_apply(v, self.gL2, self.P, self.dtype)
