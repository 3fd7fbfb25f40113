"""The wavelet dictionary W of the paper: the concatenation of the first M = 8
Daubechies orthonormal wavelet bases (db1 .. db8; Sect. 3, Sect. 5, App. A.1),
x = W alpha = sum_b Psi_b alpha_b, alpha = (alpha_1, .., alpha_M), each alpha_b
an N x N array of 2-D wavelet coefficients.  TEST INFRASTRUCTURE ONLY, like the
rest of this package.

Readings (the paper does not fix them): periodic boundaries, separable 2-D
transform (rows, then columns, at each level), 4 decomposition levels, the
coefficients of each basis in the usual nested layout (approximation of the
coarsest level in the top-left corner).

Filters: db_p has 2p taps, obtained by spectral factorisation.  With
y = sin^2(w/2), |H(w)|^2 = 2 cos^{2p}(w/2) Q(y), Q(y) = sum_{k<p} C(p-1+k, k) y^k;
each root y_j of Q gives the pair of roots z, 1/z of z^2 - (2 - 4 y_j) z + 1
(y = (2 - z - 1/z)/4), and the minimum-phase filter keeps the root inside the
unit circle: H(z) ~ (1 + z^-1)^p prod_j (1 - z_j z^-1), scaled to sum sqrt(2).
The high-pass filter is g[n] = (-1)^n h[2p - 1 - n].

Analysis of one level along an axis of length n (periodic):
    lo[i] = sum_k h[k] x[(2 i + k) mod n],  hi[i] = sum_k g[k] x[(2 i + k) mod n],
stored as [lo, hi]; synthesis is its transpose (the transform is orthonormal).
"""
from __future__ import annotations

from functools import lru_cache
from math import comb

import numpy as np

LEVELS = 4
M = 8


def daubechies(p: int) -> np.ndarray:
    """Low-pass taps of db_p (2p taps, sum sqrt(2), minimum phase)."""
    return _daubechies(p).copy()


@lru_cache(maxsize=None)
def _daubechies(p: int) -> np.ndarray:
    q = np.array([comb(p - 1 + k, k) for k in range(p)], dtype=np.float64)  # Q(y) = sum q_k y^k
    h = np.array([1.0])
    for _ in range(p):
        h = np.convolve(h, [1.0, 1.0])  # (1 + z^-1)^p
    if p > 1:
        for y in np.roots(q[::-1]):
            # z^2 - (2 - 4y) z + 1 = 0; keep the root inside the unit circle
            b = 2.0 - 4.0 * y
            disc = np.sqrt(b * b - 4.0 + 0j)
            z1, z2 = (b + disc) / 2.0, (b - disc) / 2.0
            z = z1 if abs(z1) < 1.0 else z2
            h = np.convolve(h, [1.0, -z])
        h = np.real_if_close(h, tol=1e6)
        h = np.real(h)
    return h * (np.sqrt(2.0) / np.sum(h))


def highpass(h: np.ndarray) -> np.ndarray:
    n = np.arange(h.size)
    return ((-1.0) ** n) * h[::-1]


def _analysis_1d(x, h, g, axis):
    """One level along `axis` (periodic): returns concat([lo, hi]) along axis."""
    x = np.moveaxis(np.asarray(x, np.float64), axis, -1)
    n = x.shape[-1]
    idx = (2 * np.arange(n // 2)[:, None] + np.arange(h.size)[None, :]) % n
    win = x[..., idx]  # (..., n/2, taps)
    out = np.concatenate([win @ h, win @ g], axis=-1)
    return np.moveaxis(out, -1, axis)


def _synthesis_1d(c, h, g, axis):
    """Transpose of _analysis_1d."""
    c = np.moveaxis(np.asarray(c, np.float64), axis, -1)
    n = c.shape[-1]
    lo, hi = c[..., : n // 2], c[..., n // 2:]
    x = np.zeros(c.shape)
    for k in range(h.size):
        pos = (2 * np.arange(n // 2) + k) % n  # distinct for a fixed k
        x[..., pos] += lo * h[k] + hi * g[k]
    return np.moveaxis(x, -1, axis)


def dwt2(x, p, levels=LEVELS):
    """Coefficients of one orthonormal basis (db_p), nested layout."""
    h = daubechies(p)
    g = highpass(h)
    c = np.array(x, dtype=np.float64, copy=True)
    s = c.shape[0]
    for _ in range(levels):
        blk = c[:s, :s]
        blk = _analysis_1d(blk, h, g, axis=1)  # rows
        blk = _analysis_1d(blk, h, g, axis=0)  # columns
        c[:s, :s] = blk
        s //= 2
    return c


def idwt2(c, p, levels=LEVELS):
    h = daubechies(p)
    g = highpass(h)
    x = np.array(c, dtype=np.float64, copy=True)
    s = x.shape[0] >> (levels - 1)
    for _ in range(levels):
        blk = x[:s, :s]
        blk = _synthesis_1d(blk, h, g, axis=0)  # columns
        blk = _synthesis_1d(blk, h, g, axis=1)  # rows
        x[:s, :s] = blk
        s *= 2
    return x


def synthesis(alpha, levels=LEVELS):
    """W alpha: alpha has shape (M, N, N)."""
    return sum(idwt2(alpha[b], b + 1, levels) for b in range(M))


def analysis(x, levels=LEVELS):
    """W^T x: shape (M, N, N)."""
    return np.stack([dwt2(x, b + 1, levels) for b in range(M)])


class InDictionary:
    """A step's problem in the coefficients alpha of W (Eqs. 4-5 as written):
    f(alpha) = f_image(W alpha), grad = W^T grad_image(W alpha)."""

    def __init__(self, prob, levels=LEVELS):
        self.prob = prob
        self.levels = levels
        self.n = prob.n

    def grad(self, alpha):
        return analysis(self.prob.grad(synthesis(alpha, self.levels)), self.levels)

    def objective(self, alpha, lam):
        f = self.prob.objective(synthesis(alpha, self.levels), lam)
        data = f[1]
        l1 = float(np.sum(np.abs(alpha)))
        return data + lam * l1, data, l1

    def normal(self, alpha):
        return analysis(self.prob.normal(synthesis(alpha, self.levels)), self.levels)
