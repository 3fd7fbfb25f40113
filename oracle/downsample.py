"""The down-sampled low-resolution image (Sect. 6.1, the remedy for the
secondary data product): step 1 (Eq. 4) reconstructs an image of N_s = N / d
pixels a side instead of N, and step 2 (Eq. 5) uses it through a decimation
operator D applied to the full-resolution image and a modified filter G_L'
on the small grid:

    F2'(x) = || G_H (i_H - H_H x) ||^2 + || G_L' (l_s - D x) ||^2 + lambda ||x||_1.

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Readings (the paper names D and "an appropriate modification of G_L" and no
more):

* d is a power of two.  The small image covers the same field of view with d
  times larger pixels, so its P_s = P / d DFT grid has the full grid's uv cell
  size: cell k of the small grid is cell k of the full grid, and ell, delta
  keep their values in cells.
* Model images are in flux per pixel (a point source of flux S is one pixel of
  value S at any pixel size), so D conserves flux: it keeps the DFT cells
  |k| < N_s / 2 of each axis of the N x N image (periodic), folds the two
  cells +-N_s / 2 onto the small grid's Nyquist cell and transforms back on
  the small grid; a constant f becomes d^2 f.
* G_L' = C_{g'} E_s on the small P_s grid with g'(k) = g_L(k) / d (the same
  radius in cells), which needs g_L to vanish outside the small band.
* The step-2 kernels use U l_s, the up-sampling that D undoes (D U = I): the
  DFT of l_s zero-filled to N x N, the Nyquist cell split in halves between
  +-N_s / 2.  In circular mode (P = N)

      || G_L' (l_s - D x) ||^2 = || G_L (U l_s - x) ||^2

  exactly (Parseval on both grids: the DFT of D x on the small band is that
  of x, the DFT of U l_s on the full band is that of l_s, and
  g'^2 / P_s^2 = g_L^2 / P^2), so step 2 with the small image is Eq. 5 with
  l = U l_s.  Zero padded, the library takes the same form (the full grid's
  G_L on E (U l_s - x)).
"""
from __future__ import annotations

import numpy as np

from .filters import squared_on_grid


def _fold_index(M: int, m: int):
    """For each full-grid index k (FFT order, length M) its small-grid index
    (length m), or -1 for |k| > m/2; both cells +-m/2 map to m/2."""
    k = np.fft.fftfreq(M) * M
    idx = np.full(M, -1, dtype=np.int64)
    inside = np.abs(k) < m / 2
    idx[inside] = (k[inside] % m).astype(np.int64)
    idx[np.abs(k) == m / 2] = m // 2
    return idx


def decimate(x: np.ndarray, d: int) -> np.ndarray:
    """D x: N x N -> N/d x N/d, flux conserving (see the module docstring)."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    m = N // d
    X = np.fft.fft2(x)
    idx = _fold_index(N, m)
    Y = np.zeros((m, m), dtype=np.complex128)
    sel = np.nonzero(idx >= 0)[0]
    for r in sel:
        for c in sel:
            Y[idx[r], idx[c]] += X[r, c]
    return np.fft.ifft2(Y).real


def upsample(ls: np.ndarray, d: int) -> np.ndarray:
    """U l_s: N_s x N_s -> N x N, the zero-filled DFT (see the module docstring)."""
    ls = np.asarray(ls, dtype=np.float64)
    m = ls.shape[0]
    N = m * d
    L = np.fft.fft2(ls)
    idx = _fold_index(N, m)
    k = np.fft.fftfreq(N) * N
    wt = np.where(np.abs(k) == m / 2, 0.5, 1.0)  # the Nyquist cell split in halves
    X = np.zeros((N, N), dtype=np.complex128)
    sel = np.nonzero(idx >= 0)[0]
    for r in sel:
        for c in sel:
            X[r, c] = L[idx[r], idx[c]] * wt[r] * wt[c]
    return np.fft.ifft2(X).real


def interpolation_matrix(N: int, d: int) -> np.ndarray:
    """The 1-D factor K (N x N_s) of U l_s = K l_s K^T, written out from the
    Dirichlet sum: K[n, j] = (1/N) sum over the small band of
    exp(2 pi i k (n - d j) / N), the pair of half Nyquist cells as a cosine."""
    m = N // d
    t = (np.arange(N)[:, None] - d * np.arange(m)[None, :]).astype(np.float64)
    acc = np.ones_like(t)
    for k in range(1, m // 2):
        acc += 2.0 * np.cos(2.0 * np.pi * k * t / N)
    acc += np.cos(np.pi * m * t / N)
    return acc / N


def small_filter_sq(Ps: int, d: int, ell, delta, sigma2, eta2) -> np.ndarray:
    """g'^2 = g_L^2 / d^2 on the small P_s grid (same radius in cells)."""
    gL2, _ = squared_on_grid(Ps, ell, delta, sigma2, eta2)
    return gL2 / (d * d)


def small_term(x, ls, d, Ps, ell, delta, sigma2, eta2) -> float:
    """|| G_L' (l_s - D x) ||^2 with G_L' = C_{g'} E_s on the P_s grid."""
    r = np.asarray(ls, dtype=np.float64) - decimate(x, d)
    m = r.shape[0]
    big = np.zeros((Ps, Ps))
    o = (Ps - m) // 2
    big[o:o + m, o:o + m] = r
    R = np.fft.fft2(big)
    g2 = small_filter_sq(Ps, d, ell, delta, sigma2, eta2)
    return float(np.sum(g2 * (R.real ** 2 + R.imag ** 2)) / (Ps * Ps))
