"""Parameter helpers and reporting.

* sigma2_hat (Sect. 4.3): the variance of the pixels of the long-baseline
  dirty image inside a 5 x 5 sliding window, averaged over all window
  positions.  Reading: only windows that fit inside the image, population
  variance (ddof = 0).  eta2_hat = 1e-3 * sigma2_hat.
* default_lambda (Sect. 5, App. A.2): lambda = c ||i~||_2 * 2^(n-1) for the
  n-th major cycle, c = 0.05 for both steps of the two-step method and 0.01
  for the single-step method.  Reading of the cycle factor: the first cycle
  uses exactly c.
* low_res_image (Sect. 3.2, one major cycle): i_L = beta + (i~_L - H_L beta),
  the deconvolved model plus the residual left after it.
* psnr: 20 log10(max|truth| / RMSE).
"""
from __future__ import annotations

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view


def sigma2_hat(img: np.ndarray, w: int = 5) -> float:
    win = sliding_window_view(np.asarray(img, dtype=np.float64), (w, w))
    return float(np.mean(np.var(win, axis=(-2, -1))))


def eta2_hat(s2: float, ratio: float = 1e-3) -> float:
    return ratio * s2


def default_lambda(dirty: np.ndarray, c: float = 0.05, cycle: int = 1) -> float:
    return c * float(np.linalg.norm(np.asarray(dirty, dtype=np.float64))) * 2.0 ** (cycle - 1)


def low_res_image(beta, dirty, H) -> np.ndarray:
    """beta + (dirty - H beta), H an ``oracle.conv.Operator``."""
    return beta + (dirty - H.apply(beta))


def psnr(img, truth) -> float:
    img = np.asarray(img, dtype=np.float64)
    truth = np.asarray(truth, dtype=np.float64)
    rmse = np.sqrt(np.mean((img - truth) ** 2))
    return 20.0 * np.log10(np.max(np.abs(truth)) / rmse)
