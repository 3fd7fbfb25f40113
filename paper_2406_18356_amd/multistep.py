"""The whole two-step reconstruction with major cycles, and the single-step
method it is compared with (Sect. 5), as sequences of library calls.

two_step   : step 1 (Eq. 4) for `cycles` major cycles on the short-baseline
             data -> the low-resolution image i_L (Sect. 3.2); sigma2_hat of the
             long-baseline dirty image, eta2_hat = 1e-3 sigma2_hat (Sect. 4.3);
             step 2 (Eq. 5) for `cycles` major cycles constrained by i_L
             (Sect. 3.3) -> the image.
             With `coarse = (d, dirty_L_s, psf_L_s)` step 1 runs on the
             N/d grid instead and step 2 takes U i_L,s (msr_upsample), the
             down-sampled low-resolution image of Sect. 6.1.
single_step: the step-1 problem on all visibilities (full PSF and dirty
             image) with its own regularisation constant (0.01 in Sect. 5).

All arithmetic runs in libmsr (msr_major_cycles and the helpers); this module
only orders the calls.
"""
from __future__ import annotations


def _dev(torch, a, dev, dtype):
    import numpy as np

    return torch.from_numpy(np.ascontiguousarray(a, np.float32 if dtype == torch.float32 else np.float64)).to(dev)


def two_step(problem, cycles=5, iters=100, c=0.05, eta_ratio=1e-3, positivity=True, precision=32, device=0,
             solver=None, coarse=None):
    """Returns (image, low-resolution image, report) for a problem with n,
    dirty_L, psf_L, dirty_H, psf_H, ell, delta; eta2 = eta_ratio sigma2_hat
    (1e-3 is the estimate of Sect. 4.3).  report["model"] is the sum of the
    step-2 cycle images (the image without the final residual).  With
    coarse = (d, dirty_L_s, psf_L_s) the returned low-resolution image is
    the N/d one that step 1 produced."""
    import torch

    from .binding import Solver

    s = solver or Solver(problem.n, positivity=positivity, precision=precision, device=device)
    dev = torch.device("cuda", device)
    T = lambda a: _dev(torch, a, dev, s.dtype)  # noqa: E731
    dh = T(problem.dirty_H)
    s.set_dirty_psf(2, dh, T(problem.psf_H))
    if coarse is None:
        s.set_dirty_psf(1, T(problem.dirty_L), T(problem.psf_L))
        i_L, _, r1 = s.major_cycles(1, cycles, iters, c=c)
        low = i_L
    else:
        d, dirty_s, psf_s = coarse
        sm = Solver(problem.n // d, positivity=positivity, precision=precision, device=device)
        sm.set_dirty_psf(1, T(dirty_s), T(psf_s))
        i_L, _, r1 = sm.major_cycles(1, cycles, iters, c=c)
        low = s.upsample(i_L, d)
        del sm
    sig2 = s.estimate_sigma2(dh)
    s.set_filters(problem.ell, problem.delta, sig2, eta_ratio * sig2)
    img, model, r2 = s.major_cycles(2, cycles, iters, c=c, low_res=low)
    report = {"sigma2": sig2, "model": model, "step1_F": [r.objective for r in r1], "step2_F": [r.objective for r in r2],
              "step1_ms": sum(r.elapsed_ms for r in r1), "step2_ms": sum(r.elapsed_ms for r in r2)}
    return img, i_L, report


def single_step(dirty, psf, n, cycles=5, iters=100, c=0.01, positivity=True, precision=32, device=0):
    """The image of the single-step method on all visibilities; the report's
    "model" is the sum of the cycle images."""
    import torch

    from .binding import Solver

    s = Solver(n, positivity=positivity, precision=precision, device=device)
    dev = torch.device("cuda", device)
    s.set_dirty_psf(1, _dev(torch, dirty, dev, s.dtype), _dev(torch, psf, dev, s.dtype))
    img, model, r = s.major_cycles(1, cycles, iters, c=c)
    return img, {"model": model, "F": [x.objective for x in r], "ms": sum(x.elapsed_ms for x in r)}
