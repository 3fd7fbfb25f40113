"""The two-step minor cycle with one major cycle per step (Sect. 3).

1. Step 1 (Eq. 4): FISTA on the short-baseline dirty image and PSF.
2. Low-resolution image i_L = beta1 + (i~_L - H_L beta1)   (Sect. 3.2).
3. sigma2_hat from the long-baseline dirty image, eta2_hat = 1e-3 sigma2_hat
   (Sect. 4.3).
4. Step 2 (Eq. 5): FISTA on the long-baseline dirty image and PSF, with the
   filters of Eqs. 6-10 and l = i_L.

Step sizes come from power iteration (times ``margin``) unless given.
"""
from __future__ import annotations

import numpy as np

from .objectives import Step1, Step2
from .fista import fista
from .lipschitz import power_iteration
from .helpers import sigma2_hat, eta2_hat, default_lambda, low_res_image


def solve_step(prob, lam, iters, theta=None, x0=None, positivity=False, seed=0, margin=1.01,
               callback=None, dtype=np.float64):
    if theta is None:
        theta, _, _ = power_iteration(prob.normal, prob.n, seed=seed)
        theta *= margin
    x0 = np.zeros((prob.n, prob.n)) if x0 is None else x0
    beta, alpha = fista(prob.grad, x0, 1.0 / theta, lam, iters, positivity=positivity,
                        callback=callback, dtype=dtype)
    return beta, alpha, theta


def two_step(dirty_L, psf_L, dirty_H, psf_H, ell, delta, iters1, iters2, positivity=False,
             c=0.05, theta1=None, theta2=None, seed=0, margin=1.01, sigma2=None, eta2=None):
    s1 = Step1(dirty_L, psf_L)
    lam1 = default_lambda(dirty_L, c)
    beta1, _, theta1 = solve_step(s1, lam1, iters1, theta1, positivity=positivity, seed=seed, margin=margin)
    i_L = low_res_image(beta1, s1.y, s1.H)
    s2_ = sigma2_hat(dirty_H) if sigma2 is None else sigma2
    e2_ = eta2_hat(s2_) if eta2 is None else eta2
    s2 = Step2(dirty_H, psf_H, i_L, ell, delta, s2_, e2_)
    lam2 = default_lambda(dirty_H, c)
    beta2, _, theta2 = solve_step(s2, lam2, iters2, theta2, positivity=positivity, seed=seed, margin=margin)
    return {
        "beta1": beta1, "i_L": i_L, "beta2": beta2,
        "lambda1": lam1, "lambda2": lam2, "theta1": theta1, "theta2": theta2,
        "sigma2": s2_, "eta2": e2_,
        "F1": s1.objective(beta1, lam1)[0], "F2": s2.objective(beta2, lam2)[0],
    }


def major_cycles(step, dirty, psf, cycles, iters, c=0.05, theta=None, positivity=False, low_res=None,
                 ell=None, delta=None, sigma2=None, eta2=None, seed=0, margin=1.01, dictionary=False):
    """Several major cycles of one step (Sect. 3.2 for step 1, Sect. 3.3 for
    step 2), the residual image of each cycle formed in the image domain.

    Cycle n solves its step's problem on the residual image
        i~_n = i~_1 - H sum_{j<n} i_j
    (the paper recomputes it from the visibilities; here the PSF convolution
    stands in for degridding and gridding), with lambda_n = c ||i~_n||_2 2^(n-1)
    and, in step 2, the constraint l_n = l - sum_{j<n} i_j; FISTA starts from
    zero and its result is the cycle's image i_n.  The step's image is
    i~_{N+1} + sum_n i_n.  Returns (image, sum of the i_n, per-cycle records).

    With ``dictionary`` each cycle runs FISTA on the coefficients of the
    db1-db8 dictionary (Sect. 3, App. A.1; ``theta`` is then the constant of
    the problem in alpha, by default M = 8 times the image operator's) and
    i_n = W alpha_K."""
    dirty = np.asarray(dirty, np.float64)
    if step == 1:
        make = lambda y, l: Step1(y, psf)  # noqa: E731
    else:
        low_res = np.asarray(low_res, np.float64)
        make = lambda y, l: Step2(y, psf, l, ell, delta, sigma2, eta2)  # noqa: E731
    msum = np.zeros_like(dirty)
    resid = dirty
    recs = []
    for n in range(1, cycles + 1):
        if n > 1:
            resid = dirty - make(dirty, low_res).H.apply(msum)
        lam = default_lambda(resid, c, cycle=n)
        prob = make(resid, None if step == 1 else low_res - msum)
        if dictionary:
            from .wavelets import InDictionary, M, synthesis

            if theta is None:
                theta = M * margin * power_iteration(prob.normal, prob.n, seed=seed)[0]
            dic = InDictionary(prob)
            alpha, _ = fista(dic.grad, np.zeros((M, prob.n, prob.n)), 1.0 / theta, lam, iters)
            beta = synthesis(alpha)
            F = dic.objective(alpha, lam)[0]
        else:
            beta, _, theta = solve_step(prob, lam, iters, theta, positivity=positivity, seed=seed, margin=margin)
            F = prob.objective(beta, lam)[0]
        recs.append({"lambda": lam, "F": F, "theta": theta})
        msum = msum + beta
    final_resid = dirty - make(dirty, low_res).H.apply(msum)
    return final_resid + msum, msum, recs
