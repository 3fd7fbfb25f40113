"""Soft thresholding and FISTA (Algorithm 1).

The prox of t ||.||_1 is tau_t(z) = sign(z) max(|z| - t, 0) (Sect. 3.4).  With
the optional positivity constraint (not in the paper) the prox of
t ||.||_1 + indicator(x >= 0) is max(z - t, 0).

Algorithm 1 solves min f + gamma ||.||_1 with a gradient step mu and the
momentum weight (k-1)/(k+2).  Reading of the threshold: a proximal-gradient
step with step size mu thresholds at mu * gamma, so t = mu * lambda.

Iteration, from x0 (default 0), for k = 1 .. K:
    beta_k  = prox_{mu lambda}(alpha_{k-1} - mu grad f(alpha_{k-1}))
    alpha_k = beta_k + (k-1)/(k+2) (beta_k - beta_{k-1})
with beta_0 = alpha_0 = x0.  K counts prox steps.  The result is beta_K
(alpha_K is returned too).
"""
from __future__ import annotations

import numpy as np


def soft_threshold(z, t):
    return np.sign(z) * np.maximum(np.abs(z) - t, 0.0)


def prox(z, t, positivity: bool):
    if positivity:
        return np.maximum(z - t, 0.0)
    return soft_threshold(z, t)


def momentum(k: int) -> float:
    return (k - 1.0) / (k + 2.0)


def fista(grad, x0, mu, lam, iters, positivity=False, momentum_on=True, callback=None, dtype=np.float64):
    """Run ``iters`` prox steps; returns (beta_K, alpha_K).

    ``callback(k, beta_k)`` is called after every step (for traces).
    ``momentum_on=False`` gives ISTA.
    """
    dt = np.dtype(dtype)
    x0 = np.asarray(x0, dtype=dt)
    beta_prev = x0.copy()
    alpha = x0.copy()
    t = dt.type(mu * lam)
    mu_ = dt.type(mu)
    beta = beta_prev
    for k in range(1, iters + 1):
        z = alpha - mu_ * grad(alpha)
        beta = prox(z, t, positivity).astype(dt)
        w = momentum(k) if momentum_on else 0.0
        alpha = beta + dt.type(w) * (beta - beta_prev)
        beta_prev = beta
        if callback is not None:
            callback(k, beta)
    return beta, alpha


def fista_from(grad, beta_k, beta_km1, k, mu, lam, iters, positivity=False, dtype=np.float64):
    """Algorithm 1 continued from iteration k: given beta_k and beta_{k-1},
    alpha_k = beta_k + (k-1)/(k+2) (beta_k - beta_{k-1}), then the same prox
    and momentum steps for k+1 .. k+iters.  Returns (beta_{k+iters},
    beta_{k+iters-1}, alpha_{k+iters}).  With beta_k = beta_{k-1} = x0 and
    k = 0 it is ``fista`` from x0."""
    dt = np.dtype(dtype)
    beta = np.asarray(beta_k, dtype=dt).copy()
    beta_prev = np.asarray(beta_km1, dtype=dt).copy()
    alpha = beta + dt.type(momentum(k) if k >= 1 else 0.0) * (beta - beta_prev)
    t = dt.type(mu * lam)
    mu_ = dt.type(mu)
    for j in range(k + 1, k + iters + 1):
        z = alpha - mu_ * grad(alpha)
        new = prox(z, t, positivity).astype(dt)
        alpha = new + dt.type(momentum(j)) * (new - beta)
        beta_prev, beta = beta, new
    return beta, beta_prev, alpha
