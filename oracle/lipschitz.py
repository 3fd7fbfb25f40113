"""Lipschitz constant of the smooth part (Sect. 3.4).

theta = 2 lambda_max(A) with A1 = H_L^T H_L for step 1 and
A2 = H_H^T G_H^T G_H H_H + G_L^T G_L for step 2 (W = I); mu = 1/theta.

For circular convolutions and a dictionary of M orthogonal bases the paper
gives the closed forms theta_L = 2 M max|H_hat_L|^2 and
theta_H = 2 M max(|G_hat_H H_hat_H|^2 + |G_hat_L|^2); here M = 1.  Otherwise
(zero padding, i.e. crops between the convolutions) lambda_max is computed
iteratively: ``power_iteration`` (the method the paper points to) and
``lanczos`` (the method the library uses: the same quantity in several
times fewer operator applications).

Start vector: a counter-based generator, so that any implementation can
reproduce it bit for bit.  v0[n] = mix(seed + n) * 2^-64 - 1/2, where mix is
one step of SplitMix64 (Steele, Lea & Flood 2014; constants as published by
Vigna): z = c + 0x9E3779B97F4A7C15, z = (z ^ z>>30) * 0xBF58476D1CE4E5B9,
z = (z ^ z>>27) * 0x94D049BB133111EB, z ^= z>>31 (all mod 2^64).
"""
from __future__ import annotations

import numpy as np

MASK = (1 << 64) - 1


def splitmix64_mix(c: int) -> int:
    z = (c + 0x9E3779B97F4A7C15) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def start_vector(n: int, seed: int) -> np.ndarray:
    """v0 for an n x n image, row-major counter order."""
    c = (np.uint64(seed) + np.arange(n * n, dtype=np.uint64)).astype(np.uint64)
    with np.errstate(over="ignore"):
        z = c + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    # exact conversion: top 53 bits -> [0, 1), as the published float step does
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return (u - 0.5).reshape(n, n)


def power_iteration(normal, n: int, seed: int = 0, max_iter: int = 200, rtol: float = 1e-6):
    """2 * lambda_max of a symmetric PSD operator ``normal`` on n x n images.

    Iterates w = A v, theta_j = 2 <v, w> / <v, v>, v <- w / ||w|| until
    |theta_j - theta_{j-1}| <= rtol * theta_j or ``max_iter`` steps.
    Returns (theta, iterations, trace).
    """
    v = start_vector(n, seed)
    v = v / np.linalg.norm(v)
    prev = None
    trace = []
    theta = 0.0
    for j in range(1, max_iter + 1):
        w = normal(v)
        theta = 2.0 * float(np.vdot(v, w)) / float(np.vdot(v, v))
        trace.append(theta)
        nw = float(np.linalg.norm(w))
        if nw == 0.0:
            return 0.0, j, trace
        v = w / nw
        if prev is not None and abs(theta - prev) <= rtol * theta:
            return theta, j, trace
        prev = theta
    return theta, max_iter, trace


def lanczos(normal, n: int, seed: int = 0, max_iter: int = 200, rtol: float = 1e-6):
    """2 * lambda_max of a symmetric PSD operator by the Lanczos iteration
    (the largest Ritz value of the tridiagonal projection onto the Krylov
    space of the same start vector v0 as ``power_iteration``).

    With q_1 = v0 / ||v0||, beta_0 = 0 and q_0 = 0, step j computes
        w = A q_j,  alpha_j = <q_j, w>,  r = w - alpha_j q_j - beta_{j-1} q_{j-1},
        beta_j = ||r||,  q_{j+1} = r / beta_j,
    and theta_j = 2 lambda_max(T_j), T_j the j x j tridiagonal matrix with
    diagonal alpha_1..alpha_j and off-diagonal beta_1..beta_{j-1}; it stops
    when |theta_j - theta_{j-1}| <= rtol * theta_j, beta_j = 0 or after
    ``max_iter`` applications.  No reorthogonalisation (the largest Ritz
    value converges first).  Returns (theta, iterations, trace).
    """
    q = start_vector(n, seed)
    q = q / np.linalg.norm(q)
    q_prev = np.zeros_like(q)
    beta = 0.0
    alphas, betas, trace = [], [], []
    prev = None
    theta = 0.0
    for j in range(1, max_iter + 1):
        w = normal(q)
        alpha = float(np.vdot(q, w))
        alphas.append(alpha)
        r = w - alpha * q - beta * q_prev
        T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
        theta = 2.0 * float(np.linalg.eigvalsh(T)[-1])
        trace.append(theta)
        if prev is not None and abs(theta - prev) <= rtol * theta:
            return theta, j, trace
        prev = theta
        beta = float(np.linalg.norm(r))
        if beta == 0.0:
            return theta, j, trace
        betas.append(beta)
        q_prev, q = q, r / beta
    return theta, max_iter, trace


def closed_form_step1(h_hat: np.ndarray) -> float:
    """2 max |h_hat|^2 (circular convolution, M = 1)."""
    return 2.0 * float(np.max(np.abs(h_hat) ** 2))


def closed_form_step2(h_hat: np.ndarray, gL2: np.ndarray, gH2: np.ndarray) -> float:
    """2 max(g_H^2 |h_hat|^2 + g_L^2) (circular convolution, M = 1)."""
    return 2.0 * float(np.max(gH2 * np.abs(h_hat) ** 2 + gL2))
