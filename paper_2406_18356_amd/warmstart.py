"""Training data, training loop and evaluation of the learned warm start.

The network (``msr_unet_*``) predicts the start of the step-2 minor cycle
from the long-baseline dirty image and the low-resolution image of step 1;
FISTA then runs to the same tolerance as from zero, so a poor prediction
costs iterations, never accuracy.  Everything numeric runs in libmsr: the
two-step solves that produce the training pairs (batched), the network's
forward and backward passes and its Adam steps.  This module only moves
tensors between those calls.
"""
from __future__ import annotations

import time

import numpy as np


def _dev_f32(torch, a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)


def solve_pairs(problems, iters1=500, iters2=3000, c=0.05, positivity=True, chunk=32, device=0):
    """Runs the two-step method on `problems` (objects with n, dirty_L, psf_L,
    dirty_H, psf_H, ell, delta; one image size) in batches of `chunk` channels.

    Returns GPU tensors (dirty_H, i_L, beta2, lambda2) stacked over the
    problems: the network's inputs and its target, the step-2 result after
    `iters2` iterations from zero with lambda = c ||i_H|| (Sect. 5)."""
    import torch

    from .binding import Batch

    dev = torch.device("cuda", device)
    dh_all, il_all, b2_all, lam_all = [], [], [], []
    for s in range(0, len(problems), chunk):
        part = problems[s:s + chunk]
        b = Batch([p.n for p in part], positivity=positivity, device=device)
        lam1, lam2, dhs = [], [], []
        for p, ch in zip(part, b.channels):
            dl, dh = _dev_f32(torch, p.dirty_L, dev), _dev_f32(torch, p.dirty_H, dev)
            ch.set_dirty_psf(1, dl, _dev_f32(torch, p.psf_L, dev))
            ch.set_dirty_psf(2, dh, _dev_f32(torch, p.psf_H, dev))
            lam1.append(ch.default_lambda(1, 1, c))
            lam2.append(ch.default_lambda(2, 1, c))
            sig2 = ch.estimate_sigma2(dh)
            ch.set_filters(p.ell, p.delta, sig2, 1e-3 * sig2)
            dhs.append(dh)
        _, il, _ = b.solve(1, lam1, iters1, image=True)
        b2, _ = b.solve(2, lam2, iters2, low_res=il)
        dh_all += dhs
        il_all += il
        b2_all += b2
        lam_all += lam2
        del b
    return torch.stack(dh_all), torch.stack(il_all), torch.stack(b2_all), lam_all


def train(net, dh, il, target, epochs=20, batch=8, lr=1e-3, seed=0, log=None):
    """Adam on the mean squared error of the network over (dh, il) -> target
    (GPU tensors, N x n x n); returns the per-epoch mean losses."""
    import torch

    g = torch.Generator().manual_seed(seed)
    n = dh.shape[0]
    losses = []
    for e in range(epochs):
        perm = torch.randperm(n, generator=g)
        tot, cnt = 0.0, 0
        for s in range(0, n - batch + 1, batch):
            idx = perm[s:s + batch].to(dh.device)
            loss = net.train_step(dh[idx].contiguous(), il[idx].contiguous(), target[idx].contiguous(), lr=lr)
            tot += loss
            cnt += 1
        losses.append(tot / max(cnt, 1))
        if log:
            log(f"warm-start training epoch {e + 1}/{epochs}: loss {losses[-1]:.4g}")
    return losses


def time_to_tol(solver, lam, low_res, f_ref, x0=None, tol=1e-6, max_iters=20000, check_every=10, warm_ms=0.0,
                momentum_k=0):
    """Step-2 time (ms, HIP events; plus `warm_ms` spent producing x0) and
    iterations to reach (F - f_ref) / |f_ref| <= tol.  With momentum_k > 0
    the run starts at iteration momentum_k + 1 from beta = x0 with zero
    velocity (msr_set_state), so that the momentum weight starts near 1
    instead of at 0 (Algorithm 1 itself restarts at k = 1)."""
    if momentum_k > 0:
        solver.set_state(2, x0, x0, momentum_k)
    _, r = solver.step2(lam, low_res, max_iters, x0=x0, check_every=check_every, tol=tol, f_ref=f_ref)
    ms = (r.time_to_tol_ms + warm_ms) if r.converged else -1.0
    return {"ms": ms, "iters": int(r.iters), "converged": bool(r.converged), "warm_start_ms": warm_ms}


def timed_forward(net, dh, il):
    """The network's warm start and its wall time in ms (synchronised)."""
    import torch

    torch.cuda.synchronize()
    t = time.perf_counter()
    x0 = net.forward(dh, il)
    torch.cuda.synchronize()
    return x0, (time.perf_counter() - t) * 1e3
