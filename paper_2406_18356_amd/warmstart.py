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

import json
import os
import time

import numpy as np


def _dev_f32(torch, a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)


def solve_pairs(problems, iters1=500, iters2=3000, c=0.05, positivity=True, chunk=32, device=0, log=None):
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
        if log:
            torch.cuda.synchronize()
            log(f"solve_pairs: {min(s + chunk, len(problems))}/{len(problems)} pairs")
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
        z = x0.to(getattr(solver, "state_dtype", x0.dtype))
        solver.set_state(2, z, z, momentum_k)
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


# --------------------------------------------------------------------------
# A certified reference objective F* for the time-to-tolerance metric
# --------------------------------------------------------------------------
def duality_gap(F, data, grad, x, lam, positivity=True):
    """Upper bound on F(x) - F* from one gradient evaluation (any array type
    with .max(), .abs() and elementwise products: NumPy or torch).

    Step 2 (and step 1) minimise f(x) + lam ||x||_1 [+ x >= 0] with
    f(x) = ||M x - y||^2, M and y stacking the filtered PSF operator and the
    constraint term.  With r = y - M x, grad f = -2 M^T r, and the dual of
    min_{x >= 0} ||M x - y||^2 + lam 1^T x is
        max_u  -||u||^2 / 4 - u^T y   subject to  M^T u >= -lam
    (|M^T u| <= lam without positivity).  The point u = -2 s r is feasible for
    s = min(1, lam / max(-grad)) (max |grad| without positivity), and its dual
    value is (2 s - s^2) f(x) - s <grad, x>, using r^T y = f - <grad, x> / 2.
    Returns (gap, s); gap = F(x) - dual >= F(x) - F* >= 0, and gap = 0 at the
    minimiser (s = 1 by the optimality conditions)."""
    worst = float((-grad).max()) if positivity else float(abs(grad).max())
    s = 1.0 if worst <= lam else lam / worst
    gx = float((grad * x).sum())
    dual = (2.0 * s - s * s) * data - s * gx
    return F - dual, s


def certified_fstar(dirty_L, psf_L, dirty_H, psf_H, ell, delta, sigma2, lam, low_res, x_start=None, chunk=5000,
                    max_iters=200000, gap_tol=1e-9, device=0, positivity=True, log=None):
    """F* of step 2 from the FP64 path on the given data (arrays or tensors,
    e.g. the float32 inputs of an FP32 solve, converted exactly): FISTA
    (Algorithm 1) continued in chunks of `chunk` iterations (msr_get_state /
    msr_set_state, so the momentum runs on) until the duality gap of the
    iterate is <= gap_tol |F|.  Returns a dict with F (the objective of the
    last iterate, >= F*), the gap (F - gap <= F* <= F), the iterations, the
    wall time and the FP64 iterate."""
    import torch

    from .binding import Solver

    dev = torch.device("cuda", device)
    T = lambda a: a.to(dev, torch.float64).contiguous() if torch.is_tensor(a) else \
        torch.from_numpy(np.ascontiguousarray(a, np.float64)).to(dev)  # noqa: E731
    dh = T(dirty_H)
    s = Solver(dh.shape[0], positivity=positivity, precision=64)
    s.set_dirty_psf(1, T(dirty_L), T(psf_L))
    s.set_dirty_psf(2, dh, T(psf_H))
    s.set_filters(ell, delta, sigma2, 1e-3 * sigma2)
    l64 = T(low_res)
    s.lipschitz(2)
    x0 = None if x_start is None else T(x_start)
    done, rec = 0, None
    t0 = time.perf_counter()
    while done < max_iters:
        if done > 0:
            s.set_state(2, bk, bp, k)
            beta, r = s.step2(lam, l64, chunk)
        else:
            beta, r = s.step2(lam, l64, chunk, x0=x0)
        bk, bp, k = s.get_state(2)
        done += chunk
        g = s.gradient(2, beta, l64)
        F, data, _ = s.objective(2, lam, beta, l64)
        gap, sc = duality_gap(F, data, g, beta, lam, positivity)
        rec = {"F": F, "gap": gap, "rel_gap": gap / abs(F), "iters": done, "scale": sc,
               "s": time.perf_counter() - t0}
        if log:
            log(f"certified F*: {done} FP64 iterations, F = {F:.15g}, gap/|F| = {gap / abs(F):.3g}")
        if gap <= gap_tol * abs(F):
            break
    rec["beta"] = beta
    return rec


WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")


def load_weights(name="unet_w32_l4_1024"):
    """Parameters of a trained warm-start network stored with the package
    (bfloat16, the order of UNet.get_params) as float32, and their record
    (how and on what they were trained).  None if the file is absent."""
    path = os.path.join(WEIGHTS, name + ".bf16")
    if not os.path.exists(path):
        return None, None
    raw = np.fromfile(path, dtype="<u2").astype(np.uint32) << 16
    with open(os.path.join(WEIGHTS, name + ".json")) as f:
        meta = json.load(f)
    return raw.view(np.float32), meta


# --------------------------------------------------------------------------
# Objective trajectories and the time to a tolerance read from them
# --------------------------------------------------------------------------
def trajectory(solver, lam, low_res, x0=None, iters=20000, every=500, momentum_k=0):
    """Step 2 run for `iters` iterations of Algorithm 1 in chunks of `every`
    (continued exactly through msr_get_state / msr_set_state), from x0 (None:
    zero) restarted at k = 1, or, with momentum_k > 0, entered at iteration
    momentum_k + 1 with zero velocity.  Records after each chunk the
    iteration count, the exact objective F (FP64 reductions) and the
    cumulative HIP-event time of the iteration loops (objective evaluations
    excluded).  Returns {"k": [...], "F": [...], "ms": [...]}."""
    import torch

    if momentum_k > 0:
        z = x0 if x0 is not None else torch.zeros_like(low_res)
        z = z.to(getattr(solver, "state_dtype", z.dtype))  # float64 iterates take a float64 state
        solver.set_state(2, z, z, momentum_k)
        x0 = None
    out = {"k": [], "F": [], "ms": []}
    done, ms = 0, 0.0
    while done < iters:
        step = min(every, iters - done)
        if done > 0:
            solver.set_state(2, bk, bp, kk)
        beta, r = solver.step2(lam, low_res, step, x0=x0 if done == 0 else None)
        bk, bp, kk = solver.get_state(2)
        done += step
        ms += r.elapsed_ms
        out["k"].append(done)
        out["F"].append(r.objective)
        out["ms"].append(ms)
    return out


def crossing(traj, f_ref, tol=1e-6, warm_ms=0.0):
    """First recorded point of a trajectory with (F - f_ref) / |f_ref| <= tol:
    {"iters", "ms" (plus warm_ms), "converged"}; iters -1 if never."""
    for k, F, ms in zip(traj["k"], traj["F"], traj["ms"]):
        if (F - f_ref) / abs(f_ref) <= tol:
            return {"iters": int(k), "ms": ms + warm_ms, "converged": True}
    return {"iters": -1, "ms": -1.0, "converged": False}
