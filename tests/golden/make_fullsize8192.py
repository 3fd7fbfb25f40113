"""Writes tests/golden/fullsize8192.npz: FP64 oracle values for the 8192^2
workload (16384^2 grid; synth preset sky8192) that the GPU parity test
compares against on a central crop and the four corners (stored as float32:
rounding 6e-8 of each value, far below the 1e-5 tolerance of the test).

Everything here is the oracle's (oracle/) on the seeded synthetic inputs
(synth/): for each step, K = 10 FISTA iterations from x0 = 0 (Algorithm 1)
and 2 iterations continued from a late state (beta_500, beta_499; the
synthetic images of synth.late_state, rounded to float32 as the GPU receives
them), with the closed-form step-size bounds
    theta_1 = 2 max|h_hat|^2,
    theta_2 = 2 (max g_H^2 max|h_hat|^2 + max g_L^2),
lambda = 0.05 ||i~|| (Sect. 5), sigma^2 from the 5 x 5 window estimator and
eta^2 = 1e-3 sigma^2 (Sect. 4.3), and the step-2 constraint l = the
short-baseline dirty image (float32-rounded).  The run takes about ten
minutes and ~25 GB of host memory.

    python tests/golden/make_fullsize8192.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import fista, helpers, objectives  # noqa: E402

K, LATE_K, CROP = 10, 500, 512


def crops(x, n):
    h = CROP // 2
    return [x[n // 2 - h:n // 2 + h, n // 2 - h:n // 2 + h], x[:64, :64], x[:64, -64:], x[-64:, :64],
            x[-64:, -64:]]


def main():
    t0 = time.time()
    log = lambda m: print(f"[{time.time() - t0:7.1f} s] {m}", flush=True)  # noqa: E731
    pr = synth.make_problem(synth.preset("sky8192"), with_full=False, progress=log)
    n = pr.n
    out = {"n": n, "crop": CROP, "K": K, "late_k": LATE_K}
    for step in (1, 2):
        if step == 1:
            prob = objectives.Step1(pr.dirty_L, pr.psf_L)
            lam = helpers.default_lambda(pr.dirty_L)
            th = 2.0 * float(np.max(np.abs(prob.H.h))) ** 2
        else:
            del prob
            low = np.asarray(pr.dirty_L, np.float32).astype(np.float64)
            sig2 = helpers.sigma2_hat(pr.dirty_H)
            out["sigma2"] = sig2
            log(f"sigma2_hat = {sig2:.6g}")
            prob = objectives.Step2(pr.dirty_H, pr.psf_H, low, pr.ell, pr.delta, sig2, 1e-3 * sig2)
            lam = helpers.default_lambda(pr.dirty_H)
            th = 2.0 * (float(np.max(prob.gH2)) * float(np.max(np.abs(prob.H.h))) ** 2 + float(np.max(prob.gL2)))
        out[f"theta{step}"], out[f"lambda{step}"] = th, lam
        log(f"step {step}: theta {th:.6g} lambda {lam:.6g}")
        b, _ = fista.fista(prob.grad, np.zeros((n, n)), 1.0 / th, lam, K, positivity=True,
                           callback=lambda k, _b: log(f"step {step} iteration {k}"))
        out[f"peak_from0{step}"] = float(np.max(np.abs(b)))
        for i, a in enumerate(crops(b, n)):
            out[f"from0{step}_{i}"] = a.astype(np.float32)
        del b
        bk, bkm1 = synth.late_state(n, seed=17 + step)
        bk, bkm1 = (np.asarray(a, np.float32).astype(np.float64) for a in (bk, bkm1))
        bl, _, _ = fista.fista_from(prob.grad, bk, bkm1, LATE_K, 1.0 / th, lam, 2, positivity=True)
        log(f"step {step} late state done")
        out[f"peak_late{step}"] = float(np.max(np.abs(bl)))
        for i, a in enumerate(crops(bl, n)):
            out[f"late{step}_{i}"] = a.astype(np.float32)
        del bl, bk, bkm1
    path = os.path.join(HERE, "fullsize8192.npz")
    np.savez_compressed(path, **out)
    log(f"wrote {path} ({os.path.getsize(path) / 1e6:.2f} MB)")


if __name__ == "__main__":
    main()
