"""The duality-gap certificate of the reference objective (warmstart.duality_gap)
against the oracle.  Weak duality: the gap bounds F(x) - F* from above at any x
(checked on both steps with the synthetic PSFs, against the best minimiser
FISTA reaches).  Exactness: with a delta PSF (H = I) the minimiser of
||y - x||^2 + lam ||x||_1 [+ x >= 0] is the closed form tau_{lam/2}(y) (its
positive part with positivity), where the gap must vanish, and the gap of
any other point must be at least its excess over that closed-form optimum
(Eqs. 4, 5; for step 2 with sigma^2 = eta^2 = 1 and the data image equal to l,
f(x) = ||l - x||^2)."""
import numpy as np
import pytest

import synth
from synth.generator import tiny
from oracle import objectives, fista, lipschitz
from paper_2406_18356_amd.warmstart import duality_gap


def _delta(P):
    d = np.zeros((P, P))
    d[P // 2, P // 2] = 1.0
    return d


@pytest.mark.parametrize("positivity", [True, False])
@pytest.mark.parametrize("step", [1, 2])
def test_gap_exact_for_the_identity_operator(positivity, step):
    pr = synth.make_problem(tiny(16, seed=4))
    y = pr.dirty_H
    if step == 1:
        prob = objectives.Step1(y, _delta(pr.P))
    else:
        prob = objectives.Step2(y, _delta(pr.P), y, pr.ell, pr.delta, 1.0, 1.0)
    lam = 0.02 * float(np.linalg.norm(y))
    xs = np.maximum(y - lam / 2, 0.0) if positivity else np.sign(y) * np.maximum(np.abs(y) - lam / 2, 0.0)
    assert np.count_nonzero(xs) > 0 and np.count_nonzero(xs) < xs.size
    F, data, _ = prob.objective(xs, lam)
    gap, s = duality_gap(F, data, prob.grad(xs), xs, lam, positivity)
    assert abs(gap) <= 1e-12 * abs(F) and s == pytest.approx(1.0, abs=1e-12)
    rng = np.random.default_rng(2)
    for x in (np.zeros_like(y), xs + 0.05 * lam * rng.normal(size=y.shape), np.abs(y)):
        if positivity:
            x = np.maximum(x, 0.0)
        Fx, dx, _ = prob.objective(x, lam)
        g, _ = duality_gap(Fx, dx, prob.grad(x), x, lam, positivity)
        assert g >= (Fx - F) - 1e-12 * abs(F)
        assert g > 0


@pytest.mark.parametrize("positivity", [True, False])
def test_gap_bounds_the_excess_with_real_psfs(positivity):
    pr = synth.make_problem(tiny(16, seed=4))
    probs = [objectives.Step1(pr.dirty_L, pr.psf_L),
             objectives.Step2(pr.dirty_H, pr.psf_H, 0.5 * pr.dirty_L, pr.ell, pr.delta, 0.7, 0.2)]
    rng = np.random.default_rng(1)
    for prob in probs:
        n = prob.n
        lam = 0.02 * float(np.linalg.norm(prob.y))
        th = 1.01 * lipschitz.power_iteration(prob.normal, n)[0]
        snaps = {}
        xb, _ = fista.fista(prob.grad, np.zeros((n, n)), 1 / th, lam, 2000, positivity=positivity,
                            callback=lambda k, b: snaps.__setitem__(k, b.copy()) if k in (10, 100, 1000) else None)
        snaps[2000] = xb
        Fb = prob.objective(xb, lam)[0]
        gaps = []
        for K in (10, 100, 1000, 2000):
            x = snaps[K]
            F, data, _ = prob.objective(x, lam)
            gap, s = duality_gap(F, data, prob.grad(x), x, lam, positivity)
            assert 0 < s <= 1
            assert gap >= (F - Fb) - 1e-12 * abs(Fb)   # F* <= F(xb): weak duality implies this
            gaps.append(gap)
        assert gaps[-1] < gaps[0]                      # and the bound tightens along the run
        x = np.abs(rng.normal(size=(n, n))) * 0.01 * (1 if positivity else np.sign(rng.normal(size=(n, n))))
        F, data, _ = prob.objective(x, lam)
        gap, _ = duality_gap(F, data, prob.grad(x), x, lam, positivity)
        assert gap >= (F - Fb) - 1e-12 * abs(Fb)
