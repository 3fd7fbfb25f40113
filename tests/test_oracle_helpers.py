"""Pins of the parameter helpers (Sect. 4.3, Sect. 5, App. A.2) and of the
two-step driver."""
import os

import numpy as np
import pytest

import synth
from synth.generator import tiny
from oracle import helpers, twostep, objectives, lipschitz

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_sigma2_hat_iid_expectation():
    """For iid N(0, s^2) pixels a 25-pixel population variance has mean (24/25) s^2."""
    rng = np.random.default_rng(0)
    s = 0.3
    vals = [helpers.sigma2_hat(rng.normal(0, s, (128, 128))) for _ in range(8)]
    assert np.mean(vals) == pytest.approx(24 / 25 * s * s, rel=5e-3)


def test_sigma2_hat_brute_force_windows():
    img = np.random.default_rng(1).normal(size=(9, 7))
    acc = []
    for i in range(9 - 4):
        for j in range(7 - 4):
            w = img[i : i + 5, j : j + 5].ravel()
            acc.append(np.mean((w - w.mean()) ** 2))
    assert helpers.sigma2_hat(img) == pytest.approx(np.mean(acc), rel=1e-13)


def test_eta2_ratio_matches_table2():
    """Table 2: eta2_hat = 1e-3 sigma2_hat in every row except Sgr B2, ell = 20
    (printed 2.2e-7 for sigma2_hat = 2.2e-5, a factor 10 off the stated rule)."""
    rows = np.loadtxt(os.path.join(GOLD, "table2_sigma_eta.txt"), comments="#")
    hits = 0
    for ds, ell, s2, s2h, e2, e2h in rows:
        if helpers.eta2_hat(s2h) == pytest.approx(e2h, rel=1e-9):
            hits += 1
        else:
            assert (ds, ell) == (1, 20)
    assert hits == 8


def test_default_lambda_schedule():
    d = np.full((4, 4), 0.5)  # ||d||_2 = 2
    assert helpers.default_lambda(d, 0.05) == pytest.approx(0.1)
    assert helpers.default_lambda(d, 0.05, cycle=3) == pytest.approx(0.4)
    assert helpers.default_lambda(d, 0.01) == pytest.approx(0.02)


def test_psnr():
    t = np.zeros((4, 4))
    t[0, 0] = 10.0
    x = t + 0.1
    assert helpers.psnr(x, t) == pytest.approx(20 * np.log10(10 / 0.1))


def test_two_step_runs_and_improves():
    pr = synth.make_problem(tiny(32, seed=2))
    r = twostep.two_step(pr.dirty_L, pr.psf_L, pr.dirty_H, pr.psf_H, pr.ell, pr.delta, 60, 60,
                         positivity=True)
    assert r["eta2"] == pytest.approx(1e-3 * r["sigma2"])
    s2 = objectives.Step2(pr.dirty_H, pr.psf_H, r["i_L"], pr.ell, pr.delta, r["sigma2"], r["eta2"])
    assert s2.objective(r["beta2"], r["lambda2"])[0] < s2.objective(np.zeros((32, 32)), r["lambda2"])[0]
    assert np.all(r["beta2"] >= 0)


def test_major_cycles_pins():
    """One cycle is the single-cycle step; with a delta PSF the residual
    bookkeeping returns the dirty image exactly; the lambda schedule doubles."""
    pr = synth.make_problem(tiny(16, seed=3))
    s1 = objectives.Step1(pr.dirty_L, pr.psf_L)
    th = 2.0 * float(np.max(np.abs(s1.H.h))) ** 2
    img, msum, recs = twostep.major_cycles(1, pr.dirty_L, pr.psf_L, 1, 30, theta=th, positivity=True)
    beta, _, _ = twostep.solve_step(s1, helpers.default_lambda(pr.dirty_L, 0.05), 30, th, positivity=True)
    np.testing.assert_allclose(msum, beta, atol=1e-14)
    np.testing.assert_allclose(img, helpers.low_res_image(beta, pr.dirty_L, s1.H), atol=1e-12)
    # delta PSF: H = I, so i~_{N+1} + sum i_n = i~_1 whatever the cycles do
    P = pr.P
    dpsf = np.zeros((P, P))
    dpsf[P // 2, P // 2] = 1.0
    img, msum, recs = twostep.major_cycles(1, pr.dirty_L, dpsf, 3, 20, theta=2.0)
    np.testing.assert_allclose(img, pr.dirty_L, atol=1e-12)
    assert np.abs(msum).max() > 0
    # the first cycle's lambda is c ||i~_1||; later ones use their residuals and 2^(n-1)
    assert recs[0]["lambda"] == pytest.approx(0.05 * np.linalg.norm(pr.dirty_L), rel=1e-12)
    # step 2: one cycle equals the single-cycle step 2
    l = pr.dirty_L * 0.5
    s2 = objectives.Step2(pr.dirty_H, pr.psf_H, l, pr.ell, pr.delta, 1.0, 1e-3)
    th2 = 1.01 * lipschitz.power_iteration(s2.normal, 16)[0]
    img2, msum2, _ = twostep.major_cycles(2, pr.dirty_H, pr.psf_H, 1, 25, theta=th2, low_res=l, ell=pr.ell,
                                          delta=pr.delta, sigma2=1.0, eta2=1e-3)
    b2, _, _ = twostep.solve_step(s2, helpers.default_lambda(pr.dirty_H, 0.05), 25, th2)
    np.testing.assert_allclose(msum2, b2, atol=1e-14)


def test_major_cycles_with_dictionary_pins():
    """In the dictionary: a delta PSF leaves the bookkeeping exact; a single
    cycle equals one dictionary FISTA run mapped through W; and with lambda
    = 0 and H = I a cycle's model converges to the dirty image itself (W W^T
    = 8 I, so W alpha can reach any image; theta = 2 x 8 for W^T W)."""
    from oracle import fista, wavelets

    pr = synth.make_problem(tiny(16, seed=3))
    P = pr.P
    dpsf = np.zeros((P, P))
    dpsf[P // 2, P // 2] = 1.0
    img, msum, recs = twostep.major_cycles(1, pr.dirty_L, dpsf, 2, 10, theta=16.0, dictionary=True)
    np.testing.assert_allclose(img, pr.dirty_L, atol=1e-12)
    assert np.abs(msum).max() > 0
    s1 = objectives.Step1(pr.dirty_L, pr.psf_L)
    th = 8 * 2.0 * float(np.max(np.abs(s1.H.h))) ** 2
    _, msum1, recs1 = twostep.major_cycles(1, pr.dirty_L, pr.psf_L, 1, 15, theta=th, dictionary=True)
    lam = helpers.default_lambda(pr.dirty_L, 0.05)
    dic = wavelets.InDictionary(s1)
    a, _ = fista.fista(dic.grad, np.zeros((8, 16, 16)), 1.0 / th, lam, 15)
    np.testing.assert_allclose(msum1, wavelets.synthesis(a), atol=1e-14)
    assert recs1[0]["F"] == pytest.approx(dic.objective(a, lam)[0], rel=1e-14)
    # lambda -> 0, H = I: FISTA on ||y - W alpha||^2 drives W alpha to y
    _, m0, _ = twostep.major_cycles(1, pr.dirty_L, dpsf, 1, 400, c=0.0, theta=16.0 * 1.01, dictionary=True)
    np.testing.assert_allclose(m0, pr.dirty_L, atol=1e-8 * np.abs(pr.dirty_L).max())


def _soft(z, t):
    """sign(z) max(|z| - t, 0), written out element by element."""
    out = np.zeros_like(z)
    for idx, v in np.ndenumerate(z):
        out[idx] = (v - t) if v > t else ((v + t) if v < -t else 0.0)
    return out


def _delta_psf(P):
    d = np.zeros((P, P))
    d[P // 2, P // 2] = 1.0
    return d


@pytest.mark.parametrize("positivity", [False, True])
def test_major_cycles_step1_closed_form(positivity):
    """Cycles n >= 2 of step 1 in closed form (Sect. 3.2, Sect. 5 / App. A.2).

    With a delta PSF, H = I and f(x) = ||i~ - x||^2, so theta = 2 gives
    mu = 1/2 and the first prox step lands on the minimiser
    tau_{lambda/2}(i~) (positive part with positivity); the momentum term is
    then zero for ever, so every cycle's FISTA result is exact after any K.
    Cycle n therefore gives i_n = tau_{lambda_n/2}(i~_n) with
    i~_n = i~_1 - sum_{j<n} i_j and lambda_n = c ||i~_n|| 2^(n-1); the
    recursion below is run independently of the oracle's operators."""
    pr = synth.make_problem(tiny(16, seed=3))
    c = 0.02
    y = pr.dirty_L
    msum = np.zeros_like(y)
    lams, parts = [], []
    for n in range(1, 4):
        resid = y - msum
        lam = c * np.sqrt(np.sum(resid * resid)) * 2.0 ** (n - 1)
        i_n = np.maximum(resid - lam / 2, 0.0) if positivity else _soft(resid, lam / 2)
        lams.append(lam)
        parts.append(i_n)
        msum = msum + i_n
    # every later cycle does something, else the pin would not see its bookkeeping
    assert all(np.abs(p).max() > 1e-3 * np.abs(y).max() for p in parts[1:])
    img, got, recs = twostep.major_cycles(1, y, _delta_psf(pr.P), 3, 3, c=c, theta=2.0, positivity=positivity)
    np.testing.assert_allclose(got, msum, atol=1e-13 * np.abs(y).max())
    np.testing.assert_allclose([r["lambda"] for r in recs], lams, rtol=1e-13)
    np.testing.assert_allclose(img, y, atol=1e-13 * np.abs(y).max())


def test_major_cycles_step2_closed_form():
    """Cycles n >= 2 of step 2 in closed form (Eq. 5's l_{L_n}, Sect. 3.3).

    With a delta PSF, sigma^2 = eta^2 = 1 (so g_H^2 + g_L^2 = 1 everywhere,
    Eqs. 6-10) and the data image equal to the constraint l, the data
    residual of cycle n and its constraint l_n = l - sum_{j<n} i_j are the
    same image, grad f = 2 E^T C_{g_H^2 + g_L^2} E (x - l_n) = 2 (x - l_n), and
    theta = 2 makes one prox step exact: i_n = tau_{lambda_n/2}(l - sum_{j<n} i_j)
    with lambda_n = c ||l - sum_{j<n} i_j|| 2^(n-1).  A constraint left at l
    (not l_n) pulls every later cycle towards l and fails this."""
    pr = synth.make_problem(tiny(16, seed=5))
    c = 0.02
    l = pr.dirty_H.copy()
    msum = np.zeros_like(l)
    lams, parts = [], []
    for n in range(1, 4):
        resid = l - msum
        lam = c * np.sqrt(np.sum(resid * resid)) * 2.0 ** (n - 1)
        i_n = _soft(resid, lam / 2)
        lams.append(lam)
        parts.append(i_n)
        msum = msum + i_n
    assert all(np.abs(p).max() > 1e-3 * np.abs(l).max() for p in parts[1:])
    img, got, recs = twostep.major_cycles(2, l, _delta_psf(pr.P), 3, 3, c=c, theta=2.0, low_res=l,
                                          ell=pr.ell, delta=pr.delta, sigma2=1.0, eta2=1.0)
    np.testing.assert_allclose(got, msum, atol=1e-12 * np.abs(l).max())
    np.testing.assert_allclose([r["lambda"] for r in recs], lams, rtol=1e-13)
