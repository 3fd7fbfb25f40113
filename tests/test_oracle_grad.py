"""Gradients of Eqs. 11-12 against central finite differences of the objectives
of Eqs. 4-5, and the closed-form special cases."""
import numpy as np
import pytest

import synth
from synth.generator import tiny
from oracle import objectives, filters, conv


@pytest.fixture(scope="module")
def prob():
    return synth.make_problem(tiny(16, seed=21))


def _fd_check(fun, grad, x, seed, h=1e-5, ndir=6):
    rng = np.random.default_rng(seed)
    g = grad(x)
    for _ in range(ndir):
        d = rng.normal(size=x.shape)
        fd = (fun(x + h * d) - fun(x - h * d)) / (2 * h)
        an = float(np.vdot(g, d))
        assert fd == pytest.approx(an, rel=1e-7, abs=1e-9 * abs(an) + 1e-12)


def test_grad_step1(prob):
    s1 = objectives.Step1(prob.dirty_L, prob.psf_L)
    x = np.random.default_rng(1).normal(size=(16, 16)) * 0.1
    _fd_check(s1.data_term, s1.grad, x, 2)


def test_grad_step2(prob):
    l = np.random.default_rng(5).normal(size=(16, 16))
    s2 = objectives.Step2(prob.dirty_H, prob.psf_H, l, prob.ell, prob.delta, 1.3, 0.7)
    x = np.random.default_rng(3).normal(size=(16, 16)) * 0.1
    _fd_check(lambda z: sum(s2.data_terms(z)), s2.grad, x, 4)


def test_grad_linear_part_is_twice_normal(prob):
    """grad f(x) - grad f(0) = 2 A x (both steps)."""
    s1 = objectives.Step1(prob.dirty_L, prob.psf_L)
    l = np.random.default_rng(5).normal(size=(16, 16))
    s2 = objectives.Step2(prob.dirty_H, prob.psf_H, l, prob.ell, prob.delta, 1.3, 0.7)
    x = np.random.default_rng(8).normal(size=(16, 16))
    z = np.zeros_like(x)
    for s in (s1, s2):
        np.testing.assert_allclose(s.grad(x) - s.grad(z), 2 * s.normal(x), atol=1e-9 * np.abs(s.grad(x)).max())


def test_step2_filter_norm_matches_spatial_definition(prob):
    """||C_g E r||^2 computed in the spectral domain equals the spatial norm of the
    filtered, zero-embedded image (Parseval)."""
    P = prob.P
    l = np.zeros((16, 16))
    s2 = objectives.Step2(prob.dirty_H, prob.psf_H, l, prob.ell, prob.delta, 1.0, 1.0)
    r = np.random.default_rng(2).normal(size=(16, 16))
    gL, gH = filters.responses(filters.radial_grid(P), prob.ell, prob.delta, 1.0, 1.0)
    filt = np.fft.ifft2(gH * np.fft.fft2(conv.embed(r, P)))
    spatial = float(np.sum(np.abs(filt) ** 2))
    assert objectives._filter_norm2(r, s2.gH2, P) == pytest.approx(spatial, rel=1e-12)


def test_step2_reduces_to_identity_case():
    """delta PSF, sigma^2 = eta^2 = 1, i_H = l  =>  f2(x) = ||l - x||^2 (g_H^2 + g_L^2 = 1)."""
    n, P = 8, 16
    psf = np.zeros((P, P))
    psf[P // 2, P // 2] = 1.0
    l = np.random.default_rng(0).normal(size=(n, n))
    s2 = objectives.Step2(l, psf, l, 3.0, 1.0, 1.0, 1.0)
    x = np.random.default_rng(1).normal(size=(n, n))
    assert sum(s2.data_terms(x)) == pytest.approx(float(np.sum((l - x) ** 2)), rel=1e-12)
    np.testing.assert_allclose(s2.grad(x), 2 * (x - l), atol=1e-12)
