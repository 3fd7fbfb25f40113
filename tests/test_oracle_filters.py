"""Pins of the filter responses (Eqs. 6-10)."""
import numpy as np
import pytest

from oracle import filters


@pytest.mark.parametrize("sigma2,eta2", [(1.0, 1.2), (2.2e-4, 2.2e-7), (3.0, 0.5)])
def test_noise_normalisation_everywhere(sigma2, eta2):
    ell, delta = 20.0, 5.0
    r = np.linspace(0, 60, 6001)
    gL, gH = filters.responses(r, ell, delta, sigma2, eta2)
    np.testing.assert_allclose(sigma2 * gH**2 + eta2 * gL**2, 1.0, rtol=1e-13)
    assert np.all(gL >= 0) and np.all(gH >= 0)


def test_flat_regions_and_limits():
    sigma2, eta2 = 1.0, 1.2  # the example parameters of Fig. 3
    ell, delta = 20.0, 5.0
    gL, gH = filters.responses(np.array([0.0, 14.9, 25.1, 100.0]), ell, delta, sigma2, eta2)
    np.testing.assert_allclose(gL[:2], 1 / np.sqrt(eta2))
    np.testing.assert_allclose(gH[:2], 0.0)
    np.testing.assert_allclose(gH[2:], 1 / np.sqrt(sigma2))
    np.testing.assert_allclose(gL[2:], 0.0)


def test_continuity_at_band_edges():
    sigma2, eta2, ell, delta = 1.0, 1.2, 20.0, 5.0
    eps = 1e-9
    for edge in (ell - delta, ell + delta):
        a = filters.responses(np.array([edge - eps, edge, edge + eps]), ell, delta, sigma2, eta2)
        for g in a:
            assert abs(g[0] - g[1]) < 1e-6 and abs(g[1] - g[2]) < 1e-6


def test_monotone_crossfade():
    r = np.linspace(15, 25, 1001)
    gL, gH = filters.responses(r, 20.0, 5.0, 1.0, 1.2)
    assert np.all(np.diff(gL) <= 1e-15)
    assert np.all(np.diff(gH) >= -1e-15)


def test_grid_uses_signed_radius():
    P = 16
    r = filters.radial_grid(P)
    assert r[0, 0] == 0
    assert r[0, P - 1] == 1.0  # index P-1 is frequency -1
    assert r[P // 2, 0] == P // 2
