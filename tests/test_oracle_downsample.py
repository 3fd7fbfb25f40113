"""Pins of the down-sampled low-resolution image oracle (Sect. 6.1): the
decimation D and up-sampling U against sampling and band-limited closed
forms, U written out as the Dirichlet-kernel matrix, and the identity
|| G_L' (l_s - D x) ||^2 = || G_L (U l_s - x) ||^2 in circular mode that lets
step 2 use the small image through U."""
import numpy as np
import pytest

from oracle import downsample as ds
from oracle.filters import squared_on_grid


@pytest.mark.parametrize("N,d", [(16, 2), (32, 4), (64, 2)])
def test_decimate_undoes_upsample(N, d):
    ls = np.random.default_rng(N).normal(size=(N // d, N // d))
    np.testing.assert_allclose(ds.decimate(ds.upsample(ls, d), d), ls, atol=1e-12)


@pytest.mark.parametrize("N,d", [(16, 2), (32, 4)])
def test_upsample_interpolates_the_coarse_samples(N, d):
    """U l_s takes the value l_s[i, j] / d^2 (the coarse pixel's flux spread
    over d^2 fine pixels) at the fine pixel (d i, d j): the Dirichlet kernel
    vanishes at the other coarse sample points."""
    ls = np.random.default_rng(1).normal(size=(N // d, N // d))
    np.testing.assert_allclose(ds.upsample(ls, d)[::d, ::d], ls / (d * d), atol=1e-12)


def test_band_limited_closed_forms():
    """A band-limited image: sampling a cosine of frequency a < N_s/2 on the
    coarse grid and up-sampling gives the cosine on the fine grid (divided by
    d^2: flux per pixel); D of the fine cosine is d^2 times its coarse
    samples."""
    N, d = 64, 4
    m = N // d
    n = np.arange(N)
    for a, b, ph in ((3, 5, 0.3), (0, 7, 1.1), (6, 0, -0.4)):
        fine = np.cos(2 * np.pi * (a * n[:, None] + b * n[None, :]) / N + ph)
        coarse = fine[::d, ::d]
        np.testing.assert_allclose(ds.upsample(coarse, d), fine / (d * d), atol=1e-12)
        np.testing.assert_allclose(ds.decimate(fine, d), coarse * d * d, atol=1e-11)
    # flux: a constant fine image of value f decimates to d^2 f
    np.testing.assert_allclose(ds.decimate(np.full((N, N), 0.7), d), np.full((m, m), 0.7 * d * d), atol=1e-12)


@pytest.mark.parametrize("N,d", [(16, 2), (32, 2), (32, 4)])
def test_interpolation_matrix_equals_fft_upsampling(N, d):
    ls = np.random.default_rng(2).normal(size=(N // d, N // d))
    K = ds.interpolation_matrix(N, d)
    np.testing.assert_allclose(K @ ls @ K.T, ds.upsample(ls, d), atol=1e-12)


@pytest.mark.parametrize("N,d,ell,delta", [(32, 2, 4.0, 1.5), (64, 4, 4.5, 2.0), (64, 2, 10.0, 3.0)])
def test_small_grid_term_equals_full_grid_term_circular(N, d, ell, delta):
    """Circular mode: the paper's small-grid term with D and G_L' equals the
    full-resolution G_L term with l = U l_s, for any x and l_s."""
    rng = np.random.default_rng(N + d)
    m = N // d
    assert ell + delta < m / 2
    s2, e2 = 0.8, 0.3
    x = rng.normal(size=(N, N))
    ls = rng.normal(size=(m, m))
    small = ds.small_term(x, ls, d, m, ell, delta, s2, e2)
    gL2, _ = squared_on_grid(N, ell, delta, s2, e2)
    R = np.fft.fft2(ds.upsample(ls, d) - x)
    full = float(np.sum(gL2 * np.abs(R) ** 2) / (N * N))
    assert small == pytest.approx(full, rel=1e-12)
