"""Pins of the oracle's convolution operator H.

* the spatial sum (the definition) = separable DFT = FFT back-end, FP64;
* adjointness, and H = H^T for a point-symmetric PSF;
* a delta PSF gives the identity;
* zero padding to P = 2N gives the linear convolution regardless of where
  the image is embedded (independent check with a hand-rolled np.convolve).
"""
import numpy as np
import pytest
from scipy.signal import convolve2d

from oracle import conv


def _rand(n, P, seed, symmetric=False):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, n))
    psf = rng.normal(size=(P, P))
    if symmetric:
        c = P // 2
        # point symmetry about (P/2, P/2): psf[c+a, c+b] = psf[c-a, c-b]
        flipped = np.roll(np.flip(psf, (0, 1)), 1, axis=(0, 1))
        psf = 0.5 * (psf + flipped)
        psf[c, c] = 1.0
    return x, psf


@pytest.mark.parametrize("n,pad", [(4, 2), (8, 2), (8, 1), (6, 2)])
def test_brute_direct_fft_agree(n, pad):
    x, psf = _rand(n, pad * n, seed=n + pad)
    b = conv.conv_brute(x, psf)
    bv = conv.conv_brute_vec(x, psf)
    d = conv.conv_direct(x, psf)
    f = conv.conv_fft(x, psf)
    s = np.max(np.abs(b))
    np.testing.assert_allclose(bv, b, atol=1e-12 * s)
    np.testing.assert_allclose(d, b, atol=1e-12 * s)
    np.testing.assert_allclose(f, b, atol=1e-12 * s)
    for adj in (True,):
        ba = conv.conv_brute(x, psf, adjoint=adj)
        np.testing.assert_allclose(conv.conv_direct(x, psf, adjoint=adj), ba, atol=1e-12 * s)
        np.testing.assert_allclose(conv.conv_fft(x, psf, adjoint=adj), ba, atol=1e-12 * s)


def test_brute_vs_fft_n16():
    x, psf = _rand(16, 32, seed=5)
    np.testing.assert_allclose(conv.conv_fft(x, psf), conv.conv_brute_vec(x, psf), atol=1e-11)


def test_linear_convolution_matches_scipy():
    """With P = 2N the operator is the linear convolution with the PSF's central part."""
    n = 8
    P = 2 * n
    x, psf = _rand(n, P, seed=9)
    c = P // 2
    # kernel K[a, b] = PSF[c + a, c + b] for a, b in (-n, n); convolve2d 'full' then take
    # the block aligned with the output grid.
    K = psf[c - n + 1 : c + n, c - n + 1 : c + n]
    full = convolve2d(x, K, mode="full")  # index (p + n - 1) for output p
    ref = full[n - 1 : 2 * n - 1, n - 1 : 2 * n - 1]
    np.testing.assert_allclose(conv.conv_fft(x, psf), ref, atol=1e-12)


def test_adjoint_identity():
    x, psf = _rand(16, 32, seed=3)
    rng = np.random.default_rng(4)
    y = rng.normal(size=(16, 16))
    op = conv.Operator(psf, 16)
    lhs = np.vdot(op.apply(x), y)
    rhs = np.vdot(x, op.adjoint(y))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_symmetric_psf_gives_self_adjoint():
    x, psf = _rand(16, 32, seed=6, symmetric=True)
    op = conv.Operator(psf, 16)
    assert np.max(np.abs(op.h.imag)) < 1e-12 * np.max(np.abs(op.h))
    np.testing.assert_allclose(op.apply(x), op.adjoint(x), atol=1e-12)


def test_delta_psf_is_identity():
    n, P = 8, 16
    psf = np.zeros((P, P))
    psf[P // 2, P // 2] = 1.0
    x = np.random.default_rng(0).normal(size=(n, n))
    np.testing.assert_allclose(conv.conv_brute(x, psf), x, atol=0)
    np.testing.assert_allclose(conv.conv_fft(x, psf), x, atol=1e-14)


def test_embedding_offset_is_irrelevant_when_padded():
    """E at offset (P-N)/2 and at offset 0 give the same cropped result for P = 2N
    (the circulant commutes with shifts and no wrap occurs)."""
    n, P = 16, 32
    x, psf = _rand(n, P, seed=12)
    h = np.fft.fft2(np.fft.ifftshift(psf))
    big = np.zeros((P, P))
    big[:n, :n] = x
    y0 = np.fft.ifft2(h * np.fft.fft2(big)).real[:n, :n]
    np.testing.assert_allclose(conv.conv_fft(x, psf), y0, atol=1e-12)
