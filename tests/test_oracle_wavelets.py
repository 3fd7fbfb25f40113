"""Pins of the wavelet dictionary oracle (db1 .. db8 concatenation, Sect. 3,
App. A.1): the filters against closed forms and their defining properties,
the transforms' orthonormality, W W^T = M I, and the Lipschitz constant of
Sect. 3.4 for circular convolutions."""
import numpy as np
import pytest

import synth
from synth.generator import tiny
from oracle import wavelets as wv, objectives, lipschitz


def test_haar_and_db2_closed_forms():
    np.testing.assert_allclose(wv.daubechies(1), [2 ** -0.5, 2 ** -0.5], atol=1e-15)
    s3 = np.sqrt(3.0)
    db2 = np.array([1 + s3, 3 + s3, 3 - s3, 1 - s3]) / (4 * np.sqrt(2.0))
    np.testing.assert_allclose(wv.daubechies(2), db2, atol=1e-13)


@pytest.mark.parametrize("p", range(1, 9))
def test_filter_properties(p):
    h = wv.daubechies(p)
    g = wv.highpass(h)
    assert h.size == 2 * p
    assert np.sum(h) == pytest.approx(np.sqrt(2.0), abs=1e-12)
    # orthonormal to its even shifts
    for m in range(p):
        s = float(np.dot(h[2 * m:], h[:h.size - 2 * m]))
        assert s == pytest.approx(1.0 if m == 0 else 0.0, abs=1e-10)
    # p vanishing moments of the wavelet
    n = np.arange(h.size, dtype=np.float64)
    for q in range(p):
        assert abs(np.sum(n ** q * g)) <= 1e-8 * np.sum(np.abs(n ** q * g))
    # H(z) = (1 + z^-1)^p R(z) with R minimum phase (roots inside the unit circle)
    r = h.copy()
    for _ in range(p):
        r, rem = np.polydiv(r, [1.0, 1.0])
        assert np.max(np.abs(rem)) <= 1e-9
    if r.size > 1:
        assert np.all(np.abs(np.roots(r)) < 1.0)


@pytest.mark.parametrize("p", [1, 3, 8])
def test_transform_orthonormal(p):
    x = np.random.default_rng(p).normal(size=(32, 32))
    c = wv.dwt2(x, p)
    assert np.linalg.norm(c) == pytest.approx(np.linalg.norm(x), rel=1e-12)
    np.testing.assert_allclose(wv.idwt2(c, p), x, atol=1e-11)
    # the nested layout: the coarsest approximation (2x2 after 4 levels of 32) holds the mean times 16
    assert c[:2, :2].mean() == pytest.approx(x.mean() * 16, rel=1e-10)


def test_dictionary_identities():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(16, 16))
    a = rng.normal(size=(8, 16, 16))
    np.testing.assert_allclose(wv.synthesis(wv.analysis(x)), 8 * x, atol=1e-10)
    assert np.sum(wv.synthesis(a) * x) == pytest.approx(np.sum(a * wv.analysis(x)), rel=1e-12)


def _power(normal, shape, iters=3000, seed=0):
    v = np.random.default_rng(seed).normal(size=shape)
    th = prev = 0.0
    for _ in range(iters):
        w = normal(v)
        th = 2.0 * float(np.sum(v * w) / np.sum(v * v))
        v = w / np.linalg.norm(w)
        if abs(th - prev) <= 1e-10 * th:
            break
        prev = th
    return th


def test_lipschitz_with_dictionary():
    """Circular convolution: theta = 2 M max|h_hat|^2 (Sect. 3.4); zero padded:
    theta(W^T A W) = M theta(A) because W W^T = M I."""
    pr = synth.make_problem(tiny(16, seed=6).replace(pad=1))
    s1 = objectives.Step1(pr.dirty_L, pr.psf_L)
    d = wv.InDictionary(s1)
    th = _power(d.normal, (8, 16, 16))
    assert th == pytest.approx(2 * 8 * float(np.max(np.abs(s1.H.h))) ** 2, rel=1e-6)
    pr2 = synth.make_problem(tiny(16, seed=7))
    s2 = objectives.Step1(pr2.dirty_L, pr2.psf_L)
    thA = _power(s2.normal, (16, 16))
    thW = _power(wv.InDictionary(s2).normal, (8, 16, 16))
    assert thW == pytest.approx(8 * thA, rel=1e-6)
