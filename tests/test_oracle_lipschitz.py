"""Pins of the Lipschitz constant: power iteration and Lanczos against the
paper's closed form for circular convolutions (Sect. 3.4, M = 1), against
dense eigensolvers, the zero-padded bound, the identity case, and the
SplitMix64 start vector."""
import numpy as np
import pytest

import synth
from synth.generator import tiny
from oracle import objectives, lipschitz, filters, conv


def test_splitmix64_published_first_output():
    # SplitMix64 seeded with 0: the first output is 0xE220A8397B1DCDAF (a widely
    # published test value of the generator); our mix(c) is that step applied to c.
    assert lipschitz.splitmix64_mix(0) == 0xE220A8397B1DCDAF
    v = lipschitz.start_vector(4, 0)
    assert v[0, 0] == pytest.approx((0xE220A8397B1DCDAF >> 11) * 2.0**-53 - 0.5, abs=0)
    assert np.all(np.abs(v) <= 0.5)


def _dense(normal, n):
    m = np.zeros((n * n, n * n))
    for i in range(n * n):
        e = np.zeros(n * n)
        e[i] = 1.0
        m[:, i] = normal(e.reshape(n, n)).ravel()
    return m


def test_circular_closed_form_step1():
    pr = synth.make_problem(tiny(16, seed=2).replace(pad=1))
    s1 = objectives.Step1(pr.dirty_L, pr.psf_L)
    th, it, _ = lipschitz.power_iteration(s1.normal, 16, seed=1, max_iter=5000, rtol=1e-13)
    cf = lipschitz.closed_form_step1(s1.H.h)
    dense = 2 * np.linalg.eigvalsh(_dense(s1.normal, 16)).max()
    assert dense == pytest.approx(cf, rel=1e-10)
    assert th == pytest.approx(cf, rel=1e-6)
    assert th <= cf * (1 + 1e-12)


def test_circular_closed_form_step2():
    pr = synth.make_problem(tiny(16, seed=2).replace(pad=1))
    l = np.zeros((16, 16))
    s2 = objectives.Step2(pr.dirty_H, pr.psf_H, l, pr.ell, pr.delta, 0.8, 0.3)
    cf = lipschitz.closed_form_step2(s2.H.h, s2.gL2, s2.gH2)
    dense = 2 * np.linalg.eigvalsh(_dense(s2.normal, 16)).max()
    assert dense == pytest.approx(cf, rel=1e-10)
    th, _, _ = lipschitz.power_iteration(s2.normal, 16, seed=3, max_iter=5000, rtol=1e-13)
    assert th == pytest.approx(cf, rel=1e-6)


def test_padded_matches_dense_and_is_bounded():
    pr = synth.make_problem(tiny(8, seed=4))
    s1 = objectives.Step1(pr.dirty_L, pr.psf_L)
    dense = 2 * np.linalg.eigvalsh(_dense(s1.normal, 8)).max()
    th, _, _ = lipschitz.power_iteration(s1.normal, 8, seed=0, max_iter=20000, rtol=1e-14)
    assert th == pytest.approx(dense, rel=1e-8)
    assert dense <= lipschitz.closed_form_step1(s1.H.h) * (1 + 1e-12)


def test_identity_case():
    n, P = 8, 16
    psf = np.zeros((P, P))
    psf[P // 2, P // 2] = 1.0
    s1 = objectives.Step1(np.zeros((n, n)), psf)
    th, it, _ = lipschitz.power_iteration(s1.normal, n, seed=0)
    assert th == pytest.approx(2.0, rel=1e-12)
    assert it <= 3


@pytest.mark.parametrize("pad,step", [(1, 1), (1, 2), (2, 1), (2, 2)])
def test_lanczos_matches_dense(pad, step):
    """Lanczos reaches the dense eigenvalue (and, circular, the closed form);
    its Ritz values never exceed it and never decrease."""
    n = 16
    pr = synth.make_problem(tiny(n, seed=2 if pad == 1 else 3).replace(pad=pad))
    if step == 1:
        prob = objectives.Step1(pr.dirty_L, pr.psf_L)
    else:
        prob = objectives.Step2(pr.dirty_H, pr.psf_H, np.zeros((n, n)), pr.ell, pr.delta, 0.8, 0.3)
    dense = 2 * np.linalg.eigvalsh(_dense(prob.normal, n)).max()
    th, it, trace = lipschitz.lanczos(prob.normal, n, seed=5, max_iter=300, rtol=1e-13)
    assert th == pytest.approx(dense, rel=1e-9)
    assert all(t <= dense * (1 + 1e-12) for t in trace)
    assert all(b >= a * (1 - 1e-12) for a, b in zip(trace, trace[1:]))
    if pad == 1:
        cf = (lipschitz.closed_form_step1(prob.H.h) if step == 1
              else lipschitz.closed_form_step2(prob.H.h, prob.gL2, prob.gH2))
        assert th == pytest.approx(cf, rel=1e-9)


def test_lanczos_identity_and_fewer_steps():
    n, P = 8, 16
    psf = np.zeros((P, P))
    psf[P // 2, P // 2] = 1.0
    s1 = objectives.Step1(np.zeros((n, n)), psf)
    th, it, _ = lipschitz.lanczos(s1.normal, n, seed=0)
    assert th == pytest.approx(2.0, rel=1e-12)
    assert it <= 2  # the Krylov space of the identity is one-dimensional
    pr = synth.make_problem(tiny(32, seed=5))
    s1 = objectives.Step1(pr.dirty_L, pr.psf_L)
    thp, itp, _ = lipschitz.power_iteration(s1.normal, 32, rtol=1e-8, max_iter=2000)
    thl, itl, _ = lipschitz.lanczos(s1.normal, 32, rtol=1e-8, max_iter=2000)
    assert itl < itp
    assert thl >= thp * (1 - 1e-8)
