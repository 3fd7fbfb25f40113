"""The wavelet dictionary on the GPU (msr_config.dictionary = 1): W alpha and
W^T x against the FP64 oracle, W W^T = 8 I at the full image size, the
Lipschitz constant of the problem in alpha (the closed form 2 M max|h_hat|^2
of Sect. 3.4 with M = 8 in circular mode), and FISTA trajectories on the
coefficients against the oracle's FISTA on InDictionary (Eqs. 4-5 with
x = W alpha, Algorithm 1).

Tolerances as in the other parity tests: max-abs error over the oracle's
peak, 1e-5 for FP32 results (2e-6 for single transforms, which sum 8 bases
of at most 4 levels x 16 taps), 1e-9 along FP64 trajectories, 1e-12 for FP64
transforms.
"""
import numpy as np
import pytest

import synth
from synth.generator import tiny

pytestmark = pytest.mark.gpu

OP_TOL = 2e-6
OP_TOL64 = 1e-12
TOL = 1e-5
TOL64 = 1e-9
SHORT_K = 10


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    print("gpu wavelets: device", torch.cuda.get_device_name(0), flush=True)
    return torch, torch.device("cuda:0")


def _t(torch_dev, a, prec=32):
    torch, dev = torch_dev
    return torch.from_numpy(np.ascontiguousarray(a, np.float32 if prec == 32 else np.float64)).to(dev)


def _solver(torch_dev, pr, prec=32, seed=0):
    from paper_2406_18356_amd import Solver

    s = Solver(pr.n, pad=pr.cfg.pad, positivity=False, precision=prec, dictionary=1, seed=seed)
    s.set_dirty_psf(1, _t(torch_dev, pr.dirty_L, prec), _t(torch_dev, pr.psf_L, prec))
    s.set_dirty_psf(2, _t(torch_dev, pr.dirty_H, prec), _t(torch_dev, pr.psf_H, prec))
    return s


def _problem(n, pad=2, seed=5):
    return synth.make_problem(tiny(n, seed=seed).replace(pad=pad))


@pytest.mark.parametrize("n", [16, 64, 128])
@pytest.mark.parametrize("prec", [32, 64])
def test_synthesis_analysis_match_oracle(torch_dev, n, prec):
    from oracle import wavelets

    print(f"wavelet transforms n={n} prec={prec}", flush=True)
    s = _solver(torch_dev, _problem(n), prec)
    rng = np.random.default_rng(n + prec)
    alpha = rng.normal(size=(8, n, n))
    # a sparse coefficient set too: single atoms of every basis and band
    sparse = np.zeros((8, n, n))
    idx = rng.integers(0, n, (40, 3))
    sparse[idx[:, 0] % 8, idx[:, 1], idx[:, 2]] = rng.normal(size=40)
    x = rng.normal(size=(n, n))
    tol = OP_TOL if prec == 32 else OP_TOL64
    for a in (alpha, sparse):
        a_in = a.astype(np.float32).astype(np.float64) if prec == 32 else a
        y = s.synthesis(_t(torch_dev, a_in, prec)).cpu().numpy()
        e = rel(y, wavelets.synthesis(a_in))
        print(f"  synthesis error {e:.3g}", flush=True)
        assert e <= tol
    x_in = x.astype(np.float32).astype(np.float64) if prec == 32 else x
    c = s.analysis(_t(torch_dev, x_in, prec)).cpu().numpy()
    e = rel(c, wavelets.analysis(x_in))
    print(f"  analysis error {e:.3g}", flush=True)
    assert e <= tol


@pytest.mark.parametrize("n", [2048])
def test_frame_identity_full_size(torch_dev, n):
    """W W^T x = 8 x for the concatenation of 8 orthonormal bases, at the
    full image size (a property that holds at any size)."""
    from paper_2406_18356_amd import Solver

    torch, dev = torch_dev
    s = Solver(n, pad=1, precision=32, dictionary=1)  # the transforms need no PSF
    g = torch.Generator(device="cpu").manual_seed(3)
    x = torch.randn((n, n), generator=g, dtype=torch.float32).to(dev)
    y = s.synthesis(s.analysis(x))
    err = float((y - 8 * x).abs().max() / (8 * x.abs().max()))
    print(f"frame identity n={n}: {err:.3g}", flush=True)
    assert err <= OP_TOL


def test_library_taps_match_oracle(torch_dev):
    """W^T of a unit impulse at (3, 5): entry (i, j) of the first-level
    high-high band of basis b is g_b[3 - 2i] g_b[5 - 2j], so the library's
    filters agree with the oracle's db_p tap by tap."""
    from oracle import wavelets

    n = 64
    s = _solver(torch_dev, _problem(n), 64)
    x = np.zeros((n, n))
    x[3, 5] = 1.0
    c = s.analysis(_t(torch_dev, x, 64)).cpu().numpy()
    for b in range(8):
        h = wavelets.daubechies(b + 1)
        g = wavelets.highpass(h)
        # level-1 HH band sits at [n/2:, n/2:]; its entry (i, j) is g[3 - 2i] g[5 - 2j] for in-range taps
        hh = c[b, n // 2:, n // 2:]
        for i in range(2):
            for j in range(3):
                ki, kj = 3 - 2 * i, 5 - 2 * j
                want = (g[ki] if ki < g.size else 0.0) * (g[kj] if kj < g.size else 0.0)
                assert hh[i, j] == pytest.approx(want, abs=1e-13)


@pytest.mark.parametrize("pad", [1, 2])
def test_lipschitz_in_coefficients(torch_dev, pad):
    from oracle import lipschitz, objectives

    n = 32
    pr = _problem(n, pad)
    s = _solver(torch_dev, pr, 64, seed=9)
    prob = objectives.Step1(pr.dirty_L, pr.psf_L)
    th, _ = s.lipschitz(1, max_iter=500, rtol=1e-9)
    tho, _, _ = lipschitz.lanczos(prob.normal, n, seed=9, max_iter=500, rtol=1e-9)
    assert th == pytest.approx(8 * tho, rel=1e-6)
    if pad == 1:  # Sect. 3.4: 2 M max |h_hat|^2 with M = 8 bases
        assert th == pytest.approx(8 * lipschitz.closed_form_step1(prob.H.h), rel=1e-4)


def _dict_case(torch_dev, n, pad, step, K, prec, seed=5, x0=None):
    from oracle import fista, lipschitz, objectives, wavelets

    pr = _problem(n, pad, seed)
    s = _solver(torch_dev, pr, prec)
    if step == 1:
        prob = objectives.Step1(pr.dirty_L, pr.psf_L)
        lam = 0.02 * np.linalg.norm(pr.dirty_L)
    else:
        l = np.asarray(pr.dirty_L, np.float32).astype(np.float64) * 0.5
        sig2 = float(np.var(pr.dirty_H))
        s.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
        prob = objectives.Step2(pr.dirty_H, pr.psf_H, l, pr.ell, pr.delta, sig2, 1e-3 * sig2)
        lam = 0.02 * np.linalg.norm(pr.dirty_H) / sig2  # the data term carries 1 / sigma^2
    theta = 8 * 1.01 * lipschitz.power_iteration(prob.normal, n)[0]
    s.set_lipschitz(step, theta)
    x0_t = None if x0 is None else _t(torch_dev, x0, prec)
    if step == 1:
        b, r = s.step1(lam, K, x0=x0_t)
    else:
        b, r = s.step2(lam, _t(torch_dev, l, prec), K, x0=x0_t)
    dic = wavelets.InDictionary(prob)
    a0 = np.zeros((8, n, n)) if x0 is None else wavelets.analysis(x0) / 8
    ao, _ = fista.fista(dic.grad, a0, 1.0 / theta, lam, K)
    return b.cpu().numpy(), wavelets.synthesis(ao), ao, r, dic, lam


@pytest.mark.parametrize("n,pad", [(16, 2), (32, 2), (32, 1)])
@pytest.mark.parametrize("step", [1, 2])
def test_dictionary_fista_f64(torch_dev, n, pad, step):
    print(f"dictionary fista f64 n={n} pad={pad} step={step}", flush=True)
    b, xo, ao, r, dic, lam = _dict_case(torch_dev, n, pad, step, 40, 64)
    assert rel(b, xo) <= TOL64
    F, data, l1 = dic.objective(ao, lam)
    assert r.objective == pytest.approx(F, rel=1e-10)
    assert r.l1_norm == pytest.approx(l1, rel=1e-10)
    assert r.iters == 40
    assert np.count_nonzero(ao) < ao.size  # the threshold is active


@pytest.mark.parametrize("step", [1, 2])
def test_dictionary_fista_short_f32(torch_dev, step):
    print(f"dictionary fista f32 step={step}", flush=True)
    b, xo, ao, r, dic, lam = _dict_case(torch_dev, 64, 2, step, SHORT_K, 32)
    assert rel(b, xo) <= TOL
    assert r.objective == pytest.approx(dic.objective(ao, lam)[0], rel=1e-5)


def test_dictionary_warm_start(torch_dev):
    """x0 is an image: alpha_0 = W^T x0 / 8 reproduces it (zero iterations),
    and a warm-started run follows the oracle's trajectory from that alpha_0."""
    n = 32
    x0 = np.random.default_rng(2).normal(size=(n, n))
    b, xo, *_ = _dict_case(torch_dev, n, 2, 1, 0, 64, x0=x0)
    assert rel(b, x0) <= OP_TOL64
    b, xo, *_ = _dict_case(torch_dev, n, 2, 1, 15, 64, x0=x0)
    assert rel(b, xo) <= TOL64


@pytest.mark.parametrize("step", [1, 2])
def test_dictionary_major_cycles_f64(torch_dev, step):
    """Major cycles (Sect. 3.2, 3.3) with every cycle solved in the
    dictionary: the library's image, model and per-cycle objectives against
    the oracle's, with the same theta."""
    from oracle import lipschitz, objectives, twostep

    n, cycles, K = 32, 2, 20
    pr = _problem(n, 2, seed=7)
    s = _solver(torch_dev, pr, 64)
    if step == 1:
        prob = objectives.Step1(pr.dirty_L, pr.psf_L)
        low = kw = None
        dirty, psf = pr.dirty_L, pr.psf_L
    else:
        low = np.asarray(pr.dirty_L) * 0.5
        sig2 = float(np.var(pr.dirty_H))
        s.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
        prob = objectives.Step2(pr.dirty_H, pr.psf_H, low, pr.ell, pr.delta, sig2, 1e-3 * sig2)
        kw = dict(ell=pr.ell, delta=pr.delta, sigma2=sig2, eta2=1e-3 * sig2)
        dirty, psf = pr.dirty_H, pr.psf_H
    theta = 8 * 1.01 * lipschitz.lanczos(prob.normal, n)[0]
    s.set_lipschitz(step, theta)
    img, model, res = s.major_cycles(step, cycles, K, c=0.05, low_res=None if low is None else _t(torch_dev, low, 64))
    ref_img, ref_model, recs = twostep.major_cycles(step, dirty, psf, cycles, K, c=0.05, theta=theta,
                                                    low_res=low, dictionary=True, **(kw or {}))
    assert rel(model.cpu().numpy(), ref_model) <= TOL64
    assert rel(img.cpu().numpy(), ref_img) <= TOL64
    for r, rec in zip(res, recs):
        assert r.objective == pytest.approx(rec["F"], rel=1e-9)


def test_dictionary_errors(torch_dev):
    from paper_2406_18356_amd import Solver
    from paper_2406_18356_amd.binding import MsrError

    with pytest.raises(MsrError):
        Solver(32, positivity=True, dictionary=1)  # no closed-form prox
    with pytest.raises(MsrError):
        Solver(8, dictionary=1)  # 4 levels need n >= 16
    plain = Solver(32)
    with pytest.raises(MsrError):
        plain.synthesis(_t(torch_dev, np.zeros((8, 32, 32))))
