"""GPU (HIP, gfx950) path against the FP64 oracle.

Tolerances.  Images: max|x_gpu - x_oracle| / max|x_oracle| <= 1e-5 for the
FP32 path (single operator applications and one FISTA step at 2e-6), and
<= 1e-9 for the FP64 path along whole FISTA trajectories.  Scalars: relative
tolerances stated per test.  Both sides run from the same seeded inputs;
FISTA runs use the same x0, lambda, K and Lipschitz constant (passed to the
library explicitly), so the comparison is of one deterministic trajectory.

Why the FP32 path is held to short trajectories: FISTA's momentum amplifies
perturbations in the poorly conditioned directions of H (unsampled uv cells)
roughly linearly in k, so the ~3e-7 rounding of each FP32 operator
application grows to ~1e-5 after a few tens of iterations and beyond it after
~100 (the growth is measured and tabulated in the design notes).  The FP64
path carries the long-trajectory parity; the FP32 path is checked on every
operator, on the one-step map at the full 2048^2 size, and on 10-step runs.
"""
import numpy as np
import pytest

import synth
from synth.generator import tiny

pytestmark = pytest.mark.gpu

TOL = 1e-5          # images: max-abs error over the oracle's peak
OP_TOL = 2e-6       # single operator applications (H x, gradients), FP32
SCALAR_TOL = 2e-6   # objectives and reductions (relative), FP32
TOL64 = 1e-9        # FP64 path, whole trajectories
OP_TOL64 = 1e-12    # FP64 path, single operators
SHORT_K = 10        # FP32 trajectory length held to TOL


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    print("gpu parity: device", torch.cuda.get_device_name(0), flush=True)
    return torch, torch.device("cuda:0")


def _t(torch_dev, a, prec=32):
    torch, dev = torch_dev
    return torch.from_numpy(np.ascontiguousarray(a, np.float32 if prec == 32 else np.float64)).to(dev)


def _problem(n, pad=2, seed=5):
    if n == 256 and pad == 2:
        return synth.make_problem(synth.preset("small256"))
    return synth.make_problem(tiny(n, seed=seed).replace(pad=pad))


def _solver(torch_dev, pr, positivity=False, prune_tol=1e-6, seed=0, prec=32):
    from paper_2406_18356_amd import Solver

    s = Solver(pr.n, pad=pr.cfg.pad, positivity=positivity, prune_tol=prune_tol, seed=seed, precision=prec)
    s.set_dirty_psf(1, _t(torch_dev, pr.dirty_L, prec), _t(torch_dev, pr.psf_L, prec))
    s.set_dirty_psf(2, _t(torch_dev, pr.dirty_H, prec), _t(torch_dev, pr.psf_H, prec))
    return s


# ----------------------------------------------------------------- operators
@pytest.mark.parametrize("n,pad", [(8, 2), (16, 2), (64, 2), (256, 2), (32, 1), (128, 1)])
def test_psf_spectrum(torch_dev, n, pad):
    from oracle import conv

    print(f"spectrum n={n} pad={pad}", flush=True)
    pr = _problem(n, pad)
    s = _solver(torch_dev, pr)
    for step, psf in ((1, pr.psf_L), (2, pr.psf_H)):
        h, kept = s.spectrum(step)
        ho = conv.psf_spectrum(psf)
        assert np.max(np.abs(ho.imag)) < 1e-9 * np.max(np.abs(ho.real))
        ho = ho.real[:, : pr.P // 2 + 1]
        peak = np.max(np.abs(ho))
        assert rel(h[:, :kept], ho[:, :kept]) <= OP_TOL
        # pruned columns only hold values below the pruning threshold (+ FP32 noise)
        if kept < ho.shape[1]:
            assert np.max(np.abs(ho[:, kept:])) <= 1e-6 * peak + 1e-7 * peak


@pytest.mark.parametrize("n,pad", [(8, 2), (32, 2), (256, 2), (16, 1), (64, 1)])
def test_apply_psf(torch_dev, n, pad):
    from oracle import conv

    pr = _problem(n, pad)
    s = _solver(torch_dev, pr)
    x = np.random.default_rng(n).normal(size=(n, n))
    for step, psf in ((1, pr.psf_L), (2, pr.psf_H)):
        y = s.apply_psf(step, _t(torch_dev, x)).cpu().numpy()
        assert rel(y, conv.conv_fft(x, psf)) <= OP_TOL


@pytest.mark.parametrize("n,pad", [(16, 2), (64, 2), (256, 2), (32, 1)])
def test_gradients(torch_dev, n, pad):
    from oracle import objectives

    pr = _problem(n, pad)
    s = _solver(torch_dev, pr)
    rng = np.random.default_rng(3)
    x = rng.normal(size=(n, n))
    l = rng.normal(size=(n, n))
    s.set_filters(pr.ell, pr.delta, 0.8, 0.3)
    s1 = objectives.Step1(pr.dirty_L, pr.psf_L)
    s2 = objectives.Step2(pr.dirty_H, pr.psf_H, l, pr.ell, pr.delta, 0.8, 0.3)
    g1 = s.gradient(1, _t(torch_dev, x)).cpu().numpy()
    g2 = s.gradient(2, _t(torch_dev, x), _t(torch_dev, l)).cpu().numpy()
    assert rel(g1, s1.grad(x)) <= OP_TOL
    assert rel(g2, s2.grad(x)) <= OP_TOL


@pytest.mark.parametrize("n,pad", [(32, 2), (256, 2), (64, 1)])
def test_objectives(torch_dev, n, pad):
    from oracle import objectives

    pr = _problem(n, pad)
    s = _solver(torch_dev, pr)
    rng = np.random.default_rng(4)
    x = rng.normal(size=(n, n)) * 0.01
    l = rng.normal(size=(n, n))
    lam = 0.37
    s.set_filters(pr.ell, pr.delta, 1.7, 2e-3)
    F1 = s.objective(1, lam, _t(torch_dev, x))
    F2 = s.objective(2, lam, _t(torch_dev, x), _t(torch_dev, l))
    o1 = objectives.Step1(pr.dirty_L, pr.psf_L).objective(x.astype(np.float32).astype(np.float64), lam)
    o2 = objectives.Step2(pr.dirty_H, pr.psf_H, l.astype(np.float32), pr.ell, pr.delta, 1.7, 2e-3).objective(
        x.astype(np.float32).astype(np.float64), lam)
    for a, b in zip(F1, o1):
        assert a == pytest.approx(b, rel=SCALAR_TOL)
    for a, b in zip(F2, o2):
        assert a == pytest.approx(b, rel=SCALAR_TOL)


@pytest.mark.parametrize("n,pad", [(16, 2), (64, 2), (32, 1)])
def test_lipschitz(torch_dev, n, pad):
    from oracle import objectives, lipschitz

    pr = _problem(n, pad)
    s = _solver(torch_dev, pr, seed=9)
    s.set_filters(pr.ell, pr.delta, 0.8, 0.3)
    s1 = objectives.Step1(pr.dirty_L, pr.psf_L)
    s2 = objectives.Step2(pr.dirty_H, pr.psf_H, np.zeros((n, n)), pr.ell, pr.delta, 0.8, 0.3)
    for step, prob in ((1, s1), (2, s2)):
        th, it = s.lipschitz(step, max_iter=500, rtol=1e-9)
        tho, ito, _ = lipschitz.lanczos(prob.normal, n, seed=9, max_iter=500, rtol=1e-9)
        print(f"lipschitz n={n} pad={pad} step={step}: {th:.12g} ({it} its) oracle {tho:.12g} ({ito})", flush=True)
        assert th == pytest.approx(tho, rel=1e-5)
        if pad == 1:  # circular: the paper's closed form (M = 1) is the exact value
            cf = (lipschitz.closed_form_step1(prob.H.h) if step == 1
                  else lipschitz.closed_form_step2(prob.H.h, prob.gL2, prob.gH2))
            assert th == pytest.approx(cf, rel=1e-4)


@pytest.mark.parametrize("n,pad", [(16, 2), (256, 2), (32, 1)])
def test_operators_f64(torch_dev, n, pad):
    """The FP64 path: H x, both gradients and both objectives to ~1e-12."""
    from oracle import conv, objectives

    pr = _problem(n, pad)
    s = _solver(torch_dev, pr, prec=64)
    rng = np.random.default_rng(11)
    x = rng.normal(size=(n, n))
    l = rng.normal(size=(n, n))
    s.set_filters(pr.ell, pr.delta, 0.8, 0.3)
    y = s.apply_psf(1, _t(torch_dev, x, 64)).cpu().numpy()
    assert rel(y, conv.conv_fft(x, pr.psf_L)) <= OP_TOL64
    s1 = objectives.Step1(pr.dirty_L, pr.psf_L)
    s2 = objectives.Step2(pr.dirty_H, pr.psf_H, l, pr.ell, pr.delta, 0.8, 0.3)
    assert rel(s.gradient(1, _t(torch_dev, x, 64)).cpu().numpy(), s1.grad(x)) <= OP_TOL64
    assert rel(s.gradient(2, _t(torch_dev, x, 64), _t(torch_dev, l, 64)).cpu().numpy(), s2.grad(x)) <= OP_TOL64
    F1 = s.objective(1, 0.3, _t(torch_dev, x, 64))
    F2 = s.objective(2, 0.3, _t(torch_dev, x, 64), _t(torch_dev, l, 64))
    assert F1[0] == pytest.approx(s1.objective(x, 0.3)[0], rel=1e-12)
    assert F2[0] == pytest.approx(s2.objective(x, 0.3)[0], rel=1e-12)


# ----------------------------------------------------------------- FISTA
def _fista_case(torch_dev, n, pad, positivity, step, K, prec=32, seed=5):
    from oracle import objectives, fista, lipschitz

    pr = _problem(n, pad, seed)
    s = _solver(torch_dev, pr, positivity=positivity, prec=prec)
    if step == 1:
        prob = objectives.Step1(pr.dirty_L, pr.psf_L)
        lam = 0.05 * np.linalg.norm(pr.dirty_L)
    else:
        l = np.asarray(pr.dirty_L, np.float32).astype(np.float64) * 0.5
        sig2 = float(np.var(pr.dirty_H))
        s.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
        prob = objectives.Step2(pr.dirty_H, pr.psf_H, l, pr.ell, pr.delta, sig2, 1e-3 * sig2)
        lam = 0.05 * np.linalg.norm(pr.dirty_H)
    theta = 1.01 * lipschitz.power_iteration(prob.normal, n)[0]
    s.set_lipschitz(step, theta)
    if step == 1:
        b, r = s.step1(lam, K)
    else:
        b, r = s.step2(lam, _t(torch_dev, l, prec), K)
    bo, _ = fista.fista(prob.grad, np.zeros((n, n)), 1.0 / theta, lam, K, positivity=positivity)
    return b.cpu().numpy(), bo, r, prob, lam


CASES = [(16, 2, False), (64, 2, True), (128, 2, False), (32, 1, True), (64, 1, False)]


@pytest.mark.parametrize("n,pad,positivity", CASES)
@pytest.mark.parametrize("step", [1, 2])
def test_fista_trajectory_f64(torch_dev, n, pad, positivity, step):
    print(f"fista f64 n={n} pad={pad} pos={positivity} step={step}", flush=True)
    b, bo, r, prob, lam = _fista_case(torch_dev, n, pad, positivity, step, 100, prec=64)
    assert rel(b, bo) <= TOL64
    assert r.objective == pytest.approx(prob.objective(bo, lam)[0], rel=1e-10)
    assert r.iters == 100
    if positivity:
        assert np.all(b >= 0)


@pytest.mark.parametrize("n,pad,positivity", CASES)
@pytest.mark.parametrize("step", [1, 2])
def test_fista_short_f32(torch_dev, n, pad, positivity, step):
    print(f"fista f32 n={n} pad={pad} pos={positivity} step={step}", flush=True)
    b, bo, r, prob, lam = _fista_case(torch_dev, n, pad, positivity, step, SHORT_K)
    assert rel(b, bo) <= TOL
    assert r.objective == pytest.approx(prob.objective(bo, lam)[0], rel=1e-5)
    if positivity:
        assert np.all(b >= 0)


def _two_step(torch_dev, prec):
    from oracle import objectives, fista, lipschitz, helpers

    pr = _problem(256)
    s = _solver(torch_dev, pr, positivity=True, prec=prec)
    K = pr.cfg.iters
    s1 = objectives.Step1(pr.dirty_L, pr.psf_L)
    th1 = 1.01 * lipschitz.power_iteration(s1.normal, 256)[0]
    lam1 = helpers.default_lambda(pr.dirty_L, 0.05)
    assert s.default_lambda(1, 1, 0.05) == pytest.approx(lam1, rel=1e-6)
    s.set_lipschitz(1, th1)
    out = {}
    b1, iL, r1 = s.step1(lam1, K, image=True)
    b1o, _ = fista.fista(s1.grad, np.zeros((256, 256)), 1 / th1, lam1, K, positivity=True)
    iLo = helpers.low_res_image(b1o, pr.dirty_L, s1.H)
    out["beta1"] = rel(b1.cpu().numpy(), b1o)
    out["i_L"] = rel(iL.cpu().numpy(), iLo)
    sig2 = helpers.sigma2_hat(pr.dirty_H)
    assert s.estimate_sigma2(_t(torch_dev, pr.dirty_H, prec)) == pytest.approx(sig2, rel=1e-6)
    eta2 = helpers.eta2_hat(sig2)
    l_in = iLo.astype(np.float32).astype(np.float64) if prec == 32 else iLo
    s2 = objectives.Step2(pr.dirty_H, pr.psf_H, l_in, pr.ell, pr.delta, sig2, eta2)
    th2 = 1.01 * lipschitz.power_iteration(s2.normal, 256)[0]
    lam2 = helpers.default_lambda(pr.dirty_H, 0.05)
    s.set_filters(pr.ell, pr.delta, sig2, eta2)
    s.set_lipschitz(2, th2)
    b2, r2 = s.step2(lam2, _t(torch_dev, l_in, prec), K)
    b2o, _ = fista.fista(s2.grad, np.zeros((256, 256)), 1 / th2, lam2, K, positivity=True)
    out["beta2"] = rel(b2.cpu().numpy(), b2o)
    out["F1"] = (r1.objective, s1.objective(b1o, lam1)[0])
    out["F2"] = (r2.objective, s2.objective(b2o, lam2)[0])
    print(f"two-step 256 precision {prec}:", out, flush=True)
    return out


def test_two_step_small_workload_f64(torch_dev):
    """The 256^2 workload end to end in FP64: 200 iterations per step, positivity on."""
    out = _two_step(torch_dev, 64)
    for k in ("beta1", "i_L", "beta2"):
        assert out[k] <= TOL64, k
    for k in ("F1", "F2"):
        assert out[k][0] == pytest.approx(out[k][1], rel=1e-12)


def test_two_step_small_workload_f32_objective(torch_dev):
    """The same workload on the FP32 path: the objectives reached after 200
    iterations agree with the oracle's."""
    out = _two_step(torch_dev, 32)
    for k in ("F1", "F2"):
        assert out[k][0] == pytest.approx(out[k][1], rel=1e-4)


def test_f32_trajectory_drift_small_workload(torch_dev):
    """Along K = 50, 100 and 200 iterations of each step of the 256^2 workload
    the FP32 GPU iterate stays within twice the distance between the oracle run
    in float32 and in float64 (the drift of FP32 FISTA itself, pinned on the
    CPU by test_float32_drift_of_fista_small256), and within 2e-4 of peak."""
    from oracle import objectives, fista, lipschitz, helpers

    pr = _problem(256)
    s = _solver(torch_dev, pr, positivity=True)
    n, Ks = 256, (50, 100, 200)

    def traj(prob, th, lam, dt):
        out = {}
        fista.fista(prob.grad, np.zeros((n, n)), 1 / th, lam, max(Ks), positivity=True, dtype=dt,
                    callback=lambda k, b: out.__setitem__(k, b.astype(np.float64)) if k in Ks else None)
        return out

    s1 = objectives.Step1(pr.dirty_L, pr.psf_L)
    th1 = 1.01 * lipschitz.power_iteration(s1.normal, n)[0]
    lam1 = helpers.default_lambda(pr.dirty_L)
    a1 = traj(s1, th1, lam1, np.float64)
    f1 = traj(objectives.Step1(pr.dirty_L, pr.psf_L, dtype=np.float32), th1, lam1, np.float32)
    iL = helpers.low_res_image(a1[200], pr.dirty_L, s1.H).astype(np.float32).astype(np.float64)
    sig2 = helpers.sigma2_hat(pr.dirty_H)
    s2 = objectives.Step2(pr.dirty_H, pr.psf_H, iL, pr.ell, pr.delta, sig2, 1e-3 * sig2)
    th2 = 1.01 * lipschitz.power_iteration(s2.normal, n)[0]
    lam2 = helpers.default_lambda(pr.dirty_H)
    a2 = traj(s2, th2, lam2, np.float64)
    f2 = traj(objectives.Step2(pr.dirty_H, pr.psf_H, iL, pr.ell, pr.delta, sig2, 1e-3 * sig2, dtype=np.float32),
              th2, lam2, np.float32)
    s.set_lipschitz(1, th1)
    s.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
    s.set_lipschitz(2, th2)
    lt = _t(torch_dev, iL)
    for K in Ks:
        g1 = rel(s.step1(lam1, K)[0].cpu().numpy(), a1[K])
        g2 = rel(s.step2(lam2, lt, K)[0].cpu().numpy(), a2[K])
        o1, o2 = rel(f1[K], a1[K]), rel(f2[K], a2[K])
        print(f"K={K}: step 1 gpu {g1:.3g} oracle-f32 {o1:.3g}; step 2 gpu {g2:.3g} oracle-f32 {o2:.3g}", flush=True)
        assert g1 <= 2 * o1 and g1 <= 2e-4
        assert g2 <= 2 * o2 and g2 <= 2e-4


@pytest.mark.parametrize("prec,tol", [(64, TOL64), (32, TOL)])
def test_step2_image(torch_dev, prec, tol):
    """msr_step2_full_res's image_out: the model plus the long-baseline residual
    image, i^ = beta_K + (i_H~ - H_H beta_K) (Sect. 3.3), against the oracle."""
    from oracle import objectives, fista, lipschitz, helpers

    n, K = 64, SHORT_K if prec == 32 else 60
    pr = _problem(n, 2, seed=6)
    s = _solver(torch_dev, pr, positivity=True, prec=prec)
    low = np.asarray(pr.dirty_L, np.float32).astype(np.float64) * 0.5
    sig2 = float(np.var(pr.dirty_H))
    s.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
    prob = objectives.Step2(pr.dirty_H, pr.psf_H, low, pr.ell, pr.delta, sig2, 1e-3 * sig2)
    th = 1.01 * lipschitz.power_iteration(prob.normal, n)[0]
    s.set_lipschitz(2, th)
    lam = helpers.default_lambda(pr.dirty_H)
    b, img, r = s.step2(lam, _t(torch_dev, low, prec), K, image=True)
    bo, _ = fista.fista(prob.grad, np.zeros((n, n)), 1 / th, lam, K, positivity=True)
    want = helpers.low_res_image(bo, pr.dirty_H, prob.H)
    assert rel(b.cpu().numpy(), bo) <= tol
    assert rel(img.cpu().numpy(), want) <= tol
    # the image is not the model: the residual part is there
    assert rel(want, bo) > 1e-3


def test_warm_start_and_degenerate_cases(torch_dev):
    from oracle import objectives, fista, lipschitz

    pr = _problem(32)
    s = _solver(torch_dev, pr)
    s1 = objectives.Step1(pr.dirty_L, pr.psf_L)
    th = 1.01 * lipschitz.power_iteration(s1.normal, 32)[0]
    s.set_lipschitz(1, th)
    lam = 0.05 * np.linalg.norm(pr.dirty_L)
    x0 = np.random.default_rng(1).normal(size=(32, 32)).astype(np.float32)
    b, _ = s.step1(lam, 30, x0=_t(torch_dev, x0))
    bo, _ = fista.fista(s1.grad, x0.astype(np.float64), 1 / th, lam, 30)
    assert rel(b.cpu().numpy(), bo) <= TOL
    # K = 0 returns x0 unchanged
    b0, r0 = s.step1(lam, 0, x0=_t(torch_dev, x0))
    np.testing.assert_array_equal(b0.cpu().numpy(), x0)
    assert r0.iters == 0
    # lambda above ||2 H^T y||_inf: the minimiser and every iterate from 0 is exactly 0
    big = 1.01 * np.max(np.abs(s1.grad(np.zeros((32, 32)))))
    bz, rz = s.step1(big, 20)
    assert np.all(bz.cpu().numpy() == 0)
    assert rz.l1_norm == 0.0
    # zero data: zero solution
    s.set_dirty_psf(1, _t(torch_dev, np.zeros((32, 32))), _t(torch_dev, pr.psf_L))
    s.set_lipschitz(1, th)
    bz2, _ = s.step1(1e-3, 10)
    assert np.all(bz2.cpu().numpy() == 0)


def test_determinism(torch_dev):
    pr = _problem(64)
    s = _solver(torch_dev, pr, positivity=True)
    lam = 0.05 * np.linalg.norm(pr.dirty_L)
    s.set_lipschitz(1, 1e6)
    a, ra = s.step1(lam, 40)
    b, rb = s.step1(lam, 40)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    assert ra.objective == rb.objective
    th1, _ = s.lipschitz(1)
    th2, _ = s.lipschitz(1)
    assert th1 == th2


def test_stopping_rule(torch_dev):
    """With f_ref = F* from a long run, the tol rule stops early and reports time to tolerance."""
    pr = _problem(64)
    s = _solver(torch_dev, pr, positivity=True)
    lam = 0.05 * np.linalg.norm(pr.dirty_L)
    _, rlong = s.step1(lam, 3000)
    fstar = rlong.objective
    _, r = s.step1(lam, 3000, check_every=5, tol=1e-3, f_ref=fstar)
    assert r.converged == 1
    assert r.iters < 3000 and r.iters % 5 == 0
    assert r.time_to_tol_ms > 0
    assert (r.objective - fstar) / abs(fstar) <= 1e-3


def test_errors(torch_dev):
    from paper_2406_18356_amd import MsrError, Solver, binding

    pr = _problem(16)
    s = Solver(16)
    bad = pr.psf_L.copy()
    bad[16, 16] = 0.5
    with pytest.raises(MsrError) as e:
        s.set_dirty_psf(1, _t(torch_dev, pr.dirty_L), _t(torch_dev, bad))
    assert e.value.status == binding.ERR_INVALID
    asym = pr.psf_L.copy()
    asym[16, 17] += 0.3
    with pytest.raises(MsrError) as e:
        s.set_dirty_psf(1, _t(torch_dev, pr.dirty_L), _t(torch_dev, asym))
    assert e.value.status == binding.ERR_INVALID
    with pytest.raises(MsrError) as e:
        s.step1(0.1, 10)
    assert e.value.status == binding.ERR_STATE
    s.set_dirty_psf(2, _t(torch_dev, pr.dirty_H), _t(torch_dev, pr.psf_H))
    with pytest.raises(MsrError) as e:
        s.step2(0.1, _t(torch_dev, pr.dirty_L), 10)
    assert e.value.status == binding.ERR_STATE
    with pytest.raises(MsrError):
        s.set_filters(10.0, 0.0, 1.0, 1.0)
    nan = pr.dirty_L.copy()
    nan[3, 3] = np.nan
    s.set_dirty_psf(1, _t(torch_dev, nan), _t(torch_dev, pr.psf_L))
    s.set_lipschitz(1, 1e4)
    with pytest.raises(MsrError) as e:
        s.step1(0.1, 10, check_every=5)
    assert e.value.status == binding.ERR_NUMERIC
    assert "iteration 5" in str(e.value)  # the first objective check names where
    # a workspace smaller than msr_workspace_bytes is refused
    import ctypes

    lib = binding.lib()
    h = ctypes.c_void_p()
    cfg = binding._cfg(16)
    assert lib.msr_init(ctypes.byref(cfg), ctypes.byref(h)) == binding.OK
    small = _t(torch_dev, np.zeros(64, np.float32))
    assert lib.msr_set_workspace(h, ctypes.c_void_p(small.data_ptr()), 256) == binding.ERR_OOM
    assert b"workspace needs" in lib.msr_last_error(h)
    lib.msr_destroy(h)


# ----------------------------------------------------------------- full size
# The benchmark workloads (2048^2 image on a 4096^2 grid; 4096^2 on 8192^2), in
# the launch configuration the benchmark times (autotuned variants).
@pytest.fixture(scope="module", params=["sky2048", "sky4096"])
def big(torch_dev, request):
    print(f"full-size workload {request.param}", flush=True)
    pr = synth.make_problem(synth.preset(request.param), with_full=False)
    s = _solver(torch_dev, pr, positivity=True)
    return pr, s


def test_full_size_psf_sampled(torch_dev, big):
    """H x at sampled pixels against the defining spatial sum (both PSFs)."""
    pr, s = big
    n, P = pr.n, pr.P
    x = np.zeros((n, n))
    rng = np.random.default_rng(7)
    idx = rng.integers(0, n, (64, 2))
    x[idx[:, 0], idx[:, 1]] = rng.normal(size=64)
    x[n // 2 - 100:n // 2 + 100, n // 2 - 100:n // 2 + 100] = rng.normal(size=(200, 200))
    x[n - 7:, :9] = rng.normal(size=(7, 9))  # a corner: wrap-around would show here
    c = P // 2
    xs = x.astype(np.float32).astype(np.float64)
    qi, qj = np.nonzero(xs)
    vals = xs[qi, qj]
    xt = _t(torch_dev, x)
    for step, psf in ((1, pr.psf_L), (2, pr.psf_H)):
        y = s.apply_psf(step, xt).cpu().numpy()
        peak = np.max(np.abs(y))
        pts = np.concatenate([rng.integers(0, n, (24, 2)), [[0, 0], [n - 1, n - 1], [0, n - 1], [n - 1, 0]]])
        for p in pts:
            ref = float(np.sum(psf[c + p[0] - qi, c + p[1] - qj] * vals))
            assert abs(y[p[0], p[1]] - ref) <= OP_TOL * peak, (step, p)


def test_full_size_one_step_map(torch_dev, big):
    """One FISTA step of each step from a nonzero x0, against the FP64 FFT oracle on the full grid."""
    from oracle import objectives, fista

    pr, s = big
    n = pr.n
    s.autotune(reps=3)
    rng = np.random.default_rng(2)
    x0 = (np.abs(rng.normal(size=(n, n))) * 1e-3).astype(np.float32)
    s1 = objectives.Step1(pr.dirty_L, pr.psf_L)
    th = 2.0 * float(np.max(np.abs(s1.H.h))) ** 2
    s.set_lipschitz(1, th)
    lam = 0.05 * np.linalg.norm(pr.dirty_L)
    b, _ = s.step1(lam, 1, x0=_t(torch_dev, x0))
    bo, _ = fista.fista(s1.grad, x0.astype(np.float64), 1 / th, lam, 1, positivity=True)
    assert rel(b.cpu().numpy(), bo) <= TOL
    del s1

    low = (np.abs(rng.normal(size=(n, n))) * 1e-2).astype(np.float32)
    sig2 = 0.5
    s.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
    s2 = objectives.Step2(pr.dirty_H, pr.psf_H, low.astype(np.float64), pr.ell, pr.delta, sig2, 1e-3 * sig2)
    th2 = 2.0 * (float(np.max(s2.gH2)) * float(np.max(np.abs(s2.H.h))) ** 2 + float(np.max(s2.gL2)))
    s.set_lipschitz(2, th2)
    lam2 = 0.05 * np.linalg.norm(pr.dirty_H)
    b2, _ = s.step2(lam2, _t(torch_dev, low), 1, x0=_t(torch_dev, x0))
    bo2, _ = fista.fista(s2.grad, x0.astype(np.float64), 1 / th2, lam2, 1, positivity=True)
    assert rel(b2.cpu().numpy(), bo2) <= TOL


# Ten FISTA iterations from x0 = 0 and two iterations from a late state
# (k = 500) on the full benchmark grids: every momentum term of the update
# epilogue is non-zero, in every built kernel variant and in the autotuned
# choice.  Step sizes are the closed-form bounds (valid for any operator of
# this form, and cheap), passed to both sides; the oracle runs its FFT back
# end in FP64 on the full grid.
FULL_K = 10
LATE_K = 500
_full_ref = {}


def _full_bounds(pr, prob, step):
    hmax = float(np.max(np.abs(prob.H.h)))
    if step == 1:
        return 2.0 * hmax ** 2
    return 2.0 * (float(np.max(prob.gH2)) * hmax ** 2 + float(np.max(prob.gL2)))


def _full_problem(pr, step):
    from oracle import objectives, helpers

    if step == 1:
        return objectives.Step1(pr.dirty_L, pr.psf_L), helpers.default_lambda(pr.dirty_L), None, None
    low = np.asarray(pr.dirty_L, np.float32).astype(np.float64)
    sig2 = helpers.sigma2_hat(pr.dirty_H)
    prob = objectives.Step2(pr.dirty_H, pr.psf_H, low, pr.ell, pr.delta, sig2, 1e-3 * sig2)
    return prob, helpers.default_lambda(pr.dirty_H), low, sig2


def _full_oracle(pr, step):
    """(theta, lambda, low, sigma2, beta_10 from 0, late state, beta_502) for one workload and step."""
    from oracle import fista

    key = (pr.cfg.n, step)
    if key not in _full_ref:
        print(f"oracle: {pr.cfg.n}^2 step {step}, {FULL_K} iterations and a late state", flush=True)
        prob, lam, low, sig2 = _full_problem(pr, step)
        th = _full_bounds(pr, prob, step)
        z = np.zeros((pr.n, pr.n))
        b10, _ = fista.fista(prob.grad, z, 1.0 / th, lam, FULL_K, positivity=True)
        bk, bkm1 = synth.late_state(pr.n, seed=17 + step)
        bk, bkm1 = (np.asarray(a, np.float32).astype(np.float64) for a in (bk, bkm1))
        bl, _, _ = fista.fista_from(prob.grad, bk, bkm1, LATE_K, 1.0 / th, lam, 2, positivity=True)
        _full_ref[key] = (th, lam, low, sig2, b10, (bk, bkm1), bl)
    return _full_ref[key]


def _full_gpu(torch_dev, s, pr, step, ref, x0_state=None):
    th, lam, low, sig2, _, _, _ = ref
    s.set_lipschitz(step, th)
    if step == 1:
        if x0_state is not None:
            s.set_state(1, *x0_state)
            return s.step1(lam, 2)[0].cpu().numpy()
        return s.step1(lam, FULL_K)[0].cpu().numpy()
    lt = _t(torch_dev, low)
    if x0_state is not None:
        s.set_state(2, *x0_state)
        return s.step2(lam, lt, 2)[0].cpu().numpy()
    return s.step2(lam, lt, FULL_K)[0].cpu().numpy()


@pytest.mark.parametrize("step", [1, 2])
def test_full_size_momentum_path(torch_dev, big, step):
    """FULL_K iterations from 0 and 2 iterations from (beta_500, beta_499) of each
    step, every built variant plus the autotuned choice, against the FP64
    oracle on the full grid at max-abs/peak <= 1e-5."""
    from paper_2406_18356_amd import MsrError

    pr, s = big
    ref = _full_oracle(pr, step)
    th, lam, low, sig2, b10, (bk, bkm1), bl = ref
    if step == 2:
        s.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
    state = (_t(torch_dev, bk), _t(torch_dev, bkm1), LATE_K)
    tried = []
    for v in list(range(4)) + ["autotuned"]:
        if v == "autotuned":
            s.autotune(reps=3)
        else:
            try:
                s.set_variants(step, v, v, v if step == 2 else -1)
            except MsrError:
                continue
        label = f"{pr.cfg.n}^2 step {step} variants {s.get_variants(step)}"
        print(f"momentum path: {label}", flush=True)
        e10 = rel(_full_gpu(torch_dev, s, pr, step, ref), b10)
        el = rel(_full_gpu(torch_dev, s, pr, step, ref, x0_state=state), bl)
        print(f"  {FULL_K} its from 0: {e10:.3g}; 2 its from k = {LATE_K}: {el:.3g}", flush=True)
        assert e10 <= TOL, label
        assert el <= TOL, label
        tried.append(v)
    assert "autotuned" in tried and len(tried) >= 3


def test_full_size_8192_momentum_path(torch_dev):
    """The 8192^2 workload (16384^2 grid, 512 antennas 4 h at 10 s, cut 10 %) in
    the autotuned launch configuration: FULL_K iterations from 0 and 2 from a
    late state, both steps, on a central 512^2 crop and the four 64^2 corners,
    against what the FP64 oracle wrote (tests/golden/make_fullsize8192.py)."""
    import os
    from paper_2406_18356_amd import Solver

    path = os.path.join(os.path.dirname(__file__), "golden", "fullsize8192.npz")
    g = np.load(path)
    cfg = synth.preset("sky8192")
    print("8192^2: synthesising the workload", flush=True)
    pr = synth.make_problem(cfg, with_full=False, progress=lambda m: print("  synth:", m, flush=True))
    assert g["n"] == pr.n
    s = _solver(torch_dev, pr, positivity=True)
    s.set_filters(pr.ell, pr.delta, float(g["sigma2"]), 1e-3 * float(g["sigma2"]))
    s.autotune(reps=3)
    low = _t(torch_dev, np.asarray(pr.dirty_L, np.float32))
    n, c = pr.n, int(g["crop"])
    h = c // 2

    def crops(x):
        return [x[n // 2 - h:n // 2 + h, n // 2 - h:n // 2 + h], x[:64, :64], x[:64, -64:], x[-64:, :64],
                x[-64:, -64:]]

    for step in (1, 2):
        th, lam = float(g[f"theta{step}"]), float(g[f"lambda{step}"])
        s.set_lipschitz(step, th)
        bk, bkm1 = synth.late_state(n, seed=17 + step)
        state = (_t(torch_dev, bk), _t(torch_dev, bkm1), LATE_K)
        for name, run in (("from0", lambda: s.step1(lam, FULL_K)[0] if step == 1 else s.step2(lam, low, FULL_K)[0]),
                          ("late", lambda: (s.set_state(step, *state), s.step1(lam, 2)[0] if step == 1
                                            else s.step2(lam, low, 2)[0])[1])):
            print(f"8192^2 step {step} {name}, variants {s.get_variants(step)}", flush=True)
            x = run().cpu().numpy()
            got = crops(x)
            peak = float(g[f"peak_{name}{step}"])
            for i, a in enumerate(got):
                want = g[f"{name}{step}_{i}"]
                err = float(np.max(np.abs(a - want))) / peak
                print(f"  crop {i}: {err:.3g}", flush=True)
                assert err <= TOL, (step, name, i)


# ----------------------------------------------------------------- major cycles
@pytest.mark.parametrize("prec,cycles,iters,tol", [(64, 3, 40, TOL64), (32, 2, SHORT_K, TOL)])
@pytest.mark.parametrize("step", [1, 2])
def test_major_cycles(torch_dev, prec, cycles, iters, tol, step):
    """Major cycles with image-domain residuals (Sect. 3.2, 3.3) against the oracle."""
    from oracle import objectives, lipschitz, twostep

    print(f"major cycles prec={prec} step={step}", flush=True)
    pr = _problem(64, 2, seed=9)
    s = _solver(torch_dev, pr, positivity=True, prec=prec)
    sig2 = float(np.var(pr.dirty_H))
    low = np.asarray(pr.dirty_L, np.float32).astype(np.float64) * 0.5
    if step == 1:
        prob = objectives.Step1(pr.dirty_L, pr.psf_L)
        dirty, psf, kw = pr.dirty_L, pr.psf_L, {}
    else:
        s.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
        prob = objectives.Step2(pr.dirty_H, pr.psf_H, low, pr.ell, pr.delta, sig2, 1e-3 * sig2)
        dirty, psf = pr.dirty_H, pr.psf_H
        kw = dict(low_res=low, ell=pr.ell, delta=pr.delta, sigma2=sig2, eta2=1e-3 * sig2)
    th = 1.01 * lipschitz.power_iteration(prob.normal, 64)[0]
    s.set_lipschitz(step, th)
    img, model, res = s.major_cycles(step, cycles, iters, low_res=_t(torch_dev, low, prec) if step == 2 else None)
    ref_img, ref_model, recs = twostep.major_cycles(step, np.asarray(dirty, np.float32 if prec == 32 else np.float64),
                                                    psf, cycles, iters, theta=th, positivity=True, **kw)
    assert rel(model.cpu().numpy(), ref_model) <= tol
    assert rel(img.cpu().numpy(), ref_img) <= tol
    for r, rec in zip(res, recs):
        assert r.objective == pytest.approx(rec["F"], rel=1e-10 if prec == 64 else 1e-5)
        assert r.iters == iters
    # the context's dirty image is unchanged: a plain solve still matches the oracle's first cycle
    lam = 0.05 * np.linalg.norm(np.asarray(dirty, np.float64))
    if step == 1:
        _, r1 = s.step1(lam, iters)
    else:
        _, r1 = s.step2(lam, _t(torch_dev, low, prec), iters)
    assert r1.objective == pytest.approx(recs[0]["F"], rel=1e-10 if prec == 64 else 1e-5)


def test_two_step_with_major_cycles_f64(torch_dev):
    """multistep.two_step (2 major cycles per step) against the oracle chain,
    with the step sizes the library's power iteration chose."""
    from oracle import twostep, helpers
    from paper_2406_18356_amd import multistep

    pr = _problem(32, 2, seed=4)
    s = _solver(torch_dev, pr, positivity=True, prec=64)
    img, i_L, rep = multistep.two_step(pr, cycles=2, iters=30, precision=64, solver=s)
    th1 = 1.01 * s.lipschitz(1)[0]
    th2 = 1.01 * s.lipschitz(2)[0]
    ref_iL, _, _ = twostep.major_cycles(1, pr.dirty_L, pr.psf_L, 2, 30, theta=th1, positivity=True)
    assert rel(i_L.cpu().numpy(), ref_iL) <= TOL64
    sig2 = helpers.sigma2_hat(pr.dirty_H)
    assert rep["sigma2"] == pytest.approx(sig2, rel=1e-12)
    ref_img, _, _ = twostep.major_cycles(2, pr.dirty_H, pr.psf_H, 2, 30, theta=th2, positivity=True, low_res=ref_iL,
                                         ell=pr.ell, delta=pr.delta, sigma2=sig2, eta2=1e-3 * sig2)
    assert rel(img.cpu().numpy(), ref_img) <= 1e-8


# ------------------------------------------------------------ checkpoints
@pytest.mark.parametrize("prec,dictionary,step", [(64, 0, 1), (64, 0, 2), (32, 0, 1), (64, 1, 2), (32, 1, 1)])
def test_checkpoint_resume(torch_dev, prec, dictionary, step):
    """K1 iterations, msr_get_state, msr_set_state on a new context, K2 more:
    the same iterate and objective as one solve of K1 + K2 iterations (FP64
    to rounding, FP32 bit for bit: the same kernels in the same order)."""
    from oracle import lipschitz, objectives
    from paper_2406_18356_amd import Solver

    n, K1, K2 = 32, 7, 9
    pr = _problem(n, 2, seed=8)
    T = lambda a: _t(torch_dev, a, prec)  # noqa: E731

    def make():
        s = Solver(n, positivity=not dictionary, precision=prec, dictionary=dictionary)
        s.set_dirty_psf(1, T(pr.dirty_L), T(pr.psf_L))
        s.set_dirty_psf(2, T(pr.dirty_H), T(pr.psf_H))
        s.set_filters(pr.ell, pr.delta, 0.8, 0.3)
        return s

    prob = (objectives.Step1(pr.dirty_L, pr.psf_L) if step == 1 else
            objectives.Step2(pr.dirty_H, pr.psf_H, np.zeros((n, n)), pr.ell, pr.delta, 0.8, 0.3))
    theta = (8 if dictionary else 1) * 1.01 * lipschitz.lanczos(prob.normal, n)[0]
    lam = 0.03 * float(np.linalg.norm(pr.dirty_L if step == 1 else pr.dirty_H))
    l = T(0.5 * pr.dirty_L)
    run = (lambda s, K: s.step1(lam, K)) if step == 1 else (lambda s, K: s.step2(lam, l, K))
    a = make()
    a.set_lipschitz(step, theta)
    full, rf = run(a, K1 + K2)
    b = make()
    b.set_lipschitz(step, theta)
    run(b, K1)
    bk, bp, k = b.get_state(step)
    assert k == K1
    c = make()
    c.set_lipschitz(step, theta)
    c.set_state(step, bk, bp, k)
    part, rp = run(c, K2)
    assert rp.iters == K2
    f, p_ = full.cpu().numpy(), part.cpu().numpy()
    if prec == 32:
        assert np.array_equal(f, p_)
    else:
        assert rel(p_, f) <= 1e-13
    assert rp.objective == pytest.approx(rf.objective, rel=1e-12 if prec == 64 else 1e-7)
    # the state is gone after another solve; a loaded state blocks major cycles
    run(c, 1)
    c.set_state(step, bk, bp, k)
    from paper_2406_18356_amd.binding import MsrError
    with pytest.raises(MsrError):
        c.major_cycles(step, 1, 2, low_res=None if step == 1 else l)
    with pytest.raises(MsrError):
        a.get_state(3 - step)


def test_maximum_size_8192_sampled(torch_dev):
    """The largest FP32 image (8192^2 on a 16384^2 grid, every spectral column
    kept): a symmetric PSF of a few delta taps makes H x and one FISTA step
    exact short sums, checked at sampled pixels (corners included, where the
    zero padding cuts the taps)."""
    from paper_2406_18356_amd import Solver

    torch, dev = torch_dev
    n, P = 8192, 16384
    c = P // 2
    taps = {(0, 0): 1.0, (3, 0): 0.3, (-3, 0): 0.3, (0, 5): -0.2, (0, -5): -0.2, (7, 7): 0.1, (-7, -7): 0.1}
    psf = torch.zeros((P, P), dtype=torch.float32)
    for (a, b), v in taps.items():
        psf[c + a, c + b] = v
    rng = np.random.default_rng(12)
    pts_x = np.concatenate([rng.integers(0, n, (200, 2)), [[0, 0], [1, 2], [n - 1, n - 1], [n - 2, n - 3]]])
    xv = np.abs(rng.normal(size=len(pts_x))).astype(np.float32) + 0.5
    x = torch.zeros((n, n), dtype=torch.float32)
    x[pts_x[:, 0], pts_x[:, 1]] = torch.from_numpy(xv)
    yv = rng.normal(size=len(pts_x)).astype(np.float32) * 0.1
    y = torch.zeros((n, n), dtype=torch.float32)
    y[pts_x[:, 0], pts_x[:, 1]] = torch.from_numpy(yv)
    X = {tuple(p): float(v) for p, v in zip(pts_x, xv)}
    Y = {tuple(p): float(v) for p, v in zip(pts_x, yv)}

    def H(p):  # (H x)[p] = sum_t psf_t x[p - t]
        return sum(v * X.get((p[0] - a, p[1] - b), 0.0) for (a, b), v in taps.items())

    def Ht_r(q):  # (H^T (H x - y))[q] = sum_t psf_t r[q + t], r on the image only
        tot = 0.0
        for (a, b), v in taps.items():
            p = (q[0] + a, q[1] + b)
            if 0 <= p[0] < n and 0 <= p[1] < n:
                tot += v * (H(p) - Y.get(p, 0.0))
        return tot

    s = Solver(n, positivity=True, precision=32)
    s.set_dirty_psf(1, y.to(dev), psf.to(dev))
    del psf
    hx = s.apply_psf(1, x.to(dev)).cpu().numpy()
    check = [tuple(p) for p in pts_x[:60]] + [(0, 0), (n - 1, n - 1), (3, 0), (n - 1, n - 6), (10, 12)]
    peak = float(np.max(np.abs(hx)))
    for p in check:
        assert abs(hx[p] - H(p)) <= OP_TOL * peak, (p, hx[p], H(p))
    theta = 2.0 * (1.0 + 0.6 + 0.4 + 0.2) ** 2  # >= 2 max |h_hat|^2
    lam = 0.2
    s.set_lipschitz(1, theta)
    b, _ = s.step1(lam, 1, x0=x.to(dev))
    b = b.cpu().numpy()
    mu = 1.0 / theta
    for q in check + [(pts_x[k][0] + 3, pts_x[k][1]) for k in range(20) if pts_x[k][0] + 3 < n]:
        want = max(X.get(q, 0.0) - mu * 2.0 * Ht_r(q) - mu * lam, 0.0)
        assert abs(b[q] - want) <= 2e-6 * max(xv.max(), 1.0), (q, b[q], want)
