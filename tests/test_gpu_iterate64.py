"""Float64 iterates with float32 transforms (msr_config.iterate_precision =
64).  Rounding the iterate to float32 every iteration is what makes FP32
FISTA drift from the FP64 trajectory and stall above the FP64 objective;
keeping beta_k and the update in float64 while the FFTs, the PSF and filter
products stay in float32 holds the trajectory to the FP64 oracle within 1e-5
of peak over hundreds of iterations, where the all-float32 path drifts to
several 1e-5.  Also: the state (float64 images) round trip, and the
combinations the mode refuses."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    print("gpu iterate64: device", torch.cuda.get_device_name(0), flush=True)
    return torch, torch.device("cuda:0")


def _t(torch_dev, a, dt=np.float32):
    torch, dev = torch_dev
    return torch.from_numpy(np.ascontiguousarray(a, dt)).to(dev)


def _solver(torch_dev, pr, iterate_precision=64, positivity=True):
    from paper_2406_18356_amd import Solver

    s = Solver(pr.n, pad=pr.cfg.pad, positivity=positivity, iterate_precision=iterate_precision)
    s.set_dirty_psf(1, _t(torch_dev, pr.dirty_L), _t(torch_dev, pr.psf_L))
    s.set_dirty_psf(2, _t(torch_dev, pr.dirty_H), _t(torch_dev, pr.psf_H))
    return s


def test_float64_iterates_follow_the_fp64_oracle(torch_dev):
    """The 256^2 workload, K = 50, 100, 200 and 400 iterations of each step
    from zero.  Up to K = 200 the float64-iterate path stays within 1e-5 of
    the FP64 oracle's peak (the all-float32 path reaches 6.6e-5 at K = 200).
    At every K it is at least five times closer to the FP64 oracle than the
    oracle run entirely in float32 is: the drift of FP32 FISTA comes from
    rounding the iterate, and the float32 transforms left here (with the
    pruned spectral columns) cost a fraction of it.  Objectives agree to
    1e-6."""
    from oracle import objectives, fista, lipschitz, helpers

    pr = synth.make_problem(synth.preset("small256"))
    n, Ks = pr.n, (50, 100, 200, 400)
    s = _solver(torch_dev, pr)

    def traj(prob, th, lam, dt=np.float64):
        out = {}
        fista.fista(prob.grad, np.zeros((n, n)), 1 / th, lam, max(Ks), positivity=True, dtype=dt,
                    callback=lambda k, b: out.__setitem__(k, b.astype(np.float64)) if k in Ks else None)
        return out

    s1 = objectives.Step1(pr.dirty_L, pr.psf_L)
    th1 = 1.01 * lipschitz.power_iteration(s1.normal, n)[0]
    lam1 = helpers.default_lambda(pr.dirty_L)
    a1 = traj(s1, th1, lam1)
    m1 = traj(objectives.Step1(pr.dirty_L, pr.psf_L, dtype=np.float32), th1, lam1, np.float32)
    iL = helpers.low_res_image(a1[200], pr.dirty_L, s1.H).astype(np.float32).astype(np.float64)
    sig2 = helpers.sigma2_hat(pr.dirty_H)
    s2 = objectives.Step2(pr.dirty_H, pr.psf_H, iL, pr.ell, pr.delta, sig2, 1e-3 * sig2)
    th2 = 1.01 * lipschitz.power_iteration(s2.normal, n)[0]
    lam2 = helpers.default_lambda(pr.dirty_H)
    a2 = traj(s2, th2, lam2)
    m2 = traj(objectives.Step2(pr.dirty_H, pr.psf_H, iL, pr.ell, pr.delta, sig2, 1e-3 * sig2, dtype=np.float32),
              th2, lam2, np.float32)
    s.set_lipschitz(1, th1)
    s.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
    s.set_lipschitz(2, th2)
    lt = _t(torch_dev, iL)
    for K in Ks:
        b1, r1 = s.step1(lam1, K)
        b2, r2 = s.step2(lam2, lt, K)
        g1, g2 = rel(b1.cpu().numpy(), a1[K]), rel(b2.cpu().numpy(), a2[K])
        f1 = abs(r1.objective - s1.objective(a1[K], lam1)[0]) / abs(s1.objective(a1[K], lam1)[0])
        f2 = abs(r2.objective - s2.objective(a2[K], lam2)[0]) / abs(s2.objective(a2[K], lam2)[0])
        o1, o2 = rel(m1[K], a1[K]), rel(m2[K], a2[K])
        print(f"K={K}: step 1 {g1:.3g} (oracle in float32 {o1:.3g}, objective {f1:.2g}), "
              f"step 2 {g2:.3g} (oracle in float32 {o2:.3g}, objective {f2:.2g})", flush=True)
        if K <= 200:
            assert g1 <= TOL and g2 <= TOL
        assert g1 <= o1 / 5 and g2 <= o2 / 5
        assert f1 <= 1e-6 and f2 <= 1e-6


def test_float64_state_round_trip(torch_dev):
    """K1 iterations, the float64 state out and into a second context, K2 more:
    the iterate of one solve of K1 + K2 iterations, bit for bit."""
    import torch

    pr = synth.make_problem(synth.preset("small256"))
    a = _solver(torch_dev, pr)
    b = _solver(torch_dev, pr)
    a.lipschitz(1)
    b.set_lipschitz(1, a.step1(1.0, 1)[1].theta)
    lam = a.default_lambda(1, 1, 0.05)
    ref, _ = a.step1(lam, 60)
    a.step1(lam, 25)
    bk, bp, k = a.get_state(1)
    assert bk.dtype == torch.float64 and k == 25
    b.set_state(1, bk, bp, k)
    out, r = b.step1(lam, 35)
    assert r.iters == 35
    assert torch.equal(out, ref)


def test_float64_iterates_refused_where_not_built(torch_dev):
    from paper_2406_18356_amd import binding
    from paper_2406_18356_amd.binding import MsrError

    pr = synth.make_problem(synth.preset("small256"))
    s = _solver(torch_dev, pr)
    s.lipschitz(1)
    with pytest.raises(MsrError) as e:
        s.major_cycles(1, 2, 5)
    assert e.value.status == binding.ERR_UNSUPPORTED


def test_float64_iterates_circular_and_checked_loop(torch_dev):
    """Circular mode (pad 1) against the FP64 oracle after 100 iterations,
    and a loop with exact objective checks every 10 iterations (the iterate
    is rounded into a scratch image for them) giving the same model and
    objective as the loop without checks."""
    import torch
    from oracle import objectives, fista, lipschitz, helpers
    from synth.generator import tiny

    pr = synth.make_problem(tiny(64, seed=9).replace(pad=1))
    s = _solver(torch_dev, pr)
    p1 = objectives.Step1(pr.dirty_L, pr.psf_L)
    th = 1.01 * lipschitz.power_iteration(p1.normal, pr.n)[0]
    lam = helpers.default_lambda(pr.dirty_L)
    ref, _ = fista.fista(p1.grad, np.zeros((pr.n, pr.n)), 1 / th, lam, 100, positivity=True)
    s.set_lipschitz(1, th)
    b, r = s.step1(lam, 100)
    print(f"circular 64^2, K = 100: {rel(b.cpu().numpy(), ref):.3g}", flush=True)
    assert rel(b.cpu().numpy(), ref) <= TOL
    b2, r2 = s.step1(lam, 100, check_every=10)
    assert torch.equal(b2, b) and r2.objective == r.objective
