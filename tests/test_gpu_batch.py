"""Batched solves (msr_batch_*): channels of mixed sizes advanced by shared
launches inside one captured HIP graph.  Each channel must match the same
problem solved alone (same kernels, same arithmetic), and the oracle."""
import numpy as np
import pytest

import synth
from synth.generator import tiny

pytestmark = pytest.mark.gpu

TOL = 1e-5
TOL64 = 1e-9
SAME = 1e-6  # batched vs single-context FP32: same arithmetic; allows for signed zeros only


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    print("gpu batch: device", torch.cuda.get_device_name(0), flush=True)
    return torch, torch.device("cuda:0")


def _t(torch_dev, a, prec=32):
    torch, dev = torch_dev
    return torch.from_numpy(np.ascontiguousarray(a, np.float32 if prec == 32 else np.float64)).to(dev)


# mixed sizes, several channels of one size (one launch per pass for them),
# different uv coverage and cuts per channel
SIZES = [(64, 11, 0.25), (32, 12, 0.3), (64, 13, 0.2), (16, 14, 0.25), (64, 15, 0.35)]


def _channels():
    return [synth.make_problem(tiny(n, seed=seed, cut=cut)) for n, seed, cut in SIZES]


def _poison(obj):
    """Fill a Batch's or Solver's workspace with NaN bytes, then hand it over
    again (which rebuilds the twiddle table): any read of an element no pass
    has written then shows up as NaN, even where a zero factor multiplies it."""
    import ctypes as C
    from paper_2406_18356_amd import Batch

    obj._ws.fill_(0xFF)
    ptr = C.c_void_p((obj._ws.data_ptr() + 255) // 256 * 256)
    if isinstance(obj, Batch):
        obj._check(obj._lib.msr_batch_set_workspace(obj._h, ptr, obj.workspace_bytes))
    else:
        obj._check(obj._lib.msr_set_workspace(obj._h, ptr, obj.workspace_bytes))


def _setup(torch_dev, solver, pr, prec, step2_low=None):
    solver.set_dirty_psf(1, _t(torch_dev, pr.dirty_L, prec), _t(torch_dev, pr.psf_L, prec))
    solver.set_dirty_psf(2, _t(torch_dev, pr.dirty_H, prec), _t(torch_dev, pr.psf_H, prec))
    sig2 = float(np.var(pr.dirty_H))
    solver.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
    return sig2


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("positivity", [True, False])
def test_batch_matches_single_channel_solves(torch_dev, prec, positivity):
    from paper_2406_18356_amd import Batch, Solver

    print(f"batch vs single prec={prec} positivity={positivity}", flush=True)
    prs = _channels()
    b = Batch([pr.n for pr in prs], positivity=positivity, precision=prec)
    singles = [Solver(pr.n, positivity=positivity, precision=prec) for pr in prs]
    for x in [b] + singles:
        _poison(x)
    for pr, ch, s in zip(prs, b.channels, singles):
        _setup(torch_dev, ch, pr, prec)
        _setup(torch_dev, s, pr, prec)
    K = 25
    lam1 = [0.05 * np.linalg.norm(pr.dirty_L) for pr in prs]
    models1, imgs1, res1 = b.solve(1, lam1, K, image=True)
    tol = TOL64 * 1e-3 if prec == 64 else SAME
    for c, (pr, s) in enumerate(zip(prs, singles)):
        s.set_lipschitz(1, res1[c].theta)  # same theta as the batch found by power iteration
        bs, ims, rs = s.step1(lam1[c], K, image=True)
        assert rel(models1[c].cpu().numpy(), bs.cpu().numpy()) <= tol, c
        assert rel(imgs1[c].cpu().numpy(), ims.cpu().numpy()) <= tol, c
        assert res1[c].objective == pytest.approx(rs.objective, rel=1e-12 if prec == 64 else 1e-6)
        assert res1[c].iters == K
    # step 2 with each channel's low-resolution image as the constraint
    low = [m.clone() for m in models1]
    lam2 = [0.05 * np.linalg.norm(pr.dirty_H) for pr in prs]
    models2, res2 = b.solve(2, lam2, K, low_res=low)
    for c, (pr, s) in enumerate(zip(prs, singles)):
        s.set_lipschitz(2, res2[c].theta)
        bs, rs = s.step2(lam2[c], low[c], K)
        assert rel(models2[c].cpu().numpy(), bs.cpu().numpy()) <= tol, c
        assert res2[c].objective == pytest.approx(rs.objective, rel=1e-12 if prec == 64 else 1e-6)
        if positivity:
            assert float(models2[c].min()) >= 0


def test_batch_frequency_channels_match_single_channel_solves(torch_dev):
    """Channels of one size whose coverage scales with frequency (350-1050
    MHz): their kept columns span about 3x, so the solve splits the size group
    (2048^2: groups of 2048^2 and larger are split) into several runs of
    similar width.  Every channel must still match its single-context solve,
    in both steps."""
    from paper_2406_18356_amd import Batch, Solver

    cfgs = synth.channel_set(4, sizes=(2048,), seed=3, n_ant=16, dt_s=600.0)
    print("frequency channels: synthesising 4 x 2048^2", flush=True)
    prs = [synth.make_problem(c, with_full=False) for c in cfgs]
    b = Batch([pr.n for pr in prs], positivity=True)
    singles = [Solver(pr.n, positivity=True) for pr in prs]
    for x in [b] + singles:
        _poison(x)
    for pr, ch, s in zip(prs, b.channels, singles):
        _setup(torch_dev, ch, pr, 32)
        _setup(torch_dev, s, pr, 32)
    K = 10
    lam1 = [0.05 * np.linalg.norm(pr.dirty_L) for pr in prs]
    models1, imgs1, res1 = b.solve(1, lam1, K, image=True)
    for c, s in enumerate(singles):
        s.set_lipschitz(1, res1[c].theta)
        bs, ims, rs = s.step1(lam1[c], K, image=True)
        assert rel(models1[c].cpu().numpy(), bs.cpu().numpy()) <= SAME, c
        assert rel(imgs1[c].cpu().numpy(), ims.cpu().numpy()) <= SAME, c
    low = [m.clone() for m in imgs1]
    lam2 = [0.05 * np.linalg.norm(pr.dirty_H) for pr in prs]
    models2, res2 = b.solve(2, lam2, K, low_res=low)
    for c, s in enumerate(singles):
        s.set_lipschitz(2, res2[c].theta)
        bs, rs = s.step2(lam2[c], low[c], K)
        assert rel(models2[c].cpu().numpy(), bs.cpu().numpy()) <= SAME, c
        assert res2[c].objective == pytest.approx(rs.objective, rel=1e-6)


def test_batch_against_oracle_and_graph_replay(torch_dev):
    """FP64 batch vs the FP64 oracle per channel; a second solve with other
    lambdas and warm starts replays the cached graph with new parameters."""
    from oracle import objectives, fista, lipschitz
    from paper_2406_18356_amd import Batch

    prs = _channels()
    b = Batch([pr.n for pr in prs], positivity=True, precision=64)
    probs, thetas = [], []
    for pr, ch in zip(prs, b.channels):
        _setup(torch_dev, ch, pr, 64)
        p1 = objectives.Step1(pr.dirty_L, pr.psf_L)
        th = 1.01 * lipschitz.power_iteration(p1.normal, pr.n)[0]
        ch.set_lipschitz(1, th)
        probs.append(p1)
        thetas.append(th)
    K = 40
    for rep, scale in enumerate((0.05, 0.02, 0.05)):
        lam = [scale * np.linalg.norm(pr.dirty_L) for pr in prs]
        x0 = None
        if rep >= 1:
            x0 = [_t(torch_dev, np.abs(np.random.default_rng(c + rep).normal(size=(pr.n, pr.n))) * 1e-2, 64)
                  for c, pr in enumerate(prs)]
        models, res = b.solve(1, lam, K, x0=x0)
        for c, pr in enumerate(prs):
            x0c = np.zeros((pr.n, pr.n)) if x0 is None else x0[c].cpu().numpy()
            bo, _ = fista.fista(probs[c].grad, x0c, 1 / thetas[c], lam[c], K, positivity=True)
            assert rel(models[c].cpu().numpy(), bo) <= TOL64, (rep, c)
            assert res[c].objective == pytest.approx(probs[c].objective(bo, lam[c])[0], rel=1e-10)


def test_batch_fp32_short_trajectory_vs_oracle(torch_dev):
    from oracle import objectives, fista, lipschitz
    from paper_2406_18356_amd import Batch

    prs = _channels()
    b = Batch([pr.n for pr in prs], positivity=True)
    _poison(b)
    K = 10
    lam, probs, ths = [], [], []
    for pr, ch in zip(prs, b.channels):
        _setup(torch_dev, ch, pr, 32)
        p1 = objectives.Step1(pr.dirty_L, pr.psf_L)
        th = 1.01 * lipschitz.power_iteration(p1.normal, pr.n)[0]
        ch.set_lipschitz(1, th)
        probs.append(p1)
        ths.append(th)
        lam.append(0.05 * np.linalg.norm(pr.dirty_L))
    models, _ = b.solve(1, lam, K)
    for c, pr in enumerate(prs):
        bo, _ = fista.fista(probs[c].grad, np.zeros((pr.n, pr.n)), 1 / ths[c], lam[c], K, positivity=True)
        assert rel(models[c].cpu().numpy(), bo) <= TOL, c


def test_batch_errors_and_zero_iterations(torch_dev):
    from paper_2406_18356_amd import Batch, binding
    from paper_2406_18356_amd.binding import MsrError

    prs = _channels()[:2]
    b = Batch([pr.n for pr in prs])
    lam = [1.0, 1.0]
    with pytest.raises(MsrError) as e:
        b.solve(1, lam, 5)  # no PSF yet
    assert e.value.status == binding.ERR_STATE
    for pr, ch in zip(prs, b.channels):
        ch.set_dirty_psf(1, _t(torch_dev, pr.dirty_L), _t(torch_dev, pr.psf_L))
        ch.set_dirty_psf(2, _t(torch_dev, pr.dirty_H), _t(torch_dev, pr.psf_H))
    with pytest.raises(MsrError) as e:
        b.solve(2, lam, 5, low_res=[ch._img() for ch in b.channels])  # no filters
    assert e.value.status == binding.ERR_STATE
    with pytest.raises(MsrError) as e:
        b.solve(1, [1.0, -1.0], 5)
    assert e.value.status == binding.ERR_INVALID
    x0 = [_t(torch_dev, np.full((pr.n, pr.n), 0.25)) for pr in prs]
    models, res = b.solve(1, lam, 0, x0=x0)  # zero iterations: the start comes back
    for m in models:
        assert float((m - 0.25).abs().max()) == 0.0
    assert all(r.iters == 0 for r in res)
