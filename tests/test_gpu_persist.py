"""The persistent batched launch (msr_batch_set_mode(batch, 1, ...)): every
channel's FISTA passes run as work items of one kernel.  Each channel must
match the same problem solved alone with the kernel variants of the same
transform size (8 complex values per thread below 4096, 16 at 4096: the
persistent kernel's blocking), whatever the channel mix; the host's give-up
flag and the wait limit must end the launch with an error, after which the
batch solves normally again."""
import numpy as np
import pytest

import synth
from synth.generator import tiny

pytestmark = pytest.mark.gpu

# The persistent launch is switched off (msr_batch_set_mode(batch, 1) returns
# MSR_ERR_UNSUPPORTED).  Its first run, test_persistent_matches_single_channel_solves,
# printed nothing for 180 s and was stopped.  Every wave of every work item
# then wrote back and invalidated its XCD's whole L2 (agent-scope fences); with
# queues per XCD and L1-only ordering instead, the same test's first solve
# still did not return within 150 s.  No cause has been shown, so these cases
# stay off the GPU.
OFF = pytest.mark.skip(reason="persistent launch switched off: its first solve did not return in two runs; "
                              "cause not found")

SAME = 1e-6  # the same arithmetic as the single-channel solve; allows for signed zeros only


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    print("gpu persist: device", torch.cuda.get_device_name(0), flush=True)
    return torch, torch.device("cuda:0")


def _t(torch_dev, a):
    torch, dev = torch_dev
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)


def _setup(torch_dev, solver, pr):
    solver.set_dirty_psf(1, _t(torch_dev, pr.dirty_L), _t(torch_dev, pr.psf_L))
    solver.set_dirty_psf(2, _t(torch_dev, pr.dirty_H), _t(torch_dev, pr.psf_H))
    sig2 = float(np.var(pr.dirty_H))
    solver.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)


def _match_variants(solver, n):
    # the persistent kernel's blocking: variant 1 (E = 8) below 4096, 0 (E = 16) at 4096
    v = 0 if n >= 4096 else 1
    for step in (1, 2):
        solver.set_variants(step, v, v, v if step == 2 else -1)


_CACHE = {}


def _problems(spec):
    key = tuple(spec)
    if key not in _CACHE:
        _CACHE[key] = [synth.make_problem(tiny(n, seed=seed, cut=cut, n_ant=24)) for n, seed, cut in spec]
    return _CACHE[key]


def _compare(torch_dev, spec, K, positivity=True, reps=1):
    from paper_2406_18356_amd import Batch, Solver

    prs = _problems(spec)
    print("persistent vs single:", [pr.n for pr in prs], "K", K, flush=True)
    b = Batch([pr.n for pr in prs], positivity=positivity)
    b.set_mode(1)
    singles = [Solver(pr.n, positivity=positivity) for pr in prs]
    for pr, ch, s in zip(prs, b.channels, singles):
        _setup(torch_dev, ch, pr)
        _setup(torch_dev, s, pr)
        _match_variants(s, pr.n)
    for rep in range(reps):
        scale = (0.05, 0.03)[rep % 2]
        lam1 = [scale * np.linalg.norm(pr.dirty_L) for pr in prs]
        x0 = None
        if rep:
            x0 = [_t(torch_dev, np.abs(np.random.default_rng(c + rep).normal(size=(pr.n, pr.n))) * 1e-3)
                  for c, pr in enumerate(prs)]
        models1, imgs1, res1 = b.solve(1, lam1, K, x0=x0, image=True)
        for c, (pr, s) in enumerate(zip(prs, singles)):
            s.set_lipschitz(1, res1[c].theta)
            bs, ims, rs = s.step1(lam1[c], K, x0=None if x0 is None else x0[c], image=True)
            assert rel(models1[c].cpu().numpy(), bs.cpu().numpy()) <= SAME, (rep, c)
            assert rel(imgs1[c].cpu().numpy(), ims.cpu().numpy()) <= SAME, (rep, c)
            assert res1[c].objective == pytest.approx(rs.objective, rel=1e-6)
            assert res1[c].iters == K
        low = [m.clone() for m in imgs1]
        lam2 = [scale * np.linalg.norm(pr.dirty_H) for pr in prs]
        models2, res2 = b.solve(2, lam2, K, low_res=low, x0=x0)
        for c, (pr, s) in enumerate(zip(prs, singles)):
            s.set_lipschitz(2, res2[c].theta)
            bs, rs = s.step2(lam2[c], low[c], K, x0=None if x0 is None else x0[c])
            assert rel(models2[c].cpu().numpy(), bs.cpu().numpy()) <= SAME, (rep, c)
            assert res2[c].objective == pytest.approx(rs.objective, rel=1e-6)
            if positivity:
                assert float(models2[c].min()) >= 0
    return b, prs


MIX = [(512, 21, 0.25), (1024, 22, 0.3), (512, 23, 0.2), (2048, 24, 0.25)]


@OFF
def test_persistent_matches_single_channel_solves(torch_dev):
    """Mixed sizes, several channels of one size; a second solve with other
    lambdas and warm starts replays the captured launch."""
    _compare(torch_dev, MIX, 30, reps=2)


@OFF
def test_persistent_without_positivity(torch_dev):
    _compare(torch_dev, MIX[:2], 20, positivity=False)


@OFF
def test_persistent_with_a_4096_channel(torch_dev):
    _compare(torch_dev, [(4096, 25, 0.25), (512, 26, 0.3)], 8)


@OFF
def test_persistent_one_channel_one_iteration(torch_dev):
    _compare(torch_dev, [(1024, 27, 0.25)], 1)


@OFF
def test_persistent_give_up_and_wait_limit(torch_dev):
    """The host's flag and a wait limit of one poll end the launch (every
    block returns) with an error; with the flag cleared and the default limit
    the batch solves as before."""
    from paper_2406_18356_amd import Batch, binding
    from paper_2406_18356_amd.binding import MsrError

    prs = _problems(MIX)
    b = Batch([pr.n for pr in prs], positivity=True)
    for pr, ch in zip(prs, b.channels):
        _setup(torch_dev, ch, pr)
    lam = [0.05 * np.linalg.norm(pr.dirty_L) for pr in prs]
    b.set_mode(1)
    ref, _ = b.solve(1, lam, 20)
    ref = [m.cpu().numpy() for m in ref]
    print("give-up flag", flush=True)
    b.give_up(True)
    with pytest.raises(MsrError) as e:
        b.solve(1, lam, 20)
    assert e.value.status == binding.ERR_HIP and "give-up" in str(e.value)
    b.give_up(False)
    print("wait limit 1", flush=True)
    b.set_mode(1, spin_limit=1)
    with pytest.raises(MsrError) as e:
        b.solve(1, lam, 20)
    assert e.value.status == binding.ERR_HIP and "spin limit" in str(e.value)
    print("recovery", flush=True)
    b.set_mode(1)
    again, _ = b.solve(1, lam, 20)
    for c in range(len(prs)):
        assert rel(again[c].cpu().numpy(), ref[c]) == 0.0, c


def test_persistent_mode_refused_while_switched_off(torch_dev):
    """msr_batch_set_mode: 2 is invalid, 1 is refused while the persistent
    launch is switched off, and the batch keeps solving in mode 0."""
    from paper_2406_18356_amd import Batch, binding
    from paper_2406_18356_amd.binding import MsrError

    prs = _problems([(256, 28, 0.25), (512, 29, 0.25)])
    b = Batch([pr.n for pr in prs])
    for pr, ch in zip(prs, b.channels):
        _setup(torch_dev, ch, pr)
    with pytest.raises(MsrError) as e:
        b.set_mode(2)
    assert e.value.status == binding.ERR_INVALID
    with pytest.raises(MsrError) as e:
        b.set_mode(1)
    assert e.value.status == binding.ERR_UNSUPPORTED and "switched off" in str(e.value)
    b.set_mode(0)
    models, res = b.solve(1, [1.0, 1.0], 5)
    assert all(r.iters == 5 for r in res)
