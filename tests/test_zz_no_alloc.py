"""The allocation-free workspace (msr_set_workspace_static) against a caller
workspace (msr_set_workspace), through the C ABI.

Two contexts of one configuration, one on a torch-allocated workspace and one
on the library's static device array, get the same dirty images, PSFs,
filters and step sizes; both steps of the two-step solve (Eqs. 4 and 5 with
Algorithm 1), the exact objective and the step-1 image must agree bit for bit
(same kernels, same launch shapes, deterministic reductions).  This is done
for two calls in a row, the second on a smaller image, which re-binds the
array to a new context and takes it from the first one.
"""
import ctypes as C

import numpy as np
import pytest

import synth
from synth.generator import tiny

pytestmark = pytest.mark.gpu


def _t(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)


def _setup(s, torch, dev, pr, th1, th2, sig2):
    s.set_dirty_psf(1, _t(torch, dev, pr.dirty_L), _t(torch, dev, pr.psf_L))
    s.set_dirty_psf(2, _t(torch, dev, pr.dirty_H), _t(torch, dev, pr.psf_H))
    s.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
    s.set_lipschitz(1, th1)
    s.set_lipschitz(2, th2)


def _run(s, lam1, lam2, iters):
    b1, iL, r1 = s.step1(lam1, iters, image=True)
    b2, r2 = s.step2(lam2, iL, iters)
    F = s.objective(2, lam2, b2, low_res=iL)
    return b1.cpu().numpy(), iL.cpu().numpy(), b2.cpu().numpy(), r1.objective, r2.objective, F


@pytest.mark.parametrize("positivity", [True])
def test_static_workspace_matches_caller_workspace(positivity):
    import torch

    from paper_2406_18356_amd import Solver, binding

    dev = torch.device("cuda:0")
    prev = None
    for n, seed in ((128, 21), (64, 22)):  # the second call is the smaller input
        print(f"no-alloc: n={n} seed={seed}", flush=True)
        assert binding.workspace_bytes(n) <= binding.STATIC_WORKSPACE_BYTES
        pr = synth.make_problem(tiny(n, seed=seed))
        ref = Solver(n, positivity=positivity)
        ref.set_dirty_psf(1, _t(torch, dev, pr.dirty_L), _t(torch, dev, pr.psf_L))
        ref.set_dirty_psf(2, _t(torch, dev, pr.dirty_H), _t(torch, dev, pr.psf_H))
        th1 = 1.01 * ref.lipschitz(1)[0]
        sig2 = ref.estimate_sigma2(_t(torch, dev, pr.dirty_H))
        ref.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
        th2 = 1.01 * ref.lipschitz(2)[0]
        lam1 = 0.05 * float(np.linalg.norm(pr.dirty_L))
        lam2 = 0.05 * float(np.linalg.norm(pr.dirty_H))

        st = Solver(n, positivity=positivity, static_workspace=True)
        assert st._ws is None
        _setup(st, torch, dev, pr, th1, th2, sig2)
        _setup(ref, torch, dev, pr, th1, th2, sig2)
        got = _run(st, lam1, lam2, 30)
        want = _run(ref, lam1, lam2, 30)
        torch.cuda.synchronize()
        for g, w in zip(got[:3], want[:3]):
            assert np.array_equal(g, w)
            assert np.abs(w).max() > 0
        assert got[3] == want[3] and got[4] == want[4]
        assert tuple(got[5]) == tuple(want[5])

        if prev is not None:
            # the new binding took the array from the previous static context
            with pytest.raises(binding.MsrError) as e:
                prev.step1(lam1, 1)
            assert e.value.status == binding.ERR_STATE
            # which can be given a caller workspace again and works
            ws = torch.empty(prev.workspace_bytes + 256, dtype=torch.uint8, device=dev)
            aligned = (ws.data_ptr() + 255) // 256 * 256
            prev._check(prev._lib.msr_set_workspace(prev._h, C.c_void_p(aligned), prev.workspace_bytes))
            prev._ws = ws
        prev = st


def test_static_workspace_rejects_large_configurations():
    import torch  # noqa: F401

    from paper_2406_18356_amd import Solver, binding

    n = 1024
    assert binding.workspace_bytes(n) > binding.STATIC_WORKSPACE_BYTES
    with pytest.raises(binding.MsrError) as e:
        Solver(n, static_workspace=True)
    assert e.value.status == binding.ERR_OOM
    assert "static workspace holds" in str(e.value)
