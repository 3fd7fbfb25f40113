"""What the trained warm start gains over the method without it, on held-out
skies of the workload it was trained for (1024^2, the network stored with the
package).  Step 2 runs from zero and from the network's prediction, both
restarted at k = 1 (Algorithm 1), with the exact objective recorded every 500
iterations; F_ref is the lower of the two runs' best objectives.

Measured on 100 held-out skies, the prediction starts about 15x closer to
F_ref than zero does, and both runs reach a 1e-5 relative objective within
about 0.1 % of each other.  The test checks both facts on two skies: the
initial gap shrinks at least fivefold, and the network's run is no more than
5 % slower than the cold one (its forward pass included)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch

    import synth
    from paper_2406_18356_amd import UNet, warmstart as ws
    from paper_2406_18356_amd.warmstart_study import base_problem

    params, meta = ws.load_weights()
    assert params is not None, "the packaged network is missing"
    print("warm start: synthesising the 1024^2 observation", flush=True)
    base = base_problem(1024)
    skies = synth.sky_set(base, 2, 2000)  # the held-out seed stream (training used 1000)
    net = UNet(1, base.n)
    net.set_params(params)
    return torch, skies, net


@pytest.mark.parametrize("i", [0, 1])
def test_learned_start_against_cold_start(setup, i):
    torch, skies, net = setup
    from paper_2406_18356_amd import Solver, warmstart as ws

    p = skies[i]
    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)  # noqa: E731
    s = Solver(p.n, positivity=True)
    dl, dh = T(p.dirty_L), T(p.dirty_H)
    s.set_dirty_psf(1, dl, T(p.psf_L))
    s.set_dirty_psf(2, dh, T(p.psf_H))
    s.lipschitz(1)
    _, il, _ = s.step1(s.default_lambda(1, 1, 0.05), 500, image=True)
    sig2 = s.estimate_sigma2(dh)
    s.set_filters(p.ell, p.delta, sig2, 1e-3 * sig2)
    s.lipschitz(2)
    lam2 = s.default_lambda(2, 1, 0.05)
    x_net, fms = ws.timed_forward(net, dh[None].contiguous(), il[None].contiguous())
    x_net = x_net[0].contiguous()
    print(f"sky {i}: trajectories", flush=True)
    cold = ws.trajectory(s, lam2, il, x0=None, iters=16000, every=500)
    warm = ws.trajectory(s, lam2, il, x0=x_net, iters=16000, every=500)
    f_ref = min(min(cold["F"]), min(warm["F"]))
    g_cold = (s.objective(2, lam2, torch.zeros_like(dh), il)[0] - f_ref) / abs(f_ref)
    g_net = (s.objective(2, lam2, x_net, il)[0] - f_ref) / abs(f_ref)
    c = ws.crossing(cold, f_ref, 1e-5)
    w = ws.crossing(warm, f_ref, 1e-5, fms)
    print(f"sky {i}: initial gap {g_cold:.3g} -> {g_net:.3g}; time to 1e-5: cold {c['ms']:.0f} ms "
          f"({c['iters']} it), network {w['ms']:.0f} ms ({w['iters']} it)", flush=True)
    assert g_net < g_cold / 5
    assert c["converged"] and w["converged"]
    assert w["ms"] <= 1.05 * c["ms"]
