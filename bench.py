#!/usr/bin/env python3
"""Benchmark: the two-step minor-cycle FISTA solve on one MI355X.

One bench step = one whole two-step reconstruction on resident inputs:
PSF spectra of both splits, the Lanczos estimate of theta_L, step 1 (K FISTA
iterations) with the low-resolution image, sigma2_hat, filters, theta_H,
step 2 (K iterations, cold start).  The reported value is FISTA iterations
(both steps) per second of that whole job.

Also reported: the per-step loop rates, the time to a 1e-6 (and 1e-5)
relative objective in step 2 read off objective trajectories from a cold
start, from the low-resolution image and from the learned warm start (the
network trained at 1024^2 stored with the package), each restarted at k = 1
and entered at a later momentum index, against the lowest objective any run
reaches; the dominant pass against its roofline (the FP32
FMA rate these kernels can reach and HBM; timed live with HIP events), the
per-PSF setup, the wavelet dictionary, the
up-sampling of a down-sampled low-resolution image, batched channels, a
synthetic partition study and the FP64 CPU oracle timed on this host.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--size 2048|4096|8192]

The default workload is the 4096^2 image; --size 8192 runs the largest one
(its synthesis takes a minute or more on the host).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FISTA iters/s & time-to-1e-6 rel objective at 4096²; warm-start vs cold"
HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
# MI355X's published FP32 vector peak (it counts packed-FP32 instructions,
# two floats per lane), and the FMA rate the library's arithmetic can reach:
# its build excludes packed FP32, so 256 CUs x 64 FMA lanes per clock x 2
# flops x 2.4 GHz.  Both are reported; the roofline fraction of record is the
# HBM one (at 10-12 flop/B the passes sit below the 157.3 TF / 8 TB/s ridge).
FP32_PUBLISHED_TFLOPS = 157.3
FP32_VECTOR_TFLOPS = 78.6
BF16_MFMA_TFLOPS = 2500.0   # MI355X dense bf16 matrix peak


def traffic_file(kernel, workload):
    """HBM traffic of one pass measured with rocprofv3 counters (see prof_summary)."""
    return os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")

WORKLOADS = {
    2048: ("sky2048", "two-step solve, 2048x2048 image on a 4096x4096 zero-padded grid: 2000 points + 50 "
                      "Gaussians, 197 antennas 8 h at 30 s, cut 20%, 500 FISTA iterations per step, positivity on"),
    4096: ("sky4096", "two-step solve, 4096x4096 image on an 8192x8192 zero-padded grid: 8000 points + 200 "
                      "Gaussians, 197 antennas 8 h at 30 s, cut 15%, 500 FISTA iterations per step, positivity on"),
    8192: ("sky8192", "two-step solve, 8192x8192 image on a 16384x16384 zero-padded grid: 32000 points + 800 "
                      "Gaussians, 512 antennas 4 h at 10 s, cut 10%, 500 FISTA iterations per step, positivity on"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def two_step(s, dev, tensors, pr, iters, torch):
    dL, pL, dH, pH = tensors
    s.set_dirty_psf(1, dL, pL)
    s.set_dirty_psf(2, dH, pH)
    s.lipschitz(1)
    lam1 = s.default_lambda(1, 1, 0.05)
    b1, iL, r1 = s.step1(lam1, iters, image=True)
    sig2 = s.estimate_sigma2(dH)
    s.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
    s.lipschitz(2)
    lam2 = s.default_lambda(2, 1, 0.05)
    b2, r2 = s.step2(lam2, iL, iters)
    return r1, r2, iL, lam2, b1


def batch_bench(torch, dev, count, iters, seed=4, sizes=(512, 1024, 2048, 4096)):
    """Mixed-size frequency channels, step 1, `iters` iterations: one batched
    solve with one launch per pass per size (iterations in one HIP graph,
    each size on its own stream) against the channels solved one after the
    other with single contexts."""
    import synth
    from paper_2406_18356_amd import Batch, Solver

    t = time.perf_counter()
    cfgs = synth.channel_set(count, sizes=sizes, seed=seed)
    done = []

    def progress(i, p):
        done.append(i)
        if len(done) % 8 == 0 or len(done) == len(cfgs):
            log(f"batch: {len(done)}/{len(cfgs)} channels generated")

    prs = synth.make_problems(cfgs, workers=16, progress=progress)
    log(f"batch: {count} channels {[p.n for p in prs]} generated in {time.perf_counter() - t:.1f} s")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)  # noqa: E731
    b = Batch([p.n for p in prs], positivity=True)
    singles = [Solver(p.n, positivity=True) for p in prs]
    lam = []
    for pr, ch, s in zip(prs, b.channels, singles):
        d, psf = T(pr.dirty_L), T(pr.psf_L)
        ch.set_dirty_psf(1, d, psf)
        s.set_dirty_psf(1, d, psf)
        lam.append(s.default_lambda(1, 1, 0.05))
    b.autotune(reps=10)
    for s in singles:
        s.autotune(reps=10)
    out = {"channels": count, "sizes": [int(p.n) for p in prs], "iters": iters, "step": 1}
    # mode 1 (one persistent launch) is switched off in the library
    for mode, name in ((0, "batched"),):
        b.set_mode(mode)
        t = time.perf_counter()
        _, res = b.solve(1, lam, iters)  # sets theta, captures the graph
        out[f"{name}_first_call_with_capture_s"] = time.perf_counter() - t
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, res = b.solve(1, lam, iters)
        out[f"{name}_wall_s"] = time.perf_counter() - t
        out[f"{name}_channel_iters_per_s"] = count * iters / (res[0].elapsed_ms * 1e-3)
        log(f"batch mode {mode}: {res[0].elapsed_ms / iters * 1e3:.1f} us per iteration of all channels")
    for ch, r, s in zip(b.channels, res, singles):
        s.set_lipschitz(1, r.theta)
    torch.cuda.synchronize()
    t = time.perf_counter()
    loop_s = 0.0
    for s, l in zip(singles, lam):
        _, r = s.step1(l, iters)
        loop_s += r.elapsed_ms * 1e-3
    out["sequential_wall_s"] = time.perf_counter() - t
    out["sequential_channel_iters_per_s"] = count * iters / loop_s
    out["speedup_loop_batched"] = out["batched_channel_iters_per_s"] / out["sequential_channel_iters_per_s"]
    out["workload"] = (f"{count} frequency channels 350-1050 MHz, sizes drawn from "
                       f"{'/'.join(str(x) for x in sizes)}, 64 antennas 4 h at 120 s, cut 15%, positivity on")
    return out


def frequency_bench(torch, dev, count=64, iters=500, workers=16, nu_lo=350.0, nu_hi=1050.0):
    """One sky, the 4096^2 workload's, observed in `count` frequency channels
    across nu_lo-nu_hi MHz with the same array: channel c's baselines scale
    with nu_c, so its longest one lands at (nu_c / nu_hi) P/4 cells and its
    cut (15 %) is taken from that radius.  Both steps batched (`iters`
    iterations each, i_L from the batched step 1) against the channels solved
    one after the other by one context of the same size."""
    import synth
    from paper_2406_18356_amd import Batch, Solver

    base = synth.preset("sky4096")
    cfgs = [base.replace(uv_fill=0.25 * (nu_lo + (nu_hi - nu_lo) * c / max(count - 1, 1)) / nu_hi)
            for c in range(count)]
    t = time.perf_counter()
    prs = synth.make_problems(cfgs, workers=workers,
                              progress=lambda i, p: log(f"frequency channels: {i} generated, "
                                                        f"{time.perf_counter() - t:.0f} s"))
    gen_s = time.perf_counter() - t
    n = base.n
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)  # noqa: E731
    b = Batch([n] * count, positivity=True)
    for pr, ch in zip(prs, b.channels):
        ch.set_dirty_psf(1, T(pr.dirty_L), T(pr.psf_L))
        dh = T(pr.dirty_H)
        ch.set_dirty_psf(2, dh, T(pr.psf_H))
        sig2 = ch.estimate_sigma2(dh)
        ch.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
    b.autotune(reps=5)
    out = {"channels": count, "n": n, "iters": iters, "generate_s": gen_s,
           "workspace_gib": b.workspace_bytes / 2**30}
    lam1 = [ch.default_lambda(1, 1, 0.05) for ch in b.channels]
    b.solve(1, lam1, iters, image=True)  # theta, graph capture
    torch.cuda.synchronize()
    _, imgs, r1 = b.solve(1, lam1, iters, image=True)
    low = [im.contiguous() for im in imgs]
    lam2 = [ch.default_lambda(2, 1, 0.05) for ch in b.channels]
    b.solve(2, lam2, iters, low_res=low)
    torch.cuda.synchronize()
    _, r2 = b.solve(2, lam2, iters, low_res=low)
    out["batched_step1_channel_iters_per_s"] = count * iters / (r1[0].elapsed_ms * 1e-3)
    out["batched_step2_channel_iters_per_s"] = count * iters / (r2[0].elapsed_ms * 1e-3)
    log(f"frequency channels: batched step 1 {r1[0].elapsed_ms / iters * 1e3:.1f} us, "
        f"step 2 {r2[0].elapsed_ms / iters * 1e3:.1f} us per iteration of all channels")
    # one context, the channels one after the other (iteration loops timed)
    s = Solver(n, positivity=True)
    ms1 = ms2 = 0.0
    for c, pr in enumerate(prs):
        s.set_dirty_psf(1, T(pr.dirty_L), T(pr.psf_L))
        dh = T(pr.dirty_H)
        s.set_dirty_psf(2, dh, T(pr.psf_H))
        sig2 = s.estimate_sigma2(dh)
        s.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
        if c == 0:
            s.autotune(reps=5)
        s.set_lipschitz(1, r1[c].theta)
        s.set_lipschitz(2, r2[c].theta)
        _, q1 = s.step1(lam1[c], iters)
        _, q2 = s.step2(lam2[c], low[c], iters)
        ms1 += q1.elapsed_ms
        ms2 += q2.elapsed_ms
        if (c + 1) % 16 == 0:
            log(f"frequency channels: {c + 1} solved one after the other")
    out["sequential_step1_channel_iters_per_s"] = count * iters / (ms1 * 1e-3)
    out["sequential_step2_channel_iters_per_s"] = count * iters / (ms2 * 1e-3)
    out["workload"] = (f"the 4096x4096 workload's sky in {count} frequency channels {nu_lo:g}-{nu_hi:g} MHz "
                       f"(197 antennas 8 h at 30 s, longest baseline and cut scaled with frequency, cut 15%), "
                       f"positivity on, {iters} iterations per step")
    return out


def unet_forward_roofline(n, base_width=32, levels=4):
    """The network's forward pass at n^2 against its per-layer roofline: each
    3x3 convolution takes the longer of its MFMA work (K padded to 32) at the
    dense bf16 peak and its HBM bytes (bf16 input, the decoder's upsampled
    half read at quarter resolution, bf16 output) at 8 TB/s; the pooling,
    head and input kernels their bytes.  Returns (mfma flops, bytes, seconds)."""
    from paper_2406_18356_amd import unet_layers

    lay = unet_layers(base_width, levels)
    lvl = [j for j in range(levels) for _ in (0, 1)] + [j for j in range(levels - 2, -1, -1) for _ in (0, 1)]
    flops = nbytes = secs = 0.0
    for i, ((ci, co, kpad), j) in enumerate(zip(lay, lvl)):
        P = (n * n) >> (2 * j)
        fl = 2.0 * P * co * kpad
        dec_first = i >= 2 * levels and (i - 2 * levels) % 2 == 0
        inb = ((P // 4) * (ci - co) + P * co) * 2 if dec_first else P * ci * 2
        b = inb + P * co * 2
        flops, nbytes = flops + fl, nbytes + b
        secs += max(fl / (BF16_MFMA_TFLOPS * 1e12), b / (HBM_PEAK_GBS * 1e9))
    for j in range(levels - 1):  # 2x2 pooling
        P, C = (n * n) >> (2 * j), base_width << j
        b = P * C * 2 + (P // 4) * C * 2
        nbytes, secs = nbytes + b, secs + b / (HBM_PEAK_GBS * 1e9)
    b = n * n * (base_width * 2 + 4 + 2 * 4 + 8 * 2)  # head (bf16 in, float out); inputs (float in, bf16 out)
    return flops, nbytes + b, secs + b / (HBM_PEAK_GBS * 1e9)


def pipeline_bench(torch, dev, count=16, iters=500, seed=5, sizes=(1024, 2048, 4096, 8192), horizon=24000,
                   every=500, workers=16):
    """The whole method on the frequency channels of one observation with
    uneven image sizes up to 8192^2: `count` channels with sizes drawn from
    `sizes` (the seed gives at least one of the largest), 512 antennas 4 h at
    10 s, cut 10 %, positivity on.  Step 1 batched (`iters` iterations), each
    channel's low-resolution image, sigma2_hat and filters, the packaged
    network's prediction of each channel's step-2 image, then step 2 batched
    from zero and from the predictions (`iters` iterations each; FP32).  On
    the first channel of the largest size, step 2's time to 1e-5 and 1e-6
    relative objectives from both starts, read off trajectories of `horizon`
    iterations (F_ref: the lower of the two runs' lowest objectives)."""
    import synth
    from paper_2406_18356_amd import Batch, UNet, warmstart as ws

    cfgs = synth.channel_set(count, sizes=sizes, seed=seed, cut=0.10, n_ant=512, hours=4.0, dt_s=10.0)
    if not any(c.n == max(sizes) for c in cfgs):
        raise ValueError(f"seed {seed} draws no channel of {max(sizes)}^2")
    t = time.perf_counter()
    prs = synth.make_problems(cfgs, workers=workers, verbose=True,
                              progress=lambda i, p: log(f"pipeline: channel {i} ({p.n}^2) generated, "
                                                        f"{time.perf_counter() - t:.0f} s"))
    gen_s = time.perf_counter() - t
    sz = [int(p.n) for p in prs]
    log(f"pipeline: {count} channels {sz} generated in {gen_s:.1f} s")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)  # noqa: E731
    b = Batch(sz, positivity=True)
    dhs = []
    for pr, ch in zip(prs, b.channels):
        ch.set_dirty_psf(1, T(pr.dirty_L), T(pr.psf_L))
        dh = T(pr.dirty_H)
        ch.set_dirty_psf(2, dh, T(pr.psf_H))
        sig2 = ch.estimate_sigma2(dh)
        ch.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
        dhs.append(dh)
    b.autotune(reps=5)
    out = {"channels": count, "sizes": sz, "iters": iters, "generate_s": gen_s,
           "workspace_gib": b.workspace_bytes / 2**30}
    # step 1, then each channel's low-resolution image
    lam1 = [ch.default_lambda(1, 1, 0.05) for ch in b.channels]
    b.solve(1, lam1, iters, image=True)  # theta, graph capture
    torch.cuda.synchronize()
    _, imgs, res1 = b.solve(1, lam1, iters, image=True)
    out["step1_channel_iters_per_s"] = count * iters / (res1[0].elapsed_ms * 1e-3)
    log(f"pipeline: step 1 {res1[0].elapsed_ms / iters * 1e3:.1f} us per iteration of all channels")
    low = [im.contiguous() for im in imgs]
    lam2 = [ch.default_lambda(2, 1, 0.05) for ch in b.channels]
    # the network's prediction of every channel (one network per image size)
    params, meta = ws.load_weights()
    x_net, fwd_ms = [None] * count, [0.0] * count
    for n in sorted(set(sz)):
        net = UNet(1, n)
        net.set_params(params)
        for c in range(count):
            if sz[c] == n:
                x, ms = ws.timed_forward(net, dhs[c][None].contiguous(), low[c][None].contiguous())
                x_net[c], fwd_ms[c] = x[0].contiguous(), ms
        del net
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        log(f"pipeline: network predictions at {n}^2 done")
    out["network_forward_ms"] = fwd_ms
    # step 2 from zero and from the predictions
    b.solve(2, lam2, iters, low_res=low)  # theta, graph capture
    torch.cuda.synchronize()
    m_cold, r_cold = b.solve(2, lam2, iters, low_res=low)
    m_warm, r_warm = b.solve(2, lam2, iters, low_res=low, x0=x_net)
    out["step2_channel_iters_per_s"] = count * iters / (r_cold[0].elapsed_ms * 1e-3)
    out["step2_warm_channel_iters_per_s"] = count * iters / (r_warm[0].elapsed_ms * 1e-3)
    log(f"pipeline: step 2 {r_cold[0].elapsed_ms / iters * 1e3:.1f} us per iteration of all channels")
    per = []
    for c, ch in enumerate(b.channels):
        f0 = ch.objective(2, lam2[c], torch.zeros_like(low[c]), low[c])[0]
        fn = ch.objective(2, lam2[c], x_net[c], low[c])[0]
        per.append({"n": sz[c], "F_cold_at_K": r_cold[c].objective, "F_warm_at_K": r_warm[c].objective,
                    "warm_minus_cold_rel": (r_warm[c].objective - r_cold[c].objective) / abs(r_cold[c].objective),
                    "F_zero": f0, "F_network": fn})
    out["per_channel"] = per
    # time to tolerance on the first channel of the largest size
    c8 = sz.index(max(sizes))
    ch = b.channels[c8]
    ch.set_lipschitz(2, r_cold[c8].theta)
    trajs = {}
    for name, x0 in (("cold", None), ("network", x_net[c8])):
        trajs[name] = ws.trajectory(ch, lam2[c8], low[c8], x0=x0, iters=horizon, every=every)
        log(f"pipeline: {sz[c8]}^2 trajectory from {name} done, F = {trajs[name]['F'][-1]:.12g}")
    f_ref = min(min(t_["F"]) for t_ in trajs.values())
    ttt = {"channel": c8, "n": sz[c8], "horizon": horizon, "every": every, "f_ref": f_ref,
           "ms_per_iter": trajs["cold"]["ms"][-1] / trajs["cold"]["k"][-1]}
    for name, warm_ms in (("cold", 0.0), ("network", fwd_ms[c8])):
        ttt[name] = {f"{tol:g}": ws.crossing(trajs[name], f_ref, tol, warm_ms) for tol in (1e-6, 1e-5)}
    out["time_to_tol"] = ttt
    out["workload"] = (f"{count} frequency channels 350-1050 MHz, sizes drawn from "
                       f"{'/'.join(str(x) for x in sizes)} (seed {seed}), 512 antennas 4 h at 10 s, cut 10%, "
                       f"positivity on; {iters} iterations per step batched; the packaged 1024^2-trained "
                       f"network as the step-2 start")
    return out


def batch_replicas(torch, pr, tensors, iL, count, iters=20):
    """`count` copies of the workload's problem as the channels of one batch
    (the kernels' work does not depend on the data, so this measures the
    batched path at the full size; the channels are identical, not the
    frequency-scaled coverages of a real observation): both steps, `iters`
    iterations each, after a first call that captures the graph."""
    from paper_2406_18356_amd import Batch

    dL, pL, dH, pH = tensors
    b = Batch([pr.n] * count, positivity=True)
    for ch in b.channels:
        ch.set_dirty_psf(1, dL, pL)
        ch.set_dirty_psf(2, dH, pH)
        sig2 = ch.estimate_sigma2(dH)
        ch.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
    b.autotune(reps=5)
    ch0 = b.channels[0]
    lam = {1: [ch0.default_lambda(1, 1, 0.05)] * count, 2: [ch0.default_lambda(2, 1, 0.05)] * count}
    out = {"channels": count, "image": pr.n, "iters": iters,
           "workload": f"{count} identical channels of the {pr.n}x{pr.n} problem in one batch, positivity on"}
    for step in (1, 2):
        low = None if step == 1 else [iL] * count
        b.solve(step, lam[step], iters, low_res=low)  # theta and graph capture
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, res = b.solve(step, lam[step], iters, low_res=low)
        wall = time.perf_counter() - t
        loop = res[0].elapsed_ms * 1e-3
        out[f"step{step}"] = {"channel_iters_per_s": count * iters / loop, "loop_ms": loop * 1e3, "wall_s": wall}
    del b
    torch.cuda.empty_cache()
    return out


def train_warm_start(torch, n=256, ntrain=256, epochs=20, iters2=3000, neval=4, seed=11):
    """Trains the learned warm start on two-step results of skies observed like
    the benchmark workload (same array and track, sky density and cut) at
    n x n, and measures step-2 time to a 1e-6 relative objective from zero
    and from the network's prediction on held-out skies.  Returns (trained
    parameters, report)."""
    import synth
    from synth.generator import SkyConfig
    from paper_2406_18356_amd import Solver, UNet, unet_init_params, warmstart as ws

    dev = torch.device("cuda:0")
    f = (n / 4096) ** 2
    cfg = synth.preset("sky4096").replace(n=n, sky=SkyConfig(max(2, int(8000 * f)), max(1, int(200 * f))), seed=seed)
    t0 = time.perf_counter()
    base = synth.make_problem(cfg, with_full=False)
    train_p, eval_p = synth.sky_set(base, ntrain, 100), synth.sky_set(base, neval, 200)
    t1 = time.perf_counter()
    dh, il, b2, _ = ws.solve_pairs(train_p, iters2=iters2)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    net = UNet(8, n)
    net.set_params(unet_init_params(seed=0))
    losses = ws.train(net, dh, il, b2, epochs=epochs, batch=8, lr=1e-3)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    params = net.get_params()
    del net, dh, il, b2
    edh, eil, _, elam = ws.solve_pairs(eval_p, iters2=1)
    net1 = UNet(1, n)
    net1.set_params(params)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)  # noqa: E731
    evals = []
    for i, p in enumerate(eval_p):
        s = Solver(n, positivity=True)
        s.set_dirty_psf(1, T(p.dirty_L), T(p.psf_L))
        s.set_dirty_psf(2, T(p.dirty_H), T(p.psf_H))
        sig2 = s.estimate_sigma2(edh[i])
        s.set_filters(p.ell, p.delta, sig2, 1e-3 * sig2)
        _, rref = s.step2(elam[i], eil[i], 20000)
        fstar = rref.objective
        cold = ws.time_to_tol(s, elam[i], eil[i], fstar)
        x0, fms = ws.timed_forward(net1, edh[i:i + 1].contiguous(), eil[i:i + 1].contiguous())
        warm = ws.time_to_tol(s, elam[i], eil[i], fstar, x0=x0[0].contiguous(), warm_ms=fms)
        g0 = s.objective(2, elam[i], torch.zeros_like(edh[i]), eil[i])[0]
        gw = s.objective(2, elam[i], x0[0].contiguous(), eil[i])[0]
        evals.append({"cold": cold, "unet_warm": warm, "initial_gap_cold": (g0 - fstar) / abs(fstar),
                      "initial_gap_unet": (gw - fstar) / abs(fstar)})
    report = {
        "train": {"image": n, "pairs": ntrain, "target_iters": iters2, "epochs": epochs, "batch": 8,
                  "loss_first_epoch": losses[0], "loss_last_epoch": losses[-1],
                  "generate_s": t1 - t0, "solve_pairs_s": t2 - t1, "train_s": t3 - t2},
        "eval_held_out": evals,
    }
    return params, report


def psnr_study(torch, cycles=5, iters=100):
    """A synthetic analogue of the paper's partition study and single-step
    comparison (Sect. 5.1, 5.3): one 512^2 sky observed by 64 antennas for 4 h
    at 120 s, reconstructed by the two-step method for each partition
    (ell, delta) in {20, 35, 55} x {1, 3, 5} (cells of a 512 grid; doubled on
    the 1024 grid used here) with `cycles` major cycles of `iters` FISTA
    iterations per step, and by the single-step method on all visibilities.
    PSNR = 20 log10(max|sky| / RMSE) against the true sky."""
    import synth
    from paper_2406_18356_amd import multistep

    def psnr(img, truth):
        rmse = float(np.sqrt(np.mean((img - truth) ** 2)))
        return 20.0 * np.log10(float(np.max(np.abs(truth))) / rmse)

    base = synth.preset("paper512")
    rows = []
    single = None
    for ell in (20, 35, 55):
        for delta in (1, 3, 5):
            cfg = base.replace(cut=ell / 128.0, delta=2.0 * delta)
            pr = synth.make_problem(cfg, with_full=single is None)
            if single is None:
                img1, rep1 = multistep.single_step(pr.dirty_full, pr.psf_full, pr.n, cycles, iters)
                single = {"psnr": psnr(img1.cpu().numpy(), pr.sky), "psnr_model": psnr(rep1["model"].cpu().numpy(),
                          pr.sky), "ms": rep1["ms"], "dirty_psnr": psnr(pr.dirty_full, pr.sky)}
            row = {"ell": ell, "delta": delta, "V_L": int(pr.counts["V_L"]), "V_H": int(pr.counts["V_H"]),
                   "V_LH": int(pr.counts["V_LH"])}
            for tag, ratio, coarse in (("", 1e-3, None), ("_eta2_eq_sigma2", 1.0, None),
                                       ("_eta2_eq_sigma2_low_res_n2", 1.0, 2)):
                lo = None
                if coarse:
                    _, dirty_s, psf_s = synth.coarse_low(pr, coarse)
                    lo = (coarse, dirty_s, psf_s)
                img, _, rep = multistep.two_step(pr, cycles, iters, eta_ratio=ratio, coarse=lo)
                row["psnr" + tag] = psnr(img.cpu().numpy(), pr.sky)
                row["psnr_model" + tag] = psnr(rep["model"].cpu().numpy(), pr.sky)
                row["ms" + tag] = rep["step1_ms"] + rep["step2_ms"]
            rows.append(row)
            log(f"partition study: ell {ell} delta {delta} done")
    return {"workload": "paper-shaped 512^2 sky, 64 antennas 4 h at 120 s, natural weighting, "
                        f"{cycles} major cycles x {iters} FISTA iterations per step, positivity on; "
                        "two-step with eta2 = 1e-3 sigma2_hat (the paper's estimate) and with eta2 = sigma2_hat; "
                        "_low_res_n2: step 1 on the 256^2 grid (the down-sampled low-resolution image of Sect. 6.1, "
                        "a quarter of the secondary data product) and step 2 on its up-sampling",
            "single_step": single, "two_step": rows}


def dictionary_bench(torch, pr, tensors, iters=50):
    """The paper's dictionary (db1-db8 concatenation, Sect. 3, App. A.1) on the
    same workload: FISTA on the 8 N^2 wavelet coefficients, positivity off
    (no closed-form prox with the dictionary).  Loop rates of both steps and
    the two wavelet passes of an iteration against the HBM roofline."""
    from paper_2406_18356_amd import Solver

    dL, pL, dH, pH = tensors
    s = Solver(pr.n, pad=2, positivity=False, prune_tol=1e-6, dictionary=1)
    s.set_dirty_psf(1, dL, pL)
    s.set_dirty_psf(2, dH, pH)
    sig2 = s.estimate_sigma2(dH)
    s.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
    s.autotune(reps=10)
    s.lipschitz(1)
    s.lipschitz(2)
    lam1, lam2 = s.default_lambda(1, 1, 0.05), s.default_lambda(2, 1, 0.05)
    s.step1(lam1, 2)  # warm
    b1, iL, r1 = s.step1(lam1, iters, image=True)
    b2, r2 = s.step2(lam2, iL, iters)
    passes = {}
    for which, name in ((4, "synthesis"), (5, "analysis_update")):
        ms, by, fl = s.time_pass(which, reps=10, step=1)
        passes[name] = {"ms": ms, "bytes": by, "flops": fl, "gbs": by / (ms * 1e-3) / 1e9,
                        "hbm_frac": by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    out = {"workload": f"the same {pr.n}x{pr.n} two-step problem, W = db1-db8 (8 x {pr.n}^2 coefficients), "
                       f"{iters} FISTA iterations per step, positivity off",
           "step1_loop_iters_per_s": r1.iters / (r1.elapsed_ms * 1e-3),
           "step2_loop_iters_per_s": r2.iters / (r2.elapsed_ms * 1e-3),
           "step1_F": r1.objective, "step2_F": r2.objective, "passes": passes}
    del s
    torch.cuda.empty_cache()
    return out


def upsample_bench(torch, s, n, factors=(2, 4), reps=5):
    """msr_upsample (the down-sampled low-resolution image, Sect. 6.1) at the
    workload size: wall time per call (the call synchronises) and its FMA
    rate against the FP32 peaks (2 N m^2 + 2 N^2 m flops, m = N / d)."""
    out = {}
    dev = torch.device("cuda:0")
    for d in factors:
        m = n // d
        small = torch.randn((m, m), generator=torch.Generator().manual_seed(d), dtype=torch.float32).to(dev)
        s.upsample(small, d)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            s.upsample(small, d)
        ms = (time.perf_counter() - t) / reps * 1e3
        fl = 2.0 * n * m * m + 2.0 * n * n * m
        tf = fl / (ms * 1e-3) / 1e12
        out[f"d{d}"] = {"ms": ms, "tflops": tf, "frac_of_published_fp32_peak": tf / FP32_PUBLISHED_TFLOPS,
                        "frac_of_unpacked_fma_peak": tf / FP32_VECTOR_TFLOPS}
    return out


def cpu_baseline(pr, budget_s=8.0):
    """The oracle on this host (bounded samples): step-1 FISTA iterations of the
    workload in FP64 and, with the oracle's dtype switch, in float32; and the
    whole 256^2 two-step workload (200 iterations per step) end to end in FP64."""
    from oracle import objectives, fista, twostep
    from oracle.conv import WORKERS
    import synth

    lam = 0.05 * float(np.linalg.norm(pr.dirty_L))
    rates = {}
    for name, dt in (("f64", np.float64), ("f32", np.float32)):
        s1 = objectives.Step1(pr.dirty_L, pr.psf_L, dtype=dt)
        theta = 2.0 * float(np.max(np.abs(s1.H.h)) ** 2)  # a valid upper bound; the rate does not depend on it
        x = np.zeros((pr.n, pr.n), dt)
        fista.fista(s1.grad, x, 1.0 / theta, lam, 1, positivity=True, dtype=dt)  # warm-up
        k, t0 = 0, time.perf_counter()
        while True:
            fista.fista(s1.grad, x, 1.0 / theta, lam, 1, positivity=True, dtype=dt)
            k += 1
            el = time.perf_counter() - t0
            if el >= budget_s or k >= 50:
                break
        rates[name] = (k / el, k, el)
        del s1
    small = synth.make_problem(synth.preset("small256"))
    t0 = time.perf_counter()
    twostep.two_step(small.dirty_L, small.psf_L, small.dirty_H, small.psf_H, small.ell, small.delta,
                     small.cfg.iters, small.cfg.iters, positivity=True)
    c1 = time.perf_counter() - t0
    return {
        "value": rates["f64"][0], "unit": "FISTA iters/s", "cores": WORKERS, "kind": "oracle",
        "sample": f"{rates['f64'][1]} step-1 FISTA iterations of the same {pr.n}x{pr.n} workload (FP64 NumPy/SciPy "
                  f"oracle, scipy.fft with {WORKERS} workers), {rates['f64'][2]:.1f} s",
        "f32_value": rates["f32"][0],
        "f32_sample": f"{rates['f32'][1]} step-1 iterations with the oracle in float32, {rates['f32'][2]:.1f} s",
        "two_step_256_s": c1,
        "two_step_256_sample": "the 256x256 two-step workload end to end (power iterations, 200 FISTA iterations "
                               "per step, i_L, sigma2_hat), FP64 oracle",
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--size", type=int, default=4096, choices=sorted(WORKLOADS))
    ap.add_argument("--iters", type=int, default=None, help="FISTA iterations per step (default: the workload's)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ttt", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-unet", action="store_true")
    ap.add_argument("--no-psnr", action="store_true")
    ap.add_argument("--psnr-iters", type=int, default=100,
                    help="FISTA iterations per major cycle and step in the partition study")
    ap.add_argument("--psnr-only", action="store_true", help="run only the partition study and print it")
    ap.add_argument("--frequency-channels", type=int, default=0, metavar="C",
                    help="run only the 4096^2 workload's sky in C frequency channels (batched against one after "
                         "the other) and print it")
    ap.add_argument("--pipeline", action="store_true",
                    help="run only the whole method on 16 channels of uneven sizes up to 8192^2 (512 antennas, "
                         "4 h at 10 s, cut 10%%) with the network's warm start, and print it")
    ap.add_argument("--no-dict", action="store_true")
    ap.add_argument("--batch-channels", type=int, default=8)
    ap.add_argument("--batch-sizes", type=int, nargs="+", default=[512, 1024, 2048, 4096],
                    help="image sizes the batch's channels are drawn from")
    ap.add_argument("--batch-replicas", type=int, default=0, metavar="C",
                    help="also batch C copies of the workload's problem (about 1.5 GiB of HBM each at 4096^2)")
    ap.add_argument("--ttt-horizon", type=int, default=24000,
                    help="step-2 iterations of every time-to-tolerance run")
    ap.add_argument("--ttt-every", type=int, default=500, help="iterations between recorded objectives")
    ap.add_argument("--ttt-momentum-k", type=int, default=3000,
                    help="momentum index at which the 'entered' runs join Algorithm 1")
    ap.add_argument("--profile-pass", type=int, nargs=3, action="append", default=None,
                    metavar=("STEP", "WHICH", "REPS"),
                    help="profiling aid (repeatable): after setup, for each triple run one 64 MiB device "
                         "copy (counter calibration and trace marker) and msr_time_pass(STEP, WHICH, REPS), "
                         "then exit")
    ap.add_argument("--kernels-only", type=int, default=0, metavar="K",
                    help="profiling aid: set up the workload, autotune, run K iterations of each step and exit")
    ap.add_argument("--unet-train", type=int, default=0, metavar="K",
                    help="with --unet-forward: also run K training steps of the network on this workload")
    ap.add_argument("--unet-forward", type=int, default=0, metavar="K",
                    help="only run K forward passes of the warm-start network (random weights) on this workload's "
                         "image size, for a kernel trace, and exit")
    ap.add_argument("--dictionary-kernels", type=int, default=0, metavar="K",
                    help="profiling aid: set up the workload with the wavelet dictionary, run K iterations of "
                         "each step and exit")
    args = ap.parse_args(argv)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the solver runs on one GPU; --gpus must be 1 (a multi-GPU split of the "
              "channels or of the image is not implemented)", file=sys.stderr)
        return 2

    import torch
    import synth
    from paper_2406_18356_amd import Solver

    if args.frequency_channels:
        rep = frequency_bench(torch, torch.device("cuda:0"), count=args.frequency_channels)
        print(json.dumps({"frequency_channels": rep}), flush=True)
        return 0

    if args.pipeline:
        rep = pipeline_bench(torch, torch.device("cuda:0"), horizon=args.ttt_horizon, every=args.ttt_every)
        print(json.dumps({"pipeline": rep}), flush=True)
        return 0

    if args.psnr_only:
        t = time.perf_counter()
        rep = psnr_study(torch, iters=args.psnr_iters)
        rep["wall_s"] = time.perf_counter() - t
        print(json.dumps({"partition_study": rep}), flush=True)
        return 0

    preset, desc = WORKLOADS[args.size]
    cfg = synth.preset(preset)
    iters = args.iters or cfg.iters
    t = time.perf_counter()
    pr = synth.make_problem(cfg, with_full=False, progress=lambda msg: log(f"workload {preset}: {msg}"))
    log(f"workload {preset}: generated in {time.perf_counter() - t:.1f} s; counts {pr.counts}")
    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)  # noqa: E731
    tensors = (T(pr.dirty_L), T(pr.psf_L), T(pr.dirty_H), T(pr.psf_H))
    s = Solver(pr.n, pad=2, positivity=True, prune_tol=1e-6)
    s.set_dirty_psf(1, tensors[0], tensors[1])
    s.set_dirty_psf(2, tensors[2], tensors[3])
    sig2 = s.estimate_sigma2(tensors[2])
    s.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)  # so that the low-band filter pass is tuned too
    if args.unet_forward:
        # weights and inputs only set the values, not the work: random weights,
        # the long-baseline dirty image and the short-baseline one as the
        # low-resolution input
        from paper_2406_18356_amd import UNet, unet_init_params

        net = UNet(1, pr.n)
        net.set_params(unet_init_params(seed=0))
        dh1, il1 = tensors[2][None].contiguous(), tensors[0][None].contiguous()
        net.forward(dh1, il1)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.unet_forward):
            net.forward(dh1, il1)
        torch.cuda.synchronize()
        log(f"unet forward {pr.n}^2: {(time.perf_counter() - t) / args.unet_forward * 1e3:.2f} ms")
        if args.unet_train:
            # training steps (forward, loss, backward, Adam) with the
            # short-baseline dirty image standing in for the target
            tg1 = tensors[0][None].contiguous()
            net.train_step(dh1, il1, tg1)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(args.unet_train):
                net.train_step(dh1, il1, tg1)
            torch.cuda.synchronize()
            log(f"unet training step {pr.n}^2: {(time.perf_counter() - t) / args.unet_train * 1e3:.2f} ms")
        return 0
    if args.dictionary_kernels:
        rep = dictionary_bench(torch, pr, tensors, iters=args.dictionary_kernels)
        log("dictionary kernels:", json.dumps(rep))
        return 0
    tuned = s.autotune(reps=20)
    log("autotune (row variant, column variant, {variant: (col ms, row ms)}):", tuned)
    torch.cuda.synchronize()
    if args.profile_pass:
        s.lipschitz(1)
        b1, iL, _ = s.step1(s.default_lambda(1, 1, 0.05), 10, image=True)
        sig2 = s.estimate_sigma2(tensors[2])
        s.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
        s.lipschitz(2)
        s.step2(s.default_lambda(2, 1, 0.05), iL, 10)
        src = torch.empty(16 * 1024 * 1024, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for step, which, reps in args.profile_pass:
            # a 64 MiB device copy before each pass: counter calibration, and a
            # marker that separates the passes in a kernel trace
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
            ms, by, fl = s.time_pass(which, reps=reps, step=step)
            torch.cuda.synchronize()
            log(f"profile-pass step {step} which {which}: {ms * 1e3:.2f} us, {by:.0f} bytes, {fl:.0f} flops")
        return 0
    if args.kernels_only:
        s.lipschitz(1)
        b1, iL, r1 = s.step1(s.default_lambda(1, 1, 0.05), args.kernels_only, image=True)
        sig2 = s.estimate_sigma2(tensors[2])
        s.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
        s.lipschitz(2)
        b2, r2 = s.step2(s.default_lambda(2, 1, 0.05), iL, args.kernels_only)
        torch.cuda.synchronize()
        log(f"kernels-only: step1 {r1.elapsed_ms / max(r1.iters, 1) * 1e3:.1f} us/it, "
            f"step2 {r2.elapsed_ms / max(r2.iters, 1) * 1e3:.1f} us/it")
        return 0

    for w in range(args.warmup):
        two_step(s, dev, tensors, pr, iters, torch)
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    for k in range(args.steps):
        res = two_step(s, dev, tensors, pr, iters, torch)
        log(f"step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    r1, r2, iL, lam2, b1 = res
    total_iters = args.steps * 2 * iters
    value = total_iters / el

    # Each pass of an iteration of both steps timed alone (HIP events on the
    # library's stream); the dominant one is the largest share of an iteration.
    # "ms" is the mean over 30 launches each between its own pair of events
    # (the duration of one dispatch, what a profiler's kernel trace reports);
    # "ms_back_to_back" the mean of 50 launches between one pair, where each
    # launch's first blocks start while the previous launch's last ones drain.
    per_iter = {(1, 0): 2, (1, 1): 1, (1, 2): 1, (2, 0): 2, (2, 1): 2, (2, 2): 1, (2, 3): 1}
    names = {0: "col_psf", 1: "row_resid", 2: "row_update", 3: "col_filter"}
    passes = {}
    for (step, which), cnt in per_iter.items():
        ms_b2b, by, fl = s.time_pass(which, reps=50, step=step)
        ms = sum(s.time_pass(which, reps=1, step=step)[0] for _ in range(30)) / 30
        passes[f"{names[which]}_step{step}"] = {
            "ms": ms, "ms_back_to_back": ms_b2b, "bytes": by, "flops": fl, "per_iter": cnt,
            "gbs": by / (ms * 1e-3) / 1e9, "tflops": fl / (ms * 1e-3) / 1e12,
        }
    dom = max(passes, key=lambda k: passes[k]["ms"] * passes[k]["per_iter"])
    d = passes[dom]
    hbm_frac = d["gbs"] / HBM_PEAK_GBS
    traffic = None
    try:
        from paper_2406_18356_amd.prof_summary import kernel_source_hash

        rec = json.load(open(traffic_file(dom, preset)))
        if rec["source_sha256"] == kernel_source_hash():
            traffic = rec["traffic_bytes"]
    except (OSError, ValueError, KeyError):
        traffic = None
    # Per iteration: the algorithmic bytes of all passes of one iteration of a
    # step (pruned spectral columns: only the kept columns are counted) over
    # the loop's measured time per iteration.
    per_iteration = {}
    for step, r in ((1, r1), (2, r2)):
        us = r.elapsed_ms / max(r.iters, 1) * 1e3
        by = sum(v["bytes"] * v["per_iter"] for k, v in passes.items() if k.endswith(f"step{step}"))
        fl = sum(v["flops"] * v["per_iter"] for k, v in passes.items() if k.endswith(f"step{step}"))
        per_iteration[f"step{step}"] = {"us": us, "algorithmic_bytes": by, "hbm_gbs": by / (us * 1e-6) / 1e9,
                                        "hbm_frac": by / (us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                                        "fp32_tflops": fl / (us * 1e-6) / 1e12}
    roofline = {"bound": "hbm", "kernel": dom, "achieved": d["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": hbm_frac, "traffic": traffic, "algorithmic_bytes": d["bytes"],
                "algorithmic_flops": d["flops"], "launch_ms": d["ms"], "launch_ms_back_to_back": d["ms_back_to_back"],
                "fp32": {"tflops": d["tflops"], "frac_of_published_peak": d["tflops"] / FP32_PUBLISHED_TFLOPS,
                         "published_peak": FP32_PUBLISHED_TFLOPS,
                         "frac_of_unpacked_fma_peak": d["tflops"] / FP32_VECTOR_TFLOPS,
                         "unpacked_fma_peak": FP32_VECTOR_TFLOPS},
                "per_iteration": per_iteration}
    log("passes:", json.dumps(passes))

    unet_report, unet_params = None, None
    if not args.no_unet and not args.no_ttt:
        from paper_2406_18356_amd import warmstart as ws

        # the network trained at 1024^2 on converged method-generated pairs and
        # stored with the package; without that file, a small one trained here
        unet_params, meta = ws.load_weights()
        if unet_params is not None:
            unet_report = {"source": "paper_2406_18356_amd/weights/unet_w32_l4_1024.bf16", **meta}
        else:
            unet_params, unet_report = train_warm_start(torch)
        log("learned warm start:", json.dumps(unet_report)[:400])

    ttt = None
    if not args.no_ttt:
        # Step 2 from each start for a fixed horizon, the exact objective
        # recorded every `every` iterations.  Starts: zero (cold), the
        # low-resolution image and the network's prediction, each restarted at
        # k = 1 (Algorithm 1) and entered at momentum index K0 with zero
        # velocity.  The reference F_ref is the lowest objective any run
        # reaches; the time to a tolerance is read off each trajectory.  The
        # FP32 iteration stalls a few 1e-5 above the FP64 minimum on these
        # workloads, so tolerances are relative to what the FP32 path reaches.
        from paper_2406_18356_amd import UNet, warmstart as ws

        H, every, K0 = args.ttt_horizon, args.ttt_every, args.ttt_momentum_k
        starts = {"cold": (None, 0.0), "low_res": (iL, 0.0)}
        if unet_params is not None:
            net = UNet(1, pr.n)
            net.set_params(unet_params)
            x0, fms = ws.timed_forward(net, tensors[2][None].contiguous(), iL[None].contiguous())
            starts["unet"] = (x0[0].contiguous(), fms)
        trajs = {}
        for name, (x0, _) in starts.items():
            for suffix, mk in (("", 0), (f"_momentum_{K0}", K0)):
                trajs[name + suffix] = ws.trajectory(s, lam2, iL, x0=x0, iters=H, every=every, momentum_k=mk)
                log(f"time to tolerance: {name + suffix} done, F = {trajs[name + suffix]['F'][-1]:.12g}")
        # The cold start with float64 iterates (float32 transforms,
        # iterate_precision 64): the FP32 runs stall a few 1e-5 above the
        # objective this one reaches, because their iterate is rounded to
        # float32 every iteration.
        s64 = Solver(pr.n, pad=2, positivity=True, prune_tol=1e-6, iterate_precision=64)
        s64.set_dirty_psf(1, tensors[0], tensors[1])
        s64.set_dirty_psf(2, tensors[2], tensors[3])
        sig2 = s64.estimate_sigma2(tensors[2])
        s64.set_filters(pr.ell, pr.delta, sig2, 1e-3 * sig2)
        s64.autotune(reps=10)
        s64.set_lipschitz(2, r2.theta)
        t64 = ws.trajectory(s64, lam2, iL, x0=None, iters=H, every=every)
        log(f"time to tolerance: cold_fp64_iterate done, F = {t64['F'][-1]:.12g}")
        del s64
        f_ref = min(min(t["F"]) for t in trajs.values())
        f_half = min(F for t in trajs.values() for k, F in zip(t["k"], t["F"]) if k <= H // 2)
        tols = (1e-6, 1e-5)
        ttt = {"tols": list(tols), "f_ref": f_ref, "horizon": H, "every": every, "momentum_k": K0,
               "f_ref_rule": "lowest exact objective of any run within the horizon",
               "f_ref_half_horizon_rel": (f_half - f_ref) / abs(f_ref),
               "ms_per_iter": trajs["cold"]["ms"][-1] / trajs["cold"]["k"][-1]}
        for name, t in trajs.items():
            base = name.split("_momentum")[0]
            x0 = starts[base][0]
            F0 = s.objective(2, lam2, x0 if x0 is not None else torch.zeros_like(iL), iL)[0]
            ttt[name] = {f"{tol:g}": ws.crossing(t, f_ref, tol, starts[base][1]) for tol in tols}
            # the same against the reference of half the horizon: how much the
            # metric depends on the reference run's length
            ttt[name].update({f"{tol:g}_half_horizon_ref": ws.crossing(t, f_half, tol, starts[base][1])
                              for tol in tols})
            ttt[name]["initial_rel_gap"] = (F0 - f_ref) / abs(f_ref)
        # the float64-iterate run against the lowest objective of every run
        f_all = min(f_ref, min(t64["F"]))
        ttt["cold_fp64_iterate"] = {f"{tol:g}": ws.crossing(t64, f_all, tol) for tol in tols}
        ttt["cold_fp64_iterate"]["ms_per_iter"] = t64["ms"][-1] / t64["k"][-1]
        ttt["f_ref_all_runs"] = f_all
        ttt["fp32_cold_best_gap_to_f_ref_all"] = (min(trajs["cold"]["F"]) - f_all) / abs(f_all)
        ttt["fp32_cold_vs_fp64_iterate_at_horizon"] = (trajs["cold"]["F"][-1] - t64["F"][-1]) / abs(t64["F"][-1])
        if "unet" in starts:
            # the network against the best non-learned start under the same entry rule
            gain = {}
            for tol in tols:
                for suffix in ("", f"_momentum_{K0}"):
                    plain = [ttt[x + suffix][f"{tol:g}"]["ms"] for x in ("cold", "low_res")]
                    plain = [v for v in plain if v >= 0]
                    u = ttt["unet" + suffix][f"{tol:g}"]["ms"]
                    key = f"{'restart_k1' if not suffix else f'entered_at_{K0}'}@{tol:g}"
                    gain[key] = 1.0 - u / min(plain) if plain and u > 0 else None
            ttt["unet_gain_over_best_plain_start"] = gain
            # the network's forward pass against the dense bf16 MFMA peak: the
            # MFMA work of every 3x3 convolution (K padded to 32) at its level
            from paper_2406_18356_amd import unet_layers

            lay = unet_layers(32, 4)
            lvl = [0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0]
            hw = pr.n * pr.n
            fl = sum(2.0 * (hw >> (2 * j)) * co * kpad for (ci, co, kpad), j in zip(lay, lvl))
            dh1, il1 = tensors[2][None].contiguous(), iL[None].contiguous()
            net.forward(dh1, il1)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                net.forward(dh1, il1)
            e1.record()
            e1.synchronize()
            fms5 = e0.elapsed_time(e1) / 5
            _, rb, rs = unet_forward_roofline(pr.n)
            ttt["unet_forward"] = {"image": pr.n, "ms": fms5, "mfma_tflops": fl / (fms5 * 1e-3) / 1e12,
                                   "mfma_frac": fl / (fms5 * 1e-3) / 1e12 / BF16_MFMA_TFLOPS,
                                   "roofline_ms": rs * 1e3, "roofline_bytes": rb,
                                   "frac_of_roofline": rs * 1e3 / fms5}
            del net
        log("time to tolerance:", json.dumps(ttt))

    # Per-PSF setup (PSF spectra and theta of both steps), which the time to
    # tolerance excludes, and the sanity ratio lambda_s / ||grad f_s(0)||_inf
    # (at or above 1 the minimiser is x = 0).
    torch.cuda.synchronize()
    t = time.perf_counter()
    s.set_dirty_psf(1, tensors[0], tensors[1])
    s.set_dirty_psf(2, tensors[2], tensors[3])
    s.set_filters(pr.ell, pr.delta, s.estimate_sigma2(tensors[2]), 1e-3 * s.estimate_sigma2(tensors[2]))
    th1, it1 = s.lipschitz(1)
    th2, it2 = s.lipschitz(2)
    torch.cuda.synchronize()
    setup = {"ms": (time.perf_counter() - t) * 1e3, "lanczos_applications": [it1, it2], "theta": [th1, th2]}
    zero = torch.zeros_like(tensors[0])
    g1 = float(s.gradient(1, zero).abs().max())
    g2 = float(s.gradient(2, zero, iL).abs().max())
    setup["lambda_over_grad0_inf"] = [s.default_lambda(1, 1, 0.05) / g1, lam2 / g2]
    log("setup:", json.dumps(setup))

    batch = None
    if not args.no_batch:
        batch = batch_bench(torch, dev, args.batch_channels, iters, sizes=tuple(args.batch_sizes))
        log("batch:", json.dumps(batch))

    dictionary = None
    if not args.no_dict:
        dictionary = dictionary_bench(torch, pr, tensors)
        log("dictionary:", json.dumps(dictionary))
    upsampling = upsample_bench(torch, s, pr.n)
    log("upsampling:", json.dumps(upsampling))

    replicas = None
    if args.batch_replicas:
        replicas = batch_replicas(torch, pr, tensors, iL, args.batch_replicas)
        log("batch replicas:", json.dumps(replicas))

    psnr = None
    if not args.no_psnr:
        psnr = psnr_study(torch, iters=args.psnr_iters)
        log("partition study:", json.dumps(psnr))

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(pr)
        log("cpu baseline:", json.dumps(cpu))

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "FISTA iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "image": pr.n, "grid": pr.P, "iters_per_step": iters,
                   "parallelism": "none (1 GPU)"},
        "step1_loop_iters_per_s": r1.iters / (r1.elapsed_ms * 1e-3),
        "step2_loop_iters_per_s": r2.iters / (r2.elapsed_ms * 1e-3),
        "autotune": {"row_variant": tuned[0], "col_variant": tuned[1]},
        "time_to_tol": ttt,
        "setup": setup,
        "learned_warm_start": unet_report,
        "batch": batch,
        "batch_replicas": replicas,
        "partition_study": psnr,
        "wavelet_dictionary": dictionary,
        "low_res_upsampling": upsampling,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
