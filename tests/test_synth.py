"""Generator checks: baseline counts, the partition identity of Table 1, Hermitian
grids and the PSF-peak normalisation."""
import os

import numpy as np
import pytest

import synth
from synth.generator import tiny, make_antennas, uv_tracks, _baselines, ArrayConfig

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_baseline_count_no_autocorrelations():
    arr = ArrayConfig(n_ant=17, hours=1.0, dt_s=600.0)
    xyz = make_antennas(arr, np.random.default_rng(0))
    assert _baselines(xyz).shape[0] == 17 * 16 // 2
    n_vis = sum(u.size for u, _ in uv_tracks(xyz, arr))
    assert n_vis == 17 * 16 // 2 * 6


def test_table1_identity_in_the_paper():
    """Table 1: every row has |V_L| + |V_H| - |V_LH| = 249600 = (64*65/2) * 120,
    i.e. samples in the overlap are counted in both sets (and the paper's
    count includes autocorrelations)."""
    rows = np.loadtxt(os.path.join(GOLD, "table1_partition_counts.txt"), comments="#")
    assert rows.shape == (9, 5)
    for ell, delta, vl, vh, vlh in rows:
        assert vl + vh - vlh == 249600
    assert 64 * 65 // 2 * 120 == 249600


def test_partition_identity_in_generator():
    pr = synth.make_problem(tiny(32))
    c = pr.counts
    assert c["V_L"] + c["V_H"] - c["V_LH"] == c["V"]
    assert c["V_LH"] > 0


def test_grids_hermitian_and_psf_normalised():
    pr = synth.make_problem(tiny(32))
    P = pr.P
    for w, psf in ((pr.w_L, pr.psf_L), (pr.w_H, pr.psf_H), (pr.w_full, pr.psf_full)):
        # w(k) = w(-k)
        neg = np.roll(np.flip(w, (0, 1)), 1, axis=(0, 1))
        np.testing.assert_array_equal(w, neg)
        assert psf[P // 2, P // 2] == pytest.approx(1.0, abs=1e-12)
        assert np.max(np.abs(psf)) <= 1.0 + 1e-12
        h = np.fft.fft2(np.fft.ifftshift(psf))
        assert np.max(np.abs(h.imag)) < 1e-9 * np.max(np.abs(h.real))
        assert np.min(h.real) > -1e-9 * np.max(h.real)
        # the spectrum is the normalised weight grid
        np.testing.assert_allclose(h.real, w * P * P / w.sum(), atol=1e-9 * np.max(h.real))


def test_uv_support_radius():
    pr = synth.make_problem(tiny(32))
    k = np.fft.fftfreq(pr.P) * pr.P
    r = np.sqrt(k[:, None] ** 2 + k[None, :] ** 2)
    assert r[pr.w_full > 0].max() <= pr.P / 4 + 1.0
    # the split grids respect the partition up to nearest-cell rounding
    assert r[pr.w_L > 0].max() <= pr.ell + pr.delta + 1.0
    assert r[pr.w_H > 0].min() >= pr.ell - pr.delta - 1.0


def test_seeded_reproducible():
    a = synth.make_problem(tiny(16, seed=3))
    b = synth.make_problem(tiny(16, seed=3))
    np.testing.assert_array_equal(a.dirty_H, b.dirty_H)
    c = synth.make_problem(tiny(16, seed=4))
    assert not np.array_equal(a.dirty_H, c.dirty_H)


def test_sky_set_does_not_depend_on_workers():
    """Member i of a sky set draws from the seed sequence [seed, i] alone, so
    the forked workers give the serial set exactly."""
    base = synth.make_problem(tiny(64, seed=3), with_full=False)
    a = synth.sky_set(base, 5, 1000)
    b = synth.sky_set(base, 5, 1000, workers=3)
    for x, y in zip(a, b):
        assert np.array_equal(x.sky, y.sky)
        assert np.array_equal(x.dirty_L, y.dirty_L) and np.array_equal(x.dirty_H, y.dirty_H)
    assert not np.array_equal(a[0].sky, a[1].sky)


def test_grid_weights_counts_every_visibility_and_its_conjugate():
    """The grids against a direct count: every sample (u, v) and its
    conjugate (-u, -v) add one to their nearest cells, for the full set and
    for the L and H splits, whatever the chunking of the baselines."""
    from synth.generator import grid_weights

    arr = ArrayConfig(n_ant=12, hours=2.0, dt_s=900.0)
    xyz = make_antennas(arr, np.random.default_rng(5))
    P, fill, ell, delta = 48, 0.25, 6.0, 2.0
    wf, wl, wh, counts = grid_weights(xyz, arr, P, fill, ell, delta)
    u = np.concatenate([a for a, _ in uv_tracks(xyz, arr, chunk=7)])
    v = np.concatenate([b for _, b in uv_tracks(xyz, arr, chunk=7)])
    scale = fill * P / np.sqrt(np.max(u * u + v * v))
    ref = {k: np.zeros((P, P)) for k in "flh"}
    for uu, vv in zip(u * scale, v * scale):
        r = np.hypot(uu, vv)
        iu, iv = int(np.rint(uu)), int(np.rint(vv))
        for k, keep in (("f", True), ("l", r <= ell + delta), ("h", r >= ell - delta)):
            if keep:
                ref[k][iv % P, iu % P] += 1
                ref[k][-iv % P, -iu % P] += 1
    np.testing.assert_array_equal(wf, ref["f"])
    np.testing.assert_array_equal(wl, ref["l"])
    np.testing.assert_array_equal(wh, ref["h"])
    assert counts["V"] == u.size and wf.sum() == 2 * u.size


def test_make_problems_does_not_depend_on_workers():
    cfgs = synth.channel_set(3, sizes=(16, 32), seed=2, n_ant=12, dt_s=1800.0)
    a = synth.make_problems(cfgs)
    b = synth.make_problems(cfgs, workers=3)
    for x, y, c in zip(a, b, cfgs):
        assert x.n == c.n
        assert np.array_equal(x.dirty_H, y.dirty_H) and np.array_equal(x.psf_L, y.psf_L)
