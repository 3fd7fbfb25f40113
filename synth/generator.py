"""Synthetic skies, arrays, uv coverage, PSFs and dirty images (NumPy, FP64).

Recipe (all draws from ``numpy.random.Generator(PCG64(seed))``):

* Sky.  Point sources on integer pixels, uniform over the image, flux
  log-uniform on [0.01, 1].  Elliptical Gaussians with both widths uniform on
  [2, 8] px (sorted so the minor width is the smaller), position angle uniform
  on [0, pi), peak log-uniform on [0.01, 1], centre uniform over the image,
  evaluated on pixel centres inside a +-4 sigma window and cut at the edges.
* Array.  Antennas at log-radial random positions (radius r_max*10^(-2U),
  azimuth uniform) in a local East/North plane at latitude -30.7 deg, tracking
  a source at declination -30 deg.  Baselines exclude autocorrelations.
  Earth-rotation (u, v) follow the standard relation between the equatorial
  baseline vector and the hour angle (Thompson, Moran & Swenson, eq. 4.1);
  w is ignored.
* Gridding.  The coordinates are scaled so that the longest sample lies at
  radius P/4 grid cells, every sample adds one count to its nearest cell
  (natural weighting) and its Hermitian partner adds one count at -k.
* Partition (Sect. 3.1 of the paper).  A sample belongs to the short-baseline
  set L when its radius is <= ell + delta, to the long-baseline set H when it
  is >= ell - delta; samples in the overlap are in both.  ell = cut * P/4 and
  delta = max(1, round(0.1 * ell)) cells.
* PSF of a set: the inverse DFT of its weight grid, scaled so the value at the
  phase centre (P/2, P/2) is exactly one.
* Dirty image of a set: the sky zero-embedded at offset (P-N)/2 in the P x P
  grid, transformed, multiplied by the set's normalised weight grid,
  transformed back and cropped, plus white Gaussian noise whose standard
  deviation is 1e-3 of the noiseless dirty image's peak (independent seeds
  per set).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import Optional

import numpy as np


# --------------------------------------------------------------------------
# configuration
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class SkyConfig:
    n_points: int = 20
    n_gauss: int = 3
    flux_lo: float = 0.01
    flux_hi: float = 1.0
    sigma_lo: float = 2.0
    sigma_hi: float = 8.0


@dataclass(frozen=True)
class ArrayConfig:
    n_ant: int = 64
    hours: float = 4.0
    dt_s: float = 60.0
    r_max: float = 4000.0  # metres; only the shape matters after uv rescaling
    latitude_deg: float = -30.7
    dec_deg: float = -30.0
    layout_seed: Optional[int] = None  # None: derived from the problem seed


@dataclass(frozen=True)
class ProblemConfig:
    n: int = 256
    pad: int = 2  # P = pad * N
    sky: SkyConfig = field(default_factory=SkyConfig)
    array: ArrayConfig = field(default_factory=ArrayConfig)
    cut: float = 0.25  # ell = cut * (P/4)
    delta: Optional[float] = None  # default max(1, round(0.1 ell))
    noise_rel: float = 1e-3
    uv_fill: float = 0.25  # longest baseline at uv_fill * P cells
    seed: int = 1
    iters: int = 200  # FISTA iterations per step quoted with the workload

    @property
    def P(self) -> int:
        return self.pad * self.n

    def replace(self, **kw) -> "ProblemConfig":
        return dataclasses.replace(self, **kw)


@dataclass
class Problem:
    cfg: ProblemConfig
    n: int
    P: int
    sky: np.ndarray  # N x N
    w_L: np.ndarray  # P x P counts (natural weights), signed-frequency FFT order
    w_H: np.ndarray
    w_full: np.ndarray
    psf_L: np.ndarray  # P x P, peak 1 at (P/2, P/2)
    psf_H: np.ndarray
    psf_full: np.ndarray
    dirty_L: np.ndarray  # N x N
    dirty_H: np.ndarray
    dirty_full: np.ndarray
    ell: float
    delta: float
    counts: dict  # |V|, |V_L|, |V_H|, |V_LH|

    def as_f32(self, name: str) -> np.ndarray:
        return np.ascontiguousarray(getattr(self, name), dtype=np.float32)


# --------------------------------------------------------------------------
# sky
# --------------------------------------------------------------------------
def _log_uniform(rng, lo, hi, size):
    return 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), size)


def make_sky(n: int, sky: SkyConfig, rng: np.random.Generator) -> np.ndarray:
    img = np.zeros((n, n), dtype=np.float64)
    if sky.n_points:
        rows = rng.integers(0, n, sky.n_points)
        cols = rng.integers(0, n, sky.n_points)
        flux = _log_uniform(rng, sky.flux_lo, sky.flux_hi, sky.n_points)
        np.add.at(img, (rows, cols), flux)
    for _ in range(sky.n_gauss):
        s = np.sort(rng.uniform(sky.sigma_lo, sky.sigma_hi, 2))
        s_min, s_maj = s[0], s[1]
        pa = rng.uniform(0.0, np.pi)
        peak = _log_uniform(rng, sky.flux_lo, sky.flux_hi, 1)[0]
        cy, cx = rng.uniform(0.0, n, 2)
        half = int(np.ceil(4.0 * s_maj))
        r0, r1 = max(0, int(cy) - half), min(n, int(cy) + half + 1)
        c0, c1 = max(0, int(cx) - half), min(n, int(cx) + half + 1)
        if r0 >= r1 or c0 >= c1:
            continue
        yy, xx = np.mgrid[r0:r1, c0:c1].astype(np.float64)
        dy, dx = yy + 0.5 - cy, xx + 0.5 - cx
        ca, sa = np.cos(pa), np.sin(pa)
        a = ca * dx + sa * dy
        b = -sa * dx + ca * dy
        img[r0:r1, c0:c1] += peak * np.exp(-0.5 * ((a / s_maj) ** 2 + (b / s_min) ** 2))
    return img


# --------------------------------------------------------------------------
# array and uv coverage
# --------------------------------------------------------------------------
def make_antennas(arr: ArrayConfig, rng: np.random.Generator) -> np.ndarray:
    """Equatorial XYZ antenna positions, shape (n_ant, 3)."""
    u = rng.uniform(0.0, 1.0, arr.n_ant)
    radius = arr.r_max * 10.0 ** (-2.0 * u)
    theta = rng.uniform(0.0, 2.0 * np.pi, arr.n_ant)
    east = radius * np.cos(theta)
    north = radius * np.sin(theta)
    lat = np.deg2rad(arr.latitude_deg)
    # local (E, N, Up=0) -> equatorial (X towards H=0 on the equator, Y east, Z pole)
    x = -np.sin(lat) * north
    y = east
    z = np.cos(lat) * north
    return np.stack([x, y, z], axis=1)


def _baselines(xyz: np.ndarray) -> np.ndarray:
    p, q = np.triu_indices(xyz.shape[0], k=1)
    return xyz[q] - xyz[p]


def _hour_angles(arr: ArrayConfig) -> np.ndarray:
    n_t = int(round(arr.hours * 3600.0 / arr.dt_s))
    h_hours = -arr.hours / 2.0 + arr.dt_s / 3600.0 * np.arange(n_t)
    return h_hours * (2.0 * np.pi / 24.0)


def uv_tracks(xyz: np.ndarray, arr: ArrayConfig, chunk: int = 16384):
    """Yield (u, v) arrays (metres) for chunks of baselines over all hour angles."""
    b = _baselines(xyz)
    ha = _hour_angles(arr)
    sh, ch = np.sin(ha), np.cos(ha)
    dec = np.deg2rad(arr.dec_deg)
    sd, cd = np.sin(dec), np.cos(dec)
    for s in range(0, b.shape[0], chunk):
        bx = b[s : s + chunk, 0:1]
        by = b[s : s + chunk, 1:2]
        bz = b[s : s + chunk, 2:3]
        u = sh[None, :] * bx + ch[None, :] * by
        v = -sd * ch[None, :] * bx + sd * sh[None, :] * by + cd * bz
        yield u.ravel(), v.ravel()


def _max_radius(xyz, arr):
    m = 0.0
    for u, v in uv_tracks(xyz, arr):
        m = max(m, float(np.max(u * u + v * v)))
    return float(np.sqrt(m))  # sqrt is monotone: the largest radius of the samples


def _reflect(w: np.ndarray) -> np.ndarray:
    """w[(-ky) mod P, (-kx) mod P]: the grid of the conjugate visibilities."""
    return np.roll(w[::-1, ::-1], 1, axis=(0, 1))


def grid_weights(xyz, arr: ArrayConfig, P: int, uv_fill: float, ell: float, delta: float, progress=None):
    """Natural-weight grids of the full set and of the L / H splits.

    Returns (w_full, w_L, w_H, counts).  Grids are P x P float64 in FFT order
    (row = v cell, column = u cell, index k mod P).  Every visibility and its
    conjugate land on the grid: the visibilities are counted per cell, and the
    conjugates are that count reflected through the origin.  `progress(message)`,
    if given, is called for every chunk of baselines.
    """
    rmax = _max_radius(xyz, arr)
    scale = uv_fill * P / rmax
    w_full = np.zeros(P * P, dtype=np.float64)
    w_L = np.zeros(P * P, dtype=np.float64)
    w_H = np.zeros(P * P, dtype=np.float64)
    n_all = n_L = n_H = n_LH = 0
    for chunk, (u, v) in enumerate(uv_tracks(xyz, arr)):
        if progress is not None:
            progress(f"gridding baseline chunk {chunk}")
        uc, vc = u * scale, v * scale
        r = np.sqrt(uc * uc + vc * vc)
        iu = np.rint(uc).astype(np.int64)
        iv = np.rint(vc).astype(np.int64)
        idx = (iv % P) * P + (iu % P)
        in_L = r <= ell + delta
        in_H = r >= ell - delta
        w_full += np.bincount(idx, minlength=P * P)
        w_L += np.bincount(idx[in_L], minlength=P * P)
        w_H += np.bincount(idx[in_H], minlength=P * P)
        n_all += r.size
        n_L += int(in_L.sum())
        n_H += int(in_H.sum())
        n_LH += int((in_L & in_H).sum())
    counts = {"V": n_all, "V_L": n_L, "V_H": n_H, "V_LH": n_LH}
    grids = []
    for w in (w_full, w_L, w_H):
        w = w.reshape(P, P)
        grids.append(w + _reflect(w))
    return grids[0], grids[1], grids[2], counts


def partition_counts(radius: np.ndarray, ell: float, delta: float) -> dict:
    in_L = radius <= ell + delta
    in_H = radius >= ell - delta
    return {
        "V": int(radius.size),
        "V_L": int(in_L.sum()),
        "V_H": int(in_H.sum()),
        "V_LH": int((in_L & in_H).sum()),
    }


# --------------------------------------------------------------------------
# PSF and dirty image formation (the imaging pipeline's output, not the solver)
# --------------------------------------------------------------------------
def _psf_from_weights(w: np.ndarray) -> np.ndarray:
    P = w.shape[0]
    tot = w.sum()
    if tot <= 0:
        raise ValueError("empty weight grid")
    img = np.fft.ifft2(w).real * (P * P / tot)
    return np.fft.fftshift(img)


def _dirty_from_weights(sky: np.ndarray, w: np.ndarray, noise_rel: float, rng) -> np.ndarray:
    n = sky.shape[0]
    P = w.shape[0]
    o = (P - n) // 2
    big = np.zeros((P, P), dtype=np.float64)
    big[o : o + n, o : o + n] = sky
    vis = np.fft.fft2(big) * (w * (P * P / w.sum()))
    clean = np.fft.ifft2(vis).real[o : o + n, o : o + n]
    sd = noise_rel * float(np.max(clean))
    return clean + rng.normal(0.0, sd, clean.shape)


def make_problem(cfg: ProblemConfig, with_full: bool = True, progress=None) -> Problem:
    """Builds the problem; ``with_full=False`` skips the all-baseline PSF/dirty
    image.  `progress(message)`, if given, is called as each stage starts (the
    largest workloads take minutes)."""
    say = progress if progress is not None else (lambda msg: None)
    n, P = cfg.n, cfg.P
    if n < 4 or (n & (n - 1)):
        raise ValueError("n must be a power of two >= 4")
    ss = np.random.SeedSequence(cfg.seed)
    s_sky, s_arr, s_nL, s_nH, s_nF = ss.spawn(5)
    sky = make_sky(n, cfg.sky, np.random.Generator(np.random.PCG64(s_sky)))
    arr_rng = np.random.Generator(
        np.random.PCG64(s_arr if cfg.array.layout_seed is None else cfg.array.layout_seed)
    )
    xyz = make_antennas(cfg.array, arr_rng)
    rmax_cells = cfg.uv_fill * P
    ell = cfg.cut * rmax_cells
    delta = cfg.delta if cfg.delta is not None else float(max(1, round(0.1 * ell)))
    say("uv extent and gridding")
    w_full, w_L, w_H, counts = grid_weights(xyz, cfg.array, P, cfg.uv_fill, ell, delta, progress)
    say("PSF of the short baselines")
    psf_L = _psf_from_weights(w_L)
    say("PSF of the long baselines")
    psf_H = _psf_from_weights(w_H)
    gen = lambda s: np.random.Generator(np.random.PCG64(s))  # noqa: E731
    say("dirty image of the short baselines")
    dirty_L = _dirty_from_weights(sky, w_L, cfg.noise_rel, gen(s_nL))
    say("dirty image of the long baselines")
    dirty_H = _dirty_from_weights(sky, w_H, cfg.noise_rel, gen(s_nH))
    if with_full:
        psf_full = _psf_from_weights(w_full)
        dirty_full = _dirty_from_weights(sky, w_full, cfg.noise_rel, gen(s_nF))
    else:
        psf_full = dirty_full = None
    return Problem(
        cfg=cfg, n=n, P=P, sky=sky,
        w_L=w_L, w_H=w_H, w_full=w_full,
        psf_L=psf_L, psf_H=psf_H, psf_full=psf_full,
        dirty_L=dirty_L, dirty_H=dirty_H, dirty_full=dirty_full,
        ell=float(ell), delta=float(delta), counts=counts,
    )


def coarse_low(pr: Problem, d: int, seed: int = 0):
    """The short-baseline split imaged on a grid of N/d pixels over the same
    field of view: pixels d times larger, the same uv cells (the coarse P/d
    grid keeps the cells |k| < P/(2d) of each axis, which must hold every
    short-baseline cell).  The coarse sky holds the flux of each d x d block
    of fine pixels.  Returns (sky_s, dirty_L_s, psf_L_s)."""
    n, P = pr.n, pr.P
    if d < 2 or (d & (d - 1)) or n // d < 2:
        raise ValueError("d must be a power of two with n / d >= 2")
    m, Ps = n // d, P // d
    k = np.fft.fftfreq(P) * P
    keep = np.abs(k) < Ps / 2
    w = pr.w_L
    if np.any(w[~keep, :]) or np.any(w[:, ~keep]):
        raise ValueError("short baselines reach beyond the coarse grid's band")
    ks = (k[keep] % Ps).astype(np.int64)
    w_s = np.zeros((Ps, Ps))
    w_s[np.ix_(ks, ks)] = w[np.ix_(keep, keep)]
    sky_s = pr.sky.reshape(m, d, m, d).sum(axis=(1, 3))
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([pr.cfg.seed, 77, d, seed])))
    return sky_s, _dirty_from_weights(sky_s, w_s, pr.cfg.noise_rel, rng), _psf_from_weights(w_s)


def _sky_member(base: Problem, seed: int, i: int):
    s_sky, s_nL, s_nH = np.random.SeedSequence([seed, i]).spawn(3)
    gen = lambda s: np.random.Generator(np.random.PCG64(s))  # noqa: E731
    sky = make_sky(base.n, base.cfg.sky, gen(s_sky))
    return (sky, _dirty_from_weights(sky, base.w_L, base.cfg.noise_rel, gen(s_nL)),
            _dirty_from_weights(sky, base.w_H, base.cfg.noise_rel, gen(s_nH)))


_SET_BASE = None


def _sky_member_of_set(args):
    seed, i = args
    return _sky_member(_SET_BASE, seed, i)


def sky_set(base: Problem, count: int, seed: int, workers: int = 1) -> list:
    """`count` problems observed with `base`'s uv coverage (same PSFs and
    partition) but new skies and noise, drawn from its sky configuration: many
    fields, or many epochs, of one observation.  Member i draws from the seed
    sequence [seed, i] alone, so the set does not depend on `workers` (forked
    processes sharing `base`)."""
    if workers > 1 and count > 1:
        import multiprocessing as mp

        global _SET_BASE
        _SET_BASE = base
        try:
            with mp.get_context("fork").Pool(workers) as pool:
                members = pool.map(_sky_member_of_set, [(seed, i) for i in range(count)], chunksize=4)
        finally:
            _SET_BASE = None
    else:
        members = [_sky_member(base, seed, i) for i in range(count)]
    return [dataclasses.replace(base, sky=sky, psf_full=None, dirty_full=None, dirty_L=dl, dirty_H=dh)
            for sky, dl, dh in members]


def _make_problem_of(args):
    i, cfg, verbose = args
    stage = (lambda msg: print(f"channel {i} ({cfg.n}^2): {msg}", flush=True)) if verbose else None
    return i, make_problem(cfg, with_full=False, progress=stage)


def make_problems(cfgs, workers: int = 1, progress=None, verbose: bool = False) -> list:
    """make_problem(cfg, with_full=False) for every configuration, in order,
    in forked worker processes when workers > 1 (a problem depends on its
    configuration alone).  `progress(i, problem)` is called as each finishes;
    with `verbose` every problem prints its stages as they start."""
    cfgs = list(cfgs)
    out = [None] * len(cfgs)
    jobs = [(i, c, verbose) for i, c in enumerate(cfgs)]
    if workers > 1 and len(cfgs) > 1:
        import multiprocessing as mp

        with mp.get_context("fork").Pool(min(workers, len(cfgs))) as pool:
            for i, pr in pool.imap_unordered(_make_problem_of, jobs, chunksize=1):
                out[i] = pr
                if progress is not None:
                    progress(i, pr)
    else:
        for job in jobs:
            i, out[i] = _make_problem_of(job)
            if progress is not None:
                progress(i, out[i])
    return out


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
PRESETS = {
    # 256^2 image, 512^2 grid: 20 points + 3 Gaussians, 64 antennas, 4 h at 60 s,
    # cut 25 %, 200 iterations per step.
    "small256": ProblemConfig(
        n=256, sky=SkyConfig(20, 3), array=ArrayConfig(64, 4.0, 60.0), cut=0.25, seed=1, iters=200
    ),
    # 2048^2 image, 4096^2 grid: 2000 points + 50 Gaussians, 197 antennas,
    # 8 h at 30 s (~19k baselines), cut 20 %, 500 iterations per step.
    "sky2048": ProblemConfig(
        n=2048, sky=SkyConfig(2000, 50), array=ArrayConfig(197, 8.0, 30.0), cut=0.20, seed=2, iters=500
    ),
    # 4096^2 image, 8192^2 grid at the same source density, cut 15 %.
    "sky4096": ProblemConfig(
        n=4096, sky=SkyConfig(8000, 200), array=ArrayConfig(197, 8.0, 30.0), cut=0.15, seed=3, iters=500
    ),
    # 8192^2 image, 16384^2 grid at the same source density: 512 antennas,
    # 4 h at 10 s, cut 10 %.
    "sky8192": ProblemConfig(
        n=8192, sky=SkyConfig(32000, 800), array=ArrayConfig(512, 4.0, 10.0), cut=0.10, seed=4, iters=500
    ),
    # the paper's data shape: 512^2 image, 64 dishes, 4 h at 120 s.
    "paper512": ProblemConfig(
        n=512, sky=SkyConfig(40, 6), array=ArrayConfig(64, 4.0, 120.0), cut=55.0 / 128.0,
        delta=5.0, seed=7, iters=100
    ),
}


def preset(name: str, **overrides) -> ProblemConfig:
    cfg = PRESETS[name]
    return cfg.replace(**overrides) if overrides else cfg


def channel_set(count: int, sizes=(512, 1024, 2048, 4096), seed: int = 4, cut: float = 0.15,
                nu_lo: float = 350.0, nu_hi: float = 1050.0, n_ant: int = 64, hours: float = 4.0,
                dt_s: float = 120.0) -> list:
    """Frequency channels of one observation with uneven image sizes.

    Channel c observes at nu_c = nu_lo + (nu_hi - nu_lo) c / (count - 1) MHz
    with one array layout; baselines in wavelengths scale with nu, so its
    longest baseline lands at (nu_c / nu_hi) P/4 cells and its cut is taken
    from that radius.  Image sizes are drawn uniformly from `sizes`; the sky
    density (sources per pixel) is that of the small preset.
    """
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sizes), size=count)
    out = []
    for c, n in enumerate(ns):
        nu = nu_lo + (nu_hi - nu_lo) * c / max(count - 1, 1)
        dens = (int(n) / 256.0) ** 2
        out.append(ProblemConfig(
            n=int(n), sky=SkyConfig(max(2, int(20 * dens)), max(1, int(3 * dens))),
            array=ArrayConfig(n_ant, hours, dt_s, layout_seed=seed), cut=cut, uv_fill=0.25 * nu / nu_hi,
            seed=1000 * seed + c, iters=500,
        ))
    return out


def late_state(n: int, seed: int = 0, scale: float = 1e-2, change: float = 0.02):
    """Two non-negative N x N images (b_k, b_km1) shaped like late iterates of a
    sparse reconstruction: b_k holds point sources and Gaussians of the small
    preset's density times `scale`; b_km1 differs from it by a relative
    change of up to `change` on every non-zero pixel and by a few isolated
    pixels present in only one of the two.  Inputs only, no solver arithmetic.
    """
    rng = np.random.default_rng(seed)
    dens = (n / 256.0) ** 2
    sky = make_sky(n, SkyConfig(max(2, int(20 * dens)), max(1, int(3 * dens))), rng)
    b_k = scale * sky
    b_km1 = b_k * (1.0 - change * rng.random((n, n)))
    m = max(4, n // 16)
    idx = rng.integers(0, n, (m, 2))
    b_km1[idx[: m // 2, 0], idx[: m // 2, 1]] += scale * rng.random(m // 2)
    b_k[idx[m // 2:, 0], idx[m // 2:, 1]] += scale * rng.random(m - m // 2)
    return b_k, b_km1


def tiny(n: int, seed: int = 11, cut: float = 0.25, n_ant: int = 16) -> ProblemConfig:
    """A small problem for tests: density ~ that of the small preset."""
    pts = max(2, (20 * n * n) // (256 * 256))
    gs = 1 if n >= 32 else 0
    return ProblemConfig(
        n=n, sky=SkyConfig(pts, gs, sigma_lo=1.0, sigma_hi=max(1.5, n / 32.0)),
        array=ArrayConfig(n_ant, 4.0, 600.0), cut=cut, seed=seed, iters=50,
    )
