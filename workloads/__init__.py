"""Seeded synthetic inputs for the ensemble flood model.

This module holds input generation only: terrain, roughness, the rain
hyetograph, per-member parameter draws, gauge placement, observation noise and
the uniform/perturbation draws a particle filter consumes.  It contains none of
the model's arithmetic (no flux, continuity, time-step or weighting formula), so
both the FP64 oracle and the HIP library can be fed from it without sharing any
method code.

Workload shapes follow the paper's case study (Sec. 4.1): 3 m cells, a storm of
roughly 60 mm in one hour, Manning roughness of urban surfaces (Tab. 1) and a
handful of depth gauges.  The paper's Fuzhou DEM, land-cover map and storm
series are not available, so seeded synthetic stand-ins with the same shapes
are used instead.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 20230216

EDGE_WALL = 0
EDGE_OPEN = 1
# edge order used everywhere: north, east, south, west
EDGE_N, EDGE_E, EDGE_S, EDGE_W = 0, 1, 2, 3


def seed_for(config: int, catchment: int = 0, stream: int = 0) -> int:
    """Seed of configuration ``config`` (1-based), catchment ``catchment``."""
    return SEED_BASE + 1000 * config + 10 * catchment + stream


# --------------------------------------------------------------------------
# rain
# --------------------------------------------------------------------------
def chicago_cumulative_mm(t_min: np.ndarray, total_mm: float = 60.0, duration_min: float = 60.0,
                          peak_frac: float = 0.4, b: float = 10.0, c: float = 0.7) -> np.ndarray:
    """Cumulative depth (mm) of a Keifer-Chu ("Chicago") design storm.

    Average intensity over a window of length tau is a/(tau+b)^c, so the depth
    falling in a window centred on the peak is P(tau) = a*tau/(tau+b)^c.  The
    advancement coefficient ``peak_frac`` places that fraction of every window
    before the peak.  ``a`` is chosen so that the whole storm delivers
    ``total_mm``.
    """
    T = duration_min
    r = peak_frac
    a = total_mm * (T + b) ** c / T

    def P(tau):
        return a * tau / (tau + b) ** c

    t = np.asarray(t_min, dtype=np.float64)
    out = np.where(
        t <= r * T,
        r * P(T) - r * P(np.maximum(r * T - t, 0.0) / r),
        r * P(T) + (1.0 - r) * P(np.maximum(t - r * T, 0.0) / (1.0 - r)),
    )
    return out


def chicago_hyetograph(total_mm: float = 60.0, duration_s: float = 3600.0, block_s: float = 300.0,
                       peak_frac: float = 0.4) -> np.ndarray:
    """Block-averaged rain rates (m/s) of the design storm, one per ``block_s`` block."""
    nb = int(round(duration_s / block_s))
    edges = np.arange(nb + 1) * block_s / 60.0
    cum = chicago_cumulative_mm(edges, total_mm, duration_s / 60.0, peak_frac)
    depth_mm = np.diff(cum)
    return depth_mm * 1e-3 / block_s


def uniform_rain(rate_mm_h: float, duration_s: float, block_s: float = 300.0) -> np.ndarray:
    nb = int(math.ceil(duration_s / block_s))
    return np.full(nb, rate_mm_h * 1e-3 / 3600.0, dtype=np.float64)


# --------------------------------------------------------------------------
# terrain
# --------------------------------------------------------------------------
def dem_plane_bumps(ny: int, nx: int, dx: float, slope: float, n_bumps: int,
                    rng: np.random.Generator) -> np.ndarray:
    """Plane falling by ``slope`` toward the south edge plus Gaussian bumps.

    Bumps: centre uniform over the grid, height U(0.5, 2) m, width sigma
    U(5, 15) cells.
    """
    r = np.arange(ny, dtype=np.float64)[:, None]
    c = np.arange(nx, dtype=np.float64)[None, :]
    z = slope * dx * (ny - 1 - r) + 0.0 * c
    for _ in range(n_bumps):
        rc = rng.uniform(0, ny)
        cc = rng.uniform(0, nx)
        hgt = rng.uniform(0.5, 2.0)
        sig = rng.uniform(5.0, 15.0)
        z = z + hgt * np.exp(-((r - rc) ** 2 + (c - cc) ** 2) / (2.0 * sig * sig))
    return z.astype(np.float32)


def fractal_terrain(ny: int, nx: int, rng: np.random.Generator, beta: float = 2.5,
                    relief: float = 15.0) -> np.ndarray:
    """Spectral-synthesis fractal surface: white noise filtered by k^(-beta/2)."""
    noise = rng.standard_normal((ny, nx))
    F = np.fft.rfft2(noise)
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.rfftfreq(nx)[None, :]
    k = np.sqrt(kx * kx + ky * ky)
    k[0, 0] = 1.0
    F = F * k ** (-beta / 2.0)
    F[0, 0] = 0.0
    z = np.fft.irfft2(F, s=(ny, nx))
    z = (z - z.min()) / max(z.max() - z.min(), 1e-30) * relief
    return z


def building_mask(ny: int, nx: int, rng: np.random.Generator, frac: float = 0.30,
                  period: int = 12, street: int = 2, tol: float = 0.005) -> np.ndarray:
    """Boolean mask of building cells.

    The grid is cut into city blocks of ``period`` cells separated by streets
    ``street`` cells wide.  Each block may hold one rectangular building of
    U{4..10} x U{4..10} cells placed at a random offset; buildings are added or
    removed at random until the covered fraction is within ``frac +- tol``.
    """
    lot = period - street
    nby = (ny + period - 1) // period
    nbx = (nx + period - 1) // period
    rects = []
    for by in range(nby):
        for bx in range(nbx):
            w = int(rng.integers(4, 11))
            hgt = int(rng.integers(4, 11))
            w = min(w, lot)
            hgt = min(hgt, lot)
            oy = by * period + street + int(rng.integers(0, lot - hgt + 1))
            ox = bx * period + street + int(rng.integers(0, lot - w + 1))
            rects.append((oy, ox, hgt, w))
    order = rng.permutation(len(rects))
    on = np.ones(len(rects), dtype=bool)
    m = np.zeros((ny, nx), dtype=bool)
    for oy, ox, hgt, w in rects:          # lots are disjoint, so painting is order-free
        m[oy:oy + hgt, ox:ox + w] = True
    area = np.array([min(oy + hgt, ny) - min(oy, ny) for oy, ox, hgt, w in rects]) * \
        np.array([min(ox + w, nx) - min(ox, nx) for oy, ox, hgt, w in rects])
    covered = int(m.sum())
    target = frac * ny * nx
    it = 0
    # remove buildings (random order) while above target, add back while below
    while abs(covered - target) > tol * ny * nx and it < 4 * len(rects):
        i = order[it % len(order)]
        it += 1
        oy, ox, hgt, w = rects[i]
        if covered > target and on[i]:
            on[i] = False
            m[oy:oy + hgt, ox:ox + w] = False
            covered -= int(area[i])
        elif covered < target and not on[i]:
            on[i] = True
            m[oy:oy + hgt, ox:ox + w] = True
            covered += int(area[i])
    return m


def dem_urban(ny: int, nx: int, rng: np.random.Generator, beta: float = 2.5, relief: float = 15.0,
              building_height: float = 10.0, building_frac: float = 0.30):
    """Urban-style DEM: fractal terrain plus raised building blocks.

    Returns ``(dem float32, building mask)``.
    """
    z = fractal_terrain(ny, nx, rng, beta, relief)
    b = building_mask(ny, nx, rng, building_frac)
    z = z + building_height * b
    return z.astype(np.float32), b


# --------------------------------------------------------------------------
# ensemble draws
# --------------------------------------------------------------------------
def lognormal(rng: np.random.Generator, n: int, mean_log: float = 0.0, sd_log: float = 0.3) -> np.ndarray:
    return np.exp(rng.normal(mean_log, sd_log, size=n))


def pick_gauges(mask_ok: np.ndarray, k: int, rng: np.random.Generator, margin: int = 2) -> np.ndarray:
    """``k`` distinct (row, col) cells where ``mask_ok`` holds, away from the edge."""
    ny, nx = mask_ok.shape
    ok = mask_ok.copy()
    ok[:margin, :] = False
    ok[-margin:, :] = False
    ok[:, :margin] = False
    ok[:, -margin:] = False
    idx = np.flatnonzero(ok)
    sel = rng.choice(idx, size=k, replace=False)
    return np.stack([sel // nx, sel % nx], axis=1).astype(np.int32)


def obs_noise(rng: np.random.Generator, truth: np.ndarray, sigma: float = 0.05) -> np.ndarray:
    """Synthetic observations: truth + N(0, sigma^2)."""
    t = np.asarray(truth, dtype=np.float64)
    return t + rng.normal(0.0, sigma, size=t.shape)


def pf_draws(rng: np.random.Generator, n_members: int, beta_sd: float = 0.05):
    """One resampling offset u0 ~ U[0,1) and per-member rain perturbations beta ~ N(1, sd^2)."""
    u0 = float(rng.uniform(0.0, 1.0))
    beta = rng.normal(1.0, beta_sd, size=n_members)
    return u0, beta


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------
@dataclass
class Catchment:
    name: str
    ny: int
    nx: int
    dx: float
    dem: np.ndarray            # float32 [ny, nx]
    manning: np.ndarray        # float32 [ny, nx]
    edge_kind: tuple
    edge_slope: tuple
    n_members: int
    n_scale: np.ndarray        # float64 [N]
    rain_mult: np.ndarray      # float64 [N]
    gauges: np.ndarray         # int32 [K, 2]
    street: np.ndarray | None = None
    truth_n_scale: float = 1.0
    truth_rain_mult: float = 1.0
    h0: np.ndarray | None = None
    # land cover (Sec. 4.1, Table 1); None: shared Manning field x member scale
    land_class: np.ndarray | None = None      # uint8 [ny, nx]: 0 hardened ground, 1 green land, 2 water
    class_runoff: np.ndarray | None = None    # [3]
    class_drain: np.ndarray | None = None     # [3] int
    class_n: np.ndarray | None = None         # [N, 3] per-member Manning n of each class
    drain: np.ndarray | None = None           # [N] drainage rate, m/s
    truth_class_n: np.ndarray | None = None   # [3]
    truth_drain: float = 0.0
    # inflow hydrographs (Sec. 4.1) and streamflow sections (Sec. 4.4); None: none
    inflow: np.ndarray | None = None          # int32 [n, 3]: edge (N, E, S, W), position, series
    inflow_q: np.ndarray | None = None        # [n_series, n_blocks] inward discharge per unit width, m^2/s
    sections: list | None = None              # int32 [n_links, 4] each: kind (0 x / 1 y), r, c, sign


@dataclass
class Workload:
    name: str
    catchments: list
    rain: np.ndarray            # m/s per block
    rain_interval: float
    t_end: float
    real_bytes: int = 4
    cfl_alpha: float = 0.7
    h_dry: float = 1e-3
    dt_cap: float = 10.0
    dt_fixed: float = 0.0
    g: float = 9.81
    pf_every: float = 0.0
    obs_sigma: float = 0.05
    sample_dt: float = 0.0
    seed: int = SEED_BASE
    extra: dict = field(default_factory=dict)


# Land cover of the synthetic city (Sec. 4.1, Table 1): streets and roofs are
# hardened ground, open lot area is green land, the lowest 3 % of the open
# ground are water bodies.  Per-member roughness is drawn uniformly within
# Table 1's initial-ensemble ranges; the drainage rate of hardened ground within
# +-50 % of the paper's 12 mm/h.
CLASS_HARD, CLASS_GREEN, CLASS_WATER = 0, 1, 2
CLASS_N_RANGE = ((0.010, 0.022), (0.08, 0.22), (0.016, 0.030))
CLASS_N_TRUTH = (0.017, 0.15, 0.020)
CLASS_RUNOFF = (1.0, 0.9, 1.0)
CLASS_DRAIN = (1, 0, 0)
DRAIN_MMH = 12.0


def land_cover(dem: np.ndarray, bmask: np.ndarray, period: int = 12, street: int = 2,
               water_frac: float = 0.03) -> np.ndarray:
    ny, nx = dem.shape
    r = np.arange(ny)[:, None] % period
    c = np.arange(nx)[None, :] % period
    streets = (r < street) | (c < street)
    cls = np.full((ny, nx), CLASS_GREEN, dtype=np.uint8)
    cls[streets | bmask] = CLASS_HARD
    green = cls == CLASS_GREEN
    if np.any(green):
        cut = np.quantile(dem[green], water_frac)
        cls[green & (dem <= cut)] = CLASS_WATER
    return cls


# Two synthetic stream outlets on the north edge (Sec. 4.1 assigns synthetic
# hydrographs to the boundary cells of two stream outlets; the paper's series
# are not available): each enters along a street, two links wide, with a
# triangular hydrograph over the 12 rain blocks, the second 0.6 of the first and
# one block later.  A streamflow section crosses each street a quarter of the way
# down (Sec. 4.4: two flow gauges), two cells wider than the street on each side.
HYDROGRAPH = (0.05, 0.10, 0.20, 0.35, 0.50, 0.45, 0.35, 0.25, 0.18, 0.12, 0.08, 0.05)


def stream_inflow(ny: int, nx: int, n_blocks: int = 12, period: int = 12):
    base = np.interp(np.arange(n_blocks), np.linspace(0, n_blocks - 1, len(HYDROGRAPH)), HYDROGRAPH)
    second = 0.6 * np.concatenate([[base[0]], base[:-1]])
    cols = sorted({min(max(period * int(round(nx * f / period)), 0), nx - 2) for f in (1 / 3, 2 / 3)})
    inflow, sections = [], []
    rs = min(ny - 1, max(1, ny // 4))
    for j, c0 in enumerate(cols):
        inflow += [(0, c0, j), (0, c0 + 1, j)]
        sections.append(np.array([(1, rs, c, 1) for c in range(max(c0 - 2, 0), min(c0 + 4, nx))], dtype=np.int32))
    q = np.array([base, second][:len(cols)])
    return np.array(inflow, dtype=np.int32), q, sections


def urban_catchment(name: str, ny: int, nx: int, n_members: int, seed: int, n_gauges: int = 5,
                    dx: float = 3.0, open_slope: float = 1e-3, with_land_cover: bool = False,
                    with_inflow: bool = False) -> Catchment:
    rng = np.random.default_rng(seed)
    dem, bmask = dem_urban(ny, nx, rng)
    manning = np.full((ny, nx), 0.03, dtype=np.float32)
    s = lognormal(rng, n_members)
    mu = lognormal(rng, n_members)
    gauges = pick_gauges(~bmask, n_gauges, rng)
    ts = float(lognormal(rng, 1)[0])
    tm = float(lognormal(rng, 1)[0])
    cat = Catchment(name=name, ny=ny, nx=nx, dx=dx, dem=dem, manning=manning,
                    edge_kind=(EDGE_OPEN,) * 4, edge_slope=(open_slope,) * 4,
                    n_members=n_members, n_scale=s, rain_mult=mu, gauges=gauges, street=~bmask,
                    truth_n_scale=ts, truth_rain_mult=tm)
    if with_land_cover:
        lrng = np.random.default_rng(seed + 5)       # its own stream: the draws above do not move
        cat.land_class = land_cover(dem, bmask)
        cat.class_runoff = np.array(CLASS_RUNOFF)
        cat.class_drain = np.array(CLASS_DRAIN, dtype=np.int32)
        lo = np.array([a for a, _ in CLASS_N_RANGE])
        hi = np.array([b for _, b in CLASS_N_RANGE])
        cat.class_n = lrng.uniform(lo, hi, size=(n_members, 3))
        cat.drain = lrng.uniform(0.5, 1.5, size=n_members) * DRAIN_MMH / 3.6e6
        cat.truth_class_n = np.array(CLASS_N_TRUTH)
        cat.truth_drain = DRAIN_MMH / 3.6e6
    if with_inflow:
        cat.inflow, cat.inflow_q, cat.sections = stream_inflow(ny, nx)
    return cat


def config1(ny: int = 128, nx: int = 128) -> Workload:
    """Plain method, one member, FP64: plane + bumps, 50 mm/h for 600 s, open south edge."""
    seed = seed_for(1)
    rng = np.random.default_rng(seed)
    dem = dem_plane_bumps(ny, nx, 3.0, 1e-3, 20, rng)
    manning = np.full((ny, nx), 0.03, dtype=np.float32)
    c = Catchment(name="plane_bumps", ny=ny, nx=nx, dx=3.0, dem=dem, manning=manning,
                  edge_kind=(EDGE_WALL, EDGE_WALL, EDGE_OPEN, EDGE_WALL),
                  edge_slope=(0.0, 0.0, 1e-3, 0.0), n_members=1,
                  n_scale=np.ones(1), rain_mult=np.ones(1),
                  gauges=np.zeros((0, 2), dtype=np.int32))
    return Workload(name="c1_plane128_fp64", catchments=[c], rain=uniform_rain(50.0, 600.0),
                    rain_interval=300.0, t_end=600.0, real_bytes=8, seed=seed)


def config2(ny: int = 1024, nx: int = 1024, n_members: int = 32) -> Workload:
    """Forward + particle filter, FP32, urban DEM, Chicago storm, PF every 300 s, 5 gauges."""
    seed = seed_for(2)
    c = urban_catchment("urban1024", ny, nx, n_members, seed, n_gauges=5)
    return Workload(name="c2_urban1024x32_pf", catchments=[c], rain=chicago_hyetograph(),
                    rain_interval=300.0, t_end=3600.0, real_bytes=4, pf_every=300.0, seed=seed)


def config3(ny: int = 1024, nx: int = 1024, n_members: int = 16) -> Workload:
    """Differentiation: 16 members, 8 gauges, 1800 s, 10 s sampling, checkpoints every 100 steps."""
    seed = seed_for(3)
    c = urban_catchment("urban1024_adj", ny, nx, n_members, seed, n_gauges=8)
    return Workload(name="c3_urban1024x16_adjoint", catchments=[c], rain=chicago_hyetograph(),
                    rain_interval=300.0, t_end=1800.0, real_bytes=4, sample_dt=10.0, seed=seed,
                    extra={"ckpt_every": 100})


def config4(members_each: int = 24, shapes=((512, 512), (768, 1536), (1024, 1024), (2000, 2000))) -> Workload:
    """Batched uneven catchments, 24 members each, PF every 300 s, 5 gauges per catchment."""
    seed = seed_for(4)
    cs = [urban_catchment(f"urban{ny}x{nx}", ny, nx, members_each, seed_for(4, j), n_gauges=5)
          for j, (ny, nx) in enumerate(shapes)]
    return Workload(name="c4_batched_uneven_96", catchments=cs, rain=chicago_hyetograph(),
                    rain_interval=300.0, t_end=1800.0, real_bytes=4, pf_every=300.0, seed=seed)


def config5(ny: int = 2000, nx: int = 2000, n_members: int = 96, with_land_cover: bool = False,
            with_inflow: bool = False) -> Workload:
    """Paper-scale single GPU: 4.0 M cells x 96 members, 3600 s, PF every 600 s, 10 gauges
    (optionally with the land cover of Sec. 4.1: class roughness, runoff, drainage)."""
    seed = seed_for(5)
    c = urban_catchment("urban2000", ny, nx, n_members, seed, n_gauges=10, with_land_cover=with_land_cover,
                        with_inflow=with_inflow)
    return Workload(name="c5_urban2000x96_pf", catchments=[c], rain=chicago_hyetograph(),
                    rain_interval=300.0, t_end=3600.0, real_bytes=4, pf_every=600.0, seed=seed,
                    extra={"adj_window": 900.0, "ckpt_every": 100})


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}
