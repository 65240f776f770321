"""Trajectory parity of GPU runs against the FP64 oracle by replay (Sec. 2.1,
Eqs. 1-5; the wet/dry rule of Eq. 3 and the remark on wet-dry fronts).

Every step of every member is replayed in the oracle with the GPU's step
length, end time and links' wet/dry decisions; the decisions themselves are
checked bit for bit against the oracle's, taken from the same state in the
kernel's precision (see tests/trajectory.py).  Bars at every checkpoint and at
the end: depth 1e-4 m on every cell, discharge 1e-4 of the largest |q| on
every link; FP64 handles 1e-9 m and 1e-9 of the largest |q|.  FP32 mass
ledgers 1e-6, FP64 1e-12.
"""
import numpy as np
import pytest

import trajectory as TR
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2302_08341_amd import flood
    flood.load_library()
    return flood


RAIN = W.chicago_hyetograph()
URBAN = W.urban_catchment("par", 97, 83, 5, W.seed_for(2, 5), n_gauges=4)   # ragged against every tile
LAND = W.urban_catchment("lc", 53, 72, 4, W.seed_for(2, 41), n_gauges=4, with_land_cover=True)
INFL = W.urban_catchment("inf", 45, 64, 4, W.seed_for(2, 61), n_gauges=3, with_inflow=True)


def _handle(fl, c, n, **kw):
    d = dict(dem=c.dem, manning=c.manning, dx=c.dx, edge_kind=c.edge_kind, edge_slope=c.edge_slope,
             n_members=n, n_scale=c.n_scale[:n], rain_mult=c.rain_mult[:n], h0=c.h0)
    if getattr(c, "land_class", None) is not None:
        d.update(land_class=c.land_class, class_runoff=c.class_runoff, class_drain=c.class_drain,
                 class_n=c.class_n[:n], drain=c.drain[:n])
    if getattr(c, "inflow", None) is not None:
        d.update(inflow=c.inflow, inflow_q=c.inflow_q)
    return fl.FloodEnsemble([d], RAIN, **kw)


def _model(orc, c, **kw):
    extra = {}
    if getattr(c, "land_class", None) is not None:
        extra.update(land_class=c.land_class, class_runoff=c.class_runoff, class_drain=c.class_drain)
    if getattr(c, "inflow", None) is not None:
        extra.update(inflow=c.inflow, inflow_q=c.inflow_q)
    extra.update(kw)
    return orc.Model(c.dem, c.manning, c.dx, RAIN, edge_kind=c.edge_kind, edge_slope=c.edge_slope, **extra)


def _member(orc, m, c, i):
    kw = {}
    if getattr(c, "land_class", None) is not None:
        kw.update(class_n=c.class_n[i], drain_rate=c.drain[i])
    return orc.Member.dry(m, s=c.n_scale[i], mu=c.rain_mult[i], h0=c.h0, **kw)


def _ledger_ok(e, tol):
    led = e.ledger()
    inflow = led.get("inflow", np.zeros_like(led["rain_in"]))
    drained = led.get("drain", np.zeros_like(led["rain_in"]))
    resid = np.abs(led["storage"] - (led["rain_in"] + inflow - led["outflow"] + led["clamp"] - drained))
    assert (resid / (led["rain_in"] + inflow)).max() <= tol, resid


@pytest.mark.parametrize("name,cat,n,t_end", [("urban", URBAN, 5, 900.0), ("land_cover", LAND, 4, 1500.0),
                                              ("inflow", INFL, 4, 1500.0)])
def test_fp32_trajectory_replay(fl, orc, name, cat, n, t_end):
    print("replay", name, flush=True)
    e = _handle(fl, cat, n, real_bytes=4)
    m = _model(orc, cat)
    refs = {i: _member(orc, m, cat, i) for i in range(n)}
    free = {i: _member(orc, m, cat, i) for i in range(n)}
    out = TR.replay(fl, orc, e, m, refs, t_end, free=free, check_every=50)
    assert out["steps"] > 100 and out["checks"] >= n * 3
    # links beyond the discharge bar are counted and each must be reproduced by the
    # oracle's own step from the GPU's state (measured: none on the urban and inflow
    # runs; on the land-cover run the drained hardened ground carries shallow sheet
    # flow a few h_dry deep whose Eq. 2 friction, h^-7/3, turns depth differences of
    # ~1e-6 m, 100 times inside the depth bar, into up to ~2e-4 of a small largest
    # discharge early in the storm)
    print(name, "link checks beyond the discharge bar:", out["q_exceed"])
    # the ledger of every term agrees with the replayed oracle's, and closes
    led = e.ledger()
    for i in range(n):
        assert led["rain_in"][i] == pytest.approx(refs[i].v_rain, rel=1e-6)
        assert led["outflow"][i] == pytest.approx(refs[i].v_out, rel=1e-4, abs=1e-6 * refs[i].v_rain)
        if name == "land_cover":
            assert led["drain"][i] == pytest.approx(refs[i].v_drain, rel=1e-4)
        if name == "inflow":
            assert led["inflow"][i] == pytest.approx(refs[i].v_in, rel=1e-6)
    _ledger_ok(e, 1e-6)


@pytest.mark.parametrize("shape", [(1, 37), (29, 1), (2, 2), (65, 64)])
def test_fp64_degenerate_grids_shallow_open_dry_start(fl, orc, shape):
    # thin, tiny and square grids, all edges open, dry start, shallow water under a
    # light uniform rain whose increments land on h_dry: the GPU's double-precision
    # decisions (difference form) are checked bit for bit and replayed
    ny, nx = shape
    rng = np.random.default_rng(ny * 1000 + nx)
    z = rng.uniform(0.0, 0.02, size=(ny, nx)).astype(np.float32).astype(np.float64)
    n = np.full((ny, nx), np.float32(0.03), dtype=np.float64)   # the library takes float rasters
    rain = W.uniform_rain(1440.0, 300.0)       # 2e-4 m per 0.5-s step: the fifth lands on h_dry = 1e-3 m
    c = dict(dem=z, manning=n, dx=3.0, edge_kind=(1, 1, 1, 1), edge_slope=(1e-3,) * 4, n_members=2,
             n_scale=np.array([1.0, 1.3]), rain_mult=np.array([1.0, 0.7]))
    e = fl.FloodEnsemble([c], rain, real_bytes=8, dt_fixed=0.5, member_interleave=1)
    m = orc.Model(z, n, 3.0, rain, edge_kind=(1, 1, 1, 1), edge_slope=(1e-3,) * 4, dt_fixed=0.5)
    refs = {i: orc.Member.dry(m, s=c["n_scale"][i], mu=c["rain_mult"][i]) for i in range(2)}
    out = TR.replay(fl, orc, e, m, refs, 300.0, check_every=100, h_tol=1e-9, q_tol=1e-9,
                    mask_mode=orc.MASK_DIFF64)
    assert out["steps"] == 600
    _ledger_ok(e, 1e-12)
