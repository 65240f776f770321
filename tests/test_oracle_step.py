"""Pins of the oracle's forward step against facts other than its own code.

Each test names what fixes the expected value: a hand closed form of Eqs. 2-3
in a special case, the worked Eq. 4 check of Sec. 4.1, an invariant (lake at
rest, mass conservation, mirror/transpose symmetry) or an independently solved
discrete steady state (rain-fed plane, Manning normal flow).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import brentq

import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")
G = 9.81


def _model(orc, z, n=0.03, dx=3.0, rain=(), edges=(0, 0, 0, 0), slopes=(0, 0, 0, 0), **kw):
    z = np.asarray(z, dtype=np.float64)
    nn = np.full(z.shape, n) if np.isscalar(n) else np.asarray(n, dtype=np.float64)
    return orc.Model(z, nn, dx, np.asarray(rain, dtype=np.float64), edge_kind=edges, edge_slope=slopes, **kw)


# ---------------------------------------------------------------------------
# Eq. 4: the worked check printed in Sec. 4.1
# ---------------------------------------------------------------------------
def test_eq4_worked_value_from_paper(orc):
    gold = json.load(open(GOLD))["eq4_worked_check"]
    z = np.zeros((3, 3))
    m = _model(orc, z, alpha=gold["k"], dx=gold["dx_m"], dt_cap=1e9, h_dry=1e-3)
    h = np.zeros((3, 3))
    h[1, 1] = gold["h_max_m"]
    dt = orc.dt_cfl(m, h)
    # Eq. 4 at the printed values: k dx / sqrt(g h_max) = 0.2524 s, which the paper
    # states is not exceeded by its fixed 0.25 s step
    assert dt == pytest.approx(0.54 * 3.0 / math.sqrt(9.81 * 4.2), rel=1e-15)
    assert dt >= gold["dt_fixed_s"]
    assert dt == pytest.approx(0.25241, abs=5e-5)


def test_dt_floor_cap_and_fixed(orc):
    z = np.zeros((2, 2))
    m = _model(orc, z, alpha=0.7, dx=3.0, dt_cap=10.0, h_dry=1e-3)
    # dry grid: depth floored at h_dry, then capped
    assert orc.dt_cfl(m, np.zeros((2, 2))) == 10.0
    h = np.full((2, 2), 1.0)
    assert orc.dt_cfl(m, h) == pytest.approx(0.7 * 3.0 / math.sqrt(9.81), rel=1e-15)
    m2 = _model(orc, z, dt_fixed=0.25)
    assert orc.dt_cfl(m2, h) == 0.25


# ---------------------------------------------------------------------------
# Eqs. 2-3: closed forms of the first step from rest (|q| = 0 => no friction)
# ---------------------------------------------------------------------------
def test_first_step_from_rest_flat_bed(orc):
    dx, dt = 3.0, 0.01
    m = _model(orc, np.zeros((1, 2)), dx=dx)
    mem = orc.Member.dry(m, h0=np.array([[1.0, 0.0]]))
    orc.step(m, mem, dt)
    # h_flow = 1, slope = -1/dx  =>  q = g dt / dx, not limited
    q = G * dt / dx
    assert mem.qx[0, 1] == pytest.approx(q, rel=1e-14)
    assert mem.qx[0, 0] == 0.0 and mem.qx[0, 2] == 0.0
    assert mem.h[0, 0] == pytest.approx(1.0 - dt / dx * q, rel=1e-14)
    assert mem.h[0, 1] == pytest.approx(dt / dx * q, rel=1e-14)


def test_first_step_flow_depth_uses_higher_bed(orc):
    # Eq. 3: h_flow = max(eta) - max(z); here 1.5 - 1.2 = 0.3 (not 0.5, not the mean)
    dx, dt = 3.0, 0.05
    z = np.array([[1.0, 1.2]])
    m = _model(orc, z, dx=dx)
    mem = orc.Member.dry(m, h0=np.array([[0.5, 0.2]]))
    orc.step(m, mem, dt)
    hf = 0.3
    slope = (1.4 - 1.5) / dx
    assert mem.qx[0, 1] == pytest.approx(-G * hf * dt * slope, rel=1e-12)
    # and the mirrored case flows the other way with the same magnitude
    m2 = _model(orc, z[:, ::-1].copy(), dx=dx)
    mem2 = orc.Member.dry(m2, h0=np.array([[0.2, 0.5]]))
    orc.step(m2, mem2, dt)
    assert mem2.qx[0, 1] == pytest.approx(G * hf * dt * slope, rel=1e-12)


def test_first_step_y_direction_matches_x(orc):
    dx, dt = 3.0, 0.05
    mx = _model(orc, np.array([[1.0, 1.2]]), dx=dx)
    my = _model(orc, np.array([[1.0], [1.2]]), dx=dx)
    a = orc.Member.dry(mx, h0=np.array([[0.5, 0.2]]))
    b = orc.Member.dry(my, h0=np.array([[0.5], [0.2]]))
    orc.step(mx, a, dt)
    orc.step(my, b, dt)
    assert b.qy[1, 0] == a.qx[0, 1]
    np.testing.assert_array_equal(b.h.ravel(), a.h.ravel())


def test_wet_dry_threshold_is_strict(orc):
    dx, dt = 3.0, 0.05
    hd = 1e-3
    m = _model(orc, np.zeros((1, 2)), dx=dx, h_dry=hd)
    mem = orc.Member.dry(m, h0=np.array([[hd, 0.0]]))   # h_flow == h_dry -> no flow
    orc.step(m, mem, dt)
    assert mem.qx[0, 1] == 0.0
    mem = orc.Member.dry(m, h0=np.array([[2 * hd, 0.0]]))
    orc.step(m, mem, dt)
    assert mem.qx[0, 1] > 0.0


def test_single_precision_wet_decision_at_the_float_threshold(orc):
    # h_dry = 1e-3 is not a float; its float rounding lies above it.  A flow depth
    # equal to that float exceeds 1e-3 (wet in double) but is not strictly above
    # the float threshold (dry when decided in float, as a float model decides it)
    dx, dt = 3.0, 0.05
    hf = float(np.float32(1e-3))
    assert hf > 1e-3
    for wet32, expect_flow in ((False, True), (True, False)):
        m = _model(orc, np.zeros((1, 2)), dx=dx, h_dry=1e-3, wet_fp32=wet32)
        mem = orc.Member.dry(m, h0=np.array([[hf, 0.0]]))
        orc.step(m, mem, dt)
        assert (mem.qx[0, 1] > 0.0) == expect_flow
    # the next float up is wet either way; so is an open edge's inner depth
    up = float(np.nextafter(np.float32(hf), np.float32(1.0)))
    m = _model(orc, np.zeros((1, 2)), dx=dx, h_dry=1e-3, wet_fp32=True)
    mem = orc.Member.dry(m, h0=np.array([[up, 0.0]]))
    orc.step(m, mem, dt)
    assert mem.qx[0, 1] > 0.0
    for h0, expect in ((hf, False), (up, True)):
        m = _model(orc, np.zeros((1, 1)), dx=dx, h_dry=1e-3, edges=(0, 1, 0, 0), slopes=(0, 1e-3, 0, 0),
                   wet_fp32=True)
        mem = orc.Member.dry(m, h0=np.array([[h0]]))
        orc.step(m, mem, dt)
        assert (mem.qx[0, 1] > 0.0) == expect


def test_single_precision_wet_decision_changes_nothing_where_floats_are_exact(orc):
    # beds and depths on a 2^-10 lattice below 16 m with h_dry on the lattice: every
    # float operation of the flow depth is exact, so deciding in float or double
    # gives the same links and a bit-identical step
    rng = np.random.default_rng(11)
    ny, nx = 40, 37
    z = rng.integers(0, 4096, size=(ny, nx)) / 1024.0
    h0 = rng.integers(0, 3, size=(ny, nx)) / 1024.0 + rng.integers(0, 2, size=(ny, nx)) * rng.integers(
        0, 600, size=(ny, nx)) / 1024.0
    out = []
    for wet32 in (False, True):
        m = _model(orc, z, dx=3.0, h_dry=1.0 / 1024.0, edges=(1, 1, 1, 1), slopes=(1e-3,) * 4, wet_fp32=wet32)
        mem = orc.Member.dry(m, h0=h0)
        orc.step(m, mem, 0.02)
        out.append((mem.h.copy(), mem.qx.copy(), mem.qy.copy()))
    for a, b in zip(*out):
        np.testing.assert_array_equal(a, b)
    assert np.count_nonzero(out[0][1]) > 50     # the step moved water over many links


def test_donor_limiter_closed_form(orc):
    # single wet cell surrounded by dry cells, long step: every link hits the
    # quarter-cell cap h dx/(4 dt) and the centre cell empties exactly
    dx, dt = 3.0, 1.0
    h0 = np.zeros((3, 3))
    h0[1, 1] = 1.0
    m = _model(orc, np.zeros((3, 3)), dx=dx)
    mem = orc.Member.dry(m, h0=h0)
    orc.step(m, mem, dt)
    cap = 1.0 * dx / (4 * dt)
    assert mem.qx[1, 2] == cap and mem.qx[1, 1] == -cap
    assert mem.qy[2, 1] == cap and mem.qy[1, 1] == -cap
    assert mem.h[1, 1] == 0.0
    for r, c in ((0, 1), (2, 1), (1, 0), (1, 2)):
        assert mem.h[r, c] == pytest.approx(0.25, rel=1e-15)
    assert mem.v_clamp == 0.0


def test_friction_relaxes_to_manning_normal_flow(orc):
    # Two enormous cells: depths change negligibly, so the link discharge relaxes
    # to the fixed point of Eq. 2, Manning's normal flow |q| = h^(5/3) sqrt(S) / n.
    dx = 1e9
    n = 0.03
    z = np.array([[0.0, -dx * 1e-4]])          # bed falls by slope 1e-4 across the link
    m = _model(orc, z, n=n, dx=dx, h_dry=1e-6)
    mem = orc.Member.dry(m, h0=np.array([[1.0, 1.0]]))
    for _ in range(4000):
        orc.step(m, mem, 2.0)
    hf = max(mem.h[0, 0] + z[0, 0], mem.h[0, 1] + z[0, 1]) - max(z[0, 0], z[0, 1])
    S = abs((mem.h[0, 1] + z[0, 1]) - (mem.h[0, 0] + z[0, 0])) / dx
    q_manning = hf ** (5.0 / 3.0) * math.sqrt(S) / n
    assert mem.qx[0, 1] == pytest.approx(q_manning, rel=1e-6)


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------
def test_lake_at_rest_with_islands(orc):
    wl = W.config1(48, 40)
    c = wl.catchments[0]
    z = c.dem.astype(np.float64)
    eta0 = float(np.quantile(z, 0.7))        # some bumps emerge as islands
    h0 = np.maximum(eta0 - z, 0.0)
    assert (h0 == 0).any() and (h0 > 0.5).any()
    m = _model(orc, z, dx=3.0, dt_fixed=0.5)
    mem = orc.Member.dry(m, h0=h0)
    orc.advance(m, mem, 500.0)                # 1000 steps
    assert mem.steps == 1000
    assert np.abs(mem.h - h0).max() <= 1e-12
    assert max(np.abs(mem.qx).max(), np.abs(mem.qy).max()) <= 1e-10


def _ledger_rel(orc, m, mem, s0):
    s = orc.storage(m, mem.h)
    return abs((s - s0) - (mem.v_rain - mem.v_out + mem.v_clamp)) / mem.v_rain


def test_mass_balance_config1(orc):
    wl = W.config1()
    m = orc.Model.from_workload(wl)
    mem = orc.Member.dry(m)
    orc.advance(m, mem, wl.t_end)
    assert mem.t == 600.0
    area = 128 * 128 * 9.0
    v_rain_closed = 50e-3 / 3600.0 * 600.0 * area
    assert mem.v_rain == pytest.approx(v_rain_closed, rel=1e-13)
    assert mem.v_out > 0.0
    assert _ledger_rel(orc, m, mem, 0.0) <= 1e-12
    assert mem.v_clamp <= 1e-14 * mem.v_rain


def test_mass_balance_urban_all_open_edges(orc):
    c = W.urban_catchment("t", 60, 50, 1, W.seed_for(2), n_gauges=2)
    rain = W.chicago_hyetograph()
    m = orc.Model(c.dem, c.manning, 3.0, rain, edge_kind=c.edge_kind, edge_slope=c.edge_slope)
    mem = orc.Member.dry(m, s=1.3, mu=1.7)
    orc.advance(m, mem, 1500.0)
    # rain volume is the closed form of the first five 300 s blocks
    v_closed = 1.7 * rain[:5].sum() * 300.0 * 60 * 50 * 9.0
    assert mem.v_rain == pytest.approx(v_closed, rel=1e-12)
    assert _ledger_rel(orc, m, mem, 0.0) <= 1e-12
    assert mem.v_clamp <= 1e-14 * mem.v_rain


def test_steps_end_exactly_on_events(orc):
    wl = W.config1(32, 32)
    m = orc.Model.from_workload(wl)
    mem = orc.Member.dry(m)
    orc.advance(m, mem, 450.0, log_dt=True)
    assert mem.t == 450.0
    ends = np.cumsum(mem.dt_log)
    # one step ends on the 300 s rain block edge (to rounding of the summation)
    assert np.min(np.abs(ends - 300.0)) < 1e-9
    orc.advance(m, mem, 600.0)
    assert mem.t == 600.0


def _random_state(rng, ny, nx):
    z = rng.uniform(0.0, 0.6, size=(ny, nx))
    h0 = rng.uniform(0.0, 0.4, size=(ny, nx)) * (rng.uniform(size=(ny, nx)) > 0.2)
    return z, h0


@pytest.mark.parametrize("kind", ["transpose", "flip_lr", "flip_ud"])
def test_symmetry(orc, kind):
    rng = np.random.default_rng(7)
    ny, nx = 23, 17
    z, h0 = _random_state(rng, ny, nx)
    ncell = rng.uniform(0.02, 0.05, size=(ny, nx))
    kw = dict(edges=(1, 1, 1, 1), slopes=(1e-3, 2e-3, 3e-3, 4e-3), rain=[1e-4, 3e-5], dt_fixed=0.2)
    m = _model(orc, z, n=ncell, **kw)
    a = orc.Member.dry(m, h0=h0, s=1.1, mu=0.9)
    orc.advance(m, a, 10.0)
    if kind == "transpose":
        f = lambda x: x.T.copy()
        sl = (kw["slopes"][3], kw["slopes"][2], kw["slopes"][1], kw["slopes"][0])   # N<->W, E<->S
    elif kind == "flip_lr":
        f = lambda x: x[:, ::-1].copy()
        sl = (kw["slopes"][0], kw["slopes"][3], kw["slopes"][2], kw["slopes"][1])   # E<->W
    else:
        f = lambda x: x[::-1, :].copy()
        sl = (kw["slopes"][2], kw["slopes"][1], kw["slopes"][0], kw["slopes"][3])   # N<->S
    kw2 = dict(kw)
    kw2["slopes"] = sl
    m2 = _model(orc, f(z), n=f(ncell), **kw2)
    b = orc.Member.dry(m2, h0=f(h0), s=1.1, mu=0.9)
    orc.advance(m2, b, 10.0)
    assert np.abs(f(a.h) - b.h).max() <= 1e-13
    assert b.v_out == pytest.approx(a.v_out, rel=1e-12)


def test_members_are_independent(orc):
    wl = W.config1(24, 20)
    m = orc.Model.from_workload(wl)
    e = orc.Ensemble(m, [1.0, 1.2, 0.8], [1.0, 0.7, 1.4])
    e.advance(200.0)
    solo = orc.Member.dry(m, s=1.2, mu=0.7)
    orc.advance(m, solo, 200.0)
    np.testing.assert_array_equal(e.members[1].h, solo.h)


# ---------------------------------------------------------------------------
# rain-fed inclined plane: exact discrete steady state and Manning outflow
# ---------------------------------------------------------------------------
def _plane_march(ny, dx, s0, n, r, se):
    """Steady depths of a 1-D rain-fed plane solved link by link from the outlet.

    At steady state the discharge through the link below row i is (i+1) r dx
    (rain of every upstream cell), Eq. 2's fixed point balances the surface
    slope against Manning friction, and the open outlet passes its Manning
    normal flow.  Solved here with a scalar root finder, independently of the
    time stepping.
    """
    h = np.zeros(ny)
    q_out = ny * r * dx
    h[ny - 1] = (n * q_out / math.sqrt(se)) ** 0.6
    for i in range(ny - 2, -1, -1):
        q = (i + 1) * r * dx

        def f(hi):
            return hi + s0 * dx - h[i + 1] - dx * n * n * q * q / hi ** (10.0 / 3.0)

        h[i] = brentq(f, 1e-6, 10.0, xtol=1e-15, rtol=1e-15)
    return h


@pytest.mark.parametrize("direction", ["south", "east", "north", "west"])
def test_rain_fed_plane_reaches_discrete_steady_state(orc, direction):
    L, Wd, dx, s0, n = 64, 3, 3.0, 1e-3, 0.03
    r = 50e-3 / 3600.0
    se = 1e-3
    zline = s0 * dx * (L - 1 - np.arange(L))        # falls toward the outlet end
    if direction == "south":
        z = np.repeat(zline[:, None], Wd, axis=1)
        edges, slopes = (0, 0, 1, 0), (0, 0, se, 0)
        prof = lambda h: h[:, 1]
    elif direction == "north":
        z = np.repeat(zline[::-1, None], Wd, axis=1)
        edges, slopes = (1, 0, 0, 0), (se, 0, 0, 0)
        prof = lambda h: h[::-1, 1]
    elif direction == "east":
        z = np.repeat(zline[None, :], Wd, axis=0)
        edges, slopes = (0, 1, 0, 0), (0, se, 0, 0)
        prof = lambda h: h[1, :]
    else:
        z = np.repeat(zline[None, ::-1], Wd, axis=0)
        edges, slopes = (0, 0, 0, 1), (0, 0, 0, se)
        prof = lambda h: h[1, ::-1]
    m = _model(orc, z, n=n, dx=dx, rain=[r] * 100, edges=edges, slopes=slopes, alpha=0.7, h_dry=1e-4,
               dt_cap=2.0)
    mem = orc.Member.dry(m)
    orc.advance(m, mem, 6 * 3600.0)
    h_exact = _plane_march(L, dx, s0, n, r, se)
    got = prof(mem.h)
    assert np.abs(got - h_exact).max() <= 1e-7 * h_exact.max()
    # kinematic-wave sanity check (approximate, since the surface slope is not s0)
    x = (np.arange(L) + 1) * dx
    h_kin = (n * r * x / math.sqrt(s0)) ** 0.6
    assert np.abs(got[L // 2:] / h_kin[L // 2:] - 1).max() < 0.15
    # every column carries the same profile and no cross-slope flow
    assert np.abs(np.diff(mem.h, axis=1 if direction in ("south", "north") else 0)).max() <= 1e-12
