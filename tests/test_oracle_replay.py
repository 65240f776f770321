"""Pins of the oracle's replay helpers: link flow depths, wet/dry decision masks,
a step with given wet/dry decisions, and a replay of given step lengths.

These serve trajectory parity (a single-precision model's run replayed in the
FP64 oracle with its step lengths and its links' decisions), so each is pinned
against a hand closed form of Eq. 3, the strict h_dry threshold of the wet/dry
rule, the oracle's own unforced step (identity when the given decisions are the
oracle's), the mass ledger, or a first step from rest in closed form.
"""
import numpy as np
import pytest

import workloads as W

G = 9.81


def _model(orc, z, n=0.03, dx=3.0, rain=(), edges=(0, 0, 0, 0), slopes=(0, 0, 0, 0), **kw):
    z = np.asarray(z, dtype=np.float64)
    nn = np.full(z.shape, n) if np.isscalar(n) else np.asarray(n, dtype=np.float64)
    return orc.Model(z, nn, dx, np.asarray(rain, dtype=np.float64), edge_kind=edges, edge_slope=slopes, **kw)


def test_link_depths_hand_values(orc):
    # Eq. 3: flow depth = higher water surface - higher bed; edges: inner depth
    z = np.array([[0.0, 0.5], [0.25, 0.0]])
    h = np.array([[1.0, 0.25], [0.5, 0.125]])
    m = _model(orc, z)
    hx, hy = orc.link_depths(m, h)
    # x-link (0,1): eta = 1.0, 0.75 -> 1.0 - 0.5;  x-link (1,1): eta = 0.75, 0.125 -> 0.75 - 0.25
    assert hx[0, 1] == 0.5 and hx[1, 1] == 0.5
    # y-link (1,0): eta = 1.0 (north), 0.75 (south) -> 1.0 - 0.25; y-link (1,1): 0.75, 0.125 -> 0.75 - 0.5
    assert hy[1, 0] == 0.75 and hy[1, 1] == 0.25
    # edge links carry the inner cell's depth
    np.testing.assert_array_equal(hx[:, 0], h[:, 0])
    np.testing.assert_array_equal(hx[:, 2], h[:, 1])
    np.testing.assert_array_equal(hy[0, :], h[0, :])
    np.testing.assert_array_equal(hy[2, :], h[1, :])


def test_link_depths_lake_at_rest(orc):
    # a flat surface eta0 over a dyadic bed (every sum exact): each link between two
    # submerged cells has flow depth eta0 - max(z1, z2)
    rng = np.random.default_rng(3)
    z = rng.integers(0, 64, size=(9, 11)) / 64.0
    eta0 = 2.0
    h = eta0 - z
    hx, hy = orc.link_depths(_model(orc, z), h)
    np.testing.assert_array_equal(hx[:, 1:-1], eta0 - np.maximum(z[:, :-1], z[:, 1:]))
    np.testing.assert_array_equal(hy[1:-1, :], eta0 - np.maximum(z[:-1, :], z[1:, :]))


def test_wet_masks_strict_threshold_edges_and_walls(orc):
    hd = 1.0 / 64.0
    z = np.zeros((2, 3))
    h = np.array([[hd, 2 * hd, 0.0], [0.0, hd, 3 * hd]])
    # N, E, S, W: N open, E wall, S open, W wall
    m = _model(orc, z, h_dry=hd, edges=(1, 0, 1, 0), slopes=(1e-3, 0, 1e-3, 0))
    wx, wy = orc.wet_masks(m, h)
    # interior x-links, flat bed: flow depth = max of the two depths, wet iff > h_dry
    assert wx[0, 1] == 1 and wx[0, 2] == 1 and wx[1, 1] == 0 and wx[1, 2] == 1
    # walls take no decision
    assert np.all(wx[:, 0] == 0) and np.all(wx[:, 3] == 0)
    # open north edge: inner depth > h_dry (strict); open south edge likewise
    np.testing.assert_array_equal(wy[0], [0, 1, 0])
    np.testing.assert_array_equal(wy[2], [0, 0, 1])
    # interior y-links: max depths (hd, 0), (2hd, hd), (0, 3hd)
    np.testing.assert_array_equal(wy[1], [0, 1, 1])
    # a flow depth equal to h_dry is dry also when decided in float (hd is a float)
    wx32, wy32 = orc.wet_masks(m, h, fp32=True)
    np.testing.assert_array_equal(wx32, wx)
    np.testing.assert_array_equal(wy32, wy)


def test_wet_masks_at_the_float_threshold(orc):
    # 1e-3 rounds up in float: a depth equal to that float is wet in double, dry in float
    hf = float(np.float32(1e-3))
    m = _model(orc, np.zeros((1, 2)), h_dry=1e-3, edges=(0, 1, 0, 0), slopes=(0, 1e-3, 0, 0))
    h = np.array([[hf, 0.0]])
    wx, _ = orc.wet_masks(m, h)
    wx32, _ = orc.wet_masks(m, h, fp32=True)
    assert wx[0, 1] == 1 and wx32[0, 1] == 0
    h = np.array([[0.0, hf]])                  # the open east edge's inner cell
    assert orc.wet_masks(m, h)[0][0, 2] == 1 and orc.wet_masks(m, h, fp32=True)[0][0, 2] == 0


def test_wet_masks_skip_inflow_links(orc):
    # an inflow link has a prescribed discharge and takes no decision
    z = np.zeros((3, 4))
    h = np.full((3, 4), 0.5)
    inflow = np.array([[0, 1, 0], [3, 2, 0]])            # north edge column 1, west edge row 2
    m = _model(orc, z, edges=(1, 1, 1, 1), slopes=(1e-3,) * 4, rain=[0.0],
               inflow=inflow, inflow_q=np.array([[0.1]]))
    wx, wy = orc.wet_masks(m, h, t=0.0)
    assert wy[0, 1] == 0 and wx[2, 0] == 0
    assert wy[0, 0] == 1 and wy[0, 2] == 1 and wx[1, 0] == 1


def test_masks_are_the_decisions_the_step_takes(orc):
    # from a random state, a link moves water in the next step only where the mask
    # calls it wet, and every wet link with a surface slope moves some
    rng = np.random.default_rng(5)
    ny, nx = 19, 23
    z = rng.uniform(0.0, 0.3, size=(ny, nx))
    h = rng.uniform(0.0, 4e-3, size=(ny, nx)) * (rng.uniform(size=(ny, nx)) > 0.3)
    m = _model(orc, z, edges=(1, 1, 1, 1), slopes=(1e-3,) * 4)
    wx, wy = orc.wet_masks(m, h)
    mem = orc.Member.dry(m, h0=h)
    orc.step(m, mem, 0.05)
    assert np.all(mem.qx[wx == 0] == 0.0) and np.all(mem.qy[wy == 0] == 0.0)
    eta = h + z
    sx = np.zeros((ny, nx + 1))
    sx[:, 1:-1] = eta[:, 1:] - eta[:, :-1]
    sy = np.zeros((ny + 1, nx))
    sy[1:-1, :] = eta[1:, :] - eta[:-1, :]
    inner_x = np.zeros_like(wx, dtype=bool)
    inner_x[:, 1:-1] = True
    inner_y = np.zeros_like(wy, dtype=bool)
    inner_y[1:-1, :] = True
    assert np.all(mem.qx[(wx == 1) & inner_x & (sx != 0)] != 0.0)
    assert np.all(mem.qy[(wy == 1) & inner_y & (sy != 0)] != 0.0)
    assert np.count_nonzero(wx) > 50 and np.count_nonzero(wx == 0) > 50


def test_forced_step_with_own_decisions_is_the_step(orc):
    wl = W.config1(30, 26)
    m = orc.Model.from_workload(wl)
    a = orc.Member.dry(m, mu=3.0)
    orc.advance(m, a, 240.0)
    b = a.copy()
    wx, wy = orc.wet_masks(m, a.h, a.t)
    dt = orc.dt_cfl(m, a.h)
    orc.step(m, a, dt)
    orc.step_forced(m, b, dt, b.t + dt, wx, wy)
    for x, y in ((a.h, b.h), (a.qx, b.qx), (a.qy, b.qy)):
        np.testing.assert_array_equal(x, y)
    assert a.t == b.t and a.v_out == b.v_out and a.v_rain == b.v_rain


def test_forced_decisions_change_only_the_forced_links(orc):
    # first step from rest on a flat-bottomed two-cell tank: a link forced dry carries
    # nothing; a link the state calls dry (flow depth 0 < depth <= h_dry) forced wet
    # carries Eq. 2 from rest, q = -g hf dt S, and the ledger still closes
    dx, dt, hd = 3.0, 0.01, 1e-3
    m = _model(orc, np.zeros((1, 2)), dx=dx, h_dry=hd)
    h0 = np.array([[0.8 * hd, 0.2 * hd]])
    own = orc.wet_masks(m, h0)
    assert own[0][0, 1] == 0
    forced_x = own[0].copy()
    forced_x[0, 1] = 1
    mem = orc.Member.dry(m, h0=h0)
    orc.step_forced(m, mem, dt, dt, forced_x, own[1])
    hf = 0.8 * hd
    S = (0.2 * hd - 0.8 * hd) / dx
    assert mem.qx[0, 1] == pytest.approx(-G * hf * dt * S, rel=1e-14)
    assert mem.h.sum() == pytest.approx(h0.sum(), rel=1e-15)
    # a deep link forced dry carries nothing
    h1 = np.array([[0.5, 0.1]])
    wx, wy = orc.wet_masks(m, h1)
    wx[0, 1] = 0
    mem = orc.Member.dry(m, h0=h1)
    orc.step_forced(m, mem, dt, dt, wx, wy)
    assert mem.qx[0, 1] == 0.0
    np.testing.assert_array_equal(mem.h, h1)


def test_forced_decisions_keep_the_ledger(orc):
    wl = W.config1(28, 24)
    m = orc.Model.from_workload(wl)
    mem = orc.Member.dry(m, mu=2.0)
    s0 = orc.storage(m, mem.h)
    rng = np.random.default_rng(2)
    for _ in range(60):
        wx, wy = orc.wet_masks(m, mem.h, mem.t)
        # flip a few decisions at random: the step stays conservative
        fx = rng.uniform(size=wx.shape) < 0.02
        fy = rng.uniform(size=wy.shape) < 0.02
        wx = np.where(fx, 1 - wx, wx).astype(np.uint8)
        wy = np.where(fy, 1 - wy, wy).astype(np.uint8)
        wx[:, 0] = wx[:, -1] = 0                  # walls stay walls (the south edge is open)
        wy[0, :] = 0
        dt = orc.dt_cfl(m, mem.h)
        orc.step_forced(m, mem, dt, mem.t + dt, wx, wy)
    s = orc.storage(m, mem.h)
    assert abs((s - s0) - (mem.v_rain - mem.v_out + mem.v_clamp)) <= 1e-12 * mem.v_rain


def test_replay_of_logged_steps_is_bit_exact(orc):
    wl = W.config1(26, 22)
    m = orc.Model.from_workload(wl)
    # end times of the steps, one step at a time, and the step lengths of a second run
    a = orc.Member.dry(m, mu=2.5)
    tes = []
    while a.t < 300.0:
        orc.advance(m, a, 300.0, max_steps=1)
        tes.append(a.t)
    b = orc.Member.dry(m, mu=2.5)
    orc.advance(m, b, 300.0, log_dt=True)
    assert len(b.dt_log) == len(tes)
    c = orc.Member.dry(m, mu=2.5)
    orc.replay(m, c, b.dt_log, tes)
    for x, y in ((b.h, c.h), (b.qx, c.qx), (b.qy, c.qy)):
        np.testing.assert_array_equal(x, y)
    assert c.t == b.t == 300.0


def test_double_difference_form_decides_as_written_off_ties(orc):
    # the difference form of Eq. 3 in double equals the literal form except where
    # the flow depth is within a rounding of h_dry; on a dyadic lattice (every
    # operation exact) the two agree everywhere, including exact ties at h_dry
    rng = np.random.default_rng(13)
    ny, nx = 33, 29
    z = rng.integers(0, 4096, size=(ny, nx)) / 1024.0
    hd = 1.0 / 1024.0
    h = rng.integers(0, 4, size=(ny, nx)) / 1024.0
    m = _model(orc, z, h_dry=hd, edges=(1, 1, 1, 1), slopes=(1e-3,) * 4)
    a = orc.wet_masks(m, h)
    b = orc.wet_masks(m, h, mode=orc.MASK_DIFF64)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    hx, hy = orc.link_depths(m, h)
    assert np.count_nonzero(hx == hd) > 10          # exact ties present, dry in both forms
    # off the lattice the two forms still agree away from h_dry
    z2 = rng.uniform(0.0, 4.0, size=(ny, nx))
    h2 = rng.uniform(0.0, 3e-3, size=(ny, nx))
    m2 = _model(orc, z2, h_dry=1e-3, edges=(1, 1, 1, 1), slopes=(1e-3,) * 4)
    a = orc.wet_masks(m2, h2)
    b = orc.wet_masks(m2, h2, mode=orc.MASK_DIFF64)
    hx, hy = orc.link_depths(m2, h2)
    far_x, far_y = np.abs(hx - 1e-3) > 1e-12, np.abs(hy - 1e-3) > 1e-12
    np.testing.assert_array_equal(a[0][far_x], b[0][far_x])
    np.testing.assert_array_equal(a[1][far_y], b[1][far_y])
