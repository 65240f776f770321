"""Pins of the oracle's discrete adjoint.

The adjoint is checked against central finite differences of the oracle's own
forward step and loss (a different code path from the reverse sweep), with the
step sequence frozen to the recorded one, and for independence from the
checkpoint interval.
"""
import numpy as np
import pytest

import workloads as W


def _wet_model(orc, rng, ny, nx, rain=(2e-4, 1e-4), n=None, edges=(1, 1, 1, 1)):
    z = rng.uniform(0.0, 0.3, size=(ny, nx))
    nn = rng.uniform(0.02, 0.05, size=(ny, nx)) if n is None else n
    m = orc.Model(z, nn, 3.0, np.asarray(rain), rain_interval=20.0, edge_kind=edges,
                  edge_slope=(1e-3, 2e-3, 3e-3, 1.5e-3), h_dry=1e-3, alpha=0.5, dt_cap=5.0)
    return m, z, nn


def _state(orc, m, rng, s=1.1, mu=0.8):
    mem = orc.Member.dry(m, s=s, mu=mu, h0=rng.uniform(0.3, 0.6, size=(m.ny, m.nx)))
    mem.qx[:] = rng.uniform(-0.05, 0.05, size=mem.qx.shape)
    mem.qy[:] = rng.uniform(-0.05, 0.05, size=mem.qy.shape)
    # walls carry no flow; open edges flow outward
    mem.qx[:, 0] = -np.abs(mem.qx[:, 0])
    mem.qx[:, -1] = np.abs(mem.qx[:, -1])
    mem.qy[0, :] = -np.abs(mem.qy[0, :])
    mem.qy[-1, :] = np.abs(mem.qy[-1, :])
    mem.t = 5.0
    return mem


def _step_out(orc, m, mem, dt):
    x = mem.copy()
    orc.step(m, x, dt)
    return np.concatenate([x.h.ravel(), x.qx.ravel(), x.qy.ravel()])


@pytest.mark.parametrize("what", ["h", "qx", "qy", "n", "mu"])
def test_single_step_transpose(orc, what):
    rng = np.random.default_rng(11)
    ny, nx = 9, 7
    m, z, nn = _wet_model(orc, rng, ny, nx)
    mem = _state(orc, m, rng)
    dt = 0.2
    wv = rng.standard_normal(ny * nx + ny * (nx + 1) + (ny + 1) * nx)
    lh = wv[:ny * nx].reshape(ny, nx)
    lqx = wv[ny * nx:ny * nx + ny * (nx + 1)].reshape(ny, nx + 1)
    lqy = wv[ny * nx + ny * (nx + 1):].reshape(ny + 1, nx)
    ah, aqx, aqy, gn, gmu = orc.adj_step(m, mem, dt, lh, lqx, lqy)
    eps = 1e-6
    if what in ("h", "qx", "qy"):
        arr = getattr(mem, what)
        v = rng.standard_normal(arr.shape)
        p, q = mem.copy(), mem.copy()
        getattr(p, what)[:] += eps * v
        getattr(q, what)[:] -= eps * v
        fd = wv @ (_step_out(orc, m, p, dt) - _step_out(orc, m, q, dt)) / (2 * eps)
        ad = {"h": ah, "qx": aqx, "qy": aqy}[what].ravel() @ v.ravel()
    elif what == "n":
        v = rng.standard_normal((ny, nx))
        mp = orc.Model(z, nn + eps * v, 3.0, np.array([2e-4, 1e-4]), rain_interval=20.0, edge_kind=(1, 1, 1, 1),
                       edge_slope=(1e-3, 2e-3, 3e-3, 1.5e-3), h_dry=1e-3)
        mm = orc.Model(z, nn - eps * v, 3.0, np.array([2e-4, 1e-4]), rain_interval=20.0, edge_kind=(1, 1, 1, 1),
                       edge_slope=(1e-3, 2e-3, 3e-3, 1.5e-3), h_dry=1e-3)
        fd = wv @ (_step_out(orc, mp, mem, dt) - _step_out(orc, mm, mem, dt)) / (2 * eps)
        ad = gn.ravel() @ v.ravel()
    else:
        p, q = mem.copy(), mem.copy()
        p.mu += eps
        q.mu -= eps
        fd = wv @ (_step_out(orc, m, p, dt) - _step_out(orc, m, q, dt)) / (2 * eps)
        ad = gmu
    assert ad == pytest.approx(fd, rel=2e-7)


def test_single_step_transpose_with_limiter_and_dry_links(orc):
    # a step long enough for donor limiting, with dry cells next to wet ones
    rng = np.random.default_rng(5)
    ny, nx = 8, 8
    m, z, nn = _wet_model(orc, rng, ny, nx)
    mem = _state(orc, m, rng)
    mem.h[2:5, 2:5] = 0.0
    mem.h[6, 6] = 2e-3
    dt = 2.5
    wv = rng.standard_normal(ny * nx + ny * (nx + 1) + (ny + 1) * nx)
    sizes = [ny * nx, ny * (nx + 1), (ny + 1) * nx]
    lh, lqx, lqy = (wv[:sizes[0]].reshape(ny, nx), wv[sizes[0]:sizes[0] + sizes[1]].reshape(ny, nx + 1),
                    wv[sizes[0] + sizes[1]:].reshape(ny + 1, nx))
    ah, aqx, aqy, gn, gmu = orc.adj_step(m, mem, dt, lh, lqx, lqy)
    v = rng.standard_normal((ny, nx))
    v[mem.h == 0] = 0.0          # perturbing a dry cell upward would change the branch
    eps = 1e-7
    p, q = mem.copy(), mem.copy()
    p.h += eps * v
    q.h -= eps * v
    fd = wv @ (_step_out(orc, m, p, dt) - _step_out(orc, m, q, dt)) / (2 * eps)
    assert ah.ravel() @ v.ravel() == pytest.approx(fd, rel=1e-6)


def _loss_setup(orc, seed=21, ny=14, nx=11, t_end=40.0):
    # sloped bed and smooth initial depth: every link keeps its flow direction, so
    # the flow depth of Eq. 3 stays away from its max() kink under small perturbations
    rng = np.random.default_rng(seed)
    r = np.arange(ny)[:, None]
    c = np.arange(nx)[None, :]
    z = 0.02 * (r + 0.7 * c) + rng.uniform(0.0, 0.003, size=(ny, nx))
    nn = rng.uniform(0.02, 0.05, size=(ny, nx))
    m = orc.Model(z, nn, 3.0, np.array([2e-4, 1e-4]), rain_interval=20.0, edge_kind=(1, 1, 1, 1),
                  edge_slope=(1e-3, 2e-3, 3e-3, 1.5e-3), h_dry=1e-3, alpha=0.5, dt_cap=5.0)
    mem0 = orc.Member.dry(m, s=1.05, mu=1.3, h0=0.4 + rng.uniform(0.0, 0.01, size=(ny, nx)))
    g = np.array([[3, 4], [9, 2], [12, 9]], dtype=np.int32)
    obs = rng.uniform(0.3, 0.5, size=(int(t_end / 10.0), 3))
    return m, z, nn, mem0, g, obs


def test_loss_gradient_matches_central_differences(orc):
    m, z, nn, mem0, g, obs = _loss_setup(orc)
    L, gn, gmu, rec = orc.adjoint(m, mem0.copy(), 40.0, 10.0, g, obs, ckpt_every=7)
    assert len(rec[0]) > 30
    # rain multiplier
    eps = 1e-4 * mem0.mu
    p, q = mem0.copy(), mem0.copy()
    p.mu += eps
    q.mu -= eps
    fd = (orc.loss(m, p, 40.0, 10.0, g, obs, replay=rec) - orc.loss(m, q, 40.0, 10.0, g, obs, replay=rec)) / (2 * eps)
    assert gmu == pytest.approx(fd, rel=1e-6)
    # Manning field: random direction and two single cells
    rng = np.random.default_rng(0)
    for v in (rng.standard_normal(nn.shape), np.eye(1, nn.size, 40).reshape(nn.shape),
              np.eye(1, nn.size, 100).reshape(nn.shape)):
        e = 1e-4 * 0.03

        def Lof(nf):
            mm = orc.Model(z, nf, 3.0, np.array([2e-4, 1e-4]), rain_interval=20.0, edge_kind=(1, 1, 1, 1),
                           edge_slope=(1e-3, 2e-3, 3e-3, 1.5e-3), h_dry=1e-3, alpha=0.5, dt_cap=5.0)
            return orc.loss(mm, mem0.copy(), 40.0, 10.0, g, obs, replay=rec)

        fd = (Lof(nn + e * v) - Lof(nn - e * v)) / (2 * e)
        assert float(np.sum(gn * v)) == pytest.approx(fd, rel=1e-5, abs=1e-12 * abs(L))


def test_replay_reproduces_the_recorded_forward(orc):
    m, z, nn, mem0, g, obs = _loss_setup(orc)
    L, gn, gmu, rec = orc.adjoint(m, mem0.copy(), 40.0, 10.0, g, obs, ckpt_every=7)
    assert orc.loss(m, mem0.copy(), 40.0, 10.0, g, obs) == L
    assert orc.loss(m, mem0.copy(), 40.0, 10.0, g, obs, replay=rec) == L


def test_checkpoint_interval_does_not_change_gradients(orc):
    m, z, nn, mem0, g, obs = _loss_setup(orc)
    ref = orc.adjoint(m, mem0.copy(), 40.0, 10.0, g, obs, ckpt_every=1)
    for k in (3, 100):
        got = orc.adjoint(m, mem0.copy(), 40.0, 10.0, g, obs, ckpt_every=k)
        assert got[0] == ref[0] and got[2] == ref[2]
        np.testing.assert_array_equal(got[1], ref[1])


def test_urban_rain_event_gradient_fd(orc):
    # Urban terrain after 20 min of rain: wet/dry fronts, puddles against buildings.
    # The adjoint is the derivative of the step map with its branches (wet/dry,
    # limiter, clamp, which surface is higher) frozen.  A perturbation of 1e-3 in
    # the rain multiplier flips some of those branches here, so the finite
    # difference is taken at 1e-5, where no branch flips.
    c = W.urban_catchment("adj", 24, 20, 1, W.seed_for(3), n_gauges=4)
    rain = W.chicago_hyetograph()
    m = orc.Model(c.dem, c.manning, 3.0, rain, edge_kind=c.edge_kind, edge_slope=c.edge_slope)
    mem0 = orc.Member.dry(m, s=1.0, mu=1.0)
    orc.advance(m, mem0, 1200.0)
    obs = np.random.default_rng(1).uniform(0.0, 0.05, size=(12, 4))
    L, gn, gmu, rec = orc.adjoint(m, mem0.copy(), 1320.0, 10.0, c.gauges, obs, ckpt_every=50)

    def fd(eps):
        p, q = mem0.copy(), mem0.copy()
        p.mu += eps
        q.mu -= eps
        return (orc.loss(m, p, 1320.0, 10.0, c.gauges, obs, replay=rec)
                - orc.loss(m, q, 1320.0, 10.0, c.gauges, obs, replay=rec)) / (2 * eps)

    assert gmu == pytest.approx(fd(1e-5), rel=1e-6)
    assert gmu == pytest.approx(fd(1e-6), rel=1e-6)
