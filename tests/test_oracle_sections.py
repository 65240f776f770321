"""Pins of the oracle's streamflow sections (Sec. 4.4: the flow is the sum of
the link fluxes across the observed section) and of the relative observation
error of Sec. 4.4 (Sigma = diag((alpha d_k)^2), alpha = 0.05), with a floor where
an observation is zero.

* Discrete continuity: over one step without clamping, the volume change of any
  rectangle of cells equals dt times the flow through the section made of its
  boundary links, oriented inward, plus the rain on it -- Eq. 1 summed over the
  rectangle, the interior links cancelling.
* Uniform channel flow (Manning normal depth, fed by an inflow hydrograph):
  every cross-section carries the inflow; the reversed section its negative.
* Relative standard deviations: scipy's Gaussian log-density with
  scale max(alpha |d|, floor) and a softmax give the weights and N_eff.
"""
import numpy as np
import pytest
from scipy.stats import norm

import workloads as W


def _rect_section(r0, r1, c0, c1):
    """Boundary links of rows r0..r1, columns c0..c1, oriented into the rectangle."""
    links = []
    for r in range(r0, r1 + 1):
        links.append((0, r, c0, +1))          # west face: x-link c0, +x points inward
        links.append((0, r, c1 + 1, -1))      # east face
    for c in range(c0, c1 + 1):
        links.append((1, r0, c, +1))          # north face
        links.append((1, r1 + 1, c, -1))      # south face
    return links


@pytest.mark.parametrize("rect", [(3, 9, 4, 12), (0, 5, 0, 7), (10, 19, 14, 21), (0, 19, 0, 21)])
def test_rectangle_section_closes_continuity(orc, rect):
    c = W.urban_catchment("sec", 20, 22, 1, W.seed_for(2, 51), n_gauges=1)
    rain = W.chicago_hyetograph()
    m = orc.Model(c.dem, c.manning, c.dx, rain, edge_kind=c.edge_kind, edge_slope=c.edge_slope)
    mem = orc.Member.dry(m, s=c.n_scale[0], mu=c.rain_mult[0])
    orc.advance(m, mem, 1500.0)
    before = mem.copy()
    dt = 0.5
    orc.step(m, mem, dt)
    assert mem.v_clamp == before.v_clamp            # no clamping in this step
    r0, r1, c0, c1 = rect
    q = orc.section_flow(m, mem, _rect_section(*rect))
    dS = (mem.h[r0:r1 + 1, c0:c1 + 1] - before.h[r0:r1 + 1, c0:c1 + 1]).sum() * c.dx ** 2
    rain_rate = mem.mu * rain[int(before.t // 300.0)]
    cells = (r1 - r0 + 1) * (c1 - c0 + 1)
    expect = dt * q + rain_rate * dt * cells * c.dx ** 2
    scale = dt * c.dx * np.abs(mem.qx).sum() + abs(expect)
    assert abs(dS - expect) <= 1e-12 * scale
    assert abs(q) > 0.0
    # the whole grid: the flow through the outer section is minus the outflow
    if rect == (0, 19, 0, 21):
        assert -dt * q == pytest.approx(mem.v_out - before.v_out, rel=1e-12)


def test_channel_cross_sections_carry_the_inflow(orc):
    ny, nx, dx, S0, n, q_in = 3, 20, 3.0, 1e-4, 0.05, 0.015
    z = np.tile(S0 * dx * (nx - np.arange(nx)), (ny, 1)).astype(np.float64)
    m = orc.Model(z, np.full((ny, nx), n), dx, np.zeros(40), edge_kind=(0, 1, 0, 0),
                  edge_slope=(0.0, S0, 0.0, 0.0), inflow=[(3, r, 0) for r in range(ny)],
                  inflow_q=np.full((1, 40), q_in))
    mem = orc.Member.dry(m)
    orc.advance(m, mem, 10800.0)
    for col in (0, 7, 20):
        sec = [(0, r, col, +1) for r in range(ny)]
        assert orc.section_flow(m, mem, sec) == pytest.approx(ny * q_in * dx, rel=1e-6)
        assert orc.section_flow(m, mem, [(k, r, c, -s) for k, r, c, s in sec]) == pytest.approx(-ny * q_in * dx,
                                                                                                rel=1e-6)
    along = [(1, r, 5, +1) for r in range(ny + 1)]
    assert orc.section_flow(m, mem, along) == 0.0


def test_section_validation(orc):
    m = orc.Model(np.zeros((3, 4)), np.full((3, 4), 0.03), 3.0, np.zeros(1))
    mem = orc.Member.dry(m)
    for bad in ([(0, 3, 0, 1)], [(0, 0, 5, 1)], [(1, 4, 0, 1)], [(1, 0, 4, 1)], [(2, 0, 0, 1)], [(0, 0, 0, 2)]):
        with pytest.raises(ValueError):
            orc.section_flow(m, mem, bad)


def test_relative_sigma_and_floor(orc):
    d = np.array([0.4, 0.0, -2.0, 1e-4, 12.0])
    floor = np.array([0.01, 0.02, 0.01, 0.01, 0.5])
    np.testing.assert_allclose(orc.obs_sigma(d, floor, 0.05), [0.02, 0.02, 0.1, 0.01, 0.6], rtol=1e-15, atol=0)
    np.testing.assert_array_equal(orc.obs_sigma(d, floor, 0.0), floor)
    with pytest.raises(ValueError):
        orc.obs_sigma(d, np.zeros(5), 0.05)      # zero observation with no floor


def test_relative_sigma_weights_match_scipy(orc):
    rng = np.random.default_rng(17)
    N, K = 24, 5
    d = np.array([0.3, 0.0, 0.8, 2.5, 40.0])     # three depths (one dry), two flows
    y = d + rng.normal(0.0, 0.05, size=(N, K)) * np.maximum(np.abs(d), 0.1)
    floor = np.array([0.01, 0.01, 0.01, 0.05, 0.05])
    lw0 = np.log(rng.uniform(0.5, 1.5, N))
    lw0 -= np.log(np.exp(lw0).sum())
    lp, w, neff = orc.pf_weights(y, d, floor, lw0, alpha=0.05)
    sig = np.maximum(0.05 * np.abs(d), floor)
    a = lw0 + norm.logpdf(y, d, sig).sum(axis=1)
    ref = np.exp(a - a.max())
    ref /= ref.sum()
    np.testing.assert_allclose(w, ref, rtol=1e-12, atol=1e-300)
    assert neff == pytest.approx(1.0 / (ref ** 2).sum(), rel=1e-12)
    # alpha = 0 is the absolute form with sigma = floor
    _, w0, _ = orc.pf_weights(y, d, floor, lw0)
    a0 = lw0 + norm.logpdf(y, d, floor).sum(axis=1)
    r0 = np.exp(a0 - a0.max())
    np.testing.assert_allclose(w0, r0 / r0.sum(), rtol=1e-12, atol=1e-300)


def test_ensemble_assimilates_depths_and_flows(orc):
    # the flows enter the likelihood after the depths, with their own sigma
    c = W.urban_catchment("sec2", 16, 18, 4, W.seed_for(2, 52), n_gauges=2)
    m = orc.Model(c.dem, c.manning, c.dx, W.chicago_hyetograph(), edge_kind=c.edge_kind, edge_slope=c.edge_slope)
    e = orc.Ensemble(m, c.n_scale[:4], c.rain_mult[:4])
    e.advance(1200.0)
    secs = [_rect_section(2, 8, 2, 9), [(0, r, 9, 1) for r in range(16)]]
    yh = orc.gauge_values(e.members, c.gauges)
    yq = np.array([[orc.section_flow(m, mm, s) for s in secs] for mm in e.members])
    obs = np.concatenate([yh[1], yq[1]])
    floor = np.full(obs.size, 1e-3)
    lw0 = e.logw.copy()
    _, w_ref, neff_ref = orc.pf_weights(np.concatenate([yh, yq], axis=1), obs, floor, lw0, alpha=0.05)
    neff, anc, res = e.assimilate(c.gauges, obs, floor, 1e-9, 0.5, sections=secs, alpha=0.05)
    assert not res and neff == pytest.approx(neff_ref, rel=1e-14)
    np.testing.assert_allclose(np.exp(e.logw), w_ref, rtol=1e-13)
