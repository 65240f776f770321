"""Pins of the oracle's land cover (Sec. 4.1, Table 1): per-member Manning n per
class, runoff coefficient of the rain per class, drainage of draining classes at
a member's rate, and the drained volume in the mass ledger.

Fixed by: the field form it generalises (one class equals a uniform field,
bit for bit), closed forms on closed flat basins (rain times the runoff
coefficient; rain minus drainage, floored at zero), Manning normal flow with
the class mean roughness, and the extended ledger identity.
"""
import numpy as np
import pytest

import workloads as W


def _model(orc, z, cls=None, runoff=None, drain=None, edges=(0, 0, 0, 0), slopes=(0, 0, 0, 0), rain=(),
           n_field=0.03, **kw):
    z = np.asarray(z, dtype=np.float64)
    return orc.Model(z, np.full(z.shape, n_field), 3.0, np.asarray(rain, dtype=np.float64), edge_kind=edges,
                     edge_slope=slopes, land_class=cls, class_runoff=runoff, class_drain=drain, **kw)


def test_one_class_equals_the_uniform_field(orc):
    c = W.urban_catchment("lc1", 30, 26, 1, W.seed_for(2, 31), n_gauges=1)
    rain = W.chicago_hyetograph()
    a = orc.Model(c.dem, np.full(c.dem.shape, 0.035), c.dx, rain, edge_kind=c.edge_kind, edge_slope=c.edge_slope)
    b = orc.Model(c.dem, np.full(c.dem.shape, 0.5), c.dx, rain, edge_kind=c.edge_kind, edge_slope=c.edge_slope,
                  land_class=np.zeros(c.dem.shape, np.uint8), class_runoff=[1.0], class_drain=[0])
    ma = orc.Member.dry(a)
    mb = orc.Member.dry(b, s=7.0, class_n=[0.035])        # the member scale does not apply to class values
    orc.advance(a, ma, 900.0)
    orc.advance(b, mb, 900.0)
    for x, y in ((ma.h, mb.h), (ma.qx, mb.qx), (ma.qy, mb.qy)):
        np.testing.assert_array_equal(x, y)
    assert ma.v_rain == mb.v_rain and mb.v_drain == 0.0


def test_runoff_coefficient_on_a_closed_flat_basin(orc):
    # walls, flat bed, uniform rain: depth = rain depth x runoff coefficient, exactly
    R = 50.0 / 3.6e6
    cls = np.zeros((6, 5), np.uint8)
    cls[2:4, 1:3] = 1
    m = _model(orc, np.zeros((6, 5)), cls, runoff=[1.0, 0.9], drain=[0, 0], rain=[R], dt_fixed=5.0, h_dry=0.01)
    mem = orc.Member.dry(m, class_n=[0.02, 0.15], mu=1.0)
    orc.advance(m, mem, 200.0)
    expect = np.where(cls == 1, 0.9, 1.0) * R * 200.0
    # depths stay below h_dry, so no link carries flow and every cell is alone
    assert expect.max() < 0.01
    np.testing.assert_allclose(mem.h, expect, rtol=1e-13)
    assert mem.v_rain == pytest.approx(expect.sum() * 9.0, rel=1e-13)


@pytest.mark.parametrize("I_mmh", [5.0, 12.0, 80.0])
def test_drainage_closed_form_and_ledger(orc, I_mmh):
    R = 40.0 / 3.6e6
    I = I_mmh / 3.6e6
    cls = np.zeros((5, 7), np.uint8)
    cls[:, 3:] = 1                                    # class 1 drains (hardened ground)
    m = _model(orc, np.zeros((5, 7)), cls, runoff=[1.0, 1.0], drain=[0, 1], rain=[R], dt_fixed=4.0)
    mem = orc.Member.dry(m, class_n=[0.03, 0.017], drain_rate=I)
    orc.advance(m, mem, 60.0)
    # each 4-s step adds R dt and then drains min(I dt, what is there)
    expect_drain_cell = max(0.0, (R - I) * 60.0)
    np.testing.assert_allclose(mem.h[:, 3:], expect_drain_cell, atol=1e-18)
    np.testing.assert_allclose(mem.h[:, :3], R * 60.0, rtol=1e-13)
    drained = min(R, I) * 60.0 * cls.sum() * 9.0
    assert mem.v_drain == pytest.approx(drained, rel=1e-12)
    storage = orc.storage(m, mem.h)
    assert storage == pytest.approx(mem.v_rain - mem.v_out + mem.v_clamp - mem.v_drain, rel=1e-12)


def test_class_roughness_sets_manning_normal_flow(orc):
    # two enormous cells: depths change negligibly, so the link relaxes to Manning's
    # normal flow |q| = h^(5/3) sqrt(S) / n_f with n_f the mean of the two cells'
    # class values for this member
    dx = 1e9
    z = np.array([[0.0, -dx * 1e-4]])
    cls = np.array([[0, 1]], np.uint8)
    m = orc.Model(z, np.full((1, 2), 0.03), dx, np.zeros(0), land_class=cls, class_runoff=[1.0, 1.0],
                  class_drain=[0, 0], h_dry=1e-6)
    mem = orc.Member.dry(m, h0=np.array([[1.0, 1.0]]), class_n=[0.02, 0.05])
    for _ in range(4000):
        orc.step(m, mem, 2.0)
    hf = max(mem.h[0, 0] + z[0, 0], mem.h[0, 1] + z[0, 1]) - max(z[0, 0], z[0, 1])
    S = abs((mem.h[0, 1] + z[0, 1]) - (mem.h[0, 0] + z[0, 0])) / dx
    nf = 0.5 * (0.02 + 0.05)
    assert mem.qx[0, 1] == pytest.approx(hf ** (5.0 / 3.0) * np.sqrt(S) / nf, rel=1e-6)


def test_mass_ledger_with_every_term(orc):
    c = W.urban_catchment("lc2", 28, 24, 1, W.seed_for(2, 32), n_gauges=1)
    rng = np.random.default_rng(6)
    cls = rng.integers(0, 3, size=c.dem.shape).astype(np.uint8)
    rain = W.chicago_hyetograph()
    m = orc.Model(c.dem, c.manning, c.dx, rain, edge_kind=c.edge_kind, edge_slope=c.edge_slope,
                  land_class=cls, class_runoff=[1.0, 0.9, 1.0], class_drain=[1, 0, 0])
    mem = orc.Member.dry(m, class_n=[0.017, 0.15, 0.02], drain_rate=12.0 / 3.6e6)
    orc.advance(m, mem, 1500.0)
    storage = orc.storage(m, mem.h)
    assert mem.v_drain > 0.0 and mem.v_out > 0.0
    assert storage == pytest.approx(mem.v_rain - mem.v_out + mem.v_clamp - mem.v_drain, rel=1e-12)
