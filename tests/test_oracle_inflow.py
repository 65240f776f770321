"""Pins of the oracle's inflow hydrographs (Sec. 4.1: boundary links at the
stream outlets carry prescribed discharge series).  An inflow link takes the
series value of the current rain block as its inward discharge per unit width,
replacing the edge's wall or open condition on that link.

* Closed flat basin: the stored volume equals the closed-form inflow volume
  (series x block length x cell width, summed), through every edge.
* Sloping channel fed at its head with an open outlet: the state tends to
  uniform flow at Manning's normal depth h = (q n / sqrt(S0))^(3/5), the closed
  form of Eq. 2's fixed point, and the outflow equals the inflow.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore")


def _basin(orc, inflow, q, ny=6, nx=8, edge_kind=(0, 0, 0, 0), n_blocks=3):
    z = np.zeros((ny, nx))
    return orc.Model(z, np.full((ny, nx), 0.03), 3.0, np.zeros(n_blocks), edge_kind=edge_kind,
                     edge_slope=(1e-3,) * 4, inflow=inflow, inflow_q=q)


@pytest.mark.parametrize("kind", [0, 1])
def test_closed_basin_holds_exactly_the_inflow_volume(orc, kind):
    # one link on every edge, two series; walls (kind 0) or open edges (kind 1)
    inflow = [(0, 2, 0), (1, 3, 1), (2, 5, 0), (3, 1, 1)]
    q = np.array([[0.010, 0.000, 0.004], [0.002, 0.006, 0.000]])
    m = _basin(orc, inflow, q, edge_kind=(kind,) * 4)
    mem = orc.Member.dry(m)
    orc.advance(m, mem, 900.0)
    expect = 3.0 * 300.0 * (2 * q[0].sum() + 2 * q[1].sum())
    assert mem.v_in == pytest.approx(expect, rel=1e-13)
    s = orc.storage(m, mem.h)
    assert s == pytest.approx(mem.v_in - mem.v_out + mem.v_clamp, rel=1e-12)
    if kind == 0:
        assert mem.v_out == 0.0 and s == pytest.approx(expect, rel=1e-12)
    else:
        assert mem.v_out > 0.0
    # each inflow link holds its series value with the inward sign
    t_last = 2
    assert mem.qy[0, 2] == q[0, t_last] and mem.qx[3, 8] == -q[1, t_last]
    assert mem.qy[6, 5] == -q[0, t_last] and mem.qx[1, 0] == q[1, t_last]


def test_inflow_ends_with_the_series(orc):
    m = _basin(orc, [(3, 2, 0)], np.array([[0.01, 0.02]]), n_blocks=2)
    mem = orc.Member.dry(m)
    orc.advance(m, mem, 900.0)
    assert mem.v_in == pytest.approx(3.0 * 300.0 * 0.03, rel=1e-13)
    assert mem.qx[2, 0] == 0.0


@pytest.mark.parametrize("q_in", [0.01, 0.02])
def test_channel_tends_to_manning_normal_depth(orc, q_in):
    ny, nx, dx, S0, n = 3, 20, 3.0, 1e-4, 0.05
    c = np.arange(nx)
    z = np.tile(S0 * dx * (nx - c), (ny, 1)).astype(np.float64)
    blocks = 40
    inflow = [(3, r, 0) for r in range(ny)]
    m = orc.Model(z, np.full((ny, nx), n), dx, np.zeros(blocks), edge_kind=(0, 1, 0, 0),
                  edge_slope=(0.0, S0, 0.0, 0.0), inflow=inflow, inflow_q=np.full((1, blocks), q_in))
    mem = orc.Member.dry(m)
    orc.advance(m, mem, 10800.0)
    hn = (q_in * n / np.sqrt(S0)) ** 0.6
    assert np.abs(mem.h / hn - 1.0).max() <= 1e-6
    assert np.abs(mem.qx / q_in - 1.0).max() <= 1e-6          # every x-link, both edges included
    assert np.abs(mem.qy).max() == 0.0
    # outflow rate over one more block equals the inflow rate
    v0, i0 = mem.v_out, mem.v_in
    orc.advance(m, mem, 11100.0)
    assert (mem.v_out - v0) == pytest.approx(mem.v_in - i0, rel=1e-6)
    assert mem.v_in - i0 == pytest.approx(ny * q_in * dx * 300.0, rel=1e-11)   # difference of two sums


def test_invalid_inflow_is_refused(orc):
    z = np.zeros((4, 5))
    for inflow, q in (([(4, 0, 0)], [[0.01]]), ([(0, 5, 0)], [[0.01]]), ([(3, 4, 0)], [[0.01]]),
                      ([(0, 1, 1)], [[0.01]]), ([(0, 1, 0), (0, 1, 0)], [[0.01]]), ([(0, 1, 0)], [[-0.01]])):
        m = orc.Model(z, np.full((4, 5), 0.03), 3.0, np.zeros(1), inflow=inflow, inflow_q=np.array(q))
        with pytest.raises(ValueError):
            orc.advance(m, orc.Member.dry(m), 10.0)


def test_adjoint_refuses_inflow(orc):
    z = np.zeros((4, 6))
    m = orc.Model(z, np.full((4, 6), 0.03), 3.0, np.zeros(1), inflow=[(3, 1, 0)], inflow_q=np.array([[0.01]]))
    with pytest.raises(ValueError):
        orc.adjoint(m, orc.Member.dry(m), 20.0, 10.0, [(1, 1)], np.zeros((2, 1)))


def test_urban_mass_ledger_with_inflow(orc):
    import workloads as W
    c = W.urban_catchment("inf", 30, 36, 1, W.seed_for(2, 53), n_gauges=1, with_inflow=True)
    m = orc.Model(c.dem, c.manning, c.dx, W.chicago_hyetograph(), edge_kind=c.edge_kind, edge_slope=c.edge_slope,
                  inflow=c.inflow, inflow_q=c.inflow_q)
    mem = orc.Member.dry(m, s=c.n_scale[0], mu=c.rain_mult[0])
    orc.advance(m, mem, 1800.0)
    expect_in = 2 * c.dx * 300.0 * c.inflow_q[:, :6].sum()
    assert mem.v_in == pytest.approx(expect_in, rel=1e-12)
    s = orc.storage(m, mem.h)
    assert s == pytest.approx(mem.v_rain + mem.v_in - mem.v_out + mem.v_clamp, rel=1e-12)
    # water of the streams reaches their sections (either way: the terrain decides)
    for sec in c.sections:
        assert orc.section_flow(m, mem, sec) != 0.0
