"""GPU inflow hydrographs, streamflow sections and the relative observation error
(Sec. 4.1, Sec. 4.4) against the FP64 oracle, through the C ABI.

Bars: FP64 trajectories 1e-9 m and 1e-9 of the largest discharge, inflow and
outflow ledger 1e-10 relative, balance 1e-12 (FP32 trajectories are held by
replay in tests/test_gpu_trajectory.py);
one FP32 step from an identical float state 1e-6 m + 4 ulp; the section operator on the
GPU's own discharges 1e-12 of the sum of |q| dx (FP64 sums in another order);
weights 1e-12 and N_eff 1e-12 from the GPU's own observations, ancestors
bit-exact given the weights; Manning normal depth of a fed channel 1e-6.
"""
import os
import tempfile

import numpy as np
import pytest

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


CAT = W.urban_catchment("inf", 45, 64, 4, W.seed_for(2, 61), n_gauges=3, with_inflow=True)   # nx % 4 == 0
RAIN = W.chicago_hyetograph()


def _cat(members=None, sections=True):
    c = CAT
    idx = np.arange(4) if members is None else np.asarray(members)
    d = dict(dem=c.dem, manning=c.manning, dx=c.dx, edge_kind=c.edge_kind, edge_slope=c.edge_slope,
             n_members=len(idx), n_scale=c.n_scale[idx], rain_mult=c.rain_mult[idx], inflow=c.inflow,
             inflow_q=c.inflow_q)
    if sections:
        d["sections"] = c.sections
    return d


def _oracle(orc, i, t_end, mu_factor=1.0, **kw):
    c = CAT
    m = orc.Model(c.dem, c.manning, c.dx, RAIN, edge_kind=c.edge_kind, edge_slope=c.edge_slope,
                  inflow=c.inflow, inflow_q=c.inflow_q, **kw)
    mem = orc.Member.dry(m, s=c.n_scale[i], mu=c.rain_mult[i] * mu_factor)
    orc.advance(m, mem, t_end)
    return m, mem


def _secs(orc, m, mem):
    return np.array([orc.section_flow(m, mem, s) for s in CAT.sections])


def test_fp64_trajectory_ledger_and_sections_match_oracle(fl, orc):
    e = fl.FloodEnsemble([_cat()], RAIN, real_bytes=8)
    e.step(1500.0)
    led = e.ledger()
    q_gpu = e.sections()
    for i in range(4):
        m, mem = _oracle(orc, i, 1500.0)
        assert np.abs(e.field(i) - mem.h).max() <= 1e-9
        qs = max(np.abs(mem.qx).max(), np.abs(mem.qy).max())
        assert np.abs(e.field(i, fl.FIELD_QX) - mem.qx).max() <= 1e-9 * qs
        assert np.abs(e.field(i, fl.FIELD_QY) - mem.qy).max() <= 1e-9 * qs
        assert led["steps"][i] == mem.steps
        assert led["inflow"][i] == pytest.approx(mem.v_in, rel=1e-12)
        assert led["outflow"][i] == pytest.approx(mem.v_out, rel=1e-10)
        assert led["rain_in"][i] == pytest.approx(mem.v_rain, rel=1e-12)
        ref = _secs(orc, m, mem)
        assert np.abs(q_gpu[i] - ref).max() <= 1e-9 * np.abs(ref).max()
    # the inflow follows the series: two links per stream, 300-s blocks
    assert led["inflow"][0] == pytest.approx(2 * CAT.dx * 300.0 * CAT.inflow_q[:, :5].sum(), rel=1e-12)
    resid = np.abs(led["storage"] - (led["rain_in"] + led["inflow"] - led["outflow"] + led["clamp"]))
    assert (resid / (led["rain_in"] + led["inflow"])).max() <= 1e-12


def test_one_step_from_an_identical_float_state(fl, orc):
    # inflow links are active at 1200 s; one step from the oracle's state rounded
    # to float, float wet/dry decisions on both sides
    m, mem = _oracle(orc, 1, 1200.0)
    h32, qx32, qy32 = (a.astype(np.float32).astype(np.float64) for a in (mem.h, mem.qx, mem.qy))
    e = fl.FloodEnsemble([_cat()], RAIN, real_bytes=4)
    e.set_state(1, h32, qx32, qy32, 1200.0)
    e.step(1200.0)
    dt = 0.05
    e.step(1200.0 + dt)
    m32, _ = _oracle(orc, 1, 0.0, wet_fp32=True)
    ref = orc.Member(h32.copy(), qx32.copy(), qy32.copy(), t=1200.0, s=CAT.n_scale[1], mu=CAT.rain_mult[1])
    orc.step(m32, ref, dt)
    tol = 1e-6 + 4.0 * np.spacing(np.abs(ref.h).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(e.field(1) - ref.h) <= tol)
    qs = max(np.abs(ref.qx).max(), np.abs(ref.qy).max())
    assert np.abs(e.field(1, fl.FIELD_QX) - ref.qx).max() <= 1e-5 * qs
    assert np.abs(e.field(1, fl.FIELD_QY) - ref.qy).max() <= 1e-5 * qs
    # the inflow links hold their series value (rounded to float)
    q = CAT.inflow_q[:, 4]
    for (edge, pos, j) in CAT.inflow:
        assert edge == 0 and e.field(1, fl.FIELD_QY)[0, pos] == np.float32(q[j])


@pytest.mark.parametrize("mi", [1, 2, 4])
def test_section_operator_on_the_gpu_fields(fl, orc, mi):
    # sections of every kind of link (edge strips, interior, both signs) on the
    # GPU's own discharges; interleaved layouts without inflow links
    c = CAT
    cat = dict(dem=c.dem, manning=c.manning, dx=c.dx, edge_kind=c.edge_kind, edge_slope=c.edge_slope,
               n_members=4, n_scale=c.n_scale[:4], rain_mult=c.rain_mult[:4])
    ny, nx = c.ny, c.nx
    secs = [np.array([(0, r, 0, 1) for r in range(ny)]),                     # west edge
            np.array([(0, r, nx, -1) for r in range(ny)]),                   # east edge, outward
            np.array([(1, 0, cc, 1) for cc in range(nx)] + [(1, ny, cc, -1) for cc in range(nx)]),
            np.array([(0, r, 17, 1) for r in range(5, 30)] + [(1, 12, cc, -1) for cc in range(3, 40)]),
            c.sections[0]]
    e = fl.FloodEnsemble([cat], RAIN, real_bytes=4, member_interleave=mi, step_kernel=1 if mi > 1 else 0)
    e.step(1200.0)
    e.set_sections(secs)
    q = e.sections()
    m = orc.Model(c.dem, c.manning, c.dx, RAIN)
    for i in range(4):
        mem = orc.Member(e.field(i), e.field(i, fl.FIELD_QX), e.field(i, fl.FIELD_QY))
        ref = np.array([orc.section_flow(m, mem, s) for s in secs])
        mag = np.array([c.dx * sum(abs(mem.qx[r, cc] if k == 0 else mem.qy[r, cc]) for k, r, cc, _ in s)
                        for s in secs])
        assert np.all(np.abs(q[i] - ref) <= 1e-12 * mag + 1e-300)
    assert np.any(np.abs(q) > 0)


def test_filter_on_depths_and_flows_with_relative_error(fl, orc):
    e = fl.FloodEnsemble([_cat()], RAIN, real_bytes=4)
    e.step(1200.0)
    g = CAT.gauges
    yh = np.array([e.field(i)[g[:, 0], g[:, 1]] for i in range(4)])
    yq = e.sections()
    y = np.concatenate([yh, yq], axis=1)
    obs = y[2] * np.array([1.03, 0.97, 1.0, 1.02, 0.99])
    obs[1] = 0.0                                   # a dry gauge: the floor applies
    floor = np.array([0.01, 0.01, 0.01, 0.05, 0.05])
    lw0 = e.weights()[0]
    neff, _, res = e.assimilate_obs(0, g, obs, floor, alpha=0.05, neff_frac=1e-9)
    assert not res
    _, w_ref, neff_ref = orc.pf_weights(y, obs, floor, lw0, alpha=0.05)
    np.testing.assert_allclose(np.exp(e.weights()[0]), w_ref, rtol=1e-12, atol=1e-300)
    assert neff == pytest.approx(neff_ref, rel=1e-12)
    # absolute form: alpha = 0 uses sigma as given
    e2 = fl.FloodEnsemble([_cat()], RAIN, real_bytes=4)
    e2.step(1200.0)
    e2.assimilate_obs(0, g, obs, floor, alpha=0.0, neff_frac=1e-9)
    _, w_abs, _ = orc.pf_weights(y, obs, floor, lw0)
    np.testing.assert_allclose(np.exp(e2.weights()[0]), w_abs, rtol=1e-12, atol=1e-300)
    # resampling moves the inflow ledger with the members
    led0 = e.ledger()
    neff, anc, res = e.assimilate_obs(0, g, y[1], np.full(5, 1e-6), alpha=0.0, neff_frac=1.0)
    assert res
    np.testing.assert_array_equal(e.ledger()["inflow"], led0["inflow"][anc])


def test_channel_reaches_manning_normal_depth_on_the_gpu(fl):
    ny, nx, dx, S0, n, q_in = 3, 20, 3.0, 1e-4, 0.05, 0.02
    z = np.tile(S0 * dx * (nx - np.arange(nx)), (ny, 1)).astype(np.float32)
    cat = dict(dem=z, manning=np.full((ny, nx), n, np.float32), dx=dx, edge_kind=(0, 1, 0, 0),
               edge_slope=(0.0, S0, 0.0, 0.0), n_members=2, inflow=[(3, r, 0) for r in range(ny)],
               inflow_q=np.full((1, 40), q_in), sections=[[(0, r, 10, 1) for r in range(ny)]])
    e = fl.FloodEnsemble([cat], np.zeros(40), real_bytes=8)
    e.step(10800.0)
    hn = (q_in * n / np.sqrt(float(np.float32(S0 * dx)) / dx)) ** 0.6
    for i in range(2):
        assert np.abs(e.field(i) / hn - 1.0).max() <= 1e-5
        assert np.abs(e.field(i, fl.FIELD_QX) / q_in - 1.0).max() <= 1e-5
    np.testing.assert_allclose(e.sections()[:, 0], ny * q_in * dx, rtol=1e-5)


def test_batched_equals_one_handle_and_snapshots(fl):
    other = W.urban_catchment("o", 32, 40, 3, W.seed_for(2, 62), n_gauges=2)
    oc = dict(dem=other.dem, manning=other.manning, dx=other.dx, edge_kind=other.edge_kind,
              edge_slope=other.edge_slope, n_members=3, n_scale=other.n_scale, rain_mult=other.rain_mult)
    b = fl.FloodEnsemble([oc, _cat()], RAIN, real_bytes=4)
    b.step(900.0)
    p = fl.FloodEnsemble([_cat()], RAIN, real_bytes=4)
    p.step(900.0)
    for i in range(4):
        np.testing.assert_array_equal(b.field(i, catchment=1), p.field(i))
    np.testing.assert_array_equal(b.ledger(1)["inflow"], p.ledger()["inflow"])
    np.testing.assert_array_equal(b.sections(1), p.sections())
    path = os.path.join(tempfile.mkdtemp(), "inf.bin")
    p.save(path)
    p.step(1200.0)
    p.load(path)
    np.testing.assert_array_equal(p.ledger()["inflow"], b.ledger(1)["inflow"])
    np.testing.assert_array_equal(p.field(2), b.field(2, catchment=1))


def test_refusals(fl):
    e = fl.FloodEnsemble([_cat()], RAIN, real_bytes=4)
    with pytest.raises(fl.FloodError) as ex:
        e.adjoint(0, 20.0, 10.0, CAT.gauges, np.zeros((2, 3)), ckpt_every=5)
    assert ex.value.status == fl.FLOOD_EINVAL
    for kw in (dict(step_kernel=1), dict(step_kernel=2), dict(member_interleave=2)):
        with pytest.raises(fl.FloodError) as ex:
            fl.FloodEnsemble([_cat()], RAIN, real_bytes=4, **kw)
        assert ex.value.status == fl.FLOOD_EINVAL
    ny, nx = CAT.ny, CAT.nx
    for bad in ([[(0, ny, 0, 1)]], [[(0, 0, nx + 1, 1)]], [[(1, ny + 1, 0, 1)]], [[(1, 0, nx, 1)]],
                [[(2, 0, 0, 1)]], [[(0, 0, 0, 0)]], [np.zeros((0, 4))], [[(0, 0, 0, 1)]] * 65):
        with pytest.raises(fl.FloodError) as ex:
            e.set_sections(bad)
        assert ex.value.status == fl.FLOOD_EINVAL
    g = CAT.gauges
    with pytest.raises(fl.FloodError) as ex:
        e.assimilate_obs(0, g, np.zeros(5), np.full(5, 0.01), alpha=-0.1)
    assert ex.value.status == fl.FLOOD_EINVAL
    with pytest.raises(fl.FloodError) as ex:
        e.assimilate_obs(0, g, np.zeros(5), np.array([0.01, 0.01, 0.0, 0.01, 0.01]), alpha=0.05)
    assert ex.value.status == fl.FLOOD_EINVAL
    e.set_sections([])
    with pytest.raises(fl.FloodError) as ex:
        e.sections()
    assert ex.value.status == fl.FLOOD_ESTATE


@pytest.mark.parametrize("rb", [8, 4])
def test_inflow_on_every_edge_matches_oracle(fl, orc, rb):
    # inflow links on all four edges (corners included) and over walls and open
    # edges, on a grid whose width spans two strips with a ragged tail; FP64 over
    # the run, FP32 one step from the same float state
    ny, nx = 37, 264
    rng = np.random.default_rng(W.seed_for(2, 63))
    z = (np.add.outer(np.linspace(0, 1.5, ny), np.linspace(0, 0.8, nx)) + rng.uniform(0, 0.3, (ny, nx)))
    z = z.astype(np.float32)
    n = np.full((ny, nx), 0.03, np.float32)
    inflow = [(0, 0, 0), (0, 131, 1), (0, nx - 1, 2), (1, 0, 3), (1, 17, 0), (1, ny - 1, 1),
              (2, 5, 2), (2, nx - 1, 3), (3, 0, 1), (3, ny - 1, 2), (3, 20, 0)]
    q = np.array([[0.02, 0.05, 0.0, 0.01], [0.03, 0.0, 0.04, 0.02], [0.0, 0.01, 0.02, 0.03],
                  [0.05, 0.05, 0.01, 0.0]])
    edge_kind, edge_slope = (1, 0, 1, 0), (1e-3, 0.0, 1e-3, 0.0)
    rain = np.array([20.0, 40.0, 10.0, 0.0]) / 3.6e6
    cat = dict(dem=z, manning=n, dx=3.0, edge_kind=edge_kind, edge_slope=edge_slope, n_members=2,
               n_scale=np.array([1.0, 1.2]), rain_mult=np.array([1.0, 0.8]), inflow=inflow, inflow_q=q)
    e = fl.FloodEnsemble([cat], rain, real_bytes=rb)
    m = orc.Model(z, n, 3.0, rain, edge_kind=edge_kind, edge_slope=edge_slope, inflow=inflow, inflow_q=q)
    if rb == 8:
        e.step(1000.0)
        led = e.ledger()
        for i, (s, mu) in enumerate(((1.0, 1.0), (1.2, 0.8))):
            mem = orc.Member.dry(m, s=s, mu=mu)
            orc.advance(m, mem, 1000.0)
            assert np.abs(e.field(i) - mem.h).max() <= 1e-9
            qs = max(np.abs(mem.qx).max(), np.abs(mem.qy).max())
            assert np.abs(e.field(i, fl.FIELD_QX) - mem.qx).max() <= 1e-9 * qs
            assert np.abs(e.field(i, fl.FIELD_QY) - mem.qy).max() <= 1e-9 * qs
            assert led["inflow"][i] == pytest.approx(mem.v_in, rel=1e-12)
            assert led["outflow"][i] == pytest.approx(mem.v_out, rel=1e-10)
        return
    mem = orc.Member.dry(m, s=1.2, mu=0.8)
    orc.advance(m, mem, 700.0)
    h32, qx32, qy32 = (a.astype(np.float32).astype(np.float64) for a in (mem.h, mem.qx, mem.qy))
    e.set_state(1, h32, qx32, qy32, 700.0)
    e.step(700.0)
    dt = 0.05
    e.step(700.0 + dt)
    m32 = orc.Model(z, n, 3.0, rain, edge_kind=edge_kind, edge_slope=edge_slope, inflow=inflow, inflow_q=q,
                    wet_fp32=True)
    ref = orc.Member(h32.copy(), qx32.copy(), qy32.copy(), t=700.0, s=1.2, mu=0.8)
    orc.step(m32, ref, dt)
    tol = 1e-6 + 4.0 * np.spacing(np.abs(ref.h).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(e.field(1) - ref.h) <= tol)
    qs = max(np.abs(ref.qx).max(), np.abs(ref.qy).max())
    assert np.abs(e.field(1, fl.FIELD_QX) - ref.qx).max() <= 1e-5 * qs
    assert np.abs(e.field(1, fl.FIELD_QY) - ref.qy).max() <= 1e-5 * qs


def test_land_cover_with_inflow_matches_oracle(fl, orc):
    # both extensions in one handle (their own kernel instantiation), FP64 over the run
    c = W.urban_catchment("lcinf", 38, 52, 3, W.seed_for(2, 64), n_gauges=2, with_land_cover=True,
                          with_inflow=True)
    cat = dict(dem=c.dem, manning=c.manning, dx=c.dx, edge_kind=c.edge_kind, edge_slope=c.edge_slope, n_members=3,
               n_scale=c.n_scale, rain_mult=c.rain_mult, land_class=c.land_class, class_runoff=c.class_runoff,
               class_drain=c.class_drain, class_n=c.class_n, drain=c.drain, inflow=c.inflow, inflow_q=c.inflow_q,
               sections=c.sections)
    e = fl.FloodEnsemble([cat], RAIN, real_bytes=8)
    e.step(1200.0)
    led = e.ledger()
    q = e.sections()
    m = orc.Model(c.dem, c.manning, c.dx, RAIN, edge_kind=c.edge_kind, edge_slope=c.edge_slope,
                  land_class=c.land_class, class_runoff=c.class_runoff, class_drain=c.class_drain, inflow=c.inflow,
                  inflow_q=c.inflow_q)
    for i in range(3):
        mem = orc.Member.dry(m, s=c.n_scale[i], mu=c.rain_mult[i], class_n=c.class_n[i], drain_rate=c.drain[i])
        orc.advance(m, mem, 1200.0)
        assert np.abs(e.field(i) - mem.h).max() <= 1e-9
        for k, v in (("inflow", mem.v_in), ("drain", mem.v_drain), ("rain_in", mem.v_rain)):
            assert led[k][i] == pytest.approx(v, rel=1e-10)
        ref = np.array([orc.section_flow(m, mem, s) for s in c.sections])
        assert np.abs(q[i] - ref).max() <= 1e-9 * max(np.abs(ref).max(), 1e-12)
    gain = led["rain_in"] + led["inflow"]
    resid = np.abs(led["storage"] - (gain - led["outflow"] + led["clamp"] - led["drain"])) / gain
    assert resid.max() <= 1e-12


def test_filter_at_the_member_limit_and_on_flows_alone(fl, orc):
    # 1024 members (the most one workgroup filters) on a small grid, observed
    # through the sections only (no depth gauge), relative error
    c = W.urban_catchment("max", 20, 24, 1024, W.seed_for(2, 65), n_gauges=1, with_inflow=True)
    cat = dict(dem=c.dem, manning=c.manning, dx=c.dx, edge_kind=c.edge_kind, edge_slope=c.edge_slope,
               n_members=1024, n_scale=c.n_scale, rain_mult=c.rain_mult, inflow=c.inflow, inflow_q=c.inflow_q,
               sections=c.sections)
    e = fl.FloodEnsemble([cat], RAIN, real_bytes=4)
    e.step(900.0)
    yq = e.sections()
    assert yq.shape == (1024, len(c.sections))
    obs = yq[17] * 1.02
    floor = np.full(len(c.sections), 1e-4)
    lw0 = e.weights()[0]
    before = {j: e.field(j) for j in range(0, 1024, 97)}
    neff, anc, res = e.assimilate_obs(0, np.zeros((0, 2), np.int32), obs, floor, alpha=0.05, neff_frac=0.8, u0=0.3)
    _, w_ref, neff_ref = orc.pf_weights(yq, obs, floor, lw0, alpha=0.05)
    assert neff == pytest.approx(neff_ref, rel=1e-12)
    if res:
        np.testing.assert_array_equal(anc, orc.systematic(w_ref, 0.3))
        for j in range(0, 1024, 97):
            if anc[j] in before:
                np.testing.assert_array_equal(e.field(j), before[anc[j]])
    else:
        np.testing.assert_allclose(np.exp(e.weights()[0]), w_ref, rtol=1e-12, atol=1e-300)
