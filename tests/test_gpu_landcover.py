"""GPU land cover (Sec. 4.1, Table 1) against the FP64 oracle, through the C ABI:
per-member Manning n per class, runoff coefficient of the rain per class,
drainage of draining classes at each member's rate, drained volume in the ledger.

Bars: FP64 1e-9 m over the run; one step from an identical float state
1e-6 m (float wet/dry decisions on both sides); ledger terms 1e-4 (FP32) /
1e-10 (FP64) relative, balance 1e-6 / 1e-12.  Member parameters follow
resampling and snapshots exactly.  The FP32 trajectory is held by replay in
tests/test_gpu_trajectory.py.
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


CAT = W.urban_catchment("lc", 53, 72, 4, W.seed_for(2, 41), n_gauges=4, with_land_cover=True)   # nx % 4 == 0
RAIN = W.chicago_hyetograph()


def _cat(n=4, members=None):
    c = CAT
    idx = np.arange(n) if members is None else np.asarray(members)
    return dict(dem=c.dem, manning=c.manning, dx=c.dx, edge_kind=c.edge_kind, edge_slope=c.edge_slope,
                n_members=len(idx), n_scale=c.n_scale[idx], rain_mult=c.rain_mult[idx], land_class=c.land_class,
                class_runoff=c.class_runoff, class_drain=c.class_drain, class_n=c.class_n[idx], drain=c.drain[idx])


def _ens(fl, n=4, **kw):
    return fl.FloodEnsemble([_cat(n)], RAIN, **kw)


def _oracle(orc, i, t_end, mu_factor=1.0, **kw):
    c = CAT
    m = orc.Model(c.dem, c.manning, c.dx, RAIN, edge_kind=c.edge_kind, edge_slope=c.edge_slope,
                  land_class=c.land_class, class_runoff=c.class_runoff, class_drain=c.class_drain, **kw)
    mem = orc.Member.dry(m, s=c.n_scale[i], mu=c.rain_mult[i] * mu_factor, class_n=c.class_n[i],
                         drain_rate=c.drain[i])
    orc.advance(m, mem, t_end)
    return m, mem


def test_fp64_trajectory_and_ledger_match_oracle(fl, orc):
    e = _ens(fl, real_bytes=8)
    e.step(1500.0)
    led = e.ledger()
    for i in range(4):
        _, mem = _oracle(orc, i, 1500.0)
        assert np.abs(e.field(i) - mem.h).max() <= 1e-9
        assert led["steps"][i] == mem.steps
        for k, v in (("rain_in", mem.v_rain), ("outflow", mem.v_out), ("drain", mem.v_drain)):
            assert led[k][i] == pytest.approx(v, rel=1e-10, abs=1e-12)
    assert np.all(led["drain"] > 0.0)
    resid = np.abs(led["storage"] - (led["rain_in"] - led["outflow"] + led["clamp"] - led["drain"])) / led["rain_in"]
    assert resid.max() <= 1e-12


def test_one_step_from_an_identical_float_state(fl, orc):
    m, mem = _oracle(orc, 2, 1200.0)
    h32 = mem.h.astype(np.float32).astype(np.float64)
    qx32 = mem.qx.astype(np.float32).astype(np.float64)
    qy32 = mem.qy.astype(np.float32).astype(np.float64)
    e = _ens(fl, real_bytes=4)
    e.set_state(2, h32, qx32, qy32, 1200.0)
    e.step(1200.0)
    dt = 0.05
    e.step(1200.0 + dt)
    m32, _ = _oracle(orc, 2, 0.0, wet_fp32=True)
    ref = orc.Member(h32.copy(), qx32.copy(), qy32.copy(), t=1200.0, s=CAT.n_scale[2], mu=CAT.rain_mult[2],
                     class_n=CAT.class_n[2].copy(), drain_rate=float(CAT.drain[2]))
    orc.step(m32, ref, dt)
    assert np.abs(e.field(2) - ref.h).max() <= 1e-6
    qs = max(np.abs(ref.qx).max(), np.abs(ref.qy).max())
    assert np.abs(e.field(2, fl.FIELD_QX) - ref.qx).max() <= 1e-5 * qs
    assert np.abs(e.field(2, fl.FIELD_QY) - ref.qy).max() <= 1e-5 * qs


def test_batched_equals_one_handle_per_member(fl):
    b = _ens(fl, real_bytes=4, track_peak=True)
    b.step(900.0)
    for i in range(4):
        p = fl.FloodEnsemble([_cat(members=[i])], RAIN, real_bytes=4, track_peak=True)
        p.step(900.0)
        np.testing.assert_array_equal(p.field(0), b.field(i))
        np.testing.assert_array_equal(p.field(0, fl.FIELD_PEAK), b.field(i, fl.FIELD_PEAK))
        # the drained volume is summed by FP64 atomics into bins chosen by the
        # workgroup id, which differs between the two launches: equal up to the
        # order of those sums
        assert p.ledger()["drain"][0] == pytest.approx(b.ledger()["drain"][i], rel=1e-12)
        p.close()


def test_member_parameters_follow_resampling_and_snapshots(fl):
    e = _ens(fl, real_bytes=4)
    e.step(1200.0)
    cn0, dr0 = e.land_params()
    np.testing.assert_array_equal(cn0, CAT.class_n[:4])
    np.testing.assert_array_equal(dr0, CAT.drain[:4])
    drained0 = e.ledger()["drain"]
    obs = e.field(1)[CAT.gauges[:, 0], CAT.gauges[:, 1]]
    neff, anc, res = e.assimilate(0, CAT.gauges, obs, np.full(4, 1e-5), 1.0, 0.4)
    assert res and len(set(anc.tolist())) < 4
    cn1, dr1 = e.land_params()
    np.testing.assert_array_equal(cn1, cn0[anc])
    np.testing.assert_array_equal(dr1, dr0[anc])
    np.testing.assert_array_equal(e.ledger()["drain"], drained0[anc])
    path = os.path.join(tempfile.mkdtemp(), "lc.bin")
    e.save(path)
    f = _ens(fl, real_bytes=4)
    f.load(path)
    np.testing.assert_array_equal(f.land_params()[0], cn1)
    np.testing.assert_array_equal(f.field(3), e.field(3))


def test_refusals(fl):
    e = _ens(fl, real_bytes=4)
    with pytest.raises(fl.FloodError) as ex:
        e.adjoint(0, 20.0, 10.0, CAT.gauges, np.zeros((2, 4)), ckpt_every=5)
    assert ex.value.status == fl.FLOOD_EINVAL
    with pytest.raises(fl.FloodError) as ex:
        fl.flood_set_params(e.h, 0, np.full(CAT.dem.shape, 0.03, np.float32), None, None)
    assert ex.value.status == fl.FLOOD_EINVAL
    for kw in (dict(step_kernel=1), dict(step_kernel=2), dict(member_interleave=4)):
        with pytest.raises(fl.FloodError) as ex:
            _ens(fl, real_bytes=4, **kw)
        assert ex.value.status == fl.FLOOD_EINVAL
    plain = fl.FloodEnsemble([dict(dem=CAT.dem, manning=CAT.manning, dx=CAT.dx, n_members=2)], RAIN, real_bytes=4)
    with pytest.raises(fl.FloodError) as ex:
        plain.land_params()
    assert ex.value.status == fl.FLOOD_ESTATE
