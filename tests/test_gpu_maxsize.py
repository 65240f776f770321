"""Largest shapes: one catchment of 4096 x 4096 cells with 160 members holds
2.7e9 values in each state array, past 2^31, so every index into the member
planes has to be 64-bit.

The last member starts from a wet state with a sloping surface and one step of
it is checked against the oracle (the bars of the one-step tests: 1e-6 m plus 4
FP32 ulp of the depth, 1e-5 of the largest discharge); dry members' steps and
mass ledgers are checked too; then a filter update whose weight falls entirely
on the last member copies it into every slot, bit-exact.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

NY = NX = 4096
N = 160
DT = 0.05          # shorter than Eq. 4 allows for every member: one step each
LAST = N - 1


@pytest.fixture(scope="module")
def fl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2302_08341_amd import flood
    flood.load_library()
    return flood


@pytest.fixture(scope="module")
def big(fl):
    assert N * NY * NX > 2 ** 31
    c = W.urban_catchment("max", NY, NX, N, W.seed_for(9, 0), n_gauges=10)
    rain = W.chicago_hyetograph()
    ens = fl.FloodEnsemble([dict(dem=c.dem, manning=c.manning, dx=c.dx, edge_kind=c.edge_kind,
                                 edge_slope=c.edge_slope, n_members=N, n_scale=c.n_scale, rain_mult=c.rain_mult)],
                           rain, real_bytes=4)
    yy, xx = np.mgrid[0:NY, 0:NX]
    h0 = (0.3 + 0.25 * np.sin(2 * np.pi * xx / 61.0) * np.cos(2 * np.pi * yy / 47.0))
    h0 = h0.astype(np.float32).astype(np.float64)
    ens.set_state(LAST, h0, np.zeros((NY, NX + 1)), np.zeros((NY + 1, NX)), 0.0)
    ens.step(DT)
    print("configuration at 4096 x 4096 x 160", ens.config(), flush=True)
    yield c, rain, h0, ens
    ens.close()


def _model(orc, c, rain):
    return orc.Model(c.dem, c.manning, c.dx, rain, edge_kind=c.edge_kind, edge_slope=c.edge_slope, wet_fp32=True)


def test_last_member_one_step_matches_oracle(fl, orc, big):
    c, rain, h0, ens = big
    ref = orc.Member(h0.copy(), np.zeros((NY, NX + 1)), np.zeros((NY + 1, NX)), t=0.0, s=c.n_scale[LAST],
                     mu=c.rain_mult[LAST])
    orc.step(_model(orc, c, rain), ref, DT)
    gh, gqx, gqy = ens.field(LAST), ens.field(LAST, fl.FIELD_QX), ens.field(LAST, fl.FIELD_QY)
    tol = 1e-6 + 4.0 * np.spacing(np.abs(ref.h).astype(np.float32)).astype(np.float64)
    d = np.abs(gh - ref.h)
    print("last member: max |dh|", d.max(), "max |q|", np.abs(ref.qx).max(), flush=True)
    assert np.all(d <= tol)
    qs = max(np.abs(ref.qx).max(), np.abs(ref.qy).max())
    assert qs > 1e-3          # the sloping surface drives real flows
    assert np.abs(gqx - ref.qx).max() <= 1e-5 * qs
    assert np.abs(gqy - ref.qy).max() <= 1e-5 * qs


@pytest.mark.parametrize("i", [0, N // 2, LAST - 1])
def test_dry_members_one_step_match_oracle(fl, orc, big, i):
    c, rain, _, ens = big
    m = _model(orc, c, rain)
    ref = orc.Member.dry(m, s=c.n_scale[i], mu=c.rain_mult[i])
    orc.step(m, ref, DT)
    assert np.abs(ens.field(i) - ref.h).max() <= 1e-6 + 4.0 * np.spacing(np.float32(ref.h.max()))


def test_every_member_stepped_once_and_ledgers_close(big):
    _, _, _, ens = big
    led = ens.ledger()
    assert np.all(led["steps"] == 1)
    assert np.all(led["t"] == DT)
    dry = np.arange(N) != LAST
    resid = np.abs(led["storage"] - (led["rain_in"] - led["outflow"] + led["clamp"]))[dry] / led["rain_in"][dry]
    assert resid.max() <= 1e-6


def test_filter_copies_the_last_member_into_every_slot(fl, big):
    # runs last: it rewrites the ensemble
    c, _, _, ens = big
    before = (ens.field(LAST), ens.field(LAST, fl.FIELD_QX), ens.field(LAST, fl.FIELD_QY))
    obs = before[0][c.gauges[:, 0], c.gauges[:, 1]]
    assert obs.min() > 0.01     # dry members hold about 1e-6 m there: their weights underflow to 0
    neff, anc, res = ens.assimilate(0, c.gauges, obs, np.full(len(obs), 1e-3), 0.8, 0.5)
    assert res and neff == pytest.approx(1.0)
    np.testing.assert_array_equal(anc, np.full(N, LAST))
    for i in (0, N // 2, LAST):
        for w, ref in zip((fl.FIELD_H, fl.FIELD_QX, fl.FIELD_QY), before):
            np.testing.assert_array_equal(ens.field(i, w), ref)
    np.testing.assert_allclose(ens.weights()[0], np.full(N, -np.log(N)), rtol=1e-15)
