"""Empty and degenerate inputs through the C ABI, against the oracle where it
has something to say: a filter update with no gauges (the prior weights stand,
and N_eff, the resampling decision and the ancestors follow them), an adjoint
with no gauges (zero loss, zero gradients), steps to the current or an
earlier time (nothing moves), systematic resampling of one particle and of
weights with zeros (bit-exact ancestors, never a zero-weight particle), and
the ensemble products of a single member (every percentile is its maximum).
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

CAT = W.urban_catchment("edges", 40, 48, 6, W.seed_for(2, 51), n_gauges=4)
RAIN = W.chicago_hyetograph()
NOG = np.zeros((0, 2), np.int32)
NONE = np.zeros(0)


@pytest.fixture(scope="module")
def fl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2302_08341_amd import flood
    flood.load_library()
    return flood


def _ens(fl, n=6, **kw):
    c = CAT
    return fl.FloodEnsemble([dict(dem=c.dem, manning=c.manning, dx=c.dx, edge_kind=c.edge_kind,
                                  edge_slope=c.edge_slope, n_members=n, n_scale=c.n_scale[:n],
                                  rain_mult=c.rain_mult[:n])], RAIN, real_bytes=4, **kw)


def test_filter_update_without_gauges_keeps_the_prior(fl, orc):
    e = _ens(fl)
    e.step(600.0)
    states = [e.field(i) for i in range(6)]
    # equal prior weights: N_eff = N, no resampling, nothing moves
    neff, anc, res = e.assimilate(0, NOG, NONE, NONE, 0.8, 0.3)
    assert neff == pytest.approx(6.0, rel=1e-15) and not res
    np.testing.assert_allclose(e.weights()[0], np.full(6, -np.log(6.0)), rtol=1e-15)
    for i in range(6):
        np.testing.assert_array_equal(e.field(i), states[i])
    # unequal prior weights (an update with gauges under a threshold no N_eff
    # reaches), then an update with no gauges under the usual threshold
    # (gauges on member 2's four deepest cells, where the members' rain multipliers
    # set them apart)
    deep = np.argsort(states[2], axis=None)[-4:]
    gauges = np.stack(np.unravel_index(deep, states[2].shape), axis=1).astype(np.int32)
    obs = states[2][gauges[:, 0], gauges[:, 1]]
    e.assimilate(0, gauges, obs, np.full(4, 0.005), 1e-9, 0.3)
    lw0 = e.weights()[0]
    neff, anc, res = e.assimilate(0, NOG, NONE, NONE, 0.8, 0.3)
    _, neff_ref, anc_ref, res_ref = orc.pf(np.zeros((6, 0)), NONE, NONE, lw0, 0.8, 0.3)
    print("prior N_eff", neff_ref, "resampled", res_ref, flush=True)
    assert res_ref, "the prior built above should be degenerate enough to resample"
    assert neff == pytest.approx(neff_ref, rel=1e-12)
    assert res == res_ref
    np.testing.assert_array_equal(anc, anc_ref)
    for i in range(6):
        np.testing.assert_array_equal(e.field(i), states[anc[i]])


def test_adjoint_without_gauges_is_zero(fl):
    e = _ens(fl, n=4)
    e.step(300.0)
    loss, gn, gm = e.adjoint(0, 320.0, 10.0, NOG, np.zeros((2, 0)), ckpt_every=5)
    assert loss == 0.0
    assert not gn.any() and not gm.any()
    assert np.all(e.ledger()["t"] == 320.0)


def test_steps_to_the_current_or_an_earlier_time_move_nothing(fl):
    e = _ens(fl, n=3)
    e.step(300.0)
    h = [e.field(i) for i in range(3)]
    q = [e.field(i, fl.FIELD_QX) for i in range(3)]
    led = e.ledger()
    for t in (300.0, 120.0, 0.0, -5.0):
        e.step(t)
    after = e.ledger()
    np.testing.assert_array_equal(after["steps"], led["steps"])
    np.testing.assert_array_equal(after["t"], led["t"])
    for i in range(3):
        np.testing.assert_array_equal(e.field(i), h[i])
        np.testing.assert_array_equal(e.field(i, fl.FIELD_QX), q[i])


@pytest.mark.parametrize("w", [[1.0], [0.0, 0.0, 1.0, 0.0], [0.5, 0.0, 0.0, 0.5], [0.0, 1e-300, 0.0, 1.0],
                               [3.0, 0.0, 1.0]])
def test_resampling_one_particle_and_zero_weights(fl, orc, w):
    w = np.array(w)
    for u0 in (0.0, 0.5, 0.999999):
        anc = fl.flood_systematic_resample(w, u0)
        np.testing.assert_array_equal(anc, orc.systematic(w, u0))
        assert np.all(w[anc] > 0.0)


def test_products_of_one_member(fl, orc):
    e = _ens(fl, n=1, track_peak=True)
    e.step(900.0)
    pk = e.field(0, fl.FIELD_PEAK)
    assert pk.max() > 0.05
    pcts = (0.1, 0.5, 1.0)
    prob, pct = e.products(0.05, pct=pcts)
    np.testing.assert_array_equal(prob, (pk >= 0.05).astype(np.float64))
    for p in pct:
        np.testing.assert_array_equal(p, pk)
    prob_ref, pct_ref = orc.ensemble_products(pk[None], 0.05, pcts)
    np.testing.assert_array_equal(prob, prob_ref)
    for p, r in zip(pct, pct_ref):
        np.testing.assert_array_equal(p, r)
