"""Pins of the oracle's ensemble products (Sec. 4.4, Figs. 15-16): probability of
the maximum depth reaching a threshold and percentiles of the maximum depth,
and the running maximum itself.

Fixed by: numpy's empirical mean and its inverted-CDF percentile for equal
weights, the equivalence of integer weights with duplicated members, the
extreme percentiles (minimum, maximum), and the maximum of a trajectory
recorded step by step.
"""
import numpy as np
import pytest

import workloads as W


def _values(rng, N, shape):
    # maximum depths with ties and exact threshold hits
    v = rng.choice([0.0, 0.05, 0.1, 0.2, 0.35, 0.8], size=(N,) + shape)
    return v + np.where(rng.random((N,) + shape) < 0.5, rng.uniform(0.0, 0.3, size=(N,) + shape), 0.0)


@pytest.mark.parametrize("N", [7, 96])
def test_equal_weights_match_numpy(orc, N):
    rng = np.random.default_rng(N)
    v = _values(rng, N, (9, 11))
    pcts = (0.1, 0.5, 0.9) if N == 96 else (0.2, 0.55, 0.93)
    prob, pc = orc.ensemble_products(v, 0.2, pcts)
    np.testing.assert_array_equal(prob, np.mean(v >= 0.2, axis=0))
    for p, got in zip(pcts, pc):
        r = p * N                                         # exact rank, or none near a rounding boundary
        assert r == round(r) or abs(r - round(r)) > 1e-6
        np.testing.assert_array_equal(got, np.percentile(v, 100 * p, axis=0, method="inverted_cdf"))


def test_integer_weights_equal_duplicated_members(orc):
    rng = np.random.default_rng(3)
    N = 12
    v = _values(rng, N, (6, 5))
    k = rng.integers(0, 4, size=N)
    k[0] = max(k[0], 1)
    dup = np.repeat(v, k, axis=0)
    pcts = (0.13, 0.5, 0.87)
    a = orc.ensemble_products(v, 0.2, pcts, weights=k.astype(float))
    b = orc.ensemble_products(dup, 0.2, pcts)
    np.testing.assert_allclose(a[0], b[0], rtol=1e-15)
    for x, y in zip(a[1], b[1]):
        np.testing.assert_array_equal(x, y)


def test_extreme_percentiles_and_zero_weights(orc):
    rng = np.random.default_rng(4)
    N = 10
    v = _values(rng, N, (4, 4))
    w = rng.uniform(0.5, 2.0, size=N)
    w[3] = 0.0                                            # a zero-weight member is never the minimum
    v[3] = -1.0
    prob, (lo, hi) = orc.ensemble_products(v, 0.2, (1e-12, 1.0), weights=w)
    keep = np.arange(N) != 3
    np.testing.assert_array_equal(lo, v[keep].min(axis=0))
    np.testing.assert_array_equal(hi, v.max(axis=0))
    # the threshold is inclusive
    v2 = np.full((3, 1, 1), 0.2)
    assert orc.ensemble_products(v2, 0.2)[0][0, 0] == 1.0


def test_running_maximum_equals_recorded_trajectory(orc):
    c = W.urban_catchment("hm", 24, 20, 1, W.seed_for(2, 11), n_gauges=1)
    rain = W.chicago_hyetograph()
    m = orc.Model(c.dem, c.manning, c.dx, rain, edge_kind=c.edge_kind, edge_slope=c.edge_slope)
    tracked = orc.Member.dry(m, s=c.n_scale[0], mu=c.rain_mult[0], track_max=True)
    plain = orc.Member.dry(m, s=c.n_scale[0], mu=c.rain_mult[0])
    seen = plain.h.copy()
    t = 0.0
    while t < 1500.0:
        t = min(t + 37.0, 1500.0)
        orc.advance(m, tracked, t)
        # the same trajectory one step at a time
        while plain.t < t:
            orc.advance(m, plain, t, max_steps=1)
            seen = np.maximum(seen, plain.h)
    np.testing.assert_array_equal(tracked.h, plain.h)
    np.testing.assert_array_equal(tracked.hmax, seen)
    assert np.any(tracked.hmax > tracked.h)                # the storm has receded somewhere
