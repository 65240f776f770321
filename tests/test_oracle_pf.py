"""Pins of the oracle's particle filter (Eqs. 9-12, systematic resampling).

Expected values come from textbook identities, scipy's Gaussian log-density
and softmax, and exact rational arithmetic on dyadic weights.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.special import softmax
from scipy.stats import norm

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def test_likelihood_matches_scipy_gaussian(orc):
    rng = np.random.default_rng(3)
    N, K = 9, 5
    y = rng.uniform(0, 1, size=(N, K))
    d = rng.uniform(0, 1, size=K)
    sig = rng.uniform(0.02, 0.2, size=K)
    prior = np.log(rng.dirichlet(np.ones(N)))
    lp, w, neff = orc.pf_weights(y, d, sig, prior)
    # Eq. 9 with diagonal covariance = product of independent normal densities;
    # Eqs. 10-11 = normalised prior x likelihood
    ll = norm.logpdf(d[None, :], loc=y, scale=sig[None, :]).sum(axis=1)
    ref = softmax(prior + ll)
    np.testing.assert_allclose(w, ref, rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(np.exp(lp), ref, rtol=1e-12)
    assert neff == pytest.approx(1.0 / np.sum(ref ** 2), rel=1e-12)


def test_equal_likelihoods_keep_uniform_weights(orc):
    N = 16
    y = np.full((N, 3), 0.4)
    lw, neff, anc, res = orc.pf(y, np.array([0.1, 0.2, 0.3]), np.full(3, 0.05), np.full(N, -np.log(N)),
                                0.8, 0.5)
    assert not res
    assert neff == pytest.approx(N, rel=1e-14)
    np.testing.assert_allclose(np.exp(lw), 1.0 / N, rtol=1e-14)
    np.testing.assert_array_equal(anc, np.arange(N))


def test_one_hot_degenerates_and_resamples(orc):
    N = 12
    y = np.full((N, 2), 5.0)
    y[7] = [0.3, 0.4]
    lw, neff, anc, res = orc.pf(y, np.array([0.3, 0.4]), np.full(2, 0.05), np.full(N, -np.log(N)), 0.8, 0.3)
    assert res
    assert neff == pytest.approx(1.0, abs=1e-12)
    np.testing.assert_array_equal(anc, 7)
    np.testing.assert_allclose(lw, -np.log(N))


def test_extreme_log_likelihoods_stay_finite(orc):
    N = 5
    y = np.array([[0.0], [10.0], [20.0], [30.0], [40.0]])   # misfits up to 40/0.05 sigma
    lp, w, neff = orc.pf_weights(y, np.array([0.0]), np.array([0.05]), np.full(N, -np.log(N)))
    assert np.all(np.isfinite(lp))
    assert w[0] == 1.0 and neff == 1.0
    assert lp[1] == pytest.approx(-0.5 * (10.0 / 0.05) ** 2, rel=1e-12)


def test_neff_closed_form(orc):
    # weights (1/2, 1/4, 1/4) from the prior alone: N_eff = 1 / (1/4 + 1/16 + 1/16) = 8/3
    prior = np.log([0.5, 0.25, 0.25])
    lp, w, neff = orc.pf_weights(np.zeros((3, 0)), np.zeros(0), np.zeros(0), prior)
    np.testing.assert_allclose(w, [0.5, 0.25, 0.25], rtol=1e-15)
    assert neff == pytest.approx(8.0 / 3.0, rel=1e-15)


def test_resampling_threshold_is_paper_value_and_strict(orc):
    frac = json.load(open(GOLD))["resampling_threshold"]["neff_frac"]
    assert frac == 0.8
    # four particles, weights (1/2,1/6,1/6,1/6): N_eff = 1/(1/4 + 3/36) = 3 < 3.2 -> resample
    prior = np.log([0.5, 1 / 6, 1 / 6, 1 / 6])
    _, neff, _, res = orc.pf(np.zeros((4, 0)), np.zeros(0), np.zeros(0), prior, frac, 0.1)
    assert neff == pytest.approx(3.0, rel=1e-14) and res
    # five particles, one with zero weight: N_eff = 4 = 0.8 N exactly -> not below -> no resampling
    prior = np.array([np.log(0.25)] * 4 + [-np.inf])
    _, neff, _, res = orc.pf(np.zeros((5, 0)), np.zeros(0), np.zeros(0), prior, frac, 0.1)
    assert neff == 4.0
    assert not res


def _brute_systematic(w_frac, u0_frac):
    """Exact rational systematic resampling: member j takes the particle whose
    cumulative-weight interval [C_{i-1}, C_i) contains (u0 + j)/N."""
    N = len(w_frac)
    C = []
    run = Fraction(0)
    for x in w_frac:
        run += x
        C.append(run)
    out = []
    for j in range(N):
        t = (u0_frac + j) / N * C[-1]
        i = next((k for k in range(N) if t < C[k]), N - 1)
        out.append(i)
    return out


@pytest.mark.parametrize("seed", range(20))
def test_systematic_exact_rational_brute_force(orc, seed):
    rng = np.random.default_rng(100 + seed)
    N = int(rng.integers(1, 40))
    # dyadic weights (k / 2^12) and a dyadic offset make every FP64 operation exact
    k = rng.integers(0, 9, size=N)
    if k.sum() == 0:
        k[0] = 1
    w = k / 4096.0
    u0 = int(rng.integers(0, 4096)) / 4096.0
    anc = orc.systematic(w, u0)
    ref = _brute_systematic([Fraction(int(x), 4096) for x in k], Fraction(int(u0 * 4096), 4096))
    np.testing.assert_array_equal(anc, ref)


@pytest.mark.parametrize("seed", range(30))
def test_systematic_count_property(orc, seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(2, 97))
    w = rng.dirichlet(np.full(N, 0.3))
    w[rng.integers(0, N)] = 0.0            # a zero-weight particle is never chosen
    w = w / w.sum()
    anc = orc.systematic(w, float(rng.uniform()))
    counts = np.bincount(anc, minlength=N)
    assert counts.sum() == N
    assert np.all(np.diff(anc) >= 0)
    assert np.all(counts[w == 0] == 0)
    # each particle is copied floor(N w) or ceil(N w) times (up to the FP64 rounding of N w)
    nw = N * w
    assert np.all(counts >= np.floor(nw - 1e-9)) and np.all(counts <= np.ceil(nw + 1e-9))


def test_ensemble_assimilate_copies_states_and_perturbs(orc):
    import workloads as W
    wl = W.config1(20, 16)
    m = orc.Model.from_workload(wl)
    e = orc.Ensemble(m, [1.0, 1.1, 0.9, 1.2], [1.0, 1.5, 0.5, 2.0])
    e.advance(300.0)
    g = np.array([[5, 5], [10, 8]])
    truth = orc.gauge_values([e.members[3]], g)[0]
    before = [x.copy() for x in e.members]
    beta = np.array([1.01, 0.99, 1.02, 0.98])
    neff, anc, res = e.assimilate(g, truth, np.full(2, 1e-6), 0.8, 0.25, beta)
    assert res and np.all(anc == 3)
    for j, x in enumerate(e.members):
        np.testing.assert_array_equal(x.h, before[3].h)
        assert x.mu == pytest.approx(2.0 * beta[j], rel=1e-15)
        assert x.s == before[3].s and x.t == before[3].t
