"""GPU parity of the forward step against the FP64 oracle (through the C ABI).

Tolerances: one FP32 step from an identical state 1e-6 m, 1e-5 of the largest
discharge, and the links' wet/dry decisions identical (both sides decide in
float from the same float state); FP64 state: 1e-9 m over the whole
plain-method run.  Members are independent, so any interleave / tiling /
batching must give bit-identical results.  FP32 trajectories are held by replay
in tests/test_gpu_trajectory.py.
"""
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


def _ens(fl, c, rain, n, **kw):
    cat = dict(dem=c.dem, manning=c.manning, dx=c.dx, edge_kind=c.edge_kind, edge_slope=c.edge_slope,
               n_members=n, n_scale=c.n_scale[:n], rain_mult=c.rain_mult[:n], h0=c.h0)
    return fl.FloodEnsemble([cat], rain, **kw)


def _orc_member(orc, c, rain, i, t_end, **kw):
    m = orc.Model(c.dem, c.manning, c.dx, rain, edge_kind=c.edge_kind, edge_slope=c.edge_slope, **kw)
    mem = orc.Member.dry(m, s=c.n_scale[i], mu=c.rain_mult[i], h0=c.h0)
    orc.advance(m, mem, t_end)
    return m, mem


URBAN = W.urban_catchment("par", 97, 83, 5, W.seed_for(2, 5), n_gauges=4)   # ragged against every tile


def test_one_step_parity_from_identical_state(fl, orc):
    rain = W.chicago_hyetograph()
    m, mem = _orc_member(orc, URBAN, rain, 2, 1200.0)
    # round the oracle state to FP32 so both sides start from the same numbers
    h32 = mem.h.astype(np.float32).astype(np.float64)
    qx32 = mem.qx.astype(np.float32).astype(np.float64)
    qy32 = mem.qy.astype(np.float32).astype(np.float64)
    e = _ens(fl, URBAN, rain, 5, real_bytes=4)
    e.set_state(2, h32, qx32, qy32, 1200.0)
    e.step(1200.0)                      # other members advance; member 2 is already there
    wx, wy = e.wet_mask(2)              # the decisions the next step takes, from this float state
    dt = 0.05                           # shorter than Eq. 4 here: exactly one step of this length
    e.step(1200.0 + dt)
    ref = orc.Member(h32.copy(), qx32.copy(), qy32.copy(), t=1200.0, s=URBAN.n_scale[2], mu=URBAN.rain_mult[2])
    # from the same float state the links' wet/dry decision is the float model's own
    m32 = orc.Model(URBAN.dem, URBAN.manning, URBAN.dx, rain, edge_kind=URBAN.edge_kind,
                    edge_slope=URBAN.edge_slope, wet_fp32=True)
    orc.step(m32, ref, dt)
    gh, gqx, gqy = e.field(2), e.field(2, fl.FIELD_QX), e.field(2, fl.FIELD_QY)
    assert np.abs(gh - ref.h).max() <= 1e-6
    qs = max(np.abs(ref.qx).max(), np.abs(ref.qy).max())
    assert np.abs(gqx - ref.qx).max() <= 1e-5 * qs and np.abs(gqy - ref.qy).max() <= 1e-5 * qs
    # the wet/dry decisions, bit for bit, and only wet links carry flow
    ox, oy = orc.wet_masks(m32, h32, 1200.0, fp32=True)
    np.testing.assert_array_equal(wx, ox)
    np.testing.assert_array_equal(wy, oy)
    assert np.all(gqx[wx == 0] == 0.0) and np.all(gqy[wy == 0] == 0.0)
    assert np.count_nonzero(wx) > 100 and np.count_nonzero(wx == 0) > 100


@pytest.mark.parametrize("sk", [1, 2])
def test_plain_method_fp64_config1(fl, orc, sk):
    wl = W.config1()
    c = wl.catchments[0]
    e = _ens(fl, c, wl.rain, 1, real_bytes=8, member_interleave=1, step_kernel=sk)
    e.step(wl.t_end)
    m = orc.Model.from_workload(wl)
    mem = orc.Member.dry(m)
    orc.advance(m, mem, wl.t_end)
    dh = np.abs(e.field(0) - mem.h).max()
    assert dh <= 1e-9, dh
    led = e.ledger()
    assert led["steps"][0] == mem.steps
    assert abs(led["rain_in"][0] - mem.v_rain) <= 1e-12 * mem.v_rain
    resid = abs(led["storage"][0] - (led["rain_in"][0] - led["outflow"][0] + led["clamp"][0])) / led["rain_in"][0]
    assert resid <= 1e-12


@pytest.mark.parametrize("mi,rows,cpb,sk,mr,mm", [(1, 1, 1, 1, 0, 1), (2, 4, 3, 1, 0, 1), (4, 2, 2, 1, 0, 1),
                                                 (8, 8, 1, 1, 0, 1), (8, 1, 4, 1, 0, 1), (1, 4, 5, 2, 1, 1),
                                                 (1, 4, 5, 2, 7, 2), (1, 4, 5, 2, 64, 4), (1, 4, 5, 2, 500, 8),
                                                 (1, 4, 5, 2, 13, 4)])
def test_interleave_and_tiling_are_bit_exact(fl, mi, rows, cpb, sk, mr, mm):
    rain = W.chicago_hyetograph()
    ref = _ens(fl, URBAN, rain, 5, real_bytes=4, member_interleave=1, tile_rows=4, chunks_per_block=5,
               step_kernel=1)
    ref.step(400.0)
    e = _ens(fl, URBAN, rain, 5, real_bytes=4, member_interleave=mi, tile_rows=rows, chunks_per_block=cpb,
             step_kernel=sk, march_rows=mr, march_members=mm)
    assert e.config()["step_kernel"] == sk
    e.step(400.0)
    for i in range(5):
        for w in (fl.FIELD_H, fl.FIELD_QX, fl.FIELD_QY):
            np.testing.assert_array_equal(e.field(i, w), ref.field(i, w))


URBAN4 = W.urban_catchment("par4", 61, 300, 3, W.seed_for(2, 4), n_gauges=3)   # nx % 4 == 0, 2 strips


@pytest.mark.parametrize("rb", [4, 8])
@pytest.mark.parametrize("mr", [1, 5, 16, 100])
@pytest.mark.parametrize("order", [0, 1, 2, 3, 4])
def test_vectorised_march_is_bit_exact(fl, rb, mr, order, monkeypatch):
    # wavefront orders: 2 takes the members in quads and pads 3 members to 4,
    # 4 cuts the rows of strips into 8 bands and pads them
    rain = W.chicago_hyetograph()
    ref = _ens(fl, URBAN4, rain, 3, real_bytes=rb, member_interleave=1, tile_rows=4, chunks_per_block=3,
               step_kernel=1)
    ref.step(350.0)
    monkeypatch.setenv("FLOOD_MARCH_ORDER", str(order))
    e = _ens(fl, URBAN4, rain, 3, real_bytes=rb, member_interleave=1, step_kernel=3, march_rows=mr)
    assert e.config()["step_kernel"] == 3
    e.step(350.0)
    for i in range(3):
        for w in (fl.FIELD_H, fl.FIELD_QX, fl.FIELD_QY):
            np.testing.assert_array_equal(e.field(i, w), ref.field(i, w))
    np.testing.assert_array_equal(e.ledger()["outflow"], ref.ledger()["outflow"])


@pytest.mark.parametrize("pf", [0, 1, 2])
@pytest.mark.parametrize("rb", [4, 8])
@pytest.mark.parametrize("mr", [1, 2, 5, 16])
def test_row_lookahead_depths_are_bit_exact(fl, pf, rb, mr, monkeypatch):
    # no lookahead, one row and two rows of loads in flight: strips of 1 and 2 rows
    # (nothing or only the prologue row ahead) and a last strip shorter than the rest
    rain = W.chicago_hyetograph()
    ref = _ens(fl, URBAN4, rain, 3, real_bytes=rb, member_interleave=1, tile_rows=4, chunks_per_block=3,
               step_kernel=1)
    ref.step(350.0)
    monkeypatch.setenv("FLOOD_MARCH_PF", str(pf))
    e = _ens(fl, URBAN4, rain, 3, real_bytes=rb, member_interleave=1, step_kernel=3, march_rows=mr)
    e.step(350.0)
    for i in range(3):
        for w in (fl.FIELD_H, fl.FIELD_QX, fl.FIELD_QY):
            np.testing.assert_array_equal(e.field(i, w), ref.field(i, w))
    np.testing.assert_array_equal(e.ledger()["outflow"], ref.ledger()["outflow"])


@pytest.mark.parametrize("bands", [16, 32, 64])
@pytest.mark.parametrize("mr", [1, 3])
def test_banded_order_is_bit_exact(fl, bands, mr, monkeypatch):
    # more bands than rows of strips are clamped; partial bands are padded
    rain = W.chicago_hyetograph()
    ref = _ens(fl, URBAN4, rain, 3, real_bytes=4, member_interleave=1, tile_rows=4, chunks_per_block=3,
               step_kernel=1)
    ref.step(350.0)
    monkeypatch.setenv("FLOOD_MARCH_ORDER", "4")
    monkeypatch.setenv("FLOOD_MARCH_BANDS", str(bands))
    e = _ens(fl, URBAN4, rain, 3, real_bytes=4, member_interleave=1, step_kernel=3, march_rows=mr)
    assert e.config()["march_order"] == 4
    e.step(350.0)
    for i in range(3):
        for w in (fl.FIELD_H, fl.FIELD_QX, fl.FIELD_QY):
            np.testing.assert_array_equal(e.field(i, w), ref.field(i, w))


@pytest.mark.parametrize("order", [0, 2, 3, 4])
@pytest.mark.parametrize("mm", [1, 2])
def test_row_march_orders_are_bit_exact(fl, order, mm, monkeypatch):
    rain = W.chicago_hyetograph()
    ref = _ens(fl, URBAN, rain, 5, real_bytes=4, member_interleave=1, tile_rows=4, chunks_per_block=5,
               step_kernel=1)
    ref.step(330.0)
    monkeypatch.setenv("FLOOD_MARCH_ORDER", str(order))
    e = _ens(fl, URBAN, rain, 5, real_bytes=4, member_interleave=1, step_kernel=2, march_rows=7, march_members=mm)
    e.step(330.0)
    for i in range(5):
        np.testing.assert_array_equal(e.field(i), ref.field(i))
        np.testing.assert_array_equal(e.field(i, fl.FIELD_QY), ref.field(i, fl.FIELD_QY))


def test_batched_equals_one_launch_per_member(fl):
    rain = W.chicago_hyetograph()
    b = _ens(fl, URBAN, rain, 5, real_bytes=4, member_interleave=4)
    b.step(300.0)
    for i in range(5):
        cat = dict(dem=URBAN.dem, manning=URBAN.manning, dx=URBAN.dx, edge_kind=URBAN.edge_kind,
                   edge_slope=URBAN.edge_slope, n_members=1, n_scale=URBAN.n_scale[i:i + 1],
                   rain_mult=URBAN.rain_mult[i:i + 1])
        p = fl.FloodEnsemble([cat], rain, real_bytes=4, member_interleave=1)
        p.step(300.0)
        np.testing.assert_array_equal(p.field(0), b.field(i))


def test_multi_catchment_batch_matches_separate_handles(fl):
    rain = W.chicago_hyetograph()
    cs = [W.urban_catchment("a", 40, 70, 3, W.seed_for(4, 0)), W.urban_catchment("b", 65, 33, 2, W.seed_for(4, 1))]
    cats = [dict(dem=c.dem, manning=c.manning, dx=c.dx, edge_kind=c.edge_kind, edge_slope=c.edge_slope,
                 n_members=c.n_members, n_scale=c.n_scale, rain_mult=c.rain_mult) for c in cs]
    b = fl.FloodEnsemble(cats, rain, real_bytes=4)
    b.step(350.0)
    for j, c in enumerate(cats):
        s = fl.FloodEnsemble([c], rain, real_bytes=4)
        s.step(350.0)
        for i in range(c["n_members"]):
            np.testing.assert_array_equal(s.field(i), b.field(i, catchment=j))


def test_graph_and_direct_launches_agree(fl, monkeypatch):
    rain = W.chicago_hyetograph()
    a = _ens(fl, URBAN, rain, 3, real_bytes=4)
    a.step(200.0)
    monkeypatch.setenv("FLOOD_NO_GRAPH", "1")
    b = _ens(fl, URBAN, rain, 3, real_bytes=4)
    b.step(200.0)
    assert b.config()["graph_steps"] == 0
    for i in range(3):
        np.testing.assert_array_equal(a.field(i), b.field(i))


def test_lake_at_rest_gpu(fl):
    # bed and surface on a 2^-10 m lattice: h = eta0 - z, the bed step and the depth
    # difference are exact in FP32 and FP64, so a still lake must stay exactly still
    wl = W.config1(64, 48)
    z = np.round(wl.catchments[0].dem.astype(np.float64) * 1024.0) / 1024.0
    eta0 = np.round(float(np.quantile(z, 0.7)) * 1024.0) / 1024.0
    h0 = np.maximum(eta0 - z, 0.0)
    assert (h0 == 0).any() and (h0 > 0.5).any()
    cat = dict(dem=z.astype(np.float32), manning=wl.catchments[0].manning, dx=3.0, edge_kind=(0, 0, 0, 0),
               edge_slope=(0, 0, 0, 0), n_members=2, h0=h0.astype(np.float32))
    for rb in (8, 4):
        e = fl.FloodEnsemble([cat], [], real_bytes=rb)
        e.step(600.0)
        assert e.ledger()["steps"][0] > 100
        for i in range(2):
            np.testing.assert_array_equal(e.field(i), h0)
            assert np.abs(e.field(i, fl.FIELD_QX)).max() == 0.0
            assert np.abs(e.field(i, fl.FIELD_QY)).max() == 0.0


@pytest.mark.parametrize("ny,nx", [(1, 1), (1, 37), (29, 1), (2, 2), (65, 64), (3, 130)])
def test_degenerate_grids(fl, orc, ny, nx):
    # deep water everywhere (no cell near the wet/dry threshold); open edges across the
    # short direction of one-cell-thick strips would empty them in seconds, so those get walls
    rng = np.random.default_rng(ny * 100 + nx)
    dem = rng.uniform(0, 0.05, size=(ny, nx)).astype(np.float32)
    h0 = (0.3 + rng.uniform(0, 0.1, size=(ny, nx))).astype(np.float32)
    man = np.full((ny, nx), 0.03, np.float32)
    rain = [2e-5, 4e-5]
    kinds = [1, 1, 1, 1]
    if ny == 1:
        kinds[0] = kinds[2] = 0
    if nx == 1:
        kinds[1] = kinds[3] = 0
    slopes = (1e-3, 2e-3, 3e-3, 4e-3)
    cat = dict(dem=dem, manning=man, dx=3.0, edge_kind=tuple(kinds), edge_slope=slopes, h0=h0,
               n_members=3, n_scale=np.array([1.0, 1.2, 0.8]), rain_mult=np.array([1.0, 2.0, 0.5]))
    e = fl.FloodEnsemble([cat], rain, real_bytes=8, rain_interval=20.0)
    e.step(10.0)
    for i in range(3):
        m = orc.Model(dem, man, 3.0, np.array(rain), rain_interval=20.0, edge_kind=tuple(kinds),
                      edge_slope=slopes)
        mem = orc.Member.dry(m, s=cat["n_scale"][i], mu=cat["rain_mult"][i], h0=h0)
        orc.advance(m, mem, 10.0)
        assert mem.h.min() > 4e-3
        assert e.ledger()["steps"][i] == mem.steps
        assert np.abs(e.field(i) - mem.h).max() <= 1e-10
        assert np.abs(e.field(i, fl.FIELD_QX) - mem.qx).max() <= 1e-10
        assert np.abs(e.field(i, fl.FIELD_QY) - mem.qy).max() <= 1e-10


def test_save_load_roundtrip(fl, tmp_path):
    rain = W.chicago_hyetograph()
    a = _ens(fl, URBAN, rain, 3, real_bytes=4)
    a.step(150.0)
    p = str(tmp_path / "snap.bin")
    a.save(p)
    a.step(300.0)
    b = _ens(fl, URBAN, rain, 3, real_bytes=4)
    b.load(p)
    b.step(300.0)
    for i in range(3):
        np.testing.assert_array_equal(a.field(i), b.field(i))


# ---------------------------------------------------------------------------
# particle filter
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(6))
def test_systematic_resampling_bit_exact_given_weights(fl, orc, seed):
    rng = np.random.default_rng(seed)
    N = [1, 7, 64, 96, 513, 1024][seed]
    w = rng.dirichlet(np.full(N, 0.2))
    if seed % 2:
        w[rng.integers(0, N, size=max(1, N // 5))] = 0.0
        if w.sum() == 0:
            w[0] = 1.0
    u0 = float(rng.uniform())
    np.testing.assert_array_equal(fl.flood_systematic_resample(w, u0), orc.systematic(w, u0))


def test_assimilation_matches_oracle(fl, orc):
    # both sides assimilate the same ensemble state (the oracle's, loaded into the GPU handle)
    rain = W.chicago_hyetograph()
    N = 6
    c = W.urban_catchment("pf", 50, 44, N, W.seed_for(2, 7), n_gauges=5)
    m = orc.Model(c.dem, c.manning, c.dx, rain, edge_kind=c.edge_kind, edge_slope=c.edge_slope)
    ens = orc.Ensemble(m, c.n_scale, c.rain_mult)
    ens.advance(600.0)
    e = _ens(fl, c, rain, N, real_bytes=8)
    for i, x in enumerate(ens.members):
        e.set_state(i, x.h, x.qx, x.qy, 600.0)
    before = [e.field(i) for i in range(N)]
    for i, x in enumerate(ens.members):
        np.testing.assert_array_equal(before[i], x.h)
    obs = orc.gauge_values([ens.members[3]], c.gauges)[0] + 0.0002
    sig = np.full(5, 0.001)
    beta = np.random.default_rng(3).normal(1, 0.05, N)
    neff_g, anc_g, res_g = e.assimilate(0, c.gauges, obs, sig, 0.8, 0.4, beta)
    neff_o, anc_o, res_o = ens.assimilate(c.gauges, obs, sig, 0.8, 0.4, beta)
    assert neff_g == pytest.approx(neff_o, rel=1e-12)
    assert res_g == res_o and res_g
    np.testing.assert_array_equal(anc_g, anc_o)
    lw, mu, s = e.weights()
    np.testing.assert_allclose(lw, ens.logw, rtol=1e-12)
    np.testing.assert_allclose(mu, [x.mu for x in ens.members], rtol=1e-15)
    for j in range(N):
        np.testing.assert_array_equal(e.field(j), before[anc_g[j]])
    # the filtered ensemble keeps stepping in step with the oracle
    e.step(900.0)
    ens.advance(900.0)
    for j in range(N):
        assert np.abs(e.field(j) - ens.members[j].h).max() <= 1e-4


def test_assimilation_weights_without_resampling(fl, orc):
    rain = W.chicago_hyetograph()
    N = 8
    c = W.urban_catchment("pf3", 40, 36, N, W.seed_for(2, 6), n_gauges=4)
    m = orc.Model(c.dem, c.manning, c.dx, rain, edge_kind=c.edge_kind, edge_slope=c.edge_slope)
    ens = orc.Ensemble(m, c.n_scale, c.rain_mult)
    ens.advance(900.0)
    e = _ens(fl, c, rain, N, real_bytes=4)
    for i, x in enumerate(ens.members):
        e.set_state(i, x.h.astype(np.float32), x.qx.astype(np.float32), x.qy.astype(np.float32), 900.0)
    # the oracle filters the same FP32-rounded depths
    for x in ens.members:
        x.h = x.h.astype(np.float32).astype(np.float64)
    obs = orc.gauge_values([ens.members[1]], c.gauges)[0]
    sig = np.full(4, 0.5)
    for k in range(3):     # repeated updates carry the weights forward (Eq. 10 prior = last posterior)
        ng, ag, rg = e.assimilate(0, c.gauges, obs + 0.01 * k, sig, 0.3, 0.5)
        no, ao, ro = ens.assimilate(c.gauges, obs + 0.01 * k, sig, 0.3, 0.5)
        assert ng == pytest.approx(no, rel=1e-12) and rg == ro
        np.testing.assert_allclose(e.weights()[0], ens.logw, rtol=1e-12, atol=1e-12)


def test_assimilation_without_resampling_keeps_states(fl, orc):
    rain = W.chicago_hyetograph()
    c = W.urban_catchment("pf2", 30, 30, 4, W.seed_for(2, 8), n_gauges=2)
    e = _ens(fl, c, rain, 4, real_bytes=4)
    e.step(300.0)
    before = [e.field(i) for i in range(4)]
    neff, anc, res = e.assimilate(0, c.gauges, np.zeros(2), np.full(2, 100.0), 0.8, 0.5)
    assert not res and neff == pytest.approx(4.0, rel=1e-6)
    np.testing.assert_array_equal(anc, np.arange(4))
    for i in range(4):
        np.testing.assert_array_equal(e.field(i), before[i])


def test_assimilate_requires_common_time(fl):
    rain = W.chicago_hyetograph()
    e = _ens(fl, URBAN, rain, 2, real_bytes=4)
    e.step(100.0)
    h = e.field(0)
    e.set_state(0, h, e.field(0, fl.FIELD_QX), e.field(0, fl.FIELD_QY), 50.0)
    with pytest.raises(fl.FloodError) as ei:
        e.assimilate(0, URBAN.gauges, np.zeros(4), np.full(4, 0.05))
    assert ei.value.status == fl.FLOOD_ESTATE


@pytest.mark.parametrize("rb", [4, 8])
def test_numeric_fault_freezes_one_member_and_spares_the_rest(fl, rb):
    # a rain multiplier far beyond any physical storm drives one member's depth to
    # a non-finite value, or to one so large that its Eq. 4 step no longer moves its
    # clock (1e300 in double precision stays finite: 1e295 m after one step, then
    # steps of 1e-148 s); the step reports ENUMERIC, that member stays frozen at the
    # step the fault was found, and the others go on exactly as in a clean run
    rain = W.chicago_hyetograph()
    bad = _ens(fl, URBAN, rain, 5, real_bytes=rb)
    ref = _ens(fl, URBAN, rain, 5, real_bytes=rb)
    bad.step(300.0)
    ref.step(300.0)
    bad.snapshot()
    mu = URBAN.rain_mult[:5].copy()
    mu[2] = 1e38 if rb == 4 else 1e300
    bad.set_params(rain_mult=mu)
    with pytest.raises(fl.FloodError) as ei:
        bad.step(600.0)
    assert ei.value.status == fl.FLOOD_ENUMERIC
    ref.step(600.0)
    led = bad.ledger()
    assert led["t"][2] < 600.0
    assert np.all(led["t"][[0, 1, 3, 4]] == 600.0)
    frozen = [bad.field(2, k) for k in (fl.FIELD_H, fl.FIELD_QX, fl.FIELD_QY)]
    assert not np.all(np.isfinite(frozen[0])) or np.nanmax(frozen[0]) > 1e30
    for i in (0, 1, 3, 4):
        for k in (fl.FIELD_H, fl.FIELD_QX, fl.FIELD_QY):
            np.testing.assert_array_equal(bad.field(i, k), ref.field(i, k))
    # later calls keep reporting it; the frozen member does not move
    with pytest.raises(fl.FloodError) as ei:
        bad.step(900.0)
    assert ei.value.status == fl.FLOOD_ENUMERIC
    ref.step(900.0)
    assert bad.ledger()["t"][2] == led["t"][2]
    for k, f in zip((fl.FIELD_H, fl.FIELD_QX, fl.FIELD_QY), frozen):
        np.testing.assert_array_equal(bad.field(2, k), f)
    for i in (0, 1, 3, 4):
        np.testing.assert_array_equal(bad.field(i), ref.field(i))
    # the filter refuses a faulted catchment
    with pytest.raises(fl.FloodError) as ei:
        bad.assimilate(0, URBAN.gauges, np.zeros(len(URBAN.gauges)), np.full(len(URBAN.gauges), 1e-2))
    assert ei.value.status == fl.FLOOD_ESTATE
    # the device snapshot brings back the clean state, parameters and status
    bad.restore()
    ref2 = _ens(fl, URBAN, rain, 5, real_bytes=rb)
    ref2.step(300.0)
    bad.step(600.0)
    ref2.step(600.0)
    for i in range(5):
        np.testing.assert_array_equal(bad.field(i), ref2.field(i))


def test_graph_timing_matches_launch_timing_and_changes_nothing(fl):
    rain = W.chicago_hyetograph()
    runs = {}
    for mode in (0, 1, 2):
        e = _ens(fl, URBAN, rain, 5, real_bytes=4)
        e.step(300.0)
        if mode:
            e.timing(mode)
        e.step(600.0)
        if mode:
            e.timing(0)
        runs[mode] = (e.get_timing(), [e.field(i) for i in range(5)], e.config())
    (a1, n1), (a2, n2) = runs[1][0], runs[2][0]
    print("per-launch events %.4f ms over %d launches; per-batch events %.4f ms per launch over %d" % (a1, n1, a2, n2))
    assert runs[2][2]["graph_steps"] > 0
    assert n1 == n2 > 0                 # the same batches of step launches
    assert 0.0 < a1 < 3.0 * a2 and 0.0 < a2 < 3.0 * a1
    for mode in (1, 2):
        for i in range(5):
            np.testing.assert_array_equal(runs[mode][1][i], runs[0][1][i])


def test_stream_probe_reports_a_bandwidth_and_refuses_bad_shapes(fl):
    for wps in (0, 3, 4):
        gbps, ms = fl.flood_probe_stream(256, 512, 4, 16, 3, wps)
        print("stream probe on 4 x 256 x 512 cells, waves per SIMD %d: %.0f GB/s, %.4f ms" % (wps, gbps, ms))
        assert 0.0 < gbps < 8000.0 and ms > 0.0
    for bad in ((0, 512, 4, 16, 3), (256, 510, 4, 16, 3), (256, 512, 0, 16, 3), (256, 512, 4, 0, 3),
                (256, 512, 4, 16, 0), (65536, 65536, 1, 16, 3), (256, 512, 4, 16, 3, 9), (256, 512, 4, 16, 3, 2)):
        with pytest.raises(fl.FloodError):
            fl.flood_probe_stream(*bad)
