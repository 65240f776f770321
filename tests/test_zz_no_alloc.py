"""The allocation-free entry point flood_systematic_resample_noalloc against the
allocating flood_systematic_resample (same kernel; systematic resampling of
Sec. 2.2 and Sec. 3.3 step IV), through the C ABI: ancestors bit-exact on two
calls in a row, the second smaller, and again at full size after it."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2302_08341_amd import flood
    flood.load_library()
    return flood


def test_noalloc_resampling_matches_the_allocating_entry_point(fl, orc):
    rng = np.random.default_rng(20240607)
    for n, u0 in ((1024, 0.731), (37, 0.052), (1024, 0.0)):
        w = rng.exponential(size=n)
        w[rng.uniform(size=n) < 0.25] = 0.0          # zero-weight particles are never chosen
        w[n // 2] += 5.0
        ref = fl.flood_systematic_resample(w, u0)
        got = fl.flood_systematic_resample_noalloc(w, u0)
        np.testing.assert_array_equal(got, ref)
        np.testing.assert_array_equal(got, orc.systematic(w, u0))
        assert np.all(w[got] > 0.0)


def test_noalloc_rejects_sizes_beyond_its_staging(fl):
    with pytest.raises(fl.FloodError) as e:
        fl.flood_systematic_resample_noalloc(np.ones(1025), 0.5)
    assert e.value.status == fl.FLOOD_EINVAL
    with pytest.raises(fl.FloodError):
        fl.flood_systematic_resample_noalloc(np.zeros(8), 0.5)
