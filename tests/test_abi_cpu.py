"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/flood.h, and rejects bad arguments before any HIP call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "flood.h")).read()
    return sorted(set(re.findall(r"\b(flood_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2302_08341_amd import flood
    if not os.path.exists(flood.LIB_PATH):
        pytest.fail("libflood.so is not built (run __graft_entry__.build())")
    return flood.load_library()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "flood_step" in names and "flood_assimilate" in names and "flood_adjoint" in names
    for n in names:
        assert hasattr(lib, n), n


def test_binding_names_match_header():
    from paper_2302_08341_amd import flood
    assert sorted(flood.EXPORTED) == _declared()
    for n in flood.EXPORTED:
        assert callable(getattr(flood, n, None)) or n in ("flood_last_error", "flood_strerror")


def test_strerror(lib):
    assert lib.flood_strerror(0) == b"ok"
    assert lib.flood_strerror(-1) == b"invalid argument"


def _grid(ny=4, nx=5, **kw):
    from paper_2302_08341_amd import flood
    dem = np.zeros((ny, nx), np.float32)
    n = np.full((ny, nx), 0.03, np.float32)
    args = dict(edge_kind=(0, 0, 1, 0), edge_slope=(0, 0, 1e-3, 0))
    args.update(kw)
    return flood.make_grid(dem, n, 3.0, **args)


@pytest.mark.parametrize("bad", ["dx", "rain", "slope", "members", "manning", "alpha", "bytes", "mi", "h0"])
def test_create_rejects_bad_arguments_before_touching_the_device(lib, bad):
    from paper_2302_08341_amd import flood
    g = _grid()
    p = flood.make_params([1e-5], real_bytes=4)
    n = 2
    if bad == "dx":
        g.dx = -1.0
    elif bad == "rain":
        p = flood.make_params([-1.0])
    elif bad == "slope":
        g = _grid(edge_kind=(1, 0, 0, 0), edge_slope=(0.0, 0, 0, 0))
    elif bad == "members":
        n = 0
    elif bad == "manning":
        dem = np.zeros((4, 5), np.float32)
        g = flood.make_grid(dem, np.zeros((4, 5), np.float32), 3.0)
    elif bad == "alpha":
        p = flood.make_params([1e-5], cfl_alpha=2.0)
    elif bad == "bytes":
        p = flood.make_params([1e-5], real_bytes=2)
    elif bad == "mi":
        p = flood.make_params([1e-5], member_interleave=3)
    elif bad == "h0":
        dem = np.zeros((4, 5), np.float32)
        g = flood.make_grid(dem, np.full((4, 5), 0.03, np.float32), 3.0, h0=np.full((4, 5), -1, np.float32))
    h = C.c_void_p()
    rc = lib.flood_create(C.byref(g), C.byref(p), n, None, None, None, C.byref(h))
    assert rc == flood.FLOOD_EINVAL
    assert not h.value
    assert lib.flood_last_error(None)


LC_GOOD = dict(class_runoff=[1.0, 0.9], class_drain=[1, 0], member_class_n=[0.02, 0.1, 0.015, 0.12],
               member_drain=[3e-6, 4e-6])


@pytest.mark.parametrize("bad", ["map_without_classes", "classes_without_map", "class_value", "runoff", "drain_flag",
                                 "class_n", "class_n_missing", "member_drain", "too_many", "kernel", "interleave"])
def test_land_cover_is_validated_before_touching_the_device(lib, bad):
    from paper_2302_08341_amd import flood
    cls = np.zeros((4, 5), np.uint8)
    cls[1:3, 2:] = 1
    kw = dict(LC_GOOD)
    g = _grid(land_class=cls)
    extra = {}
    if bad == "map_without_classes":
        kw = {}
    elif bad == "classes_without_map":
        g = _grid()
    elif bad == "class_value":
        cls2 = cls.copy()
        cls2[0, 0] = 2
        g = _grid(land_class=cls2)
    elif bad == "runoff":
        kw["class_runoff"] = [1.0, 1.2]
    elif bad == "drain_flag":
        kw["class_drain"] = [2, 0]
    elif bad == "class_n":
        kw["member_class_n"] = [0.02, 0.0, 0.015, 0.12]
    elif bad == "class_n_missing":
        kw["member_class_n"] = None
    elif bad == "member_drain":
        kw["member_drain"] = [1e-6, -1e-6]
    elif bad == "too_many":
        kw.update(class_runoff=[1.0] * 5, class_drain=[0] * 5, member_class_n=[0.02] * 10)
    elif bad == "kernel":
        extra = dict(step_kernel=1)
    elif bad == "interleave":
        extra = dict(member_interleave=2)
    p = flood.make_params([1e-5], real_bytes=4, **kw, **extra)
    h = C.c_void_p()
    rc = lib.flood_create(C.byref(g), C.byref(p), 2, None, None, None, C.byref(h))
    assert rc == flood.FLOOD_EINVAL, bad
    assert not h.value
    assert lib.flood_last_error(None)


@pytest.mark.parametrize("bad", ["edge", "position", "series_index", "duplicate", "negative_q", "nan_q",
                                 "n_series", "missing_q", "missing_links", "too_many", "kernel", "interleave"])
def test_inflow_is_validated_before_touching_the_device(lib, bad):
    from paper_2302_08341_amd import flood
    g = _grid()                                     # 4 x 5 cells
    inflow = [(0, 2, 0), (3, 1, 1)]
    q = [[0.01, 0.02], [0.0, 0.03]]
    extra = {}
    if bad == "edge":
        inflow = [(4, 0, 0)]
    elif bad == "position":
        inflow = [(1, 4, 0)]                         # east edge has rows 0..3
    elif bad == "series_index":
        inflow = [(0, 0, 2)]
    elif bad == "duplicate":
        inflow = [(0, 2, 0), (0, 2, 1)]
    elif bad == "negative_q":
        q = [[0.01, -0.02], [0.0, 0.03]]
    elif bad == "nan_q":
        q = [[0.01, float("nan")], [0.0, 0.03]]
    elif bad == "n_series":
        q = [[0.01, 0.0]] * 5
        inflow = [(0, 0, 4)]
    elif bad == "kernel":
        extra = dict(step_kernel=2)
    elif bad == "interleave":
        extra = dict(member_interleave=4)
    p = flood.make_params([1e-5, 2e-5], real_bytes=4, inflow=inflow, inflow_q=q, **extra)
    if bad == "missing_q":
        p.inflow_q = None
    elif bad == "missing_links":
        p.inflow = None
    elif bad == "too_many":
        p.n_inflow = 2 * (4 + 5) + 1
    h = C.c_void_p()
    rc = lib.flood_create(C.byref(g), C.byref(p), 2, None, None, None, C.byref(h))
    assert rc == flood.FLOOD_EINVAL, bad
    assert not h.value
    assert lib.flood_last_error(None)


def test_section_and_observation_calls_reject_a_null_handle(lib):
    from paper_2302_08341_amd import flood
    assert lib.flood_set_sections(None, 0, 0, None, None) == flood.FLOOD_EINVAL
    assert lib.flood_get_sections(None, 0, None) == flood.FLOOD_EINVAL
    assert lib.flood_assimilate_obs(None, 0, 0, None, None, None, 0.05, 0.8, 0.5, None, None, None,
                                    None) == flood.FLOOD_EINVAL


def test_null_handle_calls_are_rejected(lib):
    from paper_2302_08341_amd import flood
    assert lib.flood_step(None, 1.0) == flood.FLOOD_EINVAL
    assert lib.flood_get_field(None, 0, 0, 0, None) == flood.FLOOD_EINVAL
    assert lib.flood_adjoint_release(None) == flood.FLOOD_EINVAL
    lib.flood_destroy(None)   # NULL-safe


def test_systematic_resample_validates(lib):
    from paper_2302_08341_amd import flood
    w = np.array([0.5, -0.1, 0.6])
    anc = np.zeros(3, np.int32)
    assert lib.flood_systematic_resample(flood._dp(w), 3, 0.5, flood._ip(anc), None) == flood.FLOOD_EINVAL
    w = np.array([0.5, 0.5])
    assert lib.flood_systematic_resample(flood._dp(w), 2, 1.0, flood._ip(anc), None) == flood.FLOOD_EINVAL


def test_no_cpu_fallback_without_device(lib):
    # on a host without a HIP device a valid creation fails loudly instead of computing on the CPU
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a device is present")
    except ImportError:
        pass
    from paper_2302_08341_amd import flood
    g = _grid()
    p = flood.make_params([1e-5])
    h = C.c_void_p()
    rc = lib.flood_create(C.byref(g), C.byref(p), 2, None, None, None, C.byref(h))
    assert rc == flood.FLOOD_EHIP


def test_valid_inflow_passes_validation(lib):
    # with no device the call gets past validation and fails at the first HIP call
    from paper_2302_08341_amd import flood
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    p = flood.make_params([1e-5, 2e-5], real_bytes=4, inflow=[(0, 2, 0), (3, 1, 1), (2, 0, 0), (1, 3, 1)],
                          inflow_q=[[0.01, 0.02], [0.0, 0.03]])
    h = C.c_void_p()
    g = _grid()
    assert lib.flood_create(C.byref(g), C.byref(p), 2, None, None, None, C.byref(h)) == flood.FLOOD_EHIP
