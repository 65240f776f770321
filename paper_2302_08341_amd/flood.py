"""ctypes binding of libflood (the C ABI in include/flood.h).

Argument marshalling only: every step of the model runs in the HIP kernels
of ``libflood.so``.  The module-level functions carry the C names
(``flood_create``, ``flood_step``, ...); :class:`FloodEnsemble` is a thin
object wrapper over them.  PyTorch, when present, only supplies the HIP
stream (``torch.cuda.current_stream()``).  There is no CPU fallback: if the
library is missing or no device is present the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libflood.so")

FLOOD_OK, FLOOD_EINVAL, FLOOD_ENOMEM, FLOOD_EHIP, FLOOD_ESTATE, FLOOD_ENUMERIC = 0, -1, -2, -3, -4, -5
EDGE_WALL, EDGE_OPEN = 0, 1
FIELD_H, FIELD_QX, FIELD_QY, FIELD_PEAK = 0, 1, 2, 3
SNAPSHOT_TAKE, SNAPSHOT_RESTORE, SNAPSHOT_RELEASE = 1, 2, 3
EXPORTED = ["flood_create", "flood_create_batch", "flood_step", "flood_assimilate", "flood_adjoint",
            "flood_get_field", "flood_set_state", "flood_set_params", "flood_get_ledger", "flood_get_weights",
            "flood_systematic_resample", "flood_ensemble_products", "flood_get_land_params", "flood_save",
            "flood_load", "flood_set_sections", "flood_get_sections", "flood_assimilate_obs",
            "flood_get_config", "flood_timing", "flood_get_timing", "flood_adjoint_release", "flood_step_n",
            "flood_get_wet_mask", "flood_log_steps", "flood_get_step_log", "flood_get_adjoint_info",
            "flood_systematic_resample_noalloc", "flood_device_snapshot", "flood_get_march_rows",
            "flood_probe_stream",
            "flood_last_error",
            "flood_strerror", "flood_destroy"]


class FloodError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (status %d): %s" % (_STATUS.get(status, "error"), status, msg))
        self.status = status


_STATUS = {FLOOD_EINVAL: "EINVAL", FLOOD_ENOMEM: "ENOMEM", FLOOD_EHIP: "EHIP", FLOOD_ESTATE: "ESTATE",
           FLOOD_ENUMERIC: "ENUMERIC"}


class FloodGrid(C.Structure):
    _fields_ = [("ny", C.c_int32), ("nx", C.c_int32), ("dx", C.c_double),
                ("dem", C.POINTER(C.c_float)), ("manning_n", C.POINTER(C.c_float)), ("h0", C.POINTER(C.c_float)),
                ("edge_kind", C.c_int32 * 4), ("edge_slope", C.c_double * 4),
                ("land_class", C.POINTER(C.c_uint8))]


class FloodParams(C.Structure):
    _fields_ = [("rain_rate", C.POINTER(C.c_double)), ("n_rain", C.c_int32), ("rain_interval", C.c_double),
                ("cfl_alpha", C.c_double), ("h_dry", C.c_double), ("dt_cap", C.c_double),
                ("dt_fixed", C.c_double), ("g", C.c_double), ("real_bytes", C.c_int32),
                ("member_interleave", C.c_int32), ("tile_rows", C.c_int32), ("chunks_per_block", C.c_int32),
                ("step_kernel", C.c_int32), ("march_rows", C.c_int32), ("march_members", C.c_int32),
                ("track_peak", C.c_int32), ("n_classes", C.c_int32), ("class_runoff", C.POINTER(C.c_double)),
                ("class_drain", C.POINTER(C.c_int32)), ("member_class_n", C.POINTER(C.c_double)),
                ("member_drain", C.POINTER(C.c_double)), ("n_inflow", C.c_int32),
                ("inflow", C.POINTER(C.c_int32)), ("n_series", C.c_int32), ("inflow_q", C.POINTER(C.c_double))]


_lib = None


def load_library():
    """Load libflood.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libflood.so not found at %s: build it with __graft_entry__.build() or "
                           "python paper_2302_08341_amd/build.py" % LIB_PATH)
    # torch carries its own HIP runtime; when torch is present it is loaded first, so
    # that the library binds to the same runtime (one HIP runtime per process)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    H = C.c_void_p
    dp, ip, lp, fp = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_float)
    sig = {
        "flood_create": [C.POINTER(FloodGrid), C.POINTER(FloodParams), C.c_int32, dp, dp, C.c_void_p,
                         C.POINTER(H)],
        "flood_create_batch": [C.c_int32, C.POINTER(FloodGrid), C.POINTER(FloodParams), ip, C.POINTER(dp),
                               C.POINTER(dp), C.c_void_p, C.POINTER(H)],
        "flood_step": [H, C.c_double],
        "flood_assimilate": [H, C.c_int32, C.c_int32, ip, dp, dp, C.c_double, C.c_double, dp, dp, ip, ip],
        "flood_adjoint": [H, C.c_int32, C.c_double, C.c_double, C.c_int32, ip, dp, C.c_int32, dp, dp, dp],
        "flood_get_field": [H, C.c_int32, C.c_int32, C.c_int32, dp],
        "flood_set_state": [H, C.c_int32, C.c_int32, dp, dp, dp, C.c_double],
        "flood_set_params": [H, C.c_int32, fp, dp, dp],
        "flood_get_ledger": [H, C.c_int32, dp, dp, dp, dp, dp, dp, dp, lp],
        "flood_set_sections": [H, C.c_int32, C.c_int32, ip, ip],
        "flood_get_sections": [H, C.c_int32, dp],
        "flood_assimilate_obs": [H, C.c_int32, C.c_int32, ip, dp, dp, C.c_double, C.c_double, C.c_double, dp, dp,
                                 ip, ip],
        "flood_get_land_params": [H, C.c_int32, dp, dp],
        "flood_get_weights": [H, C.c_int32, dp, dp, dp],
        "flood_systematic_resample": [dp, C.c_int32, C.c_double, ip, C.c_void_p],
        "flood_systematic_resample_noalloc": [dp, C.c_int32, C.c_double, ip, C.c_void_p],
        "flood_device_snapshot": [H, C.c_int32],
        "flood_get_march_rows": [H, C.c_int32, ip],
        "flood_probe_stream": [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, dp,
                               dp],
        "flood_ensemble_products": [H, C.c_int32, C.c_double, C.c_int32, dp, dp, dp, dp],
        "flood_save": [H, C.c_char_p],
        "flood_load": [H, C.c_char_p],
        "flood_get_config": [H, ip, ip, ip, ip, ip, ip, ip, ip],
        "flood_timing": [H, C.c_int32],
        "flood_get_timing": [H, dp, lp],
        "flood_adjoint_release": [H],
        "flood_step_n": [H, C.c_double, C.c_int64],
        "flood_get_wet_mask": [H, C.c_int32, C.c_int32, C.POINTER(C.c_uint8), C.POINTER(C.c_uint8)],
        "flood_log_steps": [H, C.c_int32],
        "flood_get_step_log": [H, C.c_int32, dp, dp, lp],
        "flood_get_adjoint_info": [H, ip, ip, ip],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int32
    lib.flood_last_error.argtypes = [H]
    lib.flood_last_error.restype = C.c_char_p
    lib.flood_strerror.argtypes = [C.c_int32]
    lib.flood_strerror.restype = C.c_char_p
    lib.flood_destroy.argtypes = [H]
    lib.flood_destroy.restype = None
    _lib = lib
    return lib


def _check(rc, handle=None):
    if rc != FLOOD_OK:
        msg = load_library().flood_last_error(handle)
        raise FloodError(rc, msg.decode() if msg else "")


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_int32))


def _fp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_float))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


def current_stream():
    """HIP stream handle of torch's current stream (None without torch or a device)."""
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


# ---------------------------------------------------------------------------
# C-named functions
# ---------------------------------------------------------------------------
def make_grid(dem, manning, dx, edge_kind=(0, 0, 0, 0), edge_slope=(0, 0, 0, 0), h0=None, land_class=None):
    dem, manning, h0 = _f32(dem), _f32(manning), _f32(h0)
    ny, nx = dem.shape
    lc = None if land_class is None else np.ascontiguousarray(np.asarray(land_class, dtype=np.uint8))
    g = FloodGrid(ny, nx, float(dx), _fp(dem), _fp(manning), _fp(h0), (C.c_int32 * 4)(*edge_kind),
                  (C.c_double * 4)(*[float(x) for x in edge_slope]),
                  lc.ctypes.data_as(C.POINTER(C.c_uint8)) if lc is not None else None)
    g._keep = (dem, manning, h0, lc)
    return g


def make_params(rain, rain_interval=300.0, cfl_alpha=0.7, h_dry=1e-3, dt_cap=10.0, dt_fixed=0.0, g=9.81,
                real_bytes=4, member_interleave=0, tile_rows=0, chunks_per_block=0, step_kernel=0, march_rows=0,
                march_members=0, track_peak=0, class_runoff=None, class_drain=None, member_class_n=None,
                member_drain=None, inflow=None, inflow_q=None):
    rain = _f64(np.asarray(rain, dtype=np.float64).ravel())
    rc = None if class_runoff is None else _f64(np.asarray(class_runoff, dtype=np.float64).ravel())
    cd = None if class_drain is None else np.ascontiguousarray(np.asarray(class_drain, dtype=np.int32).ravel())
    cn = None if member_class_n is None else _f64(np.asarray(member_class_n, dtype=np.float64).ravel())
    md = None if member_drain is None else _f64(np.asarray(member_drain, dtype=np.float64).ravel())
    inf = None if inflow is None else np.ascontiguousarray(np.asarray(inflow, dtype=np.int32).reshape(-1, 3))
    iq = None if inflow_q is None else _f64(np.atleast_2d(np.asarray(inflow_q, dtype=np.float64)))
    n_inf = 0 if inf is None else inf.shape[0]
    n_ser = 0 if iq is None or n_inf == 0 else iq.shape[0]
    p = FloodParams(_dp(rain) if rain.size else None, int(rain.size), float(rain_interval), float(cfl_alpha),
                    float(h_dry), float(dt_cap), float(dt_fixed), float(g), int(real_bytes),
                    int(member_interleave), int(tile_rows), int(chunks_per_block), int(step_kernel),
                    int(march_rows), int(march_members), int(bool(track_peak)),
                    0 if rc is None else int(rc.size), _dp(rc) if rc is not None else None,
                    cd.ctypes.data_as(C.POINTER(C.c_int32)) if cd is not None else None,
                    _dp(cn) if cn is not None else None, _dp(md) if md is not None else None,
                    n_inf, _ip(inf) if n_inf else None, n_ser, _dp(iq) if n_ser and iq.size else None)
    p._keep = (rain, rc, cd, cn, md, inf, iq)
    return p


def flood_create_batch(grids, params, members, n_scale=None, rain_mult=None, stream=None):
    lib = load_library()
    n = len(grids)
    G = (FloodGrid * n)(*grids)
    P = (FloodParams * n)(*params)
    M = np.ascontiguousarray(members, dtype=np.int32)
    keep = []
    ns = (C.POINTER(C.c_double) * n)()
    rm = (C.POINTER(C.c_double) * n)()
    for i in range(n):
        a = _f64(n_scale[i]) if n_scale is not None and n_scale[i] is not None else None
        b = _f64(rain_mult[i]) if rain_mult is not None and rain_mult[i] is not None else None
        keep += [a, b]
        ns[i] = _dp(a) if a is not None else C.POINTER(C.c_double)()
        rm[i] = _dp(b) if b is not None else C.POINTER(C.c_double)()
    h = C.c_void_p()
    rc = lib.flood_create_batch(n, G, P, _ip(M), ns, rm, stream, C.byref(h))
    _check(rc, None)
    return h


def flood_create(grid, params, n_members, n_scale=None, rain_mult=None, stream=None):
    return flood_create_batch([grid], [params], [n_members], [n_scale], [rain_mult], stream)


def flood_step(h, t_end):
    _check(load_library().flood_step(h, float(t_end)), h)


def flood_step_n(h, t_end, max_steps):
    _check(load_library().flood_step_n(h, float(t_end), int(max_steps)), h)


def flood_get_wet_mask(h, catchment, member, ny, nx):
    wx = np.zeros((ny, nx + 1), dtype=np.uint8)
    wy = np.zeros((ny + 1, nx), dtype=np.uint8)
    u8 = C.POINTER(C.c_uint8)
    rc = load_library().flood_get_wet_mask(h, int(catchment), int(member), wx.ctypes.data_as(u8),
                                           wy.ctypes.data_as(u8))
    _check(rc, h)
    return wx, wy


def flood_log_steps(h, capacity):
    _check(load_library().flood_log_steps(h, int(capacity)), h)


def flood_get_step_log(h, catchment, n_members, capacity):
    dt = np.zeros((n_members, capacity))
    te = np.zeros((n_members, capacity))
    cnt = np.zeros(n_members, dtype=np.int64)
    rc = load_library().flood_get_step_log(h, int(catchment), _dp(dt), _dp(te),
                                           cnt.ctypes.data_as(C.POINTER(C.c_int64)))
    _check(rc, h)
    return dt, te, cnt


def flood_assimilate(h, catchment, gauges, obs, sigma, neff_frac=0.8, u0=0.5, beta=None, n_members=None):
    g = np.ascontiguousarray(np.asarray(gauges, dtype=np.int32).reshape(-1, 2))
    obs, sigma, beta = _f64(obs), _f64(sigma), _f64(beta)
    N = n_members
    neff = C.c_double(0)
    anc = np.zeros(N, dtype=np.int32)
    res = C.c_int32(0)
    rc = load_library().flood_assimilate(h, int(catchment), g.shape[0], _ip(g), _dp(obs), _dp(sigma),
                                         float(neff_frac), float(u0), _dp(beta), C.byref(neff), _ip(anc),
                                         C.byref(res))
    _check(rc, h)
    return neff.value, anc, bool(res.value)


def flood_assimilate_obs(h, catchment, gauges, obs, sigma, alpha=0.0, neff_frac=0.8, u0=0.5, beta=None,
                         n_members=None):
    """Filter cycle on depth gauges followed by every registered streamflow section;
    obs and sigma hold the depths first, then the flows; alpha > 0: relative error
    with sigma as its floor."""
    g = np.ascontiguousarray(np.asarray(gauges, dtype=np.int32).reshape(-1, 2))
    obs, sigma, beta = _f64(obs), _f64(sigma), _f64(beta)
    N = n_members
    neff = C.c_double(0)
    anc = np.zeros(N, dtype=np.int32)
    res = C.c_int32(0)
    rc = load_library().flood_assimilate_obs(h, int(catchment), g.shape[0], _ip(g), _dp(obs), _dp(sigma),
                                             float(alpha), float(neff_frac), float(u0), _dp(beta), C.byref(neff),
                                             _ip(anc), C.byref(res))
    _check(rc, h)
    return neff.value, anc, bool(res.value)


def flood_set_sections(h, catchment, sections):
    """Register streamflow sections: a list of [n_links, 4] arrays (kind 0 x-link / 1 y-link,
    r, c, sign) in the host discharge layouts."""
    secs = [np.asarray(s, dtype=np.int32).reshape(-1, 4) for s in sections]
    counts = np.array([x.shape[0] for x in secs], dtype=np.int32)
    links = np.ascontiguousarray(np.concatenate(secs) if secs else np.zeros((0, 4), np.int32), dtype=np.int32)
    _check(load_library().flood_set_sections(h, int(catchment), len(secs), _ip(counts) if len(secs) else None,
                                             _ip(links) if links.size else None), h)


def flood_get_sections(h, catchment, n_members, n_sections):
    out = np.zeros(max(n_members * n_sections, 1))
    _check(load_library().flood_get_sections(h, int(catchment), _dp(out)), h)
    return out[:n_members * n_sections].reshape(n_members, n_sections)


def flood_adjoint(h, catchment, t_end, sample_dt, gauges, obs, ckpt_every, ny, nx, n_members):
    g = np.ascontiguousarray(np.asarray(gauges, dtype=np.int32).reshape(-1, 2))
    obs = _f64(obs)
    loss = C.c_double(0)
    gn = np.zeros(ny * nx)
    gm = np.zeros(n_members)
    rc = load_library().flood_adjoint(h, int(catchment), float(t_end), float(sample_dt), g.shape[0], _ip(g),
                                      _dp(obs), int(ckpt_every), C.byref(loss), _dp(gn), _dp(gm))
    _check(rc, h)
    return loss.value, gn.reshape(ny, nx), gm


def flood_get_field(h, catchment, member, which, shape):
    out = np.zeros(shape, dtype=np.float64)
    _check(load_library().flood_get_field(h, int(catchment), int(member), int(which), _dp(out)), h)
    return out


def flood_ensemble_products(h, catchment, threshold, pct, weights, ny, nx, n_members):
    pct = _f64(np.asarray(pct, dtype=np.float64).ravel())
    w = None if weights is None else _f64(weights)
    if w is not None and w.size != n_members:
        raise ValueError("weights must have one entry per member")
    prob = np.zeros(ny * nx)
    out = np.zeros(max(pct.size, 1) * ny * nx)
    _check(load_library().flood_ensemble_products(h, int(catchment), float(threshold), int(pct.size),
                                                  _dp(pct) if pct.size else None,
                                                  _dp(w) if w is not None else None, _dp(prob), _dp(out)), h)
    return prob.reshape(ny, nx), out[:pct.size * ny * nx].reshape(pct.size, ny, nx)


def flood_set_state(h, catchment, member, hh, qx, qy, t):
    hh, qx, qy = _f64(hh), _f64(qx), _f64(qy)
    _check(load_library().flood_set_state(h, int(catchment), int(member), _dp(hh), _dp(qx), _dp(qy), float(t)), h)


def flood_set_params(h, catchment, manning=None, n_scale=None, rain_mult=None):
    manning, n_scale, rain_mult = _f32(manning), _f64(n_scale), _f64(rain_mult)
    _check(load_library().flood_set_params(h, int(catchment), _fp(manning), _dp(n_scale), _dp(rain_mult)), h)


def flood_get_ledger(h, catchment, n_members):
    out = {k: np.zeros(n_members) for k in ("storage", "rain_in", "outflow", "clamp", "drain", "inflow", "t")}
    steps = np.zeros(n_members, dtype=np.int64)
    rc = load_library().flood_get_ledger(h, int(catchment), _dp(out["storage"]), _dp(out["rain_in"]),
                                         _dp(out["outflow"]), _dp(out["clamp"]), _dp(out["drain"]),
                                         _dp(out["inflow"]), _dp(out["t"]), steps.ctypes.data_as(C.POINTER(C.c_int64)))
    _check(rc, h)
    out["steps"] = steps
    return out


def flood_get_land_params(h, catchment, n_members, n_classes):
    cn = np.zeros(n_members * max(n_classes, 1))
    dr = np.zeros(n_members)
    _check(load_library().flood_get_land_params(h, int(catchment), _dp(cn), _dp(dr)), h)
    return cn[:n_members * n_classes].reshape(n_members, n_classes), dr


def flood_get_weights(h, catchment, n_members):
    lw, rm, ns = np.zeros(n_members), np.zeros(n_members), np.zeros(n_members)
    _check(load_library().flood_get_weights(h, int(catchment), _dp(lw), _dp(rm), _dp(ns)), h)
    return lw, rm, ns


def flood_systematic_resample(w, u0, stream=None):
    w = _f64(w)
    anc = np.zeros(w.size, dtype=np.int32)
    _check(load_library().flood_systematic_resample(_dp(w), w.size, float(u0), _ip(anc), stream), None)
    return anc


def flood_systematic_resample_noalloc(w, u0, stream=None):
    """flood_systematic_resample without any device allocation (library staging array)."""
    w = _f64(w)
    anc = np.zeros(w.size, dtype=np.int32)
    rc = load_library().flood_systematic_resample_noalloc(_dp(w), w.size, float(u0), _ip(anc), stream)
    _check(rc, None)
    return anc


def flood_probe_stream(ny, nx, n_members, rows, reps=5, waves_per_simd=0):
    """(GB/s, ms per launch) of a streaming kernel with the row-marching step's access
    pattern and no arithmetic (see flood_probe_stream in include/flood.h)."""
    gbps, ms = C.c_double(0.0), C.c_double(0.0)
    _check(load_library().flood_probe_stream(int(ny), int(nx), int(n_members), int(rows), int(reps),
                                            int(waves_per_simd), current_stream(), C.byref(gbps), C.byref(ms)))
    return gbps.value, ms.value


def flood_get_march_rows(h, catchment):
    v = C.c_int32(0)
    _check(load_library().flood_get_march_rows(h, int(catchment), C.byref(v)), h)
    return int(v.value)


def flood_device_snapshot(h, op):
    _check(load_library().flood_device_snapshot(h, int(op)), h)


def flood_save(h, path):
    _check(load_library().flood_save(h, path.encode()), h)


def flood_load(h, path):
    _check(load_library().flood_load(h, path.encode()), h)


def flood_get_config(h):
    v = [C.c_int32(0) for _ in range(8)]
    _check(load_library().flood_get_config(h, *[C.byref(x) for x in v]), h)
    return {"member_interleave": v[0].value, "tile_rows": v[1].value, "chunks_per_block": v[2].value,
            "graph_steps": v[3].value, "step_kernel": v[4].value, "march_rows": v[5].value,
            "march_members": v[6].value, "march_order": v[7].value}


def flood_adjoint_release(h):
    """Free the scratch flood_adjoint keeps on the handle between calls."""
    _check(load_library().flood_adjoint_release(h), h)


TIMING_LAUNCH, TIMING_BATCH = 1, 2


def flood_timing(h, mode):
    """mode: 0 / False off, 1 / True an event pair around every step launch with the
    graph path off, 2 an event pair around every captured batch of steps."""
    _check(load_library().flood_timing(h, int(mode)), h)


def flood_get_timing(h):
    avg = C.c_double(0)
    n = C.c_int64(0)
    _check(load_library().flood_get_timing(h, C.byref(avg), C.byref(n)), h)
    return avg.value, n.value


def flood_get_adjoint_info(h):
    g, n, sg = C.c_int32(0), C.c_int32(0), C.c_int32(0)
    _check(load_library().flood_get_adjoint_info(h, C.byref(g), C.byref(n), C.byref(sg)), h)
    return {"groups": g.value, "group_size": n.value, "segments": sg.value}


def flood_destroy(h):
    if h:
        load_library().flood_destroy(h)


# ---------------------------------------------------------------------------
# object wrapper
# ---------------------------------------------------------------------------
class FloodEnsemble:
    """Ensemble of one or more catchments resident on the GPU."""

    def __init__(self, catchments, rain, rain_interval=300.0, cfl_alpha=0.7, h_dry=1e-3, dt_cap=10.0,
                 dt_fixed=0.0, g=9.81, real_bytes=4, member_interleave=0, tile_rows=0, chunks_per_block=0,
                 step_kernel=0, march_rows=0, march_members=0, track_peak=False, stream="torch"):
        self.catchments = list(catchments)
        grids, params = [], []
        for c in self.catchments:
            grids.append(make_grid(c["dem"], c["manning"], c["dx"], c.get("edge_kind", (0, 0, 0, 0)),
                                   c.get("edge_slope", (0, 0, 0, 0)), c.get("h0"), c.get("land_class")))
            params.append(make_params(rain, rain_interval, cfl_alpha, h_dry, dt_cap, dt_fixed, g, real_bytes,
                                      member_interleave, tile_rows, chunks_per_block, step_kernel, march_rows,
                                      march_members, track_peak, c.get("class_runoff"), c.get("class_drain"),
                                      c.get("class_n"), c.get("drain"), c.get("inflow"), c.get("inflow_q")))
        self._keep = (grids, params)
        self.stream = current_stream() if stream == "torch" else stream
        self.h = flood_create_batch(grids, params, [c["n_members"] for c in self.catchments],
                                    [c.get("n_scale") for c in self.catchments],
                                    [c.get("rain_mult") for c in self.catchments], self.stream)
        self._n_sections = [0] * len(self.catchments)
        for i, c in enumerate(self.catchments):
            if c.get("sections") is not None and len(c["sections"]):
                self.set_sections(c["sections"], i)

    @classmethod
    def from_workload(cls, wl, catchments=None, members=None, **over):
        cs = []
        for i, c in enumerate(wl.catchments):
            if catchments is not None and i not in catchments:
                continue
            n = c.n_members if members is None else members
            d = dict(dem=c.dem, manning=c.manning, dx=c.dx, edge_kind=c.edge_kind, edge_slope=c.edge_slope,
                     h0=c.h0, n_members=n, n_scale=c.n_scale[:n], rain_mult=c.rain_mult[:n])
            if getattr(c, "land_class", None) is not None:
                d.update(land_class=c.land_class, class_runoff=c.class_runoff, class_drain=c.class_drain,
                         class_n=c.class_n[:n], drain=c.drain[:n])
            if getattr(c, "inflow", None) is not None:
                d.update(inflow=c.inflow, inflow_q=c.inflow_q)
            if getattr(c, "sections", None) is not None:
                d.update(sections=c.sections)
            cs.append(d)
        kw = dict(rain_interval=wl.rain_interval, cfl_alpha=wl.cfl_alpha, h_dry=wl.h_dry, dt_cap=wl.dt_cap,
                  dt_fixed=wl.dt_fixed, g=wl.g, real_bytes=wl.real_bytes)
        kw.update(over)
        return cls(cs, wl.rain, **kw)

    def shape(self, c=0):
        d = self.catchments[c]["dem"]
        return d.shape

    def n_members(self, c=0):
        return self.catchments[c]["n_members"]

    def step(self, t_end):
        flood_step(self.h, t_end)

    def step_n(self, t_end, max_steps):
        """At most max_steps steps of every member toward t_end (flood_step_n)."""
        flood_step_n(self.h, t_end, max_steps)

    def wet_mask(self, member, catchment=0):
        """(wet_x [ny, nx+1], wet_y [ny+1, nx]) uint8: the links' wet/dry decision for the next step."""
        ny, nx = self.shape(catchment)
        return flood_get_wet_mask(self.h, catchment, member, ny, nx)

    def log_steps(self, capacity):
        """Open (restart) the step log with capacity entries per member; 0 closes it."""
        self._log_cap = int(capacity)
        flood_log_steps(self.h, capacity)

    def step_log(self, catchment=0):
        """(dt [N, cap], t_end [N, cap], count [N]) logged since log_steps."""
        return flood_get_step_log(self.h, catchment, self.n_members(catchment), self._log_cap)

    def assimilate(self, catchment, gauges, obs, sigma, neff_frac=0.8, u0=0.5, beta=None):
        return flood_assimilate(self.h, catchment, gauges, obs, sigma, neff_frac, u0, beta,
                                n_members=self.n_members(catchment))

    def assimilate_obs(self, catchment, gauges, obs, sigma, alpha=0.0, neff_frac=0.8, u0=0.5, beta=None):
        """Depth gauges and the registered streamflow sections together (see flood_assimilate_obs)."""
        return flood_assimilate_obs(self.h, catchment, gauges, obs, sigma, alpha, neff_frac, u0, beta,
                                    n_members=self.n_members(catchment))

    def set_sections(self, sections, catchment=0):
        flood_set_sections(self.h, catchment, sections)
        self._n_sections[catchment] = len(sections)

    def sections(self, catchment=0):
        """Discharge through every registered section, [N, n_sections] (m^3/s)."""
        return flood_get_sections(self.h, catchment, self.n_members(catchment), self._n_sections[catchment])

    def adjoint(self, catchment, t_end, sample_dt, gauges, obs, ckpt_every=100):
        ny, nx = self.shape(catchment)
        return flood_adjoint(self.h, catchment, t_end, sample_dt, gauges, obs, ckpt_every, ny, nx,
                             self.n_members(catchment))

    def field(self, member, which=FIELD_H, catchment=0):
        ny, nx = self.shape(catchment)
        shape = {FIELD_H: (ny, nx), FIELD_QX: (ny, nx + 1), FIELD_QY: (ny + 1, nx), FIELD_PEAK: (ny, nx)}[which]
        return flood_get_field(self.h, catchment, member, which, shape)

    def products(self, threshold, pct=(), weights=None, catchment=0):
        """(probability map [ny, nx], percentile maps [len(pct), ny, nx]) of the running
        maximum depth; needs track_peak=True."""
        ny, nx = self.shape(catchment)
        return flood_ensemble_products(self.h, catchment, threshold, pct, weights, ny, nx,
                                       self.n_members(catchment))

    def set_state(self, member, h, qx, qy, t, catchment=0):
        flood_set_state(self.h, catchment, member, h, qx, qy, t)

    def set_params(self, catchment=0, manning=None, n_scale=None, rain_mult=None):
        flood_set_params(self.h, catchment, manning, n_scale, rain_mult)

    def ledger(self, catchment=0):
        return flood_get_ledger(self.h, catchment, self.n_members(catchment))

    def weights(self, catchment=0):
        return flood_get_weights(self.h, catchment, self.n_members(catchment))

    def land_params(self, catchment=0):
        """(member class roughness [N, n_classes], member drainage rates [N]) of a land-cover catchment."""
        c = self.catchments[catchment]
        k = 0 if c.get("class_runoff") is None else len(c["class_runoff"])
        return flood_get_land_params(self.h, catchment, self.n_members(catchment), k)

    def save(self, path):
        flood_save(self.h, path)

    def march_rows(self, catchment=0):
        """Rows per strip of the row-marching step kernels for one catchment."""
        return flood_get_march_rows(self.h, catchment)

    def snapshot(self):
        """Keep every member's state on the device (flood_device_snapshot, TAKE)."""
        flood_device_snapshot(self.h, SNAPSHOT_TAKE)

    def restore(self):
        """Return to the last device snapshot (flood_device_snapshot, RESTORE)."""
        flood_device_snapshot(self.h, SNAPSHOT_RESTORE)

    def snapshot_release(self):
        flood_device_snapshot(self.h, SNAPSHOT_RELEASE)

    def load(self, path):
        flood_load(self.h, path)

    def config(self):
        return flood_get_config(self.h)

    def timing(self, mode):
        flood_timing(self.h, mode)

    def get_timing(self):
        return flood_get_timing(self.h)

    def adjoint_info(self):
        """Member groups, group size and tape segments of the last adjoint call."""
        return flood_get_adjoint_info(self.h)

    def adjoint_release(self):
        """Free the adjoint's scratch (tape, checkpoints) held since the last adjoint call."""
        flood_adjoint_release(self.h)

    def close(self):
        if self.h:
            flood_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
