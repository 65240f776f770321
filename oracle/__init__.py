"""FP64 serial CPU oracle of the ensemble flood model (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product library (``paper_2302_08341_amd``) never
imports, links or calls it; the two share no code.  The arithmetic lives in
``flood_oracle.c`` (plain C, double precision, contraction off); this module
only marshals arguments and performs the particle filter's member copy, which
is plain array copying.

Where the paper is silent or ambiguous, the C source states the reading it
takes beside the code that takes it (wet/dry threshold, donor limiter, open
edges, land cover, inflow links, sections, relative observation error).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "flood_oracle.c")
# FLOOD_ORACLE_LIB names another build of the same source (the sanitizer build
# of the CPU test suite); it is loaded as it is, never rebuilt
_LIB_ENV = os.environ.get("FLOOD_ORACLE_LIB")
_LIB = _LIB_ENV or os.path.join(_HERE, "_liborc.so")

EDGE_WALL, EDGE_OPEN = 0, 1


_CFLAGS = ["-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (serial, -O2, no FP contraction)."""
    if _LIB_ENV:
        return _LIB
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2"] + _CFLAGS + ["-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitized(path: str) -> str:
    """Compile the same source with AddressSanitizer and UndefinedBehaviorSanitizer
    (every report fatal) into path; load it by setting FLOOD_ORACLE_LIB and
    preloading gcc's libasan."""
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all"] + _CFLAGS + ["-o", path, _SRC, "-lm"])
    return path


class _Model(C.Structure):
    _fields_ = [("ny", C.c_int32), ("nx", C.c_int32), ("dx", C.c_double),
                ("z", C.POINTER(C.c_double)), ("n", C.POINTER(C.c_double)),
                ("edge_kind", C.c_int32 * 4), ("edge_slope", C.c_double * 4),
                ("rain", C.POINTER(C.c_double)), ("n_rain", C.c_int32), ("rain_interval", C.c_double),
                ("alpha", C.c_double), ("h_dry", C.c_double), ("dt_cap", C.c_double),
                ("dt_fixed", C.c_double), ("g", C.c_double), ("wet_fp32", C.c_int32),
                ("cls", C.POINTER(C.c_uint8)), ("n_classes", C.c_int32),
                ("class_runoff", C.POINTER(C.c_double)), ("class_drain", C.POINTER(C.c_int32)),
                ("n_inflow", C.c_int32), ("inflow", C.POINTER(C.c_int32)), ("inflow_q", C.POINTER(C.c_double)),
                ("n_series", C.c_int32)]


class _Member(C.Structure):
    _fields_ = [("h", C.POINTER(C.c_double)), ("qx", C.POINTER(C.c_double)), ("qy", C.POINTER(C.c_double)),
                ("t", C.c_double), ("s", C.c_double), ("mu", C.c_double),
                ("v_rain", C.c_double), ("v_out", C.c_double), ("v_clamp", C.c_double),
                ("steps", C.c_int64), ("hmax", C.POINTER(C.c_double)),
                ("class_n", C.POINTER(C.c_double)), ("drain_rate", C.c_double), ("v_drain", C.c_double),
                ("v_in", C.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not _LIB_ENV and (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build(force=True)
        lib = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        lp = C.POINTER(C.c_int64)
        Mp = C.POINTER(_Model)
        Sp = C.POINTER(_Member)
        lib.orc_dt_cfl.restype = C.c_double
        lib.orc_dt_cfl.argtypes = [Mp, dp]
        lib.orc_step.argtypes = [Mp, Sp, C.c_double]
        u8 = C.POINTER(C.c_uint8)
        lib.orc_step_forced.argtypes = [Mp, Sp, C.c_double, C.c_double, u8, u8]
        lib.orc_link_depths.argtypes = [Mp, dp, dp, dp]
        lib.orc_wet_masks.argtypes = [Mp, dp, C.c_double, C.c_int32, u8, u8]
        lib.orc_advance.argtypes = [Mp, Sp, C.c_double, C.c_int64, dp, C.c_int64, lp]
        lib.orc_storage.restype = C.c_double
        lib.orc_storage.argtypes = [Mp, dp]
        lib.orc_pf_weights.argtypes = [C.c_int32, C.c_int32, dp, dp, dp, dp, dp, dp, dp]
        lib.orc_systematic.argtypes = [C.c_int32, dp, C.c_double, ip]
        lib.orc_section_flow.argtypes = [Mp, dp, dp, C.c_int32, ip, dp]
        lib.orc_obs_sigma.argtypes = [C.c_int32, dp, dp, C.c_double, dp]
        lib.orc_pf.argtypes = [C.c_int32, C.c_int32, dp, dp, dp, dp, C.c_double, C.c_double, dp, ip, ip]
        lib.orc_loss.argtypes = [Mp, Sp, C.c_double, C.c_double, C.c_int32, ip, dp, dp, dp, C.c_int64, dp]
        lib.orc_adjoint.argtypes = [Mp, Sp, C.c_double, C.c_double, C.c_int32, ip, dp, C.c_int32, dp, dp, dp,
                                    dp, dp, C.c_int64, lp]
        lib.orc_adj_step.argtypes = [Mp, C.c_double, C.c_double, dp, dp, dp, C.c_double, C.c_double, dp, dp, dp,
                                     dp, dp]
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Model:
    """Static description of one catchment: grid, bed, roughness, edges, rain, step policy."""

    def __init__(self, dem, manning, dx, rain, rain_interval=300.0, edge_kind=(0, 0, 0, 0),
                 edge_slope=(0.0, 0.0, 0.0, 0.0), alpha=0.7, h_dry=1e-3, dt_cap=10.0, dt_fixed=0.0, g=9.81,
                 wet_fp32=False, land_class=None, class_runoff=None, class_drain=None, inflow=None, inflow_q=None):
        """wet_fp32: take each link's wet/dry decision in single precision (flow depth
        in difference form, rounded to float, against h_dry rounded to float), as a
        single-precision model does; for comparisons from the same float state.

        land_class [ny, nx] (uint8 < n_classes), class_runoff [n_classes] and
        class_drain [n_classes] switch on land cover (Sec. 4.1, Table 1): each member
        then carries its own Manning n per class and a drainage rate (Member.class_n,
        Member.drain_rate), rain is scaled by the cell's runoff coefficient, and
        draining classes lose water at the member's rate, up to what they hold.

        inflow [n, 3] (edge N=0 E=1 S=2 W=3, position along the edge, series index)
        and inflow_q [n_series, n_rain] (inward discharge per unit width, m^2/s,
        piecewise constant over the rain blocks) prescribe inflow hydrographs on
        edge links (Sec. 4.1)."""
        self.z = _f64(dem)
        self.n = _f64(manning)
        self.ny, self.nx = self.z.shape
        self.dx = float(dx)
        self.rain = _f64(rain).ravel()
        if self.rain.size == 0:
            self.rain = np.zeros(1)
            n_rain = 0
        else:
            n_rain = self.rain.size
        if land_class is not None:
            self.cls = np.ascontiguousarray(np.asarray(land_class, dtype=np.uint8))
            assert self.cls.shape == self.z.shape
            self.class_runoff = _f64(class_runoff).ravel()
            self.class_drain = np.ascontiguousarray(np.asarray(class_drain, dtype=np.int32).ravel())
            self.n_classes = self.class_runoff.size
            assert self.class_drain.size == self.n_classes and int(self.cls.max()) < self.n_classes
            cls_p = self.cls.ctypes.data_as(C.POINTER(C.c_uint8))
            rc_p, dr_p = _dp(self.class_runoff), self.class_drain.ctypes.data_as(C.POINTER(C.c_int32))
        else:
            self.cls = None
            self.n_classes = 0
            cls_p, rc_p, dr_p = C.POINTER(C.c_uint8)(), C.POINTER(C.c_double)(), C.POINTER(C.c_int32)()
        if inflow is not None and len(inflow) > 0:
            self.inflow = np.ascontiguousarray(np.asarray(inflow, dtype=np.int32).reshape(-1, 3))
            self.inflow_q = np.ascontiguousarray(np.asarray(inflow_q, dtype=np.float64))
            assert self.inflow_q.ndim == 2 and self.inflow_q.shape[1] == n_rain
            inf_p, infq_p = _ip(self.inflow), _dp(self.inflow_q)
            n_inf, n_ser = self.inflow.shape[0], self.inflow_q.shape[0]
        else:
            self.inflow = self.inflow_q = None
            inf_p, infq_p, n_inf, n_ser = C.POINTER(C.c_int32)(), C.POINTER(C.c_double)(), 0, 0
        self._m = _Model(self.ny, self.nx, self.dx, _dp(self.z), _dp(self.n),
                         (C.c_int32 * 4)(*edge_kind), (C.c_double * 4)(*edge_slope),
                         _dp(self.rain), n_rain, float(rain_interval), float(alpha), float(h_dry),
                         float(dt_cap), float(dt_fixed), float(g), int(bool(wet_fp32)),
                         cls_p, int(self.n_classes), rc_p, dr_p, n_inf, inf_p, infq_p, n_ser)
        self.edge_kind = tuple(edge_kind)
        self.edge_slope = tuple(edge_slope)
        self.h_dry = h_dry
        self.g = g

    @classmethod
    def from_workload(cls, wl, catchment=0, **over):
        c = wl.catchments[catchment]
        kw = dict(rain_interval=wl.rain_interval, edge_kind=c.edge_kind, edge_slope=c.edge_slope,
                  alpha=wl.cfl_alpha, h_dry=wl.h_dry, dt_cap=wl.dt_cap, dt_fixed=wl.dt_fixed, g=wl.g)
        if getattr(c, "land_class", None) is not None:
            kw.update(land_class=c.land_class, class_runoff=c.class_runoff, class_drain=c.class_drain)
        if getattr(c, "inflow", None) is not None:
            kw.update(inflow=c.inflow, inflow_q=c.inflow_q)
        kw.update(over)
        return cls(c.dem, c.manning, c.dx, wl.rain, **kw)

    @property
    def ptr(self):
        return C.byref(self._m)


@dataclass
class Member:
    h: np.ndarray
    qx: np.ndarray
    qy: np.ndarray
    t: float = 0.0
    s: float = 1.0
    mu: float = 1.0
    v_rain: float = 0.0
    v_out: float = 0.0
    v_clamp: float = 0.0
    steps: int = 0
    dt_log: list = field(default_factory=list)
    hmax: Optional[np.ndarray] = None     # running maximum depth, when tracked
    class_n: Optional[np.ndarray] = None  # land cover: this member's Manning n per class
    drain_rate: float = 0.0               # land cover: drainage rate, m/s
    v_drain: float = 0.0
    v_in: float = 0.0                     # volume entered through inflow links

    @classmethod
    def dry(cls, model: Model, s=1.0, mu=1.0, h0=None, track_max=False, class_n=None, drain_rate=0.0):
        h = np.zeros((model.ny, model.nx)) if h0 is None else _f64(h0).copy()
        return cls(h=h, qx=np.zeros((model.ny, model.nx + 1)), qy=np.zeros((model.ny + 1, model.nx)),
                   s=float(s), mu=float(mu), hmax=h.copy() if track_max else None,
                   class_n=None if class_n is None else _f64(class_n).ravel().copy(),
                   drain_rate=float(drain_rate))

    def copy(self):
        return Member(self.h.copy(), self.qx.copy(), self.qy.copy(), self.t, self.s, self.mu, self.v_rain,
                      self.v_out, self.v_clamp, self.steps, list(self.dt_log),
                      None if self.hmax is None else self.hmax.copy(),
                      None if self.class_n is None else self.class_n.copy(), self.drain_rate, self.v_drain,
                      self.v_in)

    def _c(self):
        for a in (self.h, self.qx, self.qy):
            assert a.flags.c_contiguous and a.dtype == np.float64
        if self.hmax is not None:
            assert self.hmax.flags.c_contiguous and self.hmax.dtype == np.float64 and self.hmax.shape == self.h.shape
        hm = _dp(self.hmax) if self.hmax is not None else C.POINTER(C.c_double)()
        cn = _dp(self.class_n) if self.class_n is not None else C.POINTER(C.c_double)()
        return _Member(_dp(self.h), _dp(self.qx), _dp(self.qy), self.t, self.s, self.mu, self.v_rain,
                       self.v_out, self.v_clamp, self.steps, hm, cn, float(self.drain_rate), self.v_drain,
                       self.v_in)

    def _back(self, cm):
        self.t, self.v_rain, self.v_out, self.v_clamp, self.steps = cm.t, cm.v_rain, cm.v_out, cm.v_clamp, cm.steps
        self.v_drain = cm.v_drain
        self.v_in = cm.v_in


def dt_cfl(model: Model, h) -> float:
    h = _f64(h)
    return _load().orc_dt_cfl(model.ptr, _dp(h))


def step(model: Model, mem: Member, dt: float) -> None:
    cm = mem._c()
    rc = _load().orc_step(model.ptr, C.byref(cm), float(dt))
    if rc:
        raise ValueError("orc_step failed: %d" % rc)
    mem._back(cm)


def _u8(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint8))


def step_forced(model: Model, mem: Member, dt: float, t_next: float, wet_x, wet_y) -> None:
    """One step of length dt ending at t_next with every link's wet/dry decision given
    (wet_x [ny, nx+1], wet_y [ny+1, nx], 1 wet / 0 dry): replay of another model's
    trajectory, its step lengths and its decisions."""
    wx = np.ascontiguousarray(wet_x, dtype=np.uint8)
    wy = np.ascontiguousarray(wet_y, dtype=np.uint8)
    assert wx.shape == (model.ny, model.nx + 1) and wy.shape == (model.ny + 1, model.nx)
    cm = mem._c()
    rc = _load().orc_step_forced(model.ptr, C.byref(cm), float(dt), float(t_next), _u8(wx), _u8(wy))
    if rc:
        raise ValueError("orc_step_forced failed: %d" % rc)
    mem._back(cm)


def replay(model: Model, mem: Member, dts, t_ends) -> None:
    """Advance mem by the given steps (lengths dts, end times t_ends), each link deciding
    wet/dry itself."""
    for dt, te in zip(dts, t_ends):
        step(model, mem, float(dt))
        mem.t = float(te)


def link_depths(model: Model, h):
    """Eq. 3 flow depth of every link as written (higher surface minus higher bed; edge
    links: the inner depth): (hx [ny, nx+1], hy [ny+1, nx])."""
    h = _f64(h)
    hx = np.zeros((model.ny, model.nx + 1))
    hy = np.zeros((model.ny + 1, model.nx))
    rc = _load().orc_link_depths(model.ptr, _dp(h), _dp(hx), _dp(hy))
    if rc:
        raise ValueError("orc_link_depths failed: %d" % rc)
    return hx, hy


MASK_LITERAL, MASK_FLOAT, MASK_DIFF64 = 0, 1, 2


def wet_masks(model: Model, h, t: float = 0.0, fp32: bool = False, mode: int = None):
    """Wet/dry decision of every link for the next step from depths h at time t (uint8
    (wet_x [ny, nx+1], wet_y [ny+1, nx])).  mode MASK_LITERAL: in double as Eq. 3 is
    written; MASK_FLOAT (or fp32=True): in single precision, flow depth in difference
    form; MASK_DIFF64: in double, difference form (a double-precision model's own)."""
    h = _f64(h)
    if mode is None:
        mode = MASK_FLOAT if fp32 else MASK_LITERAL
    wx = np.zeros((model.ny, model.nx + 1), dtype=np.uint8)
    wy = np.zeros((model.ny + 1, model.nx), dtype=np.uint8)
    rc = _load().orc_wet_masks(model.ptr, _dp(h), float(t), int(mode), _u8(wx), _u8(wy))
    if rc:
        raise ValueError("orc_wet_masks failed: %d" % rc)
    return wx, wy


def advance(model: Model, mem: Member, t_end: float, max_steps: int = 10 ** 12, log_dt: bool = False) -> int:
    cm = mem._c()
    n = C.c_int64(0)
    cap = 0
    buf = None
    if log_dt:
        cap = 1 << 20
        buf = np.zeros(cap)
    rc = _load().orc_advance(model.ptr, C.byref(cm), float(t_end), int(max_steps), _dp(buf), cap, C.byref(n))
    if rc:
        raise ValueError("orc_advance failed: %d" % rc)
    mem._back(cm)
    if log_dt:
        mem.dt_log.extend(buf[:min(n.value, cap)].tolist())
    return n.value


def storage(model: Model, h) -> float:
    h = _f64(h)
    return _load().orc_storage(model.ptr, _dp(h))


def section_flow(model: Model, mem: Member, links) -> float:
    """Streamflow through a section (Sec. 4.4), m^3/s: links [n, 4] = (kind 0 x-link /
    1 y-link, r, c, sign) in the oracle's link indexing."""
    l = np.ascontiguousarray(np.asarray(links, dtype=np.int32).reshape(-1, 4))
    out = C.c_double(0.0)
    rc = _load().orc_section_flow(model.ptr, _dp(mem.qx), _dp(mem.qy), l.shape[0], _ip(l), C.byref(out))
    if rc:
        raise ValueError("orc_section_flow failed: %d" % rc)
    return out.value


def obs_sigma(d, floor, alpha: float) -> np.ndarray:
    """Eq. 9's standard deviations: max(alpha |d_k|, floor_k) (alpha = 0: floor_k)."""
    d, floor = _f64(d).ravel(), _f64(floor).ravel()
    out = np.zeros(d.size)
    rc = _load().orc_obs_sigma(d.size, _dp(d), _dp(floor), float(alpha), _dp(out))
    if rc:
        raise ValueError("orc_obs_sigma failed: %d" % rc)
    return out


def pf_weights(y, d, sigma, logw_prior, alpha: float = 0.0):
    """Posterior log-weights, weights and N_eff; sigma is the floor of the relative
    standard deviation when alpha > 0 (obs_sigma)."""
    y = _f64(y)
    N, K = y.shape
    d, lw = _f64(d), _f64(logw_prior)
    sigma = obs_sigma(d, sigma, alpha) if alpha > 0.0 else _f64(sigma)
    lp = np.zeros(N)
    w = np.zeros(N)
    neff = C.c_double(0.0)
    rc = _load().orc_pf_weights(N, K, _dp(y), _dp(d), _dp(sigma), _dp(lw), _dp(lp), _dp(w), C.byref(neff))
    if rc:
        raise ValueError("orc_pf_weights failed: %d" % rc)
    return lp, w, neff.value


def systematic(w, u0: float) -> np.ndarray:
    w = _f64(w)
    anc = np.zeros(w.size, dtype=np.int32)
    rc = _load().orc_systematic(w.size, _dp(w), float(u0), _ip(anc))
    if rc:
        raise ValueError("orc_systematic failed: %d" % rc)
    return anc


def pf(y, d, sigma, logw, neff_frac: float, u0: float, alpha: float = 0.0):
    """Filter update; returns (new logw, neff, ancestors, resampled).  alpha > 0:
    relative standard deviations with sigma as their floor (obs_sigma)."""
    y = _f64(y)
    N, K = y.shape
    d = _f64(d)
    sigma = obs_sigma(d, sigma, alpha) if alpha > 0.0 else _f64(sigma)
    lw = _f64(logw).copy()
    neff = C.c_double(0.0)
    anc = np.zeros(N, dtype=np.int32)
    res = C.c_int32(0)
    rc = _load().orc_pf(N, K, _dp(y), _dp(d), _dp(sigma), _dp(lw), float(neff_frac), float(u0),
                        C.byref(neff), _ip(anc), C.byref(res))
    if rc:
        raise ValueError("orc_pf failed: %d" % rc)
    return lw, neff.value, anc, bool(res.value)


def gauge_values(members, gauges) -> np.ndarray:
    """Observation operator: depth at each gauge cell for every member, [N, K]."""
    g = np.asarray(gauges, dtype=np.int64).reshape(-1, 2)
    return np.array([[m.h[r, c] for r, c in g] for m in members], dtype=np.float64).reshape(len(members), len(g))


class Ensemble:
    """Members of one catchment plus their log-weights (equal at start)."""

    def __init__(self, model: Model, s, mu, h0=None, class_n=None, drain=None):
        self.model = model
        self.members = [Member.dry(model, s[i], mu[i], h0,
                                   class_n=None if class_n is None else class_n[i],
                                   drain_rate=0.0 if drain is None else drain[i]) for i in range(len(s))]
        self.logw = np.full(len(s), -np.log(len(s)))

    def advance(self, t_end: float, log_dt=False):
        return [advance(self.model, m, t_end, log_dt=log_dt) for m in self.members]

    def assimilate(self, gauges, obs, sigma, neff_frac, u0, beta=None, sections=(), alpha=0.0):
        """Filter cycle steps I-V of Sec. 3.3: gauge values, weights, N_eff, resampling, replacement.
        sections: streamflow sections (links as in section_flow) observed after the
        depth gauges; obs and sigma then hold the depths first, then the flows."""
        y = gauge_values(self.members, gauges)
        if len(sections):
            yq = np.array([[section_flow(self.model, m, sec) for sec in sections] for m in self.members])
            y = np.concatenate([y, yq], axis=1)
        lw, neff, anc, res = pf(y, obs, sigma, self.logw, neff_frac, u0, alpha)
        self.logw = lw
        if res:
            old = [m.copy() for m in self.members]
            self.members = [old[a].copy() for a in anc]
            if beta is not None:
                for j, m in enumerate(self.members):
                    m.mu = m.mu * float(beta[j])
        return neff, anc, res


def loss(model: Model, mem: Member, t_end, sample_dt, gauges, obs, replay=None) -> float:
    g = np.ascontiguousarray(np.asarray(gauges, dtype=np.int32).reshape(-1, 2))
    obs = _f64(obs)
    K = g.shape[0]
    cm = mem._c()
    out = C.c_double(0.0)
    rdt = rte = None
    nrep = 0
    if replay is not None:
        rdt, rte = _f64(replay[0]), _f64(replay[1])
        nrep = rdt.size
    rc = _load().orc_loss(model.ptr, C.byref(cm), float(t_end), float(sample_dt), K, _ip(g), _dp(obs),
                          _dp(rdt), _dp(rte), nrep, C.byref(out))
    if rc:
        raise ValueError("orc_loss failed: %d" % rc)
    mem._back(cm)
    return out.value


def adjoint(model: Model, mem: Member, t_end, sample_dt, gauges, obs, ckpt_every=100):
    """(loss, grad_n [ny,nx], grad_mu, (dt seq, end-time seq)) of one member."""
    g = np.ascontiguousarray(np.asarray(gauges, dtype=np.int32).reshape(-1, 2))
    obs = _f64(obs)
    K = g.shape[0]
    cm = mem._c()
    L = C.c_double(0.0)
    gmu = C.c_double(0.0)
    gn = np.zeros((model.ny, model.nx))
    cap = 1 << 20
    dts = np.zeros(cap)
    tes = np.zeros(cap)
    ns = C.c_int64(0)
    rc = _load().orc_adjoint(model.ptr, C.byref(cm), float(t_end), float(sample_dt), K, _ip(g), _dp(obs),
                             int(ckpt_every), C.byref(L), _dp(gn), C.byref(gmu), _dp(dts), _dp(tes), cap,
                             C.byref(ns))
    if rc:
        raise ValueError("orc_adjoint failed: %d" % rc)
    mem._back(cm)
    n = ns.value
    return L.value, gn, gmu.value, (dts[:n].copy(), tes[:n].copy())


def adj_step(model: Model, mem: Member, dt, lh, lqx, lqy):
    """Reverse one step of length dt from mem's state; returns (lh, lqx, lqy, grad_n, grad_mu)."""
    lh, lqx, lqy = _f64(lh).copy(), _f64(lqx).copy(), _f64(lqy).copy()
    gn = np.zeros((model.ny, model.nx))
    gmu = C.c_double(0.0)
    rc = _load().orc_adj_step(model.ptr, float(mem.s), float(mem.mu), _dp(mem.h), _dp(mem.qx), _dp(mem.qy),
                              float(dt), float(mem.t), _dp(lh), _dp(lqx), _dp(lqy), _dp(gn), C.byref(gmu))
    if rc:
        raise ValueError("orc_adj_step failed: %d" % rc)
    return lh, lqx, lqy, gn, gmu.value


def ensemble_products(hmax, threshold, pcts=(), weights=None):
    """Ensemble products of the maximum depth (Sec. 4.4, Figs. 15-16).

    hmax: [N, ...] running maximum depth of each member (any cell shape after the
    member axis).  weights: non-negative member weights (None: equal).  With
    W = sum of the weights:
      prob[c]   = (sum of w_m over members with hmax_m[c] >= threshold) / W
      pct_p[c]  = min{ hmax_k[c] : sum of w_m over members with hmax_m[c] <= hmax_k[c]
                                   >= p W }         (inverted distribution function)
    Every weight sum runs over members in index order in FP64, as written.
    Returns (prob, [pct for each p])."""
    v = np.asarray(hmax, dtype=np.float64)
    N = v.shape[0]
    w = np.ones(N) if weights is None else np.asarray(weights, dtype=np.float64)
    W = 0.0
    for m in range(N):
        W += w[m]
    hit = np.zeros(v.shape[1:])
    for m in range(N):
        hit = hit + np.where(v[m] >= threshold, w[m], 0.0)
    prob = hit / W
    best = [np.full(v.shape[1:], np.inf) for _ in pcts]
    for k in range(N):
        cum = np.zeros(v.shape[1:])
        for m in range(N):
            cum = cum + np.where(v[m] <= v[k], w[m], 0.0)
        for i, p in enumerate(pcts):
            take = (cum >= p * W) & (v[k] < best[i])
            best[i] = np.where(take, v[k], best[i])
    return prob, best
