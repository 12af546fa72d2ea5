"""Python binding of libtb.so, the gfx950 template-bank coherent orbital search
(arXiv:2112.11991) behind include/tb.h.

Argument marshalling only: every step of the search runs in the library's HIP
kernels.  Functions keep the C names (``tb_plan``, ``tb_load_series``,
``tb_search_templates``, ``tb_get_candidates`` ...); :class:`Plan` wraps them
for convenience.  Importing fails loudly when the library has not been built
(``python paper_2112_11991_amd/build.py``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtb.so")

TB_OK = 0
TB_ERR_INVALID_ARG = -1
TB_ERR_OOM = -2
TB_ERR_BUDGET = -3
TB_ERR_DEVICE = -4
TB_ERR_OVERFLOW = -5
TB_ERR_NOT_READY = -6
TB_ERR_UNKNOWN_ID = -7
TB_ERR_TOO_LARGE = -8
TB_NOALLOC_SCRATCH_BYTES = 160 << 20  # fixed device scratch of tb_search_templates_noalloc, per GPU
TB_MEM_HOST = 0
TB_MEM_DEVICE = 1
TB_SERIES_WHITENING = 2  # OR into the load flags: whiten once from the series' own spectrum
TB_DELAY_SERIES = 1  # tb_config.flags: Roemer delay from the App. B series (ELL7) instead of BT-Newton
TB_ZAP_MAX = 65536  # most birdie intervals per series
TB_BANK_CIRCULAR = 0  # bank coordinates (P_orb, tau, alpha)
TB_BANK_ELLIPTICAL = 1  # (P_orb, tau, alpha, e, psi)


class TbConfig(C.Structure):
    _fields_ = [
        ("max_log2n", C.c_uint32),
        ("harm_max", C.c_uint32),
        ("whiten_window", C.c_uint32),
        ("batch_templates", C.c_uint32),
        ("threshold_sigma", C.c_double),
        ("fmin_hz", C.c_double),
        ("fmax_hz", C.c_double),
        ("hbm_budget_bytes", C.c_uint64),
        ("ring_capacity", C.c_uint64),
        ("stream", C.c_void_p),
        ("device", C.c_int32),
        ("lanes", C.c_uint32),
        ("flags", C.c_uint32),
        ("tile_points", C.c_uint32),
    ]


class TbTemplate(C.Structure):
    _fields_ = [
        ("porb_s", C.c_double),
        ("tau_lts", C.c_double),
        ("alpha_rad", C.c_double),
        ("ecc", C.c_double),
        ("omega_rad", C.c_double),
    ]


TEMPLATE_DTYPE = np.dtype(
    [("porb_s", "<f8"), ("tau_lts", "<f8"), ("alpha_rad", "<f8"), ("ecc", "<f8"), ("omega_rad", "<f8")]
)
CANDIDATE_DTYPE = np.dtype(
    [
        ("series_id", "<u4"),
        ("template_id", "<u4"),
        ("bin", "<u4"),
        ("log2_harm", "u1"),
        ("reserved", "u1", (3,)),
        ("power", "<f4"),
        ("sigma", "<f4"),
        ("freq_hz", "<f8"),
    ]
)
assert CANDIDATE_DTYPE.itemsize == 32 and TEMPLATE_DTYPE.itemsize == C.sizeof(TbTemplate) == 40
assert C.sizeof(TbConfig) == 80

EXPORTS = [
    "tb_default_config", "tb_plan", "tb_destroy", "tb_load_series", "tb_unload_series", "tb_search_templates",
    "tb_poll", "tb_get_candidates", "tb_release", "tb_synchronize", "tb_strerror", "tb_inspect_template",
    "tb_thresholds", "tb_last_request_ms", "tb_profile", "tb_profile_read", "tb_stream_copy", "tb_memory",
    "tb_set_budget", "tb_distill", "tb_zap_series", "tb_bank_density", "tb_dedisperse", "tb_set_shape",
    "tb_search_templates_noalloc", "tb_bank_propose", "tb_bank_count", "tb_bank_select", "tb_serve",
]

# tb_serve_request / tb_serve_result records
SERVE_REQUEST_DTYPE = np.dtype([("t_arrival_s", "<f8"), ("series_id", "<i4"), ("count", "<u4"),
                                ("templates", "<u8"), ("first_template_id", "<u4"), ("reserved", "<u4")])
SERVE_RESULT_DTYPE = np.dtype([("t_admit_s", "<f8"), ("t_done_s", "<f8"), ("cand_offset", "<u8"),
                               ("n_copied", "<u8"), ("n_total", "<u8"), ("status", "<i4"), ("reserved", "<u4")])
assert SERVE_REQUEST_DTYPE.itemsize == 32 and SERVE_RESULT_DTYPE.itemsize == 48
TB_SERVE_SATURATE = 1


class TbBankMetric(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("nodes", C.c_uint32), ("tobs_s", C.c_double), ("fmax_hz", C.c_double)]


class TbBankPriors(C.Structure):
    _fields_ = [("porb_min_s", C.c_double), ("porb_max_s", C.c_double), ("m_pulsar_min_msun", C.c_double),
                ("m_comp_max_msun", C.c_double), ("ecc_max", C.c_double)]


class TbFilterbank(C.Structure):
    _fields_ = [("nchan", C.c_uint32), ("nbits", C.c_uint32), ("nsamp", C.c_uint64), ("fch1_mhz", C.c_double),
                ("foff_mhz", C.c_double), ("tsamp_s", C.c_double)]


class TbError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__("%s: %s (%d)" % (what, tb_strerror(status), status))


def _load():
    # torch ships its own HIP runtime (same soname as ROCm's).  Loading it
    # first makes libtb.so bind to that one runtime, so that torch streams and
    # device pointers handed to the library are valid in it; two runtimes in
    # one process would not see each other's devices.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            "libtb.so is not built at %s; run `python paper_2112_11991_amd/build.py` (hipcc, gfx950)" % LIB_PATH
        )
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    vp, i32, u32, i64, u64 = C.c_void_p, C.c_int32, C.c_uint32, C.c_int64, C.c_uint64
    L.tb_default_config.argtypes = [P(TbConfig)]
    L.tb_default_config.restype = None
    L.tb_plan.argtypes = [P(TbConfig), P(vp)]
    L.tb_destroy.argtypes = [vp]
    L.tb_load_series.argtypes = [vp, vp, u64, C.c_double, u32, P(i32)]
    L.tb_unload_series.argtypes = [vp, i32]
    L.tb_search_templates.argtypes = [vp, i32, vp, u32, u32, P(i64)]
    L.tb_search_templates_noalloc.argtypes = [vp, i32, vp, u32, u32, vp, u64, P(u64)]
    L.tb_poll.argtypes = [vp, i64]
    L.tb_get_candidates.argtypes = [vp, i64, vp, u64, P(u64), C.c_int]
    L.tb_release.argtypes = [vp, i64]
    L.tb_synchronize.argtypes = [vp]
    L.tb_strerror.argtypes = [C.c_int]
    L.tb_strerror.restype = C.c_char_p
    L.tb_inspect_template.argtypes = [vp, i32, P(TbTemplate), vp, vp, vp, vp]
    L.tb_thresholds.argtypes = [vp, vp]
    L.tb_last_request_ms.argtypes = [vp, i64, P(C.c_double)]
    L.tb_profile.argtypes = [vp, C.c_int]
    L.tb_profile_read.argtypes = [vp, vp, vp, P(u64)]
    L.tb_stream_copy.argtypes = [vp, vp, vp, u64, u32, P(C.c_double)]
    L.tb_memory.argtypes = [vp, P(u64), P(u64)]
    L.tb_set_budget.argtypes = [vp, u64]
    L.tb_distill.argtypes = [vp, u64, u32, u32, u32, vp, vp, P(u64)]
    L.tb_zap_series.argtypes = [vp, i32, vp, vp, u32]
    L.tb_set_shape.argtypes = [vp, u32, u32, u32]
    L.tb_bank_density.argtypes = [vp, P(TbBankMetric), vp, u64, vp, P(C.c_double)]
    L.tb_dedisperse.argtypes = [vp, P(TbFilterbank), vp, u32, vp, u32, vp, P(u64), P(C.c_double)]
    L.tb_bank_propose.argtypes = [vp, P(TbBankMetric), P(TbBankPriors), vp, u64, vp, vp, vp, P(C.c_double)]
    L.tb_bank_count.argtypes = [C.c_double, u32, C.c_double, C.c_double, P(C.c_double)]
    L.tb_bank_select.argtypes = [vp, vp, u64, C.c_double, vp, P(u64), P(u64)]
    L.tb_serve.argtypes = [vp, vp, u32, C.c_double, u32, vp, u64, vp, vp]
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("tb_default_config", "tb_strerror"):
            f.restype = C.c_int
    return L


_L = _load()


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, int):
        return C.c_void_p(a)
    return a.ctypes.data_as(C.c_void_p)


def _check(st: int, what: str):
    if st != TB_OK:
        raise TbError(st, what)


# ---------------------------------------------------------------- C names --
def tb_default_config() -> TbConfig:
    c = TbConfig()
    _L.tb_default_config(C.byref(c))
    return c


def tb_strerror(status: int) -> str:
    return _L.tb_strerror(int(status)).decode()


def tb_plan(cfg: TbConfig) -> int:
    h = C.c_void_p()
    _check(_L.tb_plan(C.byref(cfg), C.byref(h)), "tb_plan")
    return h.value


def tb_destroy(plan: int) -> None:
    _check(_L.tb_destroy(C.c_void_p(plan)), "tb_destroy")


def tb_load_series(plan: int, data, tsamp: float, n: int | None = None, flags: int = TB_MEM_HOST) -> int:
    """data: float32 numpy array (TB_MEM_HOST) or a device address (TB_MEM_DEVICE, n required);
    flags may also carry TB_SERIES_WHITENING."""
    sid = C.c_int32(-1)
    if (flags & TB_MEM_DEVICE) == TB_MEM_HOST:
        data = np.ascontiguousarray(data, dtype=np.float32)
        n = data.size
    _check(_L.tb_load_series(C.c_void_p(plan), _ptr(data), int(n), float(tsamp), int(flags), C.byref(sid)),
           "tb_load_series")
    return sid.value


def tb_unload_series(plan: int, series_id: int) -> None:
    _check(_L.tb_unload_series(C.c_void_p(plan), int(series_id)), "tb_unload_series")


def as_templates(templates) -> np.ndarray:
    if isinstance(templates, np.ndarray) and templates.dtype.names == TEMPLATE_DTYPE.names:
        return np.ascontiguousarray(templates.astype(TEMPLATE_DTYPE, copy=False))
    arr = np.zeros(len(templates), dtype=TEMPLATE_DTYPE)
    for i, t in enumerate(templates):
        arr[i] = tuple(float(v) for v in t)
    return arr


def tb_search_templates(plan: int, series_id: int, templates, first_template_id: int = 0) -> int:
    arr = as_templates(templates)
    rid = C.c_int64(0)
    _check(_L.tb_search_templates(C.c_void_p(plan), int(series_id), _ptr(arr), len(arr), int(first_template_id),
                                  C.byref(rid)), "tb_search_templates")
    return rid.value


def tb_search_templates_noalloc(plan: int, series_id: int, templates, first_template_id: int = 0,
                                capacity: int = 1 << 16, allow_overflow: bool = False):
    """The allocation-free search (blocking): (sorted candidates, n_total).
    On overflow (allow_overflow) the capacity records kept are returned."""
    arr = as_templates(templates)
    out = np.zeros(int(capacity), dtype=CANDIDATE_DTYPE)
    n = C.c_uint64(0)
    st = _L.tb_search_templates_noalloc(C.c_void_p(plan), int(series_id), _ptr(arr), len(arr),
                                        int(first_template_id), _ptr(out) if out.size else None, out.size,
                                        C.byref(n))
    if not (st == TB_ERR_OVERFLOW and allow_overflow):
        _check(st, "tb_search_templates_noalloc")
    return out[:min(out.size, int(n.value))], int(n.value)


def tb_serve(plan: int, requests, time_scale: float = 1.0, saturate: bool = False, capacity: int = 1 << 20):
    """Runs a request stream through the library's serving loop.  requests:
    (t_arrival_s, series_id, templates, first_template_id) tuples.  Returns
    (results SERVE_RESULT_DTYPE in request order, candidates of all requests
    in completion order, (most in flight, budget waits)); a request's records
    are candidates[cand_offset : cand_offset + n_copied]."""
    tms = [as_templates(r[2]) for r in requests]  # kept alive through the call
    req = np.zeros(len(requests), dtype=SERVE_REQUEST_DTYPE)
    for i, (r, a) in enumerate(zip(requests, tms)):
        req[i] = (float(r[0]), int(r[1]), len(a), a.ctypes.data if a.size else 0, int(r[3]), 0)
    res = np.zeros(len(requests), dtype=SERVE_RESULT_DTYPE)
    out = np.zeros(int(capacity), dtype=CANDIDATE_DTYPE)
    stats = np.zeros(2, dtype=np.uint32)
    _check(_L.tb_serve(C.c_void_p(plan), _ptr(req), req.size, float(time_scale),
                       TB_SERVE_SATURATE if saturate else 0, _ptr(out) if out.size else None, out.size,
                       _ptr(res), _ptr(stats)), "tb_serve")
    used = int((res["cand_offset"] + res["n_copied"]).max()) if res.size else 0
    return res, out[:used], (int(stats[0]), int(stats[1]))


def tb_poll(plan: int, request_id: int) -> bool:
    st = _L.tb_poll(C.c_void_p(plan), int(request_id))
    if st == TB_ERR_NOT_READY:
        return False
    _check(st, "tb_poll")
    return True


def tb_get_candidates(plan: int, request_id: int, blocking: bool = True, allow_overflow: bool = False,
                      ring_capacity: int | None = None):
    """Returns (candidates structured array, n_total); None if not ready and
    not blocking.  On overflow (allow_overflow) only the ring_capacity records
    kept are returned."""
    n = C.c_uint64(0)
    st = _L.tb_get_candidates(C.c_void_p(plan), int(request_id), None, 0, C.byref(n), int(bool(blocking)))
    if st == TB_ERR_NOT_READY and not blocking:
        return None
    if st not in (TB_OK, TB_ERR_OVERFLOW):
        _check(st, "tb_get_candidates")
    out = np.zeros(int(n.value), dtype=CANDIDATE_DTYPE)
    st = _L.tb_get_candidates(C.c_void_p(plan), int(request_id), _ptr(out), out.size, C.byref(n), 1)
    if st == TB_ERR_OVERFLOW and allow_overflow:
        keep = out.size if ring_capacity is None else min(out.size, int(ring_capacity))
        return out[:keep], int(n.value)
    _check(st, "tb_get_candidates")
    return out, int(n.value)


def tb_release(plan: int, request_id: int) -> None:
    _check(_L.tb_release(C.c_void_p(plan), int(request_id)), "tb_release")


def tb_synchronize(plan: int) -> None:
    _check(_L.tb_synchronize(C.c_void_p(plan)), "tb_synchronize")


def tb_thresholds(plan: int) -> np.ndarray:
    out = np.zeros(5, dtype=np.float32)
    _check(_L.tb_thresholds(C.c_void_p(plan), _ptr(out)), "tb_thresholds")
    return out


def tb_last_request_ms(plan: int, request_id: int) -> float:
    ms = C.c_double(0.0)
    _check(_L.tb_last_request_ms(C.c_void_p(plan), int(request_id), C.byref(ms)), "tb_last_request_ms")
    return ms.value


def tb_profile(plan: int, every: int) -> None:
    """Time every `every`-th wave (True = 1, False/0 = off)."""
    _check(_L.tb_profile(C.c_void_p(plan), int(every)), "tb_profile")


def tb_profile_read(plan: int):
    """(ms[6], launches[6], templates): delay polynomials, pass 1, pass 2, medians,
    whitening, harmonic sum."""
    ms = np.zeros(6, dtype=np.float64)
    ln = np.zeros(6, dtype=np.uint64)
    t = C.c_uint64(0)
    _check(_L.tb_profile_read(C.c_void_p(plan), _ptr(ms), _ptr(ln), C.byref(t)), "tb_profile_read")
    return ms, ln, int(t.value)


def tb_bank_density(plan: int, kind: int, tobs_s: float, fmax_hz: float, points, nodes: int = 128):
    """Proper-volume density of the random template bank at the points
    (TEMPLATE_DTYPE array): (densities, kernel milliseconds)."""
    pts = np.ascontiguousarray(points, dtype=TEMPLATE_DTYPE)
    out = np.zeros(max(1, pts.size), dtype=np.float64)
    ms = C.c_double(0.0)
    m = TbBankMetric(int(kind), int(nodes), float(tobs_s), float(fmax_hz))
    _check(_L.tb_bank_density(C.c_void_p(plan), C.byref(m), _ptr(pts), pts.size, _ptr(out), C.byref(ms)),
           "tb_bank_density")
    return out[: pts.size], ms.value


def tb_bank_propose(plan: int, kind: int, tobs_s: float, fmax_hz: float, priors: TbBankPriors, u,
                    nodes: int = 128):
    """Maps uniform draws u (count x 3 circular, x 5 elliptical) to prior points:
    (points, weights density/pdf, (volume, standard error, largest weight), kernel ms)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    count = u.shape[0]
    pts = np.zeros(count, dtype=TEMPLATE_DTYPE)
    w = np.zeros(count, dtype=np.float64)
    st = np.zeros(3, dtype=np.float64)
    ms = C.c_double(0.0)
    m = TbBankMetric(int(kind), int(nodes), float(tobs_s), float(fmax_hz))
    _check(_L.tb_bank_propose(None if plan is None else C.c_void_p(plan), C.byref(m), C.byref(priors), _ptr(u),
                              count, _ptr(pts), _ptr(w), _ptr(st) if count > 1 else None, C.byref(ms)),
           "tb_bank_propose")
    return pts, w, (float(st[0]), float(st[1]), float(st[2])), ms.value


def tb_bank_count(volume: float, n: int, coverage: float, mismatch: float) -> float:
    out = C.c_double(0.0)
    _check(_L.tb_bank_count(float(volume), int(n), float(coverage), float(mismatch), C.byref(out)), "tb_bank_count")
    return out.value


def tb_bank_select(weights, u, wmax: float):
    """(indices kept, number kept, number of weights above wmax)."""
    w = np.ascontiguousarray(weights, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    keep = np.zeros(w.size, dtype=np.uint8)
    nk, na = C.c_uint64(0), C.c_uint64(0)
    _check(_L.tb_bank_select(_ptr(w), _ptr(u), w.size, float(wmax), _ptr(keep), C.byref(nk), C.byref(na)),
           "tb_bank_select")
    return np.flatnonzero(keep), nk.value, na.value


def tb_dedisperse(plan: int, data, fch1_mhz: float, foff_mhz: float, tsamp_s: float, dms, out=None,
                  nchan: int | None = None, nsamp: int | None = None, nbits: int = 8):
    """data: uint8 (nsamp, nchan) numpy array of 8-bit samples (or, nbits = 4,
    (nsamp, nchan / 2) packed pairs with nchan given) on the host, or a device
    address with nchan and nsamp given.  out: device address of ndm * nout
    floats, or None to only compute nout.  Returns (nout, kernel milliseconds)."""
    flags = TB_MEM_HOST
    if isinstance(data, int):
        flags = TB_MEM_DEVICE
    else:
        data = np.ascontiguousarray(data, dtype=np.uint8)
        nsamp = data.shape[0]
        if nbits == 8:
            nchan = data.shape[1]
    dm = np.ascontiguousarray(dms, dtype=np.float64)
    fb = TbFilterbank(int(nchan), int(nbits), int(nsamp), float(fch1_mhz), float(foff_mhz), float(tsamp_s))
    nout = C.c_uint64(0)
    ms = C.c_double(0.0)
    _check(_L.tb_dedisperse(C.c_void_p(plan), C.byref(fb), _ptr(data), flags, _ptr(dm), dm.size,
                            C.c_void_p(out) if out is not None else None, C.byref(nout), C.byref(ms)),
           "tb_dedisperse")
    return nout.value, ms.value


def tb_zap_series(plan: int, series_id: int, intervals) -> None:
    """intervals: (lo_hz, hi_hz) pairs whose bins are zeroed after whitening
    for every later search on the series; empty clears the list."""
    z = np.ascontiguousarray(np.asarray(intervals, dtype=np.float64).reshape(-1, 2).T)
    lo, hi = np.ascontiguousarray(z[0]), np.ascontiguousarray(z[1])
    _check(_L.tb_zap_series(C.c_void_p(plan), int(series_id), _ptr(lo), _ptr(hi), lo.size), "tb_zap_series")


def tb_distill(cands, max_ratio: int = 16, tol: int = 16, ppm: int = 0):
    """Candidate grouping on the host: (kept candidates in strength order,
    group sizes).  tol: sixteenths of a fundamental bin; ppm: parts per
    million of the target frequency."""
    c = np.ascontiguousarray(cands, dtype=CANDIDATE_DTYPE)
    out = np.zeros(max(1, c.size), dtype=CANDIDATE_DTYPE)
    grp = np.zeros(max(1, c.size), dtype=np.uint32)
    nk = C.c_uint64(0)
    _check(_L.tb_distill(_ptr(c), c.size, int(max_ratio), int(tol), int(ppm), _ptr(out), _ptr(grp), C.byref(nk)),
           "tb_distill")
    return out[: nk.value], grp[: nk.value]


def tb_stream_copy(plan: int, dst: int, src: int, nbytes: int, reps: int = 10) -> float:
    ms = C.c_double(0.0)
    _check(_L.tb_stream_copy(C.c_void_p(plan), C.c_void_p(dst), C.c_void_p(src), int(nbytes), int(reps),
                             C.byref(ms)), "tb_stream_copy")
    return ms.value


def tb_memory(plan: int):
    """(held bytes, budget bytes)."""
    h = C.c_uint64(0)
    b = C.c_uint64(0)
    _check(_L.tb_memory(C.c_void_p(plan), C.byref(h), C.byref(b)), "tb_memory")
    return int(h.value), int(b.value)


def tb_set_budget(plan: int, budget_bytes: int) -> None:
    _check(_L.tb_set_budget(C.c_void_p(plan), int(budget_bytes)), "tb_set_budget")


def tb_inspect_template(plan: int, series_id: int, template, n: int, harm_max: int = 16, whiten_window: int = 4096,
                        want=("src", "power", "medians", "sums")):
    t = TbTemplate(*[float(v) for v in template])
    nb = n // 2 + 1
    nblk = (n // 2 + whiten_window - 1) // whiten_window
    nf = int(harm_max).bit_length()
    out = dict(
        src=np.zeros(n, dtype=np.int32) if "src" in want else None,
        power=np.zeros(nb, dtype=np.float32) if "power" in want else None,
        medians=np.zeros(nblk, dtype=np.float32) if "medians" in want else None,
        sums=np.zeros((nf, nb), dtype=np.float32) if "sums" in want else None,
    )
    _check(_L.tb_inspect_template(C.c_void_p(plan), int(series_id), C.byref(t), _ptr(out["src"]),
                                  _ptr(out["power"]), _ptr(out["medians"]), _ptr(out["sums"])),
           "tb_inspect_template")
    return out


# ------------------------------------------------------------- convenience --
class Plan:
    """Owns one tb_plan_t; keyword arguments override tb_default_config()."""

    def __init__(self, **kw):
        self.cfg = tb_default_config()
        for k, v in kw.items():
            if k == "stream":
                v = C.c_void_p(int(v)) if v else None
            setattr(self.cfg, k, v)
        self.handle = tb_plan(self.cfg)
        self.series_n = {}

    def close(self):
        if self.handle:
            tb_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_series(self, data, tsamp, n=None, flags=TB_MEM_HOST) -> int:
        sid = tb_load_series(self.handle, data, tsamp, n=n, flags=flags)
        self.series_n[sid] = int(n if (flags & TB_MEM_DEVICE) else np.asarray(data).size)
        return sid

    def bank_density(self, kind, tobs_s, fmax_hz, points, nodes=128):
        return tb_bank_density(self.handle, kind, tobs_s, fmax_hz, points, nodes)

    def bank_propose(self, kind, tobs_s, fmax_hz, priors, u, nodes=128):
        return tb_bank_propose(self.handle, kind, tobs_s, fmax_hz, priors, u, nodes)

    def dedisperse(self, data, fch1_mhz, foff_mhz, tsamp_s, dms, out=None, nchan=None, nsamp=None, nbits=8):
        return tb_dedisperse(self.handle, data, fch1_mhz, foff_mhz, tsamp_s, dms, out, nchan, nsamp, nbits)

    def set_shape(self, log2n, tile_points=0, batch_templates=0):
        """Launch shape for series of 2^log2n samples (before that length is used)."""
        _check(_L.tb_set_shape(C.c_void_p(self.handle), int(log2n), int(tile_points), int(batch_templates)),
               "tb_set_shape")

    def zap(self, sid, intervals):
        """Birdie intervals (lo_hz, hi_hz) for the series; [] clears them."""
        tb_zap_series(self.handle, sid, intervals)

    def unload_series(self, sid):
        tb_unload_series(self.handle, sid)
        self.series_n.pop(sid, None)

    def submit(self, sid, templates, first_template_id=0) -> int:
        return tb_search_templates(self.handle, sid, templates, first_template_id)

    def poll(self, rid) -> bool:
        return tb_poll(self.handle, rid)

    def candidates(self, rid, blocking=True, allow_overflow=False):
        return tb_get_candidates(self.handle, rid, blocking, allow_overflow, self.cfg.ring_capacity)

    def release(self, rid):
        tb_release(self.handle, rid)

    def serve(self, requests, time_scale=1.0, saturate=False, capacity=1 << 20):
        return tb_serve(self.handle, requests, time_scale, saturate, capacity)

    def search(self, sid, templates, first_template_id=0):
        """Submit, wait, fetch and release: the sorted candidate array."""
        rid = self.submit(sid, templates, first_template_id)
        try:
            cands, _ = self.candidates(rid)
        finally:
            self.release(rid)
        return cands

    def search_noalloc(self, sid, templates, first_template_id=0, capacity=1 << 16, allow_overflow=False):
        """The allocation-free search: (sorted candidates, n_total)."""
        return tb_search_templates_noalloc(self.handle, sid, templates, first_template_id, capacity,
                                           allow_overflow)

    def inspect(self, sid, template, want=("src", "power", "medians", "sums")):
        return tb_inspect_template(self.handle, sid, template, self.series_n[sid], self.cfg.harm_max,
                                   self.cfg.whiten_window, want)

    def thresholds(self):
        return tb_thresholds(self.handle)

    def synchronize(self):
        tb_synchronize(self.handle)

    def request_ms(self, rid) -> float:
        return tb_last_request_ms(self.handle, rid)

    def memory(self):
        return tb_memory(self.handle)

    def set_budget(self, budget_bytes):
        tb_set_budget(self.handle, budget_bytes)

    def profile(self, every=1):
        """Time every `every`-th wave (0 stops)."""
        tb_profile(self.handle, int(every))

    def profile_read(self):
        return tb_profile_read(self.handle)
