"""CPU oracle for the per-template coherent orbital search (arXiv:2112.11991).

TEST INFRASTRUCTURE ONLY.  Thin ctypes marshalling over ``tbo.c``, a plain
double-precision C restatement of the method (see ``tbo.h`` for the passage
each step follows).  Only the tests, the smoke check and the benchmark's CPU
baseline may import this package; the product library never does, and the
two share no code.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tbo.c")
_LIB_PATH = os.path.join(_HERE, "libtbo.so")


def build(force: bool = False) -> str:
    """Compile tbo.c into libtbo.so next to it (gcc, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "tbo.h"))
    ):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm", "-lpthread"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Template(C.Structure):
    _fields_ = [
        ("porb_s", C.c_double),
        ("tau_lts", C.c_double),
        ("alpha_rad", C.c_double),
        ("ecc", C.c_double),
        ("omega_rad", C.c_double),
    ]


class Config(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("tsamp", C.c_double),
        ("harm_max", C.c_int32),
        ("whiten_window", C.c_int64),
        ("threshold_sigma", C.c_double),
        ("fmin_hz", C.c_double),
        ("fmax_hz", C.c_double),
        ("series_whitening", C.c_int32),
        ("delay_model", C.c_int32),
        ("nzap", C.c_int32),
        ("zap_lo_hz", C.c_void_p),
        ("zap_hi_hz", C.c_void_p),
    ]


class Candidate(C.Structure):
    _fields_ = [
        ("series_id", C.c_uint32),
        ("template_id", C.c_uint32),
        ("bin", C.c_uint32),
        ("log2_harm", C.c_int32),
        ("power", C.c_double),
        ("sigma", C.c_double),
        ("freq_hz", C.c_double),
    ]


CANDIDATE_DTYPE = np.dtype(
    [
        ("series_id", "<u4"),
        ("template_id", "<u4"),
        ("bin", "<u4"),
        ("log2_harm", "<i4"),
        ("power", "<f8"),
        ("sigma", "<f8"),
        ("freq_hz", "<f8"),
    ]
)
assert CANDIDATE_DTYPE.itemsize == C.sizeof(Candidate)

TEMPLATE_DTYPE = np.dtype(
    [("porb_s", "<f8"), ("tau_lts", "<f8"), ("alpha_rad", "<f8"), ("ecc", "<f8"), ("omega_rad", "<f8")]
)

_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = _bind(C.CDLL(build()))
    return _lib


def build_variant(source_text: str, out_dir: str) -> str:
    """Compile an edited copy of tbo.c (for planting mistakes in tests)."""
    src = os.path.join(out_dir, "tbo.c")
    with open(src, "w") as f:
        f.write(source_text)
    hdr = os.path.join(out_dir, "tbo.h")
    with open(os.path.join(_HERE, "tbo.h")) as a, open(hdr, "w") as b:
        b.write(a.read())
    so = os.path.join(out_dir, "libtbo_variant.so")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-w", "-o", so, src, "-lm", "-lpthread"])
    return so


class use_library:
    """Context manager: route every call of this module to another build."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = _bind(C.CDLL(self.path))
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


def _bind(L):
    P = C.POINTER
    L.tbo_mean_subtract.argtypes = [C.c_void_p, C.c_int64, C.c_void_p]
    L.tbo_kepler.argtypes = [C.c_double, C.c_double, P(C.c_int32)]
    L.tbo_kepler.restype = C.c_double
    L.tbo_roemer_delay.argtypes = [P(Template), C.c_double]
    L.tbo_roemer_delay.restype = C.c_double
    L.tbo_resample_index.argtypes = [P(Template), C.c_int64, C.c_double, C.c_void_p, C.c_void_p]
    L.tbo_roemer_delay_series.argtypes = [P(Template), C.c_double]
    L.tbo_roemer_delay_series.restype = C.c_double
    L.tbo_resample_index_model.argtypes = [P(Template), C.c_int64, C.c_double, C.c_int32, C.c_void_p, C.c_void_p]
    L.tbo_resample.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
    L.tbo_dft_naive.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
    L.tbo_fft.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
    L.tbo_power.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
    L.tbo_whiten.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p]
    L.tbo_series_levels.argtypes = [C.c_void_p, P(Config), C.c_void_p, C.c_void_p]
    L.tbo_series_levels.restype = C.c_int
    L.tbo_zap.argtypes = [C.c_void_p, C.c_int64, C.c_double, C.c_void_p, C.c_void_p, C.c_int32]
    L.tbo_zap.restype = None
    L.tbo_harmsum.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]
    L.tbo_threshold.argtypes = [C.c_int32, C.c_double]
    L.tbo_threshold.restype = C.c_double
    L.tbo_log_tail.argtypes = [C.c_int32, C.c_double]
    L.tbo_log_tail.restype = C.c_double
    L.tbo_sigma.argtypes = [C.c_int32, C.c_double]
    L.tbo_sigma.restype = C.c_double
    L.tbo_template_stages.argtypes = [
        C.c_void_p, P(Config), P(Template), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p
    ]
    L.tbo_template_stages.restype = C.c_int
    L.tbo_search.argtypes = [
        C.c_void_p, P(Config), C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int32,
        C.c_void_p, C.c_int64, P(C.c_int64),
    ]
    L.tbo_search.restype = C.c_int
    L.tbo_dispersion_constant.argtypes = []
    L.tbo_dispersion_constant.restype = C.c_double
    L.tbo_dedisperse.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int64, C.c_double, C.c_double, C.c_double,
                                 C.c_void_p, C.c_int32, C.c_void_p]
    L.tbo_dedisperse.restype = C.c_int64
    L.tbo_distill.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                              P(C.c_int64)]
    L.tbo_distill.restype = C.c_int
    return L


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _tmpl(t) -> Template:
    if isinstance(t, Template):
        return t
    if isinstance(t, dict):
        return Template(t["porb_s"], t["tau_lts"], t["alpha_rad"], t.get("ecc", 0.0), t.get("omega_rad", 0.0))
    if isinstance(t, np.void):
        return Template(*(float(t[f]) for f in TEMPLATE_DTYPE.names))
    return Template(*[float(v) for v in t])


def _templates_array(templates) -> np.ndarray:
    if isinstance(templates, np.ndarray) and templates.dtype == TEMPLATE_DTYPE:
        return np.ascontiguousarray(templates)
    arr = np.zeros(len(templates), dtype=TEMPLATE_DTYPE)
    for i, t in enumerate(templates):
        tt = _tmpl(t)
        arr[i] = (tt.porb_s, tt.tau_lts, tt.alpha_rad, tt.ecc, tt.omega_rad)
    return arr


def config(n, tsamp, harm_max=16, whiten_window=4096, threshold_sigma=6.0, fmin_hz=1.0, fmax_hz=0.0,
           series_whitening=False, delay_model=0, zap=()) -> Config:
    """delay_model: 0 BT with the Newton Kepler solve, 1 the App. B series.
    zap: (lo_hz, hi_hz) intervals whose bins are zeroed after whitening."""
    c = Config(int(n), float(tsamp), int(harm_max), int(whiten_window), float(threshold_sigma),
               float(fmin_hz), float(fmax_hz), int(bool(series_whitening)), int(delay_model))
    if len(zap):
        z = np.ascontiguousarray(np.asarray(zap, dtype=np.float64).reshape(-1, 2).T)
        c._zap = z  # keeps the arrays alive with the config
        c.nzap = z.shape[1]
        c.zap_lo_hz = z[0].ctypes.data
        c.zap_hi_hz = z[1].ctypes.data
    return c


def mean_subtract(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty_like(x)
    lib().tbo_mean_subtract(_ptr(x), x.size, _ptr(out))
    return out


def kepler(M: float, e: float):
    it = C.c_int32(0)
    E = lib().tbo_kepler(float(M), float(e), C.byref(it))
    return E, it.value


def roemer_delay(t, time_s: float) -> float:
    tt = _tmpl(t)
    return lib().tbo_roemer_delay(C.byref(tt), float(time_s))


def resample_index(t, n: int, tsamp: float):
    tt = _tmpl(t)
    delta = np.empty(n, dtype=np.float64)
    src = np.empty(n, dtype=np.int64)
    lib().tbo_resample_index(C.byref(tt), int(n), float(tsamp), _ptr(delta), _ptr(src))
    return src, delta


def roemer_delay_series(t, time_s: float) -> float:
    tt = _tmpl(t)
    return lib().tbo_roemer_delay_series(C.byref(tt), float(time_s))


def resample_index_model(t, n: int, tsamp: float, model: int):
    tt = _tmpl(t)
    delta = np.empty(n)
    src = np.empty(n, dtype=np.int64)
    lib().tbo_resample_index_model(C.byref(tt), int(n), float(tsamp), int(model), _ptr(delta), _ptr(src))
    return src, delta


def resample(x0: np.ndarray, src: np.ndarray) -> np.ndarray:
    x0 = np.ascontiguousarray(x0, dtype=np.float32)
    src = np.ascontiguousarray(src, dtype=np.int64)
    y = np.empty(x0.size, dtype=np.float64)
    lib().tbo_resample(_ptr(x0), x0.size, _ptr(src), _ptr(y))
    return y


def dft_naive(y: np.ndarray):
    y = np.ascontiguousarray(y, dtype=np.float64)
    n = y.size
    re = np.empty(n // 2 + 1)
    im = np.empty(n // 2 + 1)
    lib().tbo_dft_naive(_ptr(y), n, _ptr(re), _ptr(im))
    return re + 1j * im


def fft(y: np.ndarray):
    y = np.ascontiguousarray(y, dtype=np.float64)
    n = y.size
    re = np.empty(n // 2 + 1)
    im = np.empty(n // 2 + 1)
    lib().tbo_fft(_ptr(y), n, _ptr(re), _ptr(im))
    return re + 1j * im


def power(X: np.ndarray) -> np.ndarray:
    re = np.ascontiguousarray(X.real, dtype=np.float64)
    im = np.ascontiguousarray(X.imag, dtype=np.float64)
    p = np.empty(re.size)
    lib().tbo_power(_ptr(re), _ptr(im), re.size, _ptr(p))
    return p


def whiten(p: np.ndarray, w: int):
    p = np.ascontiguousarray(p, dtype=np.float64)
    nb = p.size
    nblk = (nb - 1 + w - 1) // w
    med = np.empty(nblk)
    phat = np.empty(nb)
    lib().tbo_whiten(_ptr(p), nb, int(w), _ptr(med), _ptr(phat))
    return phat, med


def series_levels(x0: np.ndarray, cfg: Config):
    """Whitening taken once from the series' own spectrum: (medians, level
    per bin k = 0..n/2, level[0] = 0)."""
    x0 = np.ascontiguousarray(x0, dtype=np.float32)
    nb = cfg.n // 2 + 1
    nblk = (nb - 1 + cfg.whiten_window - 1) // cfg.whiten_window
    med = np.empty(nblk)
    lev = np.empty(nb)
    if lib().tbo_series_levels(_ptr(x0), C.byref(cfg), _ptr(med), _ptr(lev)) != 0:
        raise ValueError("tbo_series_levels failed")
    return med, lev


def harmsum(phat: np.ndarray, harm_max: int = 16) -> np.ndarray:
    phat = np.ascontiguousarray(phat, dtype=np.float64)
    nf = int(harm_max).bit_length()
    s = np.empty((nf, phat.size))
    lib().tbo_harmsum(_ptr(phat), phat.size, int(harm_max), _ptr(s))
    return s


def threshold(h: int, sigma: float) -> float:
    return lib().tbo_threshold(int(h), float(sigma))


def log_tail(h: int, s: float) -> float:
    return lib().tbo_log_tail(int(h), float(s))


def sigma_of(h: int, s: float) -> float:
    return lib().tbo_sigma(int(h), float(s))


def template_stages(x0: np.ndarray, cfg: Config, t):
    """Per-stage outputs of one template: dict(src, p, med, phat, s)."""
    x0 = np.ascontiguousarray(x0, dtype=np.float32)
    n = cfg.n
    nb = n // 2 + 1
    nblk = (nb - 1 + cfg.whiten_window - 1) // cfg.whiten_window
    nf = int(cfg.harm_max).bit_length()
    src = np.empty(n, dtype=np.int64)
    p = np.empty(nb)
    med = np.empty(nblk)
    phat = np.empty(nb)
    s = np.empty((nf, nb))
    tt = _tmpl(t)
    rc = lib().tbo_template_stages(_ptr(x0), C.byref(cfg), C.byref(tt), _ptr(src), _ptr(p), _ptr(med),
                                   _ptr(phat), _ptr(s))
    if rc != 0:
        raise ValueError("tbo_template_stages: bad arguments")
    return dict(src=src, p=p, med=med, phat=phat, s=s)


def search(x0: np.ndarray, cfg: Config, templates, first_template_id: int = 0, series_id: int = 0,
           nthreads: int = 0) -> np.ndarray:
    """All candidates of the given templates, sorted by (template, fold, bin)."""
    x0 = np.ascontiguousarray(x0, dtype=np.float32)
    arr = _templates_array(templates)
    if nthreads <= 0:
        nthreads = os.cpu_count() or 1
    ntot = C.c_int64(0)
    cap = 4096
    while True:
        out = np.zeros(cap, dtype=CANDIDATE_DTYPE)
        rc = lib().tbo_search(_ptr(x0), C.byref(cfg), _ptr(arr), len(arr), int(first_template_id),
                              int(series_id), int(nthreads), _ptr(out), cap, C.byref(ntot))
        if rc != 0:
            raise ValueError("tbo_search failed")
        if ntot.value <= cap:
            return out[: ntot.value]
        cap = ntot.value


def distill(cands: np.ndarray, max_ratio: int = 16, tol: int = 16, ppm: int = 0):
    """Candidate grouping: (kept candidates in strength order, group sizes).
    tol: sixteenths of a fundamental bin; ppm: parts per million of the target."""
    c = np.ascontiguousarray(cands, dtype=CANDIDATE_DTYPE)
    out = np.zeros(max(1, c.size), dtype=CANDIDATE_DTYPE)
    grp = np.zeros(max(1, c.size), dtype=np.int64)
    nk = C.c_int64(0)
    if lib().tbo_distill(_ptr(c), c.size, int(max_ratio), int(tol), int(ppm), _ptr(out), _ptr(grp),
                         C.byref(nk)) != 0:
        raise ValueError("tbo_distill: bad arguments")
    return out[: nk.value], grp[: nk.value]


def dispersion_constant() -> float:
    return lib().tbo_dispersion_constant()


def dedisperse(data: np.ndarray, fch1_mhz: float, foff_mhz: float, tsamp: float, dms, nbits: int = 8,
               nchan: int | None = None) -> np.ndarray:
    """data: uint8 (nsamp, nchan) time-major 8-bit samples, or for nbits = 4
    (nsamp, nchan / 2) bytes of packed pairs (nchan given).  Returns (ndm, nout)
    float32."""
    data = np.ascontiguousarray(data, dtype=np.uint8)
    nsamp = data.shape[0]
    if nbits == 8:
        nchan = data.shape[1]
    dm = np.ascontiguousarray(dms, dtype=np.float64)
    args = (_ptr(data), int(nbits), int(nchan), nsamp, float(fch1_mhz), float(foff_mhz), float(tsamp), _ptr(dm),
            dm.size)
    nout = lib().tbo_dedisperse(*args, None)
    if nout < 1:
        raise ValueError("tbo_dedisperse: bad arguments")
    out = np.empty((dm.size, nout), dtype=np.float32)
    lib().tbo_dedisperse(*args, _ptr(out))
    return out
