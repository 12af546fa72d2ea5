"""Seeded synthetic inputs for the coherent orbital search.

This module only *makes inputs*: noise, red noise, binary-pulsar pulse trains,
template draws and request traces.  It holds none of the search's arithmetic
(no resampling, transform, whitening, harmonic sum or thresholding) and is the
only code that both the oracle side and the GPU side use.

Pulse trains follow the signal model of Sec. 2.1 (rotational phase
f0 (t + Delta(t)), harmonics of a narrow pulse, additive noise).  The orbital
delay of an injected pulsar is evaluated through the Bessel-function series of
cos E and sqrt(1-e^2) sin E in the mean anomaly (the expansion of Sec. 2.2 /
App. B carried to convergence), which is independent of the Newton solve the
search itself uses.

Workloads stand in for the paper's simulated and survey data (Table 2: 2^24
samples at 256 us; HTRU 64 us data, Sec. 5.2), none of which exist here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.special import jv

SEED_ROOT = (2112, 11991)
TEMPLATE_DTYPE = np.dtype(
    [("porb_s", "<f8"), ("tau_lts", "<f8"), ("alpha_rad", "<f8"), ("ecc", "<f8"), ("omega_rad", "<f8")]
)
HOUR = 3600.0


def streams(cfg: int, k: int = 6):
    """Independent generators for one configuration: noise, red noise,
    templates, injections, arrivals, spare."""
    ss = np.random.SeedSequence(list(SEED_ROOT) + [int(cfg)])
    return [np.random.default_rng(s) for s in ss.spawn(k)]


def white_noise(n: int, rng: np.random.Generator, sigma: float = 1.0) -> np.ndarray:
    return rng.standard_normal(n) * sigma


def red_noise(n: int, tsamp: float, rng: np.random.Generator, f_knee: float = 1.0) -> np.ndarray:
    """Random walk (1/f^2 spectrum) whose power equals unit white noise at
    f_knee: step sigma = 2 pi f_knee tsamp."""
    step = 2.0 * math.pi * f_knee * tsamp
    return np.cumsum(rng.standard_normal(n) * step)


def orbit_delay(t: np.ndarray, porb_s: float, tau_lts: float, alpha_rad: float,
                ecc: float = 0.0, omega_rad: float = 0.0) -> np.ndarray:
    """Orbital light-travel delay tau [sin(psi) cos E + cos(psi) sqrt(1-e^2) sin E]
    of the Doppler phase (Sec. 2.1) at times t, with cos E and sin E from their
    Bessel series in the mean anomaly M = 2 pi t / P_orb + alpha."""
    M = 2.0 * math.pi / porb_s * np.asarray(t, dtype=np.float64) + alpha_rad
    if ecc == 0.0:
        cosE = np.cos(M)
        sinE_b = np.sin(M)
    else:
        cosE = np.full_like(M, -0.5 * ecc)
        sinE_b = np.zeros_like(M)
        beta = math.sqrt(1.0 - ecc * ecc)
        for k in range(1, 200):
            ck = (jv(k - 1, k * ecc) - jv(k + 1, k * ecc)) / k
            sk = beta * 2.0 * jv(k, k * ecc) / (k * ecc)
            if abs(ck) < 1e-18 and abs(sk) < 1e-18:
                break
            cosE += ck * np.cos(k * M)
            sinE_b += sk * np.sin(k * M)
    return tau_lts * (math.sin(omega_rad) * cosE + math.cos(omega_rad) * sinE_b)


@dataclass
class Orbit:
    porb_s: float
    tau_lts: float
    alpha_rad: float
    ecc: float = 0.0
    omega_rad: float = 0.0

    def as_template(self) -> np.ndarray:
        a = np.zeros(1, dtype=TEMPLATE_DTYPE)
        a[0] = (self.porb_s, self.tau_lts, self.alpha_rad, self.ecc, self.omega_rad)
        return a


def pulse_train(n: int, tsamp: float, p_spin: float, duty: float, orbit: Orbit | None,
                chunk: int = 1 << 20) -> np.ndarray:
    """Noise-free Gaussian pulse train with FWHM duty * p_spin, rotational phase
    f0 (t + Delta(t)) (Sec. 2.1), evaluated in chunks."""
    out = np.empty(n, dtype=np.float64)
    f0 = 1.0 / p_spin
    sig = duty / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        t = np.arange(a, b, dtype=np.float64) * tsamp
        d = orbit_delay(t, orbit.porb_s, orbit.tau_lts, orbit.alpha_rad, orbit.ecc, orbit.omega_rad) \
            if orbit is not None else 0.0
        ph = f0 * (t + d)
        w = ph - np.floor(ph + 0.5)
        out[a:b] = np.exp(-0.5 * (w / sig) ** 2)
    return out


def inject(series: np.ndarray, train: np.ndarray, snr: float, noise_sigma: float = 1.0) -> np.ndarray:
    """Add the train scaled so that its matched-filter S/N sqrt(sum g^2)/sigma,
    g the mean-subtracted train, equals snr."""
    g = train - train.mean()
    amp = snr * noise_sigma / math.sqrt(float(np.dot(g, g)))
    return series + amp * g


def uniform_templates(rng: np.random.Generator, count: int, porb_h=(1.0, 10.0), tau=(0.0, 2.0),
                      ecc_max: float = 0.0) -> np.ndarray:
    """Templates drawn uniformly: P_orb [h], tau [lt-s], alpha in [0, 2 pi);
    elliptical draws add e in [0, ecc_max) and psi in [0, 2 pi)."""
    a = np.zeros(count, dtype=TEMPLATE_DTYPE)
    a["porb_s"] = rng.uniform(porb_h[0], porb_h[1], count) * HOUR
    a["tau_lts"] = rng.uniform(tau[0], tau[1], count)
    a["alpha_rad"] = rng.uniform(0.0, 2.0 * math.pi, count)
    if ecc_max > 0.0:
        a["ecc"] = rng.uniform(0.0, ecc_max, count)
        a["omega_rad"] = rng.uniform(0.0, 2.0 * math.pi, count)
    return a


@dataclass
class Workload:
    name: str
    tsamp: float
    series: list = field(default_factory=list)     # float32 arrays
    templates: np.ndarray | None = None
    truths: list = field(default_factory=list)     # (series index, Orbit, p_spin)
    whiten_window: int = 4096
    harm_max: int = 16
    sigma: float = 6.0
    fmin_hz: float = 1.0


def c1_tiny(n_templates: int = 64) -> Workload:
    """One series, 2^17 samples at 64 us: N(0,1) noise plus a 20 ms pulsar
    (5% duty, S/N 15) in a circular orbit P_orb = 2 h, tau = 0.5 lt-s,
    alpha = 1.0; 64 uniform circular templates plus the true one."""
    rn, _, rt, _, _, _ = streams(1)
    n, ts = 1 << 17, 64e-6
    orb = Orbit(2.0 * HOUR, 0.5, 1.0)
    x = inject(white_noise(n, rn), pulse_train(n, ts, 0.020, 0.05, orb), 15.0)
    tm = np.concatenate([uniform_templates(rt, n_templates, (1.5, 3.0), (0.0, 1.0)), orb.as_template()])
    return Workload("c1_circular_2^17", ts, [x.astype(np.float32)], tm, [(0, orb, 0.020)])


def c2_survey(n_templates: int = 20000, n: int = 1 << 23) -> Workload:
    """One series, 2^23 samples at 64 us (537 s): N(0,1) noise, a random-walk
    red-noise component, and a 25 ms pulsar (S/N 15) with P_orb = 1.5 h,
    tau = 1.2 lt-s, alpha = 1.0; uniform circular templates P_orb in [1, 10] h,
    tau in [0, 2] lt-s."""
    rn, rr, rt, _, _, _ = streams(2)
    ts = 64e-6
    orb = Orbit(1.5 * HOUR, 1.2, 1.0)
    x = white_noise(n, rn) + red_noise(n, ts, rr)
    x = inject(x, pulse_train(n, ts, 0.025, 0.05, orb), 15.0)
    tm = uniform_templates(rt, n_templates, (1.0, 10.0), (0.0, 2.0))
    return Workload("c2_circular_2^23", ts, [x.astype(np.float32)], tm, [(0, orb, 0.025)])


def c3_elliptical(n_templates: int = 50000, n: int = 1 << 24) -> Workload:
    """One series, 2^24 samples at 256 us (71.6 min), the shape of Table 2:
    noise plus a 30 ms pulsar (S/N 15) with e = 0.08, psi = 2.0, P_orb = 8 h,
    tau = 3 lt-s, alpha = 1.0; templates P_orb in [5, 20] h, tau in [0, 6],
    e in [0, 0.1), psi and alpha in [0, 2 pi)."""
    rn, _, rt, _, _, _ = streams(3)
    ts = 256e-6
    orb = Orbit(8.0 * HOUR, 3.0, 1.0, 0.08, 2.0)
    x = inject(white_noise(n, rn), pulse_train(n, ts, 0.030, 0.05, orb), 15.0)
    tm = uniform_templates(rt, n_templates, (5.0, 20.0), (0.0, 6.0), ecc_max=0.1)
    return Workload("c3_elliptical_2^24", ts, [x.astype(np.float32)], tm, [(0, orb, 0.030)])


def table3_series(n: int = 1 << 24) -> Workload:
    """The series of the paper's circular-search timing (Tables 2 and 3): one
    series of 2^24 samples at 256 us (71.6 min), noise plus a 30 ms pulsar (5%
    duty, S/N 15) in a circular orbit P_orb = 8 h, tau = 10 lt-s, alpha = 1.0.
    The bank (the Table 1 circular random bank) is drawn by the caller."""
    rn, _, _, _, _, _ = streams(7)
    ts = 256e-6
    orb = Orbit(8.0 * HOUR, 10.0, 1.0)
    x = inject(white_noise(n, rn), pulse_train(n, ts, 0.030, 0.05, orb), 15.0)
    return Workload("t3_circular_2^24", ts, [x.astype(np.float32)], None, [(0, orb, 0.030)])


def c4_batched(n_series: int = 32, n_templates: int = 4096, log2_lengths=(20, 21, 22, 23)) -> Workload:
    """32 series (DM trials) of lengths drawn from 2^20..2^23 at 64 us, 4 of
    them with circular binaries (P_spin 20-40 ms, S/N 15); 4096 shared circular
    templates with the wide prior."""
    rn, rr, rt, ri, _, _ = streams(4)
    ts = 64e-6
    lens = [1 << int(v) for v in ri.choice(log2_lengths, n_series)]
    carriers = set(ri.choice(n_series, 4, replace=False).tolist())
    w = Workload("c4_batched", ts)
    for i, n in enumerate(lens):
        x = white_noise(n, rn)
        if i in carriers:
            orb = Orbit(ri.uniform(1.0, 10.0) * HOUR, ri.uniform(0.0, 2.0), ri.uniform(0.0, 2 * math.pi))
            ps = ri.uniform(0.020, 0.040)
            x = inject(x, pulse_train(n, ts, ps, 0.05, orb), 15.0)
            w.truths.append((i, orb, ps))
        w.series.append(x.astype(np.float32))
    w.templates = uniform_templates(rt, n_templates, (1.0, 10.0), (0.0, 2.0))
    return w


def request_trace(n_requests: int = 400, rate_hz: float = 50.0, pool: int = 16,
                  log2_lengths=(20, 21, 22, 23, 24), seed_cfg: int = 5):
    """Served stream: Poisson arrivals; each request picks one of a pool of
    series uniformly and carries 256-4096 templates, elliptical (C3 prior) with
    probability 0.3, else circular (wide C2 prior)."""
    rn, _, rt, ri, ra, _ = streams(seed_cfg)
    lens = [1 << int(v) for v in ri.choice(log2_lengths, pool)]
    arrivals = np.cumsum(ra.exponential(1.0 / rate_hz, n_requests))
    reqs = []
    for i in range(n_requests):
        sid = int(ri.integers(0, pool))
        cnt = int(ri.integers(256, 4097))
        if ri.uniform() < 0.3:
            tm = uniform_templates(rt, cnt, (5.0, 20.0), (0.0, 6.0), ecc_max=0.1)
        else:
            tm = uniform_templates(rt, cnt, (1.0, 10.0), (0.0, 2.0))
        reqs.append(dict(t_arrival=float(arrivals[i]), series=sid, templates=tm))
    return lens, reqs


def pool_series(lens, seed_cfg: int = 5):
    rn = streams(seed_cfg)[0]
    return [white_noise(n, rn).astype(np.float32) for n in lens]
