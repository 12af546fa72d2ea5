"""Random template banks (Secs. 2.3-2.7) on the GPU density kernel.

The proper volume of a prior region is estimated by Monte Carlo from the
kernel's densities at uniform draws over the region; the number of random
templates follows from coverage and mismatch; templates are then drawn from
the same uniform proposals and kept with probability proportional to
density / proposal pdf.  Prior region (Table 1): P_orb uniform in a range,
tau uniform below the Kepler limit for the given pulsar and companion masses,
alpha (and psi) uniform in [0, 2 pi), e uniform below e_max.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import TEMPLATE_DTYPE, TB_BANK_CIRCULAR, TB_BANK_ELLIPTICAL

GM_SUN_OVER_C3 = 4.925490947e-6  # s


def kepler_tau_limit(porb_s, m_pulsar_min, m_comp_max, theta=1.0):
    """Largest tau = a_p sin(i)/c [lt-s] at P_orb for a pulsar of at least
    m_pulsar_min and a companion of at most m_comp_max solar masses."""
    omega = 2.0 * math.pi / np.asarray(porb_s, dtype=np.float64)
    return theta * GM_SUN_OVER_C3 ** (1.0 / 3.0) * omega ** (-2.0 / 3.0) * m_comp_max \
        / (m_pulsar_min + m_comp_max) ** (2.0 / 3.0)


@dataclass
class Priors:
    porb_s: tuple            # (min, max)
    m_pulsar_min: float = 1.4
    m_comp_max: float = 8.0
    ecc_max: float = 0.0     # 0: circular bank


def _draw(kind, pr: Priors, rng, count):
    """Uniform proposals over the prior region and their pdf."""
    a = np.zeros(count, dtype=TEMPLATE_DTYPE)
    a["porb_s"] = rng.uniform(pr.porb_s[0], pr.porb_s[1], count)
    lim = kepler_tau_limit(a["porb_s"], pr.m_pulsar_min, pr.m_comp_max)
    a["tau_lts"] = rng.uniform(0.0, 1.0, count) * lim
    a["alpha_rad"] = rng.uniform(0.0, 2.0 * math.pi, count)
    pdf = 1.0 / ((pr.porb_s[1] - pr.porb_s[0]) * lim * 2.0 * math.pi)
    if kind == TB_BANK_ELLIPTICAL:
        a["ecc"] = rng.uniform(0.0, pr.ecc_max, count)
        a["omega_rad"] = rng.uniform(0.0, 2.0 * math.pi, count)
        pdf = pdf / (pr.ecc_max * 2.0 * math.pi)
    return a, pdf


def template_count(volume, n, coverage, mismatch):
    """ln(1 - eta) / ln(1 - m^(n/2) C_n / V)."""
    cn = math.pi ** (n / 2.0) / math.gamma(n / 2.0 + 1.0)
    x = mismatch ** (n / 2.0) * cn / volume
    return math.log(1.0 - coverage) / math.log1p(-x)


def volume(plan, kind, tobs_s, fmax_hz, pr: Priors, rng, points=1 << 18, nodes=128):
    """(V, standard error, largest density / pdf seen) by Monte Carlo."""
    pts, pdf = _draw(kind, pr, rng, points)
    dens, _ = plan.bank_density(kind, tobs_s, fmax_hz, pts, nodes)
    r = dens / pdf
    return float(r.mean()), float(r.std(ddof=1) / math.sqrt(r.size)), float(r.max())


def generate(plan, kind, tobs_s, fmax_hz, pr: Priors, coverage, mismatch, rng, volume_points=1 << 18,
             batch=1 << 18, nodes=128, headroom=1.25):
    """A random bank: (templates, info).  The acceptance scale is the largest
    density/pdf of the volume pass times `headroom`; proposals above it are
    always kept (their count is reported)."""
    n = 3 if kind == TB_BANK_CIRCULAR else 5
    V, err, rmax = volume(plan, kind, tobs_s, fmax_hz, pr, rng, volume_points, nodes)
    count = int(math.ceil(template_count(V, n, coverage, mismatch)))
    wmax = rmax * headroom
    out, over, drawn = [], 0, 0
    kept = 0
    while kept < count:
        pts, pdf = _draw(kind, pr, rng, batch)
        dens, _ = plan.bank_density(kind, tobs_s, fmax_hz, pts, nodes)
        w = dens / pdf
        u = rng.uniform(0.0, 1.0, batch)
        sel = np.flatnonzero(u * wmax < w)
        over += int(np.count_nonzero(w > wmax))
        drawn += batch
        take = sel[: count - kept]
        out.append(pts[take])
        kept += take.size
    bank = np.concatenate(out) if out else np.zeros(0, dtype=TEMPLATE_DTYPE)
    return bank, dict(volume=V, volume_err=err, count=count, proposals=drawn, above_scale=over)
