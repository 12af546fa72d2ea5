"""Random template banks (Secs. 2.3-2.7) through the library's bank calls.

The proper volume of a prior region is the Monte-Carlo mean of density /
proposal pdf over uniform proposals (tb_bank_propose, which maps the draws to
the prior region of Table 1 and takes the densities on the GPU); the number of
random templates follows from coverage and mismatch (tb_bank_count); templates
are drawn from the same proposals and kept by the rejection step
(tb_bank_select).  This module only draws the uniform numbers and orders the
calls.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import TB_BANK_CIRCULAR, TEMPLATE_DTYPE, TbBankPriors, tb_bank_count, tb_bank_select


@dataclass
class Priors:
    porb_s: tuple            # (min, max)
    m_pulsar_min: float = 1.4
    m_comp_max: float = 8.0
    ecc_max: float = 0.0     # 0: circular bank

    def c(self) -> TbBankPriors:
        return TbBankPriors(float(self.porb_s[0]), float(self.porb_s[1]), float(self.m_pulsar_min),
                            float(self.m_comp_max), float(self.ecc_max))


def uniforms(kind, rng, count):
    """The draws a proposal consumes: (count, 3) circular, (count, 5) elliptical."""
    return rng.uniform(0.0, 1.0, (count, 3 if kind == TB_BANK_CIRCULAR else 5))


def proposals(plan, kind, tobs_s, fmax_hz, pr: Priors, rng, count, nodes=128):
    """(points, weights density/pdf, (volume, standard error, largest weight))."""
    pts, w, stats, _ = plan.bank_propose(kind, tobs_s, fmax_hz, pr.c(), uniforms(kind, rng, count), nodes)
    return pts, w, stats


def template_count(volume, n, coverage, mismatch):
    return tb_bank_count(volume, n, coverage, mismatch)


def volume(plan, kind, tobs_s, fmax_hz, pr: Priors, rng, points=1 << 18, nodes=128):
    """(V, standard error, largest density / pdf seen) by Monte Carlo."""
    return proposals(plan, kind, tobs_s, fmax_hz, pr, rng, points, nodes)[2]


def generate(plan, kind, tobs_s, fmax_hz, pr: Priors, coverage, mismatch, rng, volume_points=1 << 18,
             batch=1 << 18, nodes=128, headroom=1.25):
    """A random bank: (templates, info).  The acceptance scale is the largest
    density/pdf of the volume pass times `headroom`; proposals above it are
    always kept (their count is reported)."""
    n = 3 if kind == TB_BANK_CIRCULAR else 5
    V, err, rmax = volume(plan, kind, tobs_s, fmax_hz, pr, rng, volume_points, nodes)
    count = int(np.ceil(template_count(V, n, coverage, mismatch)))
    wmax = rmax * headroom
    out, over, drawn, kept = [], 0, 0, 0
    while kept < count:
        pts, w, _ = proposals(plan, kind, tobs_s, fmax_hz, pr, rng, batch, nodes)
        sel, _, above = tb_bank_select(w, rng.uniform(0.0, 1.0, batch), wmax)
        over += above
        drawn += batch
        take = sel[: count - kept]
        out.append(pts[take])
        kept += take.size
    bank = np.concatenate(out) if out else np.zeros(0, dtype=TEMPLATE_DTYPE)
    return bank, dict(volume=V, volume_err=err, count=count, proposals=drawn, above_scale=over)
