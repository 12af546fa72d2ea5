"""Comparison rules between the HIP path and the oracle.

- Resampling indices: equal, except where the oracle's delay sits within 1e-9
  samples of a rounding tie (|frac(delta) - 1/2| < 1e-9); those are exempt and
  counted.
- Whitened powers: |P^_gpu - P^_oracle| <= 1e-4 max(P^_oracle, 1) (relative,
  floored at the noise level, which whitening puts at 1).
- Fold sums: |S_gpu - S_oracle| <= 1e-4 (S_oracle + h), the bound the power
  rule gives for a sum of h of them.
- Raw powers: relative 1e-4 with the floor at the local noise level
  (block median / ln 2).
- Candidates: the same (template, fold, bin) sets except records whose power
  lies within 1e-4 of the fold threshold; matched records agree under the fold
  rule.
"""
import math

import numpy as np

TIE = 1e-9
REL = 1e-4


def tie_exempt(delta: np.ndarray) -> np.ndarray:
    fr = delta - np.floor(delta)
    return np.abs(fr - 0.5) < TIE


def check_indices(src_gpu: np.ndarray, src_or: np.ndarray, delta_or: np.ndarray) -> int:
    ex = tie_exempt(delta_or)
    bad = (src_gpu.astype(np.int64) != src_or) & ~ex
    assert not bad.any(), "index mismatch at %s" % np.flatnonzero(bad)[:10]
    return int(ex.sum())


def check_power(p_gpu, p_or, med_or, w):
    m = p_or.size - 1
    b = np.minimum((np.arange(p_or.size) - 1).clip(0) // w, med_or.size - 1)
    floor = med_or[b] / math.log(2.0)
    err = np.abs(p_gpu.astype(np.float64) - p_or)
    lim = REL * np.maximum(p_or, floor)
    assert np.all(err <= lim), "power off by %.3g x limit at bin %d" % (
        float(np.max(err / lim)), int(np.argmax(err / lim)))
    assert m >= 1


def check_medians(med_gpu, med_or):
    err = np.abs(med_gpu.astype(np.float64) - med_or)
    assert np.all(err <= REL * med_or), "median off: max rel %.3g" % float(np.max(err / med_or))


def check_phat(phat_gpu, phat_or):
    err = np.abs(phat_gpu.astype(np.float64) - phat_or)
    lim = REL * np.maximum(phat_or, 1.0)
    assert np.all(err <= lim), "whitened power off by %.3g x limit at bin %d" % (
        float(np.max(err / lim)), int(np.argmax(err / lim)))


def check_sums(s_gpu, s_or):
    for l in range(s_or.shape[0]):
        h = 1 << l
        err = np.abs(s_gpu[l].astype(np.float64) - s_or[l])
        lim = REL * (s_or[l] + h)
        assert np.all(err <= lim), "fold %d off by %.3g x limit at bin %d" % (
            h, float(np.max(err / lim)), int(np.argmax(err / lim)))


def check_candidates(c_gpu, c_or, thr):
    """thr: per-fold thresholds (index log2 h).  Returns (#matched, #exempt)."""
    key = lambda c: (int(c["template_id"]), int(c["log2_harm"]), int(c["bin"]))
    G = {key(c): c for c in c_gpu}
    O = {key(c): c for c in c_or}
    assert len(G) == len(c_gpu) and len(O) == len(c_or), "duplicate records"
    exempt = 0
    for k in set(G) ^ set(O):
        c = G.get(k) if k in G else O[k]
        t = thr[k[1]]
        assert abs(float(c["power"]) - t) <= REL * t, "candidate %s only on one side (S=%.6g thr=%.6g)" % (
            k, float(c["power"]), t)
        exempt += 1
    for k in set(G) & set(O):
        h = 1 << k[1]
        sg, so = float(G[k]["power"]), float(O[k]["power"])
        assert abs(sg - so) <= REL * (so + h), "candidate %s power %.7g vs %.7g" % (k, sg, so)
        assert abs(float(G[k]["sigma"]) - float(O[k]["sigma"])) <= 1e-3 * max(1.0, float(O[k]["sigma"])) + \
            abs(sg - so), "candidate %s sigma" % (k,)
        assert G[k]["series_id"] == O[k]["series_id"]
        assert abs(float(G[k]["freq_hz"]) - float(O[k]["freq_hz"])) <= 1e-12 * float(O[k]["freq_hz"]) + 1e-15
    return len(set(G) & set(O)), exempt
