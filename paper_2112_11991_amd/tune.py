"""Autotuner for the launch shape of each series length: FFT points per
workgroup (8192 or 16384) and templates per wave, chosen by timing the search
itself on the device.

For each length it loads one seeded noise series into a fresh plan per
candidate shape, searches a fixed bank once to warm up, then times `reps`
searches of it and keeps the shape with the highest templates/s.  The result
is applied to a plan with Plan.set_shape before that length is used.
"""
from __future__ import annotations

import json
import math
import time

import numpy as np

from . import TEMPLATE_DTYPE, Plan


def _bank(count, rng):
    a = np.zeros(count, dtype=TEMPLATE_DTYPE)
    a["porb_s"] = rng.uniform(1.0, 10.0, count) * 3600.0
    a["tau_lts"] = rng.uniform(0.0, 2.0, count)
    a["alpha_rad"] = rng.uniform(0.0, 2.0 * math.pi, count)
    return a


def autotune(log2ns, tsamp=64e-6, tiles=(8192, 16384), batches=(4, 8, 16, 32, 64), reps=2, work=1 << 30,
             plan_kw=None, seed=2112, log=None):
    """{log2n: {"tile_points", "batch_templates", "templates_per_s", "tried": [...]}}.
    Each timing searches about `work` samples in total (templates x n)."""
    rng = np.random.default_rng(seed)
    out = {}
    for lg in log2ns:
        n = 1 << lg
        x = rng.standard_normal(n).astype(np.float32)
        count = max(64, int(work // n))
        bank = _bank(count, rng)
        tried = []
        for tile in tiles:
            for b in batches:
                if b > count:
                    continue
                with Plan(**(plan_kw or {})) as plan:
                    plan.set_shape(lg, tile, b)
                    sid = plan.load_series(x, tsamp)
                    plan.search(sid, bank[:b])
                    t0 = time.perf_counter()
                    for _ in range(reps):
                        plan.search(sid, bank)
                    rate = reps * count / (time.perf_counter() - t0)
                tried.append({"tile_points": tile, "batch_templates": b, "templates_per_s": rate})
                if log:
                    log("tune 2^%d tile %d batch %d: %.0f templates/s" % (lg, tile, b, rate))
        best = max(tried, key=lambda r: r["templates_per_s"])
        out[lg] = dict(best, tried=tried)
    return out


def apply(plan, tuned):
    """Sets every tuned length's shape on a plan that has not used it yet."""
    for lg, r in tuned.items():
        plan.set_shape(int(lg), r["tile_points"], r["batch_templates"])


def save(tuned, path):
    with open(path, "w") as f:
        json.dump({str(k): v for k, v in tuned.items()}, f, indent=1)


def load(path):
    with open(path) as f:
        return {int(k): v for k, v in json.load(f).items()}
