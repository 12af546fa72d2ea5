"""Request streams through the library's continuous-batching loop (tb_serve).

Requests (a resident series plus a chunk of templates) arrive over time.  The
library admits each one as soon as it has arrived and the plan's HBM budget
allows, spreads admitted requests over the plan's lanes so that their kernels
overlap on the device, and collects each request's candidates the moment its
device work has finished.  Per-request latency is arrival -> candidates
retrievable.

This module only builds the request records and reads back the per-request
results; the loop itself runs in the library.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import TB_ERR_OVERFLOW, Plan


@dataclass
class Request:
    t_arrival: float          # seconds after the start of the trace
    series: int               # index into the loop's series list
    templates: np.ndarray     # TEMPLATE_DTYPE records
    first_template_id: int = 0
    # filled by the loop
    t_admit: float | None = None
    t_done: float | None = None
    candidates: np.ndarray | None = None
    n_total: int = 0
    overflow: bool = False


@dataclass
class ServeReport:
    n_requests: int
    templates: int
    samples_x_templates: float
    makespan_s: float
    latencies_s: np.ndarray = field(repr=False)
    max_in_flight: int = 0
    budget_waits: int = 0

    @property
    def p50_ms(self) -> float:
        return float(np.percentile(self.latencies_s, 50) * 1e3)

    @property
    def p99_ms(self) -> float:
        return float(np.percentile(self.latencies_s, 99) * 1e3)

    @property
    def templates_per_s(self) -> float:
        return self.templates / self.makespan_s

    def as_dict(self) -> dict:
        return {"requests": self.n_requests, "templates": self.templates, "makespan_s": self.makespan_s,
                "templates_per_s": self.templates_per_s, "p50_ms": self.p50_ms, "p99_ms": self.p99_ms,
                "max_in_flight": self.max_in_flight, "budget_waits": self.budget_waits}


def serve(plan: Plan, series_ids: list[int], series_len: list[int], requests: list[Request],
          realtime: bool = True, time_scale: float = 1.0, capacity: int = 1 << 20) -> ServeReport:
    """Runs the trace to completion.  With realtime=False every request is
    taken as arrived at t = 0 (a saturation run).  time_scale stretches the
    arrival times (2.0 = half the arrival rate).  capacity: candidate records
    kept over the whole trace."""
    res, cands, (max_in_flight, budget_waits) = plan.serve(
        [(r.t_arrival, series_ids[r.series], r.templates, r.first_template_id) for r in requests],
        time_scale=time_scale, saturate=not realtime, capacity=capacity)
    for r, o in zip(requests, res):
        r.t_admit, r.t_done = float(o["t_admit_s"]), float(o["t_done_s"])
        r.candidates = cands[int(o["cand_offset"]):int(o["cand_offset"] + o["n_copied"])]
        r.n_total, r.overflow = int(o["n_total"]), int(o["status"]) == TB_ERR_OVERFLOW
    arrival = np.array([r.t_arrival * time_scale if realtime else 0.0 for r in requests])
    done = res["t_done_s"]
    makespan = float(done.max() - arrival.min())
    ntemp = int(sum(len(r.templates) for r in requests))
    work = float(sum(len(r.templates) * series_len[r.series] for r in requests))
    return ServeReport(len(requests), ntemp, work, makespan, done - arrival, max_in_flight, budget_waits)
