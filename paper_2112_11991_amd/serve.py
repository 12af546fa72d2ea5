"""Continuous-batching request loop over the C ABI.

Requests (a resident series plus a chunk of templates) arrive over time.  The
loop admits each one as soon as it has arrived and the plan's HBM budget
allows (tb_search_templates returns TB_ERR_BUDGET otherwise and the request
waits for completions to free memory), spreads admitted requests over the
plan's lanes so that their kernels overlap on the device, and collects each
request's candidates the moment its device work has finished.  Per-request
latency is arrival -> candidates retrievable.

Nothing here computes any part of the search: it only orders calls to the
library.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import TB_ERR_BUDGET, Plan, TbError


@dataclass
class Request:
    t_arrival: float          # seconds after the start of the trace
    series: int               # index into the loop's series list
    templates: np.ndarray     # TEMPLATE_DTYPE records
    first_template_id: int = 0
    # filled by the loop
    rid: int | None = None
    t_admit: float | None = None
    t_done: float | None = None
    candidates: np.ndarray | None = None
    n_total: int = 0


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
          realtime: bool = True, poll_s: float = 2e-4, time_scale: float = 1.0) -> ServeReport:
    """Runs the trace to completion.  With realtime=False every request is
    taken as arrived at t = 0 (a saturation run).  time_scale stretches the
    arrival times (2.0 = half the arrival rate)."""
    pending = sorted(requests, key=lambda r: r.t_arrival)
    waiting: list[Request] = []
    running: list[Request] = []
    done: list[Request] = []
    t0 = time.perf_counter()
    max_in_flight = 0
    budget_waits = 0
    i = 0
    while i < len(pending) or waiting or running:
        now = time.perf_counter() - t0
        while i < len(pending) and (not realtime or pending[i].t_arrival * time_scale <= now):
            waiting.append(pending[i])
            i += 1
        # admit in arrival order while memory allows
        while waiting:
            r = waiting[0]
            try:
                r.rid = plan.submit(series_ids[r.series], r.templates, r.first_template_id)
            except TbError as e:
                if e.status != TB_ERR_BUDGET or not running:
                    raise
                budget_waits += 1
                break
            r.t_admit = time.perf_counter() - t0
            running.append(waiting.pop(0))
        max_in_flight = max(max_in_flight, len(running))
        progressed = False
        still = []
        for r in running:
            if plan.poll(r.rid):
                r.t_done = time.perf_counter() - t0
                r.candidates, r.n_total = plan.candidates(r.rid, blocking=True, allow_overflow=True)
                plan.release(r.rid)
                done.append(r)
                progressed = True
            else:
                still.append(r)
        running = still
        if not progressed and running:
            time.sleep(poll_s)
        elif not running and not waiting and i < len(pending) and realtime:
            time.sleep(max(0.0, min(poll_s * 10, pending[i].t_arrival * time_scale - (time.perf_counter() - t0))))
    makespan = max(r.t_done for r in done) - (min(r.t_arrival for r in done) * time_scale if realtime else 0.0)
    lat = np.array([r.t_done - (r.t_arrival * time_scale if realtime else 0.0) for r in done])
    ntemp = int(sum(len(r.templates) for r in done))
    work = float(sum(len(r.templates) * series_len[r.series] for r in done))
    return ServeReport(len(done), ntemp, work, makespan, lat, max_in_flight, budget_waits)
