"""Benchmark of the template-bank coherent orbital search on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload c2|c1|c3|c4|c5|t3]

One step is one pass of the whole search (resample, FFT, power, whitening,
harmonic sum, peaks) over the workload's template bank, with the series
already resident in HBM.  The default workload is the circular survey-scale
search: one 2^23-sample series at 64 us with red noise and a pulsar, 20,000
uniform circular templates.  c4 is the batched uneven-length search (32
series x 4096 templates, one step = all series), c5 the served request stream
(p50/p99 latency beside throughput), t3 the paper's own circular-search timing
(one 2^24-sample series at 256 us, the Table 1 random bank drawn by the
library; its line carries vs_baseline against the paper's Table 3 time).
Prints one JSON line on stdout;
progress goes to stderr.  Only one GPU is used: --gpus above 1 exits with a
message.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (a wave64 instruction
# takes four cycles of a 16-lane SIMD; packed FP32 is not used)
PEAK_VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9
KERNELS = ["k_chunk_polys (per-template delay polynomials)", "k_fft1 (resample + FFT pass 1)",
           "k_fft2 (FFT pass 2 + R2C + power)", "k_median_whiten (block medians + whitening)", "(unused class)",
           "k_harmsum (harmonic sum + peaks)"]
KERNEL_SHORT = ["k_chunk_polys", "k_fft1", "k_fft2", "k_median_whiten", "-", "k_harmsum"]
PROFILE_EVERY = 16  # time one wave in this many inside the timed region
METRIC = "templates/s (resample+FFT+harmsum+peaks) at N=2^23 FP32"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name: str, templates: int | None):
    import synth

    if name == "c1":
        return synth.c1_tiny() if templates is None else synth.c1_tiny(templates - 1)
    if name == "c2":
        return synth.c2_survey(templates or 20000)
    if name == "c3":
        return synth.c3_elliptical(templates or 50000)
    if name == "c4":
        return synth.c4_batched(n_templates=templates or 4096)
    if name == "t3":
        return synth.table3_series()
    raise SystemExit("unknown workload " + name)


def table1_bank(tb, w, templates=None):
    """The Table 1 circular random bank (72-minute observation, P_orb 6-12 h,
    pulsar mass >= 1.4, companion <= 8 solar masses, f_max 66.67 Hz, 90 %
    coverage at mismatch 0.2), drawn by the library's bank calls: about
    10,100 templates, the paper's 10,128 within the Monte-Carlo error.  The
    2^24-sample series at 256 us lasts 71.6 minutes."""
    from paper_2112_11991_amd import bank

    pr = bank.Priors(porb_s=(6 * 3600.0, 12 * 3600.0), m_pulsar_min=1.4, m_comp_max=8.0)
    with tb.Plan() as plan:
        tm, info = bank.generate(plan, tb.TB_BANK_CIRCULAR, 72.0 * 60.0, 66.67, pr, 0.9, 0.2,
                                 np.random.default_rng(2112))
    return tm[:templates] if templates else tm, info


def default_tile(n: int) -> int:
    """FFT points per workgroup when the plan chooses (mirrors the library)."""
    return 16384 if n // 2 >= (1 << 23) else 8192


def describe(w, name):
    n = [int(s.size) for s in w.series]
    if name == "c4":
        return {"workload": "batched uneven-length search: %d series of 2^20..2^23 samples at 64 us, %d shared circular "
                            "templates each, 16 harmonics, 6 sigma" % (len(n), len(w.templates)),
                "series": len(n), "samples_total": int(sum(n)), "templates": int(len(w.templates))}
    kind = "elliptical" if w.templates["ecc"].max() > 0 else "circular"
    drawn = "Table 1 random-bank" if name == "t3" else "uniform"
    return {"workload": "%s search: one series N=2^%d at %g us, %d %s %s templates, 16 harmonics, 6 sigma, "
                        "whitening W=4096" % (w.name, int(math.log2(n[0])), w.tsamp * 1e6, len(w.templates), drawn,
                                              kind),
            "n": n[0], "tsamp_s": w.tsamp, "templates": int(len(w.templates)), "harmonics": 16,
            "whiten_window": 4096}


def kernel_bytes(n: int, templates_per_launch: float, tile: int = 8192, series_whitening: bool = False):
    """Algorithmic HBM bytes per launch of each kernel class, for series length n:
    the delay polynomials write 48 B per 16 tile points; pass 1 writes the
    4n-byte exchange per template and reads the 4n-byte series once per launch;
    pass 2 reads 4n and writes 2n (and, for a series whitened once, reads its
    2n-byte factors once per launch); the medians and whitening read the
    2n-byte spectrum and write the whitened one; the harmonic sum reads it once
    (first touch)."""
    b = templates_per_launch
    return [48.0 * min(tile, n // 2) / 16 * b, 4.0 * n * b + 4.0 * n,
            6.0 * n * b + (2.0 * n if series_whitening else 0.0), 4.0 * n * b, 0.0, 2.0 * n * b]


def wave_shape(n: int, batch: int = 0):
    """Templates per wave B and per pass-1/2 launch BY the library uses for
    series of n samples (mirrors its defaults)."""
    M = n // 2
    B = batch or min(256, max(4, (1 << 28) // M))
    return B, max(1, min(B, (1 << 24) // M))


def pass1_launches(n: int, templates: int, batch: int = 0) -> int:
    """Pass-1 launches (each reads the series once) of one request."""
    B, BY = wave_shape(n, batch)
    full, rest = divmod(templates, B)
    return full * (-(-B // BY)) + (-(-rest // BY) if rest else 0)


def traffic_record(kernel: str, workload_name: str, what: str = "traffic"):
    """A committed rocprofv3 counter record (HBM traffic, or VALU
    instructions) per launch, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "%s_%s_%s.json" % (what, kernel, workload_name))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    src = os.path.join(ROOT, "paper_2112_11991_amd", "csrc", "tb_kernels.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if rec.get("source_sha256") != sha:
        return None
    return rec


TRACE_SUMMARY = {"c2": "kernel_trace_c2_n2e23.md", "c2_series_whitening": "kernel_trace_c2_series_whitening_n2e23.md"}


def trace_average(kernel: str, workload_name: str):
    """The kernel's average launch duration in the committed rocprofv3 kernel
    trace of this workload (microseconds), if that trace was taken on the
    current kernel source."""
    name = TRACE_SUMMARY.get(workload_name)
    if name is None:
        return None
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        text = f.read()
    src = os.path.join(ROOT, "paper_2112_11991_amd", "csrc", "tb_kernels.hip")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() not in text:
            return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.split("|")]
        if len(cells) > 4 and cells[1].startswith("`%s<" % kernel):
            return {"avg_us": float(cells[4]), "calls": int(cells[2]), "file": "profiles/" + name}
    return None


# The paper's own search times (Table 3; NVIDIA Quadro RTX 6000, precision not
# stated), for one 2^24-sample series at 256 us, divided by its template
# counts.  Context from other hardware, for a different bank and timing that
# may include work outside this path: never a vs_baseline.
PAPER_CONTEXT = {
    "hardware": "NVIDIA Quadro RTX 6000 (paper, Table 3)",
    "series": "N=2^24 at 256 us",
    "circular": {"templates": 10128, "minutes": 1.2, "templates_per_s": 10128 / 72.0},
    "elliptical": {"templates": 2047716, "minutes": 990.0, "templates_per_s": 2047716 / (990.0 * 60.0)},
}


def host_threads():
    """Threads for the CPU oracle: every core this process may use, i.e. its
    CPU affinity, capped by OMP_NUM_THREADS where the host sets it (a GPU
    job's share of a shared host); with the basis stated."""
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    omp = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    if omp and omp < aff:
        return omp, "OMP_NUM_THREADS=%d (CPU affinity %d, nproc %s)" % (omp, aff, os.cpu_count())
    return aff, "CPU affinity %d (nproc %s)" % (aff, os.cpu_count())


def cpu_baseline(w, seconds_hint: float, series_whitening: bool = False, delay_series: bool = False):
    import oracle

    oracle.build()
    threads, share = host_threads()
    x = w.series[0]
    n = x.size
    cfg = oracle.config(n, w.tsamp, series_whitening=series_whitening, delay_model=int(delay_series))
    x0 = oracle.mean_subtract(x)
    t0 = time.perf_counter()
    oracle.search(x0, cfg, w.templates[:1], nthreads=1)
    one = time.perf_counter() - t0
    count = max(threads, int(seconds_hint / max(one, 1e-3)) * threads)
    count = min(count, len(w.templates))
    t0 = time.perf_counter()
    oracle.search(x0, cfg, w.templates[:count], nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": count / dt, "unit": "templates/s", "cores": threads, "kind": "oracle",
            "sample": "first %d templates of the same bank on the same series (N=%d), FP64 C oracle, %d threads, "
                      "%.1f s" % (count, n, threads, dt),
            "single_thread_templates_per_s": 1.0 / one, "cores_basis": share, "nproc": os.cpu_count()}


def kernel_report(plan, n_avg: float, workload_name: str, tile: int, series_whitening: bool = False):
    ms, launches, tmpl = plan.profile_read()
    plan.profile(False)
    per = []
    for k in range(len(KERNELS)):
        if not launches[k]:
            continue
        L = max(1, int(launches[k]))
        avg_ms = ms[k] / L
        byt = kernel_bytes(int(n_avg), tmpl / L, tile, series_whitening)[k]
        per.append({"kernel": KERNEL_SHORT[k], "desc": KERNELS[k], "launches": int(launches[k]), "avg_ms": avg_ms,
                    "total_ms": float(ms[k]), "bytes_per_launch": byt,
                    "gbs": byt / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None})
    d = max(per, key=lambda r: r["total_ms"])
    tr = traffic_record(d["kernel"], workload_name)
    hbm = {"achieved": d["gbs"], "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": d["gbs"] / PEAK_HBM_GBS}
    roof = dict(bound="hbm", kernel=d["kernel"], **hbm)
    roof.update({"traffic": None if tr is None else tr["bytes_per_launch"], "avg_launch_ms": d["avg_ms"],
                 "templates_per_launch": tmpl / max(1, d["launches"])})
    ta = trace_average(d["kernel"], workload_name)
    if ta is not None:
        # events bracket each sampled kernel, so their interval also holds its
        # dispatch after the preceding event; the trace times the kernel alone
        roof["trace_avg_launch_ms"] = ta["avg_us"] * 1e-3
        roof["events_over_trace"] = d["avg_ms"] / (ta["avg_us"] * 1e-3)
        roof["trace_file"] = ta["file"]
    vr = traffic_record(d["kernel"], workload_name, "valu")
    if vr is not None:
        # VALU issue: the counted wave instructions x 64 lanes over the live launch time
        lanes = 64.0 * vr["valu_insts_per_dispatch"]
        ach = lanes / (d["avg_ms"] * 1e-3)
        valu = {"achieved": ach / 1e12, "peak": PEAK_VALU_LANE_OPS / 1e12, "unit": "T lane-ops/s",
                "frac": ach / PEAK_VALU_LANE_OPS, "lane_ops_per_point": vr.get("lane_ops_per_point")}
        roof["hbm"], roof["valu"] = hbm, valu
        if valu["frac"] > hbm["frac"]:
            roof.update(bound="alu", achieved=valu["achieved"], peak=valu["peak"], unit=valu["unit"],
                        frac=valu["frac"])
    return per, roof


def grouping_report(tb, cands, with_oracle: bool):
    """Candidate grouping (tb_distill, host) of one step's candidates: time per
    call and groups kept, for the default rule and with a 1e-3 relative
    tolerance; the oracle's grouping of the same list timed beside it."""
    rep = {"candidates": int(cands.size), "unit": "candidates/s"}
    for name, kw in (("default", dict()), ("ppm1000", dict(ppm=1000))):
        tb.tb_distill(cands, **kw)
        reps = 20
        t0 = time.perf_counter()
        for _ in range(reps):
            kept, _ = tb.tb_distill(cands, **kw)
        dt = (time.perf_counter() - t0) / reps
        rep[name] = {"params": dict(max_ratio=16, tol=16, ppm=kw.get("ppm", 0)), "groups": int(kept.size),
                     "ms": 1e3 * dt, "value": cands.size / dt if dt > 0 else None}
    if with_oracle and cands.size:
        import oracle

        oracle.build()
        o = np.zeros(cands.size, dtype=oracle.CANDIDATE_DTYPE)
        for f in ("series_id", "template_id", "bin", "log2_harm", "power", "sigma", "freq_hz"):
            o[f] = cands[f]
        t0 = time.perf_counter()
        ko, _ = oracle.distill(o)
        dt = time.perf_counter() - t0
        rep["oracle_default"] = {"groups": int(ko.size), "ms": 1e3 * dt, "value": cands.size / dt, "cores": 1}
    return rep


def dedispersion_report(tb, torch, with_oracle: bool):
    """Dedispersion of an 8-bit filterbank shaped like the paper's simulations
    (Table 2: 1024 channels from 1181.8 MHz by 0.390625 MHz, 256 us) over
    2^20 samples (1 GiB, device-resident) into 128 DM trials 0-500 pc cm^-3.
    Rate in channel-sample additions per second of device time (one LDS byte
    read and one integer add each), against the chip's VALU issue rate of
    256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz; the oracle timed on a sample."""
    nchan, nsamp, ndm = 1024, 1 << 20, 128
    f1, df, ts = 1181.804688, 0.390625, 256e-6
    dms = np.linspace(0.0, 500.0, ndm)
    g = torch.Generator(device="cuda").manual_seed(2112)
    x = torch.randint(0, 256, (nsamp, nchan), dtype=torch.uint8, device="cuda", generator=g)
    with tb.Plan() as plan:
        nout, _ = plan.dedisperse(x.data_ptr(), f1, df, ts, dms, nchan=nchan, nsamp=nsamp)
        out = torch.empty(ndm * nout, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        plan.dedisperse(x.data_ptr(), f1, df, ts, dms, out=out.data_ptr(), nchan=nchan, nsamp=nsamp)
        _, ms = plan.dedisperse(x.data_ptr(), f1, df, ts, dms, out=out.data_ptr(), nchan=nchan, nsamp=nsamp)
    adds = float(nchan) * nout * ndm
    peak = 256 * 4 * 16 * 2.4e9
    rep = {"workload": "1024 channels x 2^20 samples (8 bit, 256 us) -> 128 DM trials 0-500", "kernel_ms": ms,
           "value": adds / (ms * 1e-3), "unit": "channel-sample adds/s", "peak": peak, "frac": adds / (ms * 1e-3) / peak,
           "input_gbs": nchan * nsamp / (ms * 1e-3) / 1e9}
    del x, out
    if with_oracle:
        import oracle

        oracle.build()
        xs = np.random.default_rng(1).integers(0, 256, (20000, 64)).astype(np.uint8)
        t0 = time.perf_counter()
        o = oracle.dedisperse(xs, f1, df * 16, ts, dms[:8])
        dt = time.perf_counter() - t0
        rep["oracle"] = {"value": o.size * 64 / dt, "sample": "64 channels x 20000 samples x 8 DMs", "cores": 1}
    return rep


def bank_report(tb, with_oracle: bool):
    """Random-template-bank density kernel on the Table 1 prior region
    (T = 1.2 h, f_max = 66.67 Hz, P_orb 6-12 h, 1.4 + 8 solar masses; e < 0.1
    for the elliptical bank): points per second of device time, 128 nodes;
    the oracle's FP64 numpy density timed beside it on a sample."""
    from paper_2112_11991_amd import bank

    T, f = 1.2 * 3600.0, 66.67
    out = {"unit": "points/s", "nodes": 128}
    rng = np.random.default_rng(2112)
    with tb.Plan() as plan:
        for name, kind, count, emax in (("circular", tb.TB_BANK_CIRCULAR, 1 << 20, 0.0),
                                        ("elliptical", tb.TB_BANK_ELLIPTICAL, 1 << 18, 0.1)):
            pr = bank.Priors(porb_s=(6 * 3600.0, 12 * 3600.0), ecc_max=emax)
            pts, _, _ = bank.proposals(plan, kind, T, f, pr, rng, count)
            plan.bank_density(kind, T, f, pts[:4096])
            _, ms = plan.bank_density(kind, T, f, pts)
            rec = {"points": count, "kernel_ms": ms, "value": count / (ms * 1e-3)}
            if with_oracle:
                from oracle import bank as obank

                k = 2000
                t0 = time.perf_counter()
                obank.density(kind, T, f, pts["porb_s"][:k], pts["tau_lts"][:k], pts["alpha_rad"][:k],
                              pts["ecc"][:k] if kind else None, pts["omega_rad"][:k] if kind else None, nodes=128)
                rec["oracle"] = {"value": k / (time.perf_counter() - t0), "sample": k, "cores": 1}
            out[name] = rec
        pr = bank.Priors(porb_s=(6 * 3600.0, 12 * 3600.0))
        V, err, _ = bank.volume(plan, tb.TB_BANK_CIRCULAR, T, f, pr, rng, points=1 << 20)
        out["table1_circular_count"] = {"value": bank.template_count(V, 3, 0.9, 0.2), "rel_err": err / V,
                                        "paper": 10128}
    return out


def stream_copy_gbs(plan, tb):
    import torch

    nbytes = 1 << 30
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    cms = tb.tb_stream_copy(plan.handle, b.data_ptr(), a.data_ptr(), nbytes, 20)
    return 2.0 * nbytes / (cms * 1e-3) / 1e9


def timed_requests(plan, sids, bank, ntemp):
    """Submits bank[:ntemp] on every series, waits for all; templates/s."""
    t0 = time.perf_counter()
    rids = [plan.submit(sid, bank[:ntemp]) for sid in sids]
    for rid in rids:
        plan.candidates(rid)
        plan.release(rid)
    return len(sids) * ntemp / (time.perf_counter() - t0)


def plain_vs_batched(tb, w, series_idx, ntemp):
    """Templates/s of the one-template-per-launch path (each kernel launched
    for one template, one stream) and of the batched path on the same subset."""
    rates = {}
    for name, kw in (("plain", dict(batch_templates=1, lanes=1)), ("batched", dict(lanes=4))):
        with tb.Plan(whiten_window=w.whiten_window, fmin_hz=w.fmin_hz, ring_capacity=1 << 16, **kw) as plan:
            sids = [plan.load_series(w.series[i], w.tsamp) for i in series_idx]
            for sid in sids:
                plan.search(sid, w.templates[:2])
            rates[name] = timed_requests(plan, sids, w.templates, ntemp)
    return rates


def run_bank(args, tb, torch):
    """c1/c2/c3/c4: every series x the whole bank per step."""
    w = workload(args.workload, args.templates)
    bank_info = None
    if args.workload == "t3":
        w.templates, bank_info = table1_bank(tb, w, args.templates)
    conf = describe(w, args.workload)
    if bank_info is not None:
        conf["bank"] = {k: bank_info[k] for k in ("volume", "volume_err", "count", "proposals")}
    conf["tile_points"] = args.tile or default_tile(max(int(x.size) for x in w.series))
    conf["requests_per_series"] = max(1, args.split)
    if args.series_whitening:
        conf["whitening"] = "once per series (levels from the series' own spectrum)"
    if args.delay_series:
        conf["delay"] = "App. B series of cos E and sqrt(1-e^2) sin E (ELL7), no Kepler solve"
    load_flags = tb.TB_SERIES_WHITENING if args.series_whitening else tb.TB_MEM_HOST
    profile_name = args.workload + ("_series_whitening" if args.series_whitening else "") + \
        ("_delay_series" if args.delay_series else "")
    # one series: waves of one stream keep the device busy (lanes add no throughput there);
    # several series: one request per series, spread over four lanes
    lanes = args.lanes or (4 if len(w.series) > 1 else 1)
    plan = tb.Plan(batch_templates=args.batch, whiten_window=w.whiten_window, harm_max=w.harm_max,
                   threshold_sigma=w.sigma, fmin_hz=w.fmin_hz, lanes=lanes, ring_capacity=1 << 18,
                   tile_points=args.tile, flags=tb.TB_DELAY_SERIES if args.delay_series else 0)
    if args.autotune:
        from paper_2112_11991_amd import tune

        lengths = sorted({int(s.size).bit_length() - 1 for s in w.series})
        t0 = time.perf_counter()
        tuned = tune.autotune(lengths, tsamp=w.tsamp, log=log)
        tune.apply(plan, tuned)
        conf["autotuned"] = {str(k): {"tile_points": v["tile_points"], "batch_templates": v["batch_templates"]}
                             for k, v in tuned.items()}
        conf["autotune_s"] = time.perf_counter() - t0
    sids = [plan.load_series(s, w.tsamp, flags=load_flags) for s in w.series]
    ntemp = len(w.templates)
    nitems = ntemp * len(sids)

    chunks = np.array_split(np.arange(ntemp), max(1, args.split))

    last = []

    def step():
        rids = [plan.submit(sid, w.templates[c[0]:c[-1] + 1], int(c[0])) for sid in sids for c in chunks if len(c)]
        ncand = 0
        last.clear()
        for rid in rids:
            c, tot = plan.candidates(rid)
            last.append(c)
            ncand += tot
            plan.release(rid)
        return ncand

    for i in range(args.warmup):
        log("warmup", i)
        step()
    torch.cuda.synchronize()
    if not args.no_profile:
        plan.profile(PROFILE_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ncand = 0
    for i in range(args.steps):
        ncand += step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = nitems * args.steps / dt
    ms_step = 1e3 * dt / args.steps
    log("timed %d steps: %.1f ms/step, %.0f templates/s, %d candidates/step" % (args.steps, ms_step, value,
                                                                                ncand // max(1, args.steps)))
    # The series are resident when the timed region starts.  The host hand-over
    # is timed apart: every series loaded once more from pageable host memory
    # (copy to HBM and its preprocessing on the device), then unloaded.
    t1 = time.perf_counter()
    extra = [plan.load_series(s, w.tsamp, flags=load_flags) for s in w.series]
    torch.cuda.synchronize()
    load_s = time.perf_counter() - t1
    for sid in extra:
        plan.unload_series(sid)
    samples_total = float(sum(s.size for s in w.series))
    metric = METRIC if args.workload == "c2" else "templates/s (%s)" % args.workload
    if args.workload == "t3":
        metric = "templates/s (the paper's circular search: N=2^24 at 256 us, Table 1 bank)"
    if args.series_whitening:
        metric += " [whitened once per series]"
    if args.delay_series:
        metric += " [series delay]"
    out = {"metric": metric, "value": value,
           "unit": "templates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": conf, "candidates_per_step": ncand // max(1, args.steps),
           "algorithmic_gbs": 12.0 * samples_total * ntemp * args.steps / dt / 1e9}
    out["pcie_inclusive"] = {
        "value": nitems / (dt / args.steps + load_s), "unit": "templates/s", "series_load_ms": 1e3 * load_s,
        "series_bytes": int(sum(s.nbytes for s in w.series)),
        "basis": "one step plus one load of every series from pageable host memory (not the headline value)"}
    out["algorithmic_hbm_frac"] = out["algorithmic_gbs"] / PEAK_HBM_GBS
    # whole path: 12n bytes per template plus the series read of every pass-1 launch
    batch = args.batch or 0
    if args.autotune:
        batch = None
    if batch is not None:
        launches = sum(pass1_launches(int(x.size), len(c), batch) for x in w.series for c in chunks if len(c))
        step_bytes = 12.0 * samples_total * ntemp + sum(
            4.0 * x.size * pass1_launches(int(x.size), len(c), batch) for x in w.series for c in chunks if len(c))
        gbs = step_bytes / (ms_step * 1e-3) / 1e9
        out["path_roofline"] = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                "frac": gbs / PEAK_HBM_GBS, "bytes_per_step": step_bytes,
                                "pass1_launches_per_step": launches}
    if not args.no_profile:
        out["kernels"], out["roofline"] = kernel_report(plan, samples_total / len(w.series), profile_name,
                                                     conf["tile_points"], args.series_whitening)
        out["stream_copy_gbs"] = stream_copy_gbs(plan, tb)
    plan.close()
    out["grouping"] = grouping_report(tb, np.concatenate(last) if last else np.zeros(0, tb.CANDIDATE_DTYPE),
                                      not args.no_cpu_baseline)
    if args.workload == "c2":
        out["bank"] = bank_report(tb, not args.no_cpu_baseline)
        out["dedispersion"] = dedispersion_report(tb, torch, not args.no_cpu_baseline)
        if not args.no_batching:
            log("batched vs one template per launch ...")
            out["batching"] = batching_report(tb)
            out["batched_vs_plain"] = {k: v["batched_vs_plain"] for k, v in out["batching"]["per_length"].items()}
        if args.serve_requests:
            out["serving"] = served(tb, torch, args.serve_requests, 4, False)
            half = out["serving"]["half_capacity"]
            # latency of the stream at half its measured capacity (at the trace's own
            # rate the latency is queueing and grows with the trace)
            out["p50_ms"], out["p99_ms"] = half["p50_ms"], half["p99_ms"]
            out["latency_basis"] = "%d-request served trace at %.2f req/s (half the measured capacity)" % (
                args.serve_requests, half["rate_req_s"])
    if args.workload == "c4" and not args.no_plain:
        idx = list(range(min(4, len(w.series))))
        rates = plain_vs_batched(tb, w, idx, 256)
        out["plain_one_template_per_launch"] = {"value": rates["plain"], "unit": "templates/s",
                                                "sample": "series %s x first 256 templates" % idx}
        out["batched_same_subset"] = {"value": rates["batched"], "unit": "templates/s"}
        out["batched_vs_plain"] = rates["batched"] / rates["plain"]
    if args.workload in ("c2", "c3", "t3"):
        out["paper_context"] = PAPER_CONTEXT
    if args.workload == "t3" and not (args.series_whitening or args.delay_series):
        # the paper's own circular search time for this series and bank size
        out["vs_baseline"] = value / PAPER_CONTEXT["circular"]["templates_per_s"]
        out["vs_baseline_basis"] = ("Table 3: 10,128 circular templates on one 2^24-sample series at 256 us in "
                                    "1.2 min on an NVIDIA Quadro RTX 6000 (140.7 templates/s)")
    if not args.no_cpu_baseline and args.workload in ("c1", "c2", "c3", "t3"):
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds, args.series_whitening, args.delay_series)
    return out


def served(tb, torch, nreq, lanes=4, with_plain=True):
    """The continuous-batching loop over a Poisson request trace (50/s; pool of
    16 series of 2^20..2^24 samples; 256-4096 templates per request, 30%%
    elliptical; 200 GB HBM budget): throughput and p50/p99 latency (arrival ->
    candidates retrievable) with the trace at its own rate (saturating: the
    trace offers several times the capacity, so latency is queueing) and
    stretched to half the measured capacity (the latency floor)."""
    import synth
    from paper_2112_11991_amd.serve import Request, serve

    lens, reqs = synth.request_trace(nreq)
    series = synth.pool_series(lens)
    tsamp = 64e-6
    plan = tb.Plan(lanes=lanes, ring_capacity=1 << 16, hbm_budget_bytes=200 * 10**9, fmin_hz=1.0)
    sids = [plan.load_series(s, tsamp) for s in series]
    for n in sorted(set(lens)):
        plan.search(sids[lens.index(n)], reqs[0]["templates"][:8])
    torch.cuda.synchronize()

    def requests():
        return [Request(r["t_arrival"], r["series"], r["templates"], 100000 * k) for k, r in enumerate(reqs)]

    log("serving %d requests at 50/s ..." % nreq)
    rep = serve(plan, sids, lens, requests(), realtime=True)
    log("  p50 %.1f ms p99 %.1f ms, %.0f templates/s" % (rep.p50_ms, rep.p99_ms, rep.templates_per_s))
    scale = 50.0 / (0.5 * rep.n_requests / rep.makespan_s)
    log("serving at %.2f req/s ..." % (50.0 / scale))
    rep2 = serve(plan, sids, lens, requests(), realtime=True, time_scale=scale)
    log("  p50 %.1f ms p99 %.1f ms" % (rep2.p50_ms, rep2.p99_ms))
    plan.close()
    out = {"workload": "served stream: %d requests, Poisson 50/s, pool of 16 series 2^20..2^24 at 64 us, 256-4096 "
                       "templates each, 30%% elliptical, HBM budget 200 GB" % nreq,
           "requests": nreq, "templates_per_s": rep.templates_per_s, "saturation": rep.as_dict(),
           "half_capacity": dict(rep2.as_dict(), rate_req_s=50.0 / scale)}
    if with_plain:
        rates = {}
        sub = requests()[:6]
        for name, kw in (("plain", dict(batch_templates=1, lanes=1)), ("served", dict(lanes=lanes))):
            with tb.Plan(ring_capacity=1 << 16, **kw) as pp:
                ps = {r.series: None for r in sub}
                for k in ps:
                    ps[k] = pp.load_series(series[k], tsamp)
                    pp.search(ps[k], sub[0].templates[:2])
                t0 = time.perf_counter()
                rids = [pp.submit(ps[r.series], r.templates[:128]) for r in sub]
                for rid in rids:
                    pp.candidates(rid)
                    pp.release(rid)
                rates[name] = sum(min(128, len(r.templates)) for r in sub) / (time.perf_counter() - t0)
        out["plain_one_template_per_launch"] = {"value": rates["plain"], "unit": "templates/s",
                                                "sample": "first 6 requests, first 128 templates each"}
        out["lanes_same_subset"] = {"value": rates["served"], "unit": "templates/s"}
        out["served_vs_plain"] = rates["served"] / rates["plain"]
    return out


def batching_report(tb, lengths=(20, 21, 22, 23), ntemp=256, tsamp=64e-6, reps=2):
    """Batched search (the library's waves of 64-256 templates, four lanes)
    against the one-template-per-launch path (every kernel launched for a
    single template, one stream) on the same noise series and the same 256
    circular templates, for each series length of the uneven-length search."""
    import synth

    rng = np.random.default_rng(2112)
    bank = synth.uniform_templates(rng, ntemp, (1.0, 10.0), (0.0, 2.0))
    out = {"templates": ntemp, "unit": "templates/s", "per_length": {}}
    for lg in lengths:
        x = rng.standard_normal(1 << lg).astype(np.float32)
        rates = {}
        for name, kw in (("plain", dict(batch_templates=1, lanes=1)), ("batched", dict(lanes=4))):
            with tb.Plan(ring_capacity=1 << 16, **kw) as plan:
                sid = plan.load_series(x, tsamp)
                plan.search(sid, bank[:8])
                best = 0.0
                for _ in range(reps):
                    t0 = time.perf_counter()
                    plan.search(sid, bank)
                    best = max(best, ntemp / (time.perf_counter() - t0))
                rates[name] = best
        out["per_length"]["2^%d" % lg] = {"plain": rates["plain"], "batched": rates["batched"],
                                          "batched_vs_plain": rates["batched"] / rates["plain"]}
        log("  2^%d: plain %.0f, batched %.0f templates/s" % (lg, rates["plain"], rates["batched"]))
    return out


def run_served(args, tb, torch):
    """c5: Poisson request stream served by the continuous-batching loop."""
    rep = served(tb, torch, args.requests, args.lanes or 4, not args.no_plain)
    sat = rep["saturation"]
    out = {"metric": "served templates/s and p50/p99 latency (request stream)", "value": rep["templates_per_s"],
           "unit": "templates/s", "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": sat["makespan_s"] * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": rep.pop("workload")}, "p50_ms": sat["p50_ms"], "p99_ms": sat["p99_ms"]}
    out.update(rep)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5", "t3"])
    ap.add_argument("--templates", type=int, default=None)
    ap.add_argument("--requests", type=int, default=400, help="requests of the c5 trace")
    ap.add_argument("--serve-requests", type=int, default=64,
                    help="requests of the short served trace in the default run (0 = none)")
    ap.add_argument("--no-batching", action="store_true",
                    help="skip the per-length batched vs one-template-per-launch comparison of the default run")
    ap.add_argument("--batch", type=int, default=0, help="templates in flight per launch (0 = library default)")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--split", type=int, default=1, help="requests the bank is cut into per series (spread over lanes)")
    ap.add_argument("--tile", type=int, default=0, help="FFT points per workgroup, 8192 or 16384 (0 = library default)")
    ap.add_argument("--series-whitening", action="store_true",
                    help="whiten once per series (levels from its own spectrum) instead of per template")
    ap.add_argument("--delay-series", action="store_true",
                    help="Roemer delay from the App. B series (ELL7) instead of BT with a Newton solve")
    ap.add_argument("--autotune", action="store_true",
                    help="choose FFT tile and templates per wave for each series length by timing them first")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="do not record per-kernel events")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-template-per-launch comparison")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the search runs on one GPU; --gpus %d is not supported (sharding the bank over GPUs is "
              "described, not implemented)" % args.gpus, file=sys.stderr)
        return 2

    import torch

    import paper_2112_11991_amd as tb

    torch.cuda.set_device(0)
    log("workload", args.workload)
    out = run_served(args, tb, torch) if args.workload == "c5" else run_bank(args, tb, torch)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
