"""Benchmark of the template-bank coherent orbital search on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload c2|c1|c3|c4]

One step is one pass of the whole search (resample, FFT, power, whitening,
harmonic sum, peaks) over the workload's full template bank, with the series
already resident in HBM.  The default workload is the circular survey-scale
search: one 2^23-sample series at 64 us with red noise and a pulsar, 20,000
uniform circular templates.  Prints one JSON line on stdout; progress goes to
stderr.  Only one GPU is used: --gpus above 1 exits with a message.
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
KERNELS = ["k_pass1 (resample + FFT pass 1)", "k_pass2 (FFT pass 2 + power)", "k_median (whitening medians)",
           "k_whiten (whitening)", "k_harmsum (harmonic sum + peaks)"]
KERNEL_SHORT = ["k_pass1", "k_pass2", "k_median", "k_whiten", "k_harmsum"]


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
    raise SystemExit("unknown workload " + name)


def describe(w, name):
    n = [int(s.size) for s in w.series]
    if name == "c4":
        return {"workload": "batched uneven-length search: %d series of 2^20..2^23 samples at 64 us, %d shared circular "
                            "templates" % (len(n), len(w.templates)), "series": len(n), "samples_total": int(sum(n)),
                "templates": int(len(w.templates))}
    kind = "elliptical" if w.templates["ecc"].max() > 0 else "circular"
    return {"workload": "%s search: one series N=2^%d at %g us, %d uniform %s templates, 16 harmonics, 6 sigma, "
                        "whitening W=4096" % (w.name, int(math.log2(n[0])), w.tsamp * 1e6, len(w.templates), kind),
            "n": n[0], "tsamp_s": w.tsamp, "templates": int(len(w.templates)), "harmonics": 16,
            "whiten_window": 4096}


def kernel_bytes(n: int, templates_per_launch: float):
    """Algorithmic HBM bytes per launch of each kernel class, for series length n:
    pass 1 writes the 4n-byte exchange per template and reads the 4n-byte series
    once per launch; pass 2 reads 4n and writes 2n; the medians read the
    2n-byte spectrum, the whitening reads and rewrites it, the harmonic sum
    reads it once (first touch)."""
    b = templates_per_launch
    return [4.0 * n * b + 4.0 * n, 6.0 * n * b, 2.0 * n * b, 4.0 * n * b, 2.0 * n * b]


def traffic_record(kernel: str):
    """Measured HBM traffic per launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % kernel)
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


def cpu_baseline(w, seconds_hint: float):
    import oracle

    oracle.build()
    threads = max(1, min(os.cpu_count() or 1, 16))
    x = w.series[0]
    n = x.size
    cfg = oracle.config(n, w.tsamp)
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
            "single_thread_templates_per_s": 1.0 / one}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--templates", type=int, default=None)
    ap.add_argument("--batch", type=int, default=0, help="templates in flight per launch (0 = library default)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="do not record per-kernel events")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus %d is not supported (multi-GPU sharding is a design "
              "note only)" % args.gpus, file=sys.stderr)
        return 2

    import torch

    import paper_2112_11991_amd as tb

    log("workload", args.workload)
    w = workload(args.workload, args.templates)
    conf = describe(w, args.workload)
    torch.cuda.set_device(0)
    plan = tb.Plan(batch_templates=args.batch, whiten_window=w.whiten_window, harm_max=w.harm_max,
                   threshold_sigma=w.sigma, fmin_hz=w.fmin_hz)
    sids = [plan.load_series(s, w.tsamp) for s in w.series]
    ntemp = len(w.templates)
    nitems = ntemp * len(sids)

    def step():
        rids = [plan.submit(sid, w.templates) for sid in sids]
        ncand = 0
        for rid in rids:
            c, tot = plan.candidates(rid)
            ncand += tot
            plan.release(rid)
        return ncand

    for i in range(args.warmup):
        log("warmup", i)
        step()
    torch.cuda.synchronize()
    if not args.no_profile:
        plan.profile(True)
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

    n_avg = float(np.mean([s.size for s in w.series]))
    samples_total = float(sum(s.size for s in w.series))
    out = {
        "metric": "templates/s (resample+FFT+harmsum+peaks) at N=2^23 FP32",
        "value": value,
        "unit": "templates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": conf,
        "candidates_per_step": ncand // max(1, args.steps),
        "algorithmic_gbs": 12.0 * samples_total * ntemp * args.steps / dt / 1e9,
    }
    out["algorithmic_hbm_frac"] = out["algorithmic_gbs"] / PEAK_HBM_GBS

    if not args.no_profile:
        ms, launches, tmpl = plan.profile_read()
        plan.profile(False)
        per = []
        for k in range(5):
            L = max(1, int(launches[k]))
            avg_ms = ms[k] / L
            byt = kernel_bytes(int(n_avg), tmpl / L)[k]
            per.append({"kernel": KERNEL_SHORT[k], "desc": KERNELS[k], "launches": int(launches[k]),
                        "avg_ms": avg_ms, "total_ms": float(ms[k]), "bytes_per_launch": byt,
                        "gbs": byt / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None})
        out["kernels"] = per
        dom = max(range(5), key=lambda k: ms[k])
        d = per[dom]
        tr = traffic_record(d["kernel"])
        out["roofline"] = {"bound": "hbm", "kernel": d["kernel"], "achieved": d["gbs"], "peak": PEAK_HBM_GBS,
                           "unit": "GB/s", "frac": d["gbs"] / PEAK_HBM_GBS,
                           "traffic": None if tr is None else tr["bytes_per_launch"],
                           "avg_launch_ms": d["avg_ms"], "templates_per_launch": tmpl / max(1, int(launches[dom]))}
        # practical ceiling: a plain streaming copy of 1 GiB
        nbytes = 1 << 30
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        cms = tb.tb_stream_copy(plan.handle, b.data_ptr(), a.data_ptr(), nbytes, 20)
        out["stream_copy_gbs"] = 2.0 * nbytes / (cms * 1e-3) / 1e9
        del a, b
    plan.close()

    if not args.no_cpu_baseline and args.workload in ("c1", "c2", "c3"):
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
