"""Checks of bench.py that need no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    """The search runs on one GPU; asking for more exits with status 2 and a
    message, before anything touches a device, and prints no JSON line."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_wave_shape_mirrors_the_library_default():
    """bench.py's accounting of pass-1 launches uses the library's default
    wave: 2^28 bins in flight (64 templates at 2^23, 32 at 2^24, at most 256),
    passes 1-2 on 2^24 / (n/2) templates per launch."""
    sys.path.insert(0, ROOT)
    import bench

    assert bench.wave_shape(1 << 23) == (64, 4)
    assert bench.wave_shape(1 << 24) == (32, 2)
    assert bench.wave_shape(1 << 20) == (256, 32)
    assert bench.wave_shape(1 << 23, 16) == (16, 4)
    # 20,000 templates at 2^23: 312 full waves of 16 launches and one of 32 templates (8 launches)
    assert bench.pass1_launches(1 << 23, 20000) == 312 * 16 + 8


def test_paper_context_rates():
    """The paper's Table 3 times divided by its template counts."""
    sys.path.insert(0, ROOT)
    import bench

    assert abs(bench.PAPER_CONTEXT["circular"]["templates_per_s"] - 140.67) < 0.01
    assert abs(bench.PAPER_CONTEXT["elliptical"]["templates_per_s"] - 34.47) < 0.01


def test_trace_average_reads_the_committed_summary():
    """The roofline line's trace figure comes from the committed C2 kernel
    trace when it was taken on the current kernel source."""
    sys.path.insert(0, ROOT)
    import bench

    t = bench.trace_average("k_fft1", "c2")
    if t is not None:
        assert t["calls"] > 0 and 10.0 < t["avg_us"] < 1000.0 and t["file"].startswith("profiles/")
    assert bench.trace_average("k_fft1", "no_such_workload") is None
