"""Parity of the HIP path (through the C ABI) with the oracle, stage by stage
and on the final candidate lists, on seeded synthetic series."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from tests import parity_rules as R

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tb():
    import paper_2112_11991_amd as tb

    return tb


def _series(n, ts, seed, red=False, orbit=None, pspin=0.02, snr=20.0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n)
    if red:
        x = x + synth.red_noise(n, ts, rng)
    if orbit is not None:
        x = synth.inject(x, synth.pulse_train(n, ts, pspin, 0.05, orbit), snr)
    return x.astype(np.float32)


def _stage_check(tb, plan, sid, x, n, ts, tm, W, harm=16):
    cfg = oracle.config(n, ts, harm_max=harm, whiten_window=W)
    x0 = oracle.mean_subtract(x)
    st = oracle.template_stages(x0, cfg, tm)
    _, delta = oracle.resample_index(tm, n, ts)
    g = plan.inspect(sid, tm)
    ex = R.check_indices(g["src"], st["src"], delta)
    R.check_power(g["power"], st["p"], st["med"], W)
    R.check_medians(g["medians"], st["med"])
    R.check_phat(g["sums"][0], st["phat"])
    R.check_sums(g["sums"], st["s"])
    return ex


CASES = [
    # (log2 n, tsamp, whitening W, template)
    (10, 64e-6, 64, (30.0, 0.01, 0.3, 0.0, 0.0)),
    (12, 64e-6, 1000, (100.0, 0.02, 2.0, 0.0, 0.0)),
    (14, 256e-6, 4096, (600.0, 0.3, 4.0, 0.0, 0.0)),
    (15, 256e-6, 3000, (900.0, 0.8, 1.0, 0.3, 2.5)),
    (17, 64e-6, 4096, (7200.0, 0.5, 1.0, 0.0, 0.0)),
    (18, 64e-6, 4096, (1800.0, 1.5, 5.5, 0.1, 0.7)),
    (19, 64e-6, 2048, (3000.0, 2.0, 0.1, 0.0, 0.0)),
    # a short orbit whose delay needs the 8-point polynomial chunks at this size
    (21, 64e-6, 4096, (380.0, 1.5, 2.0, 0.05, 1.0)),
    # a delay swing (about 12,000 samples) beyond the zero rows around the
    # resident series (8,223 samples at 2^16): the exact per-sample path,
    # though the polynomials would be accurate
    (16, 64e-6, 4096, (100.0, 3.0, 0.5, 0.0, 0.0)),
    # whitening windows at the ends of their range: one bin per block (every
    # whitened bin is ln 2), and blocks wider than 4096 bins (32 values per
    # thread), whole and with a short last block
    (10, 64e-6, 1, (30.0, 0.01, 0.3, 0.0, 0.0)),
    (17, 64e-6, 8192, (7200.0, 0.5, 1.0, 0.0, 0.0)),
    (16, 64e-6, 5000, (3000.0, 0.4, 2.0, 0.05, 0.3)),
]


@pytest.mark.parametrize("lg,ts,W,tm", CASES)
def test_stages_match_oracle(tb, lg, ts, W, tm):
    n = 1 << lg
    _say("stages n=2^%d W=%d tm=%s" % (lg, W, tm))
    x = _series(n, ts, seed=lg, red=True, orbit=synth.Orbit(*tm), pspin=0.013)
    with tb.Plan(whiten_window=W) as plan:
        sid = plan.load_series(x, ts)
        ex = _stage_check(tb, plan, sid, x, n, ts, tm, W)
        _say("  tie-exempt indices:", ex)


TILE_CASES = [
    # 16384-point tiles (one workgroup per CU): pass-1 columns C1 = 16 .. 1, pass-2 transforms of 16 and 64 points
    (15, 256e-6, 3000, (900.0, 0.8, 1.0, 0.3, 2.5)),
    (17, 64e-6, 4096, (7200.0, 0.5, 1.0, 0.0, 0.0)),
    (19, 64e-6, 2048, (3000.0, 2.0, 0.1, 0.0, 0.0)),
    (21, 64e-6, 4096, (3600.0, 1.2, 4.0, 0.05, 1.5)),
]


@pytest.mark.parametrize("lg,ts,W,tm", TILE_CASES)
def test_stages_match_oracle_16384_point_tiles(tb, lg, ts, W, tm):
    n = 1 << lg
    _say("stages (16384-point tiles) n=2^%d W=%d tm=%s" % (lg, W, tm))
    x = _series(n, ts, seed=100 + lg, red=True, orbit=synth.Orbit(*tm), pspin=0.017)
    with tb.Plan(whiten_window=W, tile_points=16384) as plan:
        sid = plan.load_series(x, ts)
        ex = _stage_check(tb, plan, sid, x, n, ts, tm, W)
        _say("  tie-exempt indices:", ex)


@pytest.mark.parametrize("kind", ["impulse", "zeros"])
def test_crowded_median_digits(tb, kind):
    """Spectra whose whitening blocks hold thousands of (nearly) equal powers:
    a unit impulse (|X_k|^2 = 1 for k >= 1 up to FP32 rounding, so the
    values of a block share the median's leading bits) and an all-zero series
    (every power exactly 0).  The radix selection of the block medians meets
    crowded digits in every pass; every stage still matches the oracle."""
    n, ts, W = 1 << 16, 64e-6, 4096
    x = np.zeros(n, np.float32)
    if kind == "impulse":
        x[12345] = 1.0
    tm = (3600.0, 0.0, 0.0, 0.0, 0.0)
    _say("crowded median digits: %s" % kind)
    with tb.Plan(whiten_window=W) as plan:
        sid = plan.load_series(x, ts)
        _stage_check(tb, plan, sid, x, n, ts, tm, W)


def test_zero_orbit_is_identity_on_gpu(tb):
    n, ts = 1 << 16, 64e-6
    x = _series(n, ts, seed=5)
    with tb.Plan() as plan:
        sid = plan.load_series(x, ts)
        for tm in [(3600.0, 0.0, 1.0, 0.0, 0.0), (5000.0, 0.0, 2.0, 0.5, 1.0)]:
            g = plan.inspect(sid, tm, want=("src",))
            assert np.array_equal(g["src"], np.arange(n, dtype=np.int32))


def test_out_of_range_source_reads_zero(tb):
    """A template whose delay sends reads past the end of the series: the
    oracle's zero fill and the GPU agree (indices and spectrum)."""
    n, ts = 1 << 13, 1e-3
    tm = (20.0, 0.5, math.pi, 0.0, 0.0)
    x = _series(n, ts, seed=6)
    with tb.Plan(whiten_window=512) as plan:
        sid = plan.load_series(x, ts)
        g = plan.inspect(sid, tm, want=("src",))
        assert (g["src"] >= n).any()
        _stage_check(tb, plan, sid, x, n, ts, tm, 512)


@pytest.mark.parametrize("harm", [1, 2, 4, 8])
def test_fewer_harmonics(tb, harm):
    n, ts = 1 << 15, 64e-6
    tm = (1200.0, 0.4, 2.2, 0.0, 0.0)
    x = _series(n, ts, seed=40 + harm, orbit=synth.Orbit(*tm), pspin=0.011)
    with tb.Plan(harm_max=harm, whiten_window=2048) as plan:
        sid = plan.load_series(x, ts)
        _stage_check(tb, plan, sid, x, n, ts, tm, 2048, harm=harm)


def test_c1_candidates_match_oracle(tb):
    """Workload of the tiny configuration: 2^17 samples, 64 + 1 circular
    templates; full candidate lists compared."""
    w = synth.c1_tiny()
    x, ts = w.series[0], w.tsamp
    n = x.size
    _say("c1 candidates: %d templates" % len(w.templates))
    with tb.Plan() as plan:
        sid = plan.load_series(x, ts)
        cg = plan.search(sid, w.templates, first_template_id=1000)
        thr = [float(v) for v in plan.thresholds()]
    co = oracle.search(oracle.mean_subtract(x), oracle.config(n, ts), w.templates, first_template_id=1000,
                       series_id=int(sid))
    matched, exempt = R.check_candidates(cg, co, [oracle.threshold(1 << l, 6.0) for l in range(5)])
    _say("  matched %d, near-threshold exempt %d" % (matched, exempt))
    assert matched > 0
    assert np.allclose(thr, [oracle.threshold(1 << l, 6.0) for l in range(5)], rtol=1e-6)
    # the strongest detection is the oracle's (2^17 samples span 0.1% of the
    # 2 h orbit, so every template recovers the pulsar about equally well)
    bg, bo = cg[np.argmax(cg["sigma"])], co[np.argmax(co["sigma"])]
    assert (bg["template_id"], bg["log2_harm"], bg["bin"]) == (bo["template_id"], bo["log2_harm"], bo["bin"])


def test_elliptical_candidates_match_oracle(tb):
    n, ts = 1 << 16, 256e-6
    rng = np.random.default_rng(77)
    tms = synth.uniform_templates(rng, 12, (0.5, 2.0), (0.0, 1.0), ecc_max=0.5)
    true = synth.Orbit(float(tms["porb_s"][3]), float(tms["tau_lts"][3]), float(tms["alpha_rad"][3]),
                       float(tms["ecc"][3]), float(tms["omega_rad"][3]))
    x = _series(n, ts, seed=78, orbit=true, pspin=0.05, snr=40.0)
    with tb.Plan(whiten_window=2048) as plan:
        sid = plan.load_series(x, ts)
        cg = plan.search(sid, tms)
    co = oracle.search(oracle.mean_subtract(x), oracle.config(n, ts, whiten_window=2048), tms,
                       series_id=int(sid))
    matched, exempt = R.check_candidates(cg, co, [oracle.threshold(1 << l, 6.0) for l in range(5)])
    _say("elliptical matched %d exempt %d" % (matched, exempt))
    assert matched > 0


def test_band_limits(tb):
    n, ts = 1 << 16, 64e-6
    tm = [(900.0, 0.2, 1.0, 0.0, 0.0), (1500.0, 0.1, 3.0, 0.0, 0.0)]
    x = _series(n, ts, seed=9, orbit=synth.Orbit(*tm[0]), pspin=0.007, snr=30.0)
    with tb.Plan(fmin_hz=30.0, fmax_hz=300.0, whiten_window=1024) as plan:
        sid = plan.load_series(x, ts)
        cg = plan.search(sid, tm)
    co = oracle.search(oracle.mean_subtract(x),
                       oracle.config(n, ts, whiten_window=1024, fmin_hz=30.0, fmax_hz=300.0), tm,
                       series_id=int(sid))
    R.check_candidates(cg, co, [oracle.threshold(1 << l, 6.0) for l in range(5)])
    assert len(cg) > 0 and cg["freq_hz"].min() >= 30.0 - 1.0 / (n * ts) and cg["freq_hz"].max() <= 300.0


def test_empty_requests(tb):
    """A request of no templates completes with no candidates on every
    entry point (queued search, allocation-free search, served stream), and
    the plan searches normally afterwards."""
    n, ts = 1 << 14, 64e-6
    x = _series(n, ts, seed=15, orbit=synth.Orbit(600.0, 0.2, 1.0), pspin=0.011, snr=30.0)
    none = np.zeros(0, dtype=tb.TEMPLATE_DTYPE)
    with tb.Plan(whiten_window=1024) as plan:
        sid = plan.load_series(x, ts)
        assert plan.search(sid, none).size == 0
        c, total = plan.search_noalloc(sid, none)
        assert c.size == 0 and total == 0
        res, cands, _ = plan.serve([(0.0, sid, none, 0), (0.0, sid, none, 5)], saturate=True)
        assert cands.size == 0 and np.all(res["n_total"] == 0) and np.all(res["status"] == tb.TB_OK)
        assert plan.search(sid, [(600.0, 0.2, 1.0, 0.0, 0.0)]).size > 0


def test_batching_invariance(tb):
    """Each template alone equals the same template inside a batch, bit for bit."""
    n, ts = 1 << 16, 64e-6
    rng = np.random.default_rng(11)
    tms = synth.uniform_templates(rng, 20, (0.2, 1.0), (0.0, 0.5))
    x = _series(n, ts, seed=12, orbit=synth.Orbit(*[float(v) for v in tms[7]]), pspin=0.009, snr=25.0)
    with tb.Plan(batch_templates=8, fmin_hz=0.5) as plan:
        sid = plan.load_series(x, ts)
        allc = plan.search(sid, tms)
        for i in [0, 7, 19]:
            one = plan.search(sid, tms[i:i + 1], first_template_id=i)
            sub = allc[allc["template_id"] == i]
            assert np.array_equal(one, sub), i


def test_ring_overflow_reports_exact_total(tb):
    n, ts = 1 << 14, 64e-6
    x = _series(n, ts, seed=13)
    tm = [(600.0, 0.1, 0.0, 0.0, 0.0)] * 3
    with tb.Plan(threshold_sigma=0.5, ring_capacity=100, whiten_window=1024) as plan:
        sid = plan.load_series(x, ts)
        rid = plan.submit(sid, tm)
        with pytest.raises(tb.TbError) as e:
            plan.candidates(rid)
        assert e.value.status == tb.TB_ERR_OVERFLOW
        kept, total = plan.candidates(rid, allow_overflow=True)
        plan.release(rid)
    co = oracle.search(oracle.mean_subtract(x), oracle.config(n, ts, whiten_window=1024, threshold_sigma=0.5), tm)
    assert len(kept) == 100
    # the exact count, up to near-threshold records
    assert abs(total - len(co)) <= max(3, int(1e-3 * len(co)))


def test_argument_errors(tb):
    n, ts = 1 << 12, 64e-6
    x = _series(n, ts, seed=14)
    with tb.Plan(max_log2n=16) as plan:
        with pytest.raises(tb.TbError) as e:
            plan.load_series(x[:1000], ts)
        assert e.value.status == tb.TB_ERR_INVALID_ARG
        with pytest.raises(tb.TbError):
            plan.load_series(np.zeros(1 << 17, np.float32), ts)
        sid = plan.load_series(x, ts)
        for bad in [(0.0, 1.0, 0.0, 0.0, 0.0), (100.0, -1.0, 0.0, 0.0, 0.0), (100.0, 1.0, 0.0, 1.0, 0.0),
                    (100.0, 1.0, float("nan"), 0.0, 0.0)]:
            with pytest.raises(tb.TbError) as e:
                plan.submit(sid, [bad])
            assert e.value.status == tb.TB_ERR_INVALID_ARG
        with pytest.raises(tb.TbError) as e:
            plan.submit(sid + 99, [(100.0, 1.0, 0.0, 0.0, 0.0)])
        assert e.value.status == tb.TB_ERR_UNKNOWN_ID
        with pytest.raises(tb.TbError) as e:
            plan.candidates(12345)
        assert e.value.status == tb.TB_ERR_UNKNOWN_ID


def test_hbm_budget_admission(tb):
    """A series is admitted while the budget holds its bytes (samples plus the
    zero rows around its columns, 4n to 5n) and refused otherwise."""
    n, ts = 1 << 16, 64e-6
    x = _series(n, ts, seed=15)
    with tb.Plan() as plan:
        plan.load_series(x, ts)  # lays out the length too
        h1 = plan.memory()[0]
        plan.load_series(x, ts)
        per = plan.memory()[0] - h1
        assert 4 * n <= per <= 5 * n
        plan.set_budget(plan.memory()[0] + per - 1)
        with pytest.raises(tb.TbError) as e:
            plan.load_series(x, ts)
        assert e.value.status == tb.TB_ERR_BUDGET
        plan.set_budget(plan.memory()[0] + per)
        plan.load_series(x, ts)


def test_device_resident_input(tb):
    import torch

    n, ts = 1 << 15, 64e-6
    x = _series(n, ts, seed=16, orbit=synth.Orbit(800.0, 0.3, 1.0), pspin=0.01)
    xd = torch.from_numpy(x).to("cuda:0")
    torch.cuda.synchronize()
    tm = [(800.0, 0.3, 1.0, 0.0, 0.0)]
    with tb.Plan() as plan:
        s_host = plan.load_series(x, ts)
        s_dev = plan.load_series(xd.data_ptr(), ts, n=n, flags=tb.TB_MEM_DEVICE)
        a = plan.search(s_host, tm)
        b = plan.search(s_dev, tm)
    assert np.array_equal(a[["template_id", "bin", "log2_harm", "power"]], b[["template_id", "bin", "log2_harm", "power"]])


def test_full_size_circular_survey(tb):
    """2^23 samples with red noise and a pulsar, in the benchmark's launch
    configuration (the library defaults: 64 templates per wave, passes 1-2 in
    groups of 4, 8192-point tiles, 64 median blocks per workgroup): bit-exact
    indices and whole-spectrum power parity for one template, candidate
    parity for all 64 templates of the wave (63 of the bank and the injected
    orbit)."""
    w = synth.c2_survey(n_templates=63)
    w.templates = np.concatenate([w.templates, w.truths[0][1].as_template()])
    x, ts = w.series[0], w.tsamp
    n = x.size
    cfg = oracle.config(n, ts)
    x0 = oracle.mean_subtract(x)
    _say("full size: 2^23, 64 templates")
    with tb.Plan() as plan:
        sid = plan.load_series(x, ts)
        cg = plan.search(sid, w.templates)
        tm0 = tuple(float(v) for v in w.templates[0])
        g = plan.inspect(sid, tm0)
    st = oracle.template_stages(x0, cfg, tm0)
    _, delta = oracle.resample_index(tm0, n, ts)
    ex = R.check_indices(g["src"], st["src"], delta)
    R.check_power(g["power"], st["p"], st["med"], 4096)
    R.check_medians(g["medians"], st["med"])
    R.check_sums(g["sums"], st["s"])
    co = oracle.search(x0, cfg, w.templates, series_id=int(sid))
    matched, exempt = R.check_candidates(cg, co, [oracle.threshold(1 << l, 6.0) for l in range(5)])
    _say("  tie-exempt %d, candidates matched %d exempt %d" % (ex, matched, exempt))
    assert matched > 0


def test_grouping_of_gpu_candidates(tb):
    """The C1 candidate list from the GPU, grouped by the library and by the
    oracle: identical kept records and group sizes; the strongest detection
    heads the first group and every candidate is in one group."""
    w = synth.c1_tiny()
    x, ts = w.series[0], w.tsamp
    with tb.Plan(threshold_sigma=4.0) as plan:
        sid = plan.load_series(x, ts)
        cg = plan.search(sid, w.templates)
    assert len(cg) > 100
    o = np.zeros(cg.size, dtype=oracle.CANDIDATE_DTYPE)
    for f in ("series_id", "template_id", "bin", "log2_harm", "power", "sigma", "freq_hz"):
        o[f] = cg[f]
    for kw in (dict(), dict(ppm=1000), dict(max_ratio=1, tol=0)):
        kept, grp = tb.tb_distill(cg, **kw)
        ko, go = oracle.distill(o, **kw)
        ok = np.zeros(kept.size, dtype=oracle.CANDIDATE_DTYPE)
        for f in ("series_id", "template_id", "bin", "log2_harm", "power", "sigma", "freq_hz"):
            ok[f] = kept[f]
        assert np.array_equal(ok, ko) and np.array_equal(grp.astype(np.int64), go), kw
        assert kept[0]["sigma"] == cg["sigma"].max() and int(grp.sum()) == len(cg)
    _say("grouping: %d candidates -> %d groups (ppm 1000)" % (len(cg), len(tb.tb_distill(cg, ppm=1000)[0])))
