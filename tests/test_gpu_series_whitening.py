"""Parity of the once-per-series whitening (series loaded with
TB_SERIES_WHITENING: levels from the series' own spectrum, applied by pass 2
to every template) with the oracle's series mode, through the C ABI."""
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


def _series(n, ts, seed, orbit=None, pspin=0.02, snr=20.0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n) + synth.red_noise(n, ts, rng)
    if orbit is not None:
        x = synth.inject(x, synth.pulse_train(n, ts, pspin, 0.05, orbit), snr)
    return x.astype(np.float32)


def _stage_check(plan, sid, x, n, ts, tm, W, harm=16):
    cfg = oracle.config(n, ts, harm_max=harm, whiten_window=W, series_whitening=True)
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
    # (log2 n, tsamp, W, template, tile points)
    (10, 64e-6, 64, (30.0, 0.01, 0.3, 0.0, 0.0), 0),
    (13, 64e-6, 1000, (100.0, 0.05, 2.0, 0.0, 0.0), 0),
    (15, 256e-6, 3000, (900.0, 0.8, 1.0, 0.3, 2.5), 0),
    (17, 64e-6, 4096, (7200.0, 0.5, 1.0, 0.0, 0.0), 16384),
    (18, 64e-6, 4096, (1800.0, 1.5, 5.5, 0.1, 0.7), 0),
    (20, 64e-6, 2048, (3000.0, 2.0, 0.1, 0.0, 0.0), 16384),
    (21, 64e-6, 4096, (380.0, 1.5, 2.0, 0.05, 1.0), 0),
]


@pytest.mark.parametrize("lg,ts,W,tm,tile", CASES)
def test_series_whitened_stages_match_oracle(tb, lg, ts, W, tm, tile):
    n = 1 << lg
    _say("series-whitened stages n=2^%d W=%d tile=%d tm=%s" % (lg, W, tile, tm))
    x = _series(n, ts, seed=200 + lg, orbit=synth.Orbit(*tm), pspin=0.013)
    with tb.Plan(whiten_window=W, tile_points=tile) as plan:
        sid = plan.load_series(x, ts, flags=tb.TB_MEM_HOST | tb.TB_SERIES_WHITENING)
        ex = _stage_check(plan, sid, x, n, ts, tm, W)
        _say("  tie-exempt indices:", ex)


def test_zero_orbit_equals_per_template_whitening_bitwise(tb):
    """With tau = 0 the series levels are the template's own: the factor
    applied in pass 2 is the float the per-template whitening multiplies by,
    so sums and candidates agree bit for bit."""
    n, ts = 1 << 18, 64e-6
    x = _series(n, ts, seed=31, orbit=synth.Orbit(3600.0, 0.3, 1.0), pspin=0.011)
    still = [(3600.0, 0.0, 1.0, 0.0, 0.0), (500.0, 0.0, 4.0, 0.4, 1.0)]
    with tb.Plan(whiten_window=4096, threshold_sigma=4.0) as plan:
        a = plan.load_series(x, ts)
        b = plan.load_series(x, ts, flags=tb.TB_SERIES_WHITENING)
        ga = plan.inspect(a, still[0])
        gb = plan.inspect(b, still[0])
        ca = plan.search(a, still)
        cb = plan.search(b, still)
    for k in ("src", "power", "medians", "sums"):
        assert np.array_equal(ga[k], gb[k]), k
    keys = ["template_id", "bin", "log2_harm", "power", "sigma", "freq_hz"]
    assert len(ca) > 0 and np.array_equal(ca[keys], cb[keys])
    assert np.all(ca["series_id"] == a) and np.all(cb["series_id"] == b)


def test_series_whitened_candidates_match_oracle(tb):
    """The tiny configuration (2^17 samples, 65 circular templates) searched
    on a series whitened once, on one lane and spread over three; per-kernel
    profile shows no median or whitening launches."""
    w = synth.c1_tiny()
    x, ts = w.series[0], w.tsamp
    n = x.size
    with tb.Plan(batch_templates=16) as plan:
        sid = plan.load_series(x, ts, flags=tb.TB_SERIES_WHITENING)
        plan.profile(1)
        cg = plan.search(sid, w.templates, first_template_id=500)
        ms, launches, ntemp = plan.profile_read()
        plan.profile(0)
    with tb.Plan(batch_templates=16, lanes=3) as plan:
        sid3 = plan.load_series(x, ts, flags=tb.TB_SERIES_WHITENING)
        c3 = plan.search(sid3, w.templates, first_template_id=500)
    assert sid3 == sid and np.array_equal(cg, c3)
    assert list(launches[3:5]) == [0, 0] and min(launches[0:3]) > 0 and launches[5] == 5 and ntemp == 65
    co = oracle.search(oracle.mean_subtract(x), oracle.config(n, ts, series_whitening=True), w.templates,
                       first_template_id=500, series_id=int(sid))
    matched, exempt = R.check_candidates(cg, co, [oracle.threshold(1 << l, 6.0) for l in range(5)])
    _say("series-whitened c1: matched %d exempt %d" % (matched, exempt))
    assert matched > 0


def test_series_whitening_memory(tb):
    """The series holds its factors and medians on top of the samples: after
    one search on each, the two plans differ by exactly that."""
    n, ts = 1 << 16, 64e-6
    x = _series(n, ts, seed=33)
    held = []
    for flags in (tb.TB_MEM_HOST, tb.TB_SERIES_WHITENING):
        with tb.Plan(whiten_window=1000) as plan:
            sid = plan.load_series(x, ts, flags=flags)
            plan.search(sid, [(600.0, 0.1, 0.0, 0.0, 0.0)])
            held.append(plan.memory()[0])
    m = n // 2
    nblk = (m + 999) // 1000
    assert held[1] - held[0] == 4 * (((m + 1 + 63) // 64) * 64 + nblk)


def test_full_size_series_whitened(tb):
    """2^23 samples with red noise and a pulsar, 8 templates in flight, series
    whitened once: whole-spectrum parity of one template, candidate parity for
    three of 17 (one of them the injected orbit)."""
    wl = synth.c2_survey(n_templates=16)
    x, ts = wl.series[0], wl.tsamp
    n = x.size
    bank = np.concatenate([wl.templates, wl.truths[0][1].as_template()])
    cfg = oracle.config(n, ts, series_whitening=True)
    x0 = oracle.mean_subtract(x)
    _say("full size series-whitened: 2^23, 17 templates")
    with tb.Plan(batch_templates=8) as plan:
        sid = plan.load_series(x, ts, flags=tb.TB_SERIES_WHITENING)
        cg = plan.search(sid, bank)
        tm0 = tuple(float(v) for v in bank[0])
        ex = _stage_check(plan, sid, x, n, ts, tm0, 4096)
    pick = [0, 7, 16]
    co = oracle.search(x0, cfg, bank[pick], series_id=int(sid))
    co["template_id"] = np.array(pick, dtype=np.uint32)[co["template_id"]]
    sub = cg[np.isin(cg["template_id"], pick)]
    matched, exempt = R.check_candidates(sub, co, [oracle.threshold(1 << l, 6.0) for l in range(5)])
    _say("  tie-exempt %d, candidates matched %d exempt %d" % (ex, matched, exempt))
    assert matched > 0


def test_series_whitening_flags(tb):
    """Unknown load flags are rejected; a device-resident series whitened once
    gives the host-loaded one's candidates."""
    import torch

    n, ts = 1 << 15, 64e-6
    x = _series(n, ts, seed=34, orbit=synth.Orbit(800.0, 0.3, 1.0), pspin=0.01)
    tm = [(800.0, 0.3, 1.0, 0.0, 0.0)]
    with tb.Plan() as plan:
        for bad in (4, 6, 1 << 31):
            with pytest.raises(tb.TbError) as e:
                plan.load_series(x, ts, flags=bad)
            assert e.value.status == tb.TB_ERR_INVALID_ARG
        xd = torch.from_numpy(x).to("cuda:0")
        torch.cuda.synchronize()
        s_host = plan.load_series(x, ts, flags=tb.TB_SERIES_WHITENING)
        s_dev = plan.load_series(xd.data_ptr(), ts, n=n, flags=tb.TB_MEM_DEVICE | tb.TB_SERIES_WHITENING)
        a = plan.search(s_host, tm)
        b = plan.search(s_dev, tm)
    assert len(a) > 0
    assert np.array_equal(a[["template_id", "bin", "log2_harm", "power"]], b[["template_id", "bin", "log2_harm", "power"]])
