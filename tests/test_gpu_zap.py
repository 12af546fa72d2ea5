"""Parity of birdie zapping (tb_zap_series: bins with lo <= k/T <= hi get a
zero whitened power before the harmonic sum) with the oracle, per-template
and once-per-series whitening, through the C ABI."""
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


def _zaps(T, M):
    f = lambda k: k / T
    return [
        (f(1), f(3)),                      # the first bins
        (f(990.5), f(1010.2)),             # across a block boundary (W = 1000), ends between bins
        (f(2000), f(2000)),                # one bin, ends exactly on it
        (f(1500), f(1600)), (f(1550), f(1700)),  # overlapping, unsorted below
        (f(M - 2), f(M) + 5.0),            # up to and past Nyquist
        (f(300), f(200)),                  # empty
        (f(700), f(705)),
    ]


@pytest.mark.parametrize("lg,ts,series_mode", [(14, 64e-6, False), (14, 64e-6, True), (18, 2.0 ** -12, False),
                                               (18, 2.0 ** -12, True)])
def test_zapped_stages_match_oracle(tb, lg, ts, series_mode):
    n = 1 << lg
    T, M = n * ts, n // 2
    zap = _zaps(T, M)
    zap = zap[4:] + zap[:4]
    tm = (1800.0, 0.4, 1.0, 0.1, 0.7)
    rng = np.random.default_rng(lg)
    x = (rng.standard_normal(n) + synth.red_noise(n, ts, rng)).astype(np.float32)
    cfg = oracle.config(n, ts, whiten_window=1000, zap=zap, series_whitening=series_mode)
    st = oracle.template_stages(oracle.mean_subtract(x), cfg, tm)
    _say("zap stages n=2^%d series=%s" % (lg, series_mode))
    with tb.Plan(whiten_window=1000) as plan:
        sid = plan.load_series(x, ts, flags=tb.TB_SERIES_WHITENING if series_mode else tb.TB_MEM_HOST)
        plan.zap(sid, zap)
        g = plan.inspect(sid, tm)
    _, delta = oracle.resample_index(tm, n, ts)
    R.check_indices(g["src"], st["src"], delta)
    R.check_power(g["power"], st["p"], st["med"], 1000)
    R.check_medians(g["medians"], st["med"])
    R.check_phat(g["sums"][0], st["phat"])
    R.check_sums(g["sums"], st["s"])
    zeroed = np.flatnonzero(st["phat"][1:] == 0.0) + 1
    assert zeroed.size > 100 and np.all(g["sums"][0][zeroed] == 0.0)


@pytest.mark.parametrize("series_mode", [False, True])
def test_clearing_restores_the_unzapped_search(tb, series_mode):
    """Zap, search, clear, search: the cleared search equals a plan that never
    zapped, bit for bit; replacing the list replaces it."""
    n, ts = 1 << 16, 64e-6
    T = n * ts
    rng = np.random.default_rng(7)
    x = (rng.standard_normal(n) + synth.red_noise(n, ts, rng)).astype(np.float32)
    tms = [(900.0, 0.2, 1.0, 0.0, 0.0), (1500.0, 0.1, 3.0, 0.05, 1.0)]
    flags = tb.TB_SERIES_WHITENING if series_mode else tb.TB_MEM_HOST
    keys = ["template_id", "bin", "log2_harm", "power", "sigma", "freq_hz"]
    with tb.Plan(threshold_sigma=3.0) as plan:
        sid = plan.load_series(x, ts, flags=flags)
        ref = plan.search(sid, tms)
        plan.zap(sid, [(0.0, 2000.0 / T)])  # bins 1..2000
        a = plan.search(sid, tms)
        plan.zap(sid, [(10.0, 20.0)])
        b = plan.search(sid, tms)
        plan.zap(sid, [])
        c = plan.search(sid, tms)
    assert len(ref) > 0 and np.array_equal(c[keys], ref[keys])
    # with bins 1..2000 zapped, no fold-1 candidate remains there
    one = a[a["log2_harm"] == 0]
    assert np.all(one["bin"] > 2000)
    assert not np.array_equal(a[keys], ref[keys]) and not np.array_equal(b[keys], ref[keys])


def test_zapped_interferer_candidates_match_oracle(tb):
    """A 50 Hz interferer with harmonics and a pulsar; zapping the interferer's
    lines: GPU and oracle candidate lists agree, and the pulsar is the best
    candidate of the template without orbit."""
    n, ts = 1 << 17, 2.0 ** -10
    t = np.arange(n) * ts
    rng = np.random.default_rng(5)
    k0 = 2861
    x = synth.inject(rng.standard_normal(n), synth.pulse_train(n, ts, n * ts / k0, 0.05, None), 25.0)
    x += sum(0.3 / m * np.cos(2 * np.pi * 50.0 * m * t) for m in range(1, 8))
    x = x.astype(np.float32)
    zap = [(50.0 * m - 0.05, 50.0 * m + 0.05) for m in range(1, 11)]
    tms = [(3600.0, 0.0, 0.0, 0.0, 0.0), (900.0, 0.1, 2.0, 0.0, 0.0)]
    with tb.Plan() as plan:
        sid = plan.load_series(x, ts)
        plan.zap(sid, zap)
        cg = plan.search(sid, tms)
    co = oracle.search(oracle.mean_subtract(x), oracle.config(n, ts, zap=zap), tms, series_id=int(sid))
    matched, exempt = R.check_candidates(cg, co, [oracle.threshold(1 << l, 6.0) for l in range(5)])
    assert matched > 0
    # the template without orbit sees the interferer's lines unsmeared, so
    # zapping removes them there and the pulsar is its best candidate
    c0 = cg[cg["template_id"] == 0]
    best = c0[np.argmax(c0["sigma"])]
    assert best["bin"] == 16 * k0 and best["log2_harm"] == 4


def test_zap_argument_errors(tb):
    n, ts = 1 << 12, 64e-6
    x = np.random.default_rng(1).standard_normal(n).astype(np.float32)
    with tb.Plan() as plan:
        sid = plan.load_series(x, ts)
        for bad in ([(float("nan"), 1.0)], [(1.0, float("inf"))]):
            with pytest.raises(tb.TbError) as e:
                plan.zap(sid, bad)
            assert e.value.status == tb.TB_ERR_INVALID_ARG
        with pytest.raises(tb.TbError) as e:
            plan.zap(sid + 5, [(1.0, 2.0)])
        assert e.value.status == tb.TB_ERR_UNKNOWN_ID
        with pytest.raises(tb.TbError) as e:
            plan.zap(sid, np.zeros((tb.TB_ZAP_MAX + 1, 2)))
        assert e.value.status == tb.TB_ERR_INVALID_ARG
        held0 = plan.memory()[0]
        T = n * ts
        plan.zap(sid, [(10 / T, 20 / T), (30 / T, 40 / T), (35 / T, 50 / T)])  # two bin ranges after merging
        assert plan.memory()[0] == held0 + 16
        plan.zap(sid, [])
        assert plan.memory()[0] == held0
