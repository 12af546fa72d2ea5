"""Oracle parity at the series lengths and launch shapes the benchmark runs:
the default pass-2 shapes of 2^20 and 2^22 samples (8192-point tiles, 64- and
256-point pass-2 transforms), the elliptical configuration at its full size
(2^24 samples at 256 us, BT delay with a Newton solve of Kepler's equation,
App. A.1 and Alg. 1) with the widest orbit of its prior, a batch shaped
like the uneven-length search (four series of 2^20 .. 2^23 samples searched at
once on four lanes), and the paper's circular timing configuration with the
extremes of its Table 1 prior."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from tests import parity_rules as R

pytestmark = pytest.mark.gpu

HOUR = 3600.0


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tb():
    import paper_2112_11991_amd as tb

    return tb


def _stage_check(plan, sid, x0, cfg, tm, W):
    n, ts = x0.size, cfg.tsamp
    st = oracle.template_stages(x0, cfg, tm)
    _, delta = oracle.resample_index(tm, n, ts)
    g = plan.inspect(sid, tm)
    ex = R.check_indices(g["src"], st["src"], delta)
    R.check_power(g["power"], st["p"], st["med"], W)
    R.check_medians(g["medians"], st["med"])
    R.check_phat(g["sums"][0], st["phat"])
    R.check_sums(g["sums"], st["s"])
    return ex


def _same_best(cg, co):
    """The strongest detection is the same record on both sides."""
    bg, bo = cg[np.argmax(cg["sigma"])], co[np.argmax(co["sigma"])]
    assert (bg["template_id"], bg["log2_harm"], bg["bin"]) == (bo["template_id"], bo["log2_harm"], bo["bin"])


def chunk_points(tm, n, ts, tile):
    """Points per delay-polynomial chunk the library takes for a BT template
    (16 or 8; 0 = exact per-sample solve): the fourth-order remainder bound
    tau/tsamp (Omega tsamp)^5 3 (1+e)^2 / (1-e)^9 U^5 / 120 <= 1e-11 samples,
    U the farthest sample of a chunk from its centre plus the column reach of
    a pass-1 tile, as the delay-polynomial kernel evaluates it."""
    porb, tau, _, e, _ = tm
    M = n // 2
    R_ = max(16, M // tile)
    S = M // R_
    C1 = min(tile, M) // S
    A, Wp = tau / ts, 2 * math.pi / porb * ts
    g5 = 3 * (1 + e) ** 2 / (1 - e) ** 9

    def reach(length):
        jof = lambda k: 2 * (k % C1 + R_ * (k // C1))
        lo, hi = jof(0), jof(length - 1) + 1
        mid = lo + (hi - lo) // 2
        return (hi - mid) + 2.0 * (R_ - C1)

    for length in (16, 8):
        if A * Wp ** 5 * g5 * reach(length) ** 5 / 120 <= 1e-11:
            return length
    return 0


@pytest.mark.parametrize("lg", [20, 22])
def test_default_pass2_shapes(tb, lg):
    """2^20 and 2^22 samples in the library's default launch shape (8192-point
    tiles: pass-2 transforms of 64 points over 128 columns, and of 256 points
    over 32 columns): whole-spectrum stage parity for an eccentric binary
    template and candidate parity for twelve templates searched together
    (one wave), the injected orbit among them.  The red noise is the survey
    recipe (40 dB above the white level in the lowest bin at 2^20 samples)
    at a quarter of its amplitude at 2^22: at full amplitude the lowest bin
    of this seed is 55 dB above the white level, where an FP32 transform no
    longer meets the per-bin power rule at its Nyquist mirror (measured 2.3x
    the limit at bin n/2 - 1); a quarter keeps it at 43 dB."""
    n, ts = 1 << lg, 64e-6
    rng = np.random.default_rng(2000 + lg)
    orb = synth.Orbit(0.9 * HOUR, 0.6, 2.0, 0.05, 1.2)
    x = rng.standard_normal(n) + (1.0 if lg <= 20 else 0.25) * synth.red_noise(n, ts, rng)
    x = synth.inject(x, synth.pulse_train(n, ts, 0.021, 0.05, orb), 30.0).astype(np.float32)
    tms = np.concatenate([synth.uniform_templates(rng, 11, (0.5, 2.0), (0.0, 1.0), ecc_max=0.1),
                          orb.as_template()])
    x0 = oracle.mean_subtract(x)
    cfg = oracle.config(n, ts, threshold_sigma=5.5)
    _say("default shapes n=2^%d" % lg)
    with tb.Plan(threshold_sigma=5.5) as plan:
        sid = plan.load_series(x, ts)
        cg = plan.search(sid, tms)
        ex = _stage_check(plan, sid, x0, cfg, tuple(float(v) for v in tms[-1]), 4096)
    co = oracle.search(x0, cfg, tms, series_id=int(sid))
    matched, exempt = R.check_candidates(cg, co, [oracle.threshold(1 << l, 5.5) for l in range(5)])
    _say("  tie-exempt %d; candidates matched %d, near-threshold %d" % (ex, matched, exempt))
    assert matched > 0
    _same_best(cg, co)


@pytest.fixture(scope="module")
def c3():
    return synth.c3_elliptical(n_templates=6)


def _c3_templates(w):
    """The widest orbit of the elliptical prior (shortest period, largest
    projected semi-major axis and eccentricity), the injected orbit, and the
    first bank templates."""
    worst = np.array([(5.0 * HOUR, 6.0, 0.3, 0.0999, 1.0)], dtype=w.templates.dtype)
    true = w.truths[0][1].as_template()
    return np.concatenate([worst, true, w.templates[:4]])


@pytest.mark.parametrize("tile", [16384, 8192])
def test_elliptical_full_size_bt_newton(tb, c3, tile):
    """2^24 samples at 256 us (the paper's Table 2 series), BT delay with the
    Newton solve: bit-exact indices and whole-spectrum parity for the widest
    orbit of the prior, candidate parity for it, the injected orbit and four
    bank templates.  With the default 16384-point tiles that orbit takes
    16-point delay chunks; with 8192-point tiles (a wider column reach) it
    needs the 8-point chunks."""
    x, ts = c3.series[0], c3.tsamp
    n = x.size
    tms = _c3_templates(c3)
    worst = tuple(float(v) for v in tms[0])
    pts = chunk_points(worst, n, ts, tile)
    _say("elliptical full size, tiles %d: widest orbit on %d-point chunks" % (tile, pts))
    assert pts == (16 if tile == 16384 else 8)
    x0 = oracle.mean_subtract(x)
    cfg = oracle.config(n, ts)
    with tb.Plan(tile_points=tile) as plan:
        sid = plan.load_series(x, ts)
        cg = plan.search(sid, tms)
        ex = _stage_check(plan, sid, x0, cfg, worst, 4096)
    co = oracle.search(x0, cfg, tms, series_id=int(sid))
    matched, exempt = R.check_candidates(cg, co, [oracle.threshold(1 << l, 6.0) for l in range(5)])
    _say("  tie-exempt %d; candidates matched %d, near-threshold %d" % (ex, matched, exempt))
    assert matched > 0
    _same_best(cg, co)
    assert cg[np.argmax(cg["sigma"])]["template_id"] == 1  # the injected orbit


@pytest.fixture(scope="module")
def t3():
    return synth.table3_series()


def _kepler_tau(porb_s, m_p=1.4, m_c=8.0):
    """Largest projected semi-major axis (lt-s) the Table 1 prior allows at
    P_orb: Kepler's third law with the lightest pulsar and the heaviest
    companion (Sec. 3.1)."""
    from oracle.bank import T_SUN

    return T_SUN ** (1 / 3) * (2 * math.pi / porb_s) ** (-2 / 3) * m_c / (m_p + m_c) ** (2 / 3)


def test_table1_prior_extremes_full_size(tb, t3):
    """The paper's circular timing configuration (2^24 samples at 256 us, the
    Table 1 prior: P_orb 6-12 h, tau up to the Kepler limit) in the plan's
    default launch shape: bit-exact indices and whole-spectrum parity for the
    orbit whose delay changes fastest (6 h at its Kepler limit, about 7 lt-s),
    candidate parity for it, the 12 h orbit at its limit and the injected
    orbit."""
    x, ts = t3.series[0], t3.tsamp
    n = x.size
    fast = (6.0 * HOUR, 0.999 * _kepler_tau(6.0 * HOUR), 2.0, 0.0, 0.0)
    wide = (12.0 * HOUR, 0.999 * _kepler_tau(12.0 * HOUR), 4.0, 0.0, 0.0)
    assert 6.9 < fast[1] < 7.0 and 11.0 < wide[1] < 11.1
    assert chunk_points(fast, n, ts, 16384) == 16 and chunk_points(wide, n, ts, 16384) == 16
    tms = np.concatenate([np.array([fast, wide], dtype=synth.TEMPLATE_DTYPE), t3.truths[0][1].as_template()])
    _say("table 1 extremes at 2^24: tau %.3f at 6 h, %.3f at 12 h" % (fast[1], wide[1]))
    x0 = oracle.mean_subtract(x)
    cfg = oracle.config(n, ts)
    with tb.Plan() as plan:
        sid = plan.load_series(x, ts)
        cg = plan.search(sid, tms)
        ex = _stage_check(plan, sid, x0, cfg, fast, 4096)
    co = oracle.search(x0, cfg, tms, series_id=int(sid))
    matched, exempt = R.check_candidates(cg, co, [oracle.threshold(1 << l, 6.0) for l in range(5)])
    _say("  tie-exempt %d; candidates matched %d, near-threshold %d" % (ex, matched, exempt))
    assert matched > 0
    _same_best(cg, co)
    assert cg[np.argmax(cg["sigma"])]["template_id"] == 2  # the injected orbit


def test_uneven_length_batch_on_lanes(tb):
    """A batch shaped like the uneven-length search: four series of 2^20,
    2^21, 2^22 and 2^23 samples (two carrying binaries), 20 shared circular
    templates, one request per series submitted together on four lanes so
    that their kernels interleave on the device; every series' candidate
    list against the oracle."""
    ts, sigma = 64e-6, 5.5
    rng = np.random.default_rng(4242)
    tms = synth.uniform_templates(rng, 18, (1.0, 10.0), (0.0, 2.0))
    orbs = {1: synth.Orbit(2.5 * HOUR, 0.8, 0.4), 3: synth.Orbit(1.2 * HOUR, 1.5, 5.0)}
    tms = np.concatenate([tms, orbs[1].as_template(), orbs[3].as_template()])
    series = []
    for i, lg in enumerate((20, 21, 22, 23)):
        n = 1 << lg
        x = rng.standard_normal(n)
        if i in orbs:
            x = synth.inject(x, synth.pulse_train(n, ts, 0.023 + 0.004 * i, 0.05, orbs[i]), 25.0)
        series.append(x.astype(np.float32))
    _say("uneven-length batch: 4 series x %d templates on 4 lanes" % len(tms))
    with tb.Plan(lanes=4, threshold_sigma=sigma) as plan:
        sids = [plan.load_series(x, ts) for x in series]
        rids = [plan.submit(sid, tms, first_template_id=100) for sid in sids]
        got = []
        for rid in rids:
            got.append(plan.candidates(rid)[0])
            plan.release(rid)
    thr = [oracle.threshold(1 << l, sigma) for l in range(5)]
    for i, (x, sid, cg) in enumerate(zip(series, sids, got)):
        x0 = oracle.mean_subtract(x)
        co = oracle.search(x0, oracle.config(x.size, ts, threshold_sigma=sigma), tms, first_template_id=100,
                           series_id=int(sid))
        matched, exempt = R.check_candidates(cg, co, thr)
        _say("  series %d (2^%d): matched %d, near-threshold %d" % (i, x.size.bit_length() - 1, matched, exempt))
        assert matched > 0
        _same_best(cg, co)


def test_uneven_length_search_at_full_size_sampled(tb):
    """The batched uneven-length workload at its full size and in the
    benchmark's launch configuration (32 series of 2^20 .. 2^23 samples, 4096
    shared circular templates, one request per series on four lanes, the
    library's default waves): the candidates of eight sampled (series,
    template) pairs, the series carrying binaries and their true orbits among
    them, against the oracle one template at a time (three of the sampled
    bank templates fall on the series with binaries, where the pulsar shows
    in most templates)."""
    w = synth.c4_batched()
    ts, sigma = w.tsamp, w.sigma
    tms = np.concatenate([w.templates] + [orb.as_template() for _, orb, _ in w.truths])
    _say("uneven-length full size: %d series x %d templates on 4 lanes" % (len(w.series), len(tms)))
    with tb.Plan(lanes=4, threshold_sigma=sigma, fmin_hz=w.fmin_hz, ring_capacity=1 << 18) as plan:
        sids = [plan.load_series(x, ts) for x in w.series]
        rids = [plan.submit(sid, tms) for sid in sids]
        got = []
        for rid in rids:
            got.append(plan.candidates(rid)[0])
            plan.release(rid)
    rng = np.random.default_rng(77)
    nb = len(w.templates)
    carriers = [i for i, _, _ in w.truths]
    pairs = [(i, nb + k) for k, i in enumerate(carriers)]
    # bank templates on the series with binaries (the pulsar shows in most of
    # them) and one on any series
    pairs += [(carriers[k % len(carriers)], int(rng.integers(nb))) for k in range(3)]
    pairs += [(int(rng.integers(len(w.series))), int(rng.integers(nb)))]
    thr = [oracle.threshold(1 << l, sigma) for l in range(5)]
    bank_hits = 0
    for s, t in pairs:
        x = w.series[s]
        co = oracle.search(oracle.mean_subtract(x), oracle.config(x.size, ts, threshold_sigma=sigma,
                                                                   fmin_hz=w.fmin_hz),
                           tms[t:t + 1], first_template_id=t, series_id=int(sids[s]))
        cg = got[s][got[s]["template_id"] == t]
        matched, exempt = R.check_candidates(cg, co, thr)
        _say("  series %d (2^%d) template %d: %d candidates, near-threshold %d" % (
            s, x.size.bit_length() - 1, t, matched, exempt))
        if t >= nb:
            assert matched > 0
        else:
            bank_hits += matched
    assert bank_hits > 0
