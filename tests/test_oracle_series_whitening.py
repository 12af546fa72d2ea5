"""Pins of the oracle's once-per-series whitening (the de-reddening taken from
the spectrum of the series itself and applied to every template searched on
it; the paper lists Fourier de-reddening among the per-series steps of its
pipeline, App. A, Sec. 5.2).

Each pin compares against a closed form, a library computation or an
invariant that a slip in the oracle would break: an impulse has a flat unit
spectrum, a template with no orbit must reproduce per-template whitening, and
the applied levels may not depend on the template."""
import math

import numpy as np

import oracle
import synth

N, TS, W = 1 << 14, 64e-6, 1000  # 9 blocks, the last one ragged
ORBITS = [(0.9, 0.4, 1.3, 0.0, 0.0), (0.6, 0.25, 4.0, 0.3, 2.0)]  # 1e3..4e3 samples of delay swing


def _red():
    rng = np.random.default_rng(21)
    x = synth.red_noise(N, TS, rng, f_knee=400.0) + rng.standard_normal(N)
    return oracle.mean_subtract(x.astype(np.float32))


def test_series_levels_of_an_impulse_are_flat(oracle_lib):
    """x = delta_0 has X_k = 1 for every k: every block median and level is 1,
    so any template's whitened power is exactly its raw power times ln 2."""
    x0 = np.zeros(N, dtype=np.float32)
    x0[0] = 1.0
    cfg = oracle.config(N, TS, whiten_window=W, series_whitening=True)
    med, lev = oracle.series_levels(x0, cfg)
    assert med.size == 9 and np.all(med == 1.0)
    assert lev[0] == 0.0 and np.all(lev[1:] == 1.0)
    for tm in ORBITS:
        st = oracle.template_stages(x0, cfg, tm)
        assert st["phat"][0] == 0.0
        assert np.array_equal(st["phat"][1:], st["p"][1:] * math.log(2))
        assert np.array_equal(st["med"], med)


def test_series_levels_of_a_silent_series_are_zero(oracle_lib):
    """An all-zero series has zero power, zero medians and zero level in every
    bin: the guard for a non-positive level gives P^ = 0, not 0/0."""
    x0 = np.zeros(N, dtype=np.float32)
    cfg = oracle.config(N, TS, whiten_window=W, series_whitening=True)
    med, lev = oracle.series_levels(x0, cfg)
    assert np.all(med == 0.0) and np.all(lev == 0.0)
    phat = oracle.template_stages(x0, cfg, ORBITS[0])["phat"]
    assert np.all(phat == 0.0)


def test_series_medians_against_library_spectrum(oracle_lib):
    """The series medians are the lower block medians of |rfft(x0)|^2 computed
    by numpy (rounding differences only)."""
    x0 = _red()
    cfg = oracle.config(N, TS, whiten_window=W, series_whitening=True)
    med, _ = oracle.series_levels(x0, cfg)
    p = np.abs(np.fft.rfft(x0.astype(np.float64))) ** 2
    m = N // 2
    for b in range(med.size):
        blk = p[1 + b * W: 1 + min(m, (b + 1) * W)]
        want = np.partition(blk, (blk.size - 1) // 2)[(blk.size - 1) // 2]
        assert abs(med[b] - want) <= 1e-9 * want


def test_zero_orbit_matches_per_template_whitening(oracle_lib):
    """With tau = 0 the template reads the series as loaded, so its own block
    medians are the series medians: both modes give identical outputs."""
    x0 = _red()
    a = oracle.template_stages(x0, oracle.config(N, TS, whiten_window=W), (3600.0, 0.0, 1.0, 0.0, 0.0))
    b = oracle.template_stages(x0, oracle.config(N, TS, whiten_window=W, series_whitening=True),
                               (3600.0, 0.0, 1.0, 0.0, 0.0))
    for key in ("p", "med", "phat", "s"):
        assert np.array_equal(a[key], b[key]), key


def test_levels_do_not_depend_on_the_template(oracle_lib):
    """Series mode: P^_k / P_k = ln2 / m(k) with the series level m for every
    template; per-template mode gives each orbit its own levels."""
    x0 = _red()
    cfg = oracle.config(N, TS, whiten_window=W, series_whitening=True)
    _, lev = oracle.series_levels(x0, cfg)
    ratios, own = [], []
    for tm in ORBITS:
        st = oracle.template_stages(x0, cfg, tm)
        k = np.arange(1, N // 2 + 1)
        k = k[st["p"][k] > 0]
        assert np.allclose(st["phat"][k] / st["p"][k], math.log(2) / lev[k], rtol=1e-14, atol=0)
        ratios.append(st["phat"][k] / st["p"][k])
        o = oracle.template_stages(x0, oracle.config(N, TS, whiten_window=W), tm)
        own.append(o["med"])
    assert np.allclose(ratios[0][:100], ratios[1][:100], rtol=1e-14)
    assert not np.array_equal(own[0], own[1])


def test_series_search_thresholds_the_series_whitened_sums(oracle_lib):
    """The multi-threaded search in series mode reports exactly the bins whose
    series-whitened harmonic sums pass the fold thresholds."""
    x0 = _red()
    cfg = oracle.config(N, TS, whiten_window=W, threshold_sigma=3.0, series_whitening=True)
    cands = oracle.search(x0, cfg, ORBITS, nthreads=2)
    T = N * TS
    kmin = max(1, math.ceil(cfg.fmin_hz * T))
    for ti, tm in enumerate(ORBITS):
        s = oracle.template_stages(x0, cfg, tm)["s"]
        got = cands[cands["template_id"] == ti]
        want = []
        for l in range(5):
            h = 1 << l
            thr = oracle.threshold(h, 3.0)
            ks = np.nonzero(s[l] > thr)[0]
            want += [(l, int(k)) for k in ks if k >= h * kmin]
        assert sorted(want) == [(int(c["log2_harm"]), int(c["bin"])) for c in got]
        assert len(want) > 0
