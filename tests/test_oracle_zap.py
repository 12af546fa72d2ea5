"""Pins of the oracle's birdie zapping (App. A / Sec. 5.2 list Fourier birdie
zapping among the per-series steps; the rule is this project's: whitened
powers of bins with lo <= k/T <= hi are zeroed before the harmonic sum).

With T = 2^14 * 2^-10 s = 16 s exactly, interval ends k/16 are exact, so the
bins expected inside are known without rounding; the rest of each spectrum
must be untouched, the fold sums must be those of the zapped spectrum, and a
strong periodic interferer that floods the candidate list disappears from it
when its lines are zapped while a pulsar is still found."""
import math

import numpy as np

import oracle
import synth

N, TS = 1 << 14, 2.0 ** -10
T = N * TS  # 16 s
TM = (300.0, 0.05, 1.0, 0.1, 2.0)


def _x(seed=3):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(N) + synth.red_noise(N, TS, rng, f_knee=5.0)
    return oracle.mean_subtract(x.astype(np.float32))


def _inside(zap):
    ks = set()
    for lo, hi in zap:
        for k in range(1, N // 2 + 1):
            if lo * T <= k <= hi * T:
                ks.add(k)
    return np.array(sorted(ks), dtype=np.int64)


def test_zapped_bins_are_zero_and_the_rest_untouched(oracle_lib):
    zap = [(10.0, 12.0),              # bins 160..192, ends exactly on bins
           (100.5 / 16, 101.5 / 16),   # 6.28..6.34 Hz: bin 101 only (ends between bins)
           (20.0, 20.0),               # a single bin, 320
           (11.5, 13.0),               # overlaps the first
           (0.0, 0.01),                # below the first bin: only k >= 1 counts, k = 0 unaffected
           (511.99, 600.0),            # up to and past Nyquist (512 Hz, bin 8192)
           (50.0, 40.0)]               # empty (lo > hi)
    x0 = _x()
    a = oracle.template_stages(x0, oracle.config(N, TS, whiten_window=1000), TM)
    b = oracle.template_stages(x0, oracle.config(N, TS, whiten_window=1000, zap=zap), TM)
    ks = _inside(zap)
    assert 101 in ks and 320 in ks and 160 in ks and 192 in ks and 193 in ks and 208 in ks and 209 not in ks
    assert 8192 in ks and 8191 not in ks and 0 not in ks
    keep = np.setdiff1d(np.arange(N // 2 + 1), ks)
    assert np.all(b["phat"][ks] == 0.0)
    assert np.array_equal(b["phat"][keep], a["phat"][keep])
    assert np.array_equal(b["p"], a["p"]) and np.array_equal(b["med"], a["med"])
    assert np.array_equal(b["s"], oracle.harmsum(b["phat"], 16))


def test_zap_function_edges(oracle_lib):
    p = np.arange(1.0, 34.0)  # bins 0..32
    z = p.copy()
    lo = np.array([0.5, 1.0]), np.array([2.0 - 1e-12, 1.0])
    oracle.lib().tbo_zap(z.ctypes.data, z.size, 4.0, lo[0].ctypes.data, lo[1].ctypes.data, 2)
    # [0.5, 2) Hz at T = 4 s: bins 2..7; [1, 1] Hz: bin 4
    assert np.array_equal(np.flatnonzero(z == 0.0), np.arange(2, 8))
    oracle.lib().tbo_zap(z.ctypes.data, z.size, 4.0, lo[0].ctypes.data, lo[1].ctypes.data, 0)
    assert np.count_nonzero(z == 0.0) == 6


def test_zapping_an_interferer_keeps_the_pulsar(oracle_lib):
    """A 50 Hz interferer with harmonics (stronger than the pulsar) fills the
    candidate list; zapping its lines leaves the pulsar as the best candidate."""
    n, ts = 1 << 17, 2.0 ** -10  # 128 s
    t = np.arange(n) * ts
    rng = np.random.default_rng(5)
    k0 = 2861  # pulsar fundamental bin: 22.35 Hz
    x = synth.inject(rng.standard_normal(n), synth.pulse_train(n, ts, n * ts / k0, 0.05, None), 25.0)
    x += sum(0.3 / m * np.cos(2 * np.pi * 50.0 * m * t) for m in range(1, 8))
    x0 = oracle.mean_subtract(x.astype(np.float32))
    tms = [(3600.0, 0.0, 0.0, 0.0, 0.0)]
    plain = oracle.search(x0, oracle.config(n, ts), tms)
    f = plain["freq_hz"] * (1 << plain["log2_harm"].astype(np.int64))  # frequency of the summed bin
    near50 = np.abs(f / 50.0 - np.round(f / 50.0)) * 50.0 < 0.05
    assert near50.sum() > 0
    zap = [(50.0 * m - 0.05, 50.0 * m + 0.05) for m in range(1, 11)]
    z = oracle.search(x0, oracle.config(n, ts, zap=zap), tms)
    fz = z["freq_hz"] * (1 << z["log2_harm"].astype(np.int64))
    assert not np.any(np.abs(fz / 50.0 - np.round(fz / 50.0)) * 50.0 < 0.04)
    best = z[np.argmax(z["sigma"])]
    assert best["bin"] == 16 * k0 and best["log2_harm"] == 4
    assert math.isclose(float(best["freq_hz"]), k0 / (n * ts), rel_tol=1e-12)
