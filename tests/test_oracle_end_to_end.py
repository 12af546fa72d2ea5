"""End-to-end pins of the oracle search: an injected binary pulsar is found at
its true template and frequency, and the demodulation recovers the isolated
pulsar's significance (pipeline mismatch of Sec. 3.1 close to zero)."""
import numpy as np

import oracle
import synth

N, TS = 1 << 20, 64e-6
T = N * TS
K0 = 3355  # f0 T integer: the fundamental sits on a bin centre
PSPIN = T / K0
ORB = synth.Orbit(600.0, 0.2, 1.0)  # T / P_orb = 0.11: orbit resolved
TRUE = (600.0, 0.2, 1.0, 0.0, 0.0)
RIVALS = [(606.0, 0.2, 1.0, 0.0, 0.0), (600.0, 0.204, 1.0, 0.0, 0.0), (600.0, 0.2, 1.05, 0.0, 0.0),
          (600.0, 0.0, 1.0, 0.0, 0.0)]


def _series(orbit):
    rng = np.random.default_rng(7)
    x = synth.inject(rng.standard_normal(N), synth.pulse_train(N, TS, PSPIN, 0.05, orbit), 60.0)
    return oracle.mean_subtract(x.astype(np.float32))


def test_injected_binary_peaks_at_true_template_and_frequency(oracle_lib):
    x0 = _series(ORB)
    cfg = oracle.config(N, TS)
    cands = oracle.search(x0, cfg, [TRUE] + RIVALS)
    best = cands[np.argmax(cands["sigma"])]
    assert best["template_id"] == 0
    assert best["log2_harm"] == 4 and best["bin"] == 16 * K0
    assert abs(best["freq_hz"] - 1.0 / PSPIN) < 1e-9
    # every rival's best is weaker
    for ti in range(1, 1 + len(RIVALS)):
        c = cands[cands["template_id"] == ti]
        assert c["sigma"].max() < best["sigma"]


def test_recovery_ratio_against_isolated_pulsar(oracle_lib):
    """m = 1 - SNR_recovered / SNR_isolated (Sec. 3.1) for the true template."""
    cfg = oracle.config(N, TS)
    b = oracle.search(_series(ORB), cfg, [TRUE])
    iso = oracle.search(_series(None), cfg, [(600.0, 0.0, 0.0, 0.0, 0.0)])
    snr = lambda c: (c["power"] - 16.0) / 4.0
    sb = snr(b[(b["log2_harm"] == 4) & (b["bin"] == 16 * K0)][0])
    si = snr(iso[(iso["log2_harm"] == 4) & (iso["bin"] == 16 * K0)][0])
    assert 1.0 - sb / si < 0.1


def test_search_output_sorted_and_consistent(oracle_lib):
    x0 = _series(ORB)
    cfg = oracle.config(N, TS, fmin_hz=20.0, fmax_hz=200.0)
    c = oracle.search(x0, cfg, [TRUE] + RIVALS, first_template_id=100, series_id=3)
    keys = list(zip(c["template_id"], c["log2_harm"], c["bin"]))
    assert keys == sorted(keys)
    assert np.all(c["series_id"] == 3) and c["template_id"].min() >= 100
    h = 2.0 ** c["log2_harm"]
    f = c["freq_hz"]
    assert np.all(f >= 20.0 - 1.0 / T) and np.all(f <= 200.0 + 1e-9)
    assert np.allclose(f, c["bin"] / (h * T))
    thr = {l: oracle.threshold(1 << l, 6.0) for l in range(5)}
    assert all(p > thr[l] for p, l in zip(c["power"], c["log2_harm"]))
    assert np.all(c["sigma"] > 6.0 - 1e-6)
