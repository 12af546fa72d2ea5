"""Pins of the oracle's dedispersion (the step before the search, App. A /
Sec. 5.2; the paper gives no formula): the dispersion constant from CODATA
constants, DM 0 as a plain channel sum, an impulse in one channel landing at
its delay, a dispersed pulse recovered exactly at its DM, band order."""
import math

import numpy as np
import pytest
import scipy.constants as sc

import oracle


def test_dispersion_constant_from_codata(oracle_lib):
    """Delay of frequency f behind infinite frequency: e^2 DM / (8 pi^2 eps0 m_e c f^2)
    with DM in m^-2; in s MHz^2 per pc cm^-3."""
    k_si = sc.e ** 2 / (8 * math.pi ** 2 * sc.epsilon_0 * sc.m_e * sc.c)  # s Hz^2 m^2
    k = k_si * sc.parsec * 1e6 / 1e12
    assert abs(oracle.dispersion_constant() / k - 1) < 2e-6


def _band(nchan=64, f1=1181.8, df=0.39):
    return f1, df, nchan


def test_zero_dm_is_the_channel_sum(oracle_lib):
    rng = np.random.default_rng(1)
    f1, df, nch = _band()
    x = rng.integers(0, 256, (3000, nch)).astype(np.uint8)
    out = oracle.dedisperse(x, f1, df, 1e-3, [0.0])
    assert out.shape == (1, 3000)
    assert np.array_equal(out[0], x.sum(axis=1).astype(np.float32))


def _delays(f1, df, nch, dm, tsamp):
    f = f1 + df * np.arange(nch)
    return np.rint(oracle.dispersion_constant() * dm * (1 / f ** 2 - 1 / f.max() ** 2) / tsamp).astype(np.int64)


def test_impulse_lands_at_its_delay(oracle_lib):
    f1, df, nch = _band()
    ts = 2e-4
    dms = [0.0, 30.0, 77.7]
    s = [_delays(f1, df, nch, d, ts) for d in dms]
    smax = max(int(v.max()) for v in s)
    n = 5000
    for c in (0, 17, nch - 1):
        x = np.zeros((n, nch), np.uint8)
        t0 = 4000
        x[t0, c] = 200
        out = oracle.dedisperse(x, f1, df, ts, dms)
        assert out.shape == (3, n - smax)
        for d in range(3):
            hit = np.flatnonzero(out[d])
            assert list(hit) == [t0 - s[d][c]] and out[d][hit[0]] == 200.0


def test_dispersed_pulse_is_recovered_at_its_dm(oracle_lib):
    """Pulses placed on the delay curve of DM 120 sum to their full height at
    DM 120 only; other trials smear them."""
    f1, df, nch = _band(128)
    ts, n = 1e-4, 20000
    rng = np.random.default_rng(3)
    x = rng.integers(0, 16, (n, nch)).astype(np.uint8)
    s = _delays(f1, df, nch, 120.0, ts)
    base = x.copy()
    for t0 in (2000, 9000):
        x[t0 + s, np.arange(nch)] += 100
    dms = np.arange(100.0, 140.5, 2.0)
    out = oracle.dedisperse(x, f1, df, ts, dms)
    ref = oracle.dedisperse(base, f1, df, ts, dms)
    gain = (out - ref).max(axis=1)
    best = int(np.argmax(gain))
    assert dms[best] == 120.0 and gain[best] == 100.0 * nch
    assert np.all(np.delete(gain, best) < 0.9 * 100.0 * nch)


def test_band_order_does_not_matter(oracle_lib):
    f1, df, nch = _band(32)
    x = np.random.default_rng(4).integers(0, 256, (4000, nch)).astype(np.uint8)
    a = oracle.dedisperse(x, f1, df, 5e-4, [0.0, 40.0, 333.0])
    f_top = f1 + df * (nch - 1)
    b = oracle.dedisperse(x[:, ::-1], f_top, -df, 5e-4, [0.0, 40.0, 333.0])
    assert np.array_equal(a, b)


def test_four_bit_samples_unpack_to_the_eight_bit_result(oracle_lib):
    """4-bit data (two channels per byte, even channel in the low nibble) gives
    exactly what the same values given as 8-bit samples give."""
    f1, df, nch = _band(32)
    v = np.random.default_rng(6).integers(0, 16, (5000, nch)).astype(np.uint8)
    packed = (v[:, 0::2] | (v[:, 1::2] << 4)).astype(np.uint8)
    dms = [0.0, 25.0, 80.0]
    assert np.array_equal(oracle.dedisperse(packed, f1, df, 2e-4, dms, nbits=4, nchan=nch),
                          oracle.dedisperse(v, f1, df, 2e-4, dms))
    with pytest.raises(ValueError):
        oracle.dedisperse(packed[:, :3], f1, df, 2e-4, dms, nbits=4, nchan=5)


def test_bad_arguments(oracle_lib):
    x = np.zeros((100, 8), np.uint8)
    for args in [(1400.0, 1.0, 1e-3, [-1.0]), (1400.0, 1.0, 0.0, [1.0]), (10.0, -2.0, 1e-3, [1.0]),
                 (1400.0, -1.0, 1e-3, [1e6])]:  # negative DM, tsamp 0, a band below 0 Hz, delays beyond the data
        with pytest.raises(ValueError):
            oracle.dedisperse(x, *args)
