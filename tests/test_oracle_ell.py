"""Pins of the oracle's series Roemer delay (App. B: cos E and sqrt(1-e^2) sin E
as series in the mean anomaly with coefficients through e^6, the paper's
ELL7; Sec. 2.2 and the discussion of the BT and ELL models).

The coefficients are recovered from the oracle's delay by a 16-point DFT over
one orbit and compared with the degree-6 Taylor polynomials of the exact
Fourier-Bessel coefficients, C_k = (J_{k-1}(ke) - J_{k+1}(ke))/k and
S_k = 2 sqrt(1-e^2) J_k(ke)/(ke), taken with 30-digit arithmetic; the delay is
compared with the exact (converged Bessel) delay within the e^7 truncation;
e = 0 reduces exactly to the circular BT delay; resampling indices follow the
exact delay; the search switches model without other change."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
import synth


def _taylor6(f, e):
    mp.mp.dps = 30
    c = mp.taylor(f, 0, 6)
    return float(sum(ci * mp.mpf(e) ** i for i, ci in enumerate(c)))


def _C_exact(k):
    if k == 0:
        return lambda e: -e / 2
    return lambda e: (mp.besselj(k - 1, k * e) - mp.besselj(k + 1, k * e)) / k


def _S_exact(k):
    # 2 sqrt(1-e^2) J_k(ke)/(ke), regular at e = 0
    return lambda e: 2 * mp.sqrt(1 - e * e) * mp.besselj(k, k * e) / (k * e) if e != 0 else (1 if k == 1 else 0)


def _coefficients_from_delay(e):
    """C_k from psi = pi/2 (delay = cos E - e), S_k from psi = 0 (delay =
    sqrt(1-e^2) sin E), tau = 1, sampled at M = 2 pi j / 16."""
    P = 1000.0
    t = np.arange(16) * P / 16
    dc = np.array([oracle.roemer_delay_series((P, 1.0, 0.0, e, math.pi / 2), ti) for ti in t]) + e
    ds = np.array([oracle.roemer_delay_series((P, 1.0, 0.0, e, 0.0), ti) for ti in t])
    Fc, Fs = np.fft.rfft(dc) / 8, np.fft.rfft(ds) / 8
    C = Fc.real[:8].copy()
    C[0] /= 2
    S = -Fs.imag[:8]
    return C, S


@pytest.mark.parametrize("e", [0.1, 0.3, 0.6])
def test_appendix_b_coefficients_are_the_bessel_taylor_polynomials(oracle_lib, e):
    C, S = _coefficients_from_delay(e)
    for k in range(8):
        assert abs(C[k] - _taylor6(_C_exact(k), e)) < 1e-13, ("C", k)
        if k:
            assert abs(S[k] - _taylor6(_S_exact(k), e)) < 1e-13, ("S", k)


@pytest.mark.parametrize("e", [0.02, 0.1, 0.2])
def test_series_delay_within_truncation_of_exact(oracle_lib, e):
    P, tau, alpha, psi = 3000.0, 1.7, 0.4, 2.2
    t = np.linspace(0.0, 2.5 * P, 1001)
    exact = synth.orbit_delay(t, P, tau, alpha, e, psi) - tau * e * math.sin(psi)
    ser = np.array([oracle.roemer_delay_series((P, tau, alpha, e, psi), ti) for ti in t])
    bt = np.array([oracle.roemer_delay((P, tau, alpha, e, psi), ti) for ti in t])
    bound = 1.3 * e**7 * tau * (abs(math.sin(psi)) + abs(math.cos(psi))) + 1e-14 * tau
    assert np.max(np.abs(ser - exact)) <= bound
    assert np.max(np.abs(bt - exact)) <= 1e-13 * tau
    if e >= 0.1:
        assert np.max(np.abs(ser - bt)) > 0.02 * e**7 * tau  # a truncated series, not the Newton solution


def test_zero_eccentricity_is_the_circular_bt_delay(oracle_lib):
    for tm in [(2000.0, 0.9, 0.7, 0.0, 0.0), (500.0, 3.0, 5.0, 0.0, 1.3)]:
        for t in [0.0, 1.0, 123.456, 1999.0, 1e4]:
            assert oracle.roemer_delay_series(tm, t) == oracle.roemer_delay(tm, t)


def test_series_indices_follow_the_exact_delay(oracle_lib):
    """e = 0.02: the e^7 truncation is 1e-8 samples, so src_j is the nearest
    integer of the exact delay except within that of a tie; src_0 = 0."""
    n, ts = 1 << 16, 64e-6
    tm = (1.5, 0.5, 1.1, 0.02, 0.6)
    src, delta = oracle.resample_index_model(tm, n, ts, 1)
    t = np.arange(n) * ts
    ex = synth.orbit_delay(t, *tm)
    d = (ex - ex[0]) / ts
    want = np.arange(n) - np.rint(d).astype(np.int64)
    tie = np.abs(d - np.floor(d) - 0.5) < 1e-6
    assert src[0] == 0 and np.array_equal(src[~tie], want[~tie])
    assert np.max(np.abs(delta - d)) < 1e-6
    src0, _ = oracle.resample_index_model(tm, n, ts, 0)
    assert np.array_equal(src0, oracle.resample_index(tm, n, ts)[0])


def test_search_with_series_delay(oracle_lib):
    """Circular templates: both models give identical candidates.  An
    eccentric pulsar (e = 0.1) is found at its true template with the series
    delay as with the Newton solve."""
    n, ts = 1 << 18, 64e-6
    T = n * ts
    k0 = 1201
    orb = synth.Orbit(900.0, 0.3, 1.0, 0.1, 2.0)
    rng = np.random.default_rng(4)
    x = synth.inject(rng.standard_normal(n), synth.pulse_train(n, ts, T / k0, 0.05, orb), 40.0)
    x0 = oracle.mean_subtract(x.astype(np.float32))
    circ = [(900.0, 0.3, 1.0, 0.0, 0.0), (700.0, 0.2, 3.0, 0.0, 0.0)]
    a = oracle.search(x0, oracle.config(n, ts, whiten_window=2048), circ)
    b = oracle.search(x0, oracle.config(n, ts, whiten_window=2048, delay_model=1), circ)
    assert np.array_equal(a, b) and len(a) > 0
    ell = [orb.as_template()[0].tolist(), (900.0, 0.3, 1.0, 0.0, 0.0), (900.0, 0.3, 1.3, 0.1, 2.0)]
    c = oracle.search(x0, oracle.config(n, ts, whiten_window=2048, delay_model=1), ell)
    best = c[np.argmax(c["sigma"])]
    assert best["template_id"] == 0 and best["log2_harm"] == 4 and best["bin"] == 16 * k0
