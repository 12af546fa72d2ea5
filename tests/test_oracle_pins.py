"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these re-types the oracle's own formula: each compares it with a
closed form, a printed table, an independent high-precision evaluation, a
library special case, brute force or an invariant.
"""
import math
import os
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest
from scipy.special import erfc, gammainccinv, gammaincc
from scipy.stats import norm

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Kepler ---
def _appb():
    coef = {}
    with open(os.path.join(GOLDEN, "appB_kepler_series.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, *terms = line.split()
            coef[name] = [(int(p), Fraction(q)) for p, q in (t.split(":") for t in terms)]
    return coef


def _series(coef, name, e):
    return sum(float(q) * e**p for p, q in coef[name])


@pytest.mark.parametrize("e", [0.02, 0.1])
def test_kepler_matches_appendix_b_series(oracle_lib, e):
    """App. B: the 7th-order series of cos E and sqrt(1-e^2) sin E agrees with
    the exact Kepler solution up to its truncation error (~e^7)."""
    coef = _appb()
    M = np.linspace(-7.0, 13.0, 2001)
    worst = 0.0
    for m in M:
        E, _ = oracle.kepler(m, e)
        c = sum(_series(coef, "C%d" % k, e) * math.cos(k * m) for k in range(8))
        s = sum(_series(coef, "S%d" % k, e) * math.sin(k * m) for k in range(1, 8))
        worst = max(worst, abs(math.cos(E) - c), abs(math.sqrt(1 - e * e) * math.sin(E) - s))
    assert worst < 1.3 * e**7 + 1e-14


@pytest.mark.parametrize("e", [0.0, 0.01, 0.1, 0.5, 0.8])
def test_kepler_against_high_precision(oracle_lib, e):
    mp.mp.dps = 40
    for m in [-3.0, 0.0, 0.3, 1.0, 2.5, 3.14159, 4.0, 9.5, 123.4]:
        E, it = oracle.kepler(m, e)
        if e == 0.0:
            assert E == m and it == 0
            continue
        Ex = mp.findroot(lambda x: x - e * mp.sin(x) - m, m)
        assert abs(E - float(Ex)) < 4e-15 * max(1.0, abs(m))
        assert abs(E - e * math.sin(E) - m) <= 1e-12


# -------------------------------------------------- delay / resample index --
def _mp_delay(t, tm):
    """Roemer delay of the BT model in 40-digit arithmetic, independent code."""
    mp.mp.dps = 40
    porb, tau, alpha, e, psi = (mp.mpf(str(v)) for v in tm)
    M = 2 * mp.pi / porb * mp.mpf(t) + alpha
    E = M if e == 0 else mp.findroot(lambda x: x - e * mp.sin(x) - M, M)
    return tau * ((mp.cos(E) - e) * mp.sin(psi) + mp.sqrt(1 - e * e) * mp.sin(E) * mp.cos(psi))


TEMPLATES = [
    (1.5 * 3600, 1.2, 1.0, 0.0, 0.0),
    (7.3 * 3600, 0.37, 4.4, 0.0, 0.0),
    (8.0 * 3600, 3.0, 1.0, 0.08, 2.0),
    (5.5 * 3600, 5.1, 0.2, 0.6, 5.0),
]


@pytest.mark.parametrize("tm", TEMPLATES)
def test_resample_index_hand_values(oracle_lib, tm):
    """src_j at j = 0, 1, N/2, N-1 against a 40-digit evaluation."""
    n, ts = 1 << 16, 64e-6
    src, delta = oracle.resample_index(tm, n, ts)
    d0 = _mp_delay(0, tm)
    for j in [0, 1, 777, n // 2, n - 1]:
        dj = (_mp_delay(mp.mpf(j) * mp.mpf(ts), tm) - d0) / mp.mpf(ts)
        assert abs(delta[j] - float(dj)) < 1e-8
        want = j - int(mp.nint(dj))
        assert src[j] == want
    assert src[0] == 0


def test_zero_orbit_is_identity(oracle_lib):
    n, ts = 1 << 14, 64e-6
    src, delta = oracle.resample_index((3600.0, 0.0, 2.0, 0.0, 0.0), n, ts)
    assert np.array_equal(src, np.arange(n)) and not delta.any()
    src, _ = oracle.resample_index((3600.0, 0.0, 2.0, 0.3, 1.0), n, ts)
    assert np.array_equal(src, np.arange(n))
    x0 = np.random.default_rng(0).standard_normal(n).astype(np.float32)
    assert np.array_equal(oracle.resample(x0, src), x0.astype(np.float64))


def test_circular_equals_elliptical_limit_and_phase_flip(oracle_lib):
    n, ts = 1 << 14, 256e-6
    a = oracle.resample_index((2000.0, 0.9, 0.7, 0.0, 0.0), n, ts)[1]
    # e=0, psi=0 through the BT expression is tau sin(M): circular phase model
    t = np.arange(n) * ts
    circ = (0.9 * np.sin(2 * np.pi / 2000.0 * t + 0.7) - 0.9 * np.sin(0.7)) / ts
    assert np.max(np.abs(a - circ)) < 1e-9
    b = oracle.resample_index((2000.0, 0.9, 0.7 + math.pi, 0.0, 0.0), n, ts)[1]
    assert np.max(np.abs(a + b)) < 1e-8


def test_out_of_range_reads_zero(oracle_lib):
    n, ts = 1 << 12, 1e-3
    tm = (20.0, 0.5, math.pi, 0.0, 0.0)  # delta down to -500 samples: reads past the end
    src, _ = oracle.resample_index(tm, n, ts)
    x0 = np.arange(1, n + 1, dtype=np.float32)
    y = oracle.resample(x0, src)
    oob = (src < 0) | (src >= n)
    assert oob.any() and np.all(y[oob] == 0.0)
    assert np.array_equal(y[~oob], x0[src[~oob]].astype(np.float64))


def test_mean_subtract(oracle_lib):
    x = (np.random.default_rng(3).standard_normal(10001) + 5.0).astype(np.float32)
    x0 = oracle.mean_subtract(x)
    m = float(mp.fsum([mp.mpf(float(v)) for v in x]) / len(x))
    assert np.array_equal(x0, (x.astype(np.float64) - m).astype(np.float32))


# -------------------------------------------------------------- DFT/power --
def test_naive_dft_brute_force_2_10(oracle_lib):
    n = 1 << 10
    y = np.random.default_rng(1).standard_normal(n)
    X = oracle.dft_naive(y)
    ref = np.fft.rfft(y)
    assert np.max(np.abs(X - ref)) < 1e-10
    # direct O(N^2) sum in 30-digit arithmetic at a few bins
    mp.mp.dps = 30
    for k in [0, 1, 37, 511, 512]:
        s = mp.fsum(mp.mpf(float(y[j])) * mp.expjpi(mp.mpf(-2 * ((k * j) % n)) / n) for j in range(n))
        assert abs(complex(s) - X[k]) < 1e-10


@pytest.mark.parametrize("lg", [10, 12, 14, 16])
def test_fft_against_library(oracle_lib, lg):
    n = 1 << lg
    y = np.random.default_rng(lg).standard_normal(n)
    assert np.max(np.abs(oracle.fft(y) - np.fft.rfft(y))) < 1e-9 * math.sqrt(n)
    if lg <= 12:
        assert np.max(np.abs(oracle.fft(y) - oracle.dft_naive(y))) < 1e-9


def test_parseval_and_pure_tone(oracle_lib):
    n = 1 << 13
    y = np.random.default_rng(5).standard_normal(n)
    p = oracle.power(oracle.fft(y))
    lhs = float(np.dot(y, y))
    rhs = (p[0] + 2 * p[1:-1].sum() + p[-1]) / n
    assert abs(lhs - rhs) < 1e-10 * lhs
    A, k0 = 0.7, 1234
    tone = A * np.cos(2 * np.pi * k0 * np.arange(n) / n)
    p = oracle.power(oracle.fft(tone))
    assert abs(p[k0] - (A * n / 2) ** 2) < 1e-9 * p[k0]
    assert np.max(np.delete(p, k0)) < 1e-12 * p[k0]


# -------------------------------------------------------------- whitening --
def test_whiten_constant_spectrum(oracle_lib):
    p = np.full(1 + 10000, 3.5)
    phat, med = oracle.whiten(p, 4096)
    assert phat[0] == 0.0
    assert np.all(phat[1:] == 3.5 * math.log(2) / 3.5)
    assert med.size == 3 and np.all(med == 3.5)


def test_whiten_linear_ramp_odd_window(oracle_lib):
    """A linear spectrum with odd W: block medians sit on the line at the block
    centres, so the interpolated level is the line itself between the first and
    last centre and is held constant outside."""
    W, m = 999, 9000  # 10 blocks, last one short (9 bins): ragged tail
    k = np.arange(m + 1, dtype=np.float64)
    a, b = 2.0, 0.01
    p = a + b * k
    phat, med = oracle.whiten(p, W)
    starts = 1 + W * np.arange(10)
    counts = np.minimum(W, m - W * np.arange(10))
    cent = starts + (counts - 1) / 2.0
    assert np.allclose(med, a + b * (starts + (counts - 1) // 2), rtol=0, atol=1e-12)
    inside = (k >= cent[0]) & (k <= cent[-2])
    # the last (short, 9-bin) block also has odd count: its centre is on the line
    inside |= (k >= cent[-2]) & (k <= cent[-1])
    assert np.allclose(phat[inside], math.log(2), rtol=1e-12)
    lo = (k >= 1) & (k < cent[0])
    assert np.allclose(phat[lo], math.log(2) * p[lo] / (a + b * cent[0]), rtol=1e-12)
    hi = k > cent[-1]
    assert np.allclose(phat[hi], math.log(2) * p[hi] / (a + b * cent[-1]), rtol=1e-12)


def test_whiten_medians_brute_force(oracle_lib):
    rng = np.random.default_rng(9)
    for W, m in [(4096, 1 << 15), (1000, 12345), (7, 100)]:
        p = rng.exponential(2.0, m + 1)
        _, med = oracle.whiten(p, W)
        for bi in range(med.size):
            blk = p[1 + bi * W: 1 + min(m, (bi + 1) * W)]
            if blk.size % 2 == 1:
                assert med[bi] == np.median(blk)
            else:
                assert med[bi] == np.partition(blk, blk.size // 2 - 1)[blk.size // 2 - 1]


def test_whiten_white_noise_statistics(oracle_lib):
    n = 1 << 17
    y = np.random.default_rng(11).standard_normal(n)
    phat, _ = oracle.whiten(oracle.power(oracle.fft(y)), 4096)
    v = phat[1:]
    assert abs(v.mean() - 1.0) < 0.02
    assert abs(np.median(v) - math.log(2)) < 0.02


# ----------------------------------------------------------- harmonic sum --
def test_harmsum_comb_closed_form(oracle_lib):
    """Harmonic comb at integer k0 on an otherwise empty spectrum: fold h at bin
    h k0 collects exactly the first h harmonics."""
    nb = 1 + 40000
    k0 = 1201
    p = np.zeros(nb)
    amps = {m: float(m * m + 1) for m in range(1, 17)}
    for m, a in amps.items():
        p[m * k0] = a
    s = oracle.harmsum(p, 16)
    for l, h in enumerate([1, 2, 4, 8, 16]):
        assert s[l, h * k0] == sum(amps[m] for m in range(1, h + 1))


def test_harmsum_direct_brute_force(oracle_lib):
    """The incremental folds equal the direct sum over m = 1..h of P at the
    nearest bin (halves up) to m k / h."""
    rng = np.random.default_rng(2)
    nb = 777
    p = rng.integers(0, 1000, nb).astype(np.float64)  # exact sums
    s = oracle.harmsum(p, 16)
    for l, h in enumerate([1, 2, 4, 8, 16]):
        for k in range(nb):
            direct = sum(p[int(Fraction(m * k, h) + Fraction(1, 2))] for m in range(1, h + 1))
            assert s[l, k] == direct, (h, k)


# ------------------------------------------------------ threshold / sigma --
def test_thresholds(oracle_lib):
    p = 0.5 * erfc(6.0 / math.sqrt(2.0))
    assert abs(oracle.threshold(1, 6.0) - (-math.log(p))) < 1e-9
    for h in [2, 4, 8, 16]:
        assert abs(oracle.threshold(h, 6.0) - gammainccinv(h, p)) < 1e-8
    for h in [1, 4, 16]:
        for sg in [3.0, 5.0, 8.0]:
            thr = oracle.threshold(h, sg)
            assert abs(gammaincc(h, thr) - norm.sf(sg)) < 1e-9 * norm.sf(sg)


def test_sigma_conversion(oracle_lib):
    for h in [1, 2, 16]:
        for s in [h + 5.0, 30.0, 80.0]:
            want = norm.isf(gammaincc(h, s))
            assert abs(oracle.sigma_of(h, s) - want) < 1e-6
    mp.mp.dps = 50
    for h, s in [(1, 2000.0), (16, 5000.0), (4, 1.0e5)]:
        q = mp.gammainc(h, s, mp.inf, regularized=True)
        z = mp.findroot(lambda x: mp.log(mp.erfc(x / mp.sqrt(2)) / 2) - mp.log(q), mp.sqrt(2 * s))
        assert abs(oracle.sigma_of(h, s) - float(z)) < 1e-6 * float(z)
        assert abs(oracle.log_tail(h, s) - float(mp.log(q))) < 1e-9 * abs(float(mp.log(q)))


def test_false_alarm_rate_on_exponential_noise(oracle_lib):
    """Whitened noise powers ~ Exp(1): per-fold exceedances of a 3-sigma
    threshold match the Gaussian tail probability (bins >= 2h so the h terms
    are distinct bins)."""
    rng = np.random.default_rng(21)
    nb = 1 << 20
    phat = rng.exponential(1.0, nb)
    s = oracle.harmsum(phat, 16)
    pt = norm.sf(3.0)
    for l, h in enumerate([1, 2, 4, 8, 16]):
        v = s[l, 2 * h:]
        cnt = int((v > oracle.threshold(h, 3.0)).sum())
        exp = pt * v.size
        assert abs(cnt - exp) < 6 * math.sqrt(exp), (h, cnt, exp)
