"""The bounds and expansions the pass-1 gather rests on (CPU, 40-digit mpmath).

Between exact solves the kernels continue the delay with a fourth-order
Taylor expansion in the mean anomaly and accept it for a template only when
the remainder bound A W'^5 g5 U^5 / 120 stays below 1e-11 samples, with
g5 >= max |F^(5)(M)| over M and psi, F the BT delay factor of App. A.1
(tau F is the Roemer delay):
  - Kepler solved by Newton (BT model): g5 = 3 (1 + e)^2 / (1 - e)^9;
  - App. B series (ELL7 model): g5 = sum_k k^5 (|C_k| + |S_k|).
These tests check the two bounds against fifth derivatives taken at 40 digits
over a grid of mean anomalies and eccentricities, and the expansion
coefficients the kernels compute (the derivatives of E(M) and F(M) written out
through Faa di Bruno's formula) against derivatives taken the same way."""
import math

import mpmath as mp
import numpy as np
import pytest

mp.mp.dps = 40


def _E(M, e):
    """Eccentric anomaly at 40 digits (Kepler's equation E - e sin E = M)."""
    M = mp.mpf(M)
    if e == 0:
        return M
    return mp.findroot(lambda E: E - e * mp.sin(E) - M, M + e * mp.sin(M))


def _parts(e):
    """The two shapes of the BT factor: F = sin(psi) a(M) + cos(psi) b(M)."""
    e = mp.mpf(e)
    beta = mp.sqrt(1 - e * e)
    return (lambda M: mp.cos(_E(M, e)) - e), (lambda M: beta * mp.sin(_E(M, e)))


def _bt_bound(e):
    return 3.0 * (1.0 + e) ** 2 / (1.0 - e) ** 9


ECCS = [0.0, 0.05, 0.1, 0.3, 0.5, 0.6, 0.8, 0.9]


@pytest.mark.parametrize("e", ECCS)
def test_bt_fifth_derivative_bound(e):
    """max over psi of |F^(5)| is sqrt(a^(5)^2 + b^(5)^2); it stays below the
    bound at every grid point, with the largest values near periastron."""
    a, b = _parts(e)
    worst = 0.0
    # dense near periastron (M = 0), where the derivatives peak
    grid = sorted(set([2 * math.pi * k / 48 for k in range(48)] + [s * 10.0 ** -p for p in range(1, 4)
                                                                   for s in (-1, 1)]))
    for M in grid:
        d5a = mp.diff(a, M, 5)
        d5b = mp.diff(b, M, 5)
        worst = max(worst, float(mp.sqrt(d5a * d5a + d5b * d5b)))
    assert worst <= _bt_bound(e), (e, worst, _bt_bound(e))
    if e > 0:
        assert worst > 1e-3 * _bt_bound(e)  # the grid reaches the steep part


def _series_coefficients(e):
    """App. B coefficients of cos E and sqrt(1-e^2) sin E (tests/golden table)."""
    e2, e3, e4, e5, e6 = e * e, e ** 3, e ** 4, e ** 5, e ** 6
    C = [-e / 2, 1 - 3 / 8 * e2 + 5 / 192 * e4 - 7 / 9216 * e6, e / 2 - e3 / 3 + e5 / 16,
         3 / 8 * e2 - 45 / 128 * e4 + 567 / 5120 * e6, e3 / 3 - 2 / 5 * e5, 125 / 384 * e4 - 4375 / 9216 * e6,
         27 / 80 * e5, 16807 / 46080 * e6]
    S = [0.0, 1 - 5 / 8 * e2 - 11 / 192 * e4 - 457 / 9216 * e6, e / 2 - 5 / 12 * e3 + e5 / 24,
         3 / 8 * e2 - 51 / 128 * e4 + 543 / 5120 * e6, e3 / 3 - 13 / 30 * e5, 125 / 384 * e4 - 4625 / 9216 * e6,
         27 / 80 * e5, 16807 / 46080 * e6]
    return C, S


@pytest.mark.parametrize("e", [0.0, 0.05, 0.1, 0.3, 0.6])
@pytest.mark.parametrize("psi", [0.0, 0.7, 2.0, 4.4])
def test_series_fifth_derivative_bound(e, psi):
    C, S = _series_coefficients(e)
    g5 = sum(k ** 5 * (abs(C[k]) + abs(S[k])) for k in range(8))
    sp, cp = mp.sin(psi), mp.cos(psi)

    def F(M):
        return sum(sp * C[k] * mp.cos(k * M) + cp * S[k] * mp.sin(k * M) for k in range(8))

    worst = max(abs(float(mp.diff(F, 2 * math.pi * j / 40, 5))) for j in range(40))
    assert worst <= g5 * (1 + 1e-12)


@pytest.mark.parametrize("e", [0.0, 0.1, 0.5, 0.8])
@pytest.mark.parametrize("psi", [0.3, 2.0])
@pytest.mark.parametrize("M", [0.0, 0.4, 2.9, 5.1])
def test_bt_expansion_coefficients(e, psi, M):
    """F^(m)(M), m = 1..4, as the kernels build them from E and q = 1/(1 - e cos E)."""
    E = float(_E(M, e))
    sE, cE = math.sin(E), math.cos(E)
    beta = math.sqrt(1 - e * e)
    sw, cw = math.sin(psi), math.cos(psi)
    FE = -sE * sw + beta * cE * cw
    FEE = -cE * sw - beta * sE * cw
    q = 1.0 / (1.0 - e * cE)
    E1 = q
    E2 = -e * sE * q ** 3
    E3 = -e * cE * q ** 4 + 3 * e * e * sE * sE * q ** 5
    E4 = e * sE * q ** 5 + 10 * e * e * sE * cE * q ** 6 - 15 * e ** 3 * sE ** 3 * q ** 7
    F1 = FE * E1
    F2 = FEE * E1 ** 2 + FE * E2
    F3 = -FE * E1 ** 3 + 3 * FEE * E1 * E2 + FE * E3
    F4 = -FEE * E1 ** 4 - 6 * FE * E1 ** 2 * E2 + FEE * (3 * E2 * E2 + 4 * E1 * E3) + FE * E4
    a, b = _parts(e)

    def F(x):
        return mp.sin(psi) * a(x) + mp.cos(psi) * b(x)

    for m, val in ((1, F1), (2, F2), (3, F3), (4, F4)):
        ref = float(mp.diff(F, M, m))
        assert abs(val - ref) <= 1e-11 * max(1.0, abs(ref)) * _bt_bound(e) ** (m / 5), (m, val, ref)


def test_remainder_bound_at_survey_extremes():
    """Chunk decisions at the workload extremes.  A chunk of L tile points of
    one pass-1 column (rows 2R samples apart) is expanded around its middle
    sample; with the column offset of other tiles (up to 2 (R - 1) samples)
    the largest |u| is R (L + 1) - 1.  C2 (2^23 samples at 64 us, R = 512 at
    8192-point tiles): the fastest orbit of the bank (P_orb 1 h, tau 2 lt-s)
    is accepted with 16-point chunks.  C3's hardest template (P_orb 5 h,
    tau 6, e 0.1 at 256 us, 2^24 samples): accepted with 16-point chunks on
    the default 16384-point tiles (R = 512), and only with 8-point chunks on
    8192-point tiles (R = 1024)."""
    def bound(tau, porb, e, ts, U):
        A, Wp = tau / ts, 2 * math.pi / porb * ts
        return A * Wp ** 5 * _bt_bound(e) * U ** 5 / 120

    def reach(R, L):
        return R * (L + 1) - 1

    assert bound(2.0, 3600.0, 0.0, 64e-6, reach(512, 16)) < 1e-11
    assert bound(6.0, 5 * 3600.0, 0.1, 256e-6, reach(512, 16)) <= 1e-11
    assert bound(6.0, 5 * 3600.0, 0.1, 256e-6, reach(1024, 16)) > 1e-11
    assert bound(6.0, 5 * 3600.0, 0.1, 256e-6, reach(1024, 8)) <= 1e-11
