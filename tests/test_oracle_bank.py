"""Pins of the oracle's random template bank (Sec. 2.3-2.7): the metric
density against a closed form, the paper's printed circular bank size, the
eccentricity degeneracy, coordinate invariance of the volume, the count
formula and the rejection step."""
import math

import numpy as np
import pytest

from oracle import bank

HOUR = 3600.0
TABLE1 = dict(T=1.2 * HOUR, f_max=66.67, porb=(6 * HOUR, 12 * HOUR), m_p=1.4, m_c=8.0, eta=0.9, m=0.2)


def test_many_orbit_limit_of_the_circular_metric(oracle_lib):
    """For Omega' >> 1 the oscillating cross terms and means vanish:
    <sin^2> = <cos^2> = 1/2, <u cos^2> = 1/4, <u^2 cos^2> = 1/6, and nothing
    couples to the frequency, so gamma~ = [[1/2, 0, 0], [0, t^2/6, t^2/4],
    [0, t^2/4, t^2/2]] in (tau', Omega', alpha) and sqrt(det) = t^2 / sqrt(96)."""
    T, f = 1000.0, 10.0
    chi = 2 * math.pi * f * T
    tp = 1e-3
    for orbits in (200.0, 400.0):
        s = bank.sqrt_det_gamma(0, T, f, T / orbits, tp * T, 0.7, nodes=8192)[0] / chi ** 3
        assert abs(s / (tp ** 2 / math.sqrt(96.0)) - 1.0) < 2.0 / (2 * math.pi * orbits) ** 0.5


def test_circular_bank_size_of_the_paper(oracle_lib):
    """Table 1 priors with e = 0 (T = 1.2 h, f_max = 66.67 Hz, P_orb 6-12 h,
    tau up to the 1.4 + 8 solar-mass limit, coverage 0.9, mismatch 0.2): the
    paper generated 10,128 circular templates (Sec. 5.1).  Monte-Carlo volume
    over 60,000 points; the count must agree within 3 standard errors."""
    c = TABLE1
    rng = np.random.default_rng(2112)
    vals, qs = [], []
    for _ in range(6):
        pts, q = bank.proposals(0, rng, 10000, c["porb"], c["m_p"], c["m_c"])
        vals.append(bank.density(0, c["T"], c["f_max"], pts["porb"], pts["tau"], pts["alpha"], nodes=128))
        qs.append(q)
    V, err = bank.volume_mc(np.concatenate(vals), np.concatenate(qs))
    n_exact, n_approx = bank.n_random(V, 3, c["eta"], c["m"])
    assert abs(n_exact - 10128) <= 3 * (err / V) * n_exact
    assert abs(n_exact / n_approx - 1) < 1e-3


def test_eccentric_metric_degenerates_at_zero_eccentricity(oracle_lib):
    """At e = 0, d/d alpha = Y d/dX - X d/dY: the elliptical metric is singular
    (smallest eigenvalue of the unit-diagonal metric at rounding level), and
    since eccentricity separates the directions at first order in e, that
    eigenvalue grows as e^2; the density grows with e."""
    T = 1.2 * HOUR
    lam = {}
    for e in (0.0, 0.001, 0.01, 0.02):
        g = bank.gamma_tilde(1, T, 8 * HOUR, 4.0, 0.4, ecc=e, psi=1.1)[0]
        d = np.sqrt(np.diag(g))
        lam[e] = np.linalg.eigvalsh(g / np.outer(d, d))[0]
    assert lam[0.0] < 1e-14
    assert abs(lam[0.01] / lam[0.001] / 100 - 1) < 0.05 and abs(lam[0.02] / lam[0.01] / 4 - 1) < 0.05
    dens = [bank.sqrt_det_gamma(1, T, 66.67, 8 * HOUR, 4.0, 0.4, ecc=e, psi=1.1)[0] for e in (0.01, 0.02, 0.05, 0.1)]
    assert dens[0] < dens[1] < dens[2] < dens[3]


def test_volume_does_not_depend_on_the_sampling_coordinates(oracle_lib):
    """Drawing Omega uniformly instead of P_orb (proposal pdf q_Omega, density
    in (Omega, tau, alpha) = sqrt(det gamma~) chi^3 T / T): the Monte-Carlo
    volumes agree within their errors."""
    c = TABLE1
    rng = np.random.default_rng(7)
    pts, q = bank.proposals(0, rng, 20000, c["porb"], c["m_p"], c["m_c"])
    V1, e1 = bank.volume_mc(bank.density(0, c["T"], c["f_max"], pts["porb"], pts["tau"], pts["alpha"], nodes=128), q)
    om = rng.uniform(2 * math.pi / c["porb"][1], 2 * math.pi / c["porb"][0], 20000)
    P = 2 * math.pi / om
    tm = bank.tau_max(P, c["m_p"], c["m_c"])
    tau = rng.uniform(0, 1, 20000) * tm
    al = rng.uniform(0, 2 * math.pi, 20000)
    dens = bank.sqrt_det_gamma(0, c["T"], c["f_max"], P, tau, al, nodes=128)  # per d tau' d Omega' d alpha
    dens = dens * (1 / c["T"]) * c["T"]  # d tau'/d tau = 1/T, d Omega'/d Omega = T
    qo = 1.0 / ((2 * math.pi / c["porb"][0] - 2 * math.pi / c["porb"][1]) * tm * 2 * math.pi)
    V2, e2 = bank.volume_mc(dens, qo)
    assert abs(V1 - V2) < 3 * math.hypot(e1, e2)


def test_count_formula(oracle_lib):
    assert math.isclose(bank.unit_ball(3), 4 * math.pi / 3)
    assert math.isclose(bank.unit_ball(5), 8 * math.pi ** 2 / 15)
    V = 1e6
    ex, ap = bank.n_random(V, 3, 0.9, 0.2)
    x = 0.2 ** 1.5 * (4 * math.pi / 3) / V
    assert math.isclose(ex, math.log(0.1) / math.log(1 - x), rel_tol=1e-8)  # log(1 - x) here rounds at ~eps/x
    assert abs(ex / ap - 1) < 1e-5
    ex, ap = bank.n_random(2.0, 3, 0.9, 0.2)  # a volume of a few template balls
    assert ex < ap and ex > 0


def test_rejection_step_follows_the_density(oracle_lib):
    """Points x ~ U(0, 1) kept with probability proportional to x follow the pdf
    2x (Kolmogorov-Smirnov against F(x) = x^2)."""
    rng = np.random.default_rng(11)
    x = rng.uniform(0, 1, 200000)
    keep = bank.select(x, np.ones_like(x), rng.uniform(0, 1, x.size))
    k = np.sort(x[keep])
    F = k ** 2
    ecdf = np.arange(1, k.size + 1) / k.size
    assert np.max(np.abs(ecdf - F)) < 1.63 / math.sqrt(k.size)  # 1 % level
    assert abs(k.size / x.size - 0.5) < 0.01
