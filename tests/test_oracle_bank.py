"""Pins of the oracle's random template bank (Sec. 2.3-2.7): the metric
density against a closed form, the paper's printed circular bank size, the
eccentricity degeneracy, coordinate invariance of the volume, the count
formula and the rejection step."""
import math
import os

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


# ---------------------------------------------------------------------------
# The projected metric pinned without the oracle's algebra.  The brute force
# below takes the phase of Sec. 2.6 in the bank's own coordinates (P_orb, tau,
# alpha[, e, psi]), differentiates it by central differences at 50 digits
# (Kepler's equation solved by mpmath's root finder), adds the spin frequency
# as a coordinate (d Phi / d kappa = chi u) and projects it out through the
# Schur complement, det(gamma) = det(g) / g_kk.  No Jacobian, no analytic
# derivative and no projection formula of the oracle is used, so a wrong
# Jacobian, a dropped derivative term, a projection sign or swapped angles in
# the oracle shows up as a different density.

T_BANK, F_BANK = 1.2 * HOUR, 66.67
# (kind, P_orb, tau, alpha, e, psi, nodes): few orbits (T/P = 0.3, 1, 3) and
# many (12), e from 0.01 to 0.5
BANK_POINTS = [
    (0, T_BANK / 0.3, 2.0, 0.4, 0.0, 0.0, 128),
    (0, T_BANK / 3.0, 0.5, 3.0, 0.0, 0.0, 128),
    (0, T_BANK / 12.0, 1.0, 5.5, 0.0, 0.0, 256),
    (1, T_BANK / 3.0, 2.0, 1.3, 0.01, 0.3, 128),
    (1, T_BANK / 0.3, 4.0, 0.4, 0.05, 2.0, 128),
    (1, T_BANK / 12.0, 1.0, 5.0, 0.1, 4.5, 256),
    (1, T_BANK / 1.0, 3.0, 2.2, 0.5, 1.1, 128),
]


def _phase_bank(mp, mpmath, kind, T, f_max, P, tau, al, e, psi, u):
    chi = 2 * mp.pi * f_max * T
    M = 2 * mp.pi * u * T / P + al
    if kind == 0:
        return chi * tau / T * mp.sin(M)
    E = mpmath.findroot(lambda x: x - e * mp.sin(x) - M, M)
    return chi * tau / T * ((mp.cos(E) - e) * mp.sin(psi) + mp.sqrt(1 - e * e) * mp.sin(E) * mp.cos(psi))


def _density_brute(kind, T, f_max, P, tau, al, e, psi, nodes, dps=50):
    import mpmath

    mp = mpmath.mp
    with mp.workdps(dps):
        x, w = np.polynomial.legendre.leggauss(nodes)
        us = [(mp.mpf(float(v)) + 1) / 2 for v in x]
        ws = [mp.mpf(float(v)) for v in w]
        tot = mp.fsum(ws)
        ws = [v / tot for v in ws]
        T, f_max = mp.mpf(T), mp.mpf(f_max)
        lam = [mp.mpf(P), mp.mpf(tau), mp.mpf(al)] + ([mp.mpf(e), mp.mpf(psi)] if kind else [])
        chi = 2 * mp.pi * f_max * T

        def phase(l, u):
            ee, pp = (l[3], l[4]) if kind else (0, 0)
            return _phase_bank(mp, mpmath, kind, T, f_max, l[0], l[1], l[2], ee, pp, u)

        rows = []
        for u in us:
            row = [chi * u]
            for a in range(len(lam)):
                h = abs(lam[a]) * mp.mpf("1e-18")
                lp, lm = list(lam), list(lam)
                lp[a] += h
                lm[a] -= h
                row.append((phase(lp, u) - phase(lm, u)) / (2 * h))
            rows.append(row)
        k = len(lam) + 1
        mean = [mp.fsum(wi * r[a] for wi, r in zip(ws, rows)) for a in range(k)]
        g = mp.matrix(k, k)
        for a in range(k):
            for b in range(k):
                g[a, b] = mp.fsum(wi * r[a] * r[b] for wi, r in zip(ws, rows)) - mean[a] * mean[b]
        return mp.sqrt(mp.det(g) / g[0, 0])


_BRUTE = {}


def _brute(pt):
    if pt not in _BRUTE:
        kind, P, tau, al, e, psi, nodes = pt
        _BRUTE[pt] = _density_brute(kind, T_BANK, F_BANK, P, tau, al, e, psi, nodes)
    return _BRUTE[pt]


def _fast(mod, pt):
    kind, P, tau, al, e, psi, nodes = pt
    return float(mod.density(kind, T_BANK, F_BANK, P, tau, al, e if kind else None, psi if kind else None,
                             nodes=nodes)[0])


def _fast_tolerance(mod, pt):
    """1e-11 + 20 n kappa eps, kappa the condition number of the FP64 metric
    scaled to unit diagonal (the FP64 route cannot do better)."""
    kind, P, tau, al, e, psi, nodes = pt
    g = mod.gamma_tilde(kind, T_BANK, P, tau, al, e if kind else None, psi if kind else None, nodes)[0]
    d = np.sqrt(np.diag(g))
    return 1e-11 + 20 * g.shape[0] * np.linalg.cond(g / np.outer(d, d)) * np.finfo(np.float64).eps


def _bank_errors(mod):
    """Per point: (|plain / brute - 1|, |fast / brute - 1| / its tolerance)."""
    out = []
    for pt in BANK_POINTS:
        kind, P, tau, al, e, psi, nodes = pt
        b = _brute(pt)
        p = mod.density_plain(kind, T_BANK, F_BANK, P, tau, al, e, psi, nodes=nodes)
        f = _fast(mod, pt)
        out.append((float(abs(p / b - 1)), abs(f / float(b) - 1) / _fast_tolerance(mod, pt)))
    return out


def test_plain_metric_is_the_brute_force_metric(oracle_lib):
    """The oracle's written-out metric (gamma_plain with the analytic Jacobian
    of the dimensionless coordinates) equals the brute-force metric of the
    phase in the bank's coordinates to 25 digits, circular and elliptical, few
    orbits and many, e from 0.01 to 0.5; the FP64 route used for volumes
    agrees within its conditioning."""
    for pt, (rp, rf) in zip(BANK_POINTS, _bank_errors(bank)):
        assert rp < 1e-25, (pt, rp)
        assert rf <= 1.0, (pt, rf)


BANK_MUTANTS = {
    "tau Jacobian dropped (FP64 route)": (
        "return s * np.asarray(tau, dtype=np.float64) * 2.0 * np.pi / (T * porb ** 2)",
        "return s * 2.0 * np.pi / (T * porb ** 2)"),
    "tau Jacobian dropped (written-out route)": (
        "else t * 2 * mp.pi / (mp.mpf(float(T)) * P ** 2)", "else 2 * mp.pi / (mp.mpf(float(T)) * P ** 2)"),
    "P_orb Jacobian 2 pi / P (circular)": ("return s * 2.0 * np.pi / porb ** 2", "return s * 2.0 * np.pi / porb"),
    "projection sign (written-out route)": (
        "g[a][b] - g[0][a] * g[0][b] / g[0][0]", "g[a][b] + g[0][a] * g[0][b] / g[0][0]"),
    "frequency not projected out (FP64 route)": (
        "r = dc - slope[:, :, None] * uc[None, None, :]", "r = dc"),
    "psi and alpha swapped (FP64 route)": (
        "s = sqrt_det_gamma(kind, T, f_max, porb, tau, alpha, ecc, psi, nodes)",
        "s = sqrt_det_gamma(kind, T, f_max, porb, tau, psi, ecc, alpha, nodes)"),
    "psi and alpha swapped (written-out route)": (
        "gamma_plain(kind, T, porb, tau, alpha, ecc, psi, nodes, dps)",
        "gamma_plain(kind, T, porb, tau, psi, ecc, alpha, nodes, dps)"),
    "sqrt(1-e^2) dropped from d/dE (FP64 route)": (
        "A = -X * sE + Y * b * cE  # d/dE", "A = -X * sE + Y * cE  # d/dE"),
    "d/d alpha without dE/dM (written-out route)": (
        "A * dEdM * u, A * dEdM]", "A * dEdM * u, A]"),
    "chi to the power n - 1 (FP64 route)": (
        "return np.sqrt(np.clip(det, 0.0, None)) * chi ** n",
        "return np.sqrt(np.clip(det, 0.0, None)) * chi ** (n - 1)"),
}


# Slips that only shear the coordinates (adding a multiple of one derivative
# to another, e.g. dropping the d sqrt(1-e^2)/de term of d/de, which lies
# along d/dY) leave every density unchanged; no density pin can see them, and
# none is listed.


@pytest.mark.parametrize("name", sorted(BANK_MUTANTS))
def test_planted_bank_mistakes_are_caught(oracle_lib, name):
    """Each plausible slip, planted in a copy of the oracle's bank module,
    moves the written-out or the FP64 density away from the brute force."""
    import types

    path = os.path.join(os.path.dirname(bank.__file__), "bank.py")
    with open(path) as f:
        src = f.read()
    old, new = BANK_MUTANTS[name]
    assert src.count(old) == 1, name
    mod = types.ModuleType("bank_mutant")
    exec(compile(src.replace(old, new), path, "exec"), mod.__dict__)
    with np.errstate(invalid="ignore"):  # a slip may leave the metric indefinite (det of NaN)
        errs = _bank_errors(mod)
    # caught: some case leaves the tolerance, NaN included
    assert any(not (rp < 1e-25 and rf <= 1.0) for rp, rf in errs), name
