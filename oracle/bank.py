"""Random template bank of Sec. 2.3-2.7: proper-volume density from the
frequency-projected phase metric, the number of random templates, and the
selection of templates with density proportional to sqrt|gamma|.

TEST INFRASTRUCTURE ONLY (part of the oracle): plain FP64 numpy, written from
the paper's definitions; the product library never imports it.

- Phase (Sec. 2.6, the equation of the dimensionless phase): Phi = chi Phi~ with
  chi = 2 pi f_max T and Phi~ = kappa u + X cos E + Y sqrt(1-e^2) sin E,
  u = t/T in [0, 1], X = tau sin(psi)/T, Y = tau cos(psi)/T, M = Omega' u + alpha,
  Omega' = Omega T, E - e sin E = M.  Circular orbits: Phi~ = kappa u +
  tau' sin(Omega' u + alpha), tau' = tau/T (psi merges into alpha).
- Metric (Sec. 2.2, the equation of the metric tensor): g_ab = <d_a Phi d_b Phi> - <d_a Phi><d_b Phi>,
  time averages over u; projected to constant frequency (Sec. 2.5):
  gamma_ab = g_ab - g_ka g_kb / g_kk.  Averages by Gauss-Legendre quadrature.
- Volume and count (Sec. 2.3, the equations of the proper volume, the total
  template count and the random-template count): V = int sqrt(det gamma) d^n lambda, C_n = pi^(n/2)/Gamma(n/2+1),
  N_R = ln(1 - eta) / ln(1 - m^(n/2) C_n / V).
- Two routes to the projected metric: gamma_plain writes the definitions
  out in mpmath (one point at a time); gamma_tilde gets the same numbers in
  FP64 through the residuals of a straight-line fit in u (vectorised, for
  Monte-Carlo volumes).  The tests pin gamma_plain by a brute-force metric
  of the phase in the bank's own coordinates (finite differences, no
  Jacobian) and hold gamma_tilde to gamma_plain.
- Coordinates of the bank (the sampling coordinates): circular
  (P_orb, tau, alpha), elliptical (P_orb, tau, alpha, e, psi).  The density in
  them is sqrt(det gamma~) chi^n times the Jacobian of the dimensionless
  coordinates: 2 pi / P^2 (circular; d tau'/d tau = 1/T, d Omega'/dP = 2 pi T/P^2),
  tau 2 pi / (T P^2) (elliptical; d(X, Y)/d(tau, psi) = tau / T^2).
"""
from __future__ import annotations

import math

import numpy as np

T_SUN = 4.925490947e-6  # G M_sun / c^3 [s]


def tau_max(porb_s, m_pulsar_min: float, m_comp_max: float, theta: float = 1.0):
    """Largest projected radius [lt-s] of Sec. 2.7 / Table 1 at P_orb (Kepler's
    third law, inclination factor theta)."""
    om = 2.0 * np.pi / np.asarray(porb_s, dtype=np.float64)
    return theta * T_SUN ** (1.0 / 3.0) * om ** (-2.0 / 3.0) * m_comp_max / (m_pulsar_min + m_comp_max) ** (2.0 / 3.0)


def _kepler(M, e):
    E = M.copy()
    for _ in range(64):
        E = E - (E - e * np.sin(E) - M) / (1.0 - e * np.cos(E))
    return E


def _derivatives(kind, T, porb, tau, alpha, ecc, psi, u):
    """d Phi~ / d lambda at the nodes u, lambda in the dimensionless
    coordinates: circular (tau', Omega', alpha), elliptical (X, Y, e, Omega',
    alpha).  Arrays (points, n, nodes)."""
    Op = (2.0 * np.pi / porb * T)[:, None]
    al = alpha[:, None]
    M = Op * u[None, :] + al
    if kind == 0:
        tp = (tau / T)[:, None]
        s, c = np.sin(M), np.cos(M)
        return np.stack([s, tp * u[None, :] * c, tp * c], axis=1)
    e = ecc[:, None]
    X = (tau * np.sin(psi) / T)[:, None]
    Y = (tau * np.cos(psi) / T)[:, None]
    E = _kepler(M, np.broadcast_to(e, M.shape))
    sE, cE = np.sin(E), np.cos(E)
    b = np.sqrt(1.0 - e * e)
    dEdM = 1.0 / (1.0 - e * cE)
    dEde = sE / (1.0 - e * cE)
    A = -X * sE + Y * b * cE  # d/dE of X cos E + Y b sin E
    de = A * dEde - Y * e / b * sE
    return np.stack([cE, b * sE, de, A * dEdM * u[None, :], A * dEdM], axis=1)


def sqrt_det_gamma(kind, T, f_max, porb, tau, alpha, ecc=None, psi=None, nodes: int = 256):
    """sqrt(det gamma) chi^n in the dimensionless coordinates (see module
    docstring); kind 0 circular (n = 3), 1 elliptical (n = 5)."""
    gam = gamma_tilde(kind, T, porb, tau, alpha, ecc, psi, nodes)
    n = gam.shape[1]
    det = np.linalg.det(gam)
    chi = 2.0 * np.pi * f_max * T
    return np.sqrt(np.clip(det, 0.0, None)) * chi ** n


def _derivatives_mp(kind, T, porb, tau, alpha, ecc, psi, u):
    """d Phi~ / d(kappa, lambda) at one node u (mpmath), lambda as in
    _derivatives: the first entry is d Phi~ / d kappa = u."""
    mp = _mp()
    Op = 2 * mp.pi / porb * T
    M = Op * u + alpha
    if kind == 0:
        tp = tau / T
        return [u, mp.sin(M), tp * u * mp.cos(M), tp * mp.cos(M)]
    e = ecc
    X, Y = tau * mp.sin(psi) / T, tau * mp.cos(psi) / T
    E = M
    for _ in range(200):
        step = (E - e * mp.sin(E) - M) / (1 - e * mp.cos(E))
        E -= step
        if abs(step) < mp.mpf(10) ** (-mp.dps + 5):
            break
    sE, cE = mp.sin(E), mp.cos(E)
    b = mp.sqrt(1 - e * e)
    dEdM = 1 / (1 - e * cE)
    dEde = sE / (1 - e * cE)
    A = -X * sE + Y * b * cE
    return [u, cE, b * sE, A * dEde - Y * e / b * sE, A * dEdM * u, A * dEdM]


def _mp():
    import mpmath

    return mpmath.mp


def gamma_plain(kind, T, porb, tau, alpha, ecc=0.0, psi=0.0, nodes: int = 128, dps: int = 40):
    """The projected metric of one point written out as the paper defines it
    (Sec. 2.2 and 2.5): g_ab = <d_a Phi~ d_b Phi~> - <d_a Phi~><d_b Phi~>
    over the coordinates (kappa, lambda), then gamma_ab = g_ab - g_ka g_kb /
    g_kk, in mpmath at dps digits so that short orbital arcs, where the
    products nearly cancel, keep their digits.  Same Gauss-Legendre nodes as
    gamma_tilde.  Returns an n x n list of mpf."""
    mp = _mp()
    with mp.workdps(dps):
        x, w = np.polynomial.legendre.leggauss(nodes)
        us = [(mp.mpf(float(v)) + 1) / 2 for v in x]
        # weights summing to 1 exactly: the average of a constant is that
        # constant, so constant parts of the derivatives cancel to all digits
        ws = [mp.mpf(float(v)) for v in w]
        tot = mp.fsum(ws)
        ws = [v / tot for v in ws]
        args = [mp.mpf(float(v)) for v in (T, porb, tau, alpha, ecc, psi)]
        d = [_derivatives_mp(kind, args[0], args[1], args[2], args[3], args[4], args[5], u) for u in us]
        k = len(d[0])
        mean = [mp.fsum(wi * di[a] for wi, di in zip(ws, d)) for a in range(k)]
        g = [[mp.fsum(wi * di[a] * di[b] for wi, di in zip(ws, d)) - mean[a] * mean[b] for b in range(k)]
             for a in range(k)]
        return [[g[a][b] - g[0][a] * g[0][b] / g[0][0] for b in range(1, k)] for a in range(1, k)]


def density_plain(kind, T, f_max, porb, tau, alpha, ecc=0.0, psi=0.0, nodes: int = 128, dps: int = 40):
    """The density of `density` from gamma_plain (one point, mpmath)."""
    mp = _mp()
    with mp.workdps(dps):
        gam = mp.matrix(gamma_plain(kind, T, porb, tau, alpha, ecc, psi, nodes, dps))
        n = gam.rows
        chi = 2 * mp.pi * mp.mpf(f_max) * mp.mpf(T)
        s = mp.sqrt(mp.det(gam)) * chi ** n
        P, t = mp.mpf(float(porb)), mp.mpf(float(tau))
        jac = 2 * mp.pi / P ** 2 if kind == 0 else t * 2 * mp.pi / (mp.mpf(float(T)) * P ** 2)
        return s * jac


def gamma_tilde(kind, T, porb, tau, alpha, ecc=None, psi=None, nodes: int = 256):
    """The frequency-projected metric of the dimensionless phase, one n x n
    matrix per point, in FP64 (vectorised; the route the bulk volumes use).
    It computes the quantity gamma_plain writes out, by another route that
    keeps its digits for short arcs in FP64; the tests hold the two
    together."""
    porb = np.atleast_1d(np.asarray(porb, dtype=np.float64))
    tau = np.broadcast_to(np.asarray(tau, dtype=np.float64), porb.shape)
    alpha = np.broadcast_to(np.asarray(alpha, dtype=np.float64), porb.shape)
    if kind == 1:
        ecc = np.broadcast_to(np.asarray(ecc, dtype=np.float64), porb.shape)
        psi = np.broadcast_to(np.asarray(psi, dtype=np.float64), porb.shape)
    x, w = np.polynomial.legendre.leggauss(nodes)
    u, w = 0.5 * (x + 1.0), 0.5 * w
    d = _derivatives(kind, T, porb, tau, alpha, ecc, psi, u)
    # g_ab - g_ka g_kb / g_kk with g_ab = <ab> - <a><b> and d_kappa Phi~ = u is
    # the average product of the residuals r_a of the derivatives after a
    # weighted least-squares fit of 1 and u (the same quantity, computed without
    # subtracting nearly equal terms when the orbital arc is short)
    dc = d - (d @ w)[:, :, None]
    uc = u - u @ w
    slope = np.einsum("pan,n->pa", dc, uc * w) / ((uc * uc) @ w)
    r = dc - slope[:, :, None] * uc[None, None, :]
    return np.einsum("pan,pbn,n->pab", r, r, w)


def density(kind, T, f_max, porb, tau, alpha, ecc=None, psi=None, nodes: int = 256):
    """Proper-volume density in the bank's coordinates (P_orb [s], tau [lt-s],
    alpha[, e, psi])."""
    porb = np.atleast_1d(np.asarray(porb, dtype=np.float64))
    s = sqrt_det_gamma(kind, T, f_max, porb, tau, alpha, ecc, psi, nodes)
    if kind == 0:
        return s * 2.0 * np.pi / porb ** 2
    return s * np.asarray(tau, dtype=np.float64) * 2.0 * np.pi / (T * porb ** 2)


def unit_ball(n: int) -> float:
    return math.pi ** (n / 2.0) / math.gamma(n / 2.0 + 1.0)


def n_random(volume: float, n: int, coverage: float, mismatch: float):
    """(exact, first-order) number of random templates."""
    x = mismatch ** (n / 2.0) * unit_ball(n) / volume
    exact = math.log(1.0 - coverage) / math.log1p(-x) if x < 1.0 else float("inf")
    approx = volume / (mismatch ** (n / 2.0) * unit_ball(n)) * math.log(1.0 / (1.0 - coverage))
    return exact, approx


def proposals(kind, rng, count, porb_range_s, m_pulsar_min, m_comp_max, ecc_max=0.0):
    """Uniform draws over the prior region of Table 1: P_orb uniform, tau
    uniform in [0, tau_max(P_orb)], alpha (and psi) uniform in [0, 2 pi), e
    uniform in [0, e_max).  Returns the points and their proposal pdf."""
    P = rng.uniform(porb_range_s[0], porb_range_s[1], count)
    tm = tau_max(P, m_pulsar_min, m_comp_max)
    tau = rng.uniform(0.0, 1.0, count) * tm
    alpha = rng.uniform(0.0, 2.0 * np.pi, count)
    q = 1.0 / ((porb_range_s[1] - porb_range_s[0]) * tm * 2.0 * np.pi)
    if kind == 0:
        return dict(porb=P, tau=tau, alpha=alpha), q
    ecc = rng.uniform(0.0, ecc_max, count)
    psi = rng.uniform(0.0, 2.0 * np.pi, count)
    return dict(porb=P, tau=tau, alpha=alpha, ecc=ecc, psi=psi), q / (ecc_max * 2.0 * np.pi)


def volume_mc(dens, q):
    """Monte-Carlo volume from densities at proposal points and their pdf:
    (estimate, standard error)."""
    r = np.asarray(dens) / np.asarray(q)
    return float(r.mean()), float(r.std(ddof=1) / math.sqrt(r.size))


def select(dens, q, uniforms, wmax=None):
    """Rejection step: point i is kept when uniforms[i] * wmax < w_i, w = dens / q
    (wmax defaults to the batch maximum).  Kept points follow dens."""
    w = np.asarray(dens) / np.asarray(q)
    if wmax is None:
        wmax = float(w.max())
    return np.flatnonzero(np.asarray(uniforms) * wmax < w)
