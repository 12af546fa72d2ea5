"""Pins of the oracle's candidate grouping (App. A: repeated detections of one
signal are grouped and the strongest kept; the grouping rule is this
project's definition, written out in oracle/tbo.c, O11).

A hand-worked example fixes the rule; a boundary case fixes how the tolerance
scales with the ratio p/q; on random lists the greedy output is checked
against the declarative form of the same rule (a candidate is kept exactly
when no stronger kept candidate is related to it, and is counted in the group
of the strongest such one); the output does not depend on input order; and
on a real search the injected pulsar's detections collapse onto its true
template."""
import math

import numpy as np
import pytest

import oracle

DT = oracle.CANDIDATE_DTYPE


def _c(series, tmpl, fold, k, sigma):
    return (series, tmpl, k, fold, 0.0, sigma, 0.0)


def _F(c):
    return int(c["bin"]) << (4 - int(c["log2_harm"]))


def test_hand_worked_example(oracle_lib):
    cands = np.array([
        _c(0, 2, 0, 1234567, 7.0),  # E: 1234567 bins, no ratio p/q <= 16 reaches it from A
        _c(0, 3, 0, 2000, 8.0),     # B: second harmonic of A
        _c(0, 1, 1, 1001, 5.0),     # D: F = 8008, |2 F - F_A| = 16 <= 2 * 16
        _c(1, 3, 0, 1000, 6.0),     # G: A's frequency in another series
        _c(0, 3, 0, 1000, 10.0),    # A: F = 16000
        _c(0, 9, 0, 1002, 4.0),     # H: F = 16032, 32 > 16 from A
        _c(0, 5, 4, 16001, 9.0),    # C: F = 16001, one sixteenth of a bin from A
    ], dtype=DT)
    kept, grp = oracle.distill(cands, max_ratio=16, tol=16)
    got = [(int(c["series_id"]), int(c["template_id"]), int(c["log2_harm"]), int(c["bin"])) for c in kept]
    assert got == [(0, 3, 0, 1000), (0, 2, 0, 1234567), (1, 3, 0, 1000), (0, 9, 0, 1002)]
    assert list(grp) == [4, 1, 1, 1]


def test_tolerance_is_measured_at_the_ratio(oracle_lib):
    """Ratio 3/2 of F_a = 1600 with tol = 16: F_b in [2384, 2416] joins, 2383
    and 2417 do not (fold-16 bins give F = k)."""
    a = _c(0, 0, 0, 100, 10.0)
    for fb, joins in [(2383, False), (2384, True), (2400, True), (2416, True), (2417, False)]:
        cands = np.array([a, _c(0, 1, 4, fb, 5.0)], dtype=DT)
        kept, grp = oracle.distill(cands, max_ratio=3, tol=16)
        assert (len(kept) == 1) == joins, fb
        assert int(grp[0]) == (2 if joins else 1)


def test_relative_tolerance_scales_with_the_target(oracle_lib):
    """ppm = 100, tol = 0, F_a = 100000: the target F_a joins within 10,
    the target 2 F_a within 20 (the tolerance is relative to p/q F_a)."""
    a = _c(0, 0, 4, 100000, 10.0)
    for fb, joins in [(100010, True), (100011, False), (99990, True), (99989, False),
                      (200020, True), (200021, False), (199980, True), (199979, False)]:
        kept, _ = oracle.distill(np.array([a, _c(0, 1, 4, fb, 5.0)], dtype=DT), max_ratio=2, tol=0, ppm=100)
        assert (len(kept) == 1) == joins, fb


def test_same_frequency_only(oracle_lib):
    """max_ratio 1, tol 0: only equal fundamentals merge, whatever the fold."""
    cands = np.array([_c(0, 0, 0, 100, 9.0), _c(0, 1, 4, 1600, 8.0), _c(0, 2, 1, 200, 7.0),
                      _c(0, 3, 4, 1601, 6.0), _c(0, 4, 0, 200, 5.0)], dtype=DT)
    kept, grp = oracle.distill(cands, max_ratio=1, tol=0)
    assert [int(c["template_id"]) for c in kept] == [0, 3, 4] and list(grp) == [3, 1, 1]


def _random_list(seed, n=300):
    rng = np.random.default_rng(seed)
    c = np.zeros(n, dtype=DT)
    c["series_id"] = rng.integers(0, 3, n)
    c["template_id"] = rng.integers(0, 50, n)
    c["log2_harm"] = rng.integers(0, 5, n)
    base = rng.integers(40, 400, n)
    mult = rng.integers(1, 5, n)
    c["bin"] = (base * mult * (1 << c["log2_harm"]) // 4 + rng.integers(-2, 3, n)).clip(1)
    c["sigma"] = np.round(rng.uniform(3.0, 12.0, n), 1)  # many ties: the secondary keys decide
    return c


def _rel(a, b, P, tol, ppm):
    """|F_b - (p/q) F_a| <= tol + ppm 1e-6 (p/q) F_a in exact rationals."""
    from fractions import Fraction

    if a["series_id"] != b["series_id"]:
        return False
    fa, fb = _F(a), _F(b)
    for p in range(1, P + 1):
        for q in range(1, P + 1):
            t = Fraction(p, q) * fa
            if abs(fb - t) <= tol + Fraction(ppm, 10**6) * t:
                return True
    return False


def _key(c):
    return (-float(c["sigma"]), int(c["series_id"]), int(c["template_id"]), int(c["log2_harm"]), int(c["bin"]))


@pytest.mark.parametrize("seed,P,tol,ppm", [(1, 16, 16, 0), (2, 4, 8, 0), (3, 1, 0, 0), (4, 8, 40, 0),
                                             (5, 16, 0, 3000), (6, 3, 16, 800)])
def test_greedy_matches_declarative_rule(oracle_lib, seed, P, tol, ppm):
    c = _random_list(seed)
    # drop exact duplicates of (series, template, fold, bin): records are unique in a search
    _, idx = np.unique(c[["series_id", "template_id", "log2_harm", "bin"]], return_index=True)
    c = c[np.sort(idx)]
    kept, grp = oracle.distill(c, max_ratio=P, tol=tol, ppm=ppm)
    order = sorted(range(len(c)), key=lambda i: _key(c[i]))
    keep_set, owner = [], {}
    for i in order:
        strong = [j for j in keep_set if _rel(c[j], c[i], P, tol, ppm)]
        if strong:
            owner[i] = strong[0]
        else:
            keep_set.append(i)
    assert [_key(c[i]) for i in keep_set] == [_key(k) for k in kept]
    want = [1 + sum(1 for v in owner.values() if v == j) for j in keep_set]
    assert list(grp) == want and sum(grp) == len(c)
    assert 0 < len(kept) < len(c) or P == 1


def test_input_order_does_not_matter(oracle_lib):
    c = _random_list(7)
    _, idx = np.unique(c[["series_id", "template_id", "log2_harm", "bin"]], return_index=True)
    c = c[idx]
    a = oracle.distill(c)
    perm = np.random.default_rng(8).permutation(len(c))
    b = oracle.distill(c[perm])
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_bad_arguments(oracle_lib):
    c = np.array([_c(0, 0, 5, 10, 1.0)], dtype=DT)
    with pytest.raises(ValueError):
        oracle.distill(c)
    for kw in (dict(max_ratio=0), dict(max_ratio=65), dict(tol=-1), dict(ppm=-1), dict(ppm=10**6 + 1)):
        with pytest.raises(ValueError):
            oracle.distill(c[:0], **kw)
    kept, grp = oracle.distill(c[:0])
    assert len(kept) == 0 and len(grp) == 0


def test_injected_pulsar_collapses_onto_true_template(oracle_lib):
    """A bin-centred binary pulsar searched with its true orbit and four
    neighbours: all detections at the pulsar's fundamental and harmonics form
    one group headed by the true template's 16-harmonic fold at 16 f0 T, once
    the tolerance admits the neighbours' residual Doppler offsets (1e-3); with
    one bin alone they form a handful of groups at f0 and its harmonics."""
    from tests import test_oracle_end_to_end as E2E

    x0 = E2E._series(E2E.ORB)
    cands = oracle.search(x0, oracle.config(E2E.N, E2E.TS), [E2E.TRUE] + E2E.RIVALS)
    kept, grp = oracle.distill(cands, ppm=1000)
    assert len(kept) == 1 and grp[0] == len(cands)
    assert kept[0]["template_id"] == 0 and kept[0]["log2_harm"] == 4 and kept[0]["bin"] == 16 * E2E.K0
    assert math.isclose(float(kept[0]["sigma"]), float(cands["sigma"].max()))
    kept, grp = oracle.distill(cands)
    assert 1 < len(kept) < 20 and grp[0] > 0.5 * len(cands)
    ratios = [(int(c["bin"]) << (4 - int(c["log2_harm"]))) / (16.0 * E2E.K0) for c in kept]
    assert all(abs(r - round(r)) < 2e-3 for r in ratios)
