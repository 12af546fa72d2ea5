"""Parity of the library's candidate grouping (tb_distill, host code behind
the C ABI) with the oracle's: the same input list gives the same kept records
in the same order and the same group sizes, bit for bit (the grouping decides
in integers and orders by the stored sigma)."""
import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module")
def tb():
    import paper_2112_11991_amd as tb

    return tb


def _to_oracle(c):
    o = np.zeros(c.size, dtype=oracle.CANDIDATE_DTYPE)
    for f in ("series_id", "template_id", "bin", "log2_harm", "power", "sigma", "freq_hz"):
        o[f] = c[f]
    return o


def _lists(tb, seed, n, nseries=4, kmax=200000, sig_decimals=2):
    rng = np.random.default_rng(seed)
    c = np.zeros(n, dtype=tb.CANDIDATE_DTYPE)
    c["series_id"] = rng.integers(0, nseries, n)
    c["template_id"] = rng.integers(0, 1000, n)
    c["log2_harm"] = rng.integers(0, 5, n)
    # clustered fundamentals: a few "pulsars" with harmonics, plus noise peaks
    f0 = rng.integers(50, kmax // 16, 24)
    pick = rng.integers(0, f0.size, n)
    harm = rng.integers(1, 9, n)
    k = f0[pick] * harm * (1 << c["log2_harm"].astype(np.int64)) // 1
    noise = rng.random(n) < 0.3
    k = np.where(noise, rng.integers(1, kmax, n), k + rng.integers(-3, 4, n))
    c["bin"] = np.clip(k, 1, None)
    c["sigma"] = np.round(rng.uniform(3.0, 30.0, n), sig_decimals)
    c["power"] = rng.uniform(10, 100, n).astype(np.float32)
    c["freq_hz"] = c["bin"] / (1 << c["log2_harm"].astype(np.int64)) / 537.0
    _, idx = np.unique(c[["series_id", "template_id", "log2_harm", "bin"]], return_index=True)
    return c[np.sort(idx)]


def _same(tb, c, **kw):
    kept, grp = tb.tb_distill(c, **kw)
    ko, go = oracle.distill(_to_oracle(c), **kw)
    assert len(kept) == len(ko)
    assert np.array_equal(_to_oracle(kept), ko)
    assert np.array_equal(grp.astype(np.int64), go)
    assert int(grp.sum()) == c.size
    return kept, grp


@pytest.mark.parametrize("seed,n,kw", [
    (1, 3000, dict()),
    (2, 3000, dict(max_ratio=1, tol=0)),
    (3, 4000, dict(max_ratio=8, tol=40, ppm=500)),
    (4, 2000, dict(max_ratio=64, tol=0, ppm=3000)),
    (5, 3000, dict(max_ratio=16, tol=16, ppm=1000)),
])
def test_library_grouping_equals_oracle(oracle_lib, tb, seed, n, kw):
    c = _lists(tb, seed, n, sig_decimals=1)  # many sigma ties
    kept, grp = _same(tb, c, **kw)
    assert 0 < len(kept) <= c.size


def test_edge_cases(oracle_lib, tb):
    D = tb.CANDIDATE_DTYPE
    empty = np.zeros(0, dtype=D)
    kept, grp = tb.tb_distill(empty)
    assert len(kept) == 0 and len(grp) == 0
    one = np.zeros(1, dtype=D)
    one["bin"], one["sigma"] = 5, 7.0
    _same(tb, one)
    # every record at the same fundamental, through every fold
    same = np.zeros(5, dtype=D)
    same["log2_harm"] = np.arange(5)
    same["bin"] = 100 << np.arange(5)
    same["sigma"] = [5, 9, 9, 1, 3]
    kept, grp = _same(tb, same, max_ratio=1, tol=0)
    assert len(kept) == 1 and grp[0] == 5 and kept[0]["log2_harm"] == 1
    # largest bins and tolerances: the integer test must not overflow
    big = np.zeros(6, dtype=D)
    big["bin"] = [0xFFFFFFFF, 0xFFFFFFF0, 0x7FFFFFFF, 0x80000000, 1, 2]
    big["sigma"] = [6, 5, 4, 3, 2, 1]
    _same(tb, big, max_ratio=64, tol=1 << 20, ppm=10**6)
    _same(tb, big, max_ratio=64, tol=0, ppm=0)


def test_input_order_and_rejects(oracle_lib, tb):
    c = _lists(tb, 9, 2000)
    a = tb.tb_distill(c, ppm=200)
    perm = np.random.default_rng(10).permutation(c.size)
    b = tb.tb_distill(c[perm], ppm=200)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    bad = c[:3].copy()
    bad["log2_harm"][1] = 5
    for arr, kw in [(bad, {}), (c[:3], dict(max_ratio=0)), (c[:3], dict(max_ratio=65)), (c[:3], dict(tol=(1 << 20) + 1)),
                    (c[:3], dict(ppm=10**6 + 1))]:
        with pytest.raises(tb.TbError) as e:
            tb.tb_distill(arr, **kw)
        assert e.value.status == tb.TB_ERR_INVALID_ARG
    nan = c[:3].copy()
    nan["sigma"][2] = np.nan
    with pytest.raises(tb.TbError):
        tb.tb_distill(nan)
