"""Host-side bank calls of the library (no GPU): the template count of a
random bank and the rejection step, against the oracle's."""
import math

import numpy as np
import pytest

from oracle import bank as obank


@pytest.fixture(scope="module")
def tb():
    import paper_2112_11991_amd as tb

    return tb


@pytest.mark.parametrize("n", [3, 5])
def test_template_count_matches_oracle(tb, n):
    for V in (50.0, 1e4, 3.3e6):
        for cov, mis in ((0.9, 0.2), (0.5, 0.05), (0.99, 0.3)):
            got = tb.tb_bank_count(V, n, cov, mis)
            want = obank.n_random(V, n, cov, mis)
            want = want[0] if isinstance(want, tuple) else want
            assert abs(got / want - 1.0) <= 1e-12, (V, n, cov, mis, got, want)


def test_template_count_rejects_bad_arguments(tb):
    for args in ((0.0, 3, 0.9, 0.2), (10.0, 3, 1.0, 0.2), (10.0, 3, 0.9, 0.0), (10.0, 0, 0.9, 0.2),
                 (1e-3, 3, 0.9, 0.2)):  # the last: one template cell is larger than the volume
        with pytest.raises(tb.TbError) as e:
            tb.tb_bank_count(*args)
        assert e.value.status == tb.TB_ERR_INVALID_ARG


def test_selection_matches_oracle(tb):
    rng = np.random.default_rng(3)
    dens = rng.exponential(1.0, 5000)
    q = rng.uniform(0.5, 2.0, 5000)
    u = rng.uniform(0.0, 1.0, 5000)
    w = dens / q
    for wmax in (float(w.max()), float(np.quantile(w, 0.8))):
        kept, nk, na = tb.tb_bank_select(w, u, wmax)
        assert np.array_equal(kept, obank.select(dens, q, u, wmax))
        assert nk == kept.size and na == int((w > wmax).sum())
    with pytest.raises(tb.TbError):
        tb.tb_bank_select(w, u, 0.0)
