"""Per-length launch shapes (tb_set_shape) and the autotuner that picks them
by timing the search on the device."""
import numpy as np
import pytest

import oracle
import synth
from tests import parity_rules as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tb():
    import paper_2112_11991_amd as tb

    return tb


def test_shape_rules(tb):
    with tb.Plan() as plan:
        for bad in [(9, 0, 0), (25, 0, 0), (17, 4096, 0), (17, 0, 5000)]:
            with pytest.raises(tb.TbError) as e:
                plan.set_shape(*bad)
            assert e.value.status == tb.TB_ERR_INVALID_ARG
        plan.set_shape(17, 16384, 3)
        plan.set_shape(17, 8192, 5)  # may change until the length is used
        plan.load_series(np.zeros(1 << 17, np.float32), 64e-6)
        with pytest.raises(tb.TbError):
            plan.set_shape(17, 16384, 3)
        plan.set_shape(18, 16384, 0)


@pytest.mark.parametrize("tile,batch", [(16384, 3), (8192, 1), (8192, 130)])
def test_shaped_search_matches_oracle(tb, tile, batch):
    """The tiny configuration under non-default shapes: one-template waves,
    ragged waves, 16384-point tiles; candidates match the oracle's."""
    w = synth.c1_tiny()
    x, ts = w.series[0], w.tsamp
    n = x.size
    with tb.Plan() as plan:
        plan.set_shape(17, tile, batch)
        sid = plan.load_series(x, ts)
        cg = plan.search(sid, w.templates)
    co = oracle.search(oracle.mean_subtract(x), oracle.config(n, ts), w.templates, series_id=int(sid))
    matched, _ = R.check_candidates(cg, co, [oracle.threshold(1 << l, 6.0) for l in range(5)])
    assert matched > 0


def test_autotune_picks_a_measured_shape(tb):
    from paper_2112_11991_amd import tune

    tuned = tune.autotune([14, 16], tiles=(8192, 16384), batches=(4, 16), reps=1, work=1 << 22)
    assert set(tuned) == {14, 16}
    for lg, r in tuned.items():
        assert len(r["tried"]) == 4 and r["templates_per_s"] == max(t["templates_per_s"] for t in r["tried"])
        assert r["tile_points"] in (8192, 16384) and r["batch_templates"] in (4, 16)
    with tb.Plan() as plan:
        tune.apply(plan, tuned)
        sid = plan.load_series(np.random.default_rng(0).standard_normal(1 << 16).astype(np.float32), 64e-6)
        plan.search(sid, [(3600.0, 0.1, 0.0, 0.0, 0.0)] * 5)
