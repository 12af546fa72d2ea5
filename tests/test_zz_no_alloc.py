"""The allocation-free search (tb_search_templates_noalloc, for callers that
cannot allocate device memory) against tb_search_templates on the same plan:
identical candidate lists on calls in a row that share the fixed scratch, the
second with a shorter series and fewer templates; a series whitened once;
overflow of the caller's buffer; work beyond the scratch refused."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tb():
    import paper_2112_11991_amd as tb

    return tb


def test_noalloc_matches_search(tb):
    ts = 64e-6
    rng = np.random.default_rng(7007)
    big, small = 1 << 16, 1 << 14
    orb = synth.Orbit(700.0, 0.2, 1.3)
    x1 = synth.inject(rng.standard_normal(big), synth.pulse_train(big, ts, 0.009, 0.05, orb), 30.0)
    x2 = synth.inject(rng.standard_normal(small), synth.pulse_train(small, ts, 0.007, 0.05, orb), 30.0)
    t1 = np.concatenate([synth.uniform_templates(rng, 39, (0.1, 0.4), (0.0, 0.4)), orb.as_template()])
    t2 = t1[-9:]
    _say("noalloc: 2^16 x 40 templates, then 2^14 x 9")
    with tb.Plan(threshold_sigma=4.5, whiten_window=1024, batch_templates=16) as plan:
        s1 = plan.load_series(x1.astype(np.float32), ts)
        s2 = plan.load_series(x2.astype(np.float32), ts)
        s3 = plan.load_series(x2.astype(np.float32), ts, flags=tb.TB_SERIES_WHITENING)
        ref1 = plan.search(s1, t1, first_template_id=5)
        ref2 = plan.search(s2, t2, first_template_id=77)
        ref3 = plan.search(s3, t2)
        got1, n1 = plan.search_noalloc(s1, t1, first_template_id=5)
        got2, n2 = plan.search_noalloc(s2, t2, first_template_id=77)
        got3, n3 = plan.search_noalloc(s3, t2)
        _say("  candidates %d, %d, %d" % (n1, n2, n3))
        assert n1 == len(ref1) > 0 and np.array_equal(got1, ref1)
        assert n2 == len(ref2) > 0 and np.array_equal(got2, ref2)
        assert n3 == len(ref3) > 0 and np.array_equal(got3, ref3)
        # a buffer smaller than the list: exact count, records a sorted subset
        few, nf = plan.search_noalloc(s1, t1, first_template_id=5, capacity=7, allow_overflow=True)
        assert nf == n1 and len(few) == 7
        key = lambda c: (int(c["template_id"]), int(c["log2_harm"]), int(c["bin"]))
        assert set(map(key, few)) <= set(map(key, ref1))
        assert [key(c) for c in few] == sorted(key(c) for c in few)
        with pytest.raises(tb.TbError) as e:
            plan.search_noalloc(s1, t1, capacity=7)
        assert e.value.status == tb.TB_ERR_OVERFLOW
        # more templates than the scratch holds (each takes 248 bytes there): refused
        # before any work
        many = np.repeat(t2[:1], tb.TB_NOALLOC_SCRATCH_BYTES // 200)
        with pytest.raises(tb.TbError) as e:
            plan.search_noalloc(s2, many)
        assert e.value.status == tb.TB_ERR_TOO_LARGE
        # the plan still works afterwards
        again, _ = plan.search_noalloc(s2, t2, first_template_id=77)
        assert np.array_equal(again, ref2)


def test_noalloc_largest_series(tb):
    """A 2^24-sample series, the longest a plan takes: one template's
    workspace (about 128 MiB) fits the fixed scratch; results equal
    tb_search_templates'."""
    n, ts = 1 << 24, 256e-6
    rng = np.random.default_rng(7008)
    orb = synth.Orbit(8 * 3600.0, 3.0, 1.0, 0.08, 2.0)
    x = synth.inject(rng.standard_normal(n), synth.pulse_train(n, ts, 0.03, 0.05, orb), 20.0).astype(np.float32)
    tms = np.concatenate([orb.as_template(), synth.uniform_templates(rng, 2, (5.0, 20.0), (0.0, 6.0), ecc_max=0.1)])
    _say("noalloc: 2^24 x 3 templates")
    with tb.Plan(threshold_sigma=5.0) as plan:
        sid = plan.load_series(x, ts)
        ref = plan.search(sid, tms)
        got, n_tot = plan.search_noalloc(sid, tms)
    _say("  candidates %d" % n_tot)
    assert n_tot == len(ref) > 0 and np.array_equal(got, ref)
