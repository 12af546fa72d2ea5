"""Lanes and the continuous-batching loop: every request's result is the same
alone and in the mix, also when the HBM budget makes requests wait."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tb():
    import paper_2112_11991_amd as tb

    return tb


def _pool():
    rng = np.random.default_rng(501)
    lens = [1 << 15, 1 << 16, 1 << 17]
    series = []
    for i, n in enumerate(lens):
        x = rng.standard_normal(n)
        if i == 1:
            x = synth.inject(x, synth.pulse_train(n, 64e-6, 0.009, 0.05, synth.Orbit(900.0, 0.2, 1.0)), 30.0)
        series.append(x.astype(np.float32))
    return lens, series


def _trace(n_req=12, seed=502):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n_req):
        cnt = int(rng.integers(16, 160))
        if rng.uniform() < 0.3:
            tm = synth.uniform_templates(rng, cnt, (0.3, 2.0), (0.0, 0.5), ecc_max=0.1)
        else:
            tm = synth.uniform_templates(rng, cnt, (0.3, 2.0), (0.0, 0.5))
        reqs.append((float(i) * 0.002, int(rng.integers(0, 3)), tm, 10000 * i))
    return reqs


def _alone(tb, series, reqs):
    out = []
    with tb.Plan(fmin_hz=2.0, ring_capacity=1 << 16) as plan:
        sids = [plan.load_series(x, 64e-6) for x in series]
        for _, s, tm, first in reqs:
            out.append(plan.search(sids[s], tm, first_template_id=first))
    return out


def test_lanes_give_identical_results(tb):
    lens, series = _pool()
    reqs = _trace()
    ref = _alone(tb, series, reqs)
    with tb.Plan(fmin_hz=2.0, ring_capacity=1 << 16, lanes=3) as plan:
        sids = [plan.load_series(x, 64e-6) for x in series]
        rids = [plan.submit(sids[s], tm, first) for _, s, tm, first in reqs]
        got = []
        for rid in rids:
            c, _ = plan.candidates(rid)
            plan.release(rid)
            got.append(c)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("tight_budget", [False, True])
def test_served_results_equal_alone(tb, tight_budget):
    from paper_2112_11991_amd.serve import Request, serve

    lens, series = _pool()
    reqs = _trace(n_req=16, seed=503)
    ref = _alone(tb, series, reqs)
    with tb.Plan(fmin_hz=2.0, ring_capacity=1 << 16, lanes=2) as plan:
        sids = [plan.load_series(x, 64e-6) for x in series]
        if tight_budget:
            # give both lanes their workspaces for every length, then leave room
            # for about two requests in flight
            warm = [plan.submit(sid, reqs[0][2][:2]) for sid in sids for _ in range(2)]
            for rid in warm:
                plan.candidates(rid)
                plan.release(rid)
            held, _ = plan.memory()
            plan.set_budget(held + int(2.5 * ((1 << 16) * 16 + 32768)))
        rq = [Request(t, s, tm, first) for t, s, tm, first in reqs]
        rep = serve(plan, sids, lens, rq, realtime=False)
    assert rep.n_requests == len(reqs)
    if tight_budget:
        assert rep.budget_waits > 0 and rep.max_in_flight <= 2
    for r, a in zip(rq, ref):
        assert np.array_equal(r.candidates, a)


def test_one_request_spread_over_idle_lanes(tb):
    """A request of many waves on a plan whose other lanes are idle runs its
    waves on all of them; the candidates are those of a single-lane plan."""
    lens, series = _pool()
    rng = np.random.default_rng(504)
    tm = synth.uniform_templates(rng, 61, (0.3, 2.0), (0.0, 0.5), ecc_max=0.05)
    out = []
    for lanes in (1, 3):
        with tb.Plan(fmin_hz=2.0, ring_capacity=1 << 16, lanes=lanes, batch_templates=8) as plan:
            sid = plan.load_series(series[1], 64e-6)
            out.append(plan.search(sid, tm, first_template_id=7))
            out.append(plan.search(sid, tm[:5], first_template_id=500))
    assert np.array_equal(out[0], out[2])
    assert np.array_equal(out[1], out[3])


def test_profile_samples_every_kth_wave(tb):
    lens, series = _pool()
    rng = np.random.default_rng(505)
    tm = synth.uniform_templates(rng, 80, (0.3, 2.0), (0.0, 0.5))
    with tb.Plan(fmin_hz=2.0, batch_templates=8) as plan:
        sid = plan.load_series(series[0], 64e-6)
        plan.profile(3)
        plan.search(sid, tm)  # 10 waves of 8: waves 0, 3, 6, 9 are timed
        ms, launches, ntemp = plan.profile_read()
        plan.profile(0)
    # block medians and whitening run as one kernel, timed as class 3
    assert list(launches) == [4, 4, 4, 4, 0, 4]
    assert ntemp == 32
    assert (ms[[0, 1, 2, 3, 5]] > 0).all() and ms[4] == 0


def test_serve_realtime_order_and_shared_capacity(tb):
    """tb_serve on a real-time trace (arrivals 2 ms apart): no request is
    admitted before it arrives or finishes before it is admitted, and every
    request's records equal its result alone.  With an output array of half
    the records, requests are filled in completion order until it is full:
    each keeps a prefix of its sorted records and those cut short report
    TB_ERR_OVERFLOW with the exact count."""
    lens, series = _pool()
    reqs = _trace(n_req=12, seed=506)
    ref = _alone(tb, series, reqs)
    total = sum(r.size for r in ref)
    with tb.Plan(fmin_hz=2.0, ring_capacity=1 << 16, lanes=2) as plan:
        sids = [plan.load_series(x, 64e-6) for x in series]
        rq = [(t, sids[s], tm, first) for t, s, tm, first in reqs]
        res, cands, (most, waits) = plan.serve(rq)
        assert waits == 0 and most >= 1
        arrival = np.array([t for t, *_ in reqs])
        assert np.all(res["t_admit_s"] >= arrival) and np.all(res["t_done_s"] >= res["t_admit_s"])
        assert np.all(res["status"] == tb.TB_OK) and cands.size == total
        for o, a in zip(res, ref):
            got = cands[int(o["cand_offset"]):int(o["cand_offset"] + o["n_copied"])]
            assert o["n_total"] == a.size and np.array_equal(got, a)

        cap = total // 2
        res, cands, _ = plan.serve(rq, saturate=True, capacity=cap)
    assert cands.size == cap and int(res["n_copied"].sum()) == cap
    short = 0
    for o, a in zip(res, ref):
        got = cands[int(o["cand_offset"]):int(o["cand_offset"] + o["n_copied"])]
        assert o["n_total"] == a.size and np.array_equal(got, a[:got.size])
        assert (o["status"] == tb.TB_ERR_OVERFLOW) == (got.size < a.size)
        short += got.size < a.size
    assert short >= 1


def test_serve_stops_on_an_error_and_releases(tb):
    """A request naming an unknown series ends the stream with that error;
    requests already admitted are waited for and released, and the same plan
    then serves the valid requests with every result equal to its result
    alone."""
    lens, series = _pool()
    reqs = _trace(n_req=6, seed=507)
    ref = _alone(tb, series, reqs)
    with tb.Plan(fmin_hz=2.0, ring_capacity=1 << 16, lanes=2) as plan:
        sids = [plan.load_series(x, 64e-6) for x in series]
        rq = [(0.0, sids[s], tm, first) for _, s, tm, first in reqs]
        bad = list(rq)
        bad[3] = (0.0, 999, rq[3][2], rq[3][3])
        with pytest.raises(tb.TbError) as e:
            plan.serve(bad, saturate=True)
        assert e.value.status == tb.TB_ERR_UNKNOWN_ID
        res, cands, _ = plan.serve(rq, saturate=True)
    assert np.all(res["status"] == tb.TB_OK)
    for o, a in zip(res, ref):
        assert np.array_equal(cands[int(o["cand_offset"]):int(o["cand_offset"] + o["n_copied"])], a)
