"""Dedispersion on the GPU (tb_dedisperse) against the oracle, bit for bit
(byte sums are exact), and dedispersion feeding the search."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from tests import parity_rules as R

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tb():
    import paper_2112_11991_amd as tb

    return tb


CASES = [
    # (nchan, nsamp, fch1, foff, tsamp, DMs): staged channels, a ragged last DM tile, descending band,
    # and delay spreads within a tile beyond the staging room (the global-memory path)
    (64, 30000, 1181.8, 0.390625, 256e-6, np.arange(0.0, 200.0, 7.0)),
    (100, 50000, 1581.4, -4.0, 64e-6, np.array([0.0, 3.3, 150.0, 151.0, 152.5, 400.0, 10.0])),
    (1024, 20000, 1181.804688, 0.390625, 256e-6, np.linspace(0.0, 300.0, 40)),
    (48, 60000, 300.0, 1.0, 1e-4, np.linspace(0.0, 60.0, 33)),
]


@pytest.mark.parametrize("nchan,nsamp,f1,df,ts,dms", CASES)
def test_dedispersion_matches_oracle_exactly(tb, nchan, nsamp, f1, df, ts, dms):
    import torch

    rng = np.random.default_rng(nchan)
    x = rng.integers(0, 256, (nsamp, nchan)).astype(np.uint8)
    want = oracle.dedisperse(x, f1, df, ts, dms)
    with tb.Plan() as plan:
        nout, _ = plan.dedisperse(x, f1, df, ts, dms)
        assert nout == want.shape[1]
        out = torch.empty(len(dms) * nout, dtype=torch.float32, device="cuda:0")
        torch.cuda.synchronize()
        _, ms = plan.dedisperse(x, f1, df, ts, dms, out=out.data_ptr())
        got = out.cpu().numpy().reshape(len(dms), nout)
        xd = torch.from_numpy(x).to("cuda:0")
        out2 = torch.empty_like(out)
        torch.cuda.synchronize()
        plan.dedisperse(xd.data_ptr(), f1, df, ts, dms, out=out2.data_ptr(), nchan=nchan, nsamp=nsamp)
        got2 = out2.cpu().numpy().reshape(len(dms), nout)
    _say("nchan %d nsamp %d ndm %d: %.3f ms" % (nchan, nsamp, len(dms), ms))
    assert np.array_equal(got, want)
    assert np.array_equal(got2, want)


def test_four_bit_filterbank_matches_oracle(tb):
    """4-bit samples (two channels per byte, even channel in the low nibble),
    Table 2's layout: host and device input, bit for bit against the oracle."""
    import torch

    nchan, nsamp, f1, df, ts = 256, 40000, 1181.804688, 0.390625, 256e-6
    dms = np.linspace(0.0, 150.0, 21)
    v = np.random.default_rng(8).integers(0, 16, (nsamp, nchan)).astype(np.uint8)
    packed = np.ascontiguousarray(v[:, 0::2] | (v[:, 1::2] << 4))
    want = oracle.dedisperse(packed, f1, df, ts, dms, nbits=4, nchan=nchan)
    assert np.array_equal(want, oracle.dedisperse(v, f1, df, ts, dms))
    with tb.Plan() as plan:
        nout, _ = plan.dedisperse(packed, f1, df, ts, dms, nchan=nchan, nbits=4)
        out = torch.empty(len(dms) * nout, dtype=torch.float32, device="cuda:0")
        torch.cuda.synchronize()
        plan.dedisperse(packed, f1, df, ts, dms, out=out.data_ptr(), nchan=nchan, nbits=4)
        got = out.cpu().numpy().reshape(len(dms), nout)
        pd = torch.from_numpy(packed).to("cuda:0")
        out2 = torch.empty_like(out)
        torch.cuda.synchronize()
        plan.dedisperse(pd.data_ptr(), f1, df, ts, dms, out=out2.data_ptr(), nchan=nchan, nsamp=nsamp, nbits=4)
        got2 = out2.cpu().numpy().reshape(len(dms), nout)
        with pytest.raises(tb.TbError):
            plan.dedisperse(packed[:, :3], f1, df, ts, dms, nchan=5, nbits=4)
    assert np.array_equal(got, want) and np.array_equal(got2, want)


def test_dedispersed_binary_pulsar_is_found(tb):
    """A 16-channel filterbank holding a binary pulsar dispersed at DM 60:
    dedispersed on the GPU, the DM-60 series is loaded straight from device
    memory and searched; the candidates match the oracle's dedisperse+search,
    the best is at the pulsar's frequency, and stronger than at DM 0."""
    import torch

    nchan, n, ts, f1, df = 16, 1 << 17, 256e-6, 1200.0, 12.5
    T = n * ts
    k0 = 1789
    orb = synth.Orbit(7200.0, 0.4, 1.0)
    rng = np.random.default_rng(12)
    dms = np.array([0.0, 30.0, 60.0, 90.0])
    f = f1 + df * np.arange(nchan)
    s = np.rint(oracle.dispersion_constant() * 60.0 * (1 / f ** 2 - 1 / f.max() ** 2) / ts).astype(int)
    pulse = synth.pulse_train(n + int(s.max()), ts, T / k0, 0.05, orb)
    x = np.empty((n + int(s.max()), nchan), np.float64)
    for c in range(nchan):
        x[:, c] = 100 + 12 * rng.standard_normal(x.shape[0])
        x[s[c]:, c] += 4.0 * pulse[: x.shape[0] - s[c]]
    x = np.clip(np.rint(x), 0, 255).astype(np.uint8)
    tms = [orb.as_template()[0].tolist(), (7200.0, 0.0, 1.0, 0.0, 0.0), (5000.0, 0.4, 2.0, 0.0, 0.0)]
    want = oracle.dedisperse(x, f1, df, ts, dms)
    with tb.Plan() as plan:
        nout, _ = plan.dedisperse(x, f1, df, ts, dms)
        out = torch.empty(len(dms) * nout, dtype=torch.float32, device="cuda:0")
        torch.cuda.synchronize()
        plan.dedisperse(x, f1, df, ts, dms, out=out.data_ptr())
        assert np.array_equal(out.cpu().numpy().reshape(len(dms), nout), want)
        nser = 1 << int(math.floor(math.log2(nout)))
        sid = plan.load_series(out.data_ptr() + 2 * nout * 4, ts, n=nser, flags=tb.TB_MEM_DEVICE)
        sid0 = plan.load_series(out.data_ptr(), ts, n=nser, flags=tb.TB_MEM_DEVICE)
        cg = plan.search(sid, tms)
        c0 = plan.search(sid0, tms)
    x0 = oracle.mean_subtract(want[2][:nser])
    co = oracle.search(x0, oracle.config(nser, ts), tms, series_id=int(sid))
    matched, _ = R.check_candidates(cg, co, [oracle.threshold(1 << l, 6.0) for l in range(5)])
    assert matched > 0
    # 33 s cover 0.5 % of the 2 h orbit, so the templates are nearly alike: the
    # pulsar is found at its frequency, and far better at its DM than at DM 0
    best = cg[np.argmax(cg["sigma"])]
    assert best["log2_harm"] == 4 and abs(best["freq_hz"] - k0 / T) < 2.0 / (nser * ts)
    assert best["sigma"] > (c0["sigma"].max() if len(c0) else 0.0) + 3.0


def test_dedispersion_argument_errors(tb):
    x = np.zeros((1000, 8), np.uint8)
    with tb.Plan() as plan:
        for args in [(1400.0, 1.0, 1e-3, [-1.0]), (1400.0, 1.0, 0.0, [1.0]), (10.0, -2.0, 1e-3, [1.0]),
                     (1400.0, -1.0, 1e-3, [1e6]), (1400.0, 1.0, 1e-3, [float("nan")])]:
            with pytest.raises(tb.TbError) as e:
                plan.dedisperse(x, *args)
            assert e.value.status == tb.TB_ERR_INVALID_ARG
