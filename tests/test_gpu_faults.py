"""Failure handling forced from the host (QRNG_FAULT, read by the library on
every call; no kernel is made to fail): an injected launch failure returns
QRNG_EDEVICE with nothing enqueued and leaves the context usable; a stale
estimate ticket (a launch that never completed) does not silence or corrupt
the next estimate; partial histograms that fail the finish's consistency
check make the estimate fail closed (m = 0, no output bits)."""
import ctypes
import math
import os

import numpy as np
import pytest

import oracle
import qrng_inputs as qi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a ROCm GPU"
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    import paper_2011_04130_amd as q
    c = q.Context(0)
    yield c
    c.close()


@pytest.fixture
def fault():
    def set_(mode):
        if mode is None:
            os.environ.pop("QRNG_FAULT", None)
        else:
            os.environ["QRNG_FAULT"] = mode
    yield set_
    os.environ.pop("QRNG_FAULT", None)


def dev(torch, words):
    return torch.from_numpy(np.ascontiguousarray(words).view(np.int64).copy()).to("cuda:0")


def test_injected_launch_failure(torch, ctx, fault):
    import paper_2011_04130_amd as q
    n, m = 100000, 60000
    xw, sw = qi.gen_bits(n, 1), qi.gen_seed_words(n + m - 1, 2)
    x, s = dev(torch, xw), dev(torch, sw)
    y = torch.full(((m + 63) // 64,), 7, dtype=torch.int64, device="cuda:0")
    samples = torch.from_numpy(qi.gen_adc(1 << 16, 20.0, seed=3)).to("cuda:0")
    fault("launch")
    for call in (lambda: ctx.hash(x, n, s, m, y=y, path=q.PATH_NTT),
                 lambda: ctx.hash(x, n, s, m, y=y, path=q.PATH_DIRECT),
                 lambda: ctx.minentropy(samples)):
        with pytest.raises(q.QrngError) as e:
            call()
        assert e.value.status == -3 and "injected" in str(e.value)
    torch.cuda.synchronize()
    assert (y.cpu() == 7).all()                     # nothing was enqueued
    fault(None)                                      # the context still works
    ctx.hash(x, n, s, m, y=y, path=q.PATH_NTT)
    assert np.array_equal(y.cpu().numpy().view(np.uint64), oracle.toeplitz_packed(xw, n, sw, m))


def _extract_case(torch, ctx):
    """The n = 2^23 workload block through qrng_extract (the estimate runs
    inside the transform's first pass and finishes by ticket)."""
    from paper_2011_04130_amd._lib import MeResult
    c = qi.config(1)
    s = qi.gen_adc(c["S"], c["sigma"], seed=c["adc_seed"])
    n = c["n"]
    sw = qi.gen_seed_words(2 * n - 1, c["seed_seed"])
    sid = ctx.register_seed(dev(torch, sw), 2 * n - 1)
    st = torch.from_numpy(s).to("cuda:0")
    rs = ctypes.sizeof(MeResult)

    def run():
        me = torch.zeros(rs, dtype=torch.uint8, device="cuda:0")
        mo = torch.full((1,), -1, dtype=torch.int64, device="cuda:0")
        y = ctx.extract(st, sid, n, m_out=mo, me_out=me)
        torch.cuda.synchronize()
        return int(mo.item()), ctx.me_result_from_bytes(me), y.cpu().numpy().view(np.uint64)
    return c, sid, run


def test_stale_ticket_does_not_silence_the_estimate(torch, ctx, fault):
    c, sid, run = _extract_case(torch, ctx)
    try:
        m0, me0, y0 = run()
        assert m0 == c["m_expected"]
        fault("ticket")
        for _ in range(2):
            m1, me1, y1 = run()
            assert m1 == m0 and me1["h_mod"] == me0["h_mod"] and me1["samples"] == c["S"]
            assert np.array_equal(y1, y0)
        fault(None)
        m2, _, y2 = run()
        assert m2 == m0 and np.array_equal(y2, y0)
    finally:
        ctx.unregister_seed(sid)


def test_failed_consistency_check_fails_closed(torch, ctx, fault):
    import paper_2011_04130_amd as q
    c, sid, run = _extract_case(torch, ctx)
    try:
        m0, me0, y0 = run()
        fault("rows")
        m1, me1, y1 = run()
        assert m1 == 0 and me1["samples"] == 0 and math.isnan(me1["h_mod"])
        assert not y1.any()                          # no output bits
        with pytest.raises(q.QrngError) as e:
            ctx.minentropy(torch.from_numpy(qi.gen_adc(1 << 16, 20.0, seed=4)).to("cuda:0"))
        assert e.value.status == -3 and "consistency" in str(e.value)
        fault(None)
        m2, me2, y2 = run()
        assert m2 == m0 and me2["h_mod"] == me0["h_mod"] and np.array_equal(y2, y0)
    finally:
        ctx.unregister_seed(sid)


def test_extract_graph_replays_and_eager_calls_interleaved(torch, ctx):
    """A captured qrng_extract carries one tag for every replay, while eager
    calls between the replays move the context's tag on: each replay then
    finds another call's tag on the ticket and must start its count afresh;
    every replay and every eager call gives the same m and bits."""
    c, sid, run = _extract_case(torch, ctx)
    try:
        m0, me0, y0 = run()
        assert m0 == c["m_expected"]
        st = torch.from_numpy(qi.gen_adc(c["S"], c["sigma"], seed=c["adc_seed"])).to("cuda:0")
        n = c["n"]
        y = torch.zeros((n + 63) // 64, dtype=torch.int64, device="cuda:0")
        mo = torch.full((1,), -1, dtype=torch.int64, device="cuda:0")
        ctx.extract(st, sid, n, y=y, m_out=mo)       # warm-up: workspaces exist before capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            ctx.extract(st, sid, n, y=y, m_out=mo)
        for k in range(3):
            y.zero_()
            mo.fill_(-1)
            g.replay()
            torch.cuda.synchronize()
            assert int(mo.item()) == m0, "replay %d" % k
            assert np.array_equal(y.cpu().numpy().view(np.uint64), y0), "replay %d" % k
            for _ in range(k + 1):                   # eager calls move the tag on
                m1, _, y1 = run()
                assert m1 == m0 and np.array_equal(y1, y0)
    finally:
        ctx.unregister_seed(sid)
