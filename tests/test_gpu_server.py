"""GPU parity of the serving loop: every request's bits against the oracle
(the concatenated hashes of the blocks it was given, cut to R bits, with the
window's own estimate deciding m_s), the same bits whether a request was
batched with others or served alone, admission by output-ring memory, and
the error paths."""
import math

import numpy as np
import pytest

import oracle
import qrng_inputs as qi

pytestmark = pytest.mark.gpu

W = 1 << 16          # samples per window
NS = 4096            # serving block length (bits)
SIGMAS = [20.0, 8.0, 33.0, 14.0, 20.0, 26.0]


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


@pytest.fixture(scope="module")
def windows():
    return [qi.gen_adc(W, s, seed=700 + k) for k, s in enumerate(SIGMAS)]


@pytest.fixture(scope="module")
def seed(torch, ctx):
    sw = qi.gen_seed_words(1 << 19, 4711)
    t = torch.from_numpy(sw.view(np.int64).copy()).to("cuda:0")
    sid = ctx.register_seed(t, 1 << 19)
    yield sid, sw
    ctx.unregister_seed(sid)


def log(msg):
    print(msg, flush=True)


def m_block(samples, n, eps=0.0):
    r = oracle.minentropy_counts(oracle.histogram(samples, 8), 8)
    return oracle.output_bits(n, 8, r["h_mod"], eps) // 64 * 64


def want_bits(windows, sw, served, n):
    """The oracle's output for one served request."""
    x = qi.samples_as_words(windows[served["window"]])
    m = served["m_block"]
    parts = []
    for b in range(served["first_block"], served["first_block"] + served["blocks"]):
        y = oracle.toeplitz_packed(x[b * n // 64:(b + 1) * n // 64], n, sw, m)
        parts.append(oracle.unpack_bits(y, m))
    bits = np.concatenate(parts)[: served["bits"]]
    return oracle.pack_bits(bits)


def serve_all(torch, srv, windows, sizes, release=True, max_iter=10000):
    """Submit all sizes, drive the loop, return {id: (served, bits words)}."""
    ids = [srv.submit(int(r)) for r in sizes]
    out, fed = {}, 0
    while fed < 2 and fed < len(windows):
        srv.feed(torch.from_numpy(windows[fed]).to("cuda:0"))
        fed += 1
    for _ in range(max_iter):
        if len(out) == len(ids):
            break
        adm = srv.step()
        got = srv.poll()
        for s in got:
            words = None
            if s["status"] == 0:
                words = srv.read(s["request_id"], s["bits"]).cpu().numpy().view(np.uint64)
                if release:
                    srv.release(s["request_id"])
            out[s["request_id"]] = (s, words)
        st = srv.stats()
        if not got and adm == 0 and st["in_flight"] == 0 and st["queued"]:
            assert fed < len(windows), "ran out of windows"
            if srv.try_feed(torch.from_numpy(windows[fed]).to("cuda:0")):
                fed += 1
        torch.cuda.synchronize()
    assert len(out) == len(ids)
    return ids, out


def test_server_requests_match_oracle(torch, ctx, windows, seed):
    sid, sw = seed
    rng = np.random.default_rng(3)
    sizes = np.floor(2.0 ** rng.uniform(3, 16, 40)).astype(np.int64)
    sizes[:4] = [1, 63, 64, 2560]
    with ctx.server(sid, W, block_bits=NS, ring_bits=1 << 22, window_slots=3) as srv:
        ids, out = serve_all(torch, srv, windows, sizes)
        stats = srv.stats()
    assert stats["bits_served"] == int(sizes.sum())
    seen = set()
    for rid, r in zip(ids, sizes):
        s, words = out[rid]
        assert s["status"] == 0 and s["bits"] == r
        assert s["m_block"] == m_block(windows[s["window"]], NS)
        assert s["blocks"] == -(-int(r) // s["m_block"])
        blk = set(range(s["first_block"], s["first_block"] + s["blocks"]))
        key = [(s["window"], b) for b in blk]
        assert not seen.intersection(key), "block handed out twice"
        seen.update(key)
        assert np.array_equal(words, want_bits(windows, sw, s, NS)), "request %d" % rid


def test_server_bits_alone_equal_bits_in_a_mix(torch, ctx, windows, seed):
    """Request X batched with others and X served alone on the same blocks
    receive the same bits."""
    sid, sw = seed
    mix = [3000, 70000, 12345, 5000, 256, 40000]
    with ctx.server(sid, W, block_bits=NS, ring_bits=1 << 22, window_slots=3) as srv:
        ids, out = serve_all(torch, srv, windows, mix)
    x, xwords = out[ids[2]]
    assert x["first_block"] > 0
    # alone: a filler request takes exactly the blocks before X's, then X
    # is submitted by itself once the filler is done
    with ctx.server(sid, W, block_bits=NS, ring_bits=1 << 22, window_slots=3) as srv:
        # whole windows before X's window, then the blocks before X's
        fill = [m_block(windows[k], NS) * (W * 8 // NS) for k in range(x["window"])]
        fill.append(x["first_block"] * x["m_block"])
        _, fout = serve_all(torch, srv, windows, fill)
        ids2 = [srv.submit(int(x["bits"]))]
        for _ in range(1000):
            srv.step()
            got = srv.poll()
            if got:
                s2 = got[0]
                w2 = srv.read(s2["request_id"], s2["bits"]).cpu().numpy().view(np.uint64)
                break
            torch.cuda.synchronize()
        else:
            raise AssertionError("request not served")
    assert (s2["window"], s2["first_block"], s2["blocks"]) == \
        (x["window"], x["first_block"], x["blocks"])
    assert np.array_equal(w2, xwords)
    assert np.array_equal(xwords, want_bits(windows, sw, x, NS))


def test_server_admission_by_ring_memory(torch, ctx, windows, seed):
    """A ring that holds a few requests: later ones wait until space is
    released, and reused ring space never corrupts an unread output."""
    sid, sw = seed
    m = m_block(windows[0], NS)
    ring = 3 * 4 * m                        # about three 4-block requests
    sizes = [4 * m - 5] * 9 + [m * 2]
    with ctx.server(sid, W, block_bits=NS, ring_bits=ring, window_slots=3) as srv:
        ids = [srv.submit(r) for r in sizes]
        srv.feed(torch.from_numpy(windows[0]).to("cuda:0"))
        srv.feed(torch.from_numpy(windows[1]).to("cuda:0"))
        first = srv.step()
        assert 1 <= first <= 3, first
        torch.cuda.synchronize()
        held, done = [], {}
        for _ in range(2000):
            for s in srv.poll():
                w = srv.read(s["request_id"], s["bits"]).cpu().numpy().view(np.uint64)
                done[s["request_id"]] = (s, w)
                held.append(s["request_id"])
            if len(held) >= 2 or (held and len(done) == len(ids)):
                srv.release(held.pop(0))    # release late: space comes back in order
            srv.step()
            torch.cuda.synchronize()
            if len(done) == len(ids):
                break
    assert len(done) == len(ids)
    for rid in ids:
        s, w = done[rid]
        assert np.array_equal(w, want_bits(windows, sw, s, NS)), "request %d" % rid


def test_server_request_larger_than_a_window_fails(torch, ctx, windows, seed):
    sid, sw = seed
    with ctx.server(sid, W, block_bits=NS, ring_bits=1 << 24, window_slots=2) as srv:
        big = srv.submit(W * 8 * 8)            # more than a window can give
        small = srv.submit(100)
        srv.feed(torch.from_numpy(windows[0]).to("cuda:0"))
        res = {}
        for _ in range(100):
            srv.step()
            for s in srv.poll():
                res[s["request_id"]] = s
            torch.cuda.synchronize()
            if len(res) == 2:
                break
        assert res[big]["status"] == -4        # EUNSUPPORTED
        assert res[small]["status"] == 0


def test_server_chooses_block_length(torch, ctx, windows, seed):
    sid, sw = seed
    with ctx.server(sid, W, block_bits=0, ring_bits=1 << 24, window_slots=2) as srv:
        st = srv.stats()
        n = st["block_bits"]
        assert n in [1 << k for k in range(12, 19)] and (W * 8) % n == 0
        ids, out = serve_all(torch, srv, windows, [1000, 20000])
        for rid in ids:
            s, w = out[rid]
            assert np.array_equal(w, want_bits(windows, sw, s, n))


def test_server_config_and_feed_errors(torch, ctx, windows, seed):
    import paper_2011_04130_amd as q
    sid, sw = seed
    for kw in (dict(block_bits=1000), dict(ring_bits=100), dict(window_slots=1),
               dict(block_bits=3 * 512 * 1024)):
        with pytest.raises(q.QrngError):
            ctx.server(sid, W, **kw)
    with pytest.raises(q.QrngError):
        ctx.server(sid + 999, W, block_bits=NS)
    with ctx.server(sid, W, block_bits=NS, ring_bits=1 << 20, window_slots=2) as srv:
        t = torch.from_numpy(windows[0]).to("cuda:0")
        assert srv.try_feed(t) and srv.try_feed(t)
        assert not srv.try_feed(t)            # both slots hold unused windows
        with pytest.raises(q.QrngError):
            srv.submit(0)
        with pytest.raises(q.QrngError):
            ctx.unregister_seed(sid)          # pinned by the live server


def test_server_vector_calls(torch, ctx, windows, seed):
    """submit_many / poll_array / release_many serve the same bits as the
    one-at-a-time calls."""
    sid, sw = seed
    sizes = [5000, 12, 30000, 2560, 777]
    with ctx.server(sid, W, block_bits=NS, ring_bits=1 << 22, window_slots=3) as srv:
        ids = srv.submit_many(sizes)
        assert list(ids) == sorted(ids) and len(ids) == len(sizes)
        srv.feed(torch.from_numpy(windows[0]).to("cuda:0"))
        done = {}
        for _ in range(1000):
            srv.step()
            got = srv.poll_array()
            for r in got:
                s = {k: int(r[k]) for k in got.dtype.names}
                done[s["request_id"]] = (s, srv.read(s["request_id"], s["bits"]).cpu().numpy()
                                         .view(np.uint64))
            srv.release_many(got["request_id"])
            torch.cuda.synchronize()
            if len(done) == len(sizes):
                break
        assert srv.stats()["ring_free_bits"] == 1 << 22
    for rid in ids:
        s, w = done[int(rid)]
        assert np.array_equal(w, want_bits(windows, sw, s, NS))


def test_server_full_size_windows(torch, ctx):
    """Windows of 2^24 samples (the serving workload's size) with the block
    length chosen by timing: requests of log-uniform size served in a mix,
    each checked against the oracle (whole requests up to 2^18 bits, the
    first and last block of larger ones)."""
    cfg = qi.config(4)
    Wf = cfg["window_samples"]
    wins = [qi.gen_adc(Wf, cfg["sigma"], seed=cfg["adc_seed"] + k) for k in range(2)]
    L = 1 << 19
    sw = qi.gen_seed_words(L, cfg["seed_seed"])
    sid = ctx.register_seed(torch.from_numpy(sw.view(np.int64).copy()).to("cuda:0"), L)
    try:
        with ctx.server(sid, Wf, block_bits=0, ring_bits=1 << 30, window_slots=2) as srv:
            n = srv.stats()["block_bits"]
            log("full-size serving, n_s=%d" % n)
            sizes = qi.request_sizes(60, cfg["r_log2_min"], cfg["r_log2_max"], cfg["arrival_seed"])
            ids, out = serve_all(torch, srv, wins, sizes)
        rng = np.random.default_rng(1)
        for rid in rng.choice(ids, 12, replace=False):
            s, w = out[rid]
            assert s["status"] == 0
            assert s["m_block"] == m_block(wins[s["window"]], n)
            if s["bits"] <= (1 << 18):
                assert np.array_equal(w, want_bits(wins, sw, s, n)), "request %d" % rid
            else:
                x = qi.samples_as_words(wins[s["window"]])
                mb = s["m_block"]
                bits = oracle.unpack_bits(w, s["bits"])
                for j in (0, s["blocks"] - 1):
                    b = s["first_block"] + j
                    yb = oracle.toeplitz_packed(x[b * n // 64:(b + 1) * n // 64], n, sw, mb)
                    want = oracle.unpack_bits(yb, mb)
                    lo = j * mb
                    hi = min(lo + mb, s["bits"])
                    assert np.array_equal(bits[lo:hi], want[:hi - lo]), "request %d" % rid
    finally:
        ctx.unregister_seed(sid)
