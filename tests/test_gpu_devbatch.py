"""GPU parity of batches described in device memory
(qrng_toeplitz_hash_batched with blocks_dev and seed_ids_or_null): uneven
blocks over every transform length up to 2^20 bits against the oracle, the
per-block seed-id array, descriptors that fail a check, and the call captured
in a HIP graph and replayed with new descriptors and raw bits written on the
device between replays."""
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


def dev(torch, words):
    return torch.from_numpy(np.ascontiguousarray(words).view(np.int64).copy()).to("cuda:0")


def host(t):
    return t.cpu().numpy().view(np.uint64)


def log(msg):
    print(msg, flush=True)


def layout(ns, ms, sids):
    """Raw blocks back to back, outputs with one guard word before each."""
    rows, xo, yo = [], 0, 1
    for n, m, sid in zip(ns, ms, sids):
        rows.append((xo, int(n), int(m), yo, int(sid)))
        xo += (int(n) + 63) // 64
        yo += (int(m) + 63) // 64 + 1
    return rows, xo, yo


def check(rows, xw, seeds, got, skip=()):
    for b, (xo, n, m, yo, sid) in enumerate(rows):
        nw = (m + 63) // 64
        assert got[yo - 1] == np.uint64(2 ** 64 - 1), "block %d: guard word written" % b
        if b in skip or m == 0:
            assert (got[yo:yo + nw] == np.uint64(2 ** 64 - 1)).all(), "block %d written" % b
            continue
        want = oracle.toeplitz_packed(xw[xo:xo + (n + 63) // 64], n, seeds[sid], m)
        assert np.array_equal(got[yo:yo + nw], want), "block %d (n=%d m=%d)" % (b, n, m)


@pytest.fixture(scope="module")
def seeds3(torch, ctx):
    """Three registered seeds of different lengths (longest 2^21 bits)."""
    lens = [1 << 21, 300001, 5000]
    sids, words = [], {}
    for g, L in enumerate(lens):
        w = qi.gen_seed_words(L, 700 + g)
        sid = ctx.register_seed(dev(torch, w), L)
        sids.append(sid)
        words[sid] = w
    yield sids, lens, words
    for sid in sids:
        ctx.unregister_seed(sid)


def uneven(rng, nb, sids, lens):
    ns, ms, ss = [], [], []
    for b in range(nb):
        g = b % 3
        L = lens[g]
        n = int(min(2 ** rng.uniform(0, 20), L))
        n = max(1, n)
        m = int(rng.integers(0, min(n, L - n + 1) + 1))
        ns.append(n)
        ms.append(m)
        ss.append(sids[g])
    return ns, ms, ss


def test_device_batch_matches_oracle(torch, ctx, seeds3):
    sids, lens, words = seeds3
    rng = np.random.default_rng(21)
    ns, ms, ss = uneven(rng, 90, sids, lens)
    ns[:4], ms[:4] = [1, 64, 65, 1 << 20], [1, 64, 0, 1 << 20]
    ss[3] = sids[0]
    rows, xwds, ywds = layout(ns, ms, ss)
    log("device batch: %d blocks, classes %s" % (
        len(rows), sorted({max(10, (n + m - 2).bit_length()) for n, m in zip(ns, ms) if m})))
    xw = qi.gen_bits(64 * xwds, 55)
    x = dev(torch, xw)
    y = torch.full((ywds + 1,), -1, dtype=torch.int64, device="cuda:0")
    blocks = ctx.block_records(rows, x, y)
    ctx.hash_batched(blocks, x, y)
    assert ctx.batched_rejected() == 0
    check(rows, xw, words, host(y))
    # the same batch again, each block through the plain single-block call
    y2 = torch.full_like(y, -1)
    for (xo, n, m, yo, sid) in rows:
        if m:
            ctx.hash_seeded(x[xo:xo + (n + 63) // 64], n, sid, m, y=y2[yo:yo + (m + 63) // 64])
    torch.cuda.synchronize()
    assert torch.equal(y, y2)


def test_device_batch_seed_id_array(torch, ctx, seeds3):
    sids, lens, words = seeds3
    rng = np.random.default_rng(22)
    ns, ms, ss = uneven(rng, 30, sids, lens)
    rows, xwds, ywds = layout(ns, ms, ss)
    xw = qi.gen_bits(64 * xwds, 56)
    x = dev(torch, xw)
    y = torch.full((ywds + 1,), -1, dtype=torch.int64, device="cuda:0")
    # descriptors name seed 0 (never registered); the array gives the ids
    blocks = ctx.block_records([(r[0], r[1], r[2], r[3], 0) for r in rows], x, y)
    ids = torch.tensor(ss, dtype=torch.int32, device="cuda:0")
    ctx.hash_batched(blocks, x, y, seed_ids=ids)
    assert ctx.batched_rejected() == 0
    check(rows, xw, words, host(y))
    # without the array every block names seed 0: all rejected, none written
    y.fill_(-1)
    ctx.hash_batched(blocks, x, y)
    assert ctx.batched_rejected() == len(rows)
    assert (host(y) == np.uint64(2 ** 64 - 1)).all()


def test_device_batch_rejects_bad_descriptors(torch, ctx, seeds3):
    import paper_2011_04130_amd as q
    sids, lens, words = seeds3
    good = [(3000, 1500, sids[2]), (40000, 20000, sids[1]), (1 << 19, 1 << 18, sids[0])]
    bad = [(2000, 2001, sids[2]),           # m > n
           (5000, 10, sids[2]),             # seed too short (5009 > 5000 bits)
           (1000, 100, 999),                # unknown seed
           (1000, 100, sids[2])]            # flags set (below)
    allb = good + bad
    rows, xwds, ywds = layout([a[0] for a in allb], [a[1] for a in allb], [a[2] for a in allb])
    xw = qi.gen_bits(64 * xwds, 57)
    x = dev(torch, xw)
    y = torch.full((ywds + 1,), -1, dtype=torch.int64, device="cuda:0")
    rec = ctx._block_records(rows, x, y)
    rec["flags"][6] = 1
    blocks = torch.from_numpy(rec.view(np.uint8).copy()).to("cuda:0")
    ctx.hash_batched(blocks, x, y)
    assert ctx.batched_rejected() == 4
    check(rows, xw, words, host(y), skip={3, 4, 5, 6})
    with pytest.raises(q.QrngError) as e:            # forced direct path: host descriptors only
        ctx.hash_batched(blocks, x, y, path=1)
    assert e.value.status == -4


def test_device_batch_graph_replays(torch, ctx, seeds3):
    """Captured once; before each replay new raw bits and new descriptors
    (shapes and seeds) are written into the same device buffers by ordinary
    eager work, and every replay is checked against the oracle."""
    sids, lens, words = seeds3
    nb = 40
    rng = np.random.default_rng(23)
    # fixed pool sizes that hold any of the batches below
    XW, YW = 64 * 1024 * 4, 64 * 1024 * 4
    x = torch.zeros(XW, dtype=torch.int64, device="cuda:0")
    y = torch.full((YW,), -1, dtype=torch.int64, device="cuda:0")
    blocks = torch.zeros(nb * 40, dtype=torch.uint8, device="cuda:0")
    ids = torch.zeros(nb, dtype=torch.int32, device="cuda:0")

    def new_batch(seed):
        r = np.random.default_rng(seed)
        while True:
            ns, ms, ss = uneven(r, nb, sids, lens)
            rows, xwds, ywds = layout(ns, ms, ss)
            if 64 * xwds <= 64 * XW and ywds + 1 <= YW:
                return rows, xwds

    rows0, xwds0 = new_batch(100)
    xw0 = qi.gen_bits(64 * XW, 200)
    x.copy_(dev(torch, xw0))
    blocks.copy_(ctx.block_records(rows0, x, y))
    ids.copy_(torch.tensor([r[4] for r in rows0], dtype=torch.int32))
    ctx.hash_batched(blocks, x, y, seed_ids=ids)          # allocates what the batch needs
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.hash_batched(blocks, x, y, seed_ids=ids)
    for rep in range(3):
        rows, _ = new_batch(101 + rep)
        xw = qi.gen_bits(64 * XW, 300 + rep)
        # eager work of the program between replays: new inputs, cleared output
        x.copy_(dev(torch, xw))
        blocks.copy_(ctx.block_records(rows, x, y))
        ids.copy_(torch.tensor([r[4] for r in rows], dtype=torch.int32))
        y.fill_(-1)
        z = torch.arange(1 << 20, device="cuda:0").sum()
        torch.cuda.synchronize()
        assert int(z) == (1 << 20) * ((1 << 20) - 1) // 2
        g.replay()
        torch.cuda.synchronize()
        log("graph replay %d" % rep)
        check(rows, xw, words, host(y))
    del g
