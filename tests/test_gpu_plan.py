"""GPU parity of plans: uneven batches fixed once (descriptors on the
device, one launch per transform-length class, HIP graph replays, tuned
launch shapes, per-block min-entropy), against the oracle."""
import ctypes
import math

import numpy as np
import pytest

import oracle
import qrng_inputs as qi

pytestmark = pytest.mark.gpu

TOL = 1e-12  # estimator scalars: same double formulas, different summation order


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


def uneven_layout(ns, ms, sids, gap=1):
    """Blocks packed back to back (x) and with a gap word between outputs (y)."""
    rows, xo, yo = [], 0, 1
    for n, m, sid in zip(ns, ms, sids):
        rows.append((xo, int(n), int(m), yo, int(sid)))
        xo += (int(n) + 63) // 64
        yo += (int(m) + 63) // 64 + gap
    return rows, xo, yo


def check_blocks(rows, xw, seeds, got, m_of=None):
    for b, (xo, n, m, yo, sid) in enumerate(rows):
        mv = m if m_of is None else m_of[b]
        want = oracle.toeplitz_packed(xw[xo:xo + (n + 63) // 64], n, seeds[sid], mv)
        nw = (mv + 63) // 64
        assert np.array_equal(got[yo:yo + nw], want), "block %d (n=%d m=%d)" % (b, n, mv)
        assert not got[yo + nw:yo + (m + 63) // 64].any(), "block %d tail" % b
        assert got[yo - 1] == np.uint64(2 ** 64 - 1), "block %d: gap word written" % b


@pytest.mark.parametrize("path", [0, 1, 2])
@pytest.mark.parametrize("graph", [False, True])
def test_plan_uneven_blocks_match_oracle(torch, ctx, path, graph):
    """Uneven n and m across several transform lengths and seeds; two
    executions with other GPU work between them give the same bits."""
    log("plan uneven path=%d graph=%d" % (path, graph))
    rng = np.random.default_rng(5 + path)
    nb = 48
    ns = np.maximum(64, (2.0 ** rng.uniform(6, 16.5, nb)).astype(np.int64))
    ns[:3] = [1, 63, 65]                       # ragged and tiny blocks
    ms = np.array([int(rng.integers(1, n + 1)) for n in ns])
    ms[3] = 0                                  # m = 0 is skipped
    sids_l = [ctx.register_seed(dev(torch, qi.gen_seed_words(2 * 2 ** 17, 900 + g)), 2 * 2 ** 17)
              for g in range(3)]
    seeds = {sid: qi.gen_seed_words(2 * 2 ** 17, 900 + g) for g, sid in enumerate(sids_l)}
    sids = [sids_l[b % 3] for b in range(nb)]
    rows, xwords, ywords = uneven_layout(ns, ms, sids)
    xw = qi.gen_bits(64 * xwords, 77)
    x = dev(torch, xw)
    y = torch.full((ywords + 1,), -1, dtype=torch.int64, device="cuda:0")
    try:
        with ctx.plan(rows, x, y, graph=graph, path=path) as pl:
            info = pl.info()
            assert info["blocks"] == nb and info["graph"] == int(graph)
            for rep in range(2):
                y.fill_(-1)
                pl.execute()
                torch.cuda.synchronize()
                got = host(y)
                check_blocks(rows, xw, seeds, got)
                # eager work of the program between replays
                z = torch.arange(1 << 20, device="cuda:0").sum()
                torch.cuda.synchronize()
                assert int(z) == (1 << 20) * ((1 << 20) - 1) // 2
    finally:
        for sid in sids_l:
            ctx.unregister_seed(sid)


def estimate_refs(samples, offs, ns, caps, eps=0.0):
    refs, ms = [], []
    for b in range(len(ns)):
        s = samples[offs[b]:offs[b] + ns[b] // 8]
        r = oracle.minentropy_counts(oracle.histogram(s, 8), 8)
        refs.append(r)
        ms.append(min(oracle.output_bits(int(ns[b]), 8, r["h_mod"], eps), int(caps[b])))
    return refs, ms


def near_integer(h):
    return abs(h - round(h)) < 1e-9


@pytest.mark.parametrize("graph", [False, True])
def test_plan_estimate_per_block(torch, ctx, graph):
    """Per-block histogram, estimate and output length on the device, then the
    hash of each block with its own m (small version of the uneven workload)."""
    cfg = dict(qi.config(3))
    cfg.update(blocks=40, group=8, log2_min=10, log2_max=16)
    log("plan estimate graph=%d" % graph)
    pool = qi.batched_pool(cfg)
    ns, offs = pool["n"], pool["byte_off"]
    caps = ns.copy()
    caps[1] = ns[1] // 4                       # a cap below the estimate's length
    sids_l = [ctx.register_seed(dev(torch, pool["seed_words"](g)), pool["seed_bits"])
              for g in range(pool["nseeds"])]
    seeds = {sid: pool["seed_words"](g) for g, sid in enumerate(sids_l)}
    sids = [sids_l[g] for g in pool["seed_of"]]
    rows = []
    yo = 1
    for b in range(len(ns)):
        rows.append((int(offs[b]) // 8, int(ns[b]), int(caps[b]), yo, sids[b]))
        yo += (int(caps[b]) + 63) // 64 + 1
    xw = qi.samples_as_words(pool["samples"])
    x = dev(torch, xw)
    y = torch.full((yo + 1,), -1, dtype=torch.int64, device="cuda:0")
    m_out = torch.full((len(ns),), -1, dtype=torch.int64, device="cuda:0")
    from paper_2011_04130_amd._lib import MeResult
    rs = ctypes.sizeof(MeResult)
    me_out = torch.zeros(len(ns) * rs, dtype=torch.uint8, device="cuda:0")
    refs, want_m = estimate_refs(pool["samples"], offs, ns, caps)
    try:
        with ctx.plan(rows, x, y, m_out=m_out, me_out=me_out, estimate=True,
                      graph=graph) as pl:
            for rep in range(2):
                y.fill_(-1)
                m_out.fill_(-1)
                pl.execute()
                torch.cuda.synchronize()
                got_m = m_out.cpu().numpy()
                me_raw = me_out.cpu().numpy()
                for b in range(len(ns)):
                    me = MeResult.from_buffer_copy(me_raw[b * rs:(b + 1) * rs].tobytes()).as_dict()
                    for k in ("mu_hat", "sigma_hat", "h_min", "d_u", "delta_h_m", "h_mod"):
                        assert abs(me[k] - refs[b][k]) <= TOL, (b, k, me[k], refs[b][k])
                    if not near_integer(refs[b]["h_mod"]):
                        assert got_m[b] == want_m[b], (b, got_m[b], want_m[b])
                check_blocks(rows, xw, seeds, host(y), m_of=[int(v) for v in got_m])
    finally:
        for sid in sids_l:
            ctx.unregister_seed(sid)


def test_plan_tune_table_roundtrip(torch, ctx):
    """Tuning picks a shape per class, the table exports and imports, and a
    plan built from the imported table gives the same bits."""
    import paper_2011_04130_amd as q
    log("plan tune")
    ns = [3000, 5000, 20000, 30000, 70000, 90000, 100000, 130000] * 3
    ms = [n // 2 for n in ns]
    sw = qi.gen_seed_words(2 ** 18, 4242)
    sid = ctx.register_seed(dev(torch, sw), 2 ** 18)
    rows, xwords, ywords = uneven_layout(ns, ms, [sid] * len(ns))
    xw = qi.gen_bits(64 * xwords, 4343)
    x = dev(torch, xw)
    y = torch.full((ywords + 1,), -1, dtype=torch.int64, device="cuda:0")
    try:
        with ctx.plan(rows, x, y, tune=True) as pl:
            pl.execute()
            torch.cuda.synchronize()
            check_blocks(rows, xw, {sid: sw}, host(y))
        table = ctx.tune_export()
        lines = [ln for ln in table.splitlines() if ln]
        entries = [ln for ln in lines if not ln.startswith("#")]
        assert entries and all(ln.startswith(("ntt ", "multi ")) for ln in entries)
        # the measured alternatives follow their entry; the choice is the fastest
        measured = {}
        for ln in lines:
            if ln.startswith("#"):
                key, _, rest = ln[2:].partition(" measured ")
                measured[key] = {int(a): float(b) for a, b in (t.split(":") for t in rest.split())}
        for ln in entries:
            if ln.startswith("ntt "):
                key, choice = ln.rsplit(" ", 1)
                assert key in measured, ln
                times = measured[key]
                assert int(choice) in times and times[int(choice)] == min(times.values()), ln
        c2 = q.Context(0)
        try:
            c2.tune_import(table)
            assert [ln for ln in c2.tune_export().splitlines()
                    if ln and not ln.startswith("#")] == entries
            sid2 = c2.register_seed(dev(torch, sw), 2 ** 18)
            y2 = torch.full_like(y, -1)
            with c2.plan([(r[0], r[1], r[2], r[3], sid2) for r in rows], x, y2, graph=True) as p2:
                p2.execute()
                torch.cuda.synchronize()
            assert torch.equal(y, y2)
        finally:
            c2.close()
    finally:
        ctx.unregister_seed(sid)


def test_plan_pins_its_seeds(torch, ctx):
    import paper_2011_04130_amd as q
    sw = qi.gen_seed_words(4096, 1)
    sid = ctx.register_seed(dev(torch, sw), 4096)
    x = dev(torch, qi.gen_bits(4096, 2))
    y = torch.zeros(64, dtype=torch.int64, device="cuda:0")
    pl = ctx.plan([(0, 2048, 1024, 0, sid)], x, y)
    with pytest.raises(q.QrngError) as e:
        ctx.unregister_seed(sid)
    assert e.value.status == -5                # EBUSY
    pl.close()
    ctx.unregister_seed(sid)


def test_plan_rejects_bad_descriptors(torch, ctx):
    import paper_2011_04130_amd as q
    sw = qi.gen_seed_words(4096, 1)
    sid = ctx.register_seed(dev(torch, sw), 4096)
    x = dev(torch, qi.gen_bits(8192, 2))
    y = torch.zeros(256, dtype=torch.int64, device="cuda:0")
    try:
        bad = [
            [(0, 2048, 1024, 0, sid), (0, 2048, 1024, 10, sid)],      # outputs overlap
            [(0, 2048, 2049, 0, sid)],                                 # m > n
            [(0, 3000, 1200, 0, sid)],                                 # seed too short
            [(0, 2048, 1024, 0, sid + 100)],                           # unknown seed
        ]
        for rows in bad:
            with pytest.raises(q.QrngError):
                ctx.plan(rows, x, y)
        with pytest.raises(q.QrngError):                               # n not a multiple of 64
            ctx.plan([(0, 2000, 100, 0, sid)], x, y,
                     m_out=torch.zeros(1, dtype=torch.int64, device="cuda:0"), estimate=True)
    finally:
        ctx.unregister_seed(sid)


def test_uneven_workload_full_size(torch, ctx):
    """The 4096-block uneven workload (n log-uniform in [2^14, 2^20], 64
    seeds, per-block estimate, output sized at n), as one graph replay.
    Every block's m against the oracle's estimate; every block bit for bit
    against the plain single-block call on the same bits (same seed prefix,
    same m), against the direct product (an independent kernel) and against
    the batch call with device-resident descriptors; blocks
    up to 2^15 bits in full and 12 rows of every larger block against the
    oracle."""
    cfg = qi.config(3)
    log("uneven workload: generating")
    pool = qi.batched_pool(cfg)
    ns, offs = pool["n"], pool["byte_off"]
    sids_l, seeds = [], {}
    for g in range(pool["nseeds"]):
        w = pool["seed_words"](g)
        sid = ctx.register_seed(dev(torch, w), pool["seed_bits"])
        sids_l.append(sid)
        seeds[sid] = w
    rows = []
    yo = 0
    for b in range(len(ns)):
        rows.append((int(offs[b]) // 8, int(ns[b]), int(ns[b]), yo, sids_l[pool["seed_of"][b]]))
        yo += (int(ns[b]) + 63) // 64
    xw = qi.samples_as_words(pool["samples"])
    x = dev(torch, xw)
    y = torch.full((yo,), -1, dtype=torch.int64, device="cuda:0")
    m_out = torch.full((len(ns),), -1, dtype=torch.int64, device="cuda:0")
    try:
        log("uneven workload: plan")
        with ctx.plan(rows, x, y, m_out=m_out, estimate=True, graph=True) as pl:
            pl.execute()
            torch.cuda.synchronize()
        got_m = m_out.cpu().numpy()
        got = host(y)
        log("uneven workload: estimates")
        refs, want_m = estimate_refs(pool["samples"], offs, ns, ns)
        for b in range(len(ns)):
            if not near_integer(refs[b]["h_mod"]):
                assert got_m[b] == want_m[b], (b, got_m[b], want_m[b])
        # the same blocks with the plan's m: one plain call per block, and the
        # direct product over the whole batch
        log("uneven workload: plain single-block calls")
        rows_m = [(xo, n, int(got_m[b]), yo_b, sid) for b, (xo, n, _, yo_b, sid) in enumerate(rows)]
        y_plain = torch.full((yo,), -1, dtype=torch.int64, device="cuda:0")
        for (xo, n, m, yo_b, sid) in rows_m:
            if m:
                ctx.hash_seeded(x[xo:xo + (n + 63) // 64], n, sid, m,
                                y=y_plain[yo_b:yo_b + (m + 63) // 64])
        log("uneven workload: direct product")
        y_dir = torch.full((yo,), -1, dtype=torch.int64, device="cuda:0")
        ctx.hash_batched_host(rows_m, x, y_dir, path=1)
        log("uneven workload: device descriptors")
        y_dev = torch.full((yo,), -1, dtype=torch.int64, device="cuda:0")
        ctx.hash_batched(ctx.block_records(rows_m, x, y_dev), x, y_dev)
        assert ctx.batched_rejected() == 0
        torch.cuda.synchronize()
        plain, direct, devb = host(y_plain), host(y_dir), host(y_dev)
        log("uneven workload: checking")
        rng = np.random.default_rng(11)
        for b in range(len(ns)):
            xo, n, cap, yo_b, sid = rows[b]
            m = int(got_m[b])
            blk = got[yo_b:yo_b + (cap + 63) // 64]
            assert not oracle.unpack_bits(blk, cap)[m:].any(), "block %d tail" % b
            nw = (m + 63) // 64
            assert np.array_equal(blk[:nw], plain[yo_b:yo_b + nw]), "block %d vs plain call" % b
            assert np.array_equal(blk[:nw], direct[yo_b:yo_b + nw]), "block %d vs direct" % b
            assert np.array_equal(blk[:nw], devb[yo_b:yo_b + nw]), "block %d vs device batch" % b
            if n <= (1 << 15):
                want = oracle.toeplitz_packed(xw[xo:xo + n // 64], n, seeds[sid], m)
                assert np.array_equal(blk[:len(want)], want), "block %d" % b
            elif m:
                r = np.unique(np.concatenate([[0, m - 1], rng.integers(0, m, 10)]))
                want = oracle.toeplitz_rows(xw[xo:xo + n // 64], n, seeds[sid], n + m - 1, r)
                bits = oracle.unpack_bits(blk, m)
                assert np.array_equal(bits[r], want), "block %d rows" % b
    finally:
        for sid in sids_l:
            ctx.unregister_seed(sid)


@pytest.mark.parametrize("estimate", [False, True])
def test_plan_persistent_multiclass_equals_per_class(torch, ctx, estimate):
    """The same uneven batch (transform lengths 2^12 .. 2^21) as the three
    persistent multi-class launches and as per-class launches (chosen through
    the tuning table), both as graphs replayed twice: identical bits, and
    against the oracle; the multi-class form takes exactly three launches
    (blocks shorter than 2^16 points join the 2^16 class)."""
    import math as _m
    log("plan persistent estimate=%d" % estimate)
    rng = np.random.default_rng(31 + estimate)
    nb = 60
    ns = (64 * np.floor(2.0 ** rng.uniform(11, 20, nb) / 64)).astype(np.int64)
    ns[:3] = [1 << 20, 64 * 97, 4096]
    ms = np.array([int(n) if estimate else int(rng.integers(1, n + 1)) for n in ns])
    L = 1 << 21
    sids_l = [ctx.register_seed(dev(torch, qi.gen_seed_words(L, 60 + g)), L) for g in range(2)]
    seeds = {sid: qi.gen_seed_words(L, 60 + g) for g, sid in enumerate(sids_l)}
    sids = [sids_l[b % 2] for b in range(nb)]
    rows, xwords, ywords = uneven_layout(ns, ms, sids)
    if estimate:
        samples = np.concatenate([qi.gen_adc(int(n) // 8, 8 + 32 * rng.random(), seed=500 + b)
                                  for b, n in enumerate(ns)])
        xw = qi.samples_as_words(samples)
    else:
        xw = qi.gen_bits(64 * xwords, 88)
    x = dev(torch, xw)
    key = "multi %d " % _m.ceil(_m.log2(nb))
    outs = {}
    try:
        for form in (1, 0):
            ctx.tune_import(key + str(form))
            y = torch.full((ywords + 1,), -1, dtype=torch.int64, device="cuda:0")
            m_out = torch.full((nb,), -1, dtype=torch.int64, device="cuda:0")
            kw = {"m_out": m_out, "estimate": True} if estimate else {}
            with ctx.plan(rows, x, y, graph=True, **kw) as pl:
                info = pl.info()
                pl.execute()
                torch.cuda.synchronize()
                if form == 1:                  # shorter classes join the 2^16 one
                    assert info["launches"] == 3
                pl.execute()                   # a replay gives the same bits
                torch.cuda.synchronize()
            outs[form] = (host(y), m_out.cpu().numpy())
        assert np.array_equal(outs[0][0], outs[1][0])
        assert np.array_equal(outs[0][1], outs[1][1])
        m_of = [int(v) for v in outs[1][1]] if estimate else None
        check_blocks(rows, xw, seeds, outs[1][0], m_of=m_of)
    finally:
        for sid in sids_l:
            ctx.unregister_seed(sid)
