"""GPU parity: the HIP library against the CPU oracle, bit for bit.

Every hash result must equal the oracle exactly (the hash is an integer
function: tolerance 0 bits).  Histogram counts must be equal; the
min-entropy scalars, computed in double on both sides by independently
written code, must agree within 1e-12 (absolute), and the derived output
length m must be equal.
"""
import math

import numpy as np
import pytest

import oracle
import qrng_inputs as qi

pytestmark = pytest.mark.gpu

TOL = 1e-12


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


# ---------------------------------------------------------------- Sec. II

ME_CASES = [
    ("single_n2^17", 16384, 20.0, 128.0, 20201101, 8),
    ("single_n2^23", 1 << 20, 20.0, 128.0, 20201102, 8),
    ("narrow", 1 << 16, 8.0, 100.0, 3, 8),
    ("wide", 1 << 16, 40.0, 128.0, 4, 8),
    ("ragged", 100003, 20.0, 128.0, 5, 8),
    ("five_bit", 50000, 5.0, 16.0, 6, 5),
    ("clipped_low", 30001, 30.0, 10.0, 7, 8),
    # the most counting workgroups a launch uses (256 partial rows), ragged tail
    ("window_2^22", (1 << 22) + 5, 20.0, 128.0, 8, 8),
]


@pytest.mark.parametrize("name,S,sigma,mu,seed,N", ME_CASES)
@pytest.mark.parametrize("u_mode", [0, 1, 2])
def test_minentropy_matches_oracle(torch, ctx, name, S, sigma, mu, seed, N, u_mode):
    log("minentropy %s u_mode=%d" % (name, u_mode))
    s = qi.gen_adc(S, sigma, mu, seed=seed, bits=N)
    want_c = oracle.histogram(s, N)
    want = oracle.minentropy_counts(want_c, N, u_mode=u_mode)
    t = torch.from_numpy(s).to("cuda:0")
    got = ctx.minentropy(t, sample_bits=N, u_mode=u_mode, want_counts=True)
    assert np.array_equal(np.array(got["counts"], dtype=np.uint64), want_c)
    for k in ("mu_hat", "sigma_hat", "h_min", "h_actual", "d_u", "delta_h_m", "h_mod"):
        assert abs(got[k] - want[k]) <= TOL, (k, got[k], want[k])
    assert got["argmax_model"] == want["argmax_model"]
    assert got["argmax_empirical"] == want["argmax_empirical"]
    import paper_2011_04130_amd as q
    n = 8 * S
    assert q.output_bits(n, N, got["h_mod"]) == oracle.output_bits(n, N, want["h_mod"])


def test_minentropy_given_model_and_misaligned_buffer(torch, ctx):
    s = qi.gen_adc(70001, 20.0, seed=8)
    t = torch.from_numpy(s).to("cuda:0")
    for off in (0, 1, 3, 13):
        sub = t[off:]
        c = oracle.histogram(s[off:], 8)
        want = oracle.minentropy_counts(c, 8, mu=127.5, sigma=19.0, u_mode=1)
        got = ctx.minentropy(sub, model=1, mu=127.5, sigma=19.0, u_mode=1, want_counts=True)
        assert np.array_equal(np.array(got["counts"], dtype=np.uint64), c)
        assert abs(got["h_mod"] - want["h_mod"]) <= TOL
        assert got["mu_hat"] == 127.5 and got["sigma_hat"] == 19.0


def test_minentropy_single_block_workload_m(torch, ctx):
    import paper_2011_04130_amd as q
    c = qi.config(0)
    s = qi.gen_adc(c["S"], c["sigma"], seed=c["adc_seed"])
    got = ctx.minentropy(torch.from_numpy(s).to("cuda:0"))
    assert abs(got["h_mod"] - round(got["h_mod"])) > 1e-9
    assert q.output_bits(c["n"], 8, got["h_mod"]) == 81920


def test_minentropy_errors_and_degenerate(torch, ctx):
    import paper_2011_04130_amd as q
    s = qi.gen_adc(4096, 5.0, 16.0, seed=9, bits=8)
    s[100] = 40
    with pytest.raises(q.QrngError):
        ctx.minentropy(torch.from_numpy(s).to("cuda:0"), sample_bits=5)
    with pytest.raises(q.QrngError):
        ctx.minentropy(torch.from_numpy(s).to("cuda:0"), model=1, sigma=0.0)
    # one out-of-range value in the last partial row of the largest launch
    big = qi.gen_adc((1 << 22) + 5, 5.0, 16.0, seed=10, bits=5)
    big[-3] = 33
    with pytest.raises(q.QrngError):
        ctx.minentropy(torch.from_numpy(big).to("cuda:0"), sample_bits=5)
    big[-3] = 31
    got = ctx.minentropy(torch.from_numpy(big).to("cuda:0"), sample_bits=5, want_counts=True)
    assert np.array_equal(np.array(got["counts"], dtype=np.uint64), oracle.histogram(big, 5))
    const = np.full(1000, 77, dtype=np.uint8)
    got = ctx.minentropy(torch.from_numpy(const).to("cuda:0"))
    want = oracle.minentropy_counts(oracle.histogram(const, 8), 8)
    assert got["h_min"] == want["h_min"] == 0.0
    assert got["h_mod"] == want["h_mod"] == 0.0


# ---------------------------------------------------------------- Sec. III.B

def ref_hash(xw, n, sw, m):
    """Oracle result as uint64 words: packed C evaluation for small blocks,
    the float64 circulant method (pinned to it) for large ones."""
    L = n + m - 1
    if n * m <= (1 << 36):
        return oracle.toeplitz_packed(xw, n, sw, m)
    r = oracle.unpack_bits(xw, n)
    a = oracle.unpack_bits(sw, L)
    return oracle.pack_bits(oracle.toeplitz_fft64(r, a, m, pad_pow2=True))


SIZES = [(1, 1), (2, 1), (5, 3), (31, 17), (64, 64), (65, 1), (100, 100), (1000, 625),
         (4095, 4000), (4096, 2560), (10007, 5003), (16384, 10240), (65536, 40960),
         (100000, 99999), (200003, 100001), (1 << 20, 655360)]


@pytest.mark.parametrize("n,m", SIZES)
@pytest.mark.parametrize("path", [1, 2, 3])
def test_hash_matches_oracle(torch, ctx, n, m, path):
    log("hash n=%d m=%d path=%d" % (n, m, path))
    rng = np.random.default_rng(n * 7919 + m)
    xw = qi.gen_bits(n, int(rng.integers(1 << 31)))
    sw = qi.gen_seed_words(n + m - 1, int(rng.integers(1 << 31)))
    want = ref_hash(xw, n, sw, m)
    y = ctx.hash(dev(torch, xw), n, dev(torch, sw), m, path=path)
    got = host(y)
    assert np.array_equal(got, want), "first mismatch word %d" % int(np.argmax(got != want))


def test_single_block_workload_both_paths(torch, ctx):
    c = qi.config(0)
    s = qi.gen_adc(c["S"], c["sigma"], seed=c["adc_seed"])
    xw = qi.samples_as_words(s)
    n, m = c["n"], 81920
    sw = qi.gen_seed_words(n + m - 1, c["seed_seed"])
    r = oracle.unpack_bits(xw, n)
    a = oracle.unpack_bits(sw, n + m - 1)
    want = oracle.pack_bits(oracle.toeplitz_bitwise(r, a, m))
    assert np.array_equal(want, oracle.toeplitz_packed(xw, n, sw, m))
    for path in (1, 2):
        got = host(ctx.hash(dev(torch, xw), n, dev(torch, sw), m, path=path))
        assert np.array_equal(got, want), path


@pytest.mark.parametrize("n,m", [(5000001, 4000003), (1 << 23, 5242880), (8388609, 8388609)])
def test_hash_block_ntt_large(torch, ctx, n, m):
    # seed length above 2^23: block-Toeplitz accumulation in the transform domain
    log("large hash n=%d m=%d" % (n, m))
    rng = np.random.default_rng(n + m)
    xw = qi.gen_bits(n, int(rng.integers(1 << 31)))
    sw = qi.gen_seed_words(n + m - 1, int(rng.integers(1 << 31)))
    want = ref_hash(xw, n, sw, m)
    got = host(ctx.hash(dev(torch, xw), n, dev(torch, sw), m, path=2))
    assert np.array_equal(got, want), "first mismatch word %d" % int(np.argmax(got != want))
    # independent spot check of sampled rows with the packed definition
    rows = np.sort(rng.choice(m, 256, replace=False))
    bits = oracle.toeplitz_rows(xw, n, sw, n + m - 1, rows)
    gb = oracle.unpack_bits(got, m)
    assert np.array_equal(gb[rows], bits)


def test_large_single_block_direct_equals_ntt(torch, ctx):
    c = qi.config(1)
    s = qi.gen_adc(c["S"], c["sigma"], seed=c["adc_seed"])
    xw = qi.samples_as_words(s)
    n, m = c["n"], c["m_expected"]
    sw = qi.gen_seed_words(n + m - 1, c["seed_seed"])
    xt, st = dev(torch, xw), dev(torch, sw)
    yd = host(ctx.hash(xt, n, st, m, path=1))
    yn = host(ctx.hash(xt, n, st, m, path=2))
    assert np.array_equal(yd, yn)
    rng = np.random.default_rng(1)
    rows = np.sort(rng.choice(m, 512, replace=False))
    bits = oracle.toeplitz_rows(xw, n, sw, n + m - 1, rows)
    assert np.array_equal(oracle.unpack_bits(yd, m)[rows], bits)


def test_m_zero_is_noop_and_arguments_checked(torch, ctx):
    import paper_2011_04130_amd as q
    xw = qi.gen_bits(1000, 1)
    sw = qi.gen_seed_words(2000, 2)
    y = torch.full((4,), 12345, dtype=torch.int64, device="cuda:0")
    ctx.hash(dev(torch, xw), 1000, dev(torch, sw), 0, y=y)
    torch.cuda.synchronize()
    assert (y.cpu() == 12345).all()
    with pytest.raises(q.QrngError):
        ctx.hash(dev(torch, xw), 100, dev(torch, sw), 101)
    with pytest.raises(q.QrngError):
        ctx.hash(dev(torch, xw), 0, dev(torch, sw), 0)
    buf = dev(torch, np.concatenate([xw, np.zeros(8, np.uint64)]))
    with pytest.raises(q.QrngError):   # output overlapping the raw block
        ctx.hash(buf, 1000, dev(torch, sw), 500, y=buf[10:])


def test_repeatable_bits(torch, ctx):
    n, m = 300000, 200000
    xw = qi.gen_bits(n, 11)
    sw = qi.gen_seed_words(n + m - 1, 12)
    xt, st = dev(torch, xw), dev(torch, sw)
    outs = [host(ctx.hash(xt, n, st, m, path=p)) for p in (1, 1, 2, 2)]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_seeded_and_batched_equal_single(torch, ctx):
    rng = np.random.default_rng(5)
    Lmax = 3 * 65536
    sw = qi.gen_seed_words(Lmax, 77)
    st = dev(torch, sw)
    sid = ctx.register_seed(st, Lmax)
    try:
        # uniform blocks at constant strides, then uneven ones at scattered offsets
        shapes = [(65536, 40960)] * 6 + [(4096, 2560)] * 5 + [(70000, 30000), (1000, 1), (64, 64)]
        x_off, y_off, blocks = 0, 3, []
        for (n, m) in shapes:
            blocks.append((x_off, n, m, y_off, sid))
            x_off += (n + 63) // 64 + int(rng.integers(0, 2))
            y_off += (m + 63) // 64 + int(rng.integers(0, 3))
        xw = qi.gen_bits(64 * x_off, 78)
        xt = dev(torch, xw)
        y_pool = torch.zeros(y_off + 4, dtype=torch.int64, device="cuda:0")
        for path in (0, 1, 2, 3):
            y_pool.zero_()
            ctx.hash_batched_host(blocks, xt, y_pool, path=path)
            yp = host(y_pool)
            for (xo, n, m, yo, _) in blocks:
                xb = xw[xo: xo + (n + 63) // 64]
                want = oracle.toeplitz_packed(xb, n, sw, m)
                assert np.array_equal(yp[yo: yo + len(want)], want), (path, n, m)
                single = host(ctx.hash_seeded(dev(torch, xb), n, sid, m, path=path))
                assert np.array_equal(single, want)
    finally:
        ctx.unregister_seed(sid)


# ------------------------------------------------ one asynchronous pass

@pytest.mark.parametrize("cfg_k,path,cap_frac", [(0, 1, 1.0), (0, 2, 1.0), (0, 2, 0.5),
                                                  (0, 3, 0.75), (1, 2, 1.0), (1, 1, 0.75)])
def test_extract_matches_oracle(torch, ctx, cfg_k, path, cap_frac):
    """Device min-entropy, device m and the hash in one call equal the oracle."""
    c = qi.config(cfg_k)
    log("extract %s path=%d cap=%.2f" % (c["name"], path, cap_frac))
    s = qi.gen_adc(c["S"], c["sigma"], seed=c["adc_seed"])
    n = 8 * c["S"]
    m_cap = int(n * cap_frac)
    ref = oracle.minentropy_counts(oracle.histogram(s, 8), 8)
    m = min(oracle.output_bits(n, 8, ref["h_mod"]), m_cap)
    sw = qi.gen_seed_words(n + m_cap - 1, c["seed_seed"])
    st = dev(torch, sw)
    sid = ctx.register_seed(st, n + m_cap - 1)
    try:
        m_out = torch.zeros(1, dtype=torch.int64, device="cuda:0")
        me_out = torch.zeros(128, dtype=torch.uint8, device="cuda:0")
        y = torch.full(((m_cap + 63) // 64,), -1, dtype=torch.int64, device="cuda:0")
        ctx.extract(torch.from_numpy(s).to("cuda:0"), sid, m_cap, y=y, m_out=m_out,
                    me_out=me_out, path=path)
        torch.cuda.synchronize()
        me = ctx.me_result_from_bytes(me_out)
        for k in ("mu_hat", "sigma_hat", "h_min", "h_actual", "d_u", "delta_h_m", "h_mod"):
            assert abs(me[k] - ref[k]) <= TOL, (k, me[k], ref[k])
        assert int(m_out.item()) == m
        xw = qi.samples_as_words(s)
        want = ref_hash(xw, n, sw, m)
        got = host(y)
        nw = (m + 63) // 64
        assert np.array_equal(got[:nw], want)
        assert not got[nw:].any()          # bits m..m_cap are written as zero
    finally:
        ctx.unregister_seed(sid)


@pytest.mark.parametrize("S", [1 << 18, 1 << 19, 1 << 20, 300008, 1 << 21])
def test_extract_estimate_in_column_pass(torch, ctx, S):
    """On the split transform (columns of 2^7, 2^8, 2^9) the estimate runs in
    extra workgroups of the first column pass, handing over through a ticket
    that each call leaves at zero: consecutive calls with different sources,
    a direct-path call in between, each against the oracle (S = 300008: a
    sample count that splits unevenly over the counting workgroups)."""
    n = 8 * S
    logn = n.bit_length() - 1
    sw = qi.gen_seed_words(2 * n - 1, 900 + logn)
    sid = ctx.register_seed(dev(torch, sw), 2 * n - 1)
    try:
        for k, (sigma, path) in enumerate([(20.0, 2), (3.0, 2), (6.5, 1), (45.0, 2)]):
            if path == 1 and logn > 21:
                continue  # the direct product at these sizes only repeats the n = 2^21 case
            if logn > 23 and k > 1:
                continue  # n = 2^24 (four raw and four output chunks): two calls suffice
            log("extract n=2^%d sigma=%.1f path=%d" % (logn, sigma, path))
            s = qi.gen_adc(S, sigma, seed=400 + 10 * logn + k)
            ref = oracle.minentropy_counts(oracle.histogram(s, 8), 8)
            m = oracle.output_bits(n, 8, ref["h_mod"])
            m_out = torch.zeros(1, dtype=torch.int64, device="cuda:0")
            me_out = torch.zeros(128, dtype=torch.uint8, device="cuda:0")
            y = torch.full(((n + 63) // 64,), -1, dtype=torch.int64, device="cuda:0")
            ctx.extract(torch.from_numpy(s).to("cuda:0"), sid, n, y=y, m_out=m_out,
                        me_out=me_out, path=path)
            torch.cuda.synchronize()
            me = ctx.me_result_from_bytes(me_out)
            for key in ("mu_hat", "sigma_hat", "h_min", "h_actual", "d_u", "delta_h_m", "h_mod"):
                assert abs(me[key] - ref[key]) <= TOL, (key, me[key], ref[key])
            assert me["samples"] == S
            assert int(m_out.item()) == m
            want = ref_hash(qi.samples_as_words(s), n, sw, m)
            got = host(y)
            nw = (m + 63) // 64
            assert np.array_equal(got[:nw], want)
            assert not got[nw:].any()
    finally:
        ctx.unregister_seed(sid)


@pytest.mark.parametrize("path", [2, 3])
def test_extract_security_term_and_given_model(torch, ctx, path):
    """The device m with a security term (m not a multiple of 32) and the
    given-model readings, on the transform and on the matrix cores (whose
    row tiles then end inside a 32-row word)."""
    c = qi.config(0)
    s = qi.gen_adc(c["S"], 12.0, seed=31)
    n = 8 * c["S"]
    sw = qi.gen_seed_words(2 * n, 32)
    sid = ctx.register_seed(dev(torch, sw), 2 * n - 1)
    try:
        for (model, mu, sigma, u_mode, eps) in [(0, 0.0, 0.0, 1, 20.0), (1, 128.0, 11.0, 2, 0.0),
                                                (1, 120.5, 12.5, 0, 3.5)]:
            ref = oracle.minentropy_counts(oracle.histogram(s, 8), 8,
                                           mu=mu if model else None,
                                           sigma=sigma if model else None, u_mode=u_mode)
            m = oracle.output_bits(n, 8, ref["h_mod"], eps)
            m_out = torch.zeros(1, dtype=torch.int64, device="cuda:0")
            y = ctx.extract(torch.from_numpy(s).to("cuda:0"), sid, n, m_out=m_out, model=model,
                            mu=mu, sigma=sigma, u_mode=u_mode, log2_inv_eps=eps, path=path)
            torch.cuda.synchronize()
            assert int(m_out.item()) == m
            want = oracle.toeplitz_packed(qi.samples_as_words(s), n, sw, m)
            got = host(y)
            assert np.array_equal(got[: len(want)], want)
            assert not got[len(want):].any()
    finally:
        ctx.unregister_seed(sid)
