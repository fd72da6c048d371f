"""GPU parity of the modified Toeplitz hash (paper Sec. III.D) against the
CPU oracle, bit for bit: k = (A, I_m) r with an (n-1)-bit seed, computed by
the library as an (n-m)-column hash plus the raw tail."""
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


def ref_modified(xw, n, aw, m):
    """The oracle's packed route; above 2^36 products of A the A-part comes
    from the oracle's float64 circulant method (pinned to the packed C hash)."""
    w = n - m
    if w * m <= (1 << 36):
        return oracle.modified_toeplitz_packed(xw, n, aw, m)
    r = oracle.unpack_bits(xw, w)
    a = oracle.unpack_bits(aw, w + m - 1)
    y = oracle.pack_bits(oracle.toeplitz_fft64(r, a, m, pad_pow2=True))
    tail = oracle.pack_bits(oracle.unpack_bits(xw, n)[w:n])
    return y ^ tail


SIZES = [(1, 1), (2, 1), (2, 2), (64, 64), (65, 1), (100, 60), (130, 97), (1000, 625),
         (4096, 2560), (10007, 5003), (65536, 40960), (100000, 99999), (200003, 150001),
         (1 << 20, 655360), (3000001, 2000001),
         # split transform with two raw and three output chunks (n-m < 2^23 < n-1)
         (1 << 24, 10485760)]


@pytest.mark.parametrize("n,m", SIZES)
@pytest.mark.parametrize("path", [1, 2])
def test_modified_matches_oracle(torch, ctx, n, m, path):
    log("modified n=%d m=%d path=%d" % (n, m, path))
    rng = np.random.default_rng(n * 104729 + m)
    xw = qi.gen_bits(n, int(rng.integers(1 << 31)))
    aw = qi.gen_seed_words(max(n - 1, 1), int(rng.integers(1 << 31)))
    want = ref_modified(xw, n, aw, m)
    got = host(ctx.modified_hash(dev(torch, xw), n, dev(torch, aw), m, path=path))
    assert np.array_equal(got, want), "first mismatch word %d" % int(np.argmax(got != want))


@pytest.mark.parametrize("n,m", [(4096, 2560), (16384, 10240), (1 << 20, 655360)])
def test_modified_matrix_core_and_auto(torch, ctx, n, m):
    rng = np.random.default_rng(n + 3 * m)
    xw = qi.gen_bits(n, int(rng.integers(1 << 31)))
    aw = qi.gen_seed_words(n - 1, int(rng.integers(1 << 31)))
    want = ref_modified(xw, n, aw, m)
    for path in (0, 3):
        if path == 3 and n > (1 << 16):
            continue
        got = host(ctx.modified_hash(dev(torch, xw), n, dev(torch, aw), m, path=path))
        assert np.array_equal(got, want), path


def test_modified_full_size_registered_seed(torch, ctx):
    """The n = 2^23 workload block with m = 5n/8: the (n-m)-column product is
    one 2^23-point transform (the ordinary hash of the same block needs the
    split transform); a registered seed of n-1 bits, twice in a row."""
    c = qi.config(1)
    s = qi.gen_adc(c["S"], c["sigma"], seed=c["adc_seed"])
    xw = qi.samples_as_words(s)
    n, m = c["n"], c["m_expected"]
    aw = qi.gen_seed_words(n - 1, c["seed_seed"])
    log("modified full size n=%d m=%d" % (n, m))
    want = ref_modified(xw, n, aw, m)
    sid = ctx.register_seed(dev(torch, aw), n - 1)
    try:
        xt = dev(torch, xw)
        y = ctx.modified_hash_seeded(xt, n, sid, m, path=2)
        assert np.array_equal(host(y), want)
        y.fill_(-1)
        ctx.modified_hash_seeded(xt, n, sid, m, y=y, path=2)
        assert np.array_equal(host(y), want)
        # sampled rows through the oracle's row-wise definition as well
        w = n - m
        rows = np.sort(np.random.default_rng(7).choice(m, 256, replace=False))
        bits = oracle.toeplitz_rows(xw, w, aw, n - 1, rows) ^ oracle.unpack_bits(xw, n)[w + rows]
        assert np.array_equal(oracle.unpack_bits(host(y), m)[rows], bits)
    finally:
        ctx.unregister_seed(sid)


def test_modified_arguments(torch, ctx):
    import paper_2011_04130_amd as q
    xw = qi.gen_bits(1000, 1)
    aw = qi.gen_seed_words(999, 2)
    y = torch.full((4,), 12345, dtype=torch.int64, device="cuda:0")
    ctx.modified_hash(dev(torch, xw), 1000, dev(torch, aw), 0, y=y)
    torch.cuda.synchronize()
    assert (y.cpu() == 12345).all()                # m = 0: nothing written
    with pytest.raises(q.QrngError):
        ctx.modified_hash(dev(torch, xw), 100, dev(torch, aw), 101)
    with pytest.raises(q.QrngError):
        ctx.modified_hash(dev(torch, xw), 0, dev(torch, aw), 0)
    sid = ctx.register_seed(dev(torch, aw), 500)
    try:
        with pytest.raises(q.QrngError):           # the block needs 999 seed bits
            ctx.modified_hash_seeded(dev(torch, xw), 1000, sid, 100)
    finally:
        ctx.unregister_seed(sid)
