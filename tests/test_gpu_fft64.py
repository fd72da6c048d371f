"""GPU parity of the paper's float64 circulant method (Sec. III.B in floating
point, the comparison path) against the CPU oracle: bit for bit, with the
reported rounding distance far below 1/2."""
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


def ref_hash(xw, n, sw, m):
    """Packed C definition for small blocks, the oracle's float64 circulant
    method (pinned to it) for large ones."""
    if n * m <= (1 << 36):
        return oracle.toeplitz_packed(xw, n, sw, m)
    r = oracle.unpack_bits(xw, n)
    a = oracle.unpack_bits(sw, n + m - 1)
    return oracle.pack_bits(oracle.toeplitz_fft64(r, a, m, pad_pow2=True))


SIZES = [(1, 1), (2, 1), (5, 3), (31, 17), (64, 64), (65, 1), (100, 100), (1000, 625),
         (4095, 4000), (4096, 2560), (10007, 5003), (65536, 40960), (200003, 100001),
         (1 << 20, 655360),
         # transform lengths 2^12, 2^16, 2^20: the first forward pass reads the bits
         (2560, 1537), (40000, 25537), (600000, 448577),
         # n+m-1 just above 2^24: a 2^25-point transform (radix 2, 16, 256, 256, 16)
         (8388609, 8388609)]


@pytest.mark.parametrize("n,m", SIZES)
def test_fft64_matches_oracle(torch, ctx, n, m):
    log("fft64 n=%d m=%d" % (n, m))
    rng = np.random.default_rng(n * 31 + m)
    xw = qi.gen_bits(n, int(rng.integers(1 << 31)))
    sw = qi.gen_seed_words(n + m - 1, int(rng.integers(1 << 31)))
    err = torch.full((1,), -1.0, dtype=torch.float64, device="cuda:0")
    got = host(ctx.hash_fft64(dev(torch, xw), n, dev(torch, sw), m, err_out=err))
    want = ref_hash(xw, n, sw, m)
    assert np.array_equal(got, want), "first mismatch word %d" % int(np.argmax(got != want))
    e = float(err.item())
    assert 0.0 <= e < 1e-6, e


def test_fft64_full_size_equals_exact_paths(torch, ctx):
    """The n = 2^23 workload block (2^24-point transform): the float64 method
    gives the exact hash (the NTT path's bits and sampled oracle rows), with
    the rounding distance it reports far below 1/2, twice in a row."""
    c = qi.config(1)
    s = qi.gen_adc(c["S"], c["sigma"], seed=c["adc_seed"])
    xw = qi.samples_as_words(s)
    n, m = c["n"], c["m_expected"]
    sw = qi.gen_seed_words(n + m - 1, c["seed_seed"])
    log("fft64 full size n=%d m=%d" % (n, m))
    xt, st = dev(torch, xw), dev(torch, sw)
    exact = host(ctx.hash(xt, n, st, m, path=2))
    err = torch.full((1,), -1.0, dtype=torch.float64, device="cuda:0")
    for _ in range(2):
        got = host(ctx.hash_fft64(xt, n, st, m, err_out=err))
        assert np.array_equal(got, exact)
        e = float(err.item())
        assert 0.0 <= e < 1e-6, e
    rows = np.sort(np.random.default_rng(3).choice(m, 256, replace=False))
    bits = oracle.toeplitz_rows(xw, n, sw, n + m - 1, rows)
    assert np.array_equal(oracle.unpack_bits(exact, m)[rows], bits)


def test_fft64_arguments(torch, ctx):
    import paper_2011_04130_amd as q
    xw = qi.gen_bits(1000, 1)
    sw = qi.gen_seed_words(2000, 2)
    with pytest.raises(q.QrngError):
        ctx.hash_fft64(dev(torch, xw), 100, dev(torch, sw), 101)
    y = torch.full((4,), 7, dtype=torch.int64, device="cuda:0")
    ctx.hash_fft64(dev(torch, xw), 1000, dev(torch, sw), 0, y=y)
    torch.cuda.synchronize()
    assert (y.cpu() == 7).all()
