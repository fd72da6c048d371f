"""GPU parity of the multi-block paths: the matrix-core product (fp4 operands) over
blocks sharing one seed, and batches of blocks against the oracle and
against the single-block call (0 differing bits)."""
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


def strided_blocks(nblk, n, m, sid, x_pad=0, y_pad=0, y0=0):
    xw, yw = (n + 63) // 64 + x_pad, (m + 63) // 64 + y_pad
    return [(b * xw, n, m, y0 + b * yw, sid) for b in range(nblk)], xw * nblk, y0 + yw * nblk


@pytest.mark.parametrize("n,m,nblk", [(64, 40, 5), (4096, 2560, 300), (4000, 2500, 129),
                                      (16384, 10240, 130), (1000, 1000, 7), (333, 1, 3),
                                      (96, 32, 1)])
@pytest.mark.parametrize("path", [1, 2, 3])
def test_shared_seed_blocks_match_oracle(torch, ctx, n, m, nblk, path):
    log("blocks n=%d m=%d B=%d path=%d" % (n, m, nblk, path))
    sw = qi.gen_seed_words(n + m - 1, n + 17 * m)
    sid = ctx.register_seed(dev(torch, sw), n + m - 1)
    try:
        blocks, xwords, ywords = strided_blocks(nblk, n, m, sid, y0=1)
        xw = qi.gen_bits(64 * xwords, nblk + n)
        yt = torch.full((ywords + 1,), -1, dtype=torch.int64, device="cuda:0")
        ctx.hash_batched_host(blocks, dev(torch, xw), yt, path=path)
        got = host(yt)
        assert got[0] == np.uint64(2 ** 64 - 1)          # untouched before the pool
        for (xo, bn, bm, yo, _) in blocks:
            want = oracle.toeplitz_packed(xw[xo: xo + (bn + 63) // 64], bn, sw, bm)
            assert np.array_equal(got[yo: yo + len(want)], want), (xo, yo)
    finally:
        ctx.unregister_seed(sid)


def test_mfma_single_block_and_sweep_slice(torch, ctx):
    # a slice of the block-length sweep: 2^12-bit blocks of Gaussian ADC data
    c = qi.config(2)
    n, m = 4096, 2560
    nblk = 1024
    s = qi.gen_adc(nblk * n // 8, c["sigma"], seed=c["adc_seed"])
    xw = qi.samples_as_words(s)
    sw = qi.gen_seed_words(n + m - 1, c["seed_seed"])
    sid = ctx.register_seed(dev(torch, sw), n + m - 1)
    try:
        blocks, _, ywords = strided_blocks(nblk, n, m, sid)
        xt = dev(torch, xw)
        outs = {}
        for path in (1, 2, 3):
            yt = torch.zeros(ywords, dtype=torch.int64, device="cuda:0")
            ctx.hash_batched_host(blocks, xt, yt, path=path)
            outs[path] = host(yt)
        assert np.array_equal(outs[1], outs[2]) and np.array_equal(outs[1], outs[3])
        for b in (0, 1, 511, 1023):
            want = oracle.toeplitz_packed(xw[b * 64:(b + 1) * 64], n, sw, m)
            assert np.array_equal(outs[3][b * 40:(b + 1) * 40], want)
        # the single-block call on the MFMA path (a batch of one)
        y1 = host(ctx.hash_seeded(xt[64:128], n, sid, m, path=3))
        assert np.array_equal(y1, outs[1][40:80])
    finally:
        ctx.unregister_seed(sid)


@pytest.fixture(scope="module")
def sweep_stream(torch):
    """The block-length sweep's 2^30-bit raw sequence (2^27 Gaussian samples)."""
    c = qi.config(2)
    s = qi.gen_adc(c["S"], c["sigma"], seed=c["adc_seed"])
    return c, qi.samples_as_words(s), dev(torch, qi.samples_as_words(s))


@pytest.mark.parametrize("lg", [12, 14, 16, 18, 20, 22, 24])
def test_sweep_full_size_every_block(torch, ctx, sweep_stream, lg):
    """The sweep at its full size, in the launch the bench times (one strided
    call over all 2^30/n blocks): every block's output of the default path
    equals the direct product's (an independent kernel) bit for bit, and up
    to 2^14 also the transform's and the matrix cores'; the first, last and
    two random blocks agree with the oracle (whole blocks up to 2^16 bits,
    sampled rows above)."""
    c, xw, xt = sweep_stream
    n = 1 << lg
    m = n * c["gamma_num"] // c["gamma_den"]
    B = c["total_bits"] // n
    log("sweep n=2^%d blocks=%d" % (lg, B))
    sw = qi.gen_seed_words(n + m - 1, c["seed_seed"])
    sid = ctx.register_seed(dev(torch, sw), n + m - 1)
    yw = (m + 63) // 64
    try:
        paths = (0, 2, 3, 1) if lg <= 14 else (0, 2, 1) if lg <= 16 else (0, 1)
        outs = {}
        for path in paths:
            yt = torch.full((B * yw,), -1, dtype=torch.int64, device="cuda:0")
            ctx.hash_strided(xt, n, n // 64, sid, m, yt, yw, B, path=path)
            outs[path] = host(yt)
            log("sweep n=2^%d path %d done" % (lg, path))
        for path in paths[1:]:
            diff = np.flatnonzero(outs[0] != outs[path])
            assert not len(diff), "path %d differs from auto in block %d" % (
                path, int(diff[0]) // yw if len(diff) else -1)
        got = outs[0]
        rng = np.random.default_rng(lg)
        for b in sorted({0, B - 1, *rng.integers(0, B, 2).tolist()}):
            xb = xw[b * (n // 64):(b + 1) * (n // 64)]
            yb = got[b * yw:(b + 1) * yw]
            if n <= (1 << 16):
                assert np.array_equal(yb, oracle.toeplitz_packed(xb, n, sw, m)), "block %d" % b
            else:
                rows = np.unique(np.concatenate([[0, m - 1], rng.integers(0, m, 24)]))
                want = oracle.toeplitz_rows(xb, n, sw, n + m - 1, rows)
                assert np.array_equal(oracle.unpack_bits(yb, m)[rows], want), "block %d" % b
    finally:
        ctx.unregister_seed(sid)


@pytest.mark.parametrize("n,nblk", [(1 << 15, 200), (3 << 14, 130), (1 << 16, 64),
                                    ((1 << 16) + 512, 40)])
def test_default_path_near_matrix_core_limit(torch, ctx, n, nblk):
    """Shared-seed batches around the default path's matrix-core limit (m n <=
    5 2^29 with >= 32 blocks, n = 2^16 at m = 5n/8): the default path's bits
    equal the transform's, the matrix cores' and the direct product's for
    every block, and the first and last blocks equal the oracle's; just above
    the limit the default is the transform."""
    m = n * 5 // 8
    log("near limit n=%d blocks=%d" % (n, nblk))
    sw = qi.gen_seed_words(n + m - 1, n + 5)
    sid = ctx.register_seed(dev(torch, sw), n + m - 1)
    xw = qi.gen_bits(nblk * n, n + 7)
    xt = dev(torch, xw)
    yw = (m + 63) // 64
    try:
        outs = {}
        for path in (0, 1, 2, 3):
            yt = torch.full((nblk * yw,), -1, dtype=torch.int64, device="cuda:0")
            ctx.hash_strided(xt, n, n // 64, sid, m, yt, yw, nblk, path=path)
            outs[path] = host(yt)
        for path in (1, 2, 3):
            assert np.array_equal(outs[0], outs[path]), "path %d differs from the default" % path
        for b in (0, nblk - 1):
            want = oracle.toeplitz_packed(xw[b * (n // 64):(b + 1) * (n // 64)], n, sw, m)
            assert np.array_equal(outs[0][b * yw:(b + 1) * yw], want), "block %d" % b
    finally:
        ctx.unregister_seed(sid)
