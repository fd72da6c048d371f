"""GPU parity of the estimator's further workloads (paper Sec. II.B-II.C):
classical-noise subtraction, the estimate on a random subset of the samples,
and the attacked-detector source of Sec. II.B -- counts bit-exact, scalars
within 1e-12, output lengths equal."""
import math

import numpy as np
import pytest

import oracle
import qrng_inputs as qi

pytestmark = pytest.mark.gpu

TOL = 1e-12
KEYS = ("mu_hat", "sigma_hat", "h_min", "h_actual", "d_u", "delta_h_m", "h_mod")


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


def log(msg):
    print(msg, flush=True)


def close(me, ref):
    for k in KEYS:
        a, b = me[k], ref[k]
        if math.isinf(a) or math.isinf(b):
            assert a == b, k
        else:
            assert abs(a - b) <= TOL, (k, a, b)


@pytest.mark.parametrize("sigma_c", [0.0, 5.0, 12.5, 40.0])
def test_quantum_model_matches_oracle(torch, ctx, sigma_c):
    import paper_2011_04130_amd as q
    log("quantum model sigma_c=%g" % sigma_c)
    s = qi.gen_adc(1 << 18, 20.0, seed=41)
    ref = oracle.minentropy_counts(oracle.histogram(s, 8), 8, sigma_classical=sigma_c)
    me = ctx.minentropy(torch.from_numpy(s).to("cuda:0"), model=q.MODEL_QUANTUM, sigma=sigma_c)
    close(me, ref)
    # the same model inside the one-call path: equal m on the device
    n = 8 * len(s)
    m = oracle.output_bits(n, 8, ref["h_mod"])
    sw = qi.gen_seed_words(2 * n - 1, 42)
    sid = ctx.register_seed(torch.from_numpy(sw.view(np.int64).copy()).to("cuda:0"), 2 * n - 1)
    try:
        m_out = torch.zeros(1, dtype=torch.int64, device="cuda:0")
        ctx.extract(torch.from_numpy(s).to("cuda:0"), sid, n, m_out=m_out,
                    model=q.MODEL_QUANTUM, sigma=sigma_c, path=q.PATH_NTT)
        torch.cuda.synchronize()
        assert int(m_out.item()) == m
    finally:
        ctx.unregister_seed(sid)


@pytest.mark.parametrize("S,offset,seed,thr", [(1 << 20, 0, 1, 1 << 29), (100003, 3, 2, 3 << 30),
                                               (65536, 8, 3, 1 << 24), (777, 5, 4, 0xFFFFFFFF)])
def test_subset_estimate_matches_oracle(torch, ctx, S, offset, seed, thr):
    log("subset S=%d offset=%d thr=%#x" % (S, offset, thr))
    s = qi.gen_adc(S + offset, 20.0, seed=50 + seed)
    dev = torch.from_numpy(s).to("cuda:0")[offset:]   # start off the 16-byte grid
    me = ctx.minentropy(dev, want_counts=True, subset_seed=seed, keep_thr=thr)
    keep = oracle.subset_mask(S, seed, thr)
    h = oracle.histogram(s[offset:][keep], 8)
    assert np.array_equal(np.array(me["counts"], np.uint64), h)
    assert me["samples"] == int(keep.sum())
    close(me, oracle.minentropy_counts(h, 8))


def test_subset_keeping_nothing_is_an_error(torch, ctx):
    import paper_2011_04130_amd as q
    s = torch.from_numpy(qi.gen_adc(64, 20.0, seed=1)).to("cuda:0")
    with pytest.raises(q.QrngError):
        ctx.minentropy(s, subset_seed=1, keep_thr=1)   # keeps about 1.5e-8 of 64 samples


@pytest.mark.parametrize("bits", [5, 8])
def test_attacked_detector_workload(torch, ctx, bits):
    """Sec. II.B's attack (V' = alpha(I) I through an N-bit ADC over [-5, 5)):
    device estimates equal the oracle's for every U reading, and the
    U = {argmax P, argmax P'} correction never exceeds the observed
    min-entropy -log2 max P' (the bound that reading guarantees)."""
    import paper_2011_04130_amd as q
    s = qi.gen_attack(1 << 20, bits, seed=60 + bits)
    h = oracle.histogram(s, bits)
    observed = -math.log2(h.max() / h.sum())
    for u in (q.U_MODEL_ARGMAX, q.U_BOTH_ARGMAX, q.U_ALL):
        me = ctx.minentropy(torch.from_numpy(s).to("cuda:0"), sample_bits=bits, u_mode=u)
        ref = oracle.minentropy_counts(h, bits, u_mode=u)
        close(me, ref)
        if u == q.U_BOTH_ARGMAX:
            assert me["h_mod"] <= observed + 1e-12


@pytest.mark.parametrize("u_mode", [0, 1])
def test_tied_model_bins_host_and_device(torch, ctx, u_mode):
    """A given model centred half way between two codes (mu = 127.5) ties
    bins 127 and 128: the default U is the lower one, the two-argmax set
    both of them and argmax P'; host finish and device finish both agree
    with the oracle."""
    import ctypes

    import paper_2011_04130_amd as q
    from paper_2011_04130_amd._lib import MeResult
    log("tied model bins u_mode=%d" % u_mode)
    s = qi.gen_adc(1 << 17, 20.0, seed=43, mu=129.0)
    ref = oracle.minentropy_counts(oracle.histogram(s, 8), 8, mu=127.5, sigma=20.0,
                                   u_mode=u_mode)
    assert ref["argmax_model"] == 127
    st = torch.from_numpy(s).to("cuda:0")
    me = ctx.minentropy(st, model=q.MODEL_GIVEN, mu=127.5, sigma=20.0, u_mode=u_mode)
    close(me, ref)
    assert me["argmax_model"] == 127
    n = 8 * len(s)
    sw = qi.gen_seed_words(2 * n - 1, 44)
    sid = ctx.register_seed(torch.from_numpy(sw.view(np.int64).copy()).to("cuda:0"), 2 * n - 1)
    try:
        rs = ctypes.sizeof(MeResult)
        me_out = torch.zeros(rs, dtype=torch.uint8, device="cuda:0")
        m_out = torch.zeros(1, dtype=torch.int64, device="cuda:0")
        ctx.extract(st, sid, n, m_out=m_out, me_out=me_out, model=q.MODEL_GIVEN, mu=127.5,
                    sigma=20.0, u_mode=u_mode)
        torch.cuda.synchronize()
        dme = ctx.me_result_from_bytes(me_out)
        close(dme, ref)
        assert dme["argmax_model"] == 127
        assert int(m_out.item()) == oracle.output_bits(n, 8, ref["h_mod"])
    finally:
        ctx.unregister_seed(sid)
