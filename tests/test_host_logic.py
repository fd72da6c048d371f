"""Host-only tier: the device-free logic of the library (the host finish of
the Sec. II estimate, the Sec. III.B output-length rule, the serving loop's
output ring) built as plain C++ with AddressSanitizer and
UndefinedBehaviorSanitizer and driven on the CPU; the C oracle likewise,
through its own self-check driver.  No GPU, no HIP runtime."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import qrng_inputs as qi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


def _build(tmp_path, name, cmd):
    exe = str(tmp_path / name)
    r = subprocess.run(cmd + ["-o", exe], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail("build failed:\n%s" % r.stderr[-3000:])
    return exe


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    tmp = tmp_path_factory.mktemp("host")
    return _build(tmp, "host_logic_test",
                  ["g++", "-std=c++17", *SAN,
                   "-I", os.path.join(ROOT, "include"),
                   "-I", os.path.join(ROOT, "paper_2011_04130_amd", "csrc"),
                   os.path.join(ROOT, "tests", "host", "host_logic_test.cpp")])


def _run(exe, text):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], input=text, capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "ERROR" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
    return r.stdout.split("\n")


def _hists():
    out = []
    for sigma in (8.0, 20.0, 40.0):
        out.append((8, oracle.histogram(qi.gen_adc(1 << 14, sigma, seed=int(sigma)), 8)))
    z = np.zeros(256, dtype=np.uint64)
    z[3] = 17
    out.append((8, z))
    out.append((5, oracle.histogram(qi.gen_attack(1 << 13, 5, seed=2), 5)))
    return out


def test_host_finish_matches_oracle(driver):
    cases, lines = [], []
    for N, c in _hists():
        for model, mu, sigma in ((0, 0.0, 0.0), (1, (1 << N) / 2 - 0.5, N * 1.5)):
            for u in (0, 1, 2):
                cases.append((N, c, model, mu, sigma, u))
                lines.append("finish %d %d %r %r %d %s" % (N, model, mu, sigma, u,
                                                         " ".join(str(int(v)) for v in c)))
    out = [ln for ln in _run(driver, "\n".join(lines) + "\n") if ln.startswith("finish")]
    assert len(out) == len(cases)
    for (N, c, model, mu, sigma, u), ln in zip(cases, out):
        f = ln.split()[1:]
        kw = {"mu": mu, "sigma": sigma} if model == 1 else {}
        ref = oracle.minentropy_counts(c, N, u_mode=u, **kw)
        for i, k in enumerate(("mu_hat", "sigma_hat", "h_min", "h_actual", "d_u",
                               "delta_h_m", "h_mod")):
            a, b = float(f[i]), ref[k]
            if math.isinf(b):
                assert math.isinf(a)
            else:
                assert abs(a - b) <= 1e-12, (k, a, b)
        assert int(f[7]) == ref["argmax_model"]


def test_output_bits_rule_matches_oracle(driver):
    cases = [(n, N, h, e) for n in (1, 64, 131072, 1 << 23, (1 << 40) + 17)
             for N in (1, 5, 8, 16) for h in (-1.0, 0.0, 0.5, 4.999, 5.0, 5.6, 8.0, 17.0)
             for e in (0.0, 0.5, 10.0, 64.0)]
    out = [ln for ln in _run(driver, "".join("bits %d %d %r %r\n" % c for c in cases))
           if ln.startswith("bits")]
    for (n, N, h, e), ln in zip(cases, out):
        assert int(ln.split()[1]) == oracle.output_bits(n, N, h, e), (n, N, h, e)


@pytest.mark.parametrize("words,seed", [(7, 1), (64, 2), (1000, 3), (4096, 4)])
def test_output_ring_invariants(driver, words, seed):
    out = [ln for ln in _run(driver, "ring %d %d 20000\n" % (words, seed))
           if ln.startswith("ring")]
    assert out and out[0].startswith("ring ok")
    alloc, rel = map(int, out[0].split()[2:])
    assert alloc > 100 and rel > 100


def test_oracle_selfcheck_under_sanitizers(tmp_path):
    """The C oracle's functions (bitwise, packed rows, packed, scalar
    estimator) on small cases, checked against each other, with the
    sanitizers watching every access."""
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = _build(tmp_path, "oracle_selfcheck",
                 ["gcc", "-std=c99", *SAN, "-fopenmp",
                  os.path.join(ROOT, "oracle", "selfcheck.c"),
                  os.path.join(ROOT, "oracle", "toeplitz_oracle.c"), "-lm"])
    out = _run(exe, "")
    assert any(ln.startswith("oracle selfcheck ok") for ln in out), out


def test_counts_consistency_guard(driver):
    """The host's guard on a full estimate's counts: bins + out-of-range
    must equal the samples counted; a lost or doubled partial histogram, or
    counts that wrap, fail it."""
    rng = np.random.default_rng(11)
    cases = []
    for K in (2, 32, 256):
        c = rng.integers(0, 1000, size=K)
        oob = int(rng.integers(0, 5))
        S = int(c.sum()) + oob
        cases.append((K, oob, S, c, 1))                        # consistent
        cases.append((K, oob, S + 1, c, 0))                    # one sample missing
        cases.append((K, oob, S - 1, c, 0))                    # one counted twice
        d = c.copy(); d[K // 2] += 17
        cases.append((K, oob, S, d, 0))                        # a row added twice
        cases.append((K, oob + 3, S, c, 0))                    # out-of-range miscounted
    big = np.zeros(4, dtype=np.uint64); big[0] = np.uint64(2**64 - 1); big[1] = np.uint64(5)
    cases.append((4, 0, 4, big, 0))                            # wraps to a small total
    cases.append((4, 0, 0, np.zeros(4, dtype=np.uint64), 1))   # empty estimate is consistent
    cases.append((4, 10, 5, np.zeros(4, dtype=np.uint64), 0))  # more out of range than samples
    text = "".join("counts %d %d %d %s\n" % (K, oob, S, " ".join(str(int(v)) for v in c))
                   for K, oob, S, c, _ in cases)
    out = [ln for ln in _run(driver, text) if ln.startswith("counts")]
    assert [int(ln.split()[1]) for ln in out] == [want for *_, want in cases]
