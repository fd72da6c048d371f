"""CPU oracle for the QRNG post-processing path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_2011_04130_amd``) and never imports it; both sides receive the same
seeded inputs from ``qrng_inputs``.

What it computes, each function citing the part of the paper it follows
(Zhao, "Performance Optimization on Practical Quantum Random Number
Generators", arXiv 2011.04130):

* ``toeplitz_bitwise`` / ``toeplitz_packed`` / ``toeplitz_rows`` -- the
  Toeplitz hash k = T r mod 2 of Sec. III.B (the m x n matrix with
  T_ij = a_{n+i-j}), written out as its definition in plain C
  (``toeplitz_oracle.c``).
* ``toeplitz_matrix`` -- the same matrix materialised (tiny sizes only).
* ``toeplitz_fft64`` -- the paper's own accelerated method (Sec. III.B,
  Definition 1 and Theorems 1-2): embed T in the (n+m-1)-square circulant,
  zero-pad r, k' = F^-1(F a . F r'), round, mod 2, keep k_n..k_{n+m-1}.
* ``modified_toeplitz`` -- Sec. III.D, k = (A, I_m) r with the (n-1)-bit seed;
  ``modified_toeplitz_packed`` the same on packed words through the
  column split (A x_low with the C hash, plus the raw tail).
* ``gaussian_model``, ``minentropy_dists``, ``minentropy_counts`` -- Sec. II:
  min-entropy -log2 max P, the statistical distance d_U over the set U, the
  finite-size correction Delta H_m = log2(d_U / 2^-(N+1) + 1) and
  H_modify = H_min - Delta H_m.
* ``output_bits`` -- the output-length rule of Sec. III.B,
  m = n H/N - 2 log2(1/eps), with H taken as whole bits per sample.

Readings of points where the paper is silent or garbled are listed in the
repository design notes; each is also stated in the docstring that uses it.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "liboracle.so")
_lib = None

# ---------------------------------------------------------------------------
# build / load of the C part
# ---------------------------------------------------------------------------


def build(force: bool = True) -> str:
    """Compile ``toeplitz_oracle.c`` into ``_build/liboracle.so`` (gcc, OpenMP)."""
    os.makedirs(_BUILD, exist_ok=True)
    src = os.path.join(_HERE, "toeplitz_oracle.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c99", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        lib.oracle_toeplitz_bitwise.argtypes = [u8p, ctypes.c_uint64, u8p,
                                                ctypes.c_uint64, u8p]
        lib.oracle_toeplitz_packed_rows.argtypes = [
            u64p, ctypes.c_uint64, u64p, ctypes.c_uint64, u64p,
            ctypes.c_uint64, u8p]
        lib.oracle_toeplitz_packed.argtypes = [u64p, ctypes.c_uint64, u64p,
                                               ctypes.c_uint64, u64p]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_minentropy_scalar.argtypes = [u64p, ctypes.c_int, ctypes.c_int,
                                                 ctypes.c_double, ctypes.c_double,
                                                 ctypes.c_int,
                                                 ctypes.POINTER(ctypes.c_double)]
        lib.oracle_minentropy_scalar.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def num_threads() -> int:
    """OpenMP threads the C oracle uses."""
    return int(_load().oracle_num_threads())


# ---------------------------------------------------------------------------
# bit helpers (layout: bit b is bit b%64 of little-endian 64-bit word b//64)
# ---------------------------------------------------------------------------


def unpack_bits(words: np.ndarray, nbits: int) -> np.ndarray:
    """uint64 words -> one uint8 (0/1) per bit, LSB first."""
    b = np.unpackbits(np.ascontiguousarray(words, dtype="<u8").view(np.uint8),
                      bitorder="little")
    return b[:nbits].copy()


def pack_bits(bits: np.ndarray) -> np.ndarray:
    """one uint8 (0/1) per bit -> uint64 words, LSB first, tail bits zero."""
    bits = np.asarray(bits, dtype=np.uint8)
    nw = (len(bits) + 63) // 64
    padded = np.zeros(nw * 64, dtype=np.uint8)
    padded[: len(bits)] = bits & 1
    return np.packbits(padded, bitorder="little").view("<u8").copy()


# ---------------------------------------------------------------------------
# Toeplitz hash (Sec. III.B)
# ---------------------------------------------------------------------------


def toeplitz_bitwise(r_bits: np.ndarray, a_bits: np.ndarray, m: int) -> np.ndarray:
    """k_i = sum_j a_{n+i-j} r_j mod 2 (the m x n matrix of Sec. III.B).

    ``r_bits``: n raw bits (uint8 0/1); ``a_bits``: at least n+m-1 seed bits.
    Returns m key bits (uint8).  Plain C, one byte per bit.
    """
    r = np.ascontiguousarray(r_bits, dtype=np.uint8)
    a = np.ascontiguousarray(a_bits, dtype=np.uint8)
    n = len(r)
    if m == 0:
        return np.zeros(0, dtype=np.uint8)
    assert len(a) >= n + m - 1, "seed shorter than n+m-1"
    k = np.zeros(m, dtype=np.uint8)
    _load().oracle_toeplitz_bitwise(_p(r, ctypes.c_uint8), n,
                                    _p(a, ctypes.c_uint8), m,
                                    _p(k, ctypes.c_uint8))
    return k


def toeplitz_packed(x_words: np.ndarray, n: int, s_words: np.ndarray, m: int) -> np.ndarray:
    """Same hash on packed words; returns ceil(m/64) uint64 words (tail zero)."""
    x = np.ascontiguousarray(x_words, dtype=np.uint64)
    s = np.ascontiguousarray(s_words, dtype=np.uint64)
    assert len(x) * 64 >= n and len(s) * 64 >= n + m - 1
    y = np.zeros(max((m + 63) // 64, 1), dtype=np.uint64)
    if m:
        _load().oracle_toeplitz_packed(_p(x, ctypes.c_uint64), n,
                                       _p(s, ctypes.c_uint64), m,
                                       _p(y, ctypes.c_uint64))
    return y[: (m + 63) // 64]


def toeplitz_rows(x_words: np.ndarray, n: int, s_words: np.ndarray, L: int,
                  rows) -> np.ndarray:
    """Selected rows y[rows[t]] of the hash (each row costs exactly n bit-ANDs)."""
    x = np.ascontiguousarray(x_words, dtype=np.uint64)
    s = np.ascontiguousarray(s_words, dtype=np.uint64)
    rr = np.ascontiguousarray(np.asarray(rows, dtype=np.uint64))
    out = np.zeros(max(len(rr), 1), dtype=np.uint8)
    if len(rr):
        assert int(rr.max()) + n <= L, "row index needs seed bits beyond L"
        _load().oracle_toeplitz_packed_rows(_p(x, ctypes.c_uint64), n,
                                            _p(s, ctypes.c_uint64), L,
                                            _p(rr, ctypes.c_uint64), len(rr),
                                            _p(out, ctypes.c_uint8))
    return out[: len(rr)]


def toeplitz_matrix(a_bits: np.ndarray, n: int, m: int) -> np.ndarray:
    """The m x n matrix of Sec. III.B materialised: T[i, j] = a_{n+i-j}.

    0-indexed: T[i, j] = a_bits[n-1+i-j].  Only for tiny n, m.
    """
    a = np.asarray(a_bits, dtype=np.uint8)
    T = np.zeros((m, n), dtype=np.uint8)
    for i in range(m):
        for j in range(n):
            T[i, j] = a[n - 1 + i - j]
    return T


def circulant_matrix(a_bits: np.ndarray, L: int) -> np.ndarray:
    """Definition 1: the L x L circulant whose first column is a_1..a_L.

    Column j+1 is column j rotated down by one, so A[i, j] = a[(i-j) mod L].
    """
    a = np.asarray(a_bits[:L], dtype=np.uint8)
    A = np.zeros((L, L), dtype=np.uint8)
    for i in range(L):
        for j in range(L):
            A[i, j] = a[(i - j) % L]
    return A


def toeplitz_fft64(r_bits: np.ndarray, a_bits: np.ndarray, m: int,
                   pad_pow2: bool = False, guard: float = 0.25) -> np.ndarray:
    """The paper's accelerated method (Sec. III.B) in float64.

    r' = (r_1..r_n, 0^{m-1}); k' = F^-1(F a . F r') is the circulant product
    A r' of Definition 1 (Theorems 1-2); round, mod 2, keep k'_n..k'_{n+m-1}.
    With ``pad_pow2`` both vectors are zero-padded to the next power of two:
    the kept rows never wrap (their indices n-1+i-j stay inside [0, n+m-1)),
    so the result is unchanged and only the transform length differs (the
    paper notes power-of-two lengths run faster, Sec. III.C).

    Exactness: every entry of k' is an integer in [0, n].  The result is
    rejected unless every kept value lies within ``guard`` of an integer.
    """
    r = np.asarray(r_bits, dtype=np.float64)
    n = len(r)
    L = n + m - 1
    if m == 0:
        return np.zeros(0, dtype=np.uint8)
    a = np.asarray(a_bits[:L], dtype=np.float64)
    nfft = L if not pad_pow2 else 1 << (L - 1).bit_length()
    fa = np.fft.rfft(a, nfft)
    fr = np.fft.rfft(r, nfft)        # rfft zero-pads r to nfft (the r' of the paper)
    kp = np.fft.irfft(fa * fr, nfft)
    kept = kp[n - 1: n - 1 + m]
    ri = np.rint(kept)
    err = float(np.max(np.abs(kept - ri))) if m else 0.0
    if not err < guard:
        raise ArithmeticError("float64 FFT rounding margin exceeded: %g" % err)
    return (ri.astype(np.int64) & 1).astype(np.uint8)


def modified_toeplitz(r_bits: np.ndarray, a_bits: np.ndarray, m: int) -> np.ndarray:
    """Sec. III.D: k = A_m r with A_m = (A, I_m) and an (n-1)-bit seed.

    A is the m x (n-m) Toeplitz block whose first row is a_{n-m}, ..., a_1 and
    last row a_{n-1}, ..., a_m: A[i, j] = a_{n-m+i-j} (1-indexed i, j), i.e.
    0-indexed A[i, j] = a_bits[n-m-1+i-j].  The identity block adds raw bit
    r_{n-m+i} to key bit k_i.  Written out as the matrix product, mod 2.
    """
    r = np.asarray(r_bits, dtype=np.uint8)
    a = np.asarray(a_bits, dtype=np.uint8)
    n = len(r)
    assert 0 <= m <= n and len(a) >= n - 1
    w = n - m
    k = np.zeros(m, dtype=np.uint8)
    for i in range(m):
        acc = 0
        for j in range(w):
            acc ^= int(a[w - 1 + i - j]) & int(r[j])
        acc ^= int(r[w + i])
        k[i] = acc
    return k


def modified_toeplitz_packed(x_words: np.ndarray, n: int, a_words: np.ndarray,
                             m: int) -> np.ndarray:
    """Sec. III.D on packed words, ceil(m/64) uint64 words (tail zero).

    The columns of (A, I_m) split the product: A times the first n-m raw bits
    is the Sec. III.B hash of an (n-m)-bit block with the same seed (A[i, j] =
    a[n-m-1+i-j], 0-indexed, is T[i][j] = s[n'-1+i-j] with n' = n-m), and I_m
    adds raw bits n-m .. n-1.  ``modified_toeplitz`` (the product written out)
    pins this route.
    """
    w = n - m
    assert 0 <= m <= n
    if w > 0:
        y = toeplitz_packed(x_words, w, a_words, m)
    else:
        y = np.zeros((m + 63) // 64, dtype=np.uint64)
    tail = pack_bits(unpack_bits(x_words, n)[w:n])
    return (y ^ tail[: len(y)]).astype(np.uint64)


# ---------------------------------------------------------------------------
# min-entropy with the statistical-distance correction (Sec. II)
# ---------------------------------------------------------------------------

U_MODEL_ARGMAX = 0   # U = {argmax P}
U_BOTH_ARGMAX = 1    # U = {argmax P, argmax P'}
U_ALL = 2            # U = every sample value (total-variation distance)
TIE_REL = 1e-9       # model probabilities this close (relative) are a tie


def _phi(z: float) -> float:
    """Standard normal CDF, Phi(z) = erfc(-z/sqrt 2)/2 (libm erfc)."""
    return 0.5 * math.erfc(-z / math.sqrt(2.0))


def gaussian_model(N: int, mu: float, sigma: float) -> np.ndarray:
    """The ideal distribution P of an N-bit ADC fed by a Gaussian (Sec. II.B).

    Value v takes the mass of [v - 1/2, v + 1/2); the two end codes 0 and
    2^N - 1 also take the clipped tails.
    """
    K = 1 << N
    P = np.empty(K, dtype=np.float64)
    if not sigma > 0:
        # every sample equal: the fitted model is a point mass
        P[:] = 0.0
        P[int(min(max(math.floor(mu + 0.5), 0), K - 1))] = 1.0
        return P
    for v in range(K):
        lo = 0.0 if v == 0 else _phi((v - 0.5 - mu) / sigma)
        hi = 1.0 if v == K - 1 else _phi((v + 0.5 - mu) / sigma)
        P[v] = hi - lo
    return P


def minentropy_dists(P: np.ndarray, Pa: np.ndarray, N: int,
                     u_mode: int = U_MODEL_ARGMAX) -> dict:
    """Sec. II.A/II.C on an ideal distribution P and an actual one P'.

    H_min = -log2 max P; H'_min = -log2 max P'; the mutual information
    I(G:E) = H_min - H'_min; d_U = (1/2) sum_{x in U} |P'(x) - P(x)|;
    Delta H_m = log2(d_U / 2^-(N+1) + 1) with N the ADC bits per sample;
    H_modify = H_min - Delta H_m.  U is the argmax of P by default (the
    chain of inequalities replaces sum_U P by 2^-H_min), the lowest value when
    several share the maximum (within TIE_REL relative) -- the reading that
    reproduces the worked example's Delta H_m of Sec. II.C, whose model has
    two equal central bins.  U_BOTH_ARGMAX takes every value that shares the
    maximum of P together with argmax P': the conservative set, whose d_U is
    at least that of any one tied value.
    """
    P = np.asarray(P, dtype=np.float64)
    Pa = np.asarray(Pa, dtype=np.float64)
    pmax = float(P.max())
    # values whose model probability equals the maximum; values within
    # TIE_REL of it count as equal (a model centred half way between two codes
    # gives two exactly equal bins, which rounding must not separate)
    tied = np.flatnonzero(P >= pmax * (1.0 - TIE_REL))
    um = int(tied[0])
    ua = int(np.argmax(Pa))         # first maximum: lowest value on ties
    h_min = -math.log2(pmax)
    h_act = -math.log2(float(Pa[ua])) if Pa[ua] > 0 else float("inf")
    if u_mode == U_MODEL_ARGMAX:
        U = [um]
    elif u_mode == U_BOTH_ARGMAX:
        U = sorted({*tied.tolist(), ua})
    elif u_mode == U_ALL:
        U = list(range(len(P)))
    else:
        raise ValueError("unknown U mode")
    d_u = 0.5 * sum(abs(float(Pa[u]) - float(P[u])) for u in U)
    delta = math.log2(d_u * 2.0 ** (N + 1) + 1.0)
    return {
        "h_min": h_min,
        "h_actual": h_act,
        "mutual_info": h_min - h_act,
        "d_u": d_u,
        "delta_h_m": delta,
        "h_mod": h_min - delta,
        "argmax_model": um,
        "argmax_empirical": ua,
    }


def minentropy_counts(counts: np.ndarray, N: int, mu: float | None = None,
                      sigma: float | None = None,
                      u_mode: int = U_MODEL_ARGMAX,
                      sigma_classical: float | None = None) -> dict:
    """Min-entropy of an ADC histogram with the correction of Sec. II.C.

    P' = counts / S is the actual distribution.  The ideal P is the Gaussian
    ADC model; its mean and standard deviation are either given or measured
    from the same samples (population moments), as the paper measures the
    noise variance (Sec. II.B).  With ``sigma_classical`` the model keeps only
    the quantum part of the measured variance, sigma_q^2 = sigma_{q+c}^2 -
    sigma_c^2 (Sec. II.B; a point mass when that is not positive).
    """
    c = np.asarray(counts, dtype=np.float64)
    S = float(c.sum())
    assert S > 0
    v = np.arange(len(c), dtype=np.float64)
    if mu is None or sigma is None:
        mu_hat = float((v * c).sum() / S)
        var = float((((v - mu_hat) ** 2) * c).sum() / S)
        if sigma_classical is not None:
            var -= float(sigma_classical) ** 2
        sigma_hat = math.sqrt(var) if var > 0 else 0.0
    else:
        mu_hat, sigma_hat = float(mu), float(sigma)
    P = gaussian_model(N, mu_hat, sigma_hat)
    out = minentropy_dists(P, c / S, N, u_mode)
    out["mu_hat"] = mu_hat
    out["sigma_hat"] = sigma_hat
    return out


def minentropy_counts_scalar(counts: np.ndarray, N: int, mu: float | None = None,
                             sigma: float | None = None,
                             u_mode: int = U_MODEL_ARGMAX) -> dict:
    """The same estimate from the C oracle's separate scalar-loop version
    (its model CDF goes through erf instead of erfc); a cross-check of
    ``minentropy_counts``, not a third reading."""
    c = np.ascontiguousarray(counts, dtype=np.uint64)
    assert len(c) == 1 << N
    out = (ctypes.c_double * 8)()
    given = mu is not None and sigma is not None
    rc = _load().oracle_minentropy_scalar(_p(c, ctypes.c_uint64), N, int(given),
                                          float(mu or 0.0), float(sigma or 0.0), u_mode, out)
    if rc:
        raise ValueError("no samples")
    keys = ("mu_hat", "sigma_hat", "h_min", "h_actual", "d_u", "delta_h_m", "h_mod")
    r = {k: float(out[i]) for i, k in enumerate(keys)}
    r["argmax_model"] = int(out[7])
    return r


SPLITMIX_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed: int, count: int) -> np.ndarray:
    """Outputs 0..count-1 of the SplitMix64 generator (Steele, Lea and Flood,
    OOPSLA 2014) from state `seed`: output t = mix(seed + (t+1) gamma), mix =
    xor-shift 30, multiply 0xbf58476d1ce4e5b9, xor-shift 27, multiply
    0x94d049bb133111eb, xor-shift 31 (all mod 2^64)."""
    with np.errstate(over="ignore"):
        t = np.arange(1, count + 1, dtype=np.uint64)
        z = np.uint64(seed & (2 ** 64 - 1)) + t * np.uint64(SPLITMIX_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def subset_mask(S: int, seed: int, keep_thr: int) -> np.ndarray:
    """The random subset of Sec. II.C's cheaper estimate: sample t is kept
    when the high 32 bits of SplitMix64 output t are below keep_thr (all
    samples when keep_thr is 0)."""
    if keep_thr == 0:
        return np.ones(S, dtype=bool)
    return (splitmix64(seed, S) >> np.uint64(32)) < np.uint64(keep_thr)


def histogram(samples: np.ndarray, N: int) -> np.ndarray:
    """Counts of each N-bit sample value (uint64)."""
    return np.bincount(np.asarray(samples, dtype=np.int64),
                       minlength=1 << N).astype(np.uint64)


def output_bits(n: int, N: int, h_mod: float, log2_inv_eps: float = 0.0) -> int:
    """Output length m = n H/N - 2 log2(1/eps) (Sec. III.B, leftover hash lemma).

    Reading: H is counted in whole bits per sample (floor of H_modify, never
    below 0 and never above the sample width N), the security term is rounded
    up, and m is clamped at 0 (it cannot exceed n once H <= N).
    """
    if math.isnan(h_mod):
        raise ValueError("h_mod is NaN")
    h = math.floor(h_mod) if math.isfinite(h_mod) else (N if h_mod > 0 else 0)
    h = min(max(h, 0), N)
    sec = math.ceil(2.0 * log2_inv_eps) if log2_inv_eps > 0 else 0
    m = (n * h) // N - sec
    return int(min(max(m, 0), n))
