"""Pins for the Toeplitz-hash oracle (CPU only).

Each test checks the oracle against something other than its own formula:
a matrix assembled from the structural description of T (first row, first
column, constant diagonals), the circulant embedding of Definition 1, linear
algebra facts (linearity, unit vectors, special seeds, a shift relation), the
appendix's rotated-seed formulation, and brute force over every input of a
tiny size.  A dropped term, a wrong sign in an index or a transposed operand
in the oracle fails at least one of them.
"""
import itertools

import numpy as np
import pytest

import oracle
import qrng_inputs as qi


def rand_bits(k, rng):
    return rng.integers(0, 2, k, dtype=np.uint8)


def structural_T(a, n, m):
    """T built from its description in Sec. III.B: first row a_n, a_{n-1}, ...,
    a_1; first column a_n, a_{n+1}, ..., a_{n+m-1}; every other entry copies
    its upper-left neighbour (T_{i,j} = T_{i+1,j+1})."""
    T = np.zeros((m, n), dtype=np.uint8)
    for j in range(n):                 # first row: a_n ... a_1 (1-indexed)
        T[0, j] = a[n - 1 - j]
    for i in range(m):                 # first column: a_n ... a_{n+m-1}
        T[i, 0] = a[n - 1 + i]
    for i in range(1, m):
        for j in range(1, n):
            T[i, j] = T[i - 1, j - 1]
    return T


def gf2_matvec(T, r):
    return (T.astype(np.int64) @ r.astype(np.int64) & 1).astype(np.uint8)


@pytest.mark.parametrize("n,m", [(1, 1), (2, 1), (5, 3), (17, 17), (40, 7),
                                 (64, 64), (63, 30), (65, 1)])
def test_bitwise_matches_structural_matrix(n, m):
    rng = np.random.default_rng(n * 1000 + m)
    for _ in range(5):
        a = rand_bits(n + m - 1, rng)
        r = rand_bits(n, rng)
        T = structural_T(a, n, m)
        assert np.array_equal(oracle.toeplitz_matrix(a, n, m), T)
        assert np.array_equal(oracle.toeplitz_bitwise(r, a, m), gf2_matvec(T, r))


def test_bruteforce_all_inputs_tiny():
    # every raw block of n <= 10 bits against the structural matrix
    rng = np.random.default_rng(7)
    for n in range(1, 11):
        m = int(rng.integers(1, n + 1))
        a = rand_bits(n + m - 1, rng)
        T = structural_T(a, n, m)
        R = np.array(list(itertools.product([0, 1], repeat=n)), dtype=np.uint8)
        want = (R.astype(np.int64) @ T.T.astype(np.int64) & 1).astype(np.uint8)
        for t in range(len(R)):
            assert np.array_equal(oracle.toeplitz_bitwise(R[t], a, m), want[t])


def test_linearity():
    rng = np.random.default_rng(11)
    n, m = 1000, 613
    a = rand_bits(n + m - 1, rng)
    x1, x2 = rand_bits(n, rng), rand_bits(n, rng)
    y1 = oracle.toeplitz_bitwise(x1, a, m)
    y2 = oracle.toeplitz_bitwise(x2, a, m)
    assert np.array_equal(oracle.toeplitz_bitwise(x1 ^ x2, a, m), y1 ^ y2)


def test_unit_vectors_give_columns():
    # T e_j is column j: seed bits a_{n-j} (top) down to a_{n+m-1-j} (1-indexed)
    rng = np.random.default_rng(12)
    n, m = 97, 41
    a = rand_bits(n + m - 1, rng)
    for j in range(n):
        e = np.zeros(n, dtype=np.uint8)
        e[j] = 1
        col = a[n - 1 - j: n - 1 - j + m]
        assert np.array_equal(oracle.toeplitz_bitwise(e, a, m), col)


def test_special_seeds():
    rng = np.random.default_rng(13)
    n, m = 300, 200
    L = n + m - 1
    x = rand_bits(n, rng)
    # a single 1 at seed position t shifts x: y_i = x_{n-1+i-t}
    for t in [0, 1, n - 1, n, L - 1, 137]:
        a = np.zeros(L, dtype=np.uint8)
        a[t] = 1
        want = np.array([x[n - 1 + i - t] if 0 <= n - 1 + i - t < n else 0
                         for i in range(m)], dtype=np.uint8)
        assert np.array_equal(oracle.toeplitz_bitwise(x, a, m), want)
    # all-ones seed: every key bit is the parity of the whole block
    a = np.ones(L, dtype=np.uint8)
    assert np.all(oracle.toeplitz_bitwise(x, a, m) == (int(x.sum()) & 1))
    # zero block
    a = rand_bits(L, rng)
    assert not oracle.toeplitz_bitwise(np.zeros(n, np.uint8), a, m).any()


def test_shift_relation():
    # x' = (0, x_0..x_{n-2}) gives y'_i = y_{i-1} xor (s_{i-1} and x_{n-1})
    rng = np.random.default_rng(14)
    n, m = 257, 129
    a = rand_bits(n + m - 1, rng)
    x = rand_bits(n, rng)
    xs = np.concatenate([[0], x[:-1]]).astype(np.uint8)
    y = oracle.toeplitz_bitwise(x, a, m)
    ys = oracle.toeplitz_bitwise(xs, a, m)
    for i in range(1, m):
        assert ys[i] == (y[i - 1] ^ (a[i - 1] & x[n - 1]))


@pytest.mark.parametrize("n,m", [(8, 3), (20, 20), (33, 5), (50, 31)])
def test_circulant_embedding(n, m):
    # Definition 1: rows n..n+m-1 of A r' with r' = (r, 0^{m-1}) equal T r
    rng = np.random.default_rng(n + 31 * m)
    L = n + m - 1
    a = rand_bits(L, rng)
    r = rand_bits(n, rng)
    rp = np.concatenate([r, np.zeros(m - 1, np.uint8)])
    A = oracle.circulant_matrix(a, L)
    # Definition 1 as stated: column j+1 starts with the last entry of column j
    for j in range(L - 1):
        assert A[0, j + 1] == A[L - 1, j]
        assert np.array_equal(A[1:, j + 1], A[:-1, j])
    kp = gf2_matvec(A, rp)
    assert np.array_equal(kp[n - 1: n - 1 + m], oracle.toeplitz_bitwise(r, a, m))


@pytest.mark.parametrize("n,m", [(16, 10), (64, 40), (100, 100), (129, 3)])
def test_appendix_formulation_is_a_seed_rotation(n, m):
    # The appendix keeps the FIRST m circulant rows; that is the text's
    # matrix for the seed rotated by n-1: s_B[t] = s_A[(t + n - 1) mod L].
    rng = np.random.default_rng(n * 7 + m)
    L = n + m - 1
    sA = rand_bits(L, rng)
    sB = np.array([sA[(t + n - 1) % L] for t in range(L)], dtype=np.uint8)
    r = rand_bits(n, rng)
    rp = np.concatenate([r, np.zeros(m - 1, np.uint8)])
    first_rows = gf2_matvec(oracle.circulant_matrix(sB, L), rp)[:m]
    assert np.array_equal(first_rows, oracle.toeplitz_bitwise(r, sA, m))


@pytest.mark.parametrize("n,m", [(1, 1), (64, 64), (65, 63), (1000, 625),
                                 (4096, 2560), (131072, 81920), (12345, 6789)])
def test_three_oracle_tiers_agree(n, m):
    rng = np.random.default_rng(n ^ m)
    L = n + m - 1
    xw = qi.gen_bits(n, int(rng.integers(1 << 30)))
    sw = qi.gen_seed_words(L, int(rng.integers(1 << 30)))   # tail bits random
    r = oracle.unpack_bits(xw, n)
    a = oracle.unpack_bits(sw, L)
    o1 = oracle.toeplitz_bitwise(r, a, m)
    o2 = oracle.toeplitz_packed(xw, n, sw, m)
    o3 = oracle.toeplitz_fft64(r, a, m)
    o3p = oracle.toeplitz_fft64(r, a, m, pad_pow2=True)
    assert np.array_equal(oracle.pack_bits(o1), o2)
    assert np.array_equal(o1, o3)
    assert np.array_equal(o1, o3p)
    rows = rng.integers(0, m, 50)
    assert np.array_equal(oracle.toeplitz_rows(xw, n, sw, L, rows), o1[rows])


def test_packed_tail_bits_are_zero_and_garbage_ignored():
    n, m = 200, 77
    rng = np.random.default_rng(3)
    xw = qi.gen_bits(n, 1)
    sw = qi.gen_seed_words(n + m - 1, 2)
    y = oracle.toeplitz_packed(xw, n, sw, m)
    assert int(y[-1]) >> (m % 64) == 0
    # flipping bits beyond n in x or beyond L in the seed changes nothing
    xw2 = xw.copy()
    xw2[-1] ^= np.uint64(~((1 << (n % 64)) - 1) & ((1 << 64) - 1))
    sw2 = sw.copy()
    L = n + m - 1
    sw2[-1] ^= np.uint64(~((1 << (L % 64)) - 1) & ((1 << 64) - 1))
    assert np.array_equal(oracle.toeplitz_packed(xw2, n, sw2, m), y)


def test_modified_toeplitz_text_formula():
    # Sec. III.D: k = (A, I_m) r.  Check against the matrix assembled from the
    # printed layout (first row a_{n-m} .. a_1 then e_1; last row a_{n-1} .. a_m
    # then e_m) and against the circulant route of the text: A_c (n x n,
    # Definition 1 on a' = (a_1..a_{n-1}, a_n)), r' = (r_1..r_{n-m}, 0^m), keep
    # rows n-m..n-1 (1-indexed), add r_{i+1} to row i.
    rng = np.random.default_rng(21)
    for n, m in [(10, 4), (33, 20), (64, 1), (50, 49)]:
        a = rand_bits(n - 1, rng)
        r = rand_bits(n, rng)
        w = n - m
        Am = np.zeros((m, n), np.uint8)
        for j in range(w):
            Am[0, j] = a[w - 1 - j]
        for i in range(m):
            Am[i, 0] = a[w - 1 + i]
        for i in range(1, m):
            for j in range(1, w):
                Am[i, j] = Am[i - 1, j - 1]
        Am[:, w:] = np.eye(m, dtype=np.uint8)
        want = gf2_matvec(Am, r)
        assert np.array_equal(oracle.modified_toeplitz(r, a, m), want)
        ap = np.concatenate([a, [int(rng.integers(0, 2))]]).astype(np.uint8)
        rp = np.concatenate([r[:w], np.zeros(m, np.uint8)])
        kp = gf2_matvec(oracle.circulant_matrix(ap, n), rp)
        assert np.array_equal(kp[w - 1: w - 1 + m] ^ r[w:], want)


def test_modified_toeplitz_packed_matches_definition():
    # the packed column-split route against the product written out, including
    # m > n - m (more key bits than A has columns), m = n (k = r), m = 1 and
    # lengths that are not multiples of 64
    rng = np.random.default_rng(23)
    for n, m in [(1, 1), (2, 1), (9, 9), (64, 40), (65, 64), (100, 1), (130, 97), (200, 150),
                 (257, 100), (300, 299)]:
        a = rand_bits(max(n - 1, 1), rng)
        r = rand_bits(n, rng)
        want = oracle.pack_bits(oracle.modified_toeplitz(r, a, m))
        got = oracle.modified_toeplitz_packed(oracle.pack_bits(r), n, oracle.pack_bits(a), m)
        assert np.array_equal(got, want), (n, m)
        if m == n:
            assert np.array_equal(got, oracle.pack_bits(r))


def test_modified_toeplitz_columns():
    # unit raw vectors read the columns of (A, I_m): e_j (j < n-m) gives
    # A[:, j] = a[n-m-1+i-j], e_{n-m+i} gives key bit i alone
    rng = np.random.default_rng(24)
    n, m = 40, 25
    a = rand_bits(n - 1, rng)
    w = n - m
    for j in range(n):
        r = np.zeros(n, np.uint8)
        r[j] = 1
        k = oracle.modified_toeplitz(r, a, m)
        if j < w:
            assert np.array_equal(k, np.array([a[w - 1 + i - j] for i in range(m)], np.uint8))
        else:
            e = np.zeros(m, np.uint8)
            e[j - w] = 1
            assert np.array_equal(k, e)
