/*
 * CPU oracle for the GF(2) Toeplitz hash -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the bench
 * may load this library.  It shares no code, header or table with the HIP
 * library: it is deliberately plain, slow and obviously correct.
 *
 * The operation (paper, Sec. III.B, the m x n Toeplitz matrix T and k = T r):
 * with 1-indexed seed a_1..a_{n+m-1} and raw bits r_1..r_n, the i-th key bit is
 *     k_i = sum_{j=1..n} a_{n+i-j} * r_j   (mod 2),   i = 1..m,
 * i.e. T_{ij} = a_{n+i-j}: the first row is a_n, a_{n-1}, ..., a_1 and every
 * row below is the row above shifted right by one with a new seed bit in
 * front.  In 0-indexed form (s[t] = a_{t+1}, x[j] = r_{j+1}, y[i] = k_{i+1}):
 *     y[i] = XOR_{j=0..n-1} ( s[n-1+i-j] AND x[j] ),   i = 0..m-1.
 *
 * Bit layout of the packed variants: bit b of a bit string lives in 64-bit
 * word b/64 at position b%64 (LSB first, little-endian words).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* O1: the definition above, one byte per bit, one row per outer iteration. */
void oracle_toeplitz_bitwise(const uint8_t *r, uint64_t n, const uint8_t *a,
                             uint64_t m, uint8_t *k)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (int64_t)m; ++i) {
        uint8_t acc = 0;
        for (uint64_t j = 0; j < n; ++j)
            acc ^= (uint8_t)(a[n - 1 + (uint64_t)i - j] & r[j] & 1u);
        k[i] = acc;
    }
}

static inline int get_bit(const uint64_t *w, uint64_t b)
{
    return (int)((w[b >> 6] >> (b & 63)) & 1u);
}

/*
 * O2: the same sum evaluated 64 terms at a time.  Reindexing j' = n-1-j turns
 * row i into  y[i] = XOR_{j'} s[i+j'] AND xr[j'],  with xr the bit reversal of
 * x, so a row is the parity of (64-bit window of s starting at bit i+64w) AND
 * (word w of xr), summed over w.  Only the rows listed in `rows` are computed;
 * out[t] receives row rows[t] (0 or 1).
 */
void oracle_toeplitz_packed_rows(const uint64_t *x, uint64_t n,
                                 const uint64_t *s, uint64_t L,
                                 const uint64_t *rows, uint64_t nrows,
                                 uint8_t *out)
{
    uint64_t nw = (n + 63) / 64;
    uint64_t sw = (L + 63) / 64;
    uint64_t *xr = (uint64_t *)calloc(nw ? nw : 1, sizeof(uint64_t));
    for (uint64_t j = 0; j < n; ++j)
        if (get_bit(x, j))
            xr[(n - 1 - j) >> 6] |= (uint64_t)1 << ((n - 1 - j) & 63);

    int64_t t;
#pragma omp parallel for schedule(dynamic, 64)
    for (t = 0; t < (int64_t)nrows; ++t) {
        uint64_t i = rows[t];
        uint64_t acc = 0;
        for (uint64_t w = 0; w < nw; ++w) {
            uint64_t b = i + 64 * w;          /* first seed bit of the window */
            uint64_t q = b >> 6, sh = b & 63;
            uint64_t lo = q < sw ? s[q] : 0;
            uint64_t hi = q + 1 < sw ? s[q + 1] : 0;
            uint64_t win = sh ? ((lo >> sh) | (hi << (64 - sh))) : lo;
            /* seed bits at or beyond L are not part of the seed */
            if (b + 64 > L) {
                uint64_t keep = L > b ? L - b : 0;
                win &= keep >= 64 ? ~(uint64_t)0 : (((uint64_t)1 << keep) - 1);
            }
            acc ^= win & xr[w];
        }
        out[t] = (uint8_t)(__builtin_popcountll(acc) & 1);
    }
    free(xr);
}

/* O2 over every row, packed into y (LSB-first words, bits >= m left zero). */
void oracle_toeplitz_packed(const uint64_t *x, uint64_t n, const uint64_t *s,
                            uint64_t m, uint64_t *y)
{
    uint64_t L = n + m - 1;
    uint64_t *rows = (uint64_t *)malloc((m ? m : 1) * sizeof(uint64_t));
    uint8_t *bits = (uint8_t *)malloc(m ? m : 1);
    for (uint64_t i = 0; i < m; ++i)
        rows[i] = i;
    oracle_toeplitz_packed_rows(x, n, s, L, rows, m, bits);
    memset(y, 0, ((m + 63) / 64) * sizeof(uint64_t));
    for (uint64_t i = 0; i < m; ++i)
        if (bits[i])
            y[i >> 6] |= (uint64_t)1 << (i & 63);
    free(rows);
    free(bits);
}

/* Number of OpenMP threads the oracle runs with (reported by the bench). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
