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

/*
 * Second, scalar-loop implementation of the min-entropy estimate of Sec. II
 * (written apart from the numpy one, as a cross-check of it): from the 2^N
 * counts of an N-bit ADC, the Gaussian model P (mean and population s.d. of
 * the counts, or the given ones), H_min = -log2 max P, the statistical
 * distance d_U = (1/2) sum_{x in U} |P'(x) - P(x)| with P' = counts / S,
 * Delta H_m = log2(d_U 2^(N+1) + 1) and H_modify = H_min - Delta H_m.
 * The model's bin v is Phi(v + 1/2) - Phi(v - 1/2) with Phi written through
 * erf (the numpy route uses erfc); codes 0 and 2^N - 1 take the tails.
 * U: 0 = the lowest value within 1e-9 (relative) of max P; 1 = every such
 * value plus the lowest value of largest count; 2 = all values.
 * out[0..7] = mu, sigma, h_min, h_actual, d_u, delta_h_m, h_mod,
 * argmax_model.  Returns 0, or -1 when S = 0.
 */
#include <math.h>

static double cdf_erf(double z) { return 0.5 * (1.0 + erf(z / sqrt(2.0))); }

int oracle_minentropy_scalar(const uint64_t *counts, int N, int given, double mu_g,
                             double sigma_g, int u_mode, double *out)
{
    const int K = 1 << N;
    double S = 0.0, mu, sigma;
    for (int v = 0; v < K; ++v) S += (double)counts[v];
    if (!(S > 0.0)) return -1;
    if (given) {
        mu = mu_g;
        sigma = sigma_g;
    } else {
        double s1 = 0.0, s2 = 0.0;
        for (int v = 0; v < K; ++v) s1 += v * (double)counts[v];
        mu = s1 / S;
        for (int v = 0; v < K; ++v) {
            const double d = v - mu;
            s2 += d * d * (double)counts[v];
        }
        sigma = s2 > 0.0 ? sqrt(s2 / S) : 0.0;
    }
    double *P = (double *)malloc(sizeof(double) * K);
    if (sigma > 0.0) {
        for (int v = 0; v < K; ++v) {
            const double hi = v == K - 1 ? 1.0 : cdf_erf((v + 0.5 - mu) / sigma);
            const double lo = v == 0 ? 0.0 : cdf_erf((v - 0.5 - mu) / sigma);
            P[v] = hi - lo;
        }
    } else {
        double at = floor(mu + 0.5);
        if (at < 0) at = 0;
        if (at > K - 1) at = K - 1;
        for (int v = 0; v < K; ++v) P[v] = v == (int)at ? 1.0 : 0.0;
    }
    double pmax = 0.0;
    int ua = 0;
    for (int v = 0; v < K; ++v) {
        if (P[v] > pmax) pmax = P[v];
        if (counts[v] > counts[ua]) ua = v;
    }
    int um = -1;
    double d = 0.0;
    for (int v = 0; v < K; ++v) {
        const int tied = P[v] >= pmax * (1.0 - 1e-9);
        if (tied && um < 0) um = v;
        int in_u;
        if (u_mode == 2) in_u = 1;
        else if (u_mode == 1) in_u = tied || v == ua;
        else in_u = 0;
        if (in_u) d += fabs((double)counts[v] / S - P[v]);
    }
    if (u_mode == 0) d = fabs((double)counts[um] / S - P[um]);
    d *= 0.5;
    const double h_min = -log2(pmax);
    const double delta = log2(d * pow(2.0, N + 1) + 1.0);
    out[0] = mu;
    out[1] = sigma;
    out[2] = h_min;
    out[3] = counts[ua] ? -log2((double)counts[ua] / S) : INFINITY;
    out[4] = d;
    out[5] = delta;
    out[6] = h_min - delta;
    out[7] = um;
    free(P);
    return 0;
}
