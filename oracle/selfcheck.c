/*
 * Self-check driver of the C oracle -- TEST INFRASTRUCTURE ONLY (built with
 * the address and undefined-behaviour sanitizers by the host-only tests).
 * Runs every function of toeplitz_oracle.c on small random cases, including
 * lengths that are not multiples of 64 and m = 1, m = n, and checks them
 * against each other: the bitwise sum (one byte per bit), the packed sum
 * over all rows and over listed rows, and the scalar estimator on a few
 * histograms (finite results, d_U within [0, 1]).  Prints
 * "oracle selfcheck ok" when everything agrees.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_toeplitz_bitwise(const uint8_t *r, uint64_t n, const uint8_t *a, uint64_t m,
                             uint8_t *k);
void oracle_toeplitz_packed_rows(const uint64_t *x, uint64_t n, const uint64_t *s, uint64_t L,
                                 const uint64_t *rows, uint64_t nrows, uint8_t *out);
void oracle_toeplitz_packed(const uint64_t *x, uint64_t n, const uint64_t *s, uint64_t m,
                            uint64_t *y);
int oracle_minentropy_scalar(const uint64_t *counts, int N, int given, double mu_g,
                             double sigma_g, int u_mode, double *out);

static uint64_t st = 0x243f6a8885a308d3ull;
static uint64_t rnd(void) { /* xorshift64 */
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    return st;
}

static int fail(const char *what, uint64_t n, uint64_t m) {
    printf("oracle selfcheck FAILED: %s (n=%llu m=%llu)\n", what, (unsigned long long)n,
           (unsigned long long)m);
    return 1;
}

int main(void) {
    const uint64_t sizes[][2] = {{1, 1}, {2, 1}, {2, 2}, {63, 30}, {64, 64}, {65, 1},
                                 {100, 77}, {129, 128}, {300, 200}, {1000, 999}};
    for (size_t t = 0; t < sizeof sizes / sizeof sizes[0]; ++t) {
        const uint64_t n = sizes[t][0], m = sizes[t][1], L = n + m - 1;
        uint8_t *r = malloc(n), *a = malloc(L), *k = malloc(m), *kr = malloc(m);
        uint64_t *x = calloc((n + 63) / 64, 8), *s = calloc((L + 63) / 64, 8);
        uint64_t *y = calloc((m + 63) / 64, 8), *rows = malloc(m * 8);
        for (uint64_t j = 0; j < n; ++j) {
            r[j] = rnd() & 1;
            x[j / 64] |= (uint64_t)r[j] << (j % 64);
        }
        for (uint64_t j = 0; j < L; ++j) {
            a[j] = rnd() & 1;
            s[j / 64] |= (uint64_t)a[j] << (j % 64);
        }
        for (uint64_t i = 0; i < m; ++i) rows[i] = m - 1 - i;
        oracle_toeplitz_bitwise(r, n, a, m, k);
        oracle_toeplitz_packed(x, n, s, m, y);
        oracle_toeplitz_packed_rows(x, n, s, L, rows, m, kr);
        for (uint64_t i = 0; i < m; ++i) {
            if (((y[i / 64] >> (i % 64)) & 1u) != k[i]) return fail("packed != bitwise", n, m);
            if (kr[m - 1 - i] != k[i]) return fail("rows != bitwise", n, m);
        }
        if (m % 64 && (y[m / 64] >> (m % 64))) return fail("output tail not zero", n, m);
        free(r); free(a); free(k); free(kr); free(x); free(s); free(y); free(rows);
    }
    uint64_t c[256] = {0};
    double out[8];
    for (int v = 0; v < 256; ++v) c[v] = 1000.0 * exp(-0.5 * (v - 128.0) * (v - 128.0) / 400.0);
    for (int u = 0; u < 3; ++u)
        for (int given = 0; given < 2; ++given) {
            if (oracle_minentropy_scalar(c, 8, given, 127.5, 20.0, u, out))
                return fail("estimator refused counts", 0, 0);
            for (int i = 0; i < 8; ++i)
                if (!isfinite(out[i])) return fail("estimator not finite", 0, 0);
            if (!(out[4] >= 0.0 && out[4] <= 1.0)) return fail("d_U outside [0, 1]", 0, 0);
        }
    uint64_t z[32] = {0};
    if (oracle_minentropy_scalar(z, 5, 0, 0, 0, 0, out) != -1)
        return fail("empty histogram accepted", 0, 0);
    printf("oracle selfcheck ok\n");
    return 0;
}
