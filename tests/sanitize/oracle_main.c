/* Drives every entry point of the oracle (oracle/ryser.c) on small inputs,
 * including the edge cases (n = 0 and 1, empty and full ranges, rejected
 * arguments), so that an AddressSanitizer + UndefinedBehaviorSanitizer build
 * sees each code path.  Prints "oracle sanitize ok" and exits 0 when every
 * call returned what its contract says. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_ryser_c128(const double *A, int n, int kahan, double *out);
int oracle_ryser_c128_ld(const double *A, int n, double *out);
int oracle_ryser_f64(const double *A, int n, int kahan, double *out);
int oracle_ryser_modp(const uint32_t *A, int n, uint32_t p, uint32_t *out);
int oracle_ryser_modp_prefix(const uint32_t *A, int n, uint32_t p, uint64_t x_end, uint32_t *out);
int oracle_ryser_modp_range(const uint32_t *A, int n, uint32_t p, uint64_t x0, uint64_t x1,
                            uint32_t *out);
int oracle_ryser_c128_range(const double *A, int n, uint64_t x0, uint64_t x1, double *out);
int oracle_ryser_f64_range(const double *A, int n, uint64_t x0, uint64_t x1, double *out);
int oracle_glynn_range_c128(const double *A, int n, uint64_t x0, uint64_t x1, double *out);
int oracle_glynn_range_f64(const double *A, int n, uint64_t x0, uint64_t x1, double *out);
int oracle_glynn_range_modp(const uint32_t *A, int n, uint32_t p, uint64_t x0, uint64_t x1,
                            uint32_t *out);
int oracle_ryser_c128_many(const double *A, int n, int count, int kahan, double *out);
int oracle_ryser_f64_many(const double *A, int n, int count, int kahan, double *out);

static int bad = 0;
#define EXPECT(c)                                                     \
    do {                                                              \
        if (!(c)) {                                                   \
            fprintf(stderr, "line %d: expected %s\n", __LINE__, #c); \
            ++bad;                                                    \
        }                                                             \
    } while (0)

int main(void)
{
    /* exactly sized heap buffers, so that an overrun is caught */
    for (int n = 0; n <= 9; ++n) {
        const size_t nn = (size_t)n * n;
        double *C = malloc(2 * nn * sizeof(double) + 1);
        double *R = malloc(nn * sizeof(double) + 1);
        uint32_t *M = malloc(nn * sizeof(uint32_t) + 1);
        uint64_t s = 88172645463325252ull + (uint64_t)n;
        for (size_t i = 0; i < nn; ++i) {
            s ^= s << 13; s ^= s >> 7; s ^= s << 17;
            C[2 * i] = (double)(s % 1000) / 500.0 - 1.0;
            C[2 * i + 1] = (double)((s >> 20) % 1000) / 500.0 - 1.0;
            R[i] = C[2 * i];
            M[i] = (uint32_t)(s % 2147483647u);
        }
        double *out2 = malloc(2 * sizeof(double));
        uint32_t *o32 = malloc(sizeof(uint32_t));
        EXPECT(oracle_ryser_c128(C, n, 1, out2) == 0);
        EXPECT(oracle_ryser_c128(C, n, 0, out2) == 0);
        EXPECT(oracle_ryser_c128_ld(C, n, out2) == 0);
        EXPECT(oracle_ryser_f64(R, n, 1, out2) == 0);
        EXPECT(oracle_ryser_modp(M, n, 2147483647u, o32) == 0);
        if (n == 0) EXPECT(o32[0] == 1);
        if (n >= 1) {
            const uint64_t T = (uint64_t)1 << (n - 1), S = (uint64_t)1 << n;
            uint32_t full = 0, a = 0, b = 0;
            EXPECT(oracle_ryser_modp_prefix(M, n, 2147483647u, S, o32) == 0);
            full = o32[0];
            EXPECT(oracle_ryser_modp_range(M, n, 2147483647u, 1, S / 2 + 1, &a) == 0);
            EXPECT(oracle_ryser_modp_range(M, n, 2147483647u, S / 2 + 1, S, &b) == 0);
            EXPECT(((uint64_t)a + b) % 2147483647u == full);
            EXPECT(oracle_ryser_modp_range(M, n, 2147483647u, 3 < S ? 3 : S, 3 < S ? 3 : S, o32) == 0);
            EXPECT(oracle_ryser_modp_range(M, n, 2147483647u, 0, 1, o32) == -1);      /* x0 >= 1 */
            EXPECT(oracle_ryser_modp_range(M, n, 2147483647u, 1, S + 1, o32) == -1);  /* past 2^n */
            EXPECT(oracle_ryser_c128_range(C, n, 1, S, out2) == 0);
            EXPECT(oracle_ryser_c128_range(C, n, S / 2 + 1, S, out2) == 0);
            EXPECT(oracle_ryser_f64_range(R, n, 1, S, out2) == 0);
            EXPECT(oracle_ryser_f64_range(R, n, 0, 1, out2) == -1);
            EXPECT(oracle_glynn_range_c128(C, n, 0, T, out2) == 0);
            EXPECT(oracle_glynn_range_c128(C, n, T, T, out2) == 0);
            EXPECT(oracle_glynn_range_f64(R, n, 0, T, out2) == 0);
            EXPECT(oracle_glynn_range_modp(M, n, 2147483647u, 0, T, o32) == 0);
            EXPECT(oracle_glynn_range_modp(M, n, 2147483647u, 0, T + 1, o32) == -1);
        }
        free(C); free(R); free(M); free(out2); free(o32);
    }
    /* batches */
    {
        const int n = 6, count = 5;
        double *C = calloc((size_t)2 * n * n * count, sizeof(double));
        double *R = calloc((size_t)n * n * count, sizeof(double));
        double *out = malloc((size_t)2 * count * sizeof(double));
        for (int i = 0; i < n * n * count; ++i) { C[2 * i] = (i % 7) * 0.1; R[i] = (i % 5) * 0.2; }
        EXPECT(oracle_ryser_c128_many(C, n, count, 1, out) == 0);
        EXPECT(oracle_ryser_f64_many(R, n, count, 1, out) == 0);
        EXPECT(oracle_ryser_f64_many(R, n, -1, 1, out) == -1);
        free(C); free(R); free(out);
    }
    /* rejected arguments */
    {
        double d[2];
        uint32_t u = 0, A1 = 5;
        EXPECT(oracle_ryser_c128(NULL, 3, 1, d) == -1);
        EXPECT(oracle_ryser_c128(d, 49, 1, d) == -1);
        EXPECT(oracle_ryser_modp(&A1, 1, 3, &u) == -1);      /* entry >= p */
        EXPECT(oracle_glynn_range_f64(d, 1, 1, 0, d) == -1);  /* x0 > x1 */
    }
    if (bad) return 1;
    printf("oracle sanitize ok\n");
    return 0;
}
