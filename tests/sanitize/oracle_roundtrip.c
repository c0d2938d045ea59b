/* Round trips of the oracle's reference codec for a sanitizer build (CPU
 * only): seeded random CSR matrices are encoded to a container file by the
 * oracle's encoder and decoded by its decoder, which must return the original
 * row pointers, columns and value bits.  Exit status 0 when all agree. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_encode(const char *path, int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr,
                  const int32_t *col, const void *vals, int dtype, int layout, int lane_nnz,
                  uint64_t seed, int first_mode, int esc_mode, int sigma);
int oracle_decode(const char *path, int32_t *row_ptr_out, int32_t *col_out, void *vals_out);

static uint64_t state = 99;
static uint64_t rnd(void) /* xorshift64 (Marsaglia) */
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return state;
}

static int one(const char *path, int64_t m, int64_t n, int maxlen, int pool, int dtype, int layout,
               int T, int first, int esc)
{
    int32_t *rp = malloc((m + 1) * sizeof(int32_t));
    int64_t cap = m * (int64_t)maxlen + 1;
    int32_t *ci = malloc(cap * sizeof(int32_t));
    double *v = malloc(cap * sizeof(double));
    float *f = malloc(cap * sizeof(float));
    double *pv = malloc(pool * sizeof(double));
    for (int i = 0; i < pool; ++i) pv[i] = (double)((int64_t)(rnd() % 2001) - 1000) / 32.0;
    int64_t nnz = 0;
    rp[0] = 0;
    for (int64_t i = 0; i < m; ++i) {
        int len = (int)(rnd() % (uint64_t)(maxlen + 1));
        int64_t c = (int64_t)(rnd() % (uint64_t)n);
        for (int k = 0; k < len && c < n; ++k) {
            ci[nnz] = (int32_t)c;
            v[nnz] = pv[rnd() % (uint64_t)pool];
            f[nnz] = (float)v[nnz];
            ++nnz;
            c += (int64_t)(rnd() % 4);
        }
        rp[i + 1] = (int32_t)nnz;
    }
    const void *vals = dtype == 2 ? (const void *)v : (const void *)f;
    int bad = oracle_encode(path, m, n, nnz, rp, ci, vals, dtype, layout, T, rnd(), first, esc, layout == 1 ? 64 * (esc + first) : 0);
    int32_t *rp2 = malloc((m + 1) * sizeof(int32_t));
    int32_t *ci2 = malloc((nnz + 1) * sizeof(int32_t));
    double *v2 = malloc((nnz + 1) * sizeof(double));
    if (!bad) bad = oracle_decode(path, rp2, ci2, v2);
    if (!bad) {
        bad = memcmp(rp, rp2, (m + 1) * sizeof(int32_t)) != 0 || memcmp(ci, ci2, nnz * sizeof(int32_t)) != 0 ||
              memcmp(vals, v2, nnz * (dtype == 2 ? 8 : 4)) != 0;
    }
    if (bad)
        printf("failure: m=%lld dtype=%d layout=%d T=%d first=%d esc=%d\n", (long long)m, dtype, layout, T, first, esc);
    free(rp); free(ci); free(v); free(f); free(pv); free(rp2); free(ci2); free(v2);
    return bad != 0;
}

int main(int argc, char **argv)
{
    const char *path = argc > 1 ? argv[1] : "oracle_roundtrip.dtans";
    int fails = 0, cases = 0;
    for (int dtype = 1; dtype <= 2; ++dtype)
        for (int layout = 1; layout <= 2; ++layout)
            for (int first = 0; first <= 1; ++first)
                for (int esc = 0; esc <= 1; ++esc) {
                    fails += one(path, 150, 300, 18, 30, dtype, layout, layout == 2 ? 12 : 0, first, esc);
                    fails += one(path, 97, 5000, 40, 700, dtype, layout, layout == 2 ? 32 : 0, first, esc);
                    fails += one(path, 3, 7, 2, 1, dtype, layout, layout == 2 ? 4 : 0, first, esc);
                    cases += 3;
                }
    printf("%d cases, %d failures\n", cases, fails);
    return fails != 0;
}
