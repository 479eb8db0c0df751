/* The oracle's direct sums (oracle/csum.c) under AddressSanitizer and UndefinedBehaviorSanitizer:
 * a small problem against a plain triple loop written here, and the invalid arguments the
 * function must refuse.  Exit status 0 on success. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_anova_rows(const double *F, int64_t N, int32_t d, int32_t L, const int32_t *win_dim,
                      const int32_t *win_feat, const double *sigma, const double *weight,
                      const double *v, const int64_t *rows, int64_t nrows, double *out);

int main(void) {
    enum { N = 57, D = 4, L = 3 };
    double *F = malloc(sizeof(double) * D * N), v[N], out[5], sig[L] = {0.3, 0.5, 0.2},
           wt[L] = {1.0, 0.5, 2.0};
    int32_t wd[L] = {3, 2, 1}, wf[6] = {0, 1, 2, 1, 3, 2};
    int64_t rows[5] = {0, 7, 19, 33, N - 1};
    unsigned s = 12345u;
    for (int k = 0; k < D * N; ++k) { s = s * 1103515245u + 12345u; F[k] = (s >> 8) / 16777216.0; }
    for (int j = 0; j < N; ++j) { s = s * 1103515245u + 12345u; v[j] = (s >> 8) / 16777216.0 - 0.5; }
    int failures = 0;
    if (oracle_anova_rows(F, N, D, L, wd, wf, sig, wt, v, rows, 5, out) != 0) ++failures;
    for (int r = 0; r < 5; ++r) {
        const int64_t i = rows[r];
        double want = 0.0;
        int off = 0;
        for (int l = 0; l < L; ++l) {
            for (int64_t j = 0; j < N; ++j) {
                double q = 0.0;
                for (int k = 0; k < wd[l]; ++k) {
                    const double t = F[wf[off + k] * N + i] - F[wf[off + k] * N + j];
                    q += t * t;
                }
                want += wt[l] * exp(-q / (sig[l] * sig[l])) * v[j];
            }
            off += wd[l];
        }
        if (fabs(out[r] - want) > 1e-12 * (1.0 + fabs(want))) {
            fprintf(stderr, "row %lld: %.17g vs %.17g\n", (long long)i, out[r], want);
            ++failures;
        }
    }
    int32_t badf[6] = {0, 1, 4, 1, 3, 2};          /* feature 4 is out of range */
    if (oracle_anova_rows(F, N, D, L, wd, badf, sig, wt, v, rows, 5, out) != 1) ++failures;
    if (oracle_anova_rows(F, 0, D, L, wd, wf, sig, wt, v, rows, 5, out) != 1) ++failures;
    if (oracle_anova_rows(F, N, D, 0, wd, wf, sig, wt, v, rows, 5, out) != 1) ++failures;
    free(F);
    printf("%d failures\n", failures);
    return failures == 0 ? 0 : 1;
}
