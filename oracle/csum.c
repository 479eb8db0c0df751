/* Direct O(|rows| N L) sums of the extended Gaussian ANOVA kernel (paper Sec. 2.6,
 * discrete ANOVA kernel), FP64, OpenMP over rows.  Test infrastructure for the oracle:
 * sampled rows of W v at sizes where the dense matrix does not fit.
 *
 *   out[r] = sum_l w_l sum_j exp(-sum_{d in W_l} (F[d][i] - F[d][j])^2 / sigma_l^2) v[j],
 *   i = rows[r].
 *
 * F is the SoA feature matrix [d][N]; windows are given by win_dim[L] and win_feat[sum dims].
 */
#include <math.h>
#include <stdint.h>

int oracle_anova_rows(const double *F, int64_t N, int32_t d,
                      int32_t L, const int32_t *win_dim, const int32_t *win_feat,
                      const double *sigma, const double *weight,
                      const double *v, const int64_t *rows, int64_t nrows, double *out)
{
    if (N <= 0 || L <= 0) return 1;
    int32_t off[256];
    if (L > 256) return 1;
    int32_t acc = 0;
    for (int32_t l = 0; l < L; ++l) {
        off[l] = acc;
        acc += win_dim[l];
        for (int32_t k = 0; k < win_dim[l]; ++k)
            if (win_feat[off[l] + k] < 0 || win_feat[off[l] + k] >= d) return 1;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t i = rows[r];
        double total = 0.0;
        for (int32_t l = 0; l < L; ++l) {
            const double inv = 1.0 / (sigma[l] * sigma[l]);
            const int32_t t = win_dim[l];
            const double *X0 = F + (int64_t)win_feat[off[l]] * N;
            const double *X1 = t > 1 ? F + (int64_t)win_feat[off[l] + 1] * N : X0;
            const double *X2 = t > 2 ? F + (int64_t)win_feat[off[l] + 2] * N : X0;
            const double x0 = X0[i], x1 = X1[i], x2 = X2[i];
            double s = 0.0;
            for (int64_t j = 0; j < N; ++j) {
                double q = (X0[j] - x0) * (X0[j] - x0);
                if (t > 1) q += (X1[j] - x1) * (X1[j] - x1);
                if (t > 2) q += (X2[j] - x2) * (X2[j] - x2);
                s += exp(-q * inv) * v[j];
            }
            total += weight[l] * s;
        }
        out[r] = total;
    }
    return 0;
}
