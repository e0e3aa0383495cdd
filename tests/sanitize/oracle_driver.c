/* Drives every entry point of the FP64 oracle on small seeded inputs, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (host code only).
 * Exits 0 when every call returns as documented; the sanitizers abort the
 * process on a memory or undefined-behaviour error. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

double oracle_kappa(const float *x, const float *y, int64_t d, int type, double gamma,
                    double coef0, int degree);
void oracle_kernel_matrix(const float *X, int64_t n, int64_t d, int64_t ldx, int type,
                          double gamma, double coef0, int degree, double *K);
void oracle_kernel_rows(const float *X, int64_t n, int64_t d, int64_t ldx, int type,
                        double gamma, double coef0, int degree, const int64_t *rows,
                        int64_t nrows, double *out);
int oracle_step(const double *K, int64_t n, int32_t k, const int32_t *labels_in, int empty_policy,
                int32_t *labels_out, double *D, double *gap, int32_t *counts_out, double *J_in,
                double *A_out, int64_t *n_changed);
int oracle_objective(const double *K, int64_t n, int32_t k, const int32_t *labels,
                     int empty_policy, double *J);
int oracle_fit(const double *K, int64_t n, int32_t k, const int32_t *labels0, int32_t max_iter,
               int check_convergence, int empty_policy, int32_t *labels_out, double *objective,
               int32_t *iters, double *J_trace, int64_t *changed_trace);
int oracle_cluster_row_sums(const float *X, int64_t n, int64_t d, int64_t ldx, int type,
                            double gamma, double coef0, int degree, const int32_t *labels,
                            int32_t k, const int64_t *rows, int64_t nrows, double *out);

static uint64_t state = 88172645463325252ull;
static double uniform(void) {  /* xorshift64, test input only */
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) / 9007199254740992.0;
}

static int run(int64_t n, int64_t d, int32_t k, int type, int empty_policy) {
    float *X = malloc(sizeof(float) * (size_t)(n * d));
    double *K = malloc(sizeof(double) * (size_t)(n * n));
    double *D = malloc(sizeof(double) * (size_t)(n * k));
    double *gap = malloc(sizeof(double) * (size_t)n);
    int32_t *l0 = malloc(sizeof(int32_t) * (size_t)n), *l1 = malloc(sizeof(int32_t) * (size_t)n);
    int32_t *cnt = malloc(sizeof(int32_t) * (size_t)k);
    double Jt[21], rs[3 * 8], kr[3 * 64];
    int64_t ct[20], rows[3] = {0, n / 2, n - 1}, nch = 0;
    for (int64_t t = 0; t < n * d; ++t) X[t] = (float)(2.0 * uniform() - 1.0);
    for (int64_t i = 0; i < n; ++i) l0[i] = (int32_t)(uniform() * k) % k;
    if (k > 2) l0[0] = l0[1] = 0;  /* leaves room for an empty cluster */
    double gamma = 1.0 / (double)d, J = 0, A = 0, obj = 0;
    int32_t iters = 0;
    int bad = 0;
    (void)oracle_kappa(X, X + (n > 1 ? d : 0), d, type, gamma, 1.0, 2);
    oracle_kernel_matrix(X, n, d, d, type, gamma, 1.0, 2, K);
    if (n <= 64) oracle_kernel_rows(X, n, d, d, type, gamma, 1.0, 2, rows, 3, kr);
    bad |= oracle_step(K, n, k, l0, empty_policy, l1, D, gap, cnt, &J, &A, &nch) != 0;
    bad |= oracle_objective(K, n, k, l1, empty_policy, &obj) != 0;
    bad |= oracle_fit(K, n, k, l0, 20, 1, empty_policy, l1, &obj, &iters, Jt, ct) != 0;
    if (k <= 8) bad |= oracle_cluster_row_sums(X, n, d, d, type, gamma, 1.0, 2, l0, k, rows, 3, rs) != 0;
    l0[n - 1] = k;  /* out of range: refused */
    bad |= oracle_step(K, n, k, l0, empty_policy, l1, D, gap, cnt, &J, &A, &nch) != -1;
    bad |= !isfinite(obj);
    free(X); free(K); free(D); free(gap); free(l0); free(l1); free(cnt);
    return bad;
}

int main(void) {
    int bad = 0;
    for (int type = 0; type < 3; ++type)
        for (int pol = 0; pol < 2; ++pol) {
            bad |= run(1, 1, 1, type, pol);
            bad |= run(7, 3, 3, type, pol);
            bad |= run(61, 5, 8, type, pol);
        }
    printf(bad ? "oracle driver: FAILED\n" : "oracle driver: ok\n");
    return bad;
}
