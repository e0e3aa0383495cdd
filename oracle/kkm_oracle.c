/*
 * Kernel K-means oracle: a plain, slow FP64 CPU implementation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library.  It shares no code,
 * header, table or helper with the HIP library and must never be called from
 * the product path.
 *
 * What it computes (paper: "Popcorn: Accelerating Kernel K-means on GPUs
 * through Sparse Linear Algebra", PPoPP'25):
 *
 *  - Kernel functions, Sec. 3.2: polynomial (gamma x.y + c)^r and Gaussian
 *    exp(-gamma ||x-y||^2 / sigma^2) with sigma = 1; "linear" is the plain inner
 *    product.  K_ij = kappa(p_i, p_j) (Sec. 2.2, kernel matrix).  The Gaussian
 *    is evaluated from the direct difference x - y, not from the norm
 *    expansion of Eq. (gauss), so the two routes check each other.
 *
 *  - Distance of point i to the centroid of cluster c in feature space,
 *    Sec. 3.1: ||phi(p_i) - c_c||^2 with c_c the mean of the cluster's feature
 *    vectors (Eq. centroids).  Expanding the square with K = P P^T gives the
 *    definition used here, term by term:
 *        d_ic = K_ii - (2/|c|) sum_{j in c} K_ij
 *                    + (1/|c|^2) sum_{j in c} sum_{l in c} K_jl .
 *    No SpMM/SpMV reformulation is used; that is what the GPU path does.
 *
 *  - The loop of Algorithms 1 and 2: every point moves to the cluster of its
 *    nearest centroid, all points against the centroids of the previous labels
 *    (batch reassignment), until no label changes or maxiter steps ran.
 *
 * Readings of points the paper leaves open (listed in the design notes):
 *  - an empty cluster has no centroid; its distance is +inf (policy 0), or,
 *    reading Algorithm 2 literally (a V row of zeros), the centroid is the
 *    origin of feature space and d_ic = K_ii (policy 1);
 *  - argmin ties go to the lowest cluster index;
 *  - J(a) = sum_i d_{i,a(i)} with the centroids of the same labels a.
 *
 * Everything is FP64; the input points are the same FP32 values the GPU gets,
 * widened exactly to double.  Built with -ffp-contract=off so every product
 * and sum is rounded as written.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_LINEAR = 0, OR_POLY = 1, OR_GAUSS = 2 };

/* Threads the OpenMP loops use (reported with the CPU timings). */
int oracle_threads(void) { return omp_get_max_threads(); }
/* Sets the threads of the following OpenMP loops (for timing at one thread). */
void oracle_set_threads(int t) { omp_set_num_threads(t > 0 ? t : 1); }
enum { OR_EMPTY_INF = 0, OR_EMPTY_ZERO_CENTROID = 1 };

/* kappa(x, y) from the definitions of Sec. 3.2 (and the inner product). */
double oracle_kappa(const float *x, const float *y, int64_t d, int type,
                    double gamma, double coef0, int degree)
{
    if (type == OR_GAUSS) {
        double sq = 0.0;
        for (int64_t l = 0; l < d; ++l) {
            double diff = (double)x[l] - (double)y[l];
            sq += diff * diff;
        }
        return exp(-gamma * sq);
    }
    double dot = 0.0;
    for (int64_t l = 0; l < d; ++l)
        dot += (double)x[l] * (double)y[l];
    if (type == OR_LINEAR)
        return dot;
    /* polynomial: (gamma * x.y + c)^r, r a positive integer */
    double base = gamma * dot + coef0;
    double v = 1.0;
    for (int r = 0; r < degree; ++r)
        v *= base;
    return v;
}

/* Full n x n kernel matrix, row-major.  kappa is symmetric in its arguments,
 * so the upper triangle is evaluated and mirrored. */
void oracle_kernel_matrix(const float *X, int64_t n, int64_t d, int64_t ldx, int type,
                          double gamma, double coef0, int degree, double *K)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i; j < n; ++j) {
            double v = oracle_kappa(X + i * ldx, X + j * ldx, d, type, gamma, coef0, degree);
            K[i * n + j] = v;
            K[j * n + i] = v;
        }
}

/* Kernel rows for selected points only: out[r * n + j] = kappa(x_rows[r], x_j). */
void oracle_kernel_rows(const float *X, int64_t n, int64_t d, int64_t ldx, int type,
                        double gamma, double coef0, int degree,
                        const int64_t *rows, int64_t nrows, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r)
        for (int64_t j = 0; j < n; ++j)
            out[r * n + j] = oracle_kappa(X + rows[r] * ldx, X + j * ldx, d, type,
                                          gamma, coef0, degree);
}

/* Cluster sizes |c|; returns -1 if a label lies outside [0, k). */
static int cluster_sizes(const int32_t *labels, int64_t n, int32_t k, int64_t *size)
{
    for (int32_t c = 0; c < k; ++c)
        size[c] = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (labels[i] < 0 || labels[i] >= k)
            return -1;
        size[labels[i]] += 1;
    }
    return 0;
}

/*
 * Squared norm of every centroid in feature space from its definition:
 *   ||c_c||^2 = (1/|c|^2) sum_{j in c} sum_{l in c} K_jl   (|c| > 0).
 * This is the quantity Sec. 3.3 obtains as diag(V K V^T) (Eq. c_norm).
 */
static void centroid_sqnorms(const double *K, int64_t n, const int32_t *labels, int32_t k,
                             const int64_t *size, double *cnorm)
{
    /* members of each cluster, in index order */
    int64_t *start = (int64_t *)calloc((size_t)k + 1, sizeof(int64_t));
    int64_t *fill = (int64_t *)calloc((size_t)k, sizeof(int64_t));
    int64_t *members = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    for (int32_t c = 0; c < k; ++c)
        start[c + 1] = start[c] + size[c];
    for (int64_t i = 0; i < n; ++i) {
        int32_t c = labels[i];
        members[start[c] + fill[c]++] = i;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t c = 0; c < k; ++c) {
        if (size[c] == 0) {
            cnorm[c] = 0.0;
            continue;
        }
        double s = 0.0;
        for (int64_t a = start[c]; a < start[c + 1]; ++a)
            for (int64_t b = start[c]; b < start[c + 1]; ++b)
                s += K[members[a] * n + members[b]];
        cnorm[c] = s / ((double)size[c] * (double)size[c]);
    }
    free(start);
    free(fill);
    free(members);
}

/*
 * One reassignment step of Algorithms 1/2 from the definition.
 *
 * In:  K (n x n), labels_in (n, values in [0,k)), empty_policy.
 * Out: labels_out[i] = argmin_c d_ic (lowest c on ties)
 *      D (n x k, row-major, nullable): d_ic, +inf for an empty cluster under policy 0
 *      gap (n, nullable): second-smallest minus smallest d_ic over finite entries
 *                         (+inf when fewer than two are finite)
 *      counts_out (k, nullable): sizes of the clusters of labels_out
 *      J_in:      sum_i d_{i, labels_in(i)}  (objective of the input labelling)
 *      A_out:     sum_i min_c d_ic
 *      n_changed: #{i : labels_out[i] != labels_in[i]}
 * Returns 0, or -1 if a label lies outside [0, k).
 */
int oracle_step(const double *K, int64_t n, int32_t k, const int32_t *labels_in,
                int empty_policy, int32_t *labels_out, double *D, double *gap,
                int32_t *counts_out, double *J_in, double *A_out, int64_t *n_changed)
{
    int64_t *size = (int64_t *)malloc((size_t)k * sizeof(int64_t));
    double *cnorm = (double *)malloc((size_t)k * sizeof(double));
    if (cluster_sizes(labels_in, n, k, size) != 0) {
        free(size);
        free(cnorm);
        return -1;
    }
    centroid_sqnorms(K, n, labels_in, k, size, cnorm);

    double J = 0.0, A = 0.0;
    int64_t changed = 0;
#pragma omp parallel for schedule(static) reduction(+ : J, A, changed)
    for (int64_t i = 0; i < n; ++i) {
        /* sum of K_ij over the members j of each cluster */
        double *rowsum = (double *)calloc((size_t)k, sizeof(double));
        for (int64_t j = 0; j < n; ++j)
            rowsum[labels_in[j]] += K[i * n + j];
        double best = INFINITY, second = INFINITY, own = 0.0;
        int32_t arg = -1;
        for (int32_t c = 0; c < k; ++c) {
            double dic;
            if (size[c] > 0)
                dic = K[i * n + i] - 2.0 * rowsum[c] / (double)size[c] + cnorm[c];
            else
                dic = (empty_policy == OR_EMPTY_ZERO_CENTROID) ? K[i * n + i] : INFINITY;
            if (D)
                D[i * k + c] = dic;
            if (c == labels_in[i])
                own = dic;
            if (dic < best) {
                second = best;
                best = dic;
                arg = c;
            } else if (dic < second) {
                second = dic;
            }
        }
        if (arg < 0) /* every distance infinite: cannot happen, the own cluster is non-empty */
            arg = labels_in[i];
        labels_out[i] = arg;
        if (gap)
            gap[i] = second - best;
        J += own;
        A += best;
        changed += (arg != labels_in[i]);
        free(rowsum);
    }
    if (counts_out) {
        for (int32_t c = 0; c < k; ++c)
            counts_out[c] = 0;
        for (int64_t i = 0; i < n; ++i)
            counts_out[labels_out[i]] += 1;
    }
    *J_in = J;
    *A_out = A;
    *n_changed = changed;
    free(size);
    free(cnorm);
    return 0;
}

/* J(a) = sum_i d_{i,a(i)} for a labelling a (no reassignment). */
int oracle_objective(const double *K, int64_t n, int32_t k, const int32_t *labels,
                     int empty_policy, double *J)
{
    int32_t *scratch = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    double A;
    int64_t ch;
    int rc = oracle_step(K, n, k, labels, empty_policy, scratch, NULL, NULL, NULL, J, &A, &ch);
    free(scratch);
    return rc;
}

/*
 * The whole loop (Algorithm 2 from "Initialize iteration counter" on).
 *
 * Runs steps until no label changes (check_convergence != 0) or max_iter
 * steps ran.  iters counts executed steps, including a final step that
 * changed nothing.  labels_out holds the last labelling, objective its J.
 * Traces (nullable, length max_iter + 1): J_trace[t] = J of the labels entering
 * step t (t = 0..iters-1) and J_trace[iters] = J(labels_out); changed_trace[t]
 * = labels changed by step t.
 */
int oracle_fit(const double *K, int64_t n, int32_t k, const int32_t *labels0,
               int32_t max_iter, int check_convergence, int empty_policy,
               int32_t *labels_out, double *objective, int32_t *iters,
               double *J_trace, int64_t *changed_trace)
{
    int32_t *cur = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *nxt = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    memcpy(cur, labels0, (size_t)n * sizeof(int32_t));
    int32_t t = 0;
    double J = 0.0, A;
    int64_t changed = -1;
    int rc = 0;
    for (; t < max_iter; ++t) {
        rc = oracle_step(K, n, k, cur, empty_policy, nxt, NULL, NULL, NULL, &J, &A, &changed);
        if (rc != 0)
            break;
        if (J_trace)
            J_trace[t] = J;
        if (changed_trace)
            changed_trace[t] = changed;
        int32_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
        if (check_convergence && changed == 0) {
            ++t;
            break;
        }
    }
    if (rc == 0) {
        /* J of the final labelling: after a no-change step it is that step's J */
        if (!(t > 0 && changed == 0))
            rc = oracle_objective(K, n, k, cur, empty_policy, &J);
        if (J_trace)
            J_trace[t] = J;
        memcpy(labels_out, cur, (size_t)n * sizeof(int32_t));
        *objective = J;
        *iters = t;
    }
    free(cur);
    free(nxt);
    return rc;
}

/*
 * Large-n checks without an n x n matrix: for selected points i, the sum of
 * kappa(x_i, x_j) over the members j of every cluster c (out[r * k + c]),
 * evaluated from the definition.  (1/|c|) times this is the E_ic term of the
 * distance.
 */
int oracle_cluster_row_sums(const float *X, int64_t n, int64_t d, int64_t ldx, int type,
                            double gamma, double coef0, int degree,
                            const int32_t *labels, int32_t k,
                            const int64_t *rows, int64_t nrows, double *out)
{
    for (int64_t i = 0; i < n; ++i)
        if (labels[i] < 0 || labels[i] >= k)
            return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        double *o = out + r * k;
        for (int32_t c = 0; c < k; ++c)
            o[c] = 0.0;
        for (int64_t j = 0; j < n; ++j)
            o[labels[j]] += oracle_kappa(X + rows[r] * ldx, X + j * ldx, d, type,
                                         gamma, coef0, degree);
    }
    return 0;
}
