/*
 * CPU oracle of the applications built on the k-means building blocks, FP64.
 * TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's
 * CPU-baseline leg load it; the product path never does.  It shares no code
 * with the GPU library (nor with kmeans_oracle.c).
 *
 * What it computes, plainly and slowly:
 *
 *   orc_spade_densities  the density step of SPADE's downsampling (section
 *     4.1, "Downsampling in Bioinformatics"): rows of the all-pairs distance
 *     matrix are visited in increasing index order; a row whose density is
 *     already set (by an earlier row that found it within the approximation
 *     width) is skipped, which is the point of the section's fused code: its
 *     distances are never computed.  A visited row i counts the samples j
 *     with dist(i, j) below the kernel width or the approximation width
 *     (that count includes i itself), and gives that count to every sample
 *     within the approximation width whose density is still unset, and to
 *     itself.  The distance is the L1 (sum of absolute differences) one of
 *     the section's generated code, evaluated in FP64 with features in
 *     increasing order; the squared Euclidean one is available as metric 1.
 *   orc_assign_metric  nearest centroid (lowest index on ties) under L1
 *     (metric 0) or squared Euclidean (metric 1) distance, FP64.
 *   orc_class_sums     the predicated per-class reduce (section 2.3) of given
 *     labels: per-class FP64 feature sums in increasing sample order, counts.
 *   orc_nb_train       multinomial naive Bayes training (named among the
 *     section 4.2 applications), with add-one (Laplace) smoothing:
 *     prior_c = n_c / n, phi_cf = (S_cf + 1) / (sum_f S_cf + d).
 *   orc_gda_train      Gaussian discriminant analysis training (named among
 *     the section 4.2 applications): class priors n_c / n, class means
 *     mu_c = S_c / n_c, and the shared covariance
 *     Sigma = (1/n) sum_i (x_i - mu_{y_i}) (x_i - mu_{y_i})^T, summed in
 *     increasing i.
 *
 * Readings fixed here (the paper states none of them): see each function.
 * Inputs are FP32 samples widened exactly to FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* distance between two FP32 rows: metric 0 = sum |a - b|, 1 = sum (a - b)^2 */
static double row_dist(const float *a, const float *b, int d, int metric)
{
    double s = 0.0;
    for (int f = 0; f < d; ++f) {
        double diff = (double)a[f] - (double)b[f];
        s += metric == 0 ? fabs(diff) : diff * diff;
    }
    return s;
}

/* distance between an FP32 sample and an FP64 centroid */
static double cen_dist(const float *x, const double *c, int d, int metric)
{
    double s = 0.0;
    for (int f = 0; f < d; ++f) {
        double diff = (double)x[f] - c[f];
        s += metric == 0 ? fabs(diff) : diff * diff;
    }
    return s;
}

/*
 * SPADE densities.  dens[n] (int32) receives every sample's density;
 * processed[n] (may be NULL) receives 1 for the rows whose distances were
 * computed, 0 for the skipped ones.  Reading: rows in increasing index order
 * (the sequential meaning of the section's loop, whose parallel versions
 * race); a density once set is never overwritten (the hand-written version
 * sets a neighbour's density only while it is still zero); a visited row's
 * own density is its count.  Returns the number of visited rows.
 */
int64_t orc_spade_densities(const float *X, int64_t n, int d, double apprx_width, double kernel_width,
                            int metric, int32_t *dens, int8_t *processed)
{
    int64_t visited = 0;
    int32_t *near = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!near) return -1;
    for (int64_t i = 0; i < n; ++i) dens[i] = 0;
    if (processed && n > 0) memset(processed, 0, (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        if (dens[i] > 0) continue;
        const float *xi = X + (size_t)i * (size_t)d;
        int64_t nnear = 0;
        int32_t c = 0;
        /* the fused row: distance, find (approximation width), count (kernel width) */
        for (int64_t j = 0; j < n; ++j) {
            double dij = row_dist(xi, X + (size_t)j * (size_t)d, d, metric);
            if (dij < apprx_width) {
                near[nnear++] = (int32_t)j;
                c++;
            } else if (dij < kernel_width) {
                c++;
            }
        }
        for (int64_t t = 0; t < nnear; ++t)
            if (dens[near[t]] == 0) dens[near[t]] = c;
        dens[i] = c;
        if (processed) processed[i] = 1;
        ++visited;
    }
    free(near);
    return visited;
}

/*
 * Nearest centroid under the given metric: labels[i] = smallest j attaining
 * min_j dist(x_i, c_j); dmin[i] = that minimum, d2nd[i] = the smallest
 * distance over j != labels[i] (+inf for k = 1).  dmin / d2nd may be NULL.
 */
void orc_assign_metric(const float *X, const double *C, int64_t n, int d, int k, int metric,
                       int32_t *labels, double *dmin, double *d2nd)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const float *x = X + (size_t)i * (size_t)d;
        double b1 = 0.0, b2 = 1.0 / 0.0;
        int32_t j1 = -1;
        for (int j = 0; j < k; ++j) {
            double dij = cen_dist(x, C + (size_t)j * (size_t)d, d, metric);
            if (j1 < 0 || dij < b1) {
                if (j1 >= 0) b2 = b1;
                b1 = dij;
                j1 = j;
            } else if (dij < b2) {
                b2 = dij;
            }
        }
        labels[i] = j1;
        if (dmin) dmin[i] = b1;
        if (d2nd) d2nd[i] = b2;
    }
}

/*
 * Per-class sums S[c][f] = sum over {i : y_i = c} of x_if (FP64, increasing
 * i) and counts cnt[c].  Returns 0, or -1 if a label lies outside [0, C).
 */
int orc_class_sums(const float *X, const int32_t *y, int64_t n, int d, int C, double *S, int64_t *cnt)
{
    memset(S, 0, sizeof(double) * (size_t)C * (size_t)d);
    for (int c = 0; c < C; ++c) cnt[c] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t c = y[i];
        if (c < 0 || c >= C) return -1;
        const float *x = X + (size_t)i * (size_t)d;
        double *s = S + (size_t)c * (size_t)d;
        for (int f = 0; f < d; ++f) s[f] += (double)x[f];
        cnt[c] += 1;
    }
    return 0;
}

/*
 * Multinomial naive Bayes with add-one smoothing.  X holds per-sample feature
 * counts (non-negative; FP32).  Outputs prior[C] = n_c / n and
 * phi[C][d] = (S_cf + 1) / (T_c + d) with T_c = sum_f S_cf (summed in
 * increasing f).  A class without samples gets prior 0 and phi = 1/d.
 * Returns 0, or -1 for a label outside [0, C).
 */
int orc_nb_train(const float *X, const int32_t *y, int64_t n, int d, int C, double *prior, double *phi)
{
    double *S = (double *)malloc(sizeof(double) * (size_t)C * (size_t)d);
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)C);
    if (!S || !cnt) { free(S); free(cnt); return -2; }
    int rc = orc_class_sums(X, y, n, d, C, S, cnt);
    if (rc) { free(S); free(cnt); return rc; }
    for (int c = 0; c < C; ++c) {
        double T = 0.0;
        for (int f = 0; f < d; ++f) T += S[(size_t)c * d + f];
        prior[c] = (double)cnt[c] / (double)n;
        for (int f = 0; f < d; ++f)
            phi[(size_t)c * d + f] = (S[(size_t)c * d + f] + 1.0) / (T + (double)d);
    }
    free(S);
    free(cnt);
    return 0;
}

/*
 * Gaussian discriminant analysis with one covariance shared by the classes.
 * Outputs prior[C] = n_c / n, mu[C][d] = S_c / n_c (0 for an empty class)
 * and sigma[d][d] = (1/n) sum_i z_i z_i^T with z_i = x_i - mu_{y_i}, every
 * product and sum in FP64, samples in increasing order.  Returns 0, or -1
 * for a label outside [0, C).
 */
int orc_gda_train(const float *X, const int32_t *y, int64_t n, int d, int C, double *prior, double *mu,
                  double *sigma)
{
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)C);
    double *z = (double *)malloc(sizeof(double) * (size_t)d);
    if (!cnt || !z) { free(cnt); free(z); return -2; }
    int rc = orc_class_sums(X, y, n, d, C, mu, cnt);
    if (rc) { free(cnt); free(z); return rc; }
    for (int c = 0; c < C; ++c) {
        prior[c] = (double)cnt[c] / (double)n;
        for (int f = 0; f < d; ++f) {
            size_t o = (size_t)c * d + f;
            mu[o] = cnt[c] > 0 ? mu[o] / (double)cnt[c] : 0.0;
        }
    }
    memset(sigma, 0, sizeof(double) * (size_t)d * (size_t)d);
    for (int64_t i = 0; i < n; ++i) {
        const float *x = X + (size_t)i * (size_t)d;
        const double *m = mu + (size_t)y[i] * (size_t)d;
        for (int f = 0; f < d; ++f) z[f] = (double)x[f] - m[f];
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) sigma[(size_t)a * d + b] += z[a] * z[b];
    }
    for (size_t o = 0; o < (size_t)d * (size_t)d; ++o) sigma[o] /= (double)n;
    free(cnt);
    free(z);
    return 0;
}
