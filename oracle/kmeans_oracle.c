/*
 * k-means (Lloyd) CPU oracle, FP64.  TEST INFRASTRUCTURE ONLY: tests, the
 * smoke check and the benchmark's CPU-baseline leg load it; the product path
 * never does.  It shares no code with the GPU library.
 *
 * What it computes, plainly and slowly:
 *
 *   The clustering step of Lloyd's method (S. P. Lloyd, "Least squares
 *   quantization in PCM", IEEE Trans. Inf. Theory 28(2), 1982), decomposed the
 *   way the paper decomposes data-parallel work (section 2.3, the DeliteOpLoop
 *   contract): a per-sample map (a collect body: the squared Euclidean distance
 *   to every centroid and the index of the nearest one) followed by a
 *   predicated reduce per label (a reduce body over the same index range: the
 *   sum and count of the samples that carry that label), and the mean as sum
 *   divided by length (section 2.1, the avg operation of the vector DSL).
 *   The distance is the fused single-pass norm/dist of section 3.4 without the
 *   square root (the square root is monotone, so the argmin is unchanged).
 *
 * Readings fixed here (the paper is silent on all of them):
 *   - distance: d_ij = sum_f (x_if - c_jf)^2, evaluated directly in FP64,
 *     features in increasing order;
 *   - ties: the lowest centroid index wins (strict < scan in index order);
 *   - objective: J_t = sum_i d_{i,L_t(i)}, against the centroids used for that
 *     assignment, summed in increasing i;
 *   - update: S_j = sum over {i : L(i) = j} of x_i in increasing i, cnt_j the
 *     member count, c_j = S_j / cnt_j; an empty cluster keeps its centroid;
 *   - one iteration = assign with C_t, then update to C_{t+1};
 *   - tolerance mode (tol >= 0): after iteration t >= 1 stop if
 *     J_{t-1} - J_t <= tol * J_{t-1} or no label changed; tol < 0 runs exactly
 *     max_iter iterations.
 *
 * Inputs X (n x d) are FP32 values widened exactly to FP64; centroids are FP64
 * throughout.  The per-point map runs under OpenMP over points; every point's
 * arithmetic is the same whatever thread runs it, and every sum over points
 * is taken sequentially in increasing i, so results do not depend on the
 * thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* squared Euclidean distance between FP32 sample x and FP64 centroid c */
static double sqdist(const float *x, const double *c, int d)
{
    double s = 0.0;
    for (int f = 0; f < d; ++f) {
        double diff = (double)x[f] - c[f];
        s += diff * diff;
    }
    return s;
}

/*
 * Assign step (the collect body of the map).  For every sample i:
 *   labels[i] = smallest j attaining min_j d_ij,
 *   dmin[i]   = that minimum,
 *   d2nd[i]   = the smallest d_ij over j != labels[i] (+inf when k == 1).
 * Returns J = sum_i dmin[i] (increasing i).  dmin / d2nd may be NULL.
 */
double orc_assign(const float *X, const double *C, int64_t n, int d, int k,
                  int32_t *labels, double *dmin, double *d2nd)
{
    double *best = dmin ? dmin : (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const float *x = X + (size_t)i * (size_t)d;
        double b1 = 0.0, b2 = 1.0 / 0.0;
        int32_t j1 = -1;
        for (int j = 0; j < k; ++j) {
            double dij = sqdist(x, C + (size_t)j * (size_t)d, d);
            if (j1 < 0 || dij < b1) {
                if (j1 >= 0) b2 = b1;
                b1 = dij;
                j1 = j;
            } else if (dij < b2) {
                b2 = dij;
            }
        }
        labels[i] = j1;
        best[i] = b1;
        if (d2nd) d2nd[i] = b2;
    }
    double J = 0.0;
    for (int64_t i = 0; i < n; ++i) J += best[i];
    if (!dmin) free(best);
    return J;
}

/*
 * Update step (the predicated reduce per label, then avg = sum / length).
 * C_new[j] = mean of the samples labelled j, or C_old[j] when none is.
 * counts[j] = number of samples labelled j.  Labels must lie in [0, k).
 * Returns 0, or -1 if a label is out of range (outputs then undefined).
 */
int orc_update(const float *X, const int32_t *labels, const double *C_old,
               int64_t n, int d, int k, double *C_new, int64_t *counts)
{
    double *S = (double *)calloc((size_t)k * (size_t)d, sizeof(double));
    if (!S) return -2;
    for (int j = 0; j < k; ++j) counts[j] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t j = labels[i];
        if (j < 0 || j >= k) { free(S); return -1; }
        const float *x = X + (size_t)i * (size_t)d;
        double *s = S + (size_t)j * (size_t)d;
        for (int f = 0; f < d; ++f) s[f] += (double)x[f];
        counts[j] += 1;
    }
    for (int j = 0; j < k; ++j) {
        for (int f = 0; f < d; ++f) {
            size_t o = (size_t)j * (size_t)d + (size_t)f;
            C_new[o] = counts[j] > 0 ? S[o] / (double)counts[j] : C_old[o];
        }
    }
    free(S);
    return 0;
}

/*
 * Lloyd iterations from C0.  Outputs: C_out = C_T (FP64), labels = L_{T-1},
 * counts of L_{T-1}, J_hist[t] = J_t, changed_hist[t] = number of samples
 * whose label differs from iteration t-1 (n at t = 0).  J_hist / changed_hist
 * hold max_iter entries and may be NULL.  Returns the number of iterations
 * run, or a negative value on allocation failure.
 */
int orc_lloyd(const float *X, const double *C0, int64_t n, int d, int k,
              int max_iter, double tol, double *C_out, int32_t *labels,
              int64_t *counts, double *J_hist, int64_t *changed_hist)
{
    size_t kd = (size_t)k * (size_t)d;
    double *C = (double *)malloc(sizeof(double) * kd);
    double *Cn = (double *)malloc(sizeof(double) * kd);
    int32_t *prev = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!C || !Cn || !prev) { free(C); free(Cn); free(prev); return -2; }
    memcpy(C, C0, sizeof(double) * kd);
    double J_prev = 0.0;
    int t = 0;
    for (t = 0; t < max_iter; ++t) {
        if (t > 0) memcpy(prev, labels, sizeof(int32_t) * (size_t)n);
        double J = orc_assign(X, C, n, d, k, labels, NULL, NULL);
        int64_t changed = n;
        if (t > 0) {
            changed = 0;
            for (int64_t i = 0; i < n; ++i) changed += (labels[i] != prev[i]);
        }
        if (J_hist) J_hist[t] = J;
        if (changed_hist) changed_hist[t] = changed;
        int rc = orc_update(X, labels, C, n, d, k, Cn, counts);
        if (rc) { free(C); free(Cn); free(prev); return rc; }
        double *tmp = C; C = Cn; Cn = tmp;
        if (tol >= 0.0 && t >= 1 && ((J_prev - J) <= tol * J_prev || changed == 0)) {
            ++t;
            break;
        }
        J_prev = J;
    }
    memcpy(C_out, C, sizeof(double) * kd);
    free(C); free(Cn); free(prev);
    return t;
}

/*
 * Objective of given labels: J = sum_i d(x_i, c_{labels[i]}) (the J of the
 * assign step when the labels are the nearest centroids), samples in
 * increasing i.  Returns -1.0 if a label is out of range.
 */
double orc_objective(const float *X, const double *C, const int32_t *labels, int64_t n, int d, int k)
{
    double J = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t j = labels[i];
        if (j < 0 || j >= k) return -1.0;
        const double *cj = C + (size_t)j * (size_t)d;
        J += sqdist(X + (size_t)i * (size_t)d, cj, d);
    }
    return J;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
