// Training kernels of the section 4.2 applications that reuse the k-means
// groupBy-label reduce (the predicated per-class sums of section 2.3):
// multinomial naive Bayes (class priors and smoothed feature probabilities
// from the per-class sums) and Gaussian discriminant analysis (class priors,
// class means and the shared covariance, whose sum of outer products is a
// dense contraction run on the FP64 matrix cores).
#include "km_internal.h"

namespace km {

// Naive Bayes from the per-class sums (in phi) and counts (in prior, as
// int64), in place: T_c = sum_f S_cf in increasing f, phi_cf =
// (S_cf + 1) / (T_c + d), prior_c = n_c / n.  One block per class.
__global__ __launch_bounds__(256) void nb_finalize_kernel(double* prior, double* phi, int32_t d, int64_t n)
{
    __shared__ double sT;
    const int c = blockIdx.x;
    double* row = phi + (size_t)c * d;
    if (threadIdx.x == 0) {
        double T = 0.0;
        for (int f = 0; f < d; ++f) T += row[f];
        sT = T + (double)d;
        const int64_t cnt = reinterpret_cast<const int64_t*>(prior)[c];
        prior[c] = (double)cnt / (double)n;
    }
    __syncthreads();
    const double den = sT;
    for (int f = threadIdx.x; f < d; f += 256) row[f] = (row[f] + 1.0) / den;
}

// GDA means from the per-class sums (in mu) and counts (in prior, as int64),
// in place: mu_c = S_c / n_c (0 for an empty class), prior_c = n_c / n.
__global__ __launch_bounds__(256) void gda_means_kernel(double* prior, double* mu, int32_t d, int64_t n)
{
    __shared__ int64_t scnt;
    const int c = blockIdx.x;
    if (threadIdx.x == 0) scnt = reinterpret_cast<const int64_t*>(prior)[c];
    __syncthreads();
    const int64_t cnt = scnt;
    double* row = mu + (size_t)c * d;
    for (int f = threadIdx.x; f < d; f += 256) row[f] = cnt > 0 ? row[f] / (double)cnt : 0.0;
    __syncthreads();
    if (threadIdx.x == 0) prior[c] = (double)cnt / (double)n;
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Region pair p of the upper triangle (ra <= rb) over R regions, row by row.
__device__ __forceinline__ void region_pair(int p, int R, int& ra, int& rb)
{
    int r = 0;
    while (p >= R - r) { p -= R - r; ++r; }
    ra = r;
    rb = r + p;
}

// Shared covariance, partial sums: block (g, p) adds z_s z_s^T, z_s = x_s -
// mu_{y_s} (FP64), over its sample range into the 64 x 64 output region pair
// p, as 4 x 4 tiles of v_mfma_f64_16x16x4_f64 (four samples per step): lane l
// supplies z[s0 + l/16][feature 16 q + l%16] for the A (row) and B (column)
// blocks, and holds rows l/16 + 4 r (r = 0..3), column l%16 of each output
// tile.
__global__ __launch_bounds__(64) void gda_cov_kernel(CovArgs a)
{
    const int g = blockIdx.x, p = blockIdx.y;
    int ra, rb;
    region_pair(p, a.R, ra, rb);
    const int lane = threadIdx.x;
    const int col = lane & 15, kq = lane >> 4;
    const int d = a.d;
    const int64_t s_begin = (a.n * g) / a.G, s_end = (a.n * (g + 1)) / a.G;
    f64x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int64_t s0 = s_begin; s0 < s_end; s0 += 4) {
        const int64_t s = s0 + kq;
        const bool valid = s < s_end;
        const int y = valid ? a.labels[s] : 0;
        const float* xr = a.X + (valid ? s : 0) * d;
        const double* mr = a.mu + (size_t)y * d;
        double za[4], zb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int fa = ra * 64 + q * 16 + col, fb = rb * 64 + q * 16 + col;
            za[q] = (valid && fa < d) ? (double)xr[fa] - mr[fa] : 0.0;
            zb[q] = (valid && fb < d) ? (double)xr[fb] - mr[fb] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(za[i], zb[j], acc[i][j], 0, 0, 0);
    }
    double* out = a.part + ((size_t)g * a.RP + p) * 64 * 64;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = i * 16 + kq + 4 * r, cc = j * 16 + col;
                out[row * 64 + cc] = acc[i][j][r];
            }
}

// sigma[a][b] = (sum over ranges g, in order, of the partial element) / n,
// the lower triangle read from the transposed upper-triangle region pair.
__global__ __launch_bounds__(256) void gda_combine_kernel(CovArgs a)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int d = a.d;
    if (e >= (int64_t)d * d) return;
    int i = (int)(e / d), j = (int)(e - (int64_t)i * d);
    if (i / 64 > j / 64) { const int t = i; i = j; j = t; }
    const int ra = i / 64, rb = j / 64;
    // index of (ra, rb) in the row-by-row upper triangle
    const int p = ra * a.R - ra * (ra - 1) / 2 + (rb - ra);
    const double* src = a.part + (size_t)p * 64 * 64 + (i % 64) * 64 + (j % 64);
    double s = 0.0;
    for (int g = 0; g < a.G; ++g) s += src[(size_t)g * a.RP * 64 * 64];
    a.sigma[e] = s / (double)a.n;
}

hipError_t launch_nb_finalize(double* prior, double* phi, int32_t k, int32_t d, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(nb_finalize_kernel, dim3(k), dim3(256), 0, s, prior, phi, d, n);
    return hipGetLastError();
}

hipError_t launch_gda_means(const CovArgs& a, int32_t k, hipStream_t s)
{
    hipLaunchKernelGGL(gda_means_kernel, dim3(k), dim3(256), 0, s, a.prior, a.mu, a.d, a.n);
    return hipGetLastError();
}

hipError_t launch_gda_cov(const CovArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(gda_cov_kernel, dim3(a.G, a.RP), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gda_combine(const CovArgs& a, hipStream_t s)
{
    const int64_t dd = (int64_t)a.d * a.d;
    hipLaunchKernelGGL(gda_combine_kernel, dim3((unsigned)((dd + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace km
