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

// Shared covariance, partial sums: block (g, p) adds z_s z_s^T, z_s = x_s -
// mu_{y_s} (FP64), over its sample range into the 64 x 64 output region pair
// p, as 4 x 4 tiles of v_mfma_f64_16x16x4_f64 (four samples per step): lane l
// supplies z[s0 + l/16][feature 16 q + l%16] for the A (row) and B (column)
// blocks, and holds rows l/16 + 4 r (r = 0..3), column l%16 of each output
// tile.  The block's kCovWaves waves take interleaved 4-sample steps of the
// range, each with the next step's samples and labels in flight while its
// MFMAs run; the class means sit in LDS when they fit.  The wave sums are
// added in wave order into the block's partial region.
constexpr int kCovWaves = 4;
constexpr int kCovMuLds = 8192;     // class means held in LDS up to k d = 8192 (64 KiB)

template <bool MU_LDS, bool DIAG>
__global__ __launch_bounds__(64 * kCovWaves) void gda_cov_kernel(CovArgs a)
{
    extern __shared__ double smem[];   // [k*d] means (MU_LDS), then [64*64] wave-sum staging
    const int g = blockIdx.x;
    int ra, rb, p;
    if constexpr (DIAG) {
        ra = rb = blockIdx.y;                            // diagonal pair (r, r)
    } else {
        int q = blockIdx.y, r = 0;                       // q-th pair (r, r') with r < r', row by row
        while (q >= a.R - 1 - r) { q -= a.R - 1 - r; ++r; }
        ra = r;
        rb = r + 1 + q;
    }
    p = ra * a.R - ra * (ra - 1) / 2 + (rb - ra);        // slot of (ra, rb) in the upper triangle
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int d = a.d;
    const int kd = MU_LDS ? a.k * d : 0;
    if constexpr (MU_LDS) {
        for (int e = tid; e < kd; e += 64 * kCovWaves) smem[e] = a.mu[e];
        __syncthreads();
    }
    const double* mu = MU_LDS ? smem : a.mu;
    double* stage = smem + kd;
    const int64_t s_begin = (a.n * g) / a.G, s_end = (a.n * (g + 1)) / a.G;
    f64x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    int fa[4], fb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) { fa[q] = ra * 64 + q * 16 + col; fb[q] = rb * 64 + q * 16 + col; }
    // raw sample values and label of this lane's sample in a step (clamped
    // addresses, so every load is unconditional; invalid values are masked
    // when used).  On a diagonal region pair the column block is the row block.
    auto fetch = [&](int64_t s0, float (&xa)[4], float (&xb)[4], int& y) {
        const int64_t s = s0 + kq;
        const bool valid = s < s_end;
        const int64_t sc = valid ? s : s_begin;
        const int yy = a.labels[sc];
        y = (valid && yy >= 0 && yy < a.k) ? yy : -1;   // a label outside [0, k) adds nothing
        const float* xr = a.X + sc * d;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            xa[q] = xr[min(fa[q], d - 1)];
            if constexpr (!DIAG) xb[q] = xr[min(fb[q], d - 1)];
        }
    };
    // PF steps in flight: step t is computed from buffer t % PF, which is
    // then refilled with step t + PF (HBM latency exceeds one step's MFMAs)
    constexpr int PF = 4;
    const int64_t step = 4 * kCovWaves;
    const int64_t first = s_begin + 4 * wave;
    float xa[PF][4], xb[PF][4] = {};
    int yb[PF];
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        yb[u] = -1;
        if (first + u * step < s_end) fetch(first + u * step, xa[u], xb[u], yb[u]);
    }
    for (int64_t s0 = first; s0 < s_end; s0 += PF * step) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int64_t su = s0 + u * step;
            if (su >= s_end) break;
            const int y = yb[u];
            double za[4], zb[4];
            const double* mr = mu + (size_t)(y < 0 ? 0 : y) * d;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double va = (double)xa[u][q] - mr[min(fa[q], d - 1)];
                za[q] = (y >= 0 && fa[q] < d) ? va : 0.0;
                if constexpr (DIAG) {
                    zb[q] = za[q];
                } else {
                    const double vb = (double)xb[u][q] - mr[min(fb[q], d - 1)];
                    zb[q] = (y >= 0 && fb[q] < d) ? vb : 0.0;
                }
            }
            yb[u] = -1;
            if (su + PF * step < s_end) fetch(su + PF * step, xa[u], xb[u], yb[u]);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(za[i], zb[j], acc[i][j], 0, 0, 0);
        }
    }
    // wave sums in wave order: wave 0 stores, each later wave adds in turn
    double* out = a.part + ((size_t)g * a.RP + p) * 64 * 64;
    for (int w = 0; w < kCovWaves; ++w) {
        if (wave == w) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int e = (i * 16 + kq + 4 * r) * 64 + j * 16 + col;
                        stage[e] = w == 0 ? acc[i][j][r] : stage[e] + acc[i][j][r];
                    }
        }
        __syncthreads();
    }
    for (int e = tid; e < 64 * 64; e += 64 * kCovWaves) out[e] = stage[e];
}

// sigma[a][b] = (sum over ranges g, in order, of the partial element) / n,
// the lower triangle read from the transposed upper-triangle region pair.
// Block c takes the 64 elements 64c .. 64c+63 of sigma; wave w sums the
// ranges [w G / W, (w+1) G / W) in increasing order, and the wave sums are
// added in wave order (a fixed order for every element).
constexpr int kCombWaves = 16;
__global__ __launch_bounds__(64 * kCombWaves) void gda_combine_kernel(CovArgs a)
{
    __shared__ double part[kCombWaves][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t e = (int64_t)blockIdx.x * 64 + lane;
    const int d = a.d;
    const bool valid = e < (int64_t)d * d;
    double s = 0.0;
    if (valid) {
        int i = (int)(e / d), j = (int)(e - (int64_t)i * d);
        if (i / 64 > j / 64) { const int t = i; i = j; j = t; }
        const int ra = i / 64, rb = j / 64;
        const int p = ra * a.R - ra * (ra - 1) / 2 + (rb - ra);   // slot of (ra, rb) in the upper triangle
        const double* src = a.part + (size_t)p * 64 * 64 + (i % 64) * 64 + (j % 64);
        const int g0 = (int)(((int64_t)wave * a.G) / kCombWaves), g1 = (int)(((int64_t)(wave + 1) * a.G) / kCombWaves);
#pragma unroll 8
        for (int g = g0; g < g1; ++g) s += src[(size_t)g * a.RP * 64 * 64];
    }
    part[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && valid) {
        double t = part[0][lane];
        for (int w = 1; w < kCombWaves; ++w) t += part[w][lane];
        a.sigma[e] = t / (double)a.n;
    }
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
    const bool mu_lds = (int64_t)a.k * a.d <= kCovMuLds;
    const size_t lds = ((mu_lds ? (size_t)a.k * a.d : 0) + 64 * 64) * sizeof(double);
    // one launch per kind of region pair: the R diagonal pairs, then the others
    const int nd = a.R, no = a.RP - a.R;
    if (mu_lds) hipLaunchKernelGGL((gda_cov_kernel<true, true>), dim3(a.G, nd), dim3(64 * kCovWaves), lds, s, a);
    else hipLaunchKernelGGL((gda_cov_kernel<false, true>), dim3(a.G, nd), dim3(64 * kCovWaves), lds, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || no == 0) return e;
    if (mu_lds) hipLaunchKernelGGL((gda_cov_kernel<true, false>), dim3(a.G, no), dim3(64 * kCovWaves), lds, s, a);
    else hipLaunchKernelGGL((gda_cov_kernel<false, false>), dim3(a.G, no), dim3(64 * kCovWaves), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_gda_combine(const CovArgs& a, hipStream_t s)
{
    const int64_t dd = (int64_t)a.d * a.d;
    hipLaunchKernelGGL(gda_combine_kernel, dim3((unsigned)((dd + 63) / 64)), dim3(64 * kCombWaves), 0, s, a);
    return hipGetLastError();
}

}  // namespace km
