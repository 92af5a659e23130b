// Assign step under a chosen metric and sample layout: squared Euclidean or
// L1 (the distance of the section 4.1 generated code, a sum of absolute
// differences), samples row-major (n x d, the section's data[i*dim + f]) or
// feature-major (d x n, struct-of-arrays, section 3.3).
//
// Canonical forms (fixed operation order, so results do not depend on the
// layout): diff = fl(x - c); features in chunks of 8, each chunk accumulated
// from 0 in feature order (squared: fused multiply-add; L1: add of |diff|);
// chunk partials summed by the pairwise tree.  The squared form is the plain
// path's distance operation for operation.  Error, relative to the exact
// distance (all terms non-negative): at most (2 + 8 + ceil(log2 P)) 2^-24
// (squared) or (1 + 8 + ceil(log2 P)) 2^-24 (L1), P = ceil(d / 8).
#include "km_dist.h"
#include "km_internal.h"

namespace km {

template <int D8, int METRIC>
__device__ __forceinline__ float dist_metric(const float (&x)[8 * D8], cfloat* c)
{
    float part[D8];
#pragma unroll
    for (int p = 0; p < D8; ++p) {
        part[p] = 0.0f;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float df = x[8 * p + q] - c[8 * p + q];
            if constexpr (METRIC == 0) part[p] = part[p] + __builtin_fabsf(df);
            else part[p] = __builtin_fmaf(df, df, part[p]);
        }
    }
#pragma unroll
    for (int s = 1; s < D8; s *= 2) {
#pragma unroll
        for (int p = 0; p + s < D8; p += 2 * s) part[p] = part[p] + part[p + s];
    }
    return part[0];
}

// Persistent grid: block b takes tiles b, b + G, ... of 256 samples (one per
// lane); labels and distances written per sample, the block's FP64 sum of
// the chosen distances (wave trees, waves in order) to partial slot b.
template <int D8, int METRIC, int LAYOUT>
__global__ __launch_bounds__(256) void assign_metric_kernel(MetricArgs a)
{
    constexpr int D = 8 * D8;
    __shared__ double redJ[kWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t n = a.n;
    const int d = a.d, k = a.k;
    const int64_t ntiles = (n + 255) / 256;
    double J = 0.0;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t i = t * 256 + tid;
        const bool valid = i < n;
        float x[D];
        if constexpr (LAYOUT == 0) {
            load_row<D8>(a.X + (valid ? i : 0) * d, d, valid, x);
        } else {
#pragma unroll
            for (int f = 0; f < D; ++f) x[f] = (valid && f < d) ? a.X[(size_t)f * n + i] : 0.0f;
        }
        float best = __builtin_huge_valf();
        int bj = 0;
        for (int j = 0; j < k; ++j) {
            const float dist = dist_metric<D8, METRIC>(x, (cfloat*)a.Cp + (size_t)j * D);
            if (dist < best) { best = dist; bj = j; }
        }
        if (valid) {
            a.labels[i] = bj;
            if (a.mindist) a.mindist[i] = best;
            J += (double)best;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) J += __shfl_xor(J, off);
    if (lane == 0) redJ[wave] = J;
    __syncthreads();
    if (tid == 0) {
        double s = redJ[0];
        for (int w = 1; w < kWaves; ++w) s += redJ[w];
        a.partJ[blockIdx.x] = s;
    }
}

template <int D8>
static void launch_d8(int metric, int layout, const MetricArgs& a, int grid, hipStream_t s)
{
    const dim3 g(grid), b(256);
    if (metric == 0 && layout == 0) hipLaunchKernelGGL((assign_metric_kernel<D8, 0, 0>), g, b, 0, s, a);
    else if (metric == 0) hipLaunchKernelGGL((assign_metric_kernel<D8, 0, 1>), g, b, 0, s, a);
    else if (layout == 0) hipLaunchKernelGGL((assign_metric_kernel<D8, 1, 0>), g, b, 0, s, a);
    else hipLaunchKernelGGL((assign_metric_kernel<D8, 1, 1>), g, b, 0, s, a);
}

hipError_t launch_assign_metric(int D8, int metric, int layout, const MetricArgs& a, int grid, hipStream_t s)
{
    switch (D8) {
    case 1: launch_d8<1>(metric, layout, a, grid, s); break;
    case 2: launch_d8<2>(metric, layout, a, grid, s); break;
    case 3: launch_d8<3>(metric, layout, a, grid, s); break;
    case 4: launch_d8<4>(metric, layout, a, grid, s); break;
    case 5: launch_d8<5>(metric, layout, a, grid, s); break;
    case 6: launch_d8<6>(metric, layout, a, grid, s); break;
    case 7: launch_d8<7>(metric, layout, a, grid, s); break;
    case 8: launch_d8<8>(metric, layout, a, grid, s); break;
    case 9: launch_d8<9>(metric, layout, a, grid, s); break;
    case 10: launch_d8<10>(metric, layout, a, grid, s); break;
    case 11: launch_d8<11>(metric, layout, a, grid, s); break;
    case 12: launch_d8<12>(metric, layout, a, grid, s); break;
    case 13: launch_d8<13>(metric, layout, a, grid, s); break;
    case 14: launch_d8<14>(metric, layout, a, grid, s); break;
    case 15: launch_d8<15>(metric, layout, a, grid, s); break;
    case 16: launch_d8<16>(metric, layout, a, grid, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace km
