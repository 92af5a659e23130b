// Finalize of one Lloyd iteration: the "combine" of the per-block activation
// records (section 2.3's generated loop merges partial records with the
// reduce function) in a fixed order, then the mean as sum / length
// (section 2.1) with the empty-cluster rule, the objective, the changed-label
// count and the tolerance decision.  Also the small helper kernels.
#include "km_internal.h"

#include <climits>

namespace km {

// Objective, changed count and the tolerance decision (one wave).
__device__ __forceinline__ void objective_wave(const FinArgs& a, int lane)
{
    double J = 0.0;
    int64_t ch = 0;
    // unrolled: the loads of several strides are in flight together (the
    // adds keep their order)
    if (a.jmode == 0) {
#pragma unroll 8
        for (int b = lane; b < a.GJ; b += 64) J += a.part.J[b];
    } else {
        const int nb = a.nJterm > 0 ? a.nJterm : finalize_blocks(a.k, a.d);
#pragma unroll 8
        for (int b = lane; b < nb; b += 64) J += a.Jterm[b];
    }
#pragma unroll 8
    for (int b = lane; b < a.GC; b += 64) ch += a.part.changed[b];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        J += __shfl_xor(J, off);
        ch += __shfl_xor(ch, off);
    }
    if (lane == 0) {
        if (a.jmode == 1) J = *a.sum_xn2 + J;
        const int t = a.iter;
        if (a.obj_hist) a.obj_hist[t] = J;
        if (a.ctrl) {
            Ctrl* c = a.ctrl;
            if (a.tol >= 0.0 && t >= 1) {
                const double Jp = c->J_prev;
                if ((Jp - J) <= a.tol * Jp || ch == 0) c->stop_iter = t;
            }
            c->J_prev = J;
            c->changed_last = ch;
            c->iters_done = t + 1;
        }
    }
}

__global__ __launch_bounds__(64) void finalize_objective_kernel(FinArgs a)
{
    if (a.ctrl != nullptr && a.ctrl->stop_iter < a.iter) return;
    objective_wave(a, threadIdx.x);
}

// The whole finalize of an iteration in one launch: block c (kFinWaves
// waves) sums the partial slots of the 64 elements 64c .. 64c+63 of the flat
// k*d sum array, wave w taking the slots [w G / W, (w+1) G / W) in increasing
// order over coalesced 512-byte rows; the wave sums are added in wave order,
// then the mean with the empty-cluster rule (and, with jmode 1, the block's
// share of the objective).  With jmode 0 and want_J one more block reduces
// the per-sample objective partials and the changed count and updates the
// control block; none of that depends on this launch's other blocks.
constexpr int kFinWaves = 16;
__global__ __launch_bounds__(64 * kFinWaves) void finalize_kernel(FinArgs a)
{
    __shared__ double sS[kFinWaves][64];
    __shared__ int32_t sC[kFinWaves][64];
    if (a.ctrl != nullptr && a.ctrl->stop_iter < a.iter) return;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    if ((int)blockIdx.x == finalize_blocks(a.k, a.d)) {
        if (wave == 0) objective_wave(a, lane);
        return;
    }
    const int64_t kd = (int64_t)a.k * a.d;
    const int64_t e = (int64_t)blockIdx.x * 64 + lane;
    const bool valid = e < kd;
    const int j = valid ? (int)(e / a.d) : 0;
    const int s0 = (int)(((int64_t)wave * a.G) / kFinWaves);
    const int s1 = (int)(((int64_t)(wave + 1) * a.G) / kFinWaves);
    double acc = 0.0;
    int32_t cacc = 0;
    if (valid) {
        const double* p = a.part.S + e;
        const int32_t* pc = a.part.cnt + j;
#pragma unroll 16
        for (int b = s0; b < s1; ++b) {
            acc += p[(size_t)b * kd];
            cacc += pc[(size_t)b * a.k];
        }
    }
    sS[wave][lane] = acc;
    sC[wave][lane] = cacc;
    __syncthreads();
    if (wave != 0) return;
    double term = 0.0;
    if (valid) {
        double S = sS[0][lane];
        int64_t c = sC[0][lane];
#pragma unroll
        for (int w = 1; w < kFinWaves; ++w) {
            S += sS[w][lane];
            c += sC[w][lane];
        }
        const int f = (int)(e - (int64_t)j * a.d);
        const float old = a.C_old ? a.C_old[(size_t)j * a.ld_old + f] : 0.0f;
        const float v = (c > 0) ? (float)(S / (double)c) : old;
        if (a.C_new) a.C_new[(size_t)j * a.ld_new + f] = v;
        if (a.Cp_out) a.Cp_out[(size_t)j * a.D + f] = v;
        if (a.counts && f == 0) a.counts[j] = c;
        if (a.S_out) a.S_out[(size_t)j * a.ld_S + f] = S;
        const double co = (double)old;
        term = (double)c * co * co - 2.0 * co * S;
    }
    if (a.jmode == 1) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) term += __shfl_xor(term, off);
        if (lane == 0) a.Jterm[a.jt_off + blockIdx.x] = term;
    }
}

// Batched finalize: block (instance, 64 elements) of 128 threads.  Wave 0
// sums the instance's partial slots for its elements in slot order, divides
// in FP64, rounds once to FP32 and applies the empty-cluster rule; wave 1 of
// the instance's first block reduces its objective partials (lane-strided,
// then xor tree) into obj_hist[iter].
__global__ __launch_bounds__(128) void batch_finalize_kernel(const BatchFinWork* __restrict__ work,
                                                             const FinArgs* __restrict__ fa, int32_t iter)
{
    const BatchFinWork w = work[blockIdx.x];
    const FinArgs a = fa[w.inst];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t kd = (int64_t)a.k * a.d;
    if (wave == 0) {
        const int64_t e = (int64_t)w.chunk * 64 + lane;
        double term = 0.0;
        if (e < kd) {
            const int j = (int)(e / a.d);
            const int f = (int)(e - (int64_t)j * a.d);
            double S = 0.0;
            int64_t c = 0;
#pragma unroll 8
            for (int b = 0; b < a.G; ++b) {
                S += a.part.S[(size_t)b * kd + e];
                c += a.part.cnt[(size_t)b * a.k + j];
            }
            const float old = a.C_old[(size_t)j * a.ld_old + f];
            const float v = (c > 0) ? (float)(S / (double)c) : old;
            a.C_new[(size_t)j * a.ld_new + f] = v;
            if (a.Cp_out) a.Cp_out[(size_t)j * a.D + f] = v;
            if (a.counts && f == 0) a.counts[j] = c;
            const double co = (double)old;
            term = (double)c * co * co - 2.0 * co * S;
        }
        if (a.jmode == 1) {
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) term += __shfl_xor(term, off);
            if (lane == 0) a.Jterm[w.chunk] = term;
        }
    } else if (w.chunk == 0 && a.jmode == 0) {
        double J = 0.0;
        for (int b = lane; b < a.GJ; b += 64) J += a.part.J[b];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) J += __shfl_xor(J, off);
        if (lane == 0 && a.obj_hist) a.obj_hist[iter] = J;
    }
}

// Batched objective with jmode 1: sum_i |x_i|^2 plus the Jterm shares of the
// instance's finalize blocks, in a fixed order; one wave per instance.
__global__ __launch_bounds__(64) void batch_objective_kernel(const FinArgs* __restrict__ fa, int32_t iter)
{
    const FinArgs a = fa[blockIdx.x];
    const int lane = threadIdx.x;
    const int nb = finalize_blocks(a.k, a.d);
    double J = 0.0;
    for (int b = lane; b < nb; b += 64) J += a.Jterm[b];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) J += __shfl_xor(J, off);
    if (lane == 0 && a.obj_hist) a.obj_hist[iter] = *a.sum_xn2 + J;
}

hipError_t launch_batch_objective(const FinArgs* fa, int ninst, int iter, hipStream_t s)
{
    hipLaunchKernelGGL(batch_objective_kernel, dim3(ninst), dim3(64), 0, s, fa, iter);
    return hipGetLastError();
}

// Batched: each instance's C (in FinArgs.C_new, row stride d) padded into its
// Cp (FinArgs.Cp_out, row stride D); one block per instance.
__global__ __launch_bounds__(256) void batch_pad_kernel(const FinArgs* __restrict__ fa)
{
    const FinArgs a = fa[blockIdx.x];
    const int64_t total = (int64_t)a.k * a.D;
    for (int64_t e = threadIdx.x; e < total; e += 256) {
        const int j = (int)(e / a.D);
        const int f = (int)(e - (int64_t)j * a.D);
        a.Cp_out[e] = (f < a.d) ? a.C_new[(size_t)j * a.d + f] : 0.0f;
    }
}

hipError_t launch_batch_finalize(const BatchFinWork* work, int nwork, const FinArgs* fa, int iter, hipStream_t s)
{
    hipLaunchKernelGGL(batch_finalize_kernel, dim3(nwork), dim3(128), 0, s, work, fa, iter);
    return hipGetLastError();
}

hipError_t launch_batch_pad(const FinArgs* fa, const float* const*, int ninst, hipStream_t s)
{
    hipLaunchKernelGGL(batch_pad_kernel, dim3(ninst), dim3(256), 0, s, fa);
    return hipGetLastError();
}

// Pads C (k x d) into Cp (k x D, zero columns d..D-1); optionally resets the
// control block.
__global__ void pad_centroids_kernel(const float* __restrict__ C, int32_t k, int32_t d, int32_t D,
                                     float* __restrict__ Cp, Ctrl* ctrl)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < (int64_t)k * D) {
        const int j = (int)(e / D);
        const int f = (int)(e - (int64_t)j * D);
        Cp[e] = (f < d) ? C[(size_t)j * d + f] : 0.0f;
    }
    if (ctrl != nullptr && e == 0) {
        ctrl->stop_iter = INT_MAX;
        ctrl->iters_done = 0;
        ctrl->J_prev = 0.0;
        ctrl->changed_last = 0;
    }
}

// Objective of an assign-only pass: slot partials in fixed lane-strided order.
__global__ void reduce_objective_kernel(const double* __restrict__ part_J, int32_t G, double* out)
{
    const int lane = threadIdx.x;
    double J = 0.0;
    for (int b = lane; b < G; b += 64) J += part_J[b];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) J += __shfl_xor(J, off);
    if (lane == 0) *out = J;
}

__global__ void copy_i32_kernel(const int32_t* __restrict__ src, int32_t* __restrict__ dst, int32_t n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// Debug-validate mode of the update from given labels: how many labels lie
// outside [0, k).  Block b counts a grid-stride share and writes part[b]; the
// host adds the partials (integers: any order gives the same total).
__global__ __launch_bounds__(256) void count_bad_labels_kernel(const int32_t* __restrict__ labels, int64_t n,
                                                               int32_t k, int32_t* __restrict__ part)
{
    __shared__ int32_t red[4];
    int32_t c = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int32_t L = labels[i];
        c += (L < 0 || L >= k) ? 1 : 0;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

hipError_t launch_count_bad_labels(const int32_t* labels, int64_t n, int32_t k, int32_t* part, int nblk,
                                   int* grid_used, hipStream_t s)
{
    const int64_t want = (n + 255) / 256;
    const int grid = (int)(want < nblk ? (want > 0 ? want : 1) : nblk);
    *grid_used = grid;
    hipLaunchKernelGGL(count_bad_labels_kernel, dim3(grid), dim3(256), 0, s, labels, n, k, part);
    return hipGetLastError();
}

hipError_t launch_finalize(const FinArgs& a, hipStream_t s)
{
    const int grid = finalize_blocks(a.k, a.d);
    const bool obj_block = a.want_J && a.jmode == 0;
    hipLaunchKernelGGL(finalize_kernel, dim3(grid + (obj_block ? 1 : 0)), dim3(64 * kFinWaves), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.want_J && a.jmode == 1) {
        hipLaunchKernelGGL(finalize_objective_kernel, dim3(1), dim3(64), 0, s, a);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_pad_centroids(const float* C, int32_t k, int32_t d, int32_t D, float* Cp, Ctrl* ctrl,
                                hipStream_t s)
{
    const int64_t total = (int64_t)k * D;
    const int grid = (int)((total + 255) / 256);
    hipLaunchKernelGGL(pad_centroids_kernel, dim3(grid > 0 ? grid : 1), dim3(256), 0, s, C, k, d, D, Cp, ctrl);
    return hipGetLastError();
}

hipError_t launch_reduce_objective(const double* part_J, int32_t G, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_objective_kernel, dim3(1), dim3(64), 0, s, part_J, G, out);
    return hipGetLastError();
}

hipError_t launch_copy_i32(const int32_t* src, int32_t* dst, int32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(copy_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

}  // namespace km
