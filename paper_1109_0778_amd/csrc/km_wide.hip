// Assign step for rows of more than 128 features (up to 1024), FP32.
//
// The sample row stays in memory (L1/L2) and is streamed in 8-feature
// chunks; kWideCJ centroids are evaluated per pass over the row.  The
// distance is the canonical direct form of the plain path, operation for
// operation: diff = fl(x - c), each chunk accumulated by FMA from 0, the
// chunk partials summed by the pairwise tree of dist_rows.  The tree is
// formed while streaming: when chunk p is done, its value is merged with the
// pending subtree of every level l at which bit l of p is set (left + right),
// and parked at the first level whose bit is clear; at the end the parked
// subtrees of the set bits of P (the number of chunks) are folded from the
// lowest level up, each as left + (accumulated right part).  This is exactly
// the left-aligned pairwise tree over P leaves, so distances, labels and the
// error bound (2 + 8 + ceil(log2 P)) 2^-24 are those of the plain path.
#include "km_dist.h"
#include "km_internal.h"

#include <climits>

namespace km {

constexpr int kWideCJ = 4;     // centroids per pass over a sample row
constexpr int kWideLevels = 8; // pairwise-tree levels for up to 128 chunks (1024 features)

__global__ __launch_bounds__(kBlock) void assign_wide_kernel(PassArgs a)
{
    __shared__ double redJ[kWaves];
    __shared__ int32_t redC[kWaves];
    if (a.ctrl != nullptr && a.ctrl->stop_iter < a.iter) return;   // converged earlier
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t n = a.n;
    const int d = a.d, k = a.k;
    const int P = (d + 7) / 8;                 // chunks
    const int D = 8 * P;                       // padded centroid row
    const bool vec = (d & 3) == 0;
    const int64_t ntiles = (n + kBlock - 1) / kBlock;
    double Jl = 0.0;
    int32_t changed = 0;
    cfloat* Cp = (cfloat*)a.Cp;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t i = t * kBlock + tid;
        const bool valid = i < n;
        const int old = (valid && a.count_changed && a.iter != 0) ? a.labels[i] : -1;
        const float* row = a.X + (valid ? i : 0) * d;
        float best = __builtin_huge_valf();
        int bj = 0;
        for (int j0 = 0; j0 < k; j0 += kWideCJ) {
            float st[kWideCJ][kWideLevels];
#pragma unroll
            for (int q = 0; q < kWideCJ; ++q)
#pragma unroll
                for (int l = 0; l < kWideLevels; ++l) st[q][l] = 0.0f;
            for (int p = 0; p < P; ++p) {
                float x[8];
                const int f0 = 8 * p;
                if (vec && f0 + 8 <= d) {
                    const float4 v0 = *reinterpret_cast<const float4*>(row + f0);
                    const float4 v1 = *reinterpret_cast<const float4*>(row + f0 + 4);
                    x[0] = v0.x; x[1] = v0.y; x[2] = v0.z; x[3] = v0.w;
                    x[4] = v1.x; x[5] = v1.y; x[6] = v1.z; x[7] = v1.w;
                } else {
#pragma unroll
                    for (int f = 0; f < 8; ++f) x[f] = f0 + f < d ? row[f0 + f] : 0.0f;
                }
#pragma unroll
                for (int q = 0; q < kWideCJ; ++q) {
                    const int j = min(j0 + q, k - 1);          // past k: a repeat, discarded below
                    cfloat* c = Cp + (size_t)j * D + f0;
                    float v = 0.0f;
#pragma unroll
                    for (int f = 0; f < 8; ++f) {
                        const float df = x[f] - c[f];
                        v = __builtin_fmaf(df, df, v);
                    }
                    bool parked = false;
#pragma unroll
                    for (int l = 0; l < kWideLevels; ++l) {
                        if (!parked) {
                            if ((p >> l) & 1) {
                                v = st[q][l] + v;
                            } else {
                                st[q][l] = v;
                                parked = true;
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < kWideCJ; ++q) {
                float r = 0.0f;
                bool have = false;
#pragma unroll
                for (int l = 0; l < kWideLevels; ++l) {
                    if ((P >> l) & 1) {
                        r = have ? st[q][l] + r : st[q][l];
                        have = true;
                    }
                }
                if (j0 + q < k && r < best) { best = r; bj = j0 + q; }
            }
        }
        if (valid) {
            if (a.count_changed) changed += (a.iter == 0) ? 1 : (old != bj);
            a.labels[i] = bj;
            if (a.mindist) a.mindist[i] = best;
            Jl += (double)best;
        }
    }
    // the plain pass's fixed-order reductions: xor tree, then waves in order
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        Jl += __shfl_xor(Jl, off);
        changed += __shfl_xor(changed, off);
    }
    if (lane == 0) { redJ[wave] = Jl; redC[wave] = changed; }
    __syncthreads();
    if (tid == 0) {
        double J = redJ[0];
        int32_t c = redC[0];
        for (int w = 1; w < kWaves; ++w) { J += redJ[w]; c += redC[w]; }
        a.part.J[blockIdx.x] = J;
        a.part.changed[blockIdx.x] = c;
    }
}

// The canonical distance of one sample row to one padded centroid row, both
// read from memory, with the streaming pairwise tree (per-lane operands).
__device__ __forceinline__ float wide_dist(const float* __restrict__ row, const float* __restrict__ c, int d)
{
    const int P = (d + 7) / 8;
    const bool vec = (d & 3) == 0;
    float st[kWideLevels];
#pragma unroll
    for (int l = 0; l < kWideLevels; ++l) st[l] = 0.0f;
    for (int p = 0; p < P; ++p) {
        const int f0 = 8 * p;
        float x[8];
        if (vec && f0 + 8 <= d) {
            const float4 v0 = *reinterpret_cast<const float4*>(row + f0);
            const float4 v1 = *reinterpret_cast<const float4*>(row + f0 + 4);
            x[0] = v0.x; x[1] = v0.y; x[2] = v0.z; x[3] = v0.w;
            x[4] = v1.x; x[5] = v1.y; x[6] = v1.z; x[7] = v1.w;
        } else {
#pragma unroll
            for (int f = 0; f < 8; ++f) x[f] = f0 + f < d ? row[f0 + f] : 0.0f;
        }
        const float4 c0 = *reinterpret_cast<const float4*>(c + f0);
        const float4 c1 = *reinterpret_cast<const float4*>(c + f0 + 4);
        const float cv[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
        float v = 0.0f;
#pragma unroll
        for (int f = 0; f < 8; ++f) {
            const float df = x[f] - cv[f];
            v = __builtin_fmaf(df, df, v);
        }
        bool parked = false;
#pragma unroll
        for (int l = 0; l < kWideLevels; ++l) {
            if (!parked) {
                if ((p >> l) & 1) {
                    v = st[l] + v;
                } else {
                    st[l] = v;
                    parked = true;
                }
            }
        }
    }
    float r = 0.0f;
    bool have = false;
#pragma unroll
    for (int l = 0; l < kWideLevels; ++l) {
        if ((P >> l) & 1) {
            r = have ? st[l] + r : st[l];
            have = true;
        }
    }
    return r;
}

// Exact recheck of the mixed path for rows of more than 128 features: one
// lane per queue entry, its candidates (or, for entries marked -1, all k
// centroids in index order) with the canonical distance; the lexicographic
// (distance, index) minimum wins.  Blocks (b, y) take every ny-th entry of
// queue region b.
__global__ __launch_bounds__(256) void recheck_wide_kernel(RecheckArgs a)
{
    __shared__ int32_t sred[kWaves];
    if (a.ctrl != nullptr && a.ctrl->stop_iter < a.iter) return;
    const int region = blockIdx.x, y = blockIdx.y, ny = gridDim.y;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int count = a.rq_count[region];
    const int32_t* rq_blk = a.rq + (size_t)region * a.rq_per_block * a.rq_ints;
    const int D = 8 * ((a.d + 7) / 8);
    int32_t changed = 0;
    for (int e = y * 256 + tid; e < count; e += ny * 256) {
        const int32_t* ent = rq_blk + (size_t)e * a.rq_ints;
        const int64_t p = ent[0];
        const int nc = ent[1];
        const int trips = nc < 0 ? a.k : nc;
        const float* row = a.X + p * a.d;
        float best = __builtin_huge_valf();
        int bj = 0;
        for (int t = 0; t < trips; ++t) {
            const int j = nc < 0 ? t : ent[kRqHead + t];
            if (j < 0 || j >= a.k) continue;
            const float dist = wide_dist(row, a.Cp + (size_t)j * D, a.d);
            if (dist < best || (dist == best && j < bj)) { best = dist; bj = j; }
        }
        if (a.count_changed) changed += (a.iter == 0) ? 1 : (a.labels[p] != bj);
        a.labels[p] = bj;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) changed += __shfl_xor(changed, off);
    if (lane == 0) sred[wave] = changed;
    __syncthreads();
    if (tid == 0) {
        int32_t c = 0;
        for (int w = 0; w < kWaves; ++w) c += sred[w];
        a.changed_part[y * a.nreg + region] = c;
    }
}

hipError_t launch_recheck_wide(const RecheckArgs& a, int G, hipStream_t s)
{
    hipLaunchKernelGGL(recheck_wide_kernel, dim3(G, kRecheckSplit), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_assign_wide(const PassArgs& a, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(assign_wide_kernel, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

int wide_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, assign_wide_kernel, kBlock, 0) != hipSuccess) return -1;
    return nb;
}

}  // namespace km
