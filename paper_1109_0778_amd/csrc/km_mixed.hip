// Mixed-precision assign for gfx950: the dense -2 X C^T term of
// |x - c|^2 = |x|^2 - 2 x.c + |c|^2 runs on the matrix cores in BF16 with
// FP32 accumulation; every sample whose nearest candidates are closer than a
// proven error band is re-checked with the canonical FP32 distance, so the
// labels are exactly those of the FP32 path.
//
// Keys.  The MFMA accumulator starts at bias_j = K + |c_j|^2 (K = 2 max|x|^2
// + 1, so every value is positive) and adds -2 x^.c^ (x^, c^ the BF16-rounded
// operands), giving e_ij = |x_i - c_j|^2 + K - |x_i|^2 up to rounding.  The
// low IB bits of the FP32 pattern of e_ij are replaced by j: positive floats
// order like their bit patterns, so one unsigned min tracks value and index.
//
// Band.  With u the unit roundoff of the operand format, for every j
//   |key_ij - e*_ij| <= B_i = 2(2u + u^2)|x_i| cmax
//                              + gamma_m emax_i + 2^-(23-IB) emax_i,
//   emax_i = K + cn2max + 2(1+u)^2 |x_i| cmax,
// (quantisation of both operands with Cauchy-Schwarz over |x_f c_f|; FP32
// accumulation of the bias and products in any order; key truncation).  The
// FP32 path's label j* satisfies e*_j* <= e*_j0 + 2.01 g d_j0 (j0 the exact
// argmin, g its canonical error bound), hence key_j* <= min_j key_ij + W_i,
//   W_i = 2 B_i + 2.01 g (|x_i| + cmax)^2.
// Samples whose candidate set {j : key_ij <= min key + W_i} has one member
// take it; the others are re-checked exactly over their candidates.
#include "km_internal.h"
#include "km_dist.h"

#include <climits>

namespace km {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

// ------------------------------------------------------------ run-level prep
// Per block: max |x|^2 (FP32) and sum |x|^2 (FP64, rows in a fixed order);
// the last block to finish is not special: a second one-wave kernel combines
// the block partials in index order.
__global__ __launch_bounds__(256) void prep_x_kernel(const float* __restrict__ X, int64_t n, int32_t d,
                                                     float* part_max, double* part_sum)
{
    __shared__ float smax[256];
    __shared__ double ssum[256];
    const int tid = threadIdx.x;
    float mx = 0.0f;
    double sm = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < n; i += (int64_t)gridDim.x * 256) {
        const float* row = X + i * d;
        float s32 = 0.0f;
        double s64 = 0.0;
        for (int f = 0; f < d; ++f) {
            const float v = row[f];
            s32 = __builtin_fmaf(v, v, s32);
            s64 += (double)v * (double)v;
        }
        mx = fmaxf(mx, s32);
        sm += s64;
    }
    smax[tid] = mx;
    ssum[tid] = sm;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if (tid < s) {
            smax[tid] = fmaxf(smax[tid], smax[tid + s]);
            ssum[tid] = ssum[tid] + ssum[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        part_max[blockIdx.x] = smax[0];
        part_sum[blockIdx.x] = ssum[0];
    }
}

__global__ void prep_x_combine_kernel(const float* part_max, const double* part_sum, int nb, XStats* xs)
{
    const int lane = threadIdx.x;
    float mx = 0.0f;
    double sm = 0.0;
    for (int b = lane; b < nb; b += 64) { mx = fmaxf(mx, part_max[b]); sm += part_sum[b]; }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        mx = fmaxf(mx, __shfl_xor(mx, off));
        sm += __shfl_xor(sm, off);
    }
    if (lane == 0) {
        // |x|^2 in FP32 is within a few ulp; the offset only needs to dominate it.
        xs->max_xn2 = mx;
        xs->K = 2.0f * mx * (1.0f + 1e-5f) + 1.0f;
        xs->sum_xn2 = sm;
    }
}

// ------------------------------------------------------ per-iteration prep
// One block: BF16 operand rows bf16(-2 c_j) (zero padded to DP features and
// kpad rows), biases K + |c_j|^2 (huge for padded rows), the band constants,
// and the recheck-queue reset.  The centroid loop invariants are hoisted here,
// out of the per-sample pass.
__global__ __launch_bounds__(256) void prep_c_kernel(const float* __restrict__ Cp, int32_t k, int32_t d,
                                                     int32_t D, int32_t kpad, int32_t DP,
                                                     const XStats* __restrict__ xs, __bf16* Ab,
                                                     float* bias, CStats* cs, int32_t* rq_count,
                                                     const Ctrl* ctrl, int32_t iter)
{
    __shared__ float smax[256];
    if (ctrl != nullptr && ctrl->stop_iter < iter) return;
    const int tid = threadIdx.x;
    const float K = xs->K;
    float cn2max = 0.0f;
    for (int j = tid; j < kpad; j += 256) {
        float s = 0.0f;
        if (j < k) {
            for (int f = 0; f < d; ++f) {
                const float v = Cp[(size_t)j * D + f];
                s = __builtin_fmaf(v, v, s);
            }
            cn2max = fmaxf(cn2max, s);
            bias[j] = K + s;
        } else {
            bias[j] = 3.0e38f;
        }
    }
    for (int64_t e = tid; e < (int64_t)kpad * DP; e += 256) {
        const int j = (int)(e / DP);
        const int f = (int)(e - (int64_t)j * DP);
        const float v = (j < k && f < d) ? -2.0f * Cp[(size_t)j * D + f] : 0.0f;
        Ab[e] = (__bf16)v;
    }
    smax[tid] = cn2max;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if (tid < s) smax[tid] = fmaxf(smax[tid], smax[tid + s]);
        __syncthreads();
    }
    if (tid == 0) {
        const float m = smax[0] * (1.0f + 1e-5f);
        cs->K = K;
        cs->cn2max = m;
        cs->cmax = sqrtf(m) * (1.0f + 1e-6f);
        cs->pad = 0.0f;
        *rq_count = 0;
    }
}

// ------------------------------------------------------------- the MFMA pass
__device__ __forceinline__ uint32_t thr_key(uint32_t m, float W, uint32_t ibm)
{
    const float v = __uint_as_float(m & ~ibm);
    return (__float_as_uint(v + W) & ~ibm) | ibm;
}

// Block = 4 waves; wave w holds the BF16 B-fragments of 2 x 32 samples (the
// 32-sample column blocks of a 32x32x16 MFMA) for the whole sweep over the
// centroids, which stream through LDS in chunks of 64 rows shared by the
// block.  Lane l of a 32x32 accumulator holds column l % 32 (one sample) and
// rows 8(i/4) + 4(l/32) + i%4, i < 16 (16 centroids); lanes l and l^32 hold
// the two halves of a sample's rows.
template <int D16>
__global__ __launch_bounds__(64 * kMixWaves) void mfma_assign_bf16(MixArgs a)
{
    constexpr int DP = 16 * D16;
    constexpr int ROWB = DP * 2 + 16;      // padded LDS row: conflict-free 16-byte reads
    constexpr int NB = kMixNB;
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned char* Abuf = smem;                                                   // [CK][ROWB]
    float* bbuf = reinterpret_cast<float*>(smem + kMixCK * ROWB);                 // [CK]
    uint32_t* cand = reinterpret_cast<uint32_t*>(bbuf + kMixCK);                  // [waves][NB][CAP][64]
    __shared__ int32_t sred[kMixWaves];

    if (a.ctrl != nullptr && a.ctrl->stop_iter < a.iter) return;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int h = lane >> 5;
    const int col = lane & 31;
    const int d = a.d;
    const int64_t n = a.n;
    const uint32_t ibm = (1u << a.IB) - 1u;
    const float K = a.cs->K, cmax = a.cs->cmax, cn2max = a.cs->cn2max;
    const float u = a.u;
    const float gm = (float)a.gamma_terms * 5.9604645e-8f;
    const float gamma_acc = gm / (1.0f - gm);
    const float trunc = __builtin_ldexpf(1.0f, a.IB - 23);
    const float P = (float)a.D8;
    const float gcan = (10.0f + (a.D8 > 1 ? ceilf(log2f(P)) : 0.0f)) * 5.9604645e-8f;
    const int nchunks = a.kpad / kMixCK;
    const int64_t ntiles = (n + kMixTile - 1) / kMixTile;
    uint32_t* mycand = cand + (size_t)wave * NB * kCandCap * 64;
    int32_t changed = 0;

    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        // --- B fragments (BF16) and |x| of this wave's 2 x 32 samples
        bf16x8 bfr[NB][D16];
        float W[NB];
        int64_t pidx[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int64_t p = t * kMixTile + (int64_t)wave * (NB * 32) + nb * 32 + col;
            pidx[nb] = p;
            const bool valid = p < n;
            const float* row = a.X + (valid ? p : 0) * d;
            float s2 = 0.0f;
#pragma unroll
            for (int s = 0; s < D16; ++s) {
                const int f0 = 16 * s + 8 * h;
                float v[8];
                if (valid && (d & 3) == 0 && f0 + 8 <= d) {
                    const float4 v0 = *reinterpret_cast<const float4*>(row + f0);
                    const float4 v1 = *reinterpret_cast<const float4*>(row + f0 + 4);
                    v[0] = v0.x; v[1] = v0.y; v[2] = v0.z; v[3] = v0.w;
                    v[4] = v1.x; v[5] = v1.y; v[6] = v1.z; v[7] = v1.w;
                } else {
#pragma unroll
                    for (int i = 0; i < 8; ++i) v[i] = (valid && f0 + i < d) ? row[f0 + i] : 0.0f;
                }
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    s2 = __builtin_fmaf(v[i], v[i], s2);
                    bfr[nb][s][i] = (__bf16)v[i];
                }
            }
            s2 += __shfl_xor(s2, 32);
            const float xn = sqrtf(s2) * (1.0f + 1e-6f);
            const float q = 2.0f * (2.0f * u + u * u);
            const float emax = K + cn2max + 2.0f * (1.0f + u) * (1.0f + u) * xn * cmax;
            const float B = q * xn * cmax + (gamma_acc + trunc) * emax;
            const float r = xn + cmax;
            W[nb] = (2.0f * B + 2.01f * gcan * r * r) * 1.001f;
        }

        uint32_t m[NB], thr[NB];
        int cnt[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) { m[nb] = 0xffffffffu; thr[nb] = 0xffffffffu; cnt[nb] = 0; }

        // --- sweep over the centroids
        for (int c = 0; c < nchunks; ++c) {
            __syncthreads();   // the previous chunk is no longer read
            {
                const uint4* src = reinterpret_cast<const uint4*>(a.Ab + (size_t)c * kMixCK * DP);
                constexpr int V = DP * 2 / 16;   // uint4 per row
                for (int e = tid; e < kMixCK * V; e += 64 * kMixWaves) {
                    const int r = e / V, q = e - r * V;
                    *reinterpret_cast<uint4*>(Abuf + r * ROWB + q * 16) = src[e];
                }
                for (int e = tid; e < kMixCK; e += 64 * kMixWaves) bbuf[e] = a.bias[(size_t)c * kMixCK + e];
            }
            __syncthreads();
#pragma unroll
            for (int tt = 0; tt < kMixCK / 32; ++tt) {
                f32x16 acc[NB];
                {
                    float bv[16];
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        const float4 b4 = *reinterpret_cast<const float4*>(bbuf + tt * 32 + 8 * g + 4 * h);
                        bv[4 * g + 0] = b4.x; bv[4 * g + 1] = b4.y; bv[4 * g + 2] = b4.z; bv[4 * g + 3] = b4.w;
                    }
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                        for (int i = 0; i < 16; ++i) acc[nb][i] = bv[i];
                }
                const unsigned char* arow = Abuf + (tt * 32 + col) * ROWB + 16 * h;
#pragma unroll
                for (int s = 0; s < D16; ++s) {
                    const bf16x8 af = *reinterpret_cast<const bf16x8*>(arow + 32 * s);
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, bfr[nb][s], acc[nb], 0, 0, 0);
                }
                // epilogue: keys, running minimum, candidate list
                const uint32_t j0 = (uint32_t)(c * kMixCK + tt * 32 + 4 * h);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    uint32_t key[16];
                    uint32_t mm = m[nb];
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        key[i] = (__float_as_uint(acc[nb][i]) & ~ibm) | (j0 + 8 * (i >> 2) + (i & 3));
                        mm = min(mm, key[i]);
                    }
                    m[nb] = mm;
                    thr[nb] = thr_key(mm, W[nb], ibm);
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        if (key[i] <= thr[nb]) {
                            if (cnt[nb] < kCandCap) mycand[(nb * kCandCap + cnt[nb]) * 64 + lane] = key[i];
                            ++cnt[nb];
                        }
                    }
                }
            }
        }

        // --- decide per sample: unique candidate, or queue an exact recheck
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const uint32_t mp = min(m[nb], (uint32_t)__shfl_xor((int)m[nb], 32));
            const uint32_t tf = thr_key(mp, W[nb], ibm);
            int vc = 0;
            const int stored = min(cnt[nb], kCandCap);
            for (int q = 0; q < stored; ++q) vc += (mycand[(nb * kCandCap + q) * 64 + lane] <= tf);
            const int ovf = cnt[nb] > kCandCap;
            const int vc_other = __shfl_xor(vc, 32);
            const int ovf_any = ovf | __shfl_xor(ovf, 32);
            const int64_t p = pidx[nb];
            const bool valid = p < n;
            // a winner index outside [0, k) can only come from non-finite keys: rescan
            const bool unique = !ovf_any && (vc + vc_other) == 1 && (int)(mp & ibm) < a.k;
            if (valid && unique && h == 0) {
                const int lab = (int)(mp & ibm);
                if (a.count_changed) changed += (a.iter == 0) ? 1 : (a.labels[p] != lab);
                a.labels[p] = lab;
            }
            int slot = 0;
            if (valid && !unique && h == 0) slot = atomicAdd(a.rq_count, 1);
            slot = __shfl(slot, col);           // lane l+32 takes lane l's slot
            const int base0 = __shfl(vc, col);  // candidates of the lower half come first
            if (valid && !unique) {
                int32_t* ent = a.rq + (size_t)slot * kRqInts;
                if (h == 0) {
                    ent[0] = (int32_t)p;
                    ent[1] = (ovf_any || (int)(mp & ibm) >= a.k) ? -1 : (vc + vc_other);
                }
                if (!ovf_any && (int)(mp & ibm) < a.k) {
                    int w = 2 + (h ? base0 : 0);
                    for (int q = 0; q < stored; ++q) {
                        const uint32_t kq = mycand[(nb * kCandCap + q) * 64 + lane];
                        if (kq <= tf) ent[w++] = (int32_t)(kq & ibm);
                    }
                }
            }
        }
    }

    // changed-label partial of this block (fixed order)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) changed += __shfl_xor(changed, off);
    if (lane == 0) sred[wave] = changed;
    __syncthreads();
    if (tid == 0) {
        int32_t c = 0;
        for (int w = 0; w < kMixWaves; ++w) c += sred[w];
        a.changed_part[blockIdx.x] = c;
    }
}

// ------------------------------------------------------------ exact recheck
// One queue entry per lane: the canonical FP32 distance (the same code as the
// plain pass) over the entry's candidates, lexicographic (distance, index)
// minimum; entries flagged -1 scan all k centroids in index order.
template <int D8>
__global__ __launch_bounds__(256) void recheck_kernel(RecheckArgs a)
{
    constexpr int D = 8 * D8;
    __shared__ int32_t sred[4];
    if (a.ctrl != nullptr && a.ctrl->stop_iter < a.iter) return;
    const int tid = threadIdx.x;
    const int count = *a.rq_count;
    int32_t changed = 0;
    for (int e = blockIdx.x * 256 + tid; e < count; e += gridDim.x * 256) {
        const int32_t* ent = a.rq + (size_t)e * kRqInts;
        const int64_t p = ent[0];
        const int nc = ent[1];
        float x[1][D];
        load_row<D8>(a.X + p * a.d, a.d, true, x[0]);
        float best = __builtin_huge_valf();
        int bj = 0;
        if (nc < 0) {
            for (int j = 0; j < a.k; ++j) {
                float dist[1];
                dist_rows<D8, 1>(x, a.Cp + (size_t)j * D, dist);
                if (dist[0] < best) { best = dist[0]; bj = j; }
            }
        } else {
            bj = 0;
            for (int q = 0; q < nc; ++q) {
                const int j = ent[2 + q];
                if (j < 0 || j >= a.k) continue;
                float dist[1];
                dist_rows<D8, 1>(x, a.Cp + (size_t)j * D, dist);
                if (dist[0] < best || (dist[0] == best && j < bj)) { best = dist[0]; bj = j; }
            }
        }
        if (a.count_changed) changed += (a.iter == 0) ? 1 : (a.labels[p] != bj);
        a.labels[p] = bj;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) changed += __shfl_xor(changed, off);
    if ((tid & 63) == 0) sred[tid >> 6] = changed;
    __syncthreads();
    if (tid == 0) a.changed_part[blockIdx.x] = sred[0] + sred[1] + sred[2] + sred[3];
}

// ------------------------------------------------------------------ launchers
hipError_t launch_prep_x(const float* X, int64_t n, int32_t d, float* part_max, double* part_sum, XStats* xs,
                         hipStream_t s)
{
    hipLaunchKernelGGL(prep_x_kernel, dim3(kXStatBlocks), dim3(256), 0, s, X, n, d, part_max, part_sum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(prep_x_combine_kernel, dim3(1), dim3(64), 0, s, part_max, part_sum, kXStatBlocks, xs);
    return hipGetLastError();
}

hipError_t launch_prep_c(const float* Cp, int32_t k, int32_t d, int32_t D, int32_t kpad, int32_t DP,
                         const XStats* xs, __bf16* Ab, float* bias, CStats* cs, int32_t* rq_count,
                         const Ctrl* ctrl, int32_t iter, hipStream_t s)
{
    hipLaunchKernelGGL(prep_c_kernel, dim3(1), dim3(256), 0, s, Cp, k, d, D, kpad, DP, xs, Ab, bias, cs, rq_count,
                       ctrl, iter);
    return hipGetLastError();
}

size_t mfma_lds_bytes(int D16)
{
    const size_t rowb = (size_t)D16 * 16 * 2 + 16;
    return kMixCK * rowb + kMixCK * sizeof(float) + (size_t)kMixWaves * kMixNB * kCandCap * 64 * sizeof(uint32_t);
}

template <int D16>
static hipError_t launch_mfma_d16(const MixArgs& a, int grid, hipStream_t s)
{
    const size_t lds = mfma_lds_bytes(D16);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&mfma_assign_bf16<D16>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((mfma_assign_bf16<D16>), dim3(grid), dim3(64 * kMixWaves), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_mfma_assign(int D16, const MixArgs& a, int grid, hipStream_t s)
{
    switch (D16) {
    case 1: return launch_mfma_d16<1>(a, grid, s);
    case 2: return launch_mfma_d16<2>(a, grid, s);
    case 3: return launch_mfma_d16<3>(a, grid, s);
    case 4: return launch_mfma_d16<4>(a, grid, s);
    case 5: return launch_mfma_d16<5>(a, grid, s);
    case 6: return launch_mfma_d16<6>(a, grid, s);
    case 7: return launch_mfma_d16<7>(a, grid, s);
    case 8: return launch_mfma_d16<8>(a, grid, s);
    default: return hipErrorInvalidValue;
    }
}

template <int D16>
static int occ_mfma()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, mfma_assign_bf16<D16>, 64 * kMixWaves,
                                                     mfma_lds_bytes(D16)) != hipSuccess)
        return -1;
    return nb;
}

int mfma_blocks_per_cu(int D16)
{
    switch (D16) {
    case 1: return occ_mfma<1>();
    case 2: return occ_mfma<2>();
    case 3: return occ_mfma<3>();
    case 4: return occ_mfma<4>();
    case 5: return occ_mfma<5>();
    case 6: return occ_mfma<6>();
    case 7: return occ_mfma<7>();
    case 8: return occ_mfma<8>();
    default: return -1;
    }
}

hipError_t launch_recheck(int D8, const RecheckArgs& a, int grid, hipStream_t s)
{
    switch (D8) {
#define KM_RC(N) case N: hipLaunchKernelGGL((recheck_kernel<N>), dim3(grid), dim3(256), 0, s, a); break;
    KM_RC(1) KM_RC(2) KM_RC(3) KM_RC(4) KM_RC(5) KM_RC(6) KM_RC(7) KM_RC(8)
    KM_RC(9) KM_RC(10) KM_RC(11) KM_RC(12) KM_RC(13) KM_RC(14) KM_RC(15) KM_RC(16)
#undef KM_RC
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace km
