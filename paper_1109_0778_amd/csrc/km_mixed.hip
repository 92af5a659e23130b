// Mixed-precision assign for gfx950: the dense -2 X C^T term of
// |x - c|^2 = |x|^2 - 2 x.c + |c|^2 runs on the matrix cores in BF16 or FP8
// (e4m3) with FP32 accumulation; every sample whose nearest candidates are
// closer than a proven error band is re-checked with the canonical FP32
// distance, so the labels are exactly those of the FP32 path.
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
//
// FP8.  Features are scaled by powers of two s_f >= max_i |x_if| / 448, so
// x~_if = x_if / s_f is exact and within the e4m3 range; centroids become
// c~_jf = c_jf s_f / r with one power of two r >= max |c_jf s_f| / 448.  Then
// x.c = r sum_f x~_f c~_f, and the MFMA forms sum_f q_f q'_f with q = e4m3(x~),
// q' = e4m3(c~) (products exact in FP32).  Keys are kept divided by 2r (exact):
// the accumulator starts at (K + |c_j|^2) / (2r) and the operand is -q'.  With
// u = 2^-4 and an absolute error eta = 2^-6 per element (covers e4m3
// subnormals whether rounded or flushed),
//   |sum x~c~ - sum q q'| <= (2u + u^2) S + (1 + u) eta (L1(c~) + L1(x~)) + D eta^2,
// S = |x| cmax / r >= sum_f |x~_f c~_f| (Cauchy-Schwarz); the accumulation and
// truncation terms are as above with every magnitude divided by 2r.
#include "km_internal.h"
#include "km_dist.h"

#include <climits>

namespace km {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

// ------------------------------------------------------------ run-level prep
// |x|^2 of one row in FP32 (fused multiply-add in feature order) and in FP64:
// 16 features per step, all loads of a step issued before their first use
// (float4 when the row is 16-byte aligned, clamped scalars otherwise).
__device__ __forceinline__ void row_norm2(const float* __restrict__ row, int d, float& s32, double& s64)
{
    s32 = 0.0f;
    s64 = 0.0;
    if ((d & 3) == 0) {
        for (int f0 = 0; f0 < d; f0 += 16) {
            float4 v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int f = f0 + 4 * q;
                v[q] = *reinterpret_cast<const float4*>(row + (f < d ? f : d - 4));
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (f0 + 4 * q < d) {
                    const float e[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        s32 = __builtin_fmaf(e[i], e[i], s32);
                        s64 += (double)e[i] * (double)e[i];
                    }
                }
            }
        }
    } else {
        for (int f0 = 0; f0 < d; f0 += 16) {
            float v[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) v[i] = row[f0 + i < d ? f0 + i : d - 1];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                if (f0 + i < d) {
                    s32 = __builtin_fmaf(v[i], v[i], s32);
                    s64 += (double)v[i] * (double)v[i];
                }
            }
        }
    }
}

// Per block: max |x|^2 (FP32) and sum |x|^2 (FP64, rows in a fixed order); a
// second one-wave kernel combines the block partials in a fixed order.
__global__ __launch_bounds__(256) void prep_x_kernel(const float* __restrict__ X, int64_t n, int32_t d,
                                                     float* part_max, double* part_sum)
{
    __shared__ float smax[256];
    __shared__ double ssum[256];
    const int tid = threadIdx.x;
    float mx = 0.0f;
    double sm = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < n; i += (int64_t)gridDim.x * 256) {
        float s32;
        double s64;
        row_norm2(X + i * d, d, s32, s64);
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

// FP8 run-level prep.  (1) Per-block max |x_f| per feature: the grid's
// threads take elements t, t + S, t + 2S, ... with S a multiple of d, so each
// thread stays on one feature.  (2) One block turns the maxima into scales.
// (3) One thread per sample writes its e4m3 row and its band inputs.
__global__ __launch_bounds__(256) void prep_fmax_kernel(const float* __restrict__ X, int64_t n, int32_t d,
                                                        int32_t DP, float* part_fmax)
{
    __shared__ uint32_t smax[16 * kMaxD16Wide];
    const int tid = threadIdx.x;
    for (int f = tid; f < DP; f += 256) smax[f] = 0u;
    __syncthreads();
    const int64_t T = (int64_t)gridDim.x * 256;
    const int64_t S = (T / d) * d;
    const int64_t t = (int64_t)blockIdx.x * 256 + tid;
    if (t < S) {
        float m = 0.0f;
        const int64_t total = n * d;
        for (int64_t e0 = t; e0 < total; e0 += 8 * S) {
            float v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {                   // 8 loads in flight, clamped addresses
                const int64_t e = e0 + q * S;
                v[q] = X[e < total ? e : t];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) m = fmaxf(m, fabsf(v[q]));   // the clamped repeat of X[t] is harmless
        }
        atomicMax(&smax[t % d], __float_as_uint(m));     // non-negative floats order like their bits
    }
    __syncthreads();
    for (int f = tid; f < DP; f += 256) part_fmax[(size_t)blockIdx.x * DP + f] = __uint_as_float(smax[f]);
}

// smallest power of two p with m / p <= limit (1 when m == 0)
__device__ __forceinline__ float pow2_scale(float m, float limit)
{
    if (!(m > 0.0f)) return 1.0f;
    int e = 0;
    (void)frexpf(m / limit, &e);            // m / limit < 2^e
    float p = __builtin_ldexpf(1.0f, e - 1);
    while (m * (1.0f / p) > limit) p *= 2.0f;
    return p;
}

__global__ __launch_bounds__(256) void prep_fscale_kernel(const float* __restrict__ part_fmax, int nb, int32_t d,
                                                          int32_t DP, float* fscale)
{
    for (int f = threadIdx.x; f < DP; f += 256) {
        float m = 0.0f;
#pragma unroll 16
        for (int b = 0; b < nb; ++b) m = fmaxf(m, part_fmax[(size_t)b * DP + f]);   // 16 loads in flight
        const float sc = f < d ? pow2_scale(m, kFp8Max) : 1.0f;
        fscale[f] = sc;
        fscale[DP + f] = 1.0f / sc;         // exact: a power of two
    }
}

__device__ __forceinline__ uint32_t fp8_of(float v)
{
    v = fminf(fmaxf(v, -kFp8Max), kFp8Max);
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false) & 0xffu;
}

// Eight features of one row per thread and chunk: a row takes G adjacent
// lanes (G = DP / 8 rounded up to a power of two, at most 16; lanes past
// DP / 8 idle), lane g holding chunks g, g + G, ... (one chunk up to DP =
// 128), so the row is read and written coalesced and its sums are completed
// by an xor tree across those lanes.
__host__ __device__ constexpr int row_lanes_q(int DP)
{
    return DP / 8 <= 2 ? 2 : DP / 8 <= 4 ? 4 : DP / 8 <= 8 ? 8 : 16;
}
__host__ __device__ constexpr int row_chunks_q(int DP) { return DP / 8 <= 16 ? 1 : (DP / 8 + 15) / 16; }

// Relative upward margin that makes sqrt of an FP32 sum of squares of a row
// (8 C sequential FMA terms per lane, then a log2 G-level tree) an upper
// bound of the exact norm: half the sum's relative error plus the rounding
// of the square root and of the product, with room to spare.
__host__ __device__ inline float norm_margin(int DP)
{
    const int C = row_chunks_q(DP), G = row_lanes_q(DP);
    const int lg = G <= 2 ? 1 : G <= 4 ? 2 : G <= 8 ? 3 : 4;
    const float m = (float)((8 * C + lg) / 2 + 4) * 5.9604645e-8f;
    return m > 1e-6f ? m : 1e-6f;
}

// Row i and chunk (lane g, pass c) of thread t (G consecutive threads per
// row, rows below n live); x[8]: the chunk's features (zero past d).
// Returns whether the thread holds a live chunk.
__device__ __forceinline__ bool row_chunk_at(const float* __restrict__ X, int64_t n, int32_t d, int32_t DP, int c,
                                             int64_t t, int64_t& i, int& f0, float (&x)[8])
{
    const int G = row_lanes_q(DP);
    i = t / G;
    f0 = 8 * ((int)(t - i * G) + G * c);
    const bool live = i < n && f0 < DP;
    const float* row = X + (live ? i : 0) * d;
    if ((d & 7) == 0) {
        // the chunk lies inside the row (DP = d rounded up to 16, chunks of 8
        // past d only when d % 16 == 8: clamp those to the row's last chunk)
        const int fc = f0 < d ? f0 : d - 8;                 // idle lanes and the chunk past d: in the row
        const float4 v0 = *reinterpret_cast<const float4*>(row + fc);
        const float4 v1 = *reinterpret_cast<const float4*>(row + fc + 4);
        const bool in = live && f0 < d;   // (f0 < d also keeps idle lanes' loads in the row)
        x[0] = in ? v0.x : 0.0f; x[1] = in ? v0.y : 0.0f; x[2] = in ? v0.z : 0.0f; x[3] = in ? v0.w : 0.0f;
        x[4] = in ? v1.x : 0.0f; x[5] = in ? v1.y : 0.0f; x[6] = in ? v1.z : 0.0f; x[7] = in ? v1.w : 0.0f;
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int f = f0 + q;
            const float v = row[f < d ? f : d - 1];
            x[q] = (live && f < d) ? v : 0.0f;
        }
    }
    return live;
}

__device__ __forceinline__ bool row_chunk(const float* __restrict__ X, int64_t n, int32_t d, int32_t DP, int c,
                                          int64_t& i, int& f0, float (&x)[8])
{
    return row_chunk_at(X, n, d, DP, c, (int64_t)blockIdx.x * 256 + threadIdx.x, i, f0, x);
}

template <typename T>
__device__ __forceinline__ T row_sum(T v, int cpr)
{
    for (int off = 1; off < cpr; off <<= 1) v += __shfl_xor(v, off);
    return v;
}

__global__ __launch_bounds__(256) void quant_x_kernel(const float* __restrict__ X, int64_t n, int32_t d, int32_t DP,
                                                      const float* __restrict__ fscale, uint8_t* Xq, float2* xst)
{
    const float* inv = fscale + DP;
    float s2 = 0.0f, l1 = 0.0f;
    int64_t i = 0;
    bool live0 = false;
    for (int c = 0; c < row_chunks_q(DP); ++c) {
        int f0;
        float x[8];
        const bool live = row_chunk(X, n, d, DP, c, i, f0, x);
        if (c == 0) live0 = live;
        uint32_t w[2] = {0u, 0u};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float xt = x[q] * inv[f0 + q < DP ? f0 + q : DP - 1];   // idle lanes: a valid index
            s2 = __builtin_fmaf(x[q], x[q], s2);
            l1 += fabsf(xt);
            w[q >> 2] |= fp8_of(xt) << (8 * (q & 3));
        }
        if (live) *reinterpret_cast<uint2*>(Xq + i * DP + f0) = make_uint2(w[0], w[1]);
    }
    s2 = row_sum(s2, row_lanes_q(DP));
    l1 = row_sum(l1, row_lanes_q(DP));
    const int G = row_lanes_q(DP);
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (live0 && t % G == 0) xst[i] = make_float2(sqrtf(s2) * (1.0f + norm_margin(DP)), l1 * (1.0f + 1e-5f));
}

// Once per call: the BF16 copy of X the BF16 MFMA passes read (rounded to
// nearest even, zero padded to DP features) and an upper bound of |x| per
// sample.
// Thread t's share (G threads per row; rows of index n or more are idle).
// With STATS, the row's first thread also folds the row into the running
// statistics: mx = max FP32 |x|^2, sm += FP64 |x|^2.
template <bool STATS = false>
__device__ __forceinline__ void quant_bf16_at(const float* __restrict__ X, int64_t n, int32_t d, int32_t DP,
                                              __bf16* Xb, float* xn, int64_t t, float* mx = nullptr,
                                              double* sm = nullptr)
{
    float s2 = 0.0f;
    double s64 = 0.0;
    int64_t i = 0;
    bool live0 = false;
    for (int c = 0; c < row_chunks_q(DP); ++c) {
        int f0;
        float x[8];
        const bool live = row_chunk_at(X, n, d, DP, c, t, i, f0, x);
        if (c == 0) live0 = live;
        bf16x8 w;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            s2 = __builtin_fmaf(x[q], x[q], s2);
            if constexpr (STATS) s64 += (double)x[q] * (double)x[q];
            w[q] = (__bf16)x[q];
        }
        if (live) *reinterpret_cast<bf16x8*>(Xb + i * DP + f0) = w;
    }
    s2 = row_sum(s2, row_lanes_q(DP));
    const int G = row_lanes_q(DP);
    if constexpr (STATS) s64 = row_sum(s64, G);
    if (live0 && t % G == 0) {
        xn[i] = sqrtf(s2) * (1.0f + norm_margin(DP));
        if constexpr (STATS) {
            *mx = fmaxf(*mx, s2);
            *sm += s64;
        }
    }
}

__global__ __launch_bounds__(256) void quant_x_bf16_kernel(const float* __restrict__ X, int64_t n, int32_t d,
                                                           int32_t DP, __bf16* Xb, float* xn)
{
    quant_bf16_at(X, n, d, DP, Xb, xn, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

// ------------------------------------------------------ per-iteration prep
// One block: BF16 operand rows bf16(-2 c_j) (zero padded to DP features and
// kpad rows), biases K + |c_j|^2 (huge for padded rows) and the band constants.
// The centroid loop invariants are hoisted here, out of the per-sample pass.
__device__ __forceinline__ void prep_c_body(const float* __restrict__ Cp, int32_t k, int32_t d, int32_t D,
                                            int32_t kpad, int32_t DP, const XStats* __restrict__ xs, __bf16* Ab,
                                            float* bias, CStats* cs, const Ctrl* ctrl, int32_t iter)
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
        const float m = smax[0] * (1.0f + fmaxf(1e-5f, (float)(d + 4) * 5.9604645e-8f));
        cs->K = K;
        cs->cn2max = m;
        cs->cmax = sqrtf(m) * (1.0f + 1e-6f);
        cs->inv2r = 1.0f;
        cs->inv_r = 2.0f;
        cs->cl1 = 0.0f;
        cs->pad[0] = cs->pad[1] = 0.0f;
    }
}

__global__ __launch_bounds__(256) void prep_c_kernel(const float* __restrict__ Cp, int32_t k, int32_t d,
                                                     int32_t D, int32_t kpad, int32_t DP,
                                                     const XStats* __restrict__ xs, __bf16* Ab,
                                                     float* bias, CStats* cs, const Ctrl* ctrl, int32_t iter)
{
    prep_c_body(Cp, k, d, D, kpad, DP, xs, Ab, bias, cs, ctrl, iter);
}

// The same, spread over kPrepRows-row blocks (large k x d): each block writes
// its rows' operands and biases and the largest |c_j|^2 among them; a
// one-wave kernel reduces those maxima into the band constants.
constexpr int kPrepRows = 32;
__global__ __launch_bounds__(256) void prep_c_rows_kernel(const float* __restrict__ Cp, int32_t k, int32_t d,
                                                          int32_t D, int32_t kpad, int32_t DP,
                                                          const XStats* __restrict__ xs, __bf16* Ab, float* bias,
                                                          float* part_cn2, const Ctrl* ctrl, int32_t iter)
{
    __shared__ float smax[kPrepRows];
    if (ctrl != nullptr && ctrl->stop_iter < iter) return;
    const int tid = threadIdx.x;
    const int r0 = blockIdx.x * kPrepRows;
    if (tid < kPrepRows) {
        const int j = r0 + tid;
        float s = 0.0f;
        if (j < k) {
            for (int f = 0; f < d; ++f) {
                const float v = Cp[(size_t)j * D + f];
                s = __builtin_fmaf(v, v, s);
            }
        }
        if (j < kpad) bias[j] = j < k ? xs->K + s : 3.0e38f;
        smax[tid] = s;
    }
    for (int e = tid; e < kPrepRows * DP; e += 256) {
        const int j = r0 + e / DP;
        const int f = e - (e / DP) * DP;
        if (j < kpad) {
            const float v = (j < k && f < d) ? -2.0f * Cp[(size_t)j * D + f] : 0.0f;
            Ab[(size_t)j * DP + f] = (__bf16)v;
        }
    }
    __syncthreads();
    if (tid == 0) {
        float m = 0.0f;
        for (int q = 0; q < kPrepRows; ++q) m = fmaxf(m, smax[q]);
        part_cn2[blockIdx.x] = m;
    }
}

__global__ __launch_bounds__(64) void prep_c_stats_kernel(const float* __restrict__ part_cn2, int nb, int32_t d,
                                                          const XStats* __restrict__ xs, CStats* cs,
                                                          const Ctrl* ctrl, int32_t iter)
{
    if (ctrl != nullptr && ctrl->stop_iter < iter) return;
    const int lane = threadIdx.x;
    float m = 0.0f;
    for (int b = lane; b < nb; b += 64) m = fmaxf(m, part_cn2[b]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if (lane == 0) {
        const float mm = m * (1.0f + fmaxf(1e-5f, (float)(d + 4) * 5.9604645e-8f));
        cs->K = xs->K;
        cs->cn2max = mm;
        cs->cmax = sqrtf(mm) * (1.0f + 1e-6f);
        cs->inv2r = 1.0f;
        cs->inv_r = 2.0f;
        cs->cl1 = 0.0f;
        cs->pad[0] = cs->pad[1] = 0.0f;
    }
}

// Batched (BF16): one block per instance.
__global__ __launch_bounds__(256) void batch_prep_c_kernel(const BatchMix* __restrict__ bm)
{
    const BatchMix& b = bm[blockIdx.x];
    prep_c_body(b.Cp, b.m.k, b.m.d, b.D, b.m.kpad, b.DP, b.xs,
                const_cast<__bf16*>(static_cast<const __bf16*>(b.m.Ab)), const_cast<float*>(b.m.bias),
                const_cast<CStats*>(b.m.cs), nullptr, 0);
}

// Batched run-level prep: row b of the work table covers rows [t0, t1) of one
// instance, writes their BF16 copy and |x| bounds, and its statistics (fixed
// order per thread, then a fixed tree) to partial slot `slot`; a one-wave
// combine per instance follows.
__global__ __launch_bounds__(256) void batch_prep_x_kernel(const BatchWork* __restrict__ work,
                                                           const BatchMix* __restrict__ bm)
{
    __shared__ float smax[256];
    __shared__ double ssum[256];
    const BatchWork w = work[blockIdx.x];
    const BatchMix& b = bm[w.inst];
    const float* X = b.m.X;
    const int d = b.m.d;
    const int tid = threadIdx.x;
    float mx = 0.0f;
    double sm = 0.0;
    // the BF16 copy of rows [t0, t1) and their |x| bounds, as quant_x_bf16_kernel,
    // with the statistics from the same reads (t0 is a multiple of 256, so the
    // G threads of a row share a wave; each row's first thread adds the row)
    const int G = row_lanes_q(b.DP);
    for (int64_t base = w.t0 * G; base < w.t1 * G; base += 256)
        quant_bf16_at<true>(X, w.t1, d, b.DP, const_cast<__bf16*>(b.m.Xb), const_cast<float*>(b.m.xn), base + tid,
                            &mx, &sm);
    smax[tid] = mx;
    ssum[tid] = sm;
    __syncthreads();
    for (int st = 128; st >= 1; st >>= 1) {
        if (tid < st) {
            smax[tid] = fmaxf(smax[tid], smax[tid + st]);
            ssum[tid] = ssum[tid] + ssum[tid + st];
        }
        __syncthreads();
    }
    if (tid == 0) {
        b.xpart_max[w.slot] = smax[0];
        b.xpart_sum[w.slot] = ssum[0];
    }
}

__global__ __launch_bounds__(64) void batch_prep_x_combine_kernel(const BatchMix* __restrict__ bm)
{
    const BatchMix& b = bm[blockIdx.x];
    const int lane = threadIdx.x;
    float mx = 0.0f;
    double sm = 0.0;
    for (int q = lane; q < b.nxb; q += 64) { mx = fmaxf(mx, b.xpart_max[q]); sm += b.xpart_sum[q]; }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        mx = fmaxf(mx, __shfl_xor(mx, off));
        sm += __shfl_xor(sm, off);
    }
    if (lane == 0) {
        b.xs->max_xn2 = mx;
        b.xs->K = 2.0f * mx * (1.0f + 1e-5f) + 1.0f;
        b.xs->sum_xn2 = sm;
    }
}

// FP8: one block.  Pass 1: |c_j|^2, the largest |c_jf s_f| and |c_j|; the
// centroid scale r; pass 2: operands e4m3(-c~), biases (K + |c_j|^2) / (2r)
// and the largest L1 norm of the scaled centroids.
__global__ __launch_bounds__(256) void prep_c_fp8_kernel(const float* __restrict__ Cp, int32_t k, int32_t d,
                                                         int32_t D, int32_t kpad, int32_t DP,
                                                         const XStats* __restrict__ xs,
                                                         const float* __restrict__ fscale, uint8_t* Aq,
                                                         float* bias, CStats* cs, const Ctrl* ctrl, int32_t iter)
{
    __shared__ float smax[256], samax[256];
    __shared__ float sr[2];
    if (ctrl != nullptr && ctrl->stop_iter < iter) return;
    const int tid = threadIdx.x;
    const float K = xs->K;
    float cn2max = 0.0f, amax = 0.0f;
    for (int j = tid; j < k; j += 256) {
        float s = 0.0f;
        for (int f = 0; f < d; ++f) {
            const float v = Cp[(size_t)j * D + f];
            s = __builtin_fmaf(v, v, s);
            amax = fmaxf(amax, fabsf(v * fscale[f]));
        }
        cn2max = fmaxf(cn2max, s);
    }
    smax[tid] = cn2max;
    samax[tid] = amax;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if (tid < s) {
            smax[tid] = fmaxf(smax[tid], smax[tid + s]);
            samax[tid] = fmaxf(samax[tid], samax[tid + s]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        const float r = pow2_scale(samax[0], kFp8Max);
        sr[0] = 1.0f / r;                   // exact
        sr[1] = 0.5f / r;
        const float m = smax[0] * (1.0f + fmaxf(1e-5f, (float)(d + 4) * 5.9604645e-8f));
        cs->cn2max = m;
        cs->cmax = sqrtf(m) * (1.0f + 1e-6f);
    }
    __syncthreads();
    const float inv_r = sr[0], inv2r = sr[1];
    float cl1 = 0.0f;
    for (int j = tid; j < kpad; j += 256) {
        float s = 0.0f, l1 = 0.0f;
        if (j < k) {
            for (int f = 0; f < d; ++f) {
                const float v = Cp[(size_t)j * D + f];
                s = __builtin_fmaf(v, v, s);
                l1 += fabsf(v * fscale[f] * inv_r);
            }
            bias[j] = (K + s) * inv2r;
        } else {
            bias[j] = 3.0e38f;
        }
        cl1 = fmaxf(cl1, l1);
    }
    for (int64_t e = tid; e < (int64_t)kpad * DP / 4; e += 256) {
        const int j = (int)(e * 4 / DP);
        const int f0 = (int)(e * 4 - (int64_t)j * DP);
        uint32_t w = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int f = f0 + q;
            const float v = (j < k && f < d) ? -(Cp[(size_t)j * D + f] * fscale[f] * inv_r) : 0.0f;
            w |= fp8_of(v) << (8 * q);
        }
        reinterpret_cast<uint32_t*>(Aq)[e] = w;
    }
    __syncthreads();                        // smax is reused below
    smax[tid] = cl1;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if (tid < s) smax[tid] = fmaxf(smax[tid], smax[tid + s]);
        __syncthreads();
    }
    if (tid == 0) {
        cs->K = K;
        cs->inv2r = inv2r;
        cs->inv_r = inv_r;
        cs->cl1 = smax[0] * (1.0f + fmaxf(1e-5f, (float)(d + 4) * 5.9604645e-8f));
        cs->pad[0] = cs->pad[1] = 0.0f;
    }
}

// ------------------------------------------------------------- the MFMA pass
// median of three: with a <= b, the second smallest of {a, b, c}
__device__ __forceinline__ uint32_t med3_u32(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ __forceinline__ uint32_t thr_key(uint32_t m, float W, uint32_t ibm)
{
    const float v = __uint_as_float(m & ~ibm);
    return (__float_as_uint(v + W) & ~ibm) | ibm;
}

// Block = 4 waves; wave w holds the B fragments of kMixNB x 32 samples (the
// 32-sample column blocks of a 32x32x16 MFMA; one block per wave measured
// fastest: fewer registers, more resident waves) for the whole sweep over the
// centroids, which stream through LDS in chunks of 64 rows shared by the
// block.  Lane l of a 32x32 accumulator holds column l % 32 (one sample) and
// rows 8(i/4) + 4(l/32) + i%4, i < 16 (16 centroids); lanes l and l^32 hold
// the two halves of a sample's rows.
// One block's share of the MFMA pass: 128-sample tiles t_first, t_first +
// t_step, ... below t_end; its recheck entries go to queue region `region`.
// STAGE 0: keys, running minimum and candidate lists over consecutive
// samples.  STAGE 1 (screen): only the two smallest keys of each sample; a
// sample whose second key lies outside its band takes the smallest, the
// others are listed in region `region` of a.amb (with their smallest key in
// a.amb_key when given).  STAGE 2: the stage-1 screen over the samples
// listed in region `region` of a.amb_in (a BF16 screen of what an FP8 screen
// left open).  STAGE 3 (refine after a screen with the same operands) over
// the samples listed in a.amb_in: the smallest key, and so the band, is the
// screen's (a.amb_key_in); the sweep lists the keys inside it and nothing
// more.
template <int D16, int FMT, int STAGE, int NW>
__device__ __forceinline__ void mfma_body(const MixArgs& a, int64_t t_first, int64_t t_end, int64_t t_step,
                                          int region, unsigned char* smem)
{
    // D16 = 0: rows of more than 128 features; the operands are streamed
    // from memory (L2) through the MFMA chain instead of being held in
    // registers (samples) and staged in LDS (centroids)
    constexpr bool WIDE = D16 == 0;
    constexpr bool F8 = FMT == FMT_FP8;
    constexpr int ES = F8 ? 1 : 2;         // operand bytes per feature
    constexpr int DP = 16 * D16;
    const int DPr = WIDE ? a.DP : DP;      // operand row width
    constexpr int ROWB = DP * ES + 16;     // padded LDS row: conflict-free reads
    constexpr int NB = mix_nb(STAGE);
    constexpr int TILE = NW * NB * 32;      // samples per block per tile
    constexpr int CHB = kMixCK * ROWB;     // bytes of one chunk buffer
    constexpr int V = DP * ES / 16;        // uint4 per centroid row
    constexpr int CAP = kCandCap;
    constexpr int SLOTS = kCandSlots;
    constexpr int RQI = kRqInts;
    constexpr int PF = WIDE ? 1 : (kMixCK * V + 64 * NW - 1) / (64 * NW);   // prefetch uint4 per thread
    // centroid chunk buffers: two, or one per chunk (a.nbuf, sized by the host)
    const int nbuf = !WIDE && a.nbuf > 2 ? a.nbuf : 2;
    unsigned char* Abuf = smem;                                                   // [nbuf][CK][ROWB]
    float* bbuf = reinterpret_cast<float*>(smem + (size_t)nbuf * CHB);            // [nbuf][CK]
    uint32_t* cand = reinterpret_cast<uint32_t*>(bbuf + nbuf * kMixCK);           // [waves][NB][SLOTS][64]
    __shared__ int32_t sred[NW];
    __shared__ int32_t blk_count;           // recheck entries queued by this block
    __shared__ int32_t blk_full;            // ... of which full scans (candidate list overflowed)

    if (a.ctrl != nullptr && a.ctrl->stop_iter < a.iter) return;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int h = lane >> 5;
    if (tid == 0) { blk_count = 0; blk_full = 0; }
    int32_t* rq_blk = a.rq + (size_t)region * a.rq_per_block * RQI;
    const int col = lane & 31;
    const int d = a.d;
    const int64_t n = a.n;
    const uint32_t ibm = (1u << a.IB) - 1u;
    const float K = a.cs->K, cmax = a.cs->cmax, cn2max = a.cs->cn2max;
    const float inv2r = a.cs->inv2r, inv_r = a.cs->inv_r, cl1 = a.cs->cl1;
    const float u = a.u;
    const float gm = (float)a.gamma_terms * 5.9604645e-8f;
    const float gamma_acc = gm / (1.0f - gm);
    const float trunc = __builtin_ldexpf(1.0f, a.IB - 23);
    const float P = (float)a.D8;
    const float gcan = (10.0f + (a.D8 > 1 ? ceilf(log2f(P)) : 0.0f)) * 5.9604645e-8f;
    const int nchunks = a.kpad / kMixCK;
    constexpr bool SCREEN = STAGE == 1 || STAGE == 2;   // two smallest keys only
    constexpr bool LISTED = STAGE >= 2;                  // a sweep over an earlier pass's open samples
    const int amb_n = LISTED ? a.amb_in_count[region] : 0;        // samples listed for this block
    const int32_t* amb_list = LISTED ? a.amb_in + (size_t)region * a.rq_per_block : nullptr;
    const uint32_t* amb_key = STAGE == 3 ? a.amb_key_in + (size_t)region * a.rq_per_block : nullptr;
    const int64_t ntiles = LISTED ? (amb_n + TILE - 1) / TILE : (n + TILE - 1) / TILE;
    const int64_t t_last = t_end < ntiles ? t_end : ntiles;
    uint32_t* mycand = cand + (size_t)wave * NB * SLOTS * 64;
    int32_t changed = 0;

    // Chunk c of the centroid operands: registers <- global, LDS buffer <- registers.
#define KM_LOAD_CHUNK(c_)                                                                 \
    {                                                                                     \
        const uint4* src_ = reinterpret_cast<const uint4*>(                               \
            static_cast<const unsigned char*>(a.Ab) + (size_t)(c_) * kMixCK * DP * ES);   \
        _Pragma("unroll") for (int i_ = 0; i_ < PF; ++i_) {                               \
            const int e_ = tid + i_ * 64 * NW;                                     \
            pr[i_] = (e_ < kMixCK * V) ? src_[e_] : make_uint4(0, 0, 0, 0);               \
        }                                                                                 \
        pb = (tid < kMixCK) ? a.bias[(size_t)(c_) * kMixCK + tid] : 0.0f;                 \
    }
#define KM_STORE_CHUNK(buf_)                                                              \
    {                                                                                     \
        _Pragma("unroll") for (int i_ = 0; i_ < PF; ++i_) {                               \
            const int e_ = tid + i_ * 64 * NW;                                     \
            if (e_ < kMixCK * V) {                                                        \
                const int row_ = e_ / V, q_ = e_ - row_ * V;                              \
                *reinterpret_cast<uint4*>(Abuf + (buf_) * CHB + row_ * ROWB + q_ * 16) = pr[i_]; \
            }                                                                             \
        }                                                                                 \
        if (tid < kMixCK) bbuf[(buf_) * kMixCK + tid] = pb;                              \
    }
    uint4 pr[PF];
    float pb = 0.0f;
    // The next chunk is prefetched one part per 32-row tile: part tt is loaded
    // at the start of tile tt and stored to the other buffer at the start of
    // tile tt + 1 (the last part after the tiles), so only PFH registers stay
    // live across a tile.
    constexpr int NTT = kMixCK / 32;                 // 32-row tiles per chunk
    constexpr int PFH = (PF + NTT - 1) / NTT;       // prefetch uint4 per thread per tile
    uint4 prh[PFH];
#define KM_LOAD_PART(c_, hf_)                                                             \
    {                                                                                     \
        const uint4* src_ = reinterpret_cast<const uint4*>(                               \
            static_cast<const unsigned char*>(a.Ab) + (size_t)(c_) * kMixCK * DP * ES);   \
        _Pragma("unroll") for (int i_ = 0; i_ < PFH; ++i_) {                              \
            const int q_ = (hf_) * PFH + i_;                                              \
            const int e_ = tid + q_ * 64 * NW;                                     \
            prh[i_] = (q_ < PF && e_ < kMixCK * V) ? src_[e_] : make_uint4(0, 0, 0, 0);   \
        }                                                                                 \
        if ((hf_) == 0) pb = (tid < kMixCK) ? a.bias[(size_t)(c_) * kMixCK + tid] : 0.0f; \
    }
#define KM_STORE_PART(buf_, hf_)                                                          \
    {                                                                                     \
        _Pragma("unroll") for (int i_ = 0; i_ < PFH; ++i_) {                              \
            const int q_ = (hf_) * PFH + i_;                                              \
            const int e_ = tid + q_ * 64 * NW;                                     \
            if (q_ < PF && e_ < kMixCK * V) {                                             \
                const int row_ = e_ / V, qq_ = e_ - row_ * V;                             \
                *reinterpret_cast<uint4*>(Abuf + (buf_) * CHB + row_ * ROWB + qq_ * 16) = prh[i_]; \
            }                                                                             \
        }                                                                                 \
        if ((hf_) == 0 && tid < kMixCK) bbuf[(buf_) * kMixCK + tid] = pb;                \
    }
    // With a buffer per chunk (two chunks, or more that the host sized the
    // buffers for) every chunk stays in LDS for the whole block: no reload per
    // tile and no barrier between chunks.
    const bool resident = !WIDE && nchunks >= 2 && nchunks == nbuf;
    int cur = 0;
    if (t_first < t_last) {
        KM_LOAD_CHUNK(0)
        KM_STORE_CHUNK(0)
        if (resident) {
            for (int c = 1; c < nchunks; ++c) {
                KM_LOAD_CHUNK(c)
                KM_STORE_CHUNK(c)
            }
        }
    }
    __syncthreads();

    for (int64_t t = t_first; t < t_last; t += t_step) {
        // --- B fragments and the band of this wave's samples
        bf16x8 bfr[NB][(F8 || WIDE) ? 1 : D16];
        long bq[NB][(F8 && !WIDE) ? D16 : 1];
        const unsigned char* brow[NB];     // WIDE: this lane's half of the sample's operand row
        float W[NB];
        int64_t pidx[NB];
        uint32_t mfix[NB];   // stage 3: the screen's smallest key of the sample
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            int64_t p = t * TILE + (int64_t)wave * (NB * 32) + nb * 32 + col;
            if constexpr (STAGE == 3) mfix[nb] = p < amb_n ? amb_key[p] : 0u;
            if constexpr (LISTED) p = p < amb_n ? (int64_t)amb_list[p] : n;   // a listed sample, or none
            pidx[nb] = p;
            const bool valid = p < n;
            if constexpr (F8) {
                const uint8_t* qrow = a.Xq + (valid ? p : 0) * DPr + 8 * h;
                if constexpr (WIDE) {
                    brow[nb] = qrow;       // an invalid sample's keys are never used
                } else {
#pragma unroll
                    for (int s = 0; s < D16; ++s) bq[nb][s] = valid ? *reinterpret_cast<const long*>(qrow + 16 * s) : 0l;
                }
                const float2 st = valid ? a.xst[p] : make_float2(0.0f, 0.0f);
                const float xn = st.x;
                const float u = a.u;
                const float eta = 0.015625f;                        // 2^-6
                const float S = xn * cmax * inv_r;
                const float Sq = (1.0f + u) * eta * (cl1 + st.y) + (float)DP * eta * eta;
                const float Eq = (2.0f * u + u * u) * S + Sq;
                const float Pq = (1.0f + u) * (1.0f + u) * S + Sq;
                const float emax = (K + cn2max) * inv2r + Pq;
                const float B = Eq + (gamma_acc + trunc) * emax;
                const float r = xn + cmax;
                W[nb] = (2.0f * B + 2.01f * gcan * r * r * inv2r) * 1.001f;
            } else {
                float xn;
                if (WIDE || a.Xb != nullptr) {
                    // the run's BF16 copy: one 16-byte load per 16 features
                    const bf16x8* xr = reinterpret_cast<const bf16x8*>(a.Xb + (valid ? p : 0) * DPr + 8 * h);
                    if constexpr (WIDE) {
                        brow[nb] = reinterpret_cast<const unsigned char*>(xr);
                    } else {
#pragma unroll
                        for (int s = 0; s < D16; ++s) bfr[nb][s] = xr[2 * s];
                    }
                    xn = valid ? a.xn[p] : 0.0f;
                } else if constexpr (!WIDE) {
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
                    xn = sqrtf(s2) * (1.0f + 1e-6f);
                }
                const float u = a.u;
                const float q = 2.0f * (2.0f * u + u * u);
                const float emax = K + cn2max + 2.0f * (1.0f + u) * (1.0f + u) * xn * cmax;
                const float B = q * xn * cmax + (gamma_acc + trunc) * emax;
                const float r = xn + cmax;
                W[nb] = (2.0f * B + 2.01f * gcan * r * r) * 1.001f;
            }
        }

        // stage 3: the final band is known before the sweep
        uint32_t tfix[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) tfix[nb] = STAGE == 3 ? thr_key(mfix[nb], W[nb], ibm) : 0u;

        // m: running minimum key; cnt: list length; cut: smallest key dropped
        // from a full list (every kept entry is below it); ovf: a full list
        // that could not be split (equal values), i.e. rescan the sample
        uint32_t m[NB], m2[NB], thr[NB], cut[NB];
        int cnt[NB], ovf[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            m[nb] = 0xffffffffu; m2[nb] = 0xffffffffu; thr[nb] = 0xffffffffu; cut[nb] = 0xffffffffu; cnt[nb] = 0; ovf[nb] = 0;
        }

        // --- sweep over the centroids; the next chunk (possibly chunk 0 of the
        // next tile) is fetched into registers while this one is computed
        for (int c = 0; c < nchunks; ++c) {
            const bool pref = !resident && nchunks > 1 && (c + 1 < nchunks || t + t_step < t_last);
            const int cnext = c + 1 < nchunks ? c + 1 : 0;
            const int buf = resident ? c : cur;
            const unsigned char* Ab_c = Abuf + buf * CHB;
            const float* bb_c = bbuf + buf * kMixCK;
            // screen: the two smallest keys of this chunk, indexed within the
            // chunk (compile-time constants); chunk base and lane offset are
            // added when the pair joins the running one
            uint32_t lm[NB], lm2[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) { lm[nb] = 0xffffffffu; lm2[nb] = 0xffffffffu; }
#pragma unroll
            for (int tt = 0; tt < kMixCK / 32; ++tt) {
                if (pref) {
                    if (tt > 0) KM_STORE_PART(cur ^ 1, tt - 1)
                    KM_LOAD_PART(cnext, tt)
                }
                f32x16 acc[NB];
                {
                    float bvv[16];
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        const float4 b4 = *reinterpret_cast<const float4*>(bb_c + tt * 32 + 8 * g + 4 * h);
                        bvv[4 * g + 0] = b4.x; bvv[4 * g + 1] = b4.y; bvv[4 * g + 2] = b4.z; bvv[4 * g + 3] = b4.w;
                    }
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                        for (int i = 0; i < 16; ++i) acc[nb][i] = bvv[i];
                }
                const unsigned char* arow = Ab_c + (tt * 32 + col) * ROWB + 8 * ES * h;
                // candidate-list stages raise the wave's priority while its MFMA
                // chain issues (the matrix pipe stays fed while other waves run
                // their longer epilogues); the screens measured faster without
                if constexpr (!SCREEN) __builtin_amdgcn_s_setprio(1);
                if constexpr (WIDE) {
                    // centroid and sample operands straight from memory, one
                    // 16-feature step at a time
                    const unsigned char* ag = static_cast<const unsigned char*>(a.Ab) +
                                              ((size_t)(c * kMixCK + tt * 32 + col) * DPr + 8 * h) * ES;
                    for (int s = 0; s < DPr / 16; ++s) {
                        if constexpr (F8) {
                            const long af = *reinterpret_cast<const long*>(ag + 16 * s);
#pragma unroll
                            for (int nb = 0; nb < NB; ++nb)
                                acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(
                                    af, *reinterpret_cast<const long*>(brow[nb] + 16 * s), acc[nb], 0, 0, 0);
                        } else {
                            const bf16x8 af = *reinterpret_cast<const bf16x8*>(ag + 32 * s);
#pragma unroll
                            for (int nb = 0; nb < NB; ++nb)
                                acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                    af, *reinterpret_cast<const bf16x8*>(brow[nb] + 32 * s), acc[nb], 0, 0, 0);
                        }
                    }
                }
                if constexpr (F8) {
                    long an = D16 > 0 ? *reinterpret_cast<const long*>(arow) : 0l;
#pragma unroll
                    for (int s = 0; s < D16; ++s) {
                        const long af = an;
                        if (s + 1 < D16) an = *reinterpret_cast<const long*>(arow + 16 * (s + 1));
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb)
                            acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(af, bq[nb][s], acc[nb], 0, 0, 0);
                    }
                } else if constexpr (!WIDE) {
                    // the next step's centroid fragment is read while this step's MFMAs run
                    bf16x8 an = *reinterpret_cast<const bf16x8*>(arow);
#pragma unroll
                    for (int s = 0; s < D16; ++s) {
                        const bf16x8 af = an;
                        if (s + 1 < D16) an = *reinterpret_cast<const bf16x8*>(arow + 32 * (s + 1));
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb)
                            acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, bfr[nb][s], acc[nb], 0, 0, 0);
                    }
                    // schedule: fragment 0's LDS read, then per step the next
                    // fragment's read ahead of this step's MFMAs
                    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
#pragma unroll
                    for (int s = 0; s + 1 < D16; ++s) {
                        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                        __builtin_amdgcn_sched_group_barrier(0x008, NB, 0);
                    }
                    __builtin_amdgcn_sched_group_barrier(0x008, NB, 0);
                }
                if constexpr (!SCREEN) __builtin_amdgcn_s_setprio(0);
                // epilogue: keys, running minimum, candidate list
                const uint32_t j0 = (uint32_t)(c * kMixCK + tt * 32 + 4 * h);
                if constexpr (SCREEN && (WIDE || D16 > 5)) {
                    // the two smallest keys of the chunk so far (lm <= lm2),
                    // one key at a time (3 VALU operations per key): at 96 or
                    // more features the MFMA chain outlasts the epilogue
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb) {
                            const uint32_t key = (__float_as_uint(acc[nb][i]) & ~ibm) | (uint32_t)(tt * 32 + 8 * (i >> 2) + (i & 3));
                            lm2[nb] = med3_u32(lm[nb], lm2[nb], key);
                            lm[nb] = min(lm[nb], key);
                        }
                    }
                    continue;
                } else if constexpr (SCREEN) {
                    // shorter chains leave the epilogue as the longer part:
                    // keys two at a time; with a <= b <= c the sorted lm, k0,
                    // k1, the new pair is (a, min(lm2, b)), where
                    // b = med3(lm, k0, k1) and a = min3(lm, k0, k1) (every
                    // other key seen is >= lm2); 9 VALU operations per 4 keys
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) {
                        uint32_t mm = lm[nb], mm2 = lm2[nb];
#pragma unroll
                        for (int i = 0; i < 16; i += 4) {
                            uint32_t key[4];
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                key[q] = (__float_as_uint(acc[nb][i + q]) & ~ibm) | (uint32_t)(tt * 32 + 8 * (i >> 2) + q);
                            const uint32_t t1 = med3_u32(mm, key[0], key[1]);
                            const uint32_t l1 = min(min(mm, key[0]), key[1]);
                            const uint32_t t2 = med3_u32(l1, key[2], key[3]);
                            mm = min(min(l1, key[2]), key[3]);
                            mm2 = min(min(mm2, t1), t2);
                        }
                        lm[nb] = mm;
                        lm2[nb] = mm2;
                    }
                    continue;
                }
                if constexpr (STAGE == 3) {
                    // list every key inside the known band; more than CAP of
                    // them leaves the sample to a full rescan
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) {
                        uint32_t* lst = mycand + nb * SLOTS * 64 + lane;
#pragma unroll
                        for (int half = 0; half < 2; ++half) {
#pragma unroll
                            for (int i = 8 * half; i < 8 * half + 8; ++i) {
                                const uint32_t key = (__float_as_uint(acc[nb][i]) & ~ibm) | (j0 + 8 * (i >> 2) + (i & 3));
                                if (key <= tfix[nb]) { lst[cnt[nb] * 64] = key; ++cnt[nb]; }
                            }
                            if (cnt[nb] > CAP) { ovf[nb] = 1; cnt[nb] = CAP; }
                        }
                    }
                    continue;
                }
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
                    const uint32_t th = thr_key(mm, W[nb], ibm);
                    thr[nb] = th;
                    uint32_t* lst = mycand + nb * SLOTS * 64 + lane;
                    const uint32_t lim = min(th, cut[nb] - 1u);
#pragma unroll
                    for (int half = 0; half < 2; ++half) {
#pragma unroll
                        for (int i = 8 * half; i < 8 * half + 8; ++i) {
                            if (key[i] <= lim) { lst[cnt[nb] * 64] = key[i]; ++cnt[nb]; }
                        }
                        if (cnt[nb] > CAP) {
                            // drop entries the (only decreasing) threshold has passed
                            int w = 0;
                            uint32_t vmax = 0;
                            for (int q = 0; q < cnt[nb]; ++q) {
                                const uint32_t v = lst[q * 64];
                                if (v <= th) { lst[w * 64] = v; ++w; vmax = max(vmax, v); }
                            }
                            // still full: halve the window above the running
                            // minimum; what falls out lowers the cut
                            while (w > CAP) {
                                const float lo = __uint_as_float(mm & ~ibm);
                                const float hi = __uint_as_float(vmax & ~ibm);
                                const uint32_t mid = (__float_as_uint(0.5f * lo + 0.5f * hi) & ~ibm) | ibm;
                                int w2 = 0;
                                uint32_t vm2 = 0;
                                for (int q = 0; q < w; ++q) {
                                    const uint32_t v = lst[q * 64];
                                    if (v <= mid) { lst[w2 * 64] = v; ++w2; vm2 = max(vm2, v); }
                                    else cut[nb] = min(cut[nb], v);
                                }
                                if (w2 == w) { ovf[nb] = 1; w = CAP; break; }
                                w = w2;
                                vmax = vm2;
                            }
                            cnt[nb] = w;
                        }
                    }
                }
            }
            if constexpr (SCREEN) {
                // index bits of the chunk (c * 64) and of the lane's rows (4h)
                // are clear in the chunk-local keys (kpad >= 64)
                const uint32_t J = (uint32_t)(c * kMixCK) | (4u * (uint32_t)h);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const uint32_t a1 = lm[nb] | J, a2 = lm2[nb] | J;
                    m2[nb] = min(min(m2[nb], a2), max(m[nb], a1));
                    m[nb] = min(m[nb], a1);
                }
            }
            if (pref) {
                KM_STORE_PART(cur ^ 1, NTT - 1)
                __syncthreads();     // next buffer complete; this one no longer read
                cur ^= 1;
            }
        }

        if constexpr (SCREEN) {
            // decide per sample: the second key outside the band leaves one
            // candidate; otherwise list the sample for the refining sweep
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const uint32_t mo = (uint32_t)__shfl_xor((int)m[nb], 32);
                const uint32_t mo2 = (uint32_t)__shfl_xor((int)m2[nb], 32);
                const uint32_t mp = min(m[nb], mo);
                const uint32_t mp2 = min(max(m[nb], mo), min(m2[nb], mo2));
                const uint32_t tf = thr_key(mp, W[nb], ibm);
                const int64_t p = pidx[nb];
                const bool valid = p < n;
                const bool unique = mp2 > tf && (int)(mp & ibm) < a.k;
                if (valid && unique && h == 0) {
                    const int lab = (int)(mp & ibm);
                    if (a.count_changed) changed += (a.iter == 0) ? 1 : (a.labels[p] != lab);
                    a.labels[p] = lab;
                }
                const uint64_t need = __ballot(valid && !unique && h == 0);
                if (need) {
                    int base = 0;
                    if (lane == 0) base = atomicAdd(&blk_count, (int)__popcll(need));
                    base = __shfl(base, 0);
                    if (valid && !unique && h == 0) {
                        const size_t at = (size_t)region * a.rq_per_block + base + (int)__popcll(need & ((1ull << col) - 1ull));
                        a.amb[at] = (int32_t)p;
                        if (a.amb_key != nullptr) a.amb_key[at] = mp;
                    }
                }
            }
            continue;
        }
        // --- decide per sample: unique candidate, or queue an exact recheck
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const uint32_t mp = STAGE == 3 ? mfix[nb] : min(m[nb], (uint32_t)__shfl_xor((int)m[nb], 32));
            const uint32_t tf = STAGE == 3 ? tfix[nb] : thr_key(mp, W[nb], ibm);
            int vc = 0;
            uint32_t lmin = 0xffffffffu;
            const int stored = cnt[nb];
            for (int q = 0; q < stored; ++q) {
                const uint32_t v = mycand[(nb * SLOTS + q) * 64 + lane];
                vc += (v <= tf);
                lmin = min(lmin, v);
            }
            const int vc_other = __shfl_xor(vc, 32);
            // a dropped key inside the final band: the list is incomplete
            int ovf_h = ovf[nb] | (cut[nb] <= tf ? 1 : 0);
            // stage 3 takes its band from the screen: the listed minimum must be
            // the screen's key exactly, else the sample is rescanned in full
            if constexpr (STAGE == 3) ovf_h |= min(lmin, (uint32_t)__shfl_xor((int)lmin, 32)) != mp ? 1 : 0;
            const int ovf_any = ovf_h | __shfl_xor(ovf_h, 32);
            const int64_t p = pidx[nb];
            const bool valid = p < n;
            // a winner index outside [0, k) can only come from non-finite keys: rescan
            const bool unique = !ovf_any && (vc + vc_other) == 1 && (int)(mp & ibm) < a.k;
            if (valid && unique && h == 0) {
                const int lab = (int)(mp & ibm);
                if (a.count_changed) changed += (a.iter == 0) ? 1 : (a.labels[p] != lab);
                a.labels[p] = lab;
            }
            // queue slots in this block's region: one LDS atomic per wave; lanes
            // l and l+32 share sample l's slot
            const uint64_t need = __ballot(valid && !unique && h == 0);
            int slot = 0;
            if (need) {
                int base = 0;
                if (lane == 0) base = atomicAdd(&blk_count, (int)__popcll(need));
                base = __shfl(base, 0);
                slot = base + (int)__popcll(need & ((1ull << col) - 1ull));
            }
            const int base0 = __shfl(vc, col);  // candidates of the lower half come first
            if (valid && !unique) {
                int32_t* ent = rq_blk + (size_t)slot * RQI;
                if (h == 0) {
                    const bool full = ovf_any || (int)(mp & ibm) >= a.k;
                    ent[0] = (int32_t)p;
                    ent[1] = full ? -1 : (vc + vc_other);
                    if (full) atomicAdd(&blk_full, 1);
                }
                if (!ovf_any && (int)(mp & ibm) < a.k) {
                    int w = kRqHead + (h ? base0 : 0);
                    for (int q = 0; q < stored; ++q) {
                        const uint32_t kq = mycand[(nb * SLOTS + q) * 64 + lane];
                        if (kq <= tf) ent[w++] = (int32_t)(kq & ibm);
                    }
                }
            }
        }
    }

#undef KM_LOAD_CHUNK
#undef KM_STORE_CHUNK
#undef KM_LOAD_PART
#undef KM_STORE_PART
    // changed-label partial of this block (fixed order)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) changed += __shfl_xor(changed, off);
    if (lane == 0) sred[wave] = changed;
    __syncthreads();
    if (tid == 0) {
        int32_t c = 0;
        for (int w = 0; w < NW; ++w) c += sred[w];
        a.changed_part[region] = c;
        if constexpr (SCREEN) {
            a.amb_count[region] = blk_count;
        } else {
            a.rq_count[region] = blk_count;
            a.rq_count[a.nreg + region] = blk_full;
        }
    }
}

// The screen is built for three resident waves per SIMD (its 64 samples per
// wave hold 64 VGPRs of operands for the whole sweep); the refine after a
// BF16 screen fits four (128 VGPRs at 128 features).
template <int D16, int FMT, int STAGE, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(STAGE == 1 || STAGE == 2 ? 3 : STAGE == 3 ? 4 : 1)))
void mfma_assign(MixArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    if constexpr (STAGE >= 2)
        mfma_body<D16, FMT, STAGE, NW>(a, 0, INT64_MAX, 1, blockIdx.x, smem);   // block b takes region b's list
    else
        mfma_body<D16, FMT, STAGE, NW>(a, blockIdx.x, INT64_MAX, gridDim.x, blockIdx.x, smem);
}

// Batched instances (BF16): row b of the work table runs tiles [t0, t1) of
// instance work[b].inst into its queue region work[b].slot.
template <int D16>
__global__ __launch_bounds__(64 * kMixWaves) void batch_mfma(const BatchWork* __restrict__ work,
                                                             const BatchMix* __restrict__ bm, int32_t iter)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const BatchWork w = work[blockIdx.x];
    MixArgs a = bm[w.inst].m;
    a.iter = iter;
    mfma_body<D16, FMT_BF16, 0, kMixWaves>(a, w.t0, w.t1, 1, w.slot, smem);
}

// ------------------------------------------------------------ exact recheck
// A group of GS lanes (GS = the chunk count rounded up to a power of two)
// evaluates one queued sample: lane q of the group owns features 8q..8q+7, so
// sample and centroid rows are read as contiguous 32-byte pieces.  Lane q
// accumulates chunk q exactly as the FP32 path does (fused multiply-add from
// 0 over its 8 features) and the chunk partials are added by the same
// pairwise tree (chunk p += chunk p+s) through lane shuffles, so every
// distance is bit-identical to the FP32 path's.  The winner is the
// lexicographic (distance, index) minimum over the candidates; entries
// flagged -1 scan all k centroids in index order.
// One level of the canonical pairwise tree over the lanes of a sample (lane
// q holds chunk q's partial): lanes q with q % 2S == 0 and q + S < D8 add the
// partial of lane q + S, fetched with a DPP row shift.
template <int S, int D8>
__device__ __forceinline__ void tree_level(float& part, int q)
{
    if constexpr (S < D8) {
        const float other = __builtin_bit_cast(
            float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, part), 0x100 + S, 0xf, 0xf, false));
        if ((q % (2 * S)) == 0 && q + S < D8) part = part + other;
    }
}

template <int D8>
__device__ __forceinline__ void recheck_body(const RecheckArgs& a, int region, int y, int ny)
{
    constexpr int D = 8 * D8;
    constexpr int GS = D8 <= 1 ? 1 : D8 <= 2 ? 2 : D8 <= 4 ? 4 : D8 <= 8 ? 8 : 16;
    constexpr int GPW = 64 / GS;
    __shared__ int32_t sred[4];
    if (a.ctrl != nullptr && a.ctrl->stop_iter < a.iter) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int q = lane % GS;
    const int grp = lane / GS;
    // ny blocks re-check the entries of one queue region, block y taking
    // every ny-th group of waves
    const int count = a.rq_count[region];
    const int32_t* rq_blk = a.rq + (size_t)region * a.rq_per_block * a.rq_ints;
    const int wave_id = y * 4 + (tid >> 6);
    const int nwaves = ny * 4;
    int32_t changed = 0;
    for (int e0 = wave_id * GPW; e0 < count; e0 += nwaves * GPW) {
        const int e = e0 + grp;
        const bool valid = e < count;
        const int32_t* ent = rq_blk + (size_t)(valid ? e : e0) * a.rq_ints;   // entry e0 < count exists
        const int64_t p = ent[0];
        const int nc = valid ? ent[1] : 0;
        // Every load below is unconditional with a clamped address (a valid
        // row, feature or list slot) and its value is masked afterwards, so
        // the loads of a batch are all in flight together.
        const int qc = q < D8 ? q : D8 - 1;
        float x[8];
        {
            const float* xr = a.X + p * a.d;
            if ((a.d & 7) == 0) {
                // every lane's eight features lie inside the row: two vector loads
                const float4 v0 = *reinterpret_cast<const float4*>(xr + 8 * qc);
                const float4 v1 = *reinterpret_cast<const float4*>(xr + 8 * qc + 4);
                const bool in = q < D8;
                x[0] = in ? v0.x : 0.0f; x[1] = in ? v0.y : 0.0f; x[2] = in ? v0.z : 0.0f; x[3] = in ? v0.w : 0.0f;
                x[4] = in ? v1.x : 0.0f; x[5] = in ? v1.y : 0.0f; x[6] = in ? v1.z : 0.0f; x[7] = in ? v1.w : 0.0f;
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int f = 8 * qc + i;
                    const float v = xr[f < a.d ? f : a.d - 1];
                    x[i] = (q < D8 && f < a.d) ? v : 0.0f;
                }
            }
        }
        // trip count: the longest candidate list of the wave
        int trips = !valid ? 0 : (nc < 0 ? a.k : nc);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) trips = max(trips, __shfl_xor(trips, off));
        float best = __builtin_huge_valf();
        int bj = 0;
        // candidates in flight per group: most lists hold two or three, and
        // four (against eight) measured 20-24% faster: fewer registers, more
        // resident waves, less work on empty slots
        constexpr int TB = 4;
        const int lastbatch = a.rq_ints - kRqHead - TB;   // the list holds a multiple of TB slots
        for (int t0 = 0; t0 < trips; t0 += TB) {
            int jj[TB];
            {
                const int4* lp = reinterpret_cast<const int4*>(ent + kRqHead + (t0 < lastbatch ? t0 : lastbatch));
                int listed[TB];
#pragma unroll
                for (int v = 0; v < TB / 4; ++v) {
                    const int4 l = lp[v];
                    listed[4 * v] = l.x; listed[4 * v + 1] = l.y; listed[4 * v + 2] = l.z; listed[4 * v + 3] = l.w;
                }
#pragma unroll
                for (int u = 0; u < TB; ++u) {
                    const int t = t0 + u;
                    const int j = (nc < 0) ? t : (t < nc ? listed[u] : -1);
                    jj[u] = (valid && j >= 0 && j < a.k && (nc >= 0 || t < a.k)) ? j : -1;
                }
            }
            float cv[TB][8];
#pragma unroll
            for (int u = 0; u < TB; ++u) {
                const float4* cr = reinterpret_cast<const float4*>(a.Cp + (size_t)(jj[u] >= 0 ? jj[u] : 0) * D + 8 * qc);
                const float4 c0 = cr[0], c1 = cr[1];
                cv[u][0] = c0.x; cv[u][1] = c0.y; cv[u][2] = c0.z; cv[u][3] = c0.w;
                cv[u][4] = c1.x; cv[u][5] = c1.y; cv[u][6] = c1.z; cv[u][7] = c1.w;
            }
#pragma unroll
            for (int u = 0; u < TB; ++u) {
                float part = 0.0f;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const float df = x[i] - (q < D8 ? cv[u][i] : 0.0f);
                    part = __builtin_fmaf(df, df, part);
                }
                // the chunk partials' pairwise tree across the sample's lanes
                // (lane q adds lane q + s; DPP row shifts stay inside a
                // 16-lane row, which holds whole samples); the distance is
                // complete in the sample's first lane, the only one that uses it
                tree_level<1, D8>(part, q);
                tree_level<2, D8>(part, q);
                tree_level<4, D8>(part, q);
                tree_level<8, D8>(part, q);
                const float dist = part;
                const int j = jj[u];
                if (j >= 0 && (dist < best || (dist == best && j < bj))) { best = dist; bj = j; }
            }
        }
        if (valid && q == 0) {
            if (a.count_changed) changed += (a.iter == 0) ? 1 : (a.labels[p] != bj);
            a.labels[p] = bj;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) changed += __shfl_xor(changed, off);
    if ((tid & 63) == 0) sred[tid >> 6] = changed;
    __syncthreads();
    if (tid == 0) a.changed_part[y * a.nreg + region] = sred[0] + sred[1] + sred[2] + sred[3];
}

template <int D8>
__global__ __launch_bounds__(256) void recheck_kernel(RecheckArgs a)
{
    recheck_body<D8>(a, blockIdx.x, blockIdx.y, gridDim.y);
}

// Batched: row b of the work table re-checks region work[b].slot of instance
// work[b].inst as split t0 of t1.
template <int D8>
__global__ __launch_bounds__(256) void batch_recheck(const BatchWork* __restrict__ work,
                                                     const BatchMix* __restrict__ bm, int32_t iter)
{
    const BatchWork w = work[blockIdx.x];
    RecheckArgs a = bm[w.inst].r;
    a.iter = iter;
    recheck_body<D8>(a, w.slot, (int)w.t0, (int)w.t1);
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

hipError_t launch_prep_x_bf16(const float* X, int64_t n, int32_t d, int32_t DP, __bf16* Xb, float* xn, hipStream_t s)
{
    const int64_t threads = n * row_lanes_q(DP);
    hipLaunchKernelGGL(quant_x_bf16_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, X, n, d, DP, Xb,
                       xn);
    return hipGetLastError();
}

hipError_t launch_prep_x_fp8(const float* X, int64_t n, int32_t d, int32_t DP, float* part_fmax, float* fscale,
                             uint8_t* Xq, float2* xst, hipStream_t s)
{
    hipLaunchKernelGGL(prep_fmax_kernel, dim3(kFmaxBlocks), dim3(256), 0, s, X, n, d, DP, part_fmax);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(prep_fscale_kernel, dim3(1), dim3(256), 0, s, part_fmax, kFmaxBlocks, d, DP, fscale);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t threads = n * row_lanes_q(DP);
    hipLaunchKernelGGL(quant_x_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, X, n, d, DP, fscale,
                       Xq, xst);
    return hipGetLastError();
}

int prep_c_blocks(int kpad) { return (kpad + kPrepRows - 1) / kPrepRows; }

hipError_t launch_prep_c(int fmt, const float* Cp, int32_t k, int32_t d, int32_t D, int32_t kpad, int32_t DP,
                         const XStats* xs, const float* fscale, void* Ab, float* bias, CStats* cs, float* part_cn2,
                         const Ctrl* ctrl, int32_t iter, hipStream_t s)
{
    if (fmt == FMT_BF16 && part_cn2 != nullptr) {
        const int nb = prep_c_blocks(kpad);
        hipLaunchKernelGGL(prep_c_rows_kernel, dim3(nb), dim3(256), 0, s, Cp, k, d, D, kpad, DP, xs,
                           static_cast<__bf16*>(Ab), bias, part_cn2, ctrl, iter);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(prep_c_stats_kernel, dim3(1), dim3(64), 0, s, part_cn2, nb, d, xs, cs, ctrl, iter);
        return hipGetLastError();
    }
    if (fmt == FMT_FP8)
        hipLaunchKernelGGL(prep_c_fp8_kernel, dim3(1), dim3(256), 0, s, Cp, k, d, D, kpad, DP, xs, fscale,
                           static_cast<uint8_t*>(Ab), bias, cs, ctrl, iter);
    else
        hipLaunchKernelGGL(prep_c_kernel, dim3(1), dim3(256), 0, s, Cp, k, d, D, kpad, DP, xs,
                           static_cast<__bf16*>(Ab), bias, cs, ctrl, iter);
    return hipGetLastError();
}

static size_t mix_row_bytes(int fmt, int D16) { return (size_t)D16 * 16 * (fmt == FMT_FP8 ? 1 : 2) + 16; }

int mix_buffers(int fmt, int D16, int kpad)
{
    const int nch = kpad / kMixCK;
    if (D16 <= 0 || nch < 3) return 2;
    return (size_t)nch * kMixCK * mix_row_bytes(fmt, D16) <= (size_t)kMixResidentBytes ? nch : 2;
}

size_t mfma_lds_bytes(int fmt, int D16, int stage, int nbuf, int waves)
{
    // (D16 = 0, rows of more than 128 features: the centroid operands are not staged)
    const size_t nb = (size_t)(D16 > 0 && nbuf > 2 ? nbuf : 2);
    return nb * kMixCK * mix_row_bytes(fmt, D16) + nb * kMixCK * sizeof(float) +
           (stage == 1 || stage == 2 ? 0 : (size_t)waves * mix_nb(stage) * kCandSlots * 64 * sizeof(uint32_t));
}

template <int D16, int FMT, int STAGE, int NW>
static hipError_t launch_mfma_d16(const MixArgs& a, int grid, hipStream_t s)
{
    const size_t lds = mfma_lds_bytes(FMT, D16, STAGE, a.nbuf, NW);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&mfma_assign<D16, FMT, STAGE, NW>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((mfma_assign<D16, FMT, STAGE, NW>), dim3(grid), dim3(64 * NW), lds, s, a);
    return hipGetLastError();
}

// (blocks of more than kMixWaves waves only for rows of at most 128 features)
template <int FMT, int STAGE, int NW>
static hipError_t launch_mfma_fs(int D16, const MixArgs& a, int grid, hipStream_t s)
{
    switch (D16) {
    case 1: return launch_mfma_d16<1, FMT, STAGE, NW>(a, grid, s);
    case 2: return launch_mfma_d16<2, FMT, STAGE, NW>(a, grid, s);
    case 3: return launch_mfma_d16<3, FMT, STAGE, NW>(a, grid, s);
    case 4: return launch_mfma_d16<4, FMT, STAGE, NW>(a, grid, s);
    case 5: return launch_mfma_d16<5, FMT, STAGE, NW>(a, grid, s);
    case 6: return launch_mfma_d16<6, FMT, STAGE, NW>(a, grid, s);
    case 7: return launch_mfma_d16<7, FMT, STAGE, NW>(a, grid, s);
    case 8: return launch_mfma_d16<8, FMT, STAGE, NW>(a, grid, s);
    default:
        if constexpr (NW == kMixWaves)
            return D16 <= kMaxD16Wide ? launch_mfma_d16<0, FMT, STAGE, NW>(a, grid, s) : hipErrorInvalidValue;
        else
            return hipErrorInvalidValue;
    }
}

template <int FMT, int STAGE>
static hipError_t launch_mfma_nw(int D16, const MixArgs& a, int grid, hipStream_t s)
{
    if constexpr (STAGE >= 1) {
        if (a.wide_blocks) return launch_mfma_fs<FMT, STAGE, mix_waves(STAGE, true)>(D16, a, grid, s);
    }
    return launch_mfma_fs<FMT, STAGE, kMixWaves>(D16, a, grid, s);
}

// The single-instance passes: BF16 and FP8 screens (stage 1), the BF16 screen
// of the FP8 screen's open samples (stage 2), the BF16 refine after a BF16
// screen (stage 3), the BF16 one-pass sweep (stage 0).
hipError_t launch_mfma_assign(int fmt, int stage, int D16, const MixArgs& a, int grid, hipStream_t s)
{
    if (stage == 1) return fmt == FMT_FP8 ? launch_mfma_nw<FMT_FP8, 1>(D16, a, grid, s)
                                          : launch_mfma_nw<FMT_BF16, 1>(D16, a, grid, s);
    if (stage == 2 && fmt == FMT_BF16) return launch_mfma_nw<FMT_BF16, 2>(D16, a, grid, s);
    if (stage == 3 && fmt == FMT_BF16) return launch_mfma_nw<FMT_BF16, 3>(D16, a, grid, s);
    if (stage == 0 && fmt == FMT_BF16) return launch_mfma_nw<FMT_BF16, 0>(D16, a, grid, s);
    return hipErrorInvalidValue;
}

template <int D16, int FMT, int STAGE, int NW>
static int occ_mfma(int nbuf)
{
    const size_t lds = mfma_lds_bytes(FMT, D16, STAGE, nbuf, NW);
    if (lds > 64 * 1024 &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(&mfma_assign<D16, FMT, STAGE, NW>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return -1;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, mfma_assign<D16, FMT, STAGE, NW>, 64 * NW, lds) !=
        hipSuccess)
        return -1;
    return nb;
}

template <int FMT, int STAGE, int NW>
static int occ_mfma_fs(int D16, int nbuf)
{
    switch (D16) {
    case 1: return occ_mfma<1, FMT, STAGE, NW>(nbuf);
    case 2: return occ_mfma<2, FMT, STAGE, NW>(nbuf);
    case 3: return occ_mfma<3, FMT, STAGE, NW>(nbuf);
    case 4: return occ_mfma<4, FMT, STAGE, NW>(nbuf);
    case 5: return occ_mfma<5, FMT, STAGE, NW>(nbuf);
    case 6: return occ_mfma<6, FMT, STAGE, NW>(nbuf);
    case 7: return occ_mfma<7, FMT, STAGE, NW>(nbuf);
    case 8: return occ_mfma<8, FMT, STAGE, NW>(nbuf);
    default:
        if constexpr (NW == kMixWaves)
            return D16 <= kMaxD16Wide ? occ_mfma<0, FMT, STAGE, NW>(nbuf) : -1;
        else
            return -1;
    }
}

template <int FMT, int STAGE>
static int occ_mfma_nw(int D16, int nbuf, bool wide_blocks)
{
    if constexpr (STAGE >= 1) {
        if (wide_blocks) return occ_mfma_fs<FMT, STAGE, mix_waves(STAGE, true)>(D16, nbuf);
    }
    return occ_mfma_fs<FMT, STAGE, kMixWaves>(D16, nbuf);
}

int mfma_blocks_per_cu(int fmt, int stage, int D16, int nbuf, bool wide_blocks)
{
    if (stage == 1) return fmt == FMT_FP8 ? occ_mfma_nw<FMT_FP8, 1>(D16, nbuf, wide_blocks)
                                          : occ_mfma_nw<FMT_BF16, 1>(D16, nbuf, wide_blocks);
    if (stage == 2 && fmt == FMT_BF16) return occ_mfma_nw<FMT_BF16, 2>(D16, nbuf, wide_blocks);
    if (stage == 3 && fmt == FMT_BF16) return occ_mfma_nw<FMT_BF16, 3>(D16, nbuf, wide_blocks);
    if (stage == 0 && fmt == FMT_BF16) return occ_mfma_nw<FMT_BF16, 0>(D16, nbuf, false);
    return -1;
}

hipError_t launch_batch_prep_x(const BatchWork* xwork, int nxwork, const BatchMix* bm, int ninst, hipStream_t s)
{
    hipLaunchKernelGGL(batch_prep_x_kernel, dim3(nxwork), dim3(256), 0, s, xwork, bm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batch_prep_x_combine_kernel, dim3(ninst), dim3(64), 0, s, bm);
    return hipGetLastError();
}

hipError_t launch_batch_prep_c(const BatchMix* bm, int ninst, hipStream_t s)
{
    hipLaunchKernelGGL(batch_prep_c_kernel, dim3(ninst), dim3(256), 0, s, bm);
    return hipGetLastError();
}

template <int D16>
static hipError_t launch_batch_mfma_d16(const BatchWork* work, int nwork, const BatchMix* bm, int iter, hipStream_t s)
{
    const size_t lds = mfma_lds_bytes(FMT_BF16, D16, 0);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&batch_mfma<D16>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((batch_mfma<D16>), dim3(nwork), dim3(64 * kMixWaves), lds, s, work, bm, iter);
    return hipGetLastError();
}

hipError_t launch_batch_mfma(int D16, const BatchWork* work, int nwork, const BatchMix* bm, int iter, hipStream_t s)
{
    switch (D16) {
    case 1: return launch_batch_mfma_d16<1>(work, nwork, bm, iter, s);
    case 2: return launch_batch_mfma_d16<2>(work, nwork, bm, iter, s);
    case 3: return launch_batch_mfma_d16<3>(work, nwork, bm, iter, s);
    case 4: return launch_batch_mfma_d16<4>(work, nwork, bm, iter, s);
    case 5: return launch_batch_mfma_d16<5>(work, nwork, bm, iter, s);
    case 6: return launch_batch_mfma_d16<6>(work, nwork, bm, iter, s);
    case 7: return launch_batch_mfma_d16<7>(work, nwork, bm, iter, s);
    case 8: return launch_batch_mfma_d16<8>(work, nwork, bm, iter, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_recheck(int D8, const BatchWork* work, int nwork, const BatchMix* bm, int iter, hipStream_t s)
{
    switch (D8) {
#define KM_BRC(N) case N: hipLaunchKernelGGL((batch_recheck<N>), dim3(nwork), dim3(256), 0, s, work, bm, iter); break;
    KM_BRC(1) KM_BRC(2) KM_BRC(3) KM_BRC(4) KM_BRC(5) KM_BRC(6) KM_BRC(7) KM_BRC(8)
    KM_BRC(9) KM_BRC(10) KM_BRC(11) KM_BRC(12) KM_BRC(13) KM_BRC(14) KM_BRC(15) KM_BRC(16)
#undef KM_BRC
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_recheck(int D8, const RecheckArgs& a, int grid, int split, hipStream_t s)
{
    switch (D8) {
#define KM_RC(N) case N: hipLaunchKernelGGL((recheck_kernel<N>), dim3(grid, split), dim3(256), 0, s, a); break;
    KM_RC(1) KM_RC(2) KM_RC(3) KM_RC(4) KM_RC(5) KM_RC(6) KM_RC(7) KM_RC(8)
    KM_RC(9) KM_RC(10) KM_RC(11) KM_RC(12) KM_RC(13) KM_RC(14) KM_RC(15) KM_RC(16)
#undef KM_RC
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace km
