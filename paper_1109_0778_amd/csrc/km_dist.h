// The canonical FP32 squared distance, shared by every kernel that must
// reproduce the plain path's distances bit for bit (the plain per-sample pass
// and the exact recheck of the mixed-precision path).
#pragma once

#include "km_internal.h"

namespace km {

// Centroid rows read by the plain pass go through the constant address space:
// every lane of a wave reads the same row, so the loads become scalar (SMEM)
// loads and the values enter the VALU as SGPR operands.
typedef __attribute__((address_space(4))) const float cfloat;

template <int D8>
__device__ __forceinline__ void load_row(const float* __restrict__ row, int d, bool valid, float (&x)[8 * D8])
{
    constexpr int D = 8 * D8;
    if (valid && (d & 3) == 0) {
#pragma unroll
        for (int q = 0; q < D / 4; ++q) {
            if (4 * q < d) {
                const float4 v = *reinterpret_cast<const float4*>(row + 4 * q);
                x[4 * q + 0] = v.x; x[4 * q + 1] = v.y; x[4 * q + 2] = v.z; x[4 * q + 3] = v.w;
            } else {
                x[4 * q + 0] = 0.f; x[4 * q + 1] = 0.f; x[4 * q + 2] = 0.f; x[4 * q + 3] = 0.f;
            }
        }
    } else {
#pragma unroll
        for (int f = 0; f < D; ++f) x[f] = (valid && f < d) ? row[f] : 0.0f;
    }
}

// Canonical FP32 squared distance of R sample rows to one centroid row:
// diff = fl(x - c); features in chunks of 8 accumulated with fused
// multiply-add starting from 0; chunk partials summed by the pairwise tree
// (p += p + s for s = 1, 2, 4, ...).  Zero padding adds exact zeros and does
// not change the value.  Error <= (2 + 8 + ceil(log2 P)) units of 2^-24 of
// the exact distance (P = number of chunks).  The centroid pointer type picks
// the load path (scalar for wave-uniform rows, vector otherwise); the
// arithmetic is the same sequence of IEEE operations either way.
template <int D8, int R, typename CP>
__device__ __forceinline__ void dist_rows(const float (&x)[R][8 * D8], CP c, float (&out)[R])
{
    float part[R][D8];
#pragma unroll
    for (int p = 0; p < D8; ++p) {
#pragma unroll
        for (int r = 0; r < R; ++r) part[r][p] = 0.0f;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float cv = c[8 * p + q];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float df = x[r][8 * p + q] - cv;
                part[r][p] = __builtin_fmaf(df, df, part[r][p]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int s = 1; s < D8; s *= 2) {
#pragma unroll
            for (int p = 0; p + s < D8; p += 2 * s) part[r][p] = part[r][p] + part[r][p + s];
        }
        out[r] = part[r][0];
    }
}

}  // namespace km
