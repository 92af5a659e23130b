// SPADE density step on gfx950 (paper section 4.1, "Downsampling in
// Bioinformatics"): rows of the all-pairs distance matrix are visited in
// increasing index order; a visited row counts the samples within the kernel
// width (or the approximation width) and hands that count to every sample
// within the approximation width whose density is still unset; a row whose
// density is already set is skipped (its distances are never formed).
//
// The order dependence is kept exactly, with the rows processed in
// speculative batches, one launch per batch b (256 samples per block):
//   claims  every undecided sample takes the count of the first visited
//           candidate of batch b-1 that has it within the approximation
//           width; visited candidates take their own count;
//   rows    every sample j against every candidate c of batch b: the
//           distance in FP64 with the features in increasing order (the same
//           IEEE operations as a sequential loop, so every threshold decision
//           is exact), the count of c (wave ballots, block LDS counters, one
//           atomic per block and candidate) and the bit "j within the
//           approximation width of c" (a 256-bit mask per sample);
//   tail    the block that finishes last (a ticket after a device-scope
//           fence) resolves batch b in candidate order from the candidates'
//           own masks (c is visited unless a visited candidate before it has
//           it within the approximation width) and selects batch b+1: the
//           next undecided rows in index order, where a row is undecided
//           when no earlier batch claimed it and no visited candidate of
//           batch b covers it; their rows are widened to FP64.
// Batch data (candidates, counts, rows, visited mask) alternate between two
// buffers, so the claims of batch b-1 and the rows of batch b share a launch.
// A candidate that an earlier one in its batch claims is wasted work (its row
// was formed speculatively); the batch size adapts to the previous batch's
// visited count.  Integer counts and first-writer claims are independent of
// scheduling, so densities are deterministic.
#include "kmeans_mi355x.h"
#include "km_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdarg>
#include <cstdio>

km_status km_set_error(km_status st, const char* msg);

namespace km {
namespace {

constexpr int kSpB = 256;               // most candidates per batch
constexpr int kSpW = kSpB / 64;         // 64-bit words of a sample's candidate mask
constexpr int kSpBMin = 32;             // fewest candidates per batch (while rows remain)
constexpr int kSpMaxD8Reg = 8;          // d <= 64: the sample row lives in registers
constexpr int kSpCG = 8;                // wide rows: candidates per pass over a sample row
constexpr int kSpSelThreads = 1024;     // the first batch's selection block
// Samples per lane: rows of at most 32 features take two (each candidate
// operand read from LDS then feeds two samples' FP64 chains), wider rows one.
__host__ __device__ constexpr int sp_rows(int D8) { return D8 > 0 && D8 <= 4 ? 2 : 1; }

struct SpadeCtrl {
    int64_t cursor;       // every row below is decided or a candidate of the current batch
    int32_t batch;        // index of the batch the next launch processes
    int32_t nc[2];        // candidates per buffer
    int32_t final_;       // no batch left: the next launch applies the last claims
    int32_t done;         // every density is set
    uint32_t ticket;      // blocks of the running launch that have finished
    int32_t last_visited; // visited candidates of the last resolved batch
    int32_t pad0;
    int64_t visited;      // visited rows so far
    int64_t batches;
    int64_t candidates;   // candidate rows formed (visited + speculative)
    uint64_t vis[2][kSpW];// visited candidates per buffer
    int64_t pad[3];
};
static_assert(sizeof(SpadeCtrl) <= 256, "control block must fit 256 bytes");

struct SpadeArgs {
    const float* X;
    int64_t n;
    int32_t d, DP;        // DP = d rounded up to 8 (candidate rows zero padded)
    double apprx, kern;   // approximation and kernel widths
    SpadeCtrl* ctrl;
    int32_t* owner;       // [n] row whose count a sample took (INT_MAX: undecided)
    int32_t* cand;        // [2][kSpB] candidate rows of a batch, increasing
    int32_t* cnt;         // [2][kSpB] count of each candidate
    double* crow;         // [2][kSpB][DP] candidate rows in FP64
    uint64_t* near;       // [n][kSpW] bit c of sample j: d(cand c, j) < apprx (the last batch formed)
    int32_t* dens;        // [n] output densities
    int8_t* visited;      // [n] output visited flags, or nullptr
};

typedef __attribute__((address_space(4))) const double cdouble;

__global__ __launch_bounds__(256) void spade_init_kernel(SpadeArgs a)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        a.owner[i] = INT_MAX;
        a.dens[i] = 0;
        if (a.visited) a.visited[i] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        SpadeCtrl c{};
        *a.ctrl = c;
    }
}

// The next B undecided rows in index order from the cursor, into buffer
// `buf`: a row is undecided when its owner is unset and (vis != nullptr) no
// candidate in `vis` covers it.  NT threads; wsum holds NT / 64 ints.
template <int NT>
__device__ void select_batch(const SpadeArgs& a, int buf, int B, const uint64_t* vis, int32_t* wsum,
                             int32_t* s_found)
{
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    int32_t* cand = a.cand + buf * kSpB;
    int64_t base = a.ctrl->cursor;
    int found = 0;
    // U chunks of NT rows per round, their owners and masks loaded before
    // any is ranked (the scan is on the critical path of every batch)
    constexpr int U = 4;
    while (found < B && base < a.n) {
        bool open[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = base + u * NT + tid;
            const int64_t ic = i < a.n ? i : a.n - 1;
            open[u] = i < a.n && a.owner[ic] == INT_MAX;
            if (vis != nullptr) {
                uint64_t m = 0ull;
#pragma unroll
                for (int w = 0; w < kSpW; ++w) m |= a.near[(size_t)ic * kSpW + w] & vis[w];
                open[u] = open[u] && m == 0ull;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = base + u * NT + tid;
            const uint64_t bal = __ballot(open[u]);
            const int below = __popcll(bal & ((1ull << lane) - 1ull));
            if (lane == 0) wsum[wave] = __popcll(bal);
            __syncthreads();
            int off = 0, tot = 0;
            for (int w = 0; w < NW; ++w) {
                const int c = wsum[w];
                off += w < wave ? c : 0;
                tot += c;
            }
            const int pos = found + off + below;
            if (open[u] && pos < B) cand[pos] = (int32_t)i;
            found += tot;
            __syncthreads();   // wsum is rewritten by the next chunk
        }
        base += U * NT;
    }
    if (tid == 0) *s_found = found;
    __syncthreads();
    const int nc = min(*s_found, B);
    if (tid == 0) {
        SpadeCtrl* c = a.ctrl;
        c->nc[buf] = nc;
        c->cursor = *s_found >= B ? (int64_t)cand[B - 1] + 1 : a.n;
        if (nc == 0) c->final_ = 1;
        c->batches += nc > 0 ? 1 : 0;
        c->candidates += nc;
    }
    int32_t* cnt = a.cnt + buf * kSpB;
    double* crow = a.crow + (size_t)buf * kSpB * a.DP;
    for (int c = tid; c < nc; c += NT) cnt[c] = 0;
    // candidate rows widened to FP64: eight loads in flight per thread
    const int total = nc * a.DP;
    for (int e0 = 0; e0 < total; e0 += 8 * NT) {
        float v[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int e = e0 + r * NT + tid;
            const int c = e / a.DP, f = e - c * a.DP;
            v[r] = (e < total && f < a.d) ? a.X[(size_t)cand[c] * a.d + f] : 0.0f;
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int e = e0 + r * NT + tid;
            if (e < total) crow[e] = (double)v[r];
        }
    }
}

// Batch 0: the first 64 rows (one block).
__global__ __launch_bounds__(kSpSelThreads) void spade_first_select_kernel(SpadeArgs a)
{
    __shared__ int32_t wsum[kSpSelThreads / 64];
    __shared__ int32_t s_found;
    select_batch<kSpSelThreads>(a, 0, 64, nullptr, wsum, &s_found);
}

// Count bookkeeping: ballot of "within either width" over the wave, one LDS
// atomic per wave and candidate.
__device__ __forceinline__ void count_within(bool within, int lane, int32_t* cnt_s, int c)
{
    const uint64_t b = __ballot(within);
    if (lane == 0 && b) atomicAdd(&cnt_s[c], (int32_t)__popcll(b));
}

// The rows of one batch against the block's samples.  D8 > 0: rows of at most
// 64 features held in registers (FP64), the candidate rows staged in LDS 64
// at a time (coalesced loads) and read back as wave-wide broadcasts, reads
// the compiler can issue ahead of the FP64 chain (whole rows of scalar
// operands could not be double-buffered in SGPRs); D8 == 0: rows streamed in
// chunks of 8 features, kSpCG candidates at a time, each sum still in
// feature order.
template <int D8, int METRIC>
__device__ __forceinline__ void batch_rows(const SpadeArgs& a, int buf, int nc, int64_t j0, int32_t* cnt_s,
                                           double* cs)
{
    const int tid = threadIdx.x, lane = tid & 63;
    const double apprx = a.apprx, kern = a.kern;
    if constexpr (D8 > 0) {
        constexpr int D = 8 * D8;
        constexpr int RR = sp_rows(D8);
        double x[RR][D];
        bool valid[RR];
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            const int64_t j = j0 + r * 256;
            valid[r] = j < a.n;
            const float* row = a.X + (valid[r] ? j : 0) * a.d;
#pragma unroll
            for (int f = 0; f < D; ++f) x[r][f] = (valid[r] && f < a.d) ? (double)row[f] : 0.0;
        }
        const double* cg = a.crow + (size_t)buf * kSpB * a.DP;
#pragma unroll
        for (int g = 0; g < kSpW; ++g) {
            const int c0 = g * 64;
            if (c0 >= nc) break;
            const int c1 = min(nc, c0 + 64);
            __syncthreads();                 // the previous chunk is no longer read
            for (int e = tid; e < (c1 - c0) * D; e += 256) cs[e] = cg[(size_t)c0 * D + e];
            __syncthreads();
            uint64_t word[RR];
#pragma unroll
            for (int r = 0; r < RR; ++r) word[r] = 0;
            for (int c = c0; c < c1; ++c) {
                const double* cr = cs + (c - c0) * D;
                double acc[RR];
#pragma unroll
                for (int r = 0; r < RR; ++r) acc[r] = 0.0;
#pragma unroll
                for (int f = 0; f < D; ++f) {
                    const double cv = cr[f];
#pragma unroll
                    for (int r = 0; r < RR; ++r) {
                        const double diff = cv - x[r][f];
                        if constexpr (METRIC == 0) acc[r] = acc[r] + __builtin_fabs(diff);
                        else acc[r] = acc[r] + diff * diff;
                    }
                }
                int within = 0;
#pragma unroll
                for (int r = 0; r < RR; ++r) {
                    const bool nr = acc[r] < apprx;
                    word[r] |= (uint64_t)nr << (c - c0);
                    within += (int)__popcll(__ballot(valid[r] && (nr || acc[r] < kern)));
                }
                if (lane == 0 && within) atomicAdd(&cnt_s[c], within);
            }
#pragma unroll
            for (int r = 0; r < RR; ++r)
                if (valid[r]) a.near[(size_t)(j0 + r * 256) * kSpW + g] = word[r];
        }
    } else {
        const int64_t j = j0;
        const bool valid = j < a.n;
        cdouble* crow = (cdouble*)(a.crow + (size_t)buf * kSpB * a.DP);
        const float* row = a.X + (valid ? j : 0) * a.d;
        const int d = a.d, DP = a.DP;
#pragma unroll
        for (int g = 0; g < kSpW; ++g) {
            const int c0 = g * 64;
            if (c0 >= nc) break;
            const int c1 = min(nc, c0 + 64);
            uint64_t word = 0;
            for (int cg = c0; cg < c1; cg += kSpCG) {
                double acc[kSpCG];
#pragma unroll
                for (int q = 0; q < kSpCG; ++q) acc[q] = 0.0;
                for (int f0 = 0; f0 < DP; f0 += 8) {
                    double x[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) x[i] = (valid && f0 + i < d) ? (double)row[f0 + i] : 0.0;
#pragma unroll
                    for (int q = 0; q < kSpCG; ++q) {
                        const int c = min(cg + q, c1 - 1);   // rows past the batch repeat the last (discarded)
                        cdouble* cr = crow + (size_t)c * DP + f0;
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            const double diff = cr[i] - x[i];
                            if constexpr (METRIC == 0) acc[q] = acc[q] + __builtin_fabs(diff);
                            else acc[q] = acc[q] + diff * diff;
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < kSpCG; ++q) {
                    const int c = cg + q;
                    if (c < c1) {
                        const bool nr = acc[q] < apprx;
                        word |= (uint64_t)nr << (c - c0);
                        count_within(valid && (nr || acc[q] < kern), lane, cnt_s, c);
                    }
                }
            }
            if (valid) a.near[(size_t)j * kSpW + g] = word;
        }
    }
}

// One batch per launch: claims of the previous batch, rows of this one, and
// (last block) its resolve and the next batch's selection.
template <int D8, int METRIC>
__global__ __launch_bounds__(256) void spade_batch_kernel(SpadeArgs a)
{
    __shared__ int32_t cnt_s[kSpB];
    __shared__ uint64_t cm[kSpB][kSpW];
    __shared__ double cs[64 * 8 * (D8 > 0 ? D8 : 1)];   // a chunk of candidate rows
    __shared__ uint64_t svis[kSpW];
    __shared__ int32_t wsum[4];
    __shared__ int32_t s_found;
    __shared__ int s_last;
    SpadeCtrl* ctrl = a.ctrl;
    if (ctrl->done) return;
    const int b = ctrl->batch;
    const int cur = b & 1, prev = cur ^ 1;
    const int nc = ctrl->final_ ? 0 : ctrl->nc[cur];
    const int tid = threadIdx.x, lane = tid & 63;
    constexpr int RR = sp_rows(D8);
    const int64_t j0 = (int64_t)blockIdx.x * (256 * RR) + tid;   // this thread's samples: j0 + 256 r
    for (int c = tid; c < kSpB; c += 256) cnt_s[c] = 0;

    // claims of batch b - 1 (its masks are still in near[])
    if (b > 0) {
        const int ncp = ctrl->nc[prev];
        const uint64_t* vp = ctrl->vis[prev];
        const int32_t* candp = a.cand + prev * kSpB;
        const int32_t* cntp = a.cnt + prev * kSpB;
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            const int64_t j = j0 + r * 256;
            if (j < a.n && a.owner[j] == INT_MAX) {
#pragma unroll
                for (int w = 0; w < kSpW; ++w) {
                    const uint64_t m = a.near[(size_t)j * kSpW + w] & vp[w];
                    if (m) {
                        const int c = w * 64 + __builtin_ctzll(m);
                        a.owner[j] = candp[c];
                        a.dens[j] = cntp[c];
                        break;
                    }
                }
            }
        }
        if (blockIdx.x == 0) {
            // visited candidates take their own count (also when the
            // approximation width admits no sample, not even the row itself);
            // the claim above writes the same values for them
            for (int c = tid; c < ncp; c += 256) {
                if ((vp[c >> 6] >> (c & 63)) & 1ull) {
                    const int32_t i = candp[c];
                    a.owner[i] = i;
                    a.dens[i] = cntp[c];
                    if (a.visited) a.visited[i] = 1;
                }
            }
        }
    }
    __syncthreads();

    if (nc > 0) batch_rows<D8, METRIC>(a, cur, nc, j0, cnt_s, cs);
    __syncthreads();
    for (int c = tid; c < nc; c += 256)
        if (cnt_s[c]) atomicAdd(&a.cnt[cur * kSpB + c], cnt_s[c]);

    // the last block to finish takes the batch's tail
    __threadfence();
    __syncthreads();
    if (tid == 0) s_last = atomicAdd(&ctrl->ticket, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    if (nc == 0) {                          // the last claims are applied: finished
        if (tid == 0) { ctrl->done = 1; ctrl->ticket = 0; ctrl->batch = b + 1; }
        return;
    }
    // resolve batch b in candidate order, 64 candidates per step: lane l
    // takes candidate 64 g + l; earlier steps' visited set is final, within
    // the step one lane after the other
    const int32_t* cand = a.cand + cur * kSpB;
    for (int e = tid; e < nc * kSpW; e += 256) {
        const int c = e / kSpW, w = e - c * kSpW;
        cm[c][w] = a.near[(size_t)cand[c] * kSpW + w];
    }
    __syncthreads();
    if (tid < 64) {
        uint64_t vis[kSpW] = {0ull, 0ull, 0ull, 0ull};
#pragma unroll
        for (int g = 0; g < kSpW; ++g) {
            const int c = 64 * g + lane;
            bool early = false;
            uint64_t intra = 0ull;
            if (c < nc) {
#pragma unroll
                for (int w = 0; w < kSpW; ++w) early |= w < g && (cm[c][w] & vis[w]) != 0ull;
                intra = cm[c][g];
            }
            uint64_t vg = 0ull;
            const int lim = min(64, nc - 64 * g);
            for (int l = 0; l < lim; ++l) {
                const bool ke = __shfl(early, l);
                const uint64_t m = __shfl(intra, l);
                if (!ke && (m & vg & ((1ull << l) - 1ull)) == 0ull) vg |= 1ull << l;
            }
            vis[g] = vg;
        }
        if (lane < kSpW) {
            svis[lane] = vis[0];
#pragma unroll
            for (int w = 1; w < kSpW; ++w) svis[lane] = lane == w ? vis[w] : svis[lane];
        }
    }
    __syncthreads();
    if (tid == 0) {
        int v = 0;
#pragma unroll
        for (int w = 0; w < kSpW; ++w) {
            ctrl->vis[cur][w] = svis[w];
            v += __popcll(svis[w]);
        }
        ctrl->visited += v;
        ctrl->last_visited = v;
    }
    // the next batch, into the other buffer: about twice this batch's visited count
    int v = 0;
#pragma unroll
    for (int w = 0; w < kSpW; ++w) v += __popcll(svis[w]);
    const int B = min(kSpB, max(kSpBMin, 2 * v));
    select_batch<256>(a, prev, B, svis, wsum, &s_found);
    if (tid == 0) {
        ctrl->ticket = 0;
        ctrl->batch = b + 1;
    }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct SpadeLayout {
    size_t ctrl, owner, cand, cnt, crow, near, total;
};

SpadeLayout spade_layout(int64_t n, int32_t d)
{
    SpadeLayout L{};
    const int DP = (d + 7) / 8 * 8;
    size_t off = 0;
    L.ctrl = off;  off = align256(off + sizeof(SpadeCtrl));
    L.owner = off; off = align256(off + (size_t)n * sizeof(int32_t));
    L.cand = off;  off = align256(off + 2 * kSpB * sizeof(int32_t));
    L.cnt = off;   off = align256(off + 2 * kSpB * sizeof(int32_t));
    L.crow = off;  off = align256(off + 2 * (size_t)kSpB * DP * sizeof(double));
    L.near = off;  off = align256(off + (size_t)n * kSpW * sizeof(uint64_t));
    L.total = off;
    return L;
}

km_status sp_fail(km_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return km_set_error(st, buf);
}

km_status sp_hip(hipError_t e, const char* what)
{
    return sp_fail(KM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

template <int D8>
void launch_batch_d8(int metric, const SpadeArgs& a, dim3 grid, hipStream_t s)
{
    if (metric == 0) hipLaunchKernelGGL((spade_batch_kernel<D8, 0>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((spade_batch_kernel<D8, 1>), grid, dim3(256), 0, s, a);
}

void launch_batch(int metric, int D8, const SpadeArgs& a, dim3 grid, hipStream_t s)
{
    switch (D8) {
    case 1: launch_batch_d8<1>(metric, a, grid, s); break;
    case 2: launch_batch_d8<2>(metric, a, grid, s); break;
    case 3: launch_batch_d8<3>(metric, a, grid, s); break;
    case 4: launch_batch_d8<4>(metric, a, grid, s); break;
    case 5: launch_batch_d8<5>(metric, a, grid, s); break;
    case 6: launch_batch_d8<6>(metric, a, grid, s); break;
    case 7: launch_batch_d8<7>(metric, a, grid, s); break;
    case 8: launch_batch_d8<8>(metric, a, grid, s); break;
    default: launch_batch_d8<0>(metric, a, grid, s); break;
    }
}

}  // namespace
}  // namespace km

using namespace km;

extern "C" {

size_t spade_workspace_bytes(int64_t n, int32_t d)
{
    if (n < 1 || n >= ((int64_t)1 << 31) || d < 1 || d > 1024) return 0;
    return spade_layout(n, d).total;
}

km_status spade_densities(const float* X, int64_t n, int32_t d, double apprx_width, double kernel_width,
                          km_metric metric, int32_t* densities, int8_t* visited, int64_t* visited_count,
                          void* ws, size_t ws_bytes, hipStream_t stream)
{
    km_set_error(KM_OK, "");
    if (n < 1 || n >= ((int64_t)1 << 31)) return sp_fail(KM_EINVAL, "n = %lld outside [1, 2^31)", (long long)n);
    if (d < 1 || d > 1024) return sp_fail(KM_EINVAL, "d = %d outside [1, 1024]", d);
    if (metric != KM_METRIC_L1 && metric != KM_METRIC_SQEUCLIDEAN)
        return sp_fail(KM_EINVAL, "unknown metric %d", (int)metric);
    if (!X || !densities) return sp_fail(KM_EINVAL, "X and densities must be non-NULL");
    if (reinterpret_cast<uintptr_t>(X) & 3u) return sp_fail(KM_EINVAL, "X must be 4-byte aligned");
    if (apprx_width != apprx_width || kernel_width != kernel_width)
        return sp_fail(KM_EINVAL, "widths must not be NaN");
    const SpadeLayout L = spade_layout(n, d);
    if (!ws) return sp_fail(KM_EWORKSPACE, "workspace pointer is NULL");
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return sp_fail(KM_EWORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total)
        return sp_fail(KM_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, L.total);

    unsigned char* w = static_cast<unsigned char*>(ws);
    SpadeArgs a{};
    a.X = X; a.n = n; a.d = d; a.DP = (d + 7) / 8 * 8;
    a.apprx = apprx_width; a.kern = kernel_width;
    a.ctrl = reinterpret_cast<SpadeCtrl*>(w + L.ctrl);
    a.owner = reinterpret_cast<int32_t*>(w + L.owner);
    a.cand = reinterpret_cast<int32_t*>(w + L.cand);
    a.cnt = reinterpret_cast<int32_t*>(w + L.cnt);
    a.crow = reinterpret_cast<double*>(w + L.crow);
    a.near = reinterpret_cast<uint64_t*>(w + L.near);
    a.dens = densities;
    a.visited = visited;
    const int D8 = (d + 7) / 8;
    const int rows_per_block = 256 * sp_rows(D8 <= kSpMaxD8Reg ? D8 : 0);
    const dim3 grid((unsigned)((n + rows_per_block - 1) / rows_per_block));
    hipError_t e;
    hipLaunchKernelGGL(spade_init_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 2048)), dim3(256), 0,
                       stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return sp_hip(e, "spade init launch");
    // batch 0, then one launch per batch (and one to apply the last claims),
    // enqueued in groups; after each group the host reads the done flag
    // (launches past the end return at once)
    hipLaunchKernelGGL(spade_first_select_kernel, dim3(1), dim3(kSpSelThreads), 0, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return sp_hip(e, "spade select launch");
    int group = 2;
    int64_t launched = 0;
    SpadeCtrl hc{};
    for (;;) {
        for (int g = 0; g < group; ++g) launch_batch(metric, D8 <= kSpMaxD8Reg ? D8 : 0, a, grid, stream);
        if ((e = hipGetLastError()) != hipSuccess) return sp_hip(e, "spade batch launch");
        launched += group;
        if ((e = hipMemcpyAsync(&hc, a.ctrl, sizeof hc, hipMemcpyDeviceToHost, stream)) != hipSuccess)
            return sp_hip(e, "hipMemcpyAsync(spade control)");
        if ((e = hipStreamSynchronize(stream)) != hipSuccess) return sp_hip(e, "hipStreamSynchronize");
        if (hc.done) break;
        if (launched > 2 * n + 64) return sp_fail(KM_EHIP, "spade: no progress after %lld launches", (long long)launched);
        group = std::min(group * 2, 64);
    }
    if (visited_count) *visited_count = hc.visited;
    return KM_OK;
}

km_status spade_stats(const void* ws, int64_t n, int32_t d, int64_t* batches, int64_t* candidates,
                      hipStream_t stream)
{
    km_set_error(KM_OK, "");
    if (!ws || n < 1 || d < 1 || d > 1024) return sp_fail(KM_EINVAL, "bad workspace or shape");
    SpadeCtrl hc{};
    const SpadeLayout L = spade_layout(n, d);
    hipError_t e = hipMemcpyAsync(&hc, static_cast<const unsigned char*>(ws) + L.ctrl, sizeof hc,
                                  hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return sp_hip(e, "hipMemcpyAsync(spade control)");
    if ((e = hipStreamSynchronize(stream)) != hipSuccess) return sp_hip(e, "hipStreamSynchronize");
    if (batches) *batches = hc.batches;
    if (candidates) *candidates = hc.candidates;
    return KM_OK;
}

}  // extern "C"
