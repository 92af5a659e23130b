// Plain FP32 Lloyd pass for gfx950: assign (map) fused with the per-label
// reduce, following the parallel-loop contract of section 2.3 (the body runs
// once per sample index, in no fixed order; writes to shared state happen only
// at disjoint places) and the fusion of section 3.5 (the assign loop and the
// reduce loop share the sample range, so they run as one pass and the label
// vector is consumed in place; the objective is a side-by-side reduction in
// the same traversal).
//
// Layout of one block (256 lanes = 4 wave64s):
//   * a tile is 256 consecutive samples, one per lane; the block walks tiles
//     blockIdx.x, blockIdx.x + gridDim.x, ...  (a fixed, schedule-independent
//     partition of the sample range);
//   * each lane holds its sample row in VGPRs (zero-padded to D = 8 * D8);
//     centroid rows are wave-uniform, so they are read with scalar loads and
//     enter the VALU as SGPR operands: no LDS traffic and no VGPRs for C;
//   * distances are the canonical direct form (dist_rows in km_dist.h);
//   * the block's activation record -- FP64 per-label sums S[k][d] and counts
//     -- is private to the block in LDS ("alloc" zeroes it, "process" adds a
//     sample, and it is merged once per block into a fixed partial slot);
//   * within a block, wave w owns the labels L with L % 4 == w and adds its
//     samples in tile order with LDS atomics that it alone issues, so the
//     order of every FP64 sum is fixed and results are bit-reproducible.
#include "km_internal.h"
#include "km_dist.h"

#include <climits>
#include <type_traits>

namespace km {


__device__ __forceinline__ void lds_add_f64(double* p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// "process": add the samples of a step (at most STEP of them: one or more
// tiles) that this wave owns to the block's activation record, in increasing
// sample order.  lab[g] is the label of sample g * 64 + lane of the step (-1:
// none, or another chunk's); row_of(pos) is the row of sample pos; the lists
// hold cap entries per buffer (the step's samples).  A row takes LPR
// lanes (lane f carries feature f: coalesced), so a wave holds NG = 64 / LPR
// row groups; label class c = L mod (4 NG) belongs to wave c / NG, row group
// c % NG.  Each group lists (and counts) its samples in LDS, two groups
// sharing a buffer from its two ends; then BG rows per group at a time are
// loaded, the next batch's loads issued before this batch's adds, rows past
// a list's end clamped to the step's first row instead of branching, so no
// load waits on another.  The adds are LDS atomics without return, which the
// wave issues, and the LDS executes, in program order; the groups of one
// instruction hold different labels, so every sum has a fixed order and
// nothing waits on the results.
template <int D8, int STEP, typename RowOf>
__device__ __forceinline__ void accumulate_step(RowOf row_of, int d, const int (&lab)[STEP / 64], int cap,
                                                int32_t* wl, double* S, int32_t* cnt, int lane, int wave)
{
    constexpr int LPR = row_lanes(D8);                          // lanes per row
    constexpr int NG = 64 / LPR;                                // row groups per wave
    constexpr int FPL = (8 * D8 + LPR - 1) / LPR;               // features per lane
    constexpr int BG = NG > 1 ? 16 : (FPL == 1 ? 32 : 16);      // rows per group per batch
    static_assert(NG * BG <= 64, "one entry per lane");
    static_assert(STEP <= 4096, "12-bit step offsets");
    // slot i of group s's list (buffers of cap entries: the samples a step can hold)
    auto slot = [cap](int s, int i) { return (s >> 1) * cap + ((s & 1) ? cap - 1 - i : i); };
    int nown[NG];
#pragma unroll
    for (int s = 0; s < NG; ++s) nown[s] = 0;
#pragma unroll
    for (int g = 0; g < STEP / 64; ++g) {
        const int L = lab[g];
        const int c = L & (kWaves * NG - 1);
        const bool own = L >= 0 && c / NG == wave;
#pragma unroll
        for (int s = 0; s < NG; ++s) {
            const bool mine = own && c % NG == s;
            const uint64_t mask = __ballot(mine);
            if (mine) {
                wl[slot(s, nown[s] + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u)))] =
                    ((L * d) << 12) | (g * 64 + lane);   // record offset of the row (< 2^19), offset in the step
                // counts are integers: any order of these adds gives the same total
                __hip_atomic_fetch_add(cnt + L, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            nown[s] += (int)__popcll(mask);
        }
    }
    const int h = lane / LPR;       // this lane's row group
    const int fl = lane % LPR;      // its first feature
    int fc[FPL];
#pragma unroll
    for (int m = 0; m < FPL; ++m) fc[m] = min(fl + LPR * m, d - 1);
    int nmax = nown[0], nmin = nown[0];
#pragma unroll
    for (int s = 1; s < NG; ++s) { nmax = max(nmax, nown[s]); nmin = min(nmin, nown[s]); }
    const int nbat = (nmax + BG - 1) / BG;
    float v0[BG][FPL], v1[BG][FPL];
    int q0 = -1, q1 = -1;
    // The entry of row u of batch b for this lane's group.  One group: lane
    // u holds it and a readlane broadcasts it.  Several groups: each lane
    // reads its group's entries from the list, four per LDS read (an odd
    // group's list runs backwards from the end of its buffer); entries past
    // the group's list read as -1.
    int nh = nown[0];
#pragma unroll
    for (int s = 1; s < NG; ++s) nh = h == s ? nown[s] : nh;
    auto entries = [&](int b) {
        if constexpr (NG == 1) {
            const int i = b * BG + lane;
            return (lane < BG && i < nown[0]) ? wl[i] : -1;
        } else {
            return 0;
        }
    };
    auto batch_entries = [&](int b, int q, int (&e)[BG]) {
        if constexpr (NG == 1) {
#pragma unroll
            for (int u = 0; u < BG; ++u) e[u] = __builtin_amdgcn_readlane(q, u);
        } else {
            const int i0 = b * BG;
#pragma unroll
            for (int u = 0; u < BG; u += 4) {
                const int4 v = *reinterpret_cast<const int4*>(wl + ((h & 1) ? slot(h, i0 + u + 3) : slot(h, i0 + u)));
                const bool rev = h & 1;
                e[u + 0] = rev ? v.w : v.x;
                e[u + 1] = rev ? v.z : v.y;
                e[u + 2] = rev ? v.y : v.z;
                e[u + 3] = rev ? v.x : v.w;
            }
            if (i0 + BG > nh) {
#pragma unroll
                for (int u = 0; u < BG; ++u) e[u] = i0 + u < nh ? e[u] : -1;
            }
        }
    };
    auto load = [&](int b, float (&v)[BG][FPL], int& q) {
        q = entries(b);
        int e[BG];
        batch_entries(b, q, e);
        const int first = NG == 1 ? e[0] : 0;     // entry 0 of a one-group batch is valid
#pragma unroll
        for (int u = 0; u < BG; ++u) {
            const float* row = row_of(e[u] >= 0 ? (e[u] & 4095) : (NG == 1 ? (first & 4095) : 0));
#pragma unroll
            for (int m = 0; m < FPL; ++m) v[u][m] = row[fc[m]];
        }
    };
    auto add = [&](int b, const float (&v)[BG][FPL], int q) {
        const bool full = b * BG + BG <= nmin;   // every group has all BG rows: no per-row test
        int e[BG];
        batch_entries(b, q, e);
#pragma unroll
        for (int u = 0; u < BG; ++u) {
            if (full || e[u] >= 0) {
                double* srow = S + (e[u] >> 12);
#pragma unroll
                for (int m = 0; m < FPL; ++m) {
                    const int f = fl + LPR * m;
                    if (f < d) lds_add_f64(srow + f, (double)v[u][m]);
                }
            }
        }
    };
    if (nbat > 0) load(0, v0, q0);
    for (int b = 0; b < nbat; b += 2) {
        if (b + 1 < nbat) load(b + 1, v1, q1);
        add(b, v0, q0);
        if (b + 1 < nbat) {
            if (b + 2 < nbat) load(b + 2, v0, q0);
            add(b + 1, v1, q1);
        }
    }
}

// Nearest centroid of each of the R rows a lane holds, over all k centroids,
// with the canonical distance.  Ties keep the lower index.
template <int D8, int R, typename CP>
__device__ __forceinline__ void nearest(const float (&x)[R][8 * D8], CP C, int k, float (&best)[R], int (&bj)[R])
{
#pragma unroll
    for (int r = 0; r < R; ++r) { best[r] = __builtin_huge_valf(); bj[r] = 0; }
    for (int j = 0; j < k; ++j) {
        float dist[R];
        dist_rows<D8, R>(x, C + (size_t)j * (8 * D8), dist);
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (dist[r] < best[r]) { best[r] = dist[r]; bj[r] = j; }
    }
}

// The per-sample pass of one block: tiles t_first, t_first + t_step, ... below
// t_end, its activation record written to partial slot `slot`; `chunk` is the
// label chunk of update passes over chunked records.
template <int D8, int MODE>
__device__ __forceinline__ void pass_body(const PassArgs& a, int64_t t_first, int64_t t_end, int64_t t_step,
                                          int slot, int chunk, unsigned char* smem)
{
    constexpr int D = 8 * D8;
    constexpr int R = plain_rows_per_lane(D8);
    constexpr bool UPD = (MODE == MODE_UPDATE);
    constexpr bool FUSED = (MODE == MODE_FUSED);
    constexpr int TILE = kBlock * R;
    __shared__ double redJ[kWaves];
    __shared__ int32_t redC[kWaves];

    if (a.ctrl != nullptr && a.ctrl->stop_iter < a.iter) return;  // converged earlier

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int k = a.k, d = a.d;
    const int64_t n = a.n;
    // Label chunk of this block (update / fused passes): labels [j0, j0 + kc).
    const int j0 = UPD ? chunk * a.kc : 0;
    const int kc = UPD ? min(a.kc, k - j0) : k;

    double* S = reinterpret_cast<double*>(smem);
    int32_t* cnt = reinterpret_cast<int32_t*>(S + ((size_t)kc * d + 1) / 2 * 2);   // 16-byte aligned
    int32_t* lbl = cnt + (((size_t)kc + 3) & ~(size_t)3);     // fused: [2][TILE] labels of a tile
    int32_t* wlist = FUSED ? lbl + 2 * TILE : lbl;             // [kWaves][list buffers][step] owned samples

    // "alloc": zero the block's activation record
    if (MODE != MODE_ASSIGN) {
        for (int e = tid; e < kc * d; e += kBlock) S[e] = 0.0;
        for (int j = tid; j < kc; j += kBlock) cnt[j] = 0;
    }
    __syncthreads();

    double Jl = 0.0;
    int32_t changed = 0;
    const int64_t ntiles = (n + TILE - 1) / TILE;
    const int64_t t_last = t_end < ntiles ? t_end : ntiles;
    const int64_t nmine = t_first < t_last ? (t_last - t_first + t_step - 1) / t_step : 0;

    // the map over one tile: nearest centroid, labels, objective, changed count
    auto assign_tile = [&](int64_t t, int (&lab)[R]) {
        float x[R][D];
        int old[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t gp = t * TILE + r * kBlock + tid;
            const bool valid = gp < n;
            // the previous label is fetched with the row, not after the sweep
            old[r] = (valid && a.count_changed && a.iter != 0) ? a.labels[gp] : -1;
            load_row<D8>(a.X + (valid ? gp : 0) * a.ldx, d, valid, x[r]);
        }
        float best[R];
        int bj[R];
        nearest<D8, R>(x, (cfloat*)a.Cp, k, best, bj);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t gp = t * TILE + r * kBlock + tid;
            lab[r] = -1;
            if (gp < n) {
                if (a.count_changed) changed += (a.iter == 0) ? 1 : (old[r] != bj[r]);
                a.labels[gp] = bj[r];
                if (a.mindist) a.mindist[gp] = best[r];
                Jl += (double)best[r];
                lab[r] = bj[r];
            }
        }
    };

    if constexpr (FUSED) {
        for (int64_t i = 0; i < nmine; ++i) {
            const int64_t t = t_first + i * t_step;
            int lab[R];
            assign_tile(t, lab);
            // "process": the tile's labels go through LDS to the waves that own them
            int32_t* lb = lbl + (i & 1) * TILE;
#pragma unroll
            for (int r = 0; r < R; ++r) lb[r * kBlock + tid] = lab[r];
            __syncthreads();    // labels of the tile complete
            int lt[TILE / 64];
#pragma unroll
            for (int g = 0; g < TILE / 64; ++g) lt[g] = lb[g * 64 + lane];
            const float* Xt = a.X + t * TILE * (int64_t)a.ldx;
            accumulate_step<D8, TILE>([&](int pos) { return Xt + pos * a.ldx; }, d, lt, TILE,
                                      wlist + wave * list_bufs(D8) * TILE, S, cnt, lane, wave);
        }
    } else if constexpr (UPD) {
        // steps of UT of the block's tiles: every wave reads the whole step's
        // labels (INT_MIN: past the last sample), the next step's in flight
        // while this one is added; labels outside [0, k) are skipped
        auto steps = [&](auto ut_c) {
            constexpr int UT = decltype(ut_c)::value;
            constexpr int NL = UT * TILE / 64;
            const int64_t nsteps = (nmine + UT - 1) / UT;
            auto tile_of = [&](int64_t st, int j) { return t_first + (st * UT + j) * t_step; };
            auto load_labels = [&](int64_t st, int (&Lv)[NL]) {
#pragma unroll
                for (int j = 0; j < UT; ++j) {
                    const bool in = st * UT + j < nmine;
#pragma unroll
                    for (int g = 0; g < TILE / 64; ++g) {
                        const int64_t gp = tile_of(st, j) * TILE + g * 64 + lane;
                        Lv[j * (TILE / 64) + g] = (in && gp < n) ? a.labels[gp] : INT_MIN;
                    }
                }
            };
            int Ln[NL];
            if (nsteps > 0) load_labels(0, Ln);
            for (int64_t st = 0; st < nsteps; ++st) {
                int L[NL];
#pragma unroll
                for (int g = 0; g < NL; ++g) L[g] = Ln[g];
                if (st + 1 < nsteps) load_labels(st + 1, Ln);
                int lab[NL];
#pragma unroll
                for (int g = 0; g < NL; ++g) {
                    lab[g] = -1;
                    if (L[g] != INT_MIN && L[g] >= j0 && L[g] < j0 + kc && L[g] < k)
                        lab[g] = L[g] - j0;   // chunk-local label
                }
                // the step's samples are consecutive (one tile, or contiguous tiles)
                const float* Xs = a.X + tile_of(st, 0) * TILE * (int64_t)a.ldx;
                auto row_of = [&](int pos) { return Xs + pos * a.ldx; };
                accumulate_step<D8, UT * TILE>(row_of, d, lab, UT * TILE, wlist + wave * list_bufs(D8) * UT * TILE,
                                               S, cnt, lane, wave);
            }
        };
        if (a.upd_tiles == kUpdTiles && t_step == 1) steps(std::integral_constant<int, kUpdTiles>());
        else steps(std::integral_constant<int, 1>());
    } else {
        for (int64_t i = 0; i < nmine; ++i) {
            int lab[R];
            assign_tile(t_first + i * t_step, lab);
        }
    }

    // Merge once per block: the activation record goes to slot `slot`,
    // labels [j0, j0 + kc) of it.
    __syncthreads();
    const int b = slot;
    if (MODE != MODE_ASSIGN) {
        double* dst = a.part.S + (size_t)b * k * d + (size_t)j0 * d;
        for (int e = tid; e < kc * d; e += kBlock) dst[e] = S[e];
        int32_t* dc = a.part.cnt + (size_t)b * k + j0;
        for (int j = tid; j < kc; j += kBlock) dc[j] = cnt[j];
    }
    // Fixed-order reductions of the scalar partials: xor tree inside the
    // wave (lane 0's value), then waves in index order.
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        Jl += __shfl_xor(Jl, off);
        changed += __shfl_xor(changed, off);
    }
    if (lane == 0) { redJ[wave] = Jl; redC[wave] = changed; }
    __syncthreads();
    if (tid == 0 && !UPD) {
        double J = redJ[0];
        int32_t c = redC[0];
        for (int w = 1; w < kWaves; ++w) { J += redJ[w]; c += redC[w]; }
        a.part.J[b] = J;
        a.part.changed[b] = c;
    }
}

// The update pass holds two batches of rows in flight; it is built for four
// resident waves per SIMD (at most 128 VGPRs).
__host__ __device__ constexpr int pass_min_waves(int mode) { return mode == MODE_UPDATE ? 4 : 1; }

template <int D8, int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(pass_min_waves(MODE))))
void plain_pass(PassArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    if (MODE == MODE_UPDATE && a.upd_tiles > 1) {
        // a stand-alone update: block b walks tiles [b T / G, (b + 1) T / G)
        const int64_t nt = (a.n + kBlock - 1) / kBlock;
        pass_body<D8, MODE>(a, (int64_t)blockIdx.x * nt / gridDim.x, (int64_t)(blockIdx.x + 1) * nt / gridDim.x, 1,
                            blockIdx.x, blockIdx.y, smem);
    } else {
        pass_body<D8, MODE>(a, blockIdx.x, INT64_MAX, gridDim.x, blockIdx.x, blockIdx.y, smem);
    }
}

// Batched instances: block b runs tiles [t0, t1) of instance work[b].inst into
// that instance's partial slot work[b].slot.
template <int D8, int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(pass_min_waves(MODE))))
void batch_pass(const BatchWork* __restrict__ work,
                                                     const PassArgs* __restrict__ insts, int32_t iter)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const BatchWork w = work[blockIdx.x];
    PassArgs a = insts[w.inst];
    a.iter = iter;
    pass_body<D8, MODE>(a, w.t0, w.t1, 1, w.slot, 0, smem);
}

// ------------------------------------------------------ partitioned update
// Large records are reduced over label chunks.  Instead of every (point
// range, chunk) block scanning all labels of its range, one pass partitions
// each kPartRows-sample sub-range by label chunk (a stable counting sort:
// chunk counts, their prefix, then each 64-sample group's lanes placed chunk
// by chunk in lane order), and the chunk blocks read just their samples.
// Within a group, the lanes of a lane's chunk are found bit by bit: one
// ballot per bit of the chunk index, kept or complemented as the lane's own
// bit is set or clear, so the cost is log2(chunks) ballots, not one round
// per distinct chunk.
__global__ __launch_bounds__(64) void partition_kernel(const int32_t* __restrict__ labels, int64_t n, int32_t k,
                                                       int32_t kc, int32_t nch, int32_t* perm, int32_t* plab,
                                                       int32_t* poff, int32_t* pcnt, const Ctrl* ctrl, int32_t iter)
{
    constexpr int G = kPartRows / 64;                     // 64-sample groups of a sub-range
    extern __shared__ __align__(16) unsigned char smem[];
    if (ctrl != nullptr && ctrl->stop_iter < iter) return;  // converged earlier
    int32_t* cnt = reinterpret_cast<int32_t*>(smem);     // [nch]
    int32_t* cur = cnt + nch;                             // [nch]
    const int lane = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kPartRows;
    const int64_t end = base + kPartRows < n ? base + kPartRows : n;
    for (int c = lane; c < nch; c += 64) cnt[c] = 0;
    // every label of the sub-range in registers (all loads in flight at once)
    int lb[G], ch[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t i = base + g * 64 + lane;
        lb[g] = i < end ? labels[i] : -1;
    }
#pragma unroll
    for (int g = 0; g < G; ++g) ch[g] = (lb[g] >= 0 && lb[g] < k) ? lb[g] / kc : -1;
    __syncthreads();
    // per group: a lane's rank among the lanes of its chunk and their number,
    // packed beside the chunk (chunk < 2^16, rank < 64, number <= 64); the
    // first lane of each chunk adds the number (distinct addresses)
    const int nbits = nch > 1 ? 32 - __builtin_clz((unsigned)(nch - 1)) : 0;
    const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int c = ch[g];
        uint64_t same = __ballot(c >= 0);
        for (int b = 0; b < nbits; ++b) {
            const bool bit = (c >> b) & 1;
            const uint64_t m = __ballot(bit);
            same &= bit ? m : ~m;
        }
        const int rank = (int)__popcll(same & lt), num = (int)__popcll(same);
        if (c >= 0) {
            if (rank == 0) __hip_atomic_fetch_add(cnt + c, num, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            ch[g] = c | (rank << 16) | (num << 23);
        }
    }
    __syncthreads();
    int carry = 0;
    for (int c0 = 0; c0 < nch; c0 += 64) {
        const int c = c0 + lane;
        const int v = c < nch ? cnt[c] : 0;
        int incl = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(incl, off);
            if (lane >= off) incl += o;
        }
        if (c < nch) {
            const int start = (int)base + carry + incl - v;
            cur[c] = start;
            poff[(int64_t)blockIdx.x * nch + c] = start;
            pcnt[(int64_t)blockIdx.x * nch + c] = v;
        }
        carry += __shfl(incl, 63);
    }
    __syncthreads();
    // scatter in sample order: a lane's slot is its chunk's cursor plus the
    // number of lower lanes of the group in the same chunk
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int c = ch[g] >= 0 ? (ch[g] & 0xffff) : -1;
        const int rank = (ch[g] >> 16) & 127, num = ch[g] >> 23;
        const int at = c >= 0 ? cur[c] : 0;
        if (c >= 0) {
            perm[at + rank] = (int32_t)(base + g * 64 + lane);
            plab[at + rank] = lb[g];
            if (rank == 0) cur[c] = at + num;    // the chunk's first lane advances its cursor
        }
    }
}

// Block (x, y): labels [y*kc, y*kc + kc') over sub-ranges [x*nsub/G, (x+1)*nsub/G);
// wave w adds the samples whose chunk-local label is congruent to w mod 4,
// in sample order (sub-range, then list order), by LDS atomics in program
// order; the record goes to partial slot x like the other update passes.
// The block's entries (sample, label) are walked kPartStep at a time, the
// next step's entries in flight while this step's rows are added, and the
// rows in batches of B with the next batch's loads issued first.
constexpr int kPartStep = 256;
template <int D8>
__global__ __launch_bounds__(kBlock) void part_update_kernel(PassArgs a)
{
    constexpr int FPL = (8 * D8 + 63) / 64;
    constexpr int B = FPL == 1 ? 32 : 16;
    constexpr int Q = kPartStep / 64;
    extern __shared__ __align__(16) unsigned char smem[];
    if (a.ctrl != nullptr && a.ctrl->stop_iter < a.iter) return;  // converged earlier
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int k = a.k, d = a.d;
    const int y = blockIdx.y;
    const int j0 = y * a.kc;
    const int kc = min(a.kc, k - j0);
    double* S = reinterpret_cast<double*>(smem);
    int32_t* cnt = reinterpret_cast<int32_t*>(S + (size_t)kc * d);
    int32_t* wrow = cnt + (((size_t)kc + 3) & ~(size_t)3);     // [kWaves][kPartStep] owned sample indices
    int32_t* woff = wrow + kWaves * kPartStep;                 // [kWaves][kPartStep] their record offsets
    for (int e = tid; e < kc * d; e += kBlock) S[e] = 0.0;
    for (int j = tid; j < kc; j += kBlock) cnt[j] = 0;
    __syncthreads();
    int32_t* wr = wrow + wave * kPartStep;
    int32_t* wo = woff + wave * kPartStep;
    int fc[FPL];
#pragma unroll
    for (int m = 0; m < FPL; ++m) fc[m] = min(lane + 64 * m, d - 1);
    const uint64_t lt = (1ull << lane) - 1ull;
    const int s1 = (int)((int64_t)(blockIdx.x + 1) * a.nsub / gridDim.x);
    // step cursor: sub-range sr, entries [q0, q0 + kPartStep) of its run of this chunk
    int sr = (int)((int64_t)blockIdx.x * a.nsub / gridDim.x);
    int q0 = 0, start = 0, num = 0;
    if (sr < s1) { start = a.poff[(int64_t)sr * a.nch + y]; num = a.pcnt[(int64_t)sr * a.nch + y]; }
    auto fetch = [&](int st, int nm, int q, int (&E)[Q], int (&L)[Q]) {
#pragma unroll
        for (int g = 0; g < Q; ++g) {
            const int i = q + g * 64 + lane;
            E[g] = i < nm ? a.perm[st + i] : -1;
            L[g] = i < nm ? a.plab[st + i] - j0 : -1;
        }
    };
    int E[Q], L[Q];
    fetch(start, num, 0, E, L);
    float v0[B][FPL], v1[B][FPL];
    while (sr < s1) {
        // the next step: the rest of this run, else the next non-empty sub-range
        int nsr = sr, nq0 = q0 + kPartStep, nstart = start, nnum = num;
        if (nq0 >= num) {
            nq0 = 0;
            nnum = 0;
            while (nnum == 0 && ++nsr < s1) {
                nstart = a.poff[(int64_t)nsr * a.nch + y];
                nnum = a.pcnt[(int64_t)nsr * a.nch + y];
            }
        }
        int En[Q], Ln[Q];
        fetch(nstart, nnum, nq0, En, Ln);
        // this step's owned entries, in order
        int nown = 0;
#pragma unroll
        for (int g = 0; g < Q; ++g) {
            const bool own = E[g] >= 0 && (L[g] & (kWaves - 1)) == wave;
            const uint64_t mask = __ballot(own);
            if (own) {
                const int at = nown + (int)__popcll(mask & lt);
                wr[at] = E[g];
                wo[at] = L[g] * d;
                __hip_atomic_fetch_add(cnt + L[g], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            nown += (int)__popcll(mask);
        }
        int r0 = -1, o0 = -1, r1 = -1, o1 = -1;
        auto load = [&](int b, float (&v)[B][FPL], int& ri, int& oi) {
            ri = (lane < B && b * B + lane < nown) ? wr[b * B + lane] : -1;
            oi = (lane < B && b * B + lane < nown) ? wo[b * B + lane] : -1;
            const int first = __builtin_amdgcn_readfirstlane(ri);   // entry b*B: always valid
#pragma unroll
            for (int u = 0; u < B; ++u) {
                int r = __builtin_amdgcn_readlane(ri, u);
                r = r >= 0 ? r : first;
                const float* row = a.X + (int64_t)r * a.ldx;
#pragma unroll
                for (int m = 0; m < FPL; ++m) v[u][m] = row[fc[m]];
            }
        };
        auto add = [&](const float (&v)[B][FPL], int oi) {
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int o = __builtin_amdgcn_readlane(oi, u);
                if (o >= 0) {
#pragma unroll
                    for (int m = 0; m < FPL; ++m) {
                        const int f = lane + 64 * m;
                        if (f < d) lds_add_f64(S + o + f, (double)v[u][m]);
                    }
                }
            }
        };
        const int nbat = (nown + B - 1) / B;
        if (nbat > 0) load(0, v0, r0, o0);
        for (int b = 0; b < nbat; b += 2) {
            if (b + 1 < nbat) load(b + 1, v1, r1, o1);
            add(v0, o0);
            if (b + 1 < nbat) {
                if (b + 2 < nbat) load(b + 2, v0, r0, o0);
                add(v1, o1);
            }
        }
#pragma unroll
        for (int g = 0; g < Q; ++g) { E[g] = En[g]; L[g] = Ln[g]; }
        sr = nsr; q0 = nq0; start = nstart; num = nnum;
    }
    __syncthreads();
    const int b = blockIdx.x;
    double* dst = a.part.S + (size_t)b * k * d + (size_t)j0 * d;
    for (int e = tid; e < kc * d; e += kBlock) dst[e] = S[e];
    int32_t* dc = a.part.cnt + (size_t)b * k + j0;
    for (int j = tid; j < kc; j += kBlock) dc[j] = cnt[j];
}

size_t part_update_lds_bytes(int kc, int d)
{
    return (size_t)kc * d * sizeof(double) + (((size_t)kc * sizeof(int32_t) + 15) & ~(size_t)15) +
           2 * kWaves * kPartStep * sizeof(int32_t);
}

// The same partition with four waves per sub-range (1024 samples each): the
// waves count their chunks separately, one wave forms the block's chunk
// offsets and each wave's cursors (wave w's samples follow waves 0..w-1's in
// every chunk), so the permutation is the one-wave kernel's exactly.
constexpr int kPartWaves = 4;
__global__ __launch_bounds__(64 * kPartWaves) void partition4_kernel(const int32_t* __restrict__ labels, int64_t n,
                                                                     int32_t k, int32_t kc, int32_t nch,
                                                                     int32_t* perm, int32_t* plab, int32_t* poff,
                                                                     int32_t* pcnt, const Ctrl* ctrl, int32_t iter)
{
    constexpr int G = kPartRows / (64 * kPartWaves);      // 64-sample groups per wave
    extern __shared__ __align__(16) unsigned char smem[];
    if (ctrl != nullptr && ctrl->stop_iter < iter) return;  // converged earlier
    int32_t* cntw = reinterpret_cast<int32_t*>(smem);    // [kPartWaves][nch]: counts, then cursors
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * kPartRows;
    const int64_t end = base + kPartRows < n ? base + kPartRows : n;
    const int64_t wbase = base + (int64_t)wave * 64 * G;
    for (int c = tid; c < kPartWaves * nch; c += 64 * kPartWaves) cntw[c] = 0;
    int lb[G], ch[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t i = wbase + g * 64 + lane;
        lb[g] = i < end ? labels[i] : -1;
    }
#pragma unroll
    for (int g = 0; g < G; ++g) ch[g] = (lb[g] >= 0 && lb[g] < k) ? lb[g] / kc : -1;
    __syncthreads();
    int32_t* mine = cntw + wave * nch;
    const int nbits = nch > 1 ? 32 - __builtin_clz((unsigned)(nch - 1)) : 0;
    const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int c = ch[g];
        uint64_t same = __ballot(c >= 0);
        for (int b = 0; b < nbits; ++b) {
            const bool bit = (c >> b) & 1;
            const uint64_t m = __ballot(bit);
            same &= bit ? m : ~m;
        }
        const int rank = (int)__popcll(same & lt), num = (int)__popcll(same);
        if (c >= 0) {
            if (rank == 0) __hip_atomic_fetch_add(mine + c, num, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            ch[g] = c | (rank << 16) | (num << 23);
        }
    }
    __syncthreads();
    if (wave == 0) {
        int carry = 0;
        for (int c0 = 0; c0 < nch; c0 += 64) {
            const int c = c0 + lane;
            int per[kPartWaves];
            int v = 0;
#pragma unroll
            for (int w = 0; w < kPartWaves; ++w) {
                per[w] = c < nch ? cntw[w * nch + c] : 0;
                v += per[w];
            }
            int incl = v;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int o = __shfl_up(incl, off);
                if (lane >= off) incl += o;
            }
            if (c < nch) {
                const int start = (int)base + carry + incl - v;
                poff[(int64_t)blockIdx.x * nch + c] = start;
                pcnt[(int64_t)blockIdx.x * nch + c] = v;
                int at = start;
#pragma unroll
                for (int w = 0; w < kPartWaves; ++w) {
                    cntw[w * nch + c] = at;
                    at += per[w];
                }
            }
            carry += __shfl(incl, 63);
        }
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int c = ch[g] >= 0 ? (ch[g] & 0xffff) : -1;
        const int rank = (ch[g] >> 16) & 127, num = ch[g] >> 23;
        const int at = c >= 0 ? mine[c] : 0;
        if (c >= 0) {
            perm[at + rank] = (int32_t)(wbase + g * 64 + lane);
            plab[at + rank] = lb[g];
            if (rank == 0) mine[c] = at + num;
        }
    }
}

hipError_t launch_partition(const PassArgs& a, int32_t* perm, int32_t* plab, int32_t* poff, int32_t* pcnt,
                            hipStream_t s)
{
    const size_t lds4 = (size_t)kPartWaves * a.nch * sizeof(int32_t);
    if (lds4 <= 64 * 1024) {
        hipLaunchKernelGGL(partition4_kernel, dim3(a.nsub), dim3(64 * kPartWaves), lds4, s, a.labels, a.n, a.k, a.kc,
                           a.nch, perm, plab, poff, pcnt, a.ctrl, a.iter);
        return hipGetLastError();
    }
    const size_t lds = 2 * (size_t)a.nch * sizeof(int32_t);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&partition_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(partition_kernel, dim3(a.nsub), dim3(64), lds, s, a.labels, a.n, a.k, a.kc, a.nch, perm,
                       plab, poff, pcnt, a.ctrl, a.iter);
    return hipGetLastError();
}

template <int D8>
static hipError_t launch_part_d8(const PassArgs& a, dim3 grid, size_t lds, hipStream_t s)
{
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&part_update_kernel<D8>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((part_update_kernel<D8>), grid, dim3(kBlock), lds, s, a);
    return hipGetLastError();
}

template <int D8>
static int part_occ_d8(size_t lds)
{
    if (lds > 64 * 1024 &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(&part_update_kernel<D8>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return -1;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, part_update_kernel<D8>, kBlock, lds) != hipSuccess)
        return -1;
    return nb;
}

hipError_t launch_part_update(int D8, const PassArgs& a, dim3 grid, size_t lds, hipStream_t s)
{
    switch (D8) {
#define KM_PU(N) case N: return launch_part_d8<N>(a, grid, lds, s);
    KM_PU(1) KM_PU(2) KM_PU(3) KM_PU(4) KM_PU(5) KM_PU(6) KM_PU(7) KM_PU(8)
    KM_PU(9) KM_PU(10) KM_PU(11) KM_PU(12) KM_PU(13) KM_PU(14) KM_PU(15) KM_PU(16)
#undef KM_PU
    default: return hipErrorInvalidValue;
    }
}

int part_update_blocks_per_cu(int D8, size_t lds)
{
    switch (D8) {
#define KM_PO(N) case N: return part_occ_d8<N>(lds);
    KM_PO(1) KM_PO(2) KM_PO(3) KM_PO(4) KM_PO(5) KM_PO(6) KM_PO(7) KM_PO(8)
    KM_PO(9) KM_PO(10) KM_PO(11) KM_PO(12) KM_PO(13) KM_PO(14) KM_PO(15) KM_PO(16)
#undef KM_PO
    default: return -1;
    }
}

template <int D8, int MODE>
static hipError_t allow_lds(size_t lds)
{
    // Dynamic LDS above 64 KiB must be opted into per kernel (gfx950 has 160 KiB per CU).
    if (lds <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&plain_pass<D8, MODE>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int D8>
static hipError_t launch_d8(Mode mode, const PassArgs& a, dim3 grid, size_t lds, hipStream_t s)
{
    hipError_t e = hipSuccess;
    switch (mode) {
    case MODE_ASSIGN: e = allow_lds<D8, MODE_ASSIGN>(lds); break;
    case MODE_UPDATE: e = allow_lds<D8, MODE_UPDATE>(lds); break;
    case MODE_FUSED:  e = allow_lds<D8, MODE_FUSED>(lds); break;
    }
    if (e != hipSuccess) return e;
    switch (mode) {
    case MODE_ASSIGN: hipLaunchKernelGGL((plain_pass<D8, MODE_ASSIGN>), grid, dim3(kBlock), lds, s, a); break;
    case MODE_UPDATE: hipLaunchKernelGGL((plain_pass<D8, MODE_UPDATE>), grid, dim3(kBlock), lds, s, a); break;
    case MODE_FUSED:  hipLaunchKernelGGL((plain_pass<D8, MODE_FUSED>), grid, dim3(kBlock), lds, s, a); break;
    }
    return hipGetLastError();
}

template <int D8>
static int occupancy_d8(Mode mode, size_t lds)
{
    int nb = 0;
    hipError_t e = hipSuccess;
    switch (mode) {
    case MODE_ASSIGN: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, plain_pass<D8, MODE_ASSIGN>, kBlock, lds); break;
    case MODE_UPDATE: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, plain_pass<D8, MODE_UPDATE>, kBlock, lds); break;
    case MODE_FUSED:  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, plain_pass<D8, MODE_FUSED>, kBlock, lds); break;
    }
    return e == hipSuccess ? nb : -1;
}

int plain_blocks_per_cu(int D8, Mode mode, size_t lds)
{
    switch (D8) {
#define KM_OCC(N) case N: return occupancy_d8<N>(mode, lds);
    KM_OCC(1) KM_OCC(2) KM_OCC(3) KM_OCC(4) KM_OCC(5) KM_OCC(6) KM_OCC(7) KM_OCC(8)
    KM_OCC(9) KM_OCC(10) KM_OCC(11) KM_OCC(12) KM_OCC(13) KM_OCC(14) KM_OCC(15) KM_OCC(16)
#undef KM_OCC
    default: return -1;
    }
}

template <int D8, int MODE>
static hipError_t launch_batch_mode(const BatchWork* work, int nwork, const PassArgs* insts, int iter, size_t lds,
                                    hipStream_t s)
{
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&batch_pass<D8, MODE>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((batch_pass<D8, MODE>), dim3(nwork), dim3(kBlock), lds, s, work, insts, iter);
    return hipGetLastError();
}

template <int D8>
static hipError_t launch_batch_d8(Mode mode, const BatchWork* work, int nwork, const PassArgs* insts, int iter,
                                  size_t lds, hipStream_t s)
{
    if (mode == MODE_UPDATE) return launch_batch_mode<D8, MODE_UPDATE>(work, nwork, insts, iter, lds, s);
    return launch_batch_mode<D8, MODE_FUSED>(work, nwork, insts, iter, lds, s);
}

hipError_t launch_batch_pass(int D8, Mode mode, const BatchWork* work, int nwork, const PassArgs* insts, int iter,
                             size_t lds, hipStream_t s)
{
    if (mode != MODE_FUSED && mode != MODE_UPDATE) return hipErrorInvalidValue;
    switch (D8) {
#define KM_BP(N) case N: return launch_batch_d8<N>(mode, work, nwork, insts, iter, lds, s);
    KM_BP(1) KM_BP(2) KM_BP(3) KM_BP(4) KM_BP(5) KM_BP(6) KM_BP(7) KM_BP(8)
    KM_BP(9) KM_BP(10) KM_BP(11) KM_BP(12) KM_BP(13) KM_BP(14) KM_BP(15) KM_BP(16)
#undef KM_BP
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_plain_pass(int D8, Mode mode, const PassArgs& a, dim3 grid, size_t lds, hipStream_t s)
{
    switch (D8) {
    case 1: return launch_d8<1>(mode, a, grid, lds, s);
    case 2: return launch_d8<2>(mode, a, grid, lds, s);
    case 3: return launch_d8<3>(mode, a, grid, lds, s);
    case 4: return launch_d8<4>(mode, a, grid, lds, s);
    case 5: return launch_d8<5>(mode, a, grid, lds, s);
    case 6: return launch_d8<6>(mode, a, grid, lds, s);
    case 7: return launch_d8<7>(mode, a, grid, lds, s);
    case 8: return launch_d8<8>(mode, a, grid, lds, s);
    case 9: return launch_d8<9>(mode, a, grid, lds, s);
    case 10: return launch_d8<10>(mode, a, grid, lds, s);
    case 11: return launch_d8<11>(mode, a, grid, lds, s);
    case 12: return launch_d8<12>(mode, a, grid, lds, s);
    case 13: return launch_d8<13>(mode, a, grid, lds, s);
    case 14: return launch_d8<14>(mode, a, grid, lds, s);
    case 15: return launch_d8<15>(mode, a, grid, lds, s);
    case 16: return launch_d8<16>(mode, a, grid, lds, s);
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------ persistent batch
// One block finalizes one instance: each element sums the instance's partial
// slots in slot order (as batch_finalize_kernel), divides in FP64, rounds
// once; wave 0 also reduces the objective partials (lane-strided, xor tree).
__device__ __forceinline__ void persist_finalize(const FinArgs& a, const float* __restrict__ c_old, float* c_next,
                                                 int32_t iter)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t kd = (int64_t)a.k * a.d;
    for (int64_t e = tid; e < kd; e += kBlock) {
        const int j = (int)(e / a.d);
        const int f = (int)(e - (int64_t)j * a.d);
        double S = 0.0;
        int64_t c = 0;
        for (int b = 0; b < a.G; ++b) {
            S += a.part.S[(size_t)b * kd + e];
            c += a.part.cnt[(size_t)b * a.k + j];
        }
        const float old = c_old[(size_t)j * a.D + f];
        const float v = (c > 0) ? (float)(S / (double)c) : old;
        a.C_new[(size_t)j * a.ld_new + f] = v;
        c_next[(size_t)j * a.D + f] = v;
        if (a.counts && f == 0) a.counts[j] = c;
    }
    // the padding columns of the next buffer stay zero
    for (int64_t e = tid; e < (int64_t)a.k * a.D; e += kBlock) {
        const int f = (int)(e % a.D);
        if (f >= a.d) c_next[e] = 0.0f;
    }
    if (wave == 0) {
        double J = 0.0;
        for (int b = lane; b < a.GJ; b += 64) J += a.part.J[b];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) J += __shfl_xor(J, off);
        if (lane == 0 && a.obj_hist) a.obj_hist[iter] = J;
    }
}

template <int D8>
__device__ __forceinline__ void persist_pass(const PassArgs& a, const BatchWork& w, unsigned char* smem)
{
    pass_body<D8, MODE_FUSED>(a, w.t0, w.t1, 1, w.slot, 0, smem);
}

__global__ __launch_bounds__(kBlock) void batch_persistent_kernel(PersistArgs p)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int64_t s_q;
    __shared__ int32_t s_flag;
    const int tid = threadIdx.x;
    const int64_t total = (int64_t)p.iters * p.nwork;
    for (;;) {
        if (tid == 0) {
            const bool stop = __hip_atomic_load(&p.ctrl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            s_q = stop ? total : __hip_atomic_fetch_add(&p.ctrl->head, (int64_t)1, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        const int64_t q = s_q;
        if (q >= total) break;                       // queue drained (or aborted): every wave leaves
        const int u = (int)(q / p.nwork);
        const BatchWork w = p.work[q - (int64_t)u * p.nwork];
        const int i = w.inst;
        // wait until instance i has published the centroids of iteration u
        if (tid == 0) {
            int64_t spins = 0;
            int ok = 1;
            while (__hip_atomic_load(&p.ready[i], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < u) {
                if (++spins > p.spin_limit ||
                    __hip_atomic_load(&p.ctrl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            if (!ok) __hip_atomic_store(&p.ctrl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_flag = ok;
        }
        __syncthreads();
        if (!s_flag) break;
        PassArgs a = p.insts[i];
        a.Cp = p.ring[i] + (int64_t)u * p.ring_stride[i];
        a.iter = p.it0 + u;
        switch ((a.d + 7) / 8) {
        case 1: persist_pass<1>(a, w, smem); break;
        case 2: persist_pass<2>(a, w, smem); break;
        case 3: persist_pass<3>(a, w, smem); break;
        case 4: persist_pass<4>(a, w, smem); break;
        case 5: persist_pass<5>(a, w, smem); break;
        case 6: persist_pass<6>(a, w, smem); break;
        case 7: persist_pass<7>(a, w, smem); break;
        default: persist_pass<8>(a, w, smem); break;
        }
        __threadfence();                             // every thread's part of the partial slot, then
        __syncthreads();                             // the count (the last block of a grid pattern)
        if (tid == 0) {
            const int32_t old = __hip_atomic_fetch_add(&p.done[i], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            s_flag = (old == p.nslots[i] - 1);
        }
        __syncthreads();
        if (s_flag) {
            // the last work row of (instance i, iteration u): finalize it
            __threadfence();
            const FinArgs& f = p.fins[i];
            const float* c_old = p.ring[i] + (int64_t)u * p.ring_stride[i];
            float* c_next = p.ring[i] + (int64_t)(u + 1) * p.ring_stride[i];
            persist_finalize(f, c_old, c_next, p.it0 + u);
            __threadfence();                         // the new centroids, then their publication
            __syncthreads();
            if (tid == 0) {
                __hip_atomic_store(&p.done[i], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&p.ready[i], u + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();                             // s_q / s_flag are rewritten next round
    }
}

// Block per instance (block 0 also resets the queue): done = ready = 0 and C
// padded into the first ring buffer.
__global__ __launch_bounds__(256) void persist_reset_kernel(PersistArgs p)
{
    const int i = blockIdx.x;
    if (i == 0 && threadIdx.x == 0) {
        p.ctrl->head = 0;
        p.ctrl->abort = 0;
    }
    if (threadIdx.x == 0) {
        p.done[i] = 0;
        p.ready[i] = 0;
    }
    const FinArgs& f = p.fins[i];
    float* c0 = p.ring[i];
    const int64_t total = (int64_t)f.k * f.D;
    for (int64_t e = threadIdx.x; e < total; e += 256) {
        const int j = (int)(e / f.D);
        const int fe = (int)(e - (int64_t)j * f.D);
        c0[e] = (fe < f.d) ? f.C_new[(size_t)j * f.ld_new + fe] : 0.0f;
    }
}

hipError_t launch_persist_reset(const PersistArgs& a, int ninst, hipStream_t s)
{
    hipLaunchKernelGGL(persist_reset_kernel, dim3(ninst), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_batch_persistent(const PersistArgs& a, int grid, size_t lds, hipStream_t s)
{
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&batch_persistent_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(batch_persistent_kernel, dim3(grid), dim3(kBlock), lds, s, a);
    return hipGetLastError();
}

int persistent_blocks_per_cu(size_t lds)
{
    if (lds > 64 * 1024 &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(&batch_persistent_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return -1;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_persistent_kernel, kBlock, lds) != hipSuccess) return -1;
    return nb;
}

}  // namespace km

