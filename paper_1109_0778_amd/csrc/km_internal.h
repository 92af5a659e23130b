// Internal declarations shared by the host API and the gfx950 kernels.
#pragma once

#include "kmeans_mi355x.h"

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace km {

// Plain-path launch geometry: one sample per lane, 256 lanes per block.
constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxD8Plain = 16;       // plain path: d <= 128 (eight-feature chunks)

// Per-sample pass variants: assign only; update from stored labels with the
// fused pass's tiles (so the two give bit-identical sums); fused assign +
// update; update over label chunks with wider tiles (records beyond LDS).
enum Mode : int { MODE_ASSIGN = 0, MODE_UPDATE = 1, MODE_FUSED = 2 };

// Device control block of one plan (lives at the head of the workspace).
struct Ctrl {
    int32_t stop_iter;    // iteration at which a tolerance stop was decided (INT32_MAX: none)
    int32_t iters_done;   // iterations completed
    int32_t pad0, pad2;
    double J_prev;        // objective of the previous iteration
    int64_t changed_last; // labels changed in the last completed iteration
    double pad1[12];
};
static_assert(sizeof(Ctrl) <= 256, "control block must fit 256 bytes");

// Per-block partial records written by the fused pass, reduced by finalize.
struct Partials {
    double* S;          // [G][k*d] per-label FP64 sums
    int32_t* cnt;       // [G][k]   per-label counts
    double* J;          // [G]      objective partials
    int32_t* changed;   // [G]      changed-label partials
};

struct PassArgs {
    const float* X;       // [n x d]
    const float* Cp;      // [k x D] centroids, rows zero-padded to D = 8 * D8
    int32_t* labels;      // [n]
    float* mindist;       // [n] or nullptr
    Partials part;
    const Ctrl* ctrl;     // early-exit control (tolerance mode), or nullptr
    int64_t n;
    int32_t d;            // features of the pass (a slice of the row when rows are reduced in slices)
    int32_t k;
    int32_t ldx;          // row stride of X (the full row length)
    int32_t iter;         // Lloyd iteration index (0 outside kmeans_lloyd)
    int32_t count_changed;// assign passes: count labels that differ from the stored ones
    int32_t kc;           // update passes: labels per chunk; block y owns labels [y*kc, y*kc+kc)
    int32_t upd_tiles;    // update pass: tiles listed and added per step (1 .. kUpdTiles); above 1 each
                          // block walks a contiguous range of tiles
    // partitioned chunk update: sample indices grouped by label chunk within
    // each kPartRows-sample sub-range, in sample order
    const int32_t* perm;  // [n]
    const int32_t* plab;  // [n] label of sample perm[i]
    const int32_t* poff;  // [nsub][nch] start of (sub-range, chunk) in perm
    const int32_t* pcnt;  // [nsub][nch] its length
    int32_t nsub, nch;
};

constexpr int kPartRows = 4096;   // samples per partition sub-range
constexpr int kPartMaxChunks = 16384;   // partition LDS: 2 ints per chunk

// One block of a batched per-sample pass.
struct BatchWork {
    int32_t inst;         // instance index
    int32_t slot;         // partial slot of the instance
    int64_t t0, t1;       // tiles [t0, t1) of the instance
};

struct FinArgs {
    Partials part;
    int32_t G;            // number of per-label partial slots (sums, counts)
    int32_t GJ;           // number of objective / changed partial slots
    int32_t k, d, D;
    const float* C_old; int32_t ld_old;   // centroids kept for empty clusters
    float* C_new;       int32_t ld_new;   // output centroids
    float* Cp_out;                        // padded copy for the next pass, or nullptr
    int64_t* counts;                      // [k] or nullptr
    Ctrl* ctrl;                           // nullptr outside kmeans_lloyd
    double* obj_hist;                     // [max_iter] or nullptr
    int32_t iter;
    double tol;                           // < 0: fixed iteration count
    int32_t want_J;                       // reduce J / changed / control
    // objective: jmode 0 sums the per-sample partials part.J[0..GJ);
    // jmode 1 uses J = sum_i |x_i|^2 + sum_j (cnt_j |c_j|^2 - 2 c_j . S_j)
    // (exact algebra on the reduce's own FP64 sums), with *sum_xn2 the first
    // term and Jterm[] the per-block second term.
    int32_t jmode;
    double* Jterm;                        // [ceil(k*d/64)] (jmode 1)
    const double* sum_xn2;                // (jmode 1)
    int32_t GC;                           // changed partial slots in part.changed
    double* S_out;                        // [k x ld_S] combined FP64 sums, or nullptr
    int32_t ld_S;                         // row stride of S_out
    int32_t jt_off;                       // (jmode 1) this launch's first block in Jterm
    int32_t nJterm;                       // (jmode 1) Jterm entries the objective sums (0: this launch's)
};

// Launchers (return the launch status).
hipError_t launch_pad_centroids(const float* C, int32_t k, int32_t d, int32_t D, float* Cp,
                                Ctrl* ctrl_reset, hipStream_t s);
hipError_t launch_plain_pass(int D8, Mode mode, const PassArgs& a, dim3 grid, size_t lds_bytes,
                             hipStream_t s);
hipError_t launch_finalize(const FinArgs& a, hipStream_t s);
__host__ __device__ inline int finalize_blocks(int k, int d) { return (int)(((int64_t)k * d + 63) / 64); }
// Batched per-sample pass (mode FUSED, or UPDATE from the labels a mixed
// assign wrote) over a work table.
hipError_t launch_batch_pass(int D8, Mode mode, const BatchWork* work, int nwork, const PassArgs* insts, int iter,
                             size_t lds_bytes, hipStream_t s);
// Batched finalize: one block per (instance, 64 elements); with jmode 1 each
// block writes its Jterm share and launch_batch_objective (one wave per
// instance) forms the objective.  batch_pad pads the instances' centroids at
// the start of a call.
struct BatchFinWork { int32_t inst; int32_t chunk; };

// Persistent batched FP32 Lloyd (one launch for up to kPersistIters
// iterations of every instance).  Resident blocks take items (iteration u,
// work row w) from a queue in iteration-major order; a block runs the fused
// pass of its item once the item's instance has published the centroids of
// iteration u; the block that completes an instance's last item of an
// iteration combines that instance's partial slots (finalize, same order as
// batch_finalize_kernel) and publishes iteration u + 1.  Waits are bounded:
// past `spin_limit` polls the launch sets `abort` and every block exits.
constexpr int kPersistIters = 32;      // iterations per launch (centroid buffers per instance: + 1)
struct PersistCtrl {
    int64_t head;         // next queue index
    int32_t abort;        // a wait exceeded its bound
    int32_t pad[13];
};
struct PersistArgs {
    const BatchWork* work;    // [nwork] work rows of one iteration, every instance
    int32_t nwork;
    int32_t iters;            // iterations of this launch
    int32_t it0;              // iteration index of the launch's first iteration
    const PassArgs* insts;    // [m] per instance (Cp replaced by the ring below)
    const FinArgs* fins;      // [m] per instance (C_old / Cp_out replaced by the ring)
    float* const* ring;       // [m] base of kPersistIters + 1 padded centroid buffers
    const int64_t* ring_stride;  // [m] floats between consecutive buffers
    const int32_t* nslots;    // [m] partial slots (work rows) per instance per iteration
    int32_t* done;            // [m] work rows finished in the current iteration
    int32_t* ready;           // [m] iterations whose centroids are published
    PersistCtrl* ctrl;
    int64_t spin_limit;
};
hipError_t launch_batch_persistent(const PersistArgs& a, int grid, size_t lds, hipStream_t s);
int persistent_blocks_per_cu(size_t lds);
// Reset of a persistent launch (head, abort, done, ready) and the padding of
// every instance's C into its first ring buffer.
hipError_t launch_persist_reset(const PersistArgs& a, int ninst, hipStream_t s);
hipError_t launch_batch_finalize(const BatchFinWork* work, int nwork, const FinArgs* fa, int iter, hipStream_t s);
hipError_t launch_batch_objective(const FinArgs* fa, int ninst, int iter, hipStream_t s);
hipError_t launch_batch_pad(const FinArgs* fa, const float* const* C_in, int ninst, hipStream_t s);
// Resident blocks per CU of the plain pass (HIP occupancy query), -1 on error.
int plain_blocks_per_cu(int D8, Mode mode, size_t lds_bytes);
// Partitioned chunk update: partition (one wave per sub-range), then blocks
// (point range x, label chunk y) over their samples only.
size_t part_update_lds_bytes(int kc, int d);
int part_update_blocks_per_cu(int D8, size_t lds_bytes);
hipError_t launch_partition(const PassArgs& a, int32_t* perm, int32_t* plab, int32_t* poff, int32_t* pcnt,
                            hipStream_t s);
hipError_t launch_part_update(int D8, const PassArgs& a, dim3 grid, size_t lds_bytes, hipStream_t s);
hipError_t launch_reduce_objective(const double* part_J, int32_t G, double* out, hipStream_t s);
hipError_t launch_copy_i32(const int32_t* src, int32_t* dst, int32_t n, hipStream_t s);
// Labels outside [0, k): per-block counts of a grid-stride scan (grid <= nblk
// blocks), written to part[0 .. grid); returns the grid used.
hipError_t launch_count_bad_labels(const int32_t* labels, int64_t n, int32_t k, int32_t* part, int nblk,
                                   int* grid_used, hipStream_t s);

// Section 4.2 applications on the per-class reduce: naive Bayes finalize
// (in place on the class sums and counts) and GDA (means in place, then the
// shared covariance from per-block 64 x 64 partial regions).
struct CovArgs {
    const float* X;          // [n x d]
    const int32_t* labels;   // [n] classes in [0, k)
    double* prior;           // [k] counts (int64) in, priors out
    double* mu;              // [k x d] sums in, means out
    double* sigma;           // [d x d] output
    double* part;            // [G][RP][64][64] partial regions
    int64_t n;
    int32_t d, k;
    int32_t R, RP, G;        // 64-feature regions, upper-triangle region pairs, sample ranges
};
hipError_t launch_nb_finalize(double* prior, double* phi, int32_t k, int32_t d, int64_t n, hipStream_t s);
hipError_t launch_gda_means(const CovArgs& a, int32_t k, hipStream_t s);
hipError_t launch_gda_cov(const CovArgs& a, hipStream_t s);
hipError_t launch_gda_combine(const CovArgs& a, hipStream_t s);

// Assign under a chosen metric (0 = L1, 1 = squared Euclidean) and sample
// layout (0 = row-major n x d, 1 = feature-major d x n).
struct MetricArgs {
    const float* X;
    const float* Cp;         // [k x 8 D8] padded centroids
    int32_t* labels;         // [n]
    float* mindist;          // [n] or nullptr
    double* partJ;           // [grid] per-block FP64 sums of the chosen distances
    int64_t n;
    int32_t d, k;
};
hipError_t launch_assign_metric(int D8, int metric, int layout, const MetricArgs& a, int grid, hipStream_t s);
// Rows of more than 128 features: streaming assign with the plain path's
// canonical distance (the per-label reduce then runs over 128-feature slices).
constexpr int kSliceD = 128;
hipError_t launch_assign_wide(const PassArgs& a, int grid, hipStream_t s);
int wide_blocks_per_cu();

// Samples per lane in the plain pass.  One: measured on MI355X at d = 64,
// k = 64, two samples per lane (sharing each SGPR centroid operand) ran 18%
// slower (3 instead of 4 resident waves per SIMD), and LDS-broadcast centroid
// operands 13% slower than SGPR operands.
constexpr int plain_rows_per_lane(int) { return 1; }
inline int plain_tile(int D8) { return kBlock * plain_rows_per_lane(D8); }
// Lanes that carry one sample row in the per-label adds: a row of at most 16
// (32) features takes a quarter (half) wave, so one load and one LDS atomic
// instruction serve four (two) samples.
__host__ __device__ constexpr int row_lanes(int D8) { return D8 <= 2 ? 16 : D8 <= 4 ? 32 : 64; }
__host__ __device__ constexpr int row_groups(int D8) { return 64 / row_lanes(D8); }
// Each wave's owned-sample lists: two row groups share a buffer, one filling
// it from the front, the other from the back.
__host__ __device__ constexpr int list_bufs(int D8) { return (row_groups(D8) + 1) / 2; }
// Tiles the update pass lists and adds per step (the fused pass: one).
constexpr int kUpdTiles = 3;
// LDS bytes the plain pass needs for given k, d (activation record + label buffers).
inline size_t plain_lds_bytes(int k, int d, Mode mode, int upd_tiles = kUpdTiles)
{
    size_t b = 0;
    if (mode != MODE_ASSIGN) {
        b += ((size_t)k * (size_t)d + 1) / 2 * 2 * sizeof(double);   // the lists start 16-byte aligned
        b += ((size_t)k * sizeof(int32_t) + 15) & ~(size_t)15;
        // fused: labels of a tile, double-buffered, and each wave's owned
        // samples of a tile; update: each wave's owned samples of a step
        const size_t lists = (size_t)kWaves * list_bufs((d + 7) / 8) * kBlock;
        b += (mode == MODE_FUSED ? 2 * (size_t)kBlock + lists : (size_t)upd_tiles * lists) * sizeof(int32_t);
    }
    return b;
}

// ---------------------------------------------------------------- mixed path
// BF16 or FP8 MFMA distances with a proven error band and an exact FP32 recheck.
enum MixFmt { FMT_BF16 = 0, FMT_FP8 = 1 };
constexpr int kMixWaves = 4;                    // waves per block
constexpr int kMixNB = 1;                       // 32-sample column blocks per wave
constexpr int kMixTile = kMixWaves * kMixNB * 32;
// The screen (two smallest keys, no candidate lists) holds two column blocks
// per wave: each centroid fragment read from LDS feeds two MFMAs.
constexpr int kMixNBScreen = 2;
__host__ __device__ constexpr int mix_nb(int stage) { return stage == 1 || stage == 2 ? kMixNBScreen : kMixNB; }
// A plan whose centroid chunks stream through LDS (more than two, not all
// resident) runs its screens in blocks of 12 waves and its refine in blocks of
// 16, one block per CU, so every chunk brought into LDS serves three (four)
// times the samples; every other MFMA pass runs blocks of kMixWaves.
constexpr int kMixWavesScreenWide = 12;
constexpr int kMixWavesRefineWide = 16;
__host__ __device__ constexpr int mix_waves(int stage, bool wide_blocks)
{
    return !wide_blocks ? kMixWaves : stage == 3 ? kMixWavesRefineWide : (stage == 1 || stage == 2) ? kMixWavesScreenWide : kMixWaves;
}
__host__ __device__ constexpr int mix_tile(int stage, bool wide_blocks = false)
{
    return mix_waves(stage, wide_blocks) * mix_nb(stage) * 32;
}
constexpr int kMixCK = 64;                      // centroids per LDS chunk
// Candidates kept per lane (half a sample's rows).  Candidate lists are only
// built by BF16 sweeps (an FP8 plan's open samples get a BF16 screen first).
constexpr int kCandCap = 7;
constexpr int kCandSlots = kCandCap + 8;        // room for 8 appends
// Recheck entry: sample, count, 2 pad, then the candidate ids, 16-byte
// aligned and rounded up to a multiple of 8.
constexpr int kRqHead = 4;
constexpr int kRqInts = kRqHead + (2 * kCandCap + 7) / 8 * 8;
constexpr int kMaxD16Mix = 8;                   // operands held in registers / LDS up to d = 128
constexpr int kMaxD16Wide = 64;                 // beyond: operands streamed from memory, up to d = 1024
constexpr int kXStatBlocks = 256;
constexpr int kFmaxBlocks = 1024;               // FP8 per-feature maxima
constexpr int kRecheckSplit = 8;                // recheck blocks per MFMA block's queue region
constexpr float kFp8Max = 448.0f;               // largest finite e4m3 (OCP "fn") value

struct XStats {                 // once per run, over all samples
    float max_xn2;              // max_i |x_i|^2 (FP32)
    float K;                    // distance offset 2 max_i |x_i|^2 + 1 (keeps keys positive)
    double sum_xn2;             // sum_i |x_i|^2 (FP64)
};
struct CStats {                 // per iteration, over the centroids
    float K, cmax, cn2max;
    float inv2r;                // keys are kept as key / (2r): 1 for BF16, 2^-(e+1) for FP8
    float inv_r;                // 1 / r (FP8 centroid scale r = 2^e), 2 for BF16 (unused)
    float cl1;                  // FP8: max_j sum_f |c~_jf| of the scaled centroids
    float pad[2];
};

struct MixArgs {
    const float* X;
    int64_t n;
    int32_t d, k, kpad;
    const void* Ab;             // [kpad][16*D16] bf16(-2 c) or e4m3(-c~), zero padded
    const float* bias;          // [kpad] (K + |c_j|^2) / (2r), padded rows huge
    const uint8_t* Xq;          // FP8: [n][16*D16] e4m3(x / s_f), zero padded
    const float2* xst;          // FP8: per sample (|x| upper bound, sum_f |x_f / s_f| upper bound)
    const __bf16* Xb;           // BF16 passes: [n][16*D16] bf16(x), zero padded, or nullptr (convert X)
    const float* xn;            // with Xb: per sample |x| upper bound
    const CStats* cs;
    float u;                    // unit roundoff of the quantised format
    int32_t IB;                 // index bits in a key
    int32_t gamma_terms;        // m of the gamma_m accumulation bound
    int32_t D8;                 // chunks of the canonical FP32 distance
    int32_t DP;                 // padded operand width (16 * ceil(d / 16))
    int32_t* labels;
    int32_t* rq;                // [nreg][rq_per_block][rq_ints] recheck entries, one region per block
    int32_t* rq_count;          // [2][nreg] entries queued in each region, then full scans among them
    int64_t rq_per_block;       // region capacity (tiles per block x samples per tile)
    int32_t nreg;               // queue regions (one per MFMA block or work row)
    int32_t* changed_part;      // [nreg]
    int32_t* amb;               // stages 1, 2: [nreg][rq_per_block] samples left open
    int32_t* amb_count;         // stages 1, 2: [nreg]
    const int32_t* amb_in;      // stages 2, 3: the previous screen's amb and amb_count
    const int32_t* amb_in_count;
    uint32_t* amb_key;          // stages 1, 2: [nreg][rq_per_block] smallest key of each listed sample
    const uint32_t* amb_key_in; // stage 3: the BF16 screen's amb_key (same operands, so the same keys)
    const Ctrl* ctrl;
    int32_t iter;
    int32_t count_changed;
    int32_t nbuf;               // LDS centroid chunk buffers: 0 or 2 stream the chunks through two
                                // buffers; the chunk count keeps every chunk for the whole block
    int32_t wide_blocks;        // 1: stages 1-3 launch in blocks of mix_waves(stage, true) waves
};

struct RecheckArgs {
    const float* X;
    const float* Cp;            // [k][8*D8] FP32 centroids (zero padded)
    int64_t n;
    int32_t d, k;
    const int32_t* rq;
    const int32_t* rq_count;    // [grid]; recheck block b takes region b
    int64_t rq_per_block;
    int32_t rq_ints;            // ints per entry
    int32_t nreg;               // queue regions; changed_part is [splits][nreg]
    int32_t* labels;
    int32_t* changed_part;      // [grid]
    const Ctrl* ctrl;
    int32_t iter;
    int32_t count_changed;
};
// Exact recheck of the mixed path for rows of more than 128 features.
hipError_t launch_recheck_wide(const RecheckArgs& a, int G, hipStream_t s);

hipError_t launch_prep_x(const float* X, int64_t n, int32_t d, float* part_max, double* part_sum,
                         XStats* xs, hipStream_t s);
// FP8 run-level prep: per-feature scales s_f (powers of two), the e4m3 copy
// of X and the per-sample band inputs.
hipError_t launch_prep_x_bf16(const float* X, int64_t n, int32_t d, int32_t DP, __bf16* Xb, float* xn, hipStream_t s);
hipError_t launch_prep_x_fp8(const float* X, int64_t n, int32_t d, int32_t DP, float* part_fmax, float* fscale,
                             uint8_t* Xq, float2* xst, hipStream_t s);
// Per-iteration centroid prep.  BF16 with part_cn2 (prep_c_blocks(kpad)
// floats): row blocks + a reduce; otherwise one block.
int prep_c_blocks(int kpad);
hipError_t launch_prep_c(int fmt, const float* Cp, int32_t k, int32_t d, int32_t D, int32_t kpad, int32_t DP,
                         const XStats* xs, const float* fscale, void* Ab, float* bias, CStats* cs, float* part_cn2,
                         const Ctrl* ctrl, int32_t iter, hipStream_t s);
// MFMA passes: stage 1 screens every sample (two smallest keys), stage 2
// (BF16) screens the samples an FP8 stage 1 listed, stage 3 (BF16) refines
// the samples the last BF16 screen listed (candidate lists inside the band
// of the screen's smallest key, recheck queue); stage 0 (the one-pass sweep
// with running candidate lists) serves short sweeps and the batched path.
hipError_t launch_mfma_assign(int fmt, int stage, int D16, const MixArgs& a, int grid, hipStream_t s);
// Chunk buffers for a plan's MFMA passes: every chunk when there are at
// least three and they fit in kMixResidentBytes, else two.  The bound keeps
// a refine block (operands + candidate lists) under 40 KiB, so the four
// blocks per CU the plans launch stay resident together.
constexpr int kMixResidentBytes = 24 * 1024;
int mix_buffers(int fmt, int D16, int kpad);
size_t mfma_lds_bytes(int fmt, int D16, int stage, int nbuf = 2, int waves = kMixWaves);
int mfma_blocks_per_cu(int fmt, int stage, int D16, int nbuf = 2, bool wide_blocks = false);
hipError_t launch_recheck(int D8, const RecheckArgs& a, int grid, int split, hipStream_t s);

// Batched mixed path: one record per instance.  The per-iteration prep and
// the |x| statistics run one block per instance; the MFMA pass and the
// recheck run over work tables (BatchWork: instance, queue region, tile range
// [t0, t1) of 128-sample tiles for the MFMA pass; instance, region, split t0
// of t1 splits for the recheck).
struct BatchMix {
    MixArgs m;
    RecheckArgs r;
    const float* Cp;            // [k][D] padded FP32 centroids
    int32_t D, DP;
    XStats* xs;
    float* xpart_max;           // [nxb] partials of the run-level statistics
    double* xpart_sum;          // [nxb]
    int32_t nxb;
};
constexpr int kPrepXRows = 4096;    // rows per block of the batched run-level statistics
// T fixed Lloyd iterations of a single-instance plan, enqueued on `stream`
// (no graph of its own, no host synchronisation); the batched call runs its
// instances of more than 128 features through it.
km_status plan_enqueue_fixed(km_plan* plan, const float* X, float* C, int32_t* labels, int64_t* counts,
                             double* obj_hist, int32_t iters, hipStream_t stream);
hipError_t launch_batch_prep_x(const BatchWork* xwork, int nxwork, const BatchMix* bm, int ninst, hipStream_t s);
hipError_t launch_batch_prep_c(const BatchMix* bm, int ninst, hipStream_t s);
hipError_t launch_batch_mfma(int D16, const BatchWork* work, int nwork, const BatchMix* bm, int iter, hipStream_t s);
hipError_t launch_batch_recheck(int D8, const BatchWork* work, int nwork, const BatchMix* bm, int iter, hipStream_t s);

}  // namespace km
