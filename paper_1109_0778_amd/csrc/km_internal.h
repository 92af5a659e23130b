// Internal declarations shared by the host API and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace km {

// Plain-path launch geometry: one sample per lane, 256 lanes per block.
constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxD8Plain = 16;       // plain path: d <= 128 (eight-feature chunks)

// Finalize geometry: 64 elements per block; the partial slots are split
// kFinSplit ways in a first stage, whose sums a second stage adds in order.
constexpr int kFinSplit = 16;

enum Mode : int { MODE_ASSIGN = 0, MODE_UPDATE = 1, MODE_FUSED = 2 };

// Device control block of one plan (lives at the head of the workspace).
struct Ctrl {
    int32_t stop_iter;    // iteration at which a tolerance stop was decided (INT32_MAX: none)
    int32_t iters_done;   // iterations completed
    int32_t bad_labels;   // update-only calls: labels outside [0, k) seen
    int32_t pad0;
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
    int32_t* bad;       // [G]      invalid-label partials (update-only)
};

struct PassArgs {
    const float* X;       // [n x d]
    const float* Cp;      // [k x D] centroids, rows zero-padded to D = 8 * D8
    int32_t* labels;      // [n]
    float* mindist;       // [n] or nullptr
    Partials part;
    const Ctrl* ctrl;     // nullptr outside kmeans_lloyd
    int64_t n;
    int32_t d;
    int32_t k;
    int32_t iter;         // Lloyd iteration index (0 outside kmeans_lloyd)
};

struct FinArgs {
    Partials part;
    double* stageS;       // [kFinSplit][k*d] first-stage sums
    int32_t* stageC;      // [kFinSplit][k*d] first-stage counts (per element)
    int32_t G;            // number of partial slots
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
};

// Launchers (return the launch status).
hipError_t launch_pad_centroids(const float* C, int32_t k, int32_t d, int32_t D, float* Cp,
                                Ctrl* ctrl_reset, hipStream_t s);
hipError_t launch_plain_pass(int D8, Mode mode, const PassArgs& a, int grid, size_t lds_bytes,
                             hipStream_t s);
hipError_t launch_finalize(const FinArgs& a, hipStream_t s);
// Resident blocks per CU of the plain pass (HIP occupancy query), -1 on error.
int plain_blocks_per_cu(int D8, Mode mode, size_t lds_bytes);
hipError_t launch_reduce_objective(const double* part_J, int32_t G, double* out, hipStream_t s);
hipError_t launch_copy_i32(const int32_t* src, int32_t* dst, int32_t n, hipStream_t s);

// Samples per lane in the plain pass.  One: measured on MI355X at d = 64,
// k = 64, two samples per lane (sharing each SGPR centroid operand) ran 18%
// slower (3 instead of 4 resident waves per SIMD), and LDS-broadcast centroid
// operands 13% slower than SGPR operands.
constexpr int plain_rows_per_lane(int) { return 1; }
inline int plain_tile(int D8) { return kBlock * plain_rows_per_lane(D8); }

// LDS bytes the plain pass needs for given k, d (activation record + label buffers).
inline size_t plain_lds_bytes(int k, int d, Mode mode)
{
    size_t b = 0;
    if (mode != MODE_ASSIGN) {
        b += (size_t)k * (size_t)d * sizeof(double);
        b += ((size_t)k * sizeof(int32_t) + 15) & ~(size_t)15;
        b += 2 * (size_t)kBlock * 2 * sizeof(int32_t);
    }
    return b;
}

}  // namespace km
