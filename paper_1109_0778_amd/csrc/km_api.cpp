// Host side of the C ABI declared in include/kmeans_mi355x.h: argument
// validation, plans and their workspaces, and the launch sequences.
#include "kmeans_mi355x.h"
#include "km_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace km;

namespace {

thread_local std::string g_err;

km_status fail(km_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

km_status hip_fail(hipError_t e, const char* what)
{
    return fail(KM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

// Shared with km_batch.cpp: record an error text for km_last_error().
km_status km_set_error(km_status st, const char* msg)
{
    g_err = msg;
    return st;
}

struct km_plan {
    int64_t n;
    int32_t d, k;
    km_precision prec;
    int device;
    int num_cu;
    int D8, D;           // padded feature count (8-feature chunks)
    bool wide = false;   // d > 128: streaming assign, per-label reduce over 128-feature slices
    int dsl = 0;         // features per reduce slice (d, or 128 when wide)
    int nsl = 1;         // reduce slices
    int D8s(int s) const { return (std::min(dsl, d - s * dsl) + 7) / 8; }
    int grid;            // blocks of the assign / fused pass (one resident wave)
    bool split;          // assign and reduce as two passes (the fused pass would lose occupancy)
    bool chunked;        // per-label record too large for one block: the reduce runs over label chunks
    int nsub = 0;        // chunked: partition sub-ranges (kPartRows samples each)
    size_t off_perm = 0, off_plab = 0, off_poff = 0, off_plen = 0;
    int kc, nch;         // update: labels per chunk, chunks
    int grid_upd;        // update: slots (point ranges) per chunk
    size_t lds_fused;    // dynamic LDS of the fused pass (whole record)
    size_t lds_upd;      // dynamic LDS of the update pass (one chunk of the record)
    int GS() const { return split ? grid_upd : grid; }
    // mixed precision (BF16 or FP8 MFMA + FP32 recheck)
    bool mixed = false;
    int fmt = FMT_BF16;
    bool cascade = false;   // screen + refine (longer centroid sweeps, and FP8); else one BF16 sweep
    // MFMA passes per iteration: one sweep; BF16 screen + refine; FP8 screen + BF16 screen + refine
    int mfma_passes() const { return !cascade ? 1 : fmt == FMT_FP8 ? 3 : 2; }
    int D16 = 0, DP = 0, kpad = 0, IB = 0;
    int upd_tiles = 1;   // update pass: tiles listed per step
    int grid_mfma = 0, grid_rc = 0;
    bool wide_blocks = false;   // MFMA stages 1-3 in blocks of mix_waves(stage, true) waves
    int rc_split = kRecheckSplit;   // recheck blocks per queue region
    int64_t rq_per_block = 0;
    size_t off_xs = 0, off_pxm = 0, off_pxs = 0, off_ab = 0, off_bias = 0, off_cs = 0, off_rq = 0,
           off_rqc = 0, off_jt = 0;
    size_t off_fsc = 0, off_pfm = 0, off_xq = 0, off_xst = 0;   // FP8 only
    size_t off_xb = 0, off_xn = 0;                              // BF16 copy of X and |x| bounds
    size_t off_ab16 = 0, off_bias16 = 0, off_cs16 = 0;           // FP8: BF16 operands of the refining pass
    size_t off_amb = 0, off_ambc = 0, off_ambk = 0;              // samples the screen left open, their keys
    size_t off_amb2 = 0, off_ambc2 = 0;                          // FP8: those the BF16 screen left open
    size_t off_pcn = 0;                                          // BF16: per-block max |c|^2
    // workspace
    unsigned char* ws;
    size_t ws_bytes;
    size_t off_ctrl, off_cp, off_pS, off_pcnt, off_pJ, off_pch, total;
    bool validate = false;   // kmeans_update checks its labels first (debug-validate mode)
    // optional per-launch timing of the per-sample pass
    std::vector<hipEvent_t> ev;   // 2 per launch
    int32_t ev_used = 0;
    bool untimed = false;    // set while a call must not record timing events
    bool timing_on() const { return !untimed && ev_used * 2 + 1 < (int32_t)ev.size(); }
    // optional graph of a whole kmeans_lloyd call, keyed by its arguments
    bool use_graph = false;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    struct GraphKey {
        const float* X; float* C; int32_t* labels; int64_t* counts; double* obj_hist;
        int32_t max_iter; double tol; int32_t ev_used;
        bool operator==(const GraphKey& o) const
        {
            return X == o.X && C == o.C && labels == o.labels && counts == o.counts && obj_hist == o.obj_hist &&
                   max_iter == o.max_iter && tol == o.tol && ev_used == o.ev_used;
        }
    } gkey{};
    void drop_graph()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        gexec = nullptr;
    }
    ~km_plan()
    {
        drop_graph();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

namespace {

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Labels per chunk of a chunked reduce: sums and count of a chunk within 44 KiB, so with the
// update pass's entry lists three blocks fit in a CU's 160 KiB of LDS.
int chunk_labels(int k, int d) { return std::max(1, std::min(k, (44 * 1024) / (8 * d + 4))); }

km_status check_plan(const km_plan* p)
{
    if (!p) return fail(KM_EINVAL, "plan is NULL");
    if (!p->ws) return fail(KM_EWORKSPACE, "no workspace bound to the plan (km_plan_set_workspace)");
    return KM_OK;
}

Partials partials_of(const km_plan* p)
{
    Partials pt;
    pt.S = reinterpret_cast<double*>(p->ws + p->off_pS);
    pt.cnt = reinterpret_cast<int32_t*>(p->ws + p->off_pcnt);
    pt.J = reinterpret_cast<double*>(p->ws + p->off_pJ);
    pt.changed = reinterpret_cast<int32_t*>(p->ws + p->off_pch);
    return pt;
}

// Launch the per-sample pass, bracketed by timing events when enabled.
hipError_t timed_pass(km_plan* p, Mode mode, const PassArgs& a, dim3 grid, size_t lds, hipStream_t s)
{
    const bool timed = p->timing_on();
    hipError_t e;
    if (timed && (e = hipEventRecord(p->ev[2 * p->ev_used], s)) != hipSuccess) return e;
    e = p->wide ? launch_assign_wide(a, (int)grid.x, s) : launch_plain_pass(p->D8, mode, a, grid, lds, s);
    if (e != hipSuccess) return e;
    if (timed) {
        if ((e = hipEventRecord(p->ev[2 * p->ev_used + 1], s)) != hipSuccess) return e;
        ++p->ev_used;
    }
    return hipSuccess;
}

PassArgs pass_args(const km_plan* p, const float* X, const float* Cp, int32_t* labels)
{
    PassArgs a{};
    a.X = X; a.Cp = Cp; a.labels = labels; a.mindist = nullptr;
    a.part = partials_of(p); a.ctrl = nullptr;
    a.n = p->n; a.d = p->d; a.ldx = p->d; a.k = p->k; a.iter = 0; a.count_changed = 0; a.kc = p->kc;
    a.upd_tiles = p->upd_tiles;
    if (p->chunked) {
        a.perm = reinterpret_cast<const int32_t*>(p->ws + p->off_perm);
        a.plab = reinterpret_cast<const int32_t*>(p->ws + p->off_plab);
        a.poff = reinterpret_cast<const int32_t*>(p->ws + p->off_poff);
        a.pcnt = reinterpret_cast<const int32_t*>(p->ws + p->off_plen);
        a.nsub = p->nsub;
        a.nch = p->nch;
    }
    return a;
}

FinArgs fin_args(const km_plan* p)
{
    FinArgs f{};
    f.part = partials_of(p);
    f.G = p->GS(); f.GJ = p->grid; f.k = p->k; f.d = p->d; f.D = p->D; f.ld_S = p->d;
    f.tol = -1.0;
    f.jmode = p->mixed ? 1 : 0;
    f.Jterm = reinterpret_cast<double*>(p->ws + p->off_jt);
    f.sum_xn2 = p->mixed ? &reinterpret_cast<const XStats*>(p->ws + p->off_xs)->sum_xn2 : nullptr;
    f.GC = p->mixed ? p->mfma_passes() * p->grid_mfma + p->grid_rc : p->grid;
    return f;
}

// The reduce from stored labels: one pass (whole record) or a 2-D grid of
// label chunks (after the samples are partitioned by chunk, unless
// `partitioned`).  D8: 8-feature chunks of the pass's rows.
hipError_t enqueue_update(km_plan* p, const PassArgs& a, int D8, bool partitioned, hipStream_t s)
{
    // without a split, the update walks exactly the fused pass's blocks and tiles
    if (!p->split) return launch_plain_pass(D8, MODE_UPDATE, a, dim3(p->grid), p->lds_upd, s);
    if (!p->chunked) return launch_plain_pass(D8, MODE_UPDATE, a, dim3(p->grid_upd, p->nch), p->lds_upd, s);
    // label chunks: partition the samples by chunk, then reduce each chunk's samples
    if (!partitioned) {
        hipError_t e = launch_partition(a, reinterpret_cast<int32_t*>(p->ws + p->off_perm),
                                        reinterpret_cast<int32_t*>(p->ws + p->off_plab),
                                        reinterpret_cast<int32_t*>(p->ws + p->off_poff),
                                        reinterpret_cast<int32_t*>(p->ws + p->off_plen), s);
        if (e != hipSuccess) return e;
    }
    return launch_part_update(D8, a, dim3(p->grid_upd, p->nch), p->lds_upd, s);
}

// The reduce from stored labels and its finalize.  Rows of more than 128
// features are reduced and finalized in 128-feature slices (the sums of a
// feature depend on that feature's column only); the counts come with the
// first slice, the objective and the stop decision with the last.
hipError_t enqueue_reduce_finalize(km_plan* p, const PassArgs& a, const FinArgs& f, hipStream_t s)
{
    hipError_t e;
    if (!p->wide) {
        if ((e = enqueue_update(p, a, p->D8, false, s)) != hipSuccess) return e;
        return launch_finalize(f, s);
    }
    int jt = 0;
    for (int sl = 0; sl < p->nsl; ++sl) {
        const int c0 = sl * p->dsl, w = std::min(p->dsl, p->d - c0);
        PassArgs as = a;
        as.X = a.X + c0;
        as.d = w;
        if ((e = enqueue_update(p, as, p->D8s(sl), sl > 0, s)) != hipSuccess) return e;
        FinArgs fs = f;
        fs.d = w;
        fs.C_old = f.C_old ? f.C_old + c0 : nullptr;
        fs.C_new = f.C_new ? f.C_new + c0 : nullptr;
        fs.Cp_out = f.Cp_out ? f.Cp_out + c0 : nullptr;
        fs.S_out = f.S_out ? f.S_out + c0 : nullptr;
        fs.counts = sl == 0 ? f.counts : nullptr;
        fs.want_J = sl == p->nsl - 1 ? f.want_J : 0;
        // (mixed plans) each slice's objective terms go to their own Jterm
        // entries, and the last slice's objective sums all of them
        fs.jt_off = jt;
        jt += finalize_blocks(p->k, w);
        fs.nJterm = jt;
        if ((e = launch_finalize(fs, s)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// Mixed path: the screening MFMA pass (the plan's format), the BF16 refining
// pass over the samples it left open (both timed, as one), and the exact
// recheck of the refining pass's queue.  Short sweeps (k <= 128, BF16) run
// one pass that keeps candidate lists for every sample instead.
hipError_t enqueue_mixed_assign(km_plan* p, const float* X, int32_t* labels, const Ctrl* ctrl, int iter,
                                int count_changed, hipStream_t s)
{
    unsigned char* ws = p->ws;
    int32_t* changed = reinterpret_cast<int32_t*>(ws + p->off_pch);
    const bool f8 = p->fmt == FMT_FP8;
    const int G = p->grid_mfma;
    const float* Cp = reinterpret_cast<const float*>(ws + p->off_cp);
    const XStats* xs = reinterpret_cast<const XStats*>(ws + p->off_xs);
    hipError_t e = launch_prep_c(p->fmt, Cp, p->k, p->d, p->D, p->kpad, p->DP, xs,
                                 f8 ? reinterpret_cast<const float*>(ws + p->off_fsc) : nullptr, ws + p->off_ab,
                                 reinterpret_cast<float*>(ws + p->off_bias), reinterpret_cast<CStats*>(ws + p->off_cs),
                                 f8 ? nullptr : reinterpret_cast<float*>(ws + p->off_pcn), ctrl, iter, s);
    if (e != hipSuccess) return e;
    if (f8 && (e = launch_prep_c(FMT_BF16, Cp, p->k, p->d, p->D, p->kpad, p->DP, xs, nullptr, ws + p->off_ab16,
                                 reinterpret_cast<float*>(ws + p->off_bias16),
                                 reinterpret_cast<CStats*>(ws + p->off_cs16),
                                 reinterpret_cast<float*>(ws + p->off_pcn), ctrl, iter, s)) != hipSuccess)
        return e;
    MixArgs m{};
    m.X = X; m.n = p->n; m.d = p->d; m.k = p->k; m.kpad = p->kpad;
    m.Ab = ws + p->off_ab;
    m.Xq = f8 ? ws + p->off_xq : nullptr;
    m.xst = f8 ? reinterpret_cast<const float2*>(ws + p->off_xst) : nullptr;
    m.Xb = f8 ? nullptr : reinterpret_cast<const __bf16*>(ws + p->off_xb);
    m.xn = f8 ? nullptr : reinterpret_cast<const float*>(ws + p->off_xn);
    m.bias = reinterpret_cast<const float*>(ws + p->off_bias);
    m.cs = reinterpret_cast<const CStats*>(ws + p->off_cs);
    m.u = f8 ? 0.0625f : 0.00390625f;        // unit roundoff: e4m3 2^-4, BF16 2^-8
    m.IB = p->IB;
    m.gamma_terms = 2 * p->DP + 8;
    m.D8 = p->D8;
    m.DP = p->DP;
    m.labels = labels;
    m.rq = reinterpret_cast<int32_t*>(ws + p->off_rq);
    m.rq_count = reinterpret_cast<int32_t*>(ws + p->off_rqc);
    m.rq_per_block = p->rq_per_block;
    m.nreg = G;
    m.changed_part = changed;
    m.amb = reinterpret_cast<int32_t*>(ws + p->off_amb);
    m.amb_count = reinterpret_cast<int32_t*>(ws + p->off_ambc);
    m.amb_key = f8 ? nullptr : reinterpret_cast<uint32_t*>(ws + p->off_ambk);
    m.amb_key_in = nullptr;
    m.ctrl = ctrl; m.iter = iter; m.count_changed = count_changed;
    m.nbuf = mix_buffers(p->fmt, p->D16, p->kpad);
    m.wide_blocks = p->wide_blocks ? 1 : 0;
    // BF16 operands (the FP8 plan's own copy); an FP8 screen's open samples
    // get a BF16 screen of their own (mb), whose keys the refine then shares
    MixArgs mb = m;
    if (f8) {
        mb.Ab = ws + p->off_ab16;
        mb.bias = reinterpret_cast<const float*>(ws + p->off_bias16);
        mb.cs = reinterpret_cast<const CStats*>(ws + p->off_cs16);
        mb.Xq = nullptr;
        mb.xst = nullptr;
        mb.Xb = reinterpret_cast<const __bf16*>(ws + p->off_xb);
        mb.xn = reinterpret_cast<const float*>(ws + p->off_xn);
        mb.u = 0.00390625f;
        mb.nbuf = mix_buffers(FMT_BF16, p->D16, p->kpad);
        mb.amb_in = m.amb;
        mb.amb_in_count = m.amb_count;
        mb.amb = reinterpret_cast<int32_t*>(ws + p->off_amb2);
        mb.amb_count = reinterpret_cast<int32_t*>(ws + p->off_ambc2);
        mb.amb_key = reinterpret_cast<uint32_t*>(ws + p->off_ambk);
        mb.changed_part = changed + G;
    }
    const MixArgs& last_screen = f8 ? mb : m;
    // the refining pass: the last screen's open samples and keys
    MixArgs m2 = mb;
    m2.amb = nullptr;
    m2.amb_count = nullptr;
    m2.amb_in = last_screen.amb;
    m2.amb_in_count = last_screen.amb_count;
    m2.amb_key = nullptr;
    m2.amb_key_in = last_screen.amb_key;
    m2.changed_part = changed + (p->mfma_passes() - 1) * G;
    // each MFMA pass is timed on its own (one event pair per launch)
    auto timed_mfma = [&](int fmt, int stage, const MixArgs& args) -> hipError_t {
        const bool timed = p->timing_on();
        hipError_t r;
        if (timed && (r = hipEventRecord(p->ev[2 * p->ev_used], s)) != hipSuccess) return r;
        if ((r = launch_mfma_assign(fmt, stage, p->D16, args, G, s)) != hipSuccess) return r;
        if (timed) {
            if ((r = hipEventRecord(p->ev[2 * p->ev_used + 1], s)) != hipSuccess) return r;
            ++p->ev_used;
        }
        return hipSuccess;
    };
    if (p->cascade) {
        if ((e = timed_mfma(p->fmt, 1, m)) != hipSuccess) return e;
        if (f8 && (e = timed_mfma(FMT_BF16, 2, mb)) != hipSuccess) return e;
        // after a BF16 screen the refine's keys are the screen's: its band is known
        if ((e = timed_mfma(FMT_BF16, 3, m2)) != hipSuccess) return e;
    } else if ((e = timed_mfma(FMT_BF16, 0, m)) != hipSuccess) {
        return e;
    }
    RecheckArgs r{};
    r.X = X; r.Cp = Cp; r.n = p->n; r.d = p->d; r.k = p->k;
    r.rq = m.rq; r.rq_count = m.rq_count; r.rq_per_block = p->rq_per_block; r.rq_ints = kRqInts;
    r.nreg = G;
    r.labels = labels; r.changed_part = changed + p->mfma_passes() * G;
    r.ctrl = ctrl; r.iter = iter; r.count_changed = count_changed;
    return p->wide ? launch_recheck_wide(r, G, s) : launch_recheck(p->D8, r, G, p->rc_split, s);
}

// Run-level prep of the mixed path (once per call, amortised over its
// iterations): |x| statistics, the BF16 copy of X with |x| bounds, and for
// FP8 the scaled e4m3 copy of X.
hipError_t enqueue_prep_x(km_plan* p, const float* X, hipStream_t s)
{
    hipError_t e = launch_prep_x(X, p->n, p->d, reinterpret_cast<float*>(p->ws + p->off_pxm),
                                 reinterpret_cast<double*>(p->ws + p->off_pxs),
                                 reinterpret_cast<XStats*>(p->ws + p->off_xs), s);
    if (e != hipSuccess) return e;
    e = launch_prep_x_bf16(X, p->n, p->d, p->DP, reinterpret_cast<__bf16*>(p->ws + p->off_xb),
                           reinterpret_cast<float*>(p->ws + p->off_xn), s);
    if (e != hipSuccess || p->fmt != FMT_FP8) return e;
    return launch_prep_x_fp8(X, p->n, p->d, p->DP, reinterpret_cast<float*>(p->ws + p->off_pfm),
                             reinterpret_cast<float*>(p->ws + p->off_fsc), p->ws + p->off_xq,
                             reinterpret_cast<float2*>(p->ws + p->off_xst), s);
}

km_status enqueue_lloyd(km_plan* plan, const float* X, float* C, int32_t* labels, int64_t* counts,
                        double* obj_hist, int32_t max_iter, double tol, hipStream_t stream);

Ctrl* ctrl_of(const km_plan* p) { return reinterpret_cast<Ctrl*>(p->ws + p->off_ctrl); }
float* cp_of(const km_plan* p) { return reinterpret_cast<float*>(p->ws + p->off_cp); }

km_status set_device(const km_plan* p)
{
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != p->device) return fail(KM_EINVAL, "plan was created on device %d but device %d is current", p->device, cur);
    return KM_OK;
}

}  // namespace

extern "C" {

const char* km_last_error(void) { return g_err.c_str(); }

km_status km_plan_create(int64_t n, int32_t d, int32_t k, km_precision prec, km_plan** out)
{
    g_err.clear();
    if (!out) return fail(KM_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n >= ((int64_t)1 << 31)) return fail(KM_EINVAL, "n = %lld outside [1, 2^31)", (long long)n);
    if (d < 1 || d > 1024) return fail(KM_EINVAL, "d = %d outside [1, 1024]", d);
    if (k < 1 || (int64_t)k > n) return fail(KM_EINVAL, "k = %d outside [1, n]", k);
    if (prec != KM_FP32 && prec != KM_BF16 && prec != KM_FP8_E4M3)
        return fail(KM_EINVAL, "unknown precision %d", (int)prec);
    if (prec != KM_FP32 && ((int64_t)k + kMixCK - 1) / kMixCK * kMixCK > 16384)
        return fail(KM_ENOTSUP, "BF16 and FP8 distances support k <= 16384 (got %d)", k);
    const int dsl = std::min<int>(d, kSliceD);   // features per reduce slice
    if (plain_lds_bytes(k, dsl, MODE_FUSED) > 80 * 1024 &&
        ((int64_t)k + chunk_labels(k, dsl) - 1) / chunk_labels(k, dsl) > kPartMaxChunks)
        return fail(KM_ENOTSUP, "k = %d needs more than %d label chunks at d = %d", k, kPartMaxChunks, d);

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    int ncu = 0;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute(multiProcessorCount)");

    km_plan* p = new (std::nothrow) km_plan();
    if (!p) return fail(KM_EINVAL, "out of host memory");
    p->n = n; p->d = d; p->k = k; p->prec = prec; p->device = dev; p->num_cu = ncu;
    p->D8 = (d + 7) / 8;
    p->D = 8 * p->D8;
    p->wide = d > kSliceD;
    p->dsl = dsl;
    p->nsl = (d + dsl - 1) / dsl;
    const int D8u = (dsl + 7) / 8;   // chunks of a full reduce slice
    const int64_t ntiles = (n + plain_tile(p->D8) - 1) / plain_tile(p->D8);

    // The per-label record (k x d FP64 + counts) lives in LDS.  The assign and
    // the reduce run fused as long as that costs the pass no resident blocks
    // (a record of a few tens of KiB); beyond that they run as two passes, the
    // reduce over the whole record up to 80 KiB and, above it, over label
    // chunks of at most 44 KiB: the samples are partitioned by chunk, then a
    // 2-D grid of (point range, label chunk) blocks reduces each chunk.
    p->lds_fused = plain_lds_bytes(k, dsl, MODE_FUSED);
    p->chunked = p->lds_fused > 80 * 1024;
    p->kc = p->chunked ? chunk_labels(k, dsl) : k;
    p->nch = (k + p->kc - 1) / p->kc;
    p->nsub = p->chunked ? (int)((n + kPartRows - 1) / kPartRows) : 0;

    // One resident wave of blocks for the persistent passes, at most 4 per CU.
    // Wide rows: the streaming assign, never fused with the reduce.
    const int per_cu_assign = p->wide ? wide_blocks_per_cu() : plain_blocks_per_cu(p->D8, MODE_ASSIGN, 0);
    const int per_cu_fused = (p->chunked || p->wide) ? 0 : plain_blocks_per_cu(p->D8, MODE_FUSED, p->lds_fused);
    if (per_cu_assign < 1 || (!p->chunked && !p->wide && per_cu_fused < 1)) {
        delete p;
        return fail(KM_EHIP, "occupancy query for the per-sample pass failed");
    }
    int per_cu = std::min(per_cu_assign, 4);
    p->split = p->chunked || p->wide || per_cu_fused < per_cu;
    // A stand-alone update lists kUpdTiles tiles per step; the update that
    // must walk the fused pass's blocks (no split) keeps its LDS and lists one.
    p->upd_tiles = p->split ? kUpdTiles : 1;
    // A stand-alone update whose record would leave fewer than three blocks
    // per CU adds label chunks instead (each block reads its range's labels
    // and adds its chunk's samples; every row is still read once).
    if (p->split && !p->chunked) {
        int c = 1;
        while (c < 4 && plain_lds_bytes((k + c - 1) / c, dsl, MODE_UPDATE, p->upd_tiles) > 53 * 1024) ++c;
        p->kc = (k + c - 1) / c;
        p->nch = (k + p->kc - 1) / p->kc;
    }
    p->lds_upd = p->chunked ? part_update_lds_bytes(p->kc, dsl) : plain_lds_bytes(p->kc, dsl, MODE_UPDATE, p->upd_tiles);
    int per_cu_upd = p->chunked ? part_update_blocks_per_cu(D8u, p->lds_upd)
                                : plain_blocks_per_cu(D8u, MODE_UPDATE, p->lds_upd);
    if (per_cu_upd < 1) {
        delete p;
        return fail(KM_EHIP, "occupancy query for the update pass failed");
    }
    if (!p->split) per_cu = std::min(per_cu, per_cu_fused);
    p->grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)ncu * per_cu, ntiles));
    per_cu_upd = std::min(per_cu_upd, 4);
    if (p->split) {
        const int64_t resident = (int64_t)ncu * per_cu_upd;
        p->grid_upd = (int)std::max<int64_t>(1, std::min<int64_t>(resident / p->nch, ntiles));
    } else {
        p->grid_upd = p->grid;
    }
    if (prec == KM_BF16 || prec == KM_FP8_E4M3) {
        p->mixed = true;
        p->fmt = prec == KM_FP8_E4M3 ? FMT_FP8 : FMT_BF16;
        p->D16 = (d + 15) / 16;
        p->DP = 16 * p->D16;
        p->kpad = (k + kMixCK - 1) / kMixCK * kMixCK;
        p->IB = 1;
        while ((1 << p->IB) < p->kpad) ++p->IB;
        p->cascade = p->fmt == FMT_FP8 || p->kpad > 2 * kMixCK;
        const int nbf = mix_buffers(FMT_BF16, p->D16, p->kpad);
        // centroid chunks that stream through LDS are reloaded for every tile:
        // wider blocks share each load among more samples
        p->wide_blocks = p->cascade && p->D16 <= 8 && p->kpad / kMixCK > 2 && nbf == 2;
        const int occ = p->cascade ? mfma_blocks_per_cu(p->fmt, 1, p->D16, mix_buffers(p->fmt, p->D16, p->kpad),
                                                        p->wide_blocks)
                                   : mfma_blocks_per_cu(FMT_BF16, 0, p->D16, nbf);
        if (occ < 1) { delete p; return fail(KM_EHIP, "occupancy query for the MFMA pass failed"); }
        const int64_t mt = (n + kMixTile - 1) / kMixTile;
        p->grid_mfma = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)ncu * std::min(occ, 4), mt));
        // blocks (b, *) take the queue region of MFMA block b; wide blocks leave
        // a third as many (larger) regions, so each gets three times the blocks
        p->rc_split = p->wide_blocks ? 3 * kRecheckSplit : kRecheckSplit;
        p->grid_rc = p->grid_mfma * p->rc_split;
        if (p->cascade && (mfma_blocks_per_cu(FMT_BF16, 3, p->D16, nbf, p->wide_blocks) < 1 ||
                           (p->fmt == FMT_FP8 && mfma_blocks_per_cu(FMT_BF16, 2, p->D16, nbf, p->wide_blocks) < 1))) {
            delete p;
            return fail(KM_EHIP, "occupancy query for the refining MFMA pass failed");
        }
        // a block's share of samples, under the screen's tile and the others'
        const int tile1 = mix_tile(1, p->wide_blocks);
        const int64_t mt1 = (n + tile1 - 1) / tile1;
        p->rq_per_block = std::max(((mt + p->grid_mfma - 1) / p->grid_mfma) * kMixTile,
                                   ((mt1 + p->grid_mfma - 1) / p->grid_mfma) * tile1);
    }

    size_t off = 0;
    p->off_ctrl = off; off = align256(off + sizeof(Ctrl));
    p->off_cp = off;   off = align256(off + (size_t)k * p->D * sizeof(float));
    p->off_pS = off;   off = align256(off + (size_t)p->GS() * k * dsl * sizeof(double));
    p->off_pcnt = off; off = align256(off + (size_t)p->GS() * k * sizeof(int32_t));
    p->off_pJ = off;   off = align256(off + (size_t)p->grid * sizeof(double));
    p->off_pch = off;  off = align256(off + (size_t)std::max(p->grid, 3 * p->grid_mfma + p->grid_rc) * sizeof(int32_t));
    if (p->chunked) {
        p->off_perm = off; off = align256(off + (size_t)n * sizeof(int32_t));
        p->off_plab = off; off = align256(off + (size_t)n * sizeof(int32_t));
        p->off_poff = off; off = align256(off + (size_t)p->nsub * p->nch * sizeof(int32_t));
        p->off_plen = off; off = align256(off + (size_t)p->nsub * p->nch * sizeof(int32_t));
    }
    p->off_jt = off;   off = align256(off + (size_t)(finalize_blocks(k, d) + p->nsl) * sizeof(double));
    if (p->mixed) {
        p->off_xs = off;   off = align256(off + sizeof(XStats));
        p->off_pxm = off;  off = align256(off + kXStatBlocks * sizeof(float));
        p->off_pxs = off;  off = align256(off + kXStatBlocks * sizeof(double));
        p->off_ab = off;   off = align256(off + (size_t)p->kpad * p->DP * (p->fmt == FMT_FP8 ? 1 : 2));
        p->off_bias = off; off = align256(off + (size_t)p->kpad * sizeof(float));
        p->off_cs = off;   off = align256(off + sizeof(CStats));
        p->off_pcn = off;  off = align256(off + (size_t)prep_c_blocks(p->kpad) * sizeof(float));
        p->off_rqc = off;  off = align256(off + 2 * (size_t)p->grid_mfma * sizeof(int32_t));
        p->off_rq = off;   off = align256(off + (size_t)p->grid_mfma * p->rq_per_block * kRqInts * sizeof(int32_t));
        p->off_amb = off;  off = align256(off + (size_t)p->grid_mfma * p->rq_per_block * sizeof(int32_t));
        p->off_ambc = off; off = align256(off + (size_t)p->grid_mfma * sizeof(int32_t));
        p->off_ambk = off; off = align256(off + (size_t)p->grid_mfma * p->rq_per_block * sizeof(uint32_t));
        if (p->fmt == FMT_FP8) {
            p->off_amb2 = off;  off = align256(off + (size_t)p->grid_mfma * p->rq_per_block * sizeof(int32_t));
            p->off_ambc2 = off; off = align256(off + (size_t)p->grid_mfma * sizeof(int32_t));
        }
        p->off_xb = off;   off = align256(off + (size_t)n * p->DP * 2);
        p->off_xn = off;   off = align256(off + (size_t)n * sizeof(float));
        if (p->fmt == FMT_FP8) {
            p->off_fsc = off; off = align256(off + 2 * (size_t)p->DP * sizeof(float));
            p->off_pfm = off; off = align256(off + (size_t)kFmaxBlocks * p->DP * sizeof(float));
            p->off_xq = off;  off = align256(off + (size_t)n * p->DP);
            p->off_xst = off; off = align256(off + (size_t)n * sizeof(float2));
            p->off_ab16 = off;   off = align256(off + (size_t)p->kpad * p->DP * 2);
            p->off_bias16 = off; off = align256(off + (size_t)p->kpad * sizeof(float));
            p->off_cs16 = off;   off = align256(off + sizeof(CStats));
        }
    }
    p->total = off;
    *out = p;
    return KM_OK;
}

size_t km_plan_workspace_bytes(const km_plan* plan) { return plan ? plan->total : 0; }

km_status km_plan_set_workspace(km_plan* plan, void* ws, size_t bytes)
{
    g_err.clear();
    if (!plan) return fail(KM_EINVAL, "plan is NULL");
    if (!ws) return fail(KM_EWORKSPACE, "workspace pointer is NULL");
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(KM_EWORKSPACE, "workspace must be 256-byte aligned");
    if (bytes < plan->total)
        return fail(KM_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu the plan needs", bytes, plan->total);
    // a captured graph holds the old workspace's addresses in its kernel arguments
    if (plan->ws != static_cast<unsigned char*>(ws)) plan->drop_graph();
    plan->ws = static_cast<unsigned char*>(ws);
    plan->ws_bytes = bytes;
    return KM_OK;
}

void km_plan_destroy(km_plan* plan) { delete plan; }

km_status kmeans_assign(km_plan* plan, const float* X, const float* C, int32_t* labels, float* mindist,
                        double* objective, hipStream_t stream)
{
    g_err.clear();
    km_status st = check_plan(plan);
    if (st != KM_OK) return st;
    if (!X || !C || !labels) return fail(KM_EINVAL, "X, C and labels must be non-NULL");
    if (!aligned16(X) || !aligned16(C)) return fail(KM_EINVAL, "X and C must be 16-byte aligned");
    if ((st = set_device(plan)) != KM_OK) return st;

    if (plan->mixed && (mindist || objective))
        return fail(KM_ENOTSUP, "mixed-precision plans return labels only from kmeans_assign (mindist and objective must be NULL)");
    hipError_t e = launch_pad_centroids(C, plan->k, plan->d, plan->D, cp_of(plan), nullptr, stream);
    if (e != hipSuccess) return hip_fail(e, "pad_centroids launch");
    if (plan->mixed) {
        if ((e = enqueue_prep_x(plan, X, stream)) != hipSuccess) return hip_fail(e, "prep_x launch");
        if ((e = enqueue_mixed_assign(plan, X, labels, nullptr, 0, 0, stream)) != hipSuccess)
            return hip_fail(e, "mixed assign launch");
        return KM_OK;
    }
    PassArgs a = pass_args(plan, X, cp_of(plan), labels);
    a.mindist = mindist;
    e = timed_pass(plan, MODE_ASSIGN, a, dim3(plan->grid), 0, stream);
    if (e != hipSuccess) return hip_fail(e, "assign pass launch");
    if (objective) {
        e = launch_reduce_objective(a.part.J, plan->grid, objective, stream);
        if (e != hipSuccess) return hip_fail(e, "objective reduce launch");
    }
    return KM_OK;
}

}  // extern "C"

namespace {

// The per-label (per-class) reduce from given labels, finalized into FP32
// means (C_new), FP64 sums (S_out) and/or int64 counts; in debug-validate
// mode the labels are checked first.
km_status enqueue_label_reduce(km_plan* plan, const float* X, const int32_t* labels, const float* C_old,
                               float* C_new, double* S_out, int64_t* counts, hipStream_t stream)
{
    hipError_t e;
    if (plan->validate) {
        // debug-validate mode: count labels outside [0, k) before anything
        // else is enqueued, so a rejected call leaves the outputs untouched
        int32_t* part = reinterpret_cast<int32_t*>(plan->ws + plan->off_pch);
        const int cap = std::max(plan->grid, 3 * plan->grid_mfma + plan->grid_rc);
        int g = 0;
        if ((e = launch_count_bad_labels(labels, plan->n, plan->k, part, cap, &g, stream)) != hipSuccess)
            return hip_fail(e, "label check launch");
        std::vector<int32_t> v((size_t)g);
        if ((e = hipMemcpyAsync(v.data(), part, v.size() * sizeof(int32_t), hipMemcpyDeviceToHost, stream)) != hipSuccess)
            return hip_fail(e, "hipMemcpyAsync(label check)");
        if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        int64_t bad = 0;
        for (int32_t c : v) bad += c;
        if (bad > 0)
            return fail(KM_EINVAL, "%lld labels lie outside [0, %d)", (long long)bad, plan->k);
    }
    PassArgs a = pass_args(plan, X, nullptr, const_cast<int32_t*>(labels));
    FinArgs f = fin_args(plan);
    f.C_old = C_old; f.ld_old = plan->d; f.C_new = C_new; f.ld_new = plan->d; f.Cp_out = nullptr;
    f.counts = counts; f.want_J = 0; f.S_out = S_out;
    e = enqueue_reduce_finalize(plan, a, f, stream);
    if (e != hipSuccess) return hip_fail(e, "update / finalize launch");
    return KM_OK;
}

km_status check_reduce_call(km_plan* plan, const float* X, const int32_t* labels)
{
    km_status st = check_plan(plan);
    if (st != KM_OK) return st;
    if (!X || !labels) return fail(KM_EINVAL, "X and labels must be non-NULL");
    if (!aligned16(X)) return fail(KM_EINVAL, "X must be 16-byte aligned");
    return set_device(plan);
}

// GDA covariance geometry: 64-feature regions, upper-triangle region pairs,
// and sample ranges (about 512 four-wave blocks in all, two per CU; at least
// 1024 samples per range).
void gda_geometry(const km_plan* p, int& R, int& RP, int& G)
{
    R = (p->d + 63) / 64;
    RP = R * (R + 1) / 2;
    const int64_t byn = std::max<int64_t>(1, (p->n + 1023) / 1024);
    G = (int)std::max<int64_t>(1, std::min<int64_t>(byn, std::max(1, 512 / RP)));
}

}  // namespace

extern "C" {

km_status kmeans_assign_metric(km_plan* plan, const float* X, km_layout layout, km_metric metric, const float* C,
                               int32_t* labels, float* mindist, double* objective, hipStream_t stream)
{
    g_err.clear();
    km_status st = check_plan(plan);
    if (st != KM_OK) return st;
    if (!X || !C || !labels) return fail(KM_EINVAL, "X, C and labels must be non-NULL");
    if (!aligned16(X) || !aligned16(C)) return fail(KM_EINVAL, "X and C must be 16-byte aligned");
    if (layout != KM_ROW_MAJOR && layout != KM_FEATURE_MAJOR) return fail(KM_EINVAL, "unknown layout %d", (int)layout);
    if (metric != KM_METRIC_L1 && metric != KM_METRIC_SQEUCLIDEAN) return fail(KM_EINVAL, "unknown metric %d", (int)metric);
    if (plan->mixed) return fail(KM_ENOTSUP, "kmeans_assign_metric needs an FP32 plan");
    if (plan->wide) return fail(KM_ENOTSUP, "kmeans_assign_metric supports d <= %d (got %d)", kSliceD, plan->d);
    if ((st = set_device(plan)) != KM_OK) return st;
    hipError_t e = launch_pad_centroids(C, plan->k, plan->d, plan->D, cp_of(plan), nullptr, stream);
    if (e != hipSuccess) return hip_fail(e, "pad_centroids launch");
    MetricArgs a{};
    a.X = X; a.Cp = cp_of(plan); a.labels = labels; a.mindist = mindist;
    a.partJ = partials_of(plan).J;
    a.n = plan->n; a.d = plan->d; a.k = plan->k;
    if ((e = launch_assign_metric(plan->D8, (int)metric, (int)layout, a, plan->grid, stream)) != hipSuccess)
        return hip_fail(e, "assign launch");
    if (objective && (e = launch_reduce_objective(a.partJ, plan->grid, objective, stream)) != hipSuccess)
        return hip_fail(e, "objective reduce launch");
    return KM_OK;
}

km_status kmeans_update(km_plan* plan, const float* X, const int32_t* labels, const float* C_old, float* C_new,
                        int64_t* counts, hipStream_t stream)
{
    g_err.clear();
    km_status st = check_reduce_call(plan, X, labels);
    if (st != KM_OK) return st;
    if (!C_old || !C_new) return fail(KM_EINVAL, "X, labels, C_old and C_new must be non-NULL");
    return enqueue_label_reduce(plan, X, labels, C_old, C_new, nullptr, counts, stream);
}

km_status km_class_sums(km_plan* plan, const float* X, const int32_t* labels, double* S, int64_t* counts,
                        hipStream_t stream)
{
    g_err.clear();
    km_status st = check_reduce_call(plan, X, labels);
    if (st != KM_OK) return st;
    if (!S) return fail(KM_EINVAL, "S must be non-NULL");
    return enqueue_label_reduce(plan, X, labels, nullptr, nullptr, S, counts, stream);
}

km_status nb_train(km_plan* plan, const float* X, const int32_t* labels, double* prior, double* phi,
                   hipStream_t stream)
{
    g_err.clear();
    km_status st = check_reduce_call(plan, X, labels);
    if (st != KM_OK) return st;
    if (!prior || !phi) return fail(KM_EINVAL, "prior and phi must be non-NULL");
    // the class sums land in phi and the counts (int64) in prior, then both
    // are finalized in place
    if ((st = enqueue_label_reduce(plan, X, labels, nullptr, nullptr, phi, reinterpret_cast<int64_t*>(prior), stream)) !=
        KM_OK)
        return st;
    hipError_t e = launch_nb_finalize(prior, phi, plan->k, plan->d, plan->n, stream);
    if (e != hipSuccess) return hip_fail(e, "naive Bayes finalize launch");
    return KM_OK;
}

size_t gda_workspace_bytes(const km_plan* plan)
{
    if (!plan) return 0;
    int R, RP, G;
    gda_geometry(plan, R, RP, G);
    return (size_t)G * RP * 64 * 64 * sizeof(double);
}

km_status gda_train(km_plan* plan, const float* X, const int32_t* labels, double* prior, double* mu,
                    double* sigma, void* ws, size_t ws_bytes, hipStream_t stream)
{
    g_err.clear();
    km_status st = check_reduce_call(plan, X, labels);
    if (st != KM_OK) return st;
    if (!prior || !mu || !sigma) return fail(KM_EINVAL, "prior, mu and sigma must be non-NULL");
    if (!ws) return fail(KM_EWORKSPACE, "GDA workspace pointer is NULL");
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(KM_EWORKSPACE, "GDA workspace must be 256-byte aligned");
    if (ws_bytes < gda_workspace_bytes(plan))
        return fail(KM_EWORKSPACE, "GDA workspace of %zu bytes is smaller than the %zu needed", ws_bytes,
                    gda_workspace_bytes(plan));
    if ((st = enqueue_label_reduce(plan, X, labels, nullptr, nullptr, mu, reinterpret_cast<int64_t*>(prior), stream)) !=
        KM_OK)
        return st;
    CovArgs a{};
    a.X = X; a.labels = labels; a.prior = prior; a.mu = mu; a.sigma = sigma;
    a.part = static_cast<double*>(ws);
    a.n = plan->n; a.d = plan->d; a.k = plan->k;
    gda_geometry(plan, a.R, a.RP, a.G);
    hipError_t e = launch_gda_means(a, plan->k, stream);
    if (e != hipSuccess) return hip_fail(e, "GDA means launch");
    // the covariance contraction is the plan's timed kernel here
    const bool timed = plan->timing_on();
    if (timed && (e = hipEventRecord(plan->ev[2 * plan->ev_used], stream)) != hipSuccess)
        return hip_fail(e, "hipEventRecord");
    if ((e = launch_gda_cov(a, stream)) != hipSuccess) return hip_fail(e, "GDA covariance launch");
    if (timed) {
        if ((e = hipEventRecord(plan->ev[2 * plan->ev_used + 1], stream)) != hipSuccess)
            return hip_fail(e, "hipEventRecord");
        ++plan->ev_used;
    }
    if ((e = launch_gda_combine(a, stream)) != hipSuccess) return hip_fail(e, "GDA combine launch");
    return KM_OK;
}

km_status kmeans_lloyd(km_plan* plan, const float* X, float* C, int32_t* labels, int64_t* counts,
                       double* obj_hist, int32_t max_iter, double tol, int32_t* iters_done, hipStream_t stream)
{
    g_err.clear();
    km_status st = check_plan(plan);
    if (st != KM_OK) return st;
    if (!X || !C || !labels) return fail(KM_EINVAL, "X, C and labels must be non-NULL");
    if (!aligned16(X) || !aligned16(C)) return fail(KM_EINVAL, "X and C must be 16-byte aligned");
    if (max_iter < 1) return fail(KM_EINVAL, "max_iter = %d must be >= 1", max_iter);
    if (tol != tol) return fail(KM_EINVAL, "tol is NaN");
    if ((st = set_device(plan)) != KM_OK) return st;

    Ctrl* ctrl = ctrl_of(plan);
    hipError_t e;
    if (plan->use_graph) {
        // Replay the captured call when the arguments are unchanged; otherwise
        // capture it on the plan's own stream (the caller's may be the null
        // stream, which cannot be captured) and replay on the caller's.
        const km_plan::GraphKey key{X, C, labels, counts, obj_hist, max_iter, tol, plan->ev_used};
        if (!plan->gexec || !(plan->gkey == key)) {
            plan->drop_graph();
            if (!plan->cap_stream && (e = hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking)) != hipSuccess)
                return hip_fail(e, "hipStreamCreateWithFlags");
            if ((e = hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                return hip_fail(e, "hipStreamBeginCapture");
            const int32_t ev_before = plan->ev_used;
            km_status cs = enqueue_lloyd(plan, X, C, labels, counts, obj_hist, max_iter, tol, plan->cap_stream);
            hipGraph_t g = nullptr;
            hipError_t ee = hipStreamEndCapture(plan->cap_stream, &g);
            if (cs != KM_OK) { if (g) (void)hipGraphDestroy(g); plan->ev_used = ev_before; return cs; }
            if (ee != hipSuccess) { plan->ev_used = ev_before; return hip_fail(ee, "hipStreamEndCapture"); }
            ee = hipGraphInstantiate(&plan->gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ee != hipSuccess) { plan->gexec = nullptr; plan->ev_used = ev_before; return hip_fail(ee, "hipGraphInstantiate"); }
            plan->gkey = key;
            plan->gkey.ev_used = plan->ev_used;
        }
        if ((e = hipGraphLaunch(plan->gexec, stream)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    } else {
        km_status es = enqueue_lloyd(plan, X, C, labels, counts, obj_hist, max_iter, tol, stream);
        if (es != KM_OK) return es;
    }
    if (iters_done) {
        if (tol < 0.0) {
            *iters_done = max_iter;
        } else {
            int32_t v = 0;
            e = hipMemcpyAsync(&v, &ctrl->iters_done, sizeof v, hipMemcpyDeviceToHost, stream);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(iters_done)");
            e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            *iters_done = v;
        }
    }
    return KM_OK;
}

km_status km_plan_set_validate(km_plan* plan, int32_t enable)
{
    g_err.clear();
    if (!plan) return fail(KM_EINVAL, "plan is NULL");
    plan->validate = enable != 0;
    return KM_OK;
}

km_status km_plan_use_graphs(km_plan* plan, int32_t enable)
{
    g_err.clear();
    if (!plan) return fail(KM_EINVAL, "plan is NULL");
    plan->use_graph = enable != 0;
    plan->drop_graph();
    return KM_OK;
}

}  // extern "C"

namespace {

// The launches of one kmeans_lloyd call, in stream order.
km_status enqueue_lloyd(km_plan* plan, const float* X, float* C, int32_t* labels, int64_t* counts,
                        double* obj_hist, int32_t max_iter, double tol, hipStream_t stream)
{
    Ctrl* ctrl = ctrl_of(plan);
    float* Cp = cp_of(plan);
    hipError_t e = launch_pad_centroids(C, plan->k, plan->d, plan->D, Cp, ctrl, stream);
    if (e != hipSuccess) return hip_fail(e, "pad_centroids launch");

    PassArgs a = pass_args(plan, X, Cp, labels);
    a.ctrl = (tol >= 0.0) ? ctrl : nullptr;
    a.count_changed = 1;
    FinArgs f = fin_args(plan);
    f.C_old = Cp; f.ld_old = plan->D; f.C_new = C; f.ld_new = plan->d; f.Cp_out = Cp;
    f.counts = counts; f.ctrl = ctrl; f.obj_hist = obj_hist; f.tol = tol; f.want_J = 1;
    if (plan->mixed && (e = enqueue_prep_x(plan, X, stream)) != hipSuccess) return hip_fail(e, "prep_x launch");
    for (int32_t t = 0; t < max_iter; ++t) {
        a.iter = t;
        f.iter = t;
        if (plan->mixed) {
            e = enqueue_mixed_assign(plan, X, labels, a.ctrl, t, 1, stream);
            if (e != hipSuccess) return hip_fail(e, "mixed assign launch");
            e = enqueue_reduce_finalize(plan, a, f, stream);
            if (e != hipSuccess) return hip_fail(e, "update / finalize launch");
        } else if (!plan->split) {
            e = timed_pass(plan, MODE_FUSED, a, dim3(plan->grid), plan->lds_fused, stream);
            if (e != hipSuccess) return hip_fail(e, "fused pass launch");
            e = launch_finalize(f, stream);
            if (e != hipSuccess) return hip_fail(e, "finalize launch");
        } else {
            e = timed_pass(plan, MODE_ASSIGN, a, dim3(plan->grid), 0, stream);
            if (e != hipSuccess) return hip_fail(e, "assign pass launch");
            e = enqueue_reduce_finalize(plan, a, f, stream);
            if (e != hipSuccess) return hip_fail(e, "update / finalize launch");
        }
    }
    return KM_OK;
}

}  // namespace

namespace km {

km_status plan_enqueue_fixed(km_plan* plan, const float* X, float* C, int32_t* labels, int64_t* counts,
                             double* obj_hist, int32_t iters, hipStream_t stream)
{
    km_status st = check_plan(plan);
    if (st != KM_OK) return st;
    return enqueue_lloyd(plan, X, C, labels, counts, obj_hist, iters, -1.0, stream);
}

}  // namespace km

extern "C" {

km_status km_plan_enable_timing(km_plan* plan, int32_t cap)
{
    g_err.clear();
    if (!plan) return fail(KM_EINVAL, "plan is NULL");
    if (cap < 0) return fail(KM_EINVAL, "cap = %d must be >= 0", cap);
    plan->drop_graph();   // a captured graph records into the old events
    for (hipEvent_t e : plan->ev) (void)hipEventDestroy(e);
    plan->ev.clear();
    plan->ev_used = 0;
    for (int32_t i = 0; i < 2 * cap; ++i) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return hip_fail(r, "hipEventCreate");
        plan->ev.push_back(e);
    }
    return KM_OK;
}

km_status km_plan_recheck_count(km_plan* plan, int64_t* count, int64_t* full_scans, hipStream_t stream)
{
    g_err.clear();
    km_status st = check_plan(plan);
    if (st != KM_OK) return st;
    if (!plan->mixed) return fail(KM_EINVAL, "the plan has no recheck queue (FP32 plan)");
    if (!count) return fail(KM_EINVAL, "count is NULL");
    std::vector<int32_t> v(2 * (size_t)plan->grid_mfma);
    hipError_t e = hipMemcpyAsync(v.data(), plan->ws + plan->off_rqc, v.size() * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(recheck counts)");
    if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    int64_t total = 0, full = 0;
    for (int b = 0; b < plan->grid_mfma; ++b) { total += v[b]; full += v[plan->grid_mfma + b]; }
    *count = total;
    if (full_scans) *full_scans = full;
    return KM_OK;
}

km_status km_plan_kernel_times(km_plan* plan, float* ms, int32_t cap, int32_t* count)
{
    g_err.clear();
    if (!plan) return fail(KM_EINVAL, "plan is NULL");
    if (!count || (cap > 0 && !ms)) return fail(KM_EINVAL, "count and ms must be non-NULL");
    int32_t m = std::min(cap, plan->ev_used);
    for (int32_t i = 0; i < m; ++i) {
        hipError_t r = hipEventSynchronize(plan->ev[2 * i + 1]);
        if (r != hipSuccess) return hip_fail(r, "hipEventSynchronize");
        r = hipEventElapsedTime(&ms[i], plan->ev[2 * i], plan->ev[2 * i + 1]);
        if (r != hipSuccess) return hip_fail(r, "hipEventElapsedTime");
    }
    *count = plan->ev_used;
    return KM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free variant of kmeans_lloyd: the plan's scratch (control block,
// padded centroids, per-block partial records, queues) lives in one
// library-owned device array instead of a caller-bound workspace.  Every GPU
// the library runs on holds its own copy of the array from the moment the
// code object is loaded until the process ends.

namespace {

static __device__ __align__(256) unsigned char scratch[KM_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_dev[kMaxDevices] = {};   // device address of `scratch`, per device

// Device address of this device's `scratch` (the host-side name is only a
// stand-in); looked up once per device, with that device current.
km_status scratch_of_device(int dev, unsigned char** out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(KM_ENOTSUP, "device %d: static scratch supports devices 0..%d", dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255u))
            return fail(KM_EHIP, "static scratch address %p is not 256-byte aligned", ptr);
        g_scratch_dev[dev] = static_cast<unsigned char*>(ptr);
    }
    *out = g_scratch_dev[dev];
    return KM_OK;
}

// Points the plan at the static scratch for the duration of one call, with
// timing off, and restores its own workspace afterwards.
struct StaticScratchScope {
    km_plan* p;
    unsigned char* ws;
    size_t bytes;
    bool untimed;
    StaticScratchScope(km_plan* plan, unsigned char* s) : p(plan), ws(plan->ws), bytes(plan->ws_bytes), untimed(plan->untimed)
    {
        p->ws = s;
        p->ws_bytes = KM_STATIC_SCRATCH_BYTES;
        p->untimed = true;
    }
    ~StaticScratchScope()
    {
        p->ws = ws;
        p->ws_bytes = bytes;
        p->untimed = untimed;
    }
};

}  // namespace

extern "C" {

km_status kmeans_lloyd_static(km_plan* plan, const float* X, float* C, int32_t* labels, int64_t* counts,
                              double* obj_hist, int32_t max_iter, double tol, int32_t* iters_done,
                              hipStream_t stream)
{
    g_err.clear();
    if (!plan) return fail(KM_EINVAL, "plan is NULL");
    if (!X || !C || !labels) return fail(KM_EINVAL, "X, C and labels must be non-NULL");
    if (!aligned16(X) || !aligned16(C)) return fail(KM_EINVAL, "X and C must be 16-byte aligned");
    if (max_iter < 1) return fail(KM_EINVAL, "max_iter = %d must be >= 1", max_iter);
    if (tol != tol) return fail(KM_EINVAL, "tol is NaN");
    if (plan->total > (size_t)KM_STATIC_SCRATCH_BYTES)
        return fail(KM_EWORKSPACE, "the plan needs %zu bytes of scratch; the static scratch holds %zu (use kmeans_lloyd "
                    "with a bound workspace)", plan->total, (size_t)KM_STATIC_SCRATCH_BYTES);
    km_status st = set_device(plan);
    if (st != KM_OK) return st;
    unsigned char* s = nullptr;
    if ((st = scratch_of_device(plan->device, &s)) != KM_OK) return st;

    StaticScratchScope scope(plan, s);
    st = enqueue_lloyd(plan, X, C, labels, counts, obj_hist, max_iter, tol, stream);
    if (st != KM_OK) return st;
    if (iters_done) {
        if (tol < 0.0) {
            *iters_done = max_iter;
        } else {
            int32_t v = 0;
            hipError_t e = hipMemcpyAsync(&v, &ctrl_of(plan)->iters_done, sizeof v, hipMemcpyDeviceToHost, stream);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(iters_done)");
            if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            *iters_done = v;
        }
    }
    return KM_OK;
}

}  // extern "C"
