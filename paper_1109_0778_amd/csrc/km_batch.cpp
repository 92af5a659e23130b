// Host side of the batched C ABI: many independent Lloyd problems advanced
// together.  FP32: every iteration is one launch of the fused per-sample pass
// per shape class (instances grouped by padded dimension and by the LDS their
// record needs) over a table of (instance, tile range, partial slot) blocks,
// plus one finalize launch over (instance, 64-element chunk) blocks.  BF16:
// per iteration one centroid-prep launch (a block per instance), the MFMA
// pass per operand width and the exact recheck per feature width over their
// own work tables, the update pass per shape class, the finalize and the
// objective; the BF16 copy of X and the |x| statistics once per call.
// Instances of more than 128 features, and every instance of an FP8 batch,
// run the single-instance launch sequence of a plan of their own on a side
// stream of the batch, forked from and joined back to the caller's stream
// within the call.
#include "kmeans_mi355x.h"
#include "km_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

using namespace km;

// Defined in km_api.cpp: sets km_last_error() text and returns the status.
km_status km_set_error(km_status st, const char* msg);

namespace {

km_status berr(km_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return km_set_error(st, buf);
}

km_status bhip(hipError_t e, const char* what)
{
    return berr(KM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

inline size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Group {
    int D8;               // D8 (pass, recheck) or D16 (MFMA pass)
    size_t lds;
    int first, count;     // range in the work table
    double cost = 0.0;    // estimated work (sum over its rows)
    int lane = 0;         // side stream it is launched on
};

constexpr int kBatchRecheckSplit = 2;   // recheck blocks per queue region
constexpr int km_side_streams = 4;      // side streams a phase's groups are spread over
constexpr int32_t kMaxTilesPerBlock = 1 << 20;   // schedule bound (keeps 2 x tiles in int range)

}  // namespace

struct km_batch {
    std::vector<km_instance> inst;         // instances of at most 128 features (the class schedule)
    // instances of more than 128 features: each runs the single-instance
    // path through a plan of its own, on a stream of its own, inside the
    // same call (and graph)
    std::vector<km_instance> wide;
    std::vector<km_plan*> wplan;
    std::vector<size_t> off_wide;
    hipStream_t wstream = nullptr;
    hipEvent_t ev_wfork = nullptr, ev_wjoin = nullptr;
    int device = 0;
    bool mixed = false;    // BF16 MFMA distances + exact FP32 recheck
    int tpb = 16;          // tiles per block (classes without their own value)
    int order = 1;         // 0: instance order, 1: decreasing work per block
    // shape classes of the per-sample pass, (D8, LDS bucket), in key order,
    // and a tiles-per-block value per class (0: tpb)
    std::vector<std::pair<int, size_t>> classes;
    std::map<std::pair<int, size_t>, int> class_tpb;
    std::vector<int> tpb_inst;             // tiles per block of each instance (its class's)
    std::vector<int64_t> rq_rows;          // recheck queue entries per region of each instance
    // derived layout
    std::vector<int> nslots;
    std::vector<size_t> off_cp, off_S, off_cnt, off_J, off_ch;
    std::vector<BatchWork> work;
    std::vector<BatchFinWork> fwork;
    std::vector<Group> groups;
    size_t off_pa = 0, off_fa = 0, off_work = 0, off_fwork = 0, total = 0;
    // mixed path
    std::vector<int> nreg;                 // MFMA queue regions per instance
    std::vector<size_t> off_xs, off_ab, off_bias, off_cs, off_rq, off_rqc, off_chg, off_jt, off_xpm, off_xps;
    std::vector<size_t> off_xb, off_xn;    // run-level BF16 copy of X and |x| bounds
    std::vector<int> nxb;
    std::vector<BatchWork> mwork, rwork, xwork;   // MFMA rows, recheck rows, statistics rows
    std::vector<Group> mgroups, rgroups;
    size_t off_bm = 0, off_mwork = 0, off_rwork = 0, off_xwork = 0;
    // side streams: the launches of one phase (one per shape class) are
    // forked onto them and joined back, so classes overlap (graph branches)
    static constexpr int kSide = km_side_streams;
    hipStream_t side[kSide] = {};
    hipEvent_t ev_fork = nullptr, ev_join[kSide] = {};
    unsigned char* ws = nullptr;
    // persistent FP32 mode: one launch per kPersistIters iterations
    bool persistent = false;
    std::vector<size_t> off_ring;          // per instance: kPersistIters + 1 padded centroid buffers
    std::vector<int64_t> ring_stride;      // floats between buffers
    std::vector<BatchWork> pwork;          // every work row, decreasing work
    size_t off_pring = 0, off_pstride = 0, off_pnsl = 0, off_pdone = 0, off_pready = 0, off_pctrl = 0, off_pwork = 0;
    size_t p_lds = 0;
    int p_grid = 1;
    // graph
    bool use_graph = false;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    int32_t g_iters = 0;
    void drop_graph()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        gexec = nullptr;
    }
    ~km_batch()
    {
        drop_graph();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (int i = 0; i < kSide; ++i) {
            if (side[i]) (void)hipStreamDestroy(side[i]);
            if (ev_join[i]) (void)hipEventDestroy(ev_join[i]);
        }
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        for (km_plan* p : wplan) km_plan_destroy(p);
        if (wstream) (void)hipStreamDestroy(wstream);
        if (ev_wfork) (void)hipEventDestroy(ev_wfork);
        if (ev_wjoin) (void)hipEventDestroy(ev_wjoin);
    }
};

namespace {

int d8_of(int d) { return (d + 7) / 8; }
int d16_of(int d) { return (d + 15) / 16; }
int kpad_of(int k) { return (k + kMixCK - 1) / kMixCK * kMixCK; }
int ib_of(int kpad)
{
    int ib = 1;
    while ((1 << ib) < kpad) ++ib;
    return ib;
}

// Rows grouped by key, optionally in decreasing cost, appended to `out`.
void emit_groups(std::map<std::pair<int, size_t>, std::vector<BatchWork>>& by, std::map<std::pair<int, size_t>,
                 std::vector<double>>& costs, int order, std::vector<BatchWork>& out, std::vector<Group>& groups)
{
    out.clear();
    groups.clear();
    for (auto& kv : by) {
        std::vector<BatchWork>& v = kv.second;
        if (order == 1) {
            std::vector<double>& c = costs[kv.first];
            std::vector<int> idx(v.size());
            for (size_t q = 0; q < idx.size(); ++q) idx[q] = (int)q;
            std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return c[a] > c[b]; });
            std::vector<BatchWork> s(v.size());
            for (size_t q = 0; q < idx.size(); ++q) s[q] = v[idx[q]];
            v.swap(s);
        }
        Group g;
        g.D8 = kv.first.first;
        g.lds = kv.first.second;
        g.first = (int)out.size();
        g.count = (int)v.size();
        for (double c : costs[kv.first]) g.cost += c;
        groups.push_back(g);
        out.insert(out.end(), v.begin(), v.end());
    }
    // launch order and side streams: largest group first, each group onto the
    // least loaded stream (longest-processing-time rule), so the long groups
    // of a phase start together instead of queueing behind short ones
    std::stable_sort(groups.begin(), groups.end(), [](const Group& a, const Group& b) { return a.cost > b.cost; });
    double load[km_side_streams] = {};
    for (Group& g : groups) {
        int best = 0;
        for (int q = 1; q < km_side_streams; ++q)
            if (load[q] < load[best]) best = q;
        g.lane = best;
        load[best] += g.cost;
    }
}

size_t lds_bucket(size_t lds)
{
    static const size_t b[] = {24 * 1024, 48 * 1024, 64 * 1024, 80 * 1024};
    for (size_t x : b)
        if (lds <= x) return x;
    return lds;
}

// Work tables and workspace layout for the current schedule.
// Schedule class of an instance: (D8, LDS bucket of the fused pass's per-label
// record).  The same partition for every precision, so a schedule tuned for
// one batch applies unchanged to the same instances at another precision.
std::pair<int, size_t> class_of(const km_batch*, const km_instance& x)
{
    return std::make_pair(d8_of(x.d), lds_bucket(plain_lds_bytes(x.k, x.d, MODE_FUSED)));
}

void layout(km_batch* B)
{
    const int m = (int)B->inst.size();
    B->nslots.assign(m, 0);
    B->tpb_inst.assign(m, B->tpb);
    B->classes.clear();
    for (const km_instance& x : B->inst) {
        const auto key = class_of(B, x);
        if (std::find(B->classes.begin(), B->classes.end(), key) == B->classes.end()) B->classes.push_back(key);
    }
    std::sort(B->classes.begin(), B->classes.end());
    B->off_cp.assign(m, 0); B->off_S.assign(m, 0); B->off_cnt.assign(m, 0);
    B->off_J.assign(m, 0); B->off_ch.assign(m, 0);
    std::map<std::pair<int, size_t>, std::vector<BatchWork>> by_group;
    std::map<std::pair<int, size_t>, std::vector<double>> costs;
    B->fwork.clear();
    size_t off = 0;
    for (int i = 0; i < m; ++i) {
        const km_instance& x = B->inst[i];
        const int D8 = d8_of(x.d);
        const int64_t tiles = (x.n + kBlock - 1) / kBlock;
        // kernel group: the pass's own LDS record size (update mode for the
        // mixed batch); the schedule class may differ from it
        const auto key = std::make_pair(D8, lds_bucket(plain_lds_bytes(x.k, x.d, B->mixed ? MODE_UPDATE : MODE_FUSED)));
        const auto ct = B->class_tpb.find(class_of(B, x));
        const int tpb = (ct != B->class_tpb.end() && ct->second > 0) ? ct->second : B->tpb;
        B->tpb_inst[i] = tpb;
        const int nb = (int)((tiles + tpb - 1) / tpb);
        B->nslots[i] = nb;
        for (int b = 0; b < nb; ++b) {
            BatchWork w;
            w.inst = i;
            w.slot = b;
            w.t0 = (int64_t)b * tpb;
            w.t1 = std::min<int64_t>(tiles, w.t0 + tpb);
            by_group[key].push_back(w);
            // the update after a BF16 assign reads rows; the fused pass also forms distances
            costs[key].push_back((double)(w.t1 - w.t0) * (B->mixed ? x.d : (double)x.k * x.d));
        }
        const int chunks = finalize_blocks(x.k, x.d);
        for (int c = 0; c < chunks; ++c) B->fwork.push_back(BatchFinWork{i, c});
        B->off_cp[i] = off;  off = al256(off + (size_t)x.k * 8 * D8 * sizeof(float));
        B->off_S[i] = off;   off = al256(off + (size_t)nb * x.k * x.d * sizeof(double));
        B->off_cnt[i] = off; off = al256(off + (size_t)nb * x.k * sizeof(int32_t));
        B->off_J[i] = off;   off = al256(off + (size_t)nb * sizeof(double));
        B->off_ch[i] = off;  off = al256(off + (size_t)nb * sizeof(int32_t));
    }
    emit_groups(by_group, costs, B->order, B->work, B->groups);
    if (B->mixed) {
        // MFMA rows of 2 * tpb 128-sample tiles (the same samples as a pass row
        // of the instance's class), one queue region per row; recheck rows:
        // kBatchRecheckSplit per region
        std::map<std::pair<int, size_t>, std::vector<BatchWork>> by_m, by_r;
        std::map<std::pair<int, size_t>, std::vector<double>> c_m, c_r;
        B->nreg.assign(m, 0);
        B->off_xs.assign(m, 0); B->off_ab.assign(m, 0); B->off_bias.assign(m, 0); B->off_cs.assign(m, 0);
        B->off_rq.assign(m, 0); B->off_rqc.assign(m, 0); B->off_chg.assign(m, 0); B->off_jt.assign(m, 0);
        B->off_xpm.assign(m, 0); B->off_xps.assign(m, 0); B->nxb.assign(m, 0);
        B->off_xb.assign(m, 0); B->off_xn.assign(m, 0);
        B->rq_rows.assign(m, 0);
        B->xwork.clear();
        for (int i = 0; i < m; ++i) {
            const km_instance& x = B->inst[i];
            const int D16 = d16_of(x.d), kpad = kpad_of(x.k);
            const int tpm = 2 * B->tpb_inst[i];
            const int64_t mt = (x.n + kMixTile - 1) / kMixTile;
            const int nr = (int)((mt + tpm - 1) / tpm);
            B->nreg[i] = nr;
            // a region holds at most its samples: no more than the instance's
            B->rq_rows[i] = std::min<int64_t>(tpm, mt) * kMixTile;
            for (int r = 0; r < nr; ++r) {
                BatchWork w;
                w.inst = i;
                w.slot = r;
                w.t0 = (int64_t)r * tpm;
                w.t1 = std::min<int64_t>(mt, w.t0 + tpm);
                by_m[std::make_pair(D16, (size_t)0)].push_back(w);
                c_m[std::make_pair(D16, (size_t)0)].push_back((double)(w.t1 - w.t0) * kpad * D16);
                for (int y = 0; y < kBatchRecheckSplit; ++y) {
                    BatchWork rw;
                    rw.inst = i;
                    rw.slot = r;
                    rw.t0 = y;
                    rw.t1 = kBatchRecheckSplit;
                    by_r[std::make_pair(d8_of(x.d), (size_t)0)].push_back(rw);
                    c_r[std::make_pair(d8_of(x.d), (size_t)0)].push_back((double)(w.t1 - w.t0) * x.d);
                }
            }
            B->off_xs[i] = off;   off = al256(off + sizeof(XStats));
            B->off_ab[i] = off;   off = al256(off + (size_t)kpad * 16 * D16 * sizeof(__bf16));
            B->off_bias[i] = off; off = al256(off + (size_t)kpad * sizeof(float));
            B->off_cs[i] = off;   off = al256(off + sizeof(CStats));
            B->off_rq[i] = off;   off = al256(off + (size_t)nr * B->rq_rows[i] * kRqInts * sizeof(int32_t));
            B->off_rqc[i] = off;  off = al256(off + 2 * (size_t)nr * sizeof(int32_t));
            B->off_chg[i] = off;  off = al256(off + (size_t)(1 + kBatchRecheckSplit) * nr * sizeof(int32_t));
            B->off_jt[i] = off;   off = al256(off + (size_t)finalize_blocks(x.k, x.d) * sizeof(double));
            const int nx = (int)((x.n + kPrepXRows - 1) / kPrepXRows);
            B->nxb[i] = nx;
            for (int b = 0; b < nx; ++b)
                B->xwork.push_back(BatchWork{i, b, (int64_t)b * kPrepXRows, std::min<int64_t>(x.n, (int64_t)(b + 1) * kPrepXRows)});
            B->off_xb[i] = off;   off = al256(off + (size_t)x.n * 16 * D16 * sizeof(__bf16));
            B->off_xn[i] = off;   off = al256(off + (size_t)x.n * sizeof(float));
            B->off_xpm[i] = off;  off = al256(off + (size_t)nx * sizeof(float));
            B->off_xps[i] = off;  off = al256(off + (size_t)nx * sizeof(double));
        }
        emit_groups(by_m, c_m, B->order, B->mwork, B->mgroups);
        emit_groups(by_r, c_r, B->order, B->rwork, B->rgroups);
        for (Group& g : B->mgroups) g.lds = mfma_lds_bytes(FMT_BF16, g.D8, 0);
        B->off_bm = off;    off = al256(off + (size_t)m * sizeof(BatchMix));
        B->off_mwork = off; off = al256(off + B->mwork.size() * sizeof(BatchWork));
        B->off_rwork = off; off = al256(off + B->rwork.size() * sizeof(BatchWork));
        B->off_xwork = off; off = al256(off + B->xwork.size() * sizeof(BatchWork));
    }
    if (B->persistent) {
        // the queue's rows: every class's, by decreasing work (t1 - t0) k d
        B->pwork = B->work;
        std::stable_sort(B->pwork.begin(), B->pwork.end(), [&](const BatchWork& a, const BatchWork& b) {
            const km_instance& xa = B->inst[a.inst];
            const km_instance& xb = B->inst[b.inst];
            return (double)(a.t1 - a.t0) * xa.k * xa.d > (double)(b.t1 - b.t0) * xb.k * xb.d;
        });
        B->off_ring.assign(m, 0);
        B->ring_stride.assign(m, 0);
        B->p_lds = 0;
        for (int i = 0; i < m; ++i) {
            const km_instance& x = B->inst[i];
            const size_t one = al256((size_t)x.k * 8 * d8_of(x.d) * sizeof(float));
            B->ring_stride[i] = (int64_t)(one / sizeof(float));
            B->off_ring[i] = off;
            off = al256(off + one * (kPersistIters + 1));
            B->p_lds = std::max(B->p_lds, plain_lds_bytes(x.k, x.d, MODE_FUSED));
        }
        B->off_pring = off;  off = al256(off + (size_t)m * sizeof(float*));
        B->off_pstride = off; off = al256(off + (size_t)m * sizeof(int64_t));
        B->off_pnsl = off;   off = al256(off + (size_t)m * sizeof(int32_t));
        B->off_pdone = off;  off = al256(off + (size_t)m * sizeof(int32_t));
        B->off_pready = off; off = al256(off + (size_t)m * sizeof(int32_t));
        B->off_pctrl = off;  off = al256(off + sizeof(PersistCtrl));
        B->off_pwork = off;  off = al256(off + B->pwork.size() * sizeof(BatchWork));
    }
    B->off_wide.assign(B->wide.size(), 0);
    for (size_t w = 0; w < B->wide.size(); ++w) {
        B->off_wide[w] = off;
        off = al256(off + km_plan_workspace_bytes(B->wplan[w]));
    }
    B->off_pa = off;    off = al256(off + (size_t)m * sizeof(PassArgs));
    B->off_fa = off;    off = al256(off + (size_t)m * sizeof(FinArgs));
    B->off_work = off;  off = al256(off + B->work.size() * sizeof(BatchWork));
    B->off_fwork = off; off = al256(off + B->fwork.size() * sizeof(BatchFinWork));
    B->total = off;
}

// hipMemcpy that skips empty tables (a batch may hold no instance of some kind).
hipError_t h2d(void* dst, const void* src, size_t bytes, hipMemcpyKind kind)
{
    return bytes == 0 ? hipSuccess : hipMemcpy(dst, src, bytes, kind);
}

// Device tables: per-instance PassArgs / FinArgs pointing into the workspace;
// the wide instances' plans get their workspace slices.
km_status upload(km_batch* B)
{
    for (size_t w = 0; w < B->wide.size(); ++w) {
        const km_status st = km_plan_set_workspace(B->wplan[w], B->ws + B->off_wide[w],
                                                   km_plan_workspace_bytes(B->wplan[w]));
        if (st != KM_OK) return st;
    }
    const int m = (int)B->inst.size();
    std::vector<PassArgs> pa(m);
    std::vector<FinArgs> fa(m);
    unsigned char* ws = B->ws;
    for (int i = 0; i < m; ++i) {
        const km_instance& x = B->inst[i];
        const int D8 = d8_of(x.d);
        Partials pt;
        pt.S = reinterpret_cast<double*>(ws + B->off_S[i]);
        pt.cnt = reinterpret_cast<int32_t*>(ws + B->off_cnt[i]);
        pt.J = reinterpret_cast<double*>(ws + B->off_J[i]);
        pt.changed = reinterpret_cast<int32_t*>(ws + B->off_ch[i]);
        float* Cp = reinterpret_cast<float*>(ws + B->off_cp[i]);
        PassArgs& a = pa[i];
        std::memset(&a, 0, sizeof a);
        a.X = x.X; a.Cp = Cp; a.labels = x.labels; a.mindist = nullptr; a.part = pt; a.ctrl = nullptr;
        a.n = x.n; a.d = x.d; a.ldx = x.d; a.k = x.k; a.iter = 0; a.count_changed = 0; a.kc = x.k; a.upd_tiles = kUpdTiles;
        FinArgs& f = fa[i];
        std::memset(&f, 0, sizeof f);
        f.part = pt; f.G = B->nslots[i]; f.GJ = B->nslots[i]; f.GC = B->nslots[i];
        f.k = x.k; f.d = x.d; f.D = 8 * D8;
        f.C_old = Cp; f.ld_old = 8 * D8; f.C_new = x.C; f.ld_new = x.d; f.Cp_out = Cp;
        f.counts = x.counts; f.ctrl = nullptr; f.obj_hist = x.obj_hist; f.tol = -1.0; f.want_J = 1; f.jmode = 0;
        if (B->mixed) {
            f.jmode = 1;
            f.Jterm = reinterpret_cast<double*>(ws + B->off_jt[i]);
            f.sum_xn2 = &reinterpret_cast<const XStats*>(ws + B->off_xs[i])->sum_xn2;
        }
    }
    std::vector<BatchMix> bm(B->mixed ? m : 0);
    for (int i = 0; B->mixed && i < m; ++i) {
        const km_instance& x = B->inst[i];
        const int D16 = d16_of(x.d), kpad = kpad_of(x.k);
        BatchMix& b = bm[i];
        std::memset(&b, 0, sizeof b);
        const int nr = B->nreg[i];
        int32_t* chg = reinterpret_cast<int32_t*>(ws + B->off_chg[i]);
        MixArgs& mm = b.m;
        mm.X = x.X; mm.n = x.n; mm.d = x.d; mm.k = x.k; mm.kpad = kpad;
        mm.Ab = ws + B->off_ab[i];
        mm.bias = reinterpret_cast<const float*>(ws + B->off_bias[i]);
        mm.cs = reinterpret_cast<const CStats*>(ws + B->off_cs[i]);
        mm.Xq = nullptr; mm.xst = nullptr;
        mm.Xb = reinterpret_cast<const __bf16*>(ws + B->off_xb[i]);   // the run's BF16 copy, written with the run-level statistics
        mm.xn = reinterpret_cast<const float*>(ws + B->off_xn[i]);
        mm.u = 0.00390625f;                  // BF16 unit roundoff 2^-8
        mm.IB = ib_of(kpad);
        mm.gamma_terms = 2 * 16 * D16 + 8;
        mm.D8 = d8_of(x.d);
        mm.labels = x.labels;
        mm.rq = reinterpret_cast<int32_t*>(ws + B->off_rq[i]);
        mm.rq_count = reinterpret_cast<int32_t*>(ws + B->off_rqc[i]);
        mm.rq_per_block = B->rq_rows[i];
        mm.nreg = nr;
        mm.changed_part = chg;
        mm.ctrl = nullptr; mm.iter = 0; mm.count_changed = 0;
        RecheckArgs& r = b.r;
        r.X = x.X; r.Cp = reinterpret_cast<const float*>(ws + B->off_cp[i]); r.n = x.n; r.d = x.d; r.k = x.k;
        r.rq = mm.rq; r.rq_count = mm.rq_count; r.rq_per_block = mm.rq_per_block; r.rq_ints = kRqInts;
        r.nreg = nr; r.labels = x.labels; r.changed_part = chg + nr; r.ctrl = nullptr; r.iter = 0; r.count_changed = 0;
        b.Cp = r.Cp;
        b.D = 8 * d8_of(x.d);
        b.DP = 16 * D16;
        b.xs = reinterpret_cast<XStats*>(ws + B->off_xs[i]);
        b.xpart_max = reinterpret_cast<float*>(ws + B->off_xpm[i]);
        b.xpart_sum = reinterpret_cast<double*>(ws + B->off_xps[i]);
        b.nxb = B->nxb[i];
    }
    hipError_t e;
    if ((e = h2d(ws + B->off_pa, pa.data(), pa.size() * sizeof(PassArgs), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = h2d(ws + B->off_fa, fa.data(), fa.size() * sizeof(FinArgs), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = h2d(ws + B->off_work, B->work.data(), B->work.size() * sizeof(BatchWork),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (e = h2d(ws + B->off_fwork, B->fwork.data(), B->fwork.size() * sizeof(BatchFinWork),
                       hipMemcpyHostToDevice)) != hipSuccess)
        return bhip(e, "hipMemcpy(batch tables)");
    if (B->mixed &&
        ((e = h2d(ws + B->off_bm, bm.data(), bm.size() * sizeof(BatchMix), hipMemcpyHostToDevice)) != hipSuccess ||
         (e = h2d(ws + B->off_mwork, B->mwork.data(), B->mwork.size() * sizeof(BatchWork),
                        hipMemcpyHostToDevice)) != hipSuccess ||
         (e = h2d(ws + B->off_rwork, B->rwork.data(), B->rwork.size() * sizeof(BatchWork),
                        hipMemcpyHostToDevice)) != hipSuccess ||
         (e = h2d(ws + B->off_xwork, B->xwork.data(), B->xwork.size() * sizeof(BatchWork),
                        hipMemcpyHostToDevice)) != hipSuccess))
        return bhip(e, "hipMemcpy(batch mixed tables)");
    if (B->persistent) {
        std::vector<float*> ring(m);
        std::vector<int32_t> nsl(m);
        for (int i = 0; i < m; ++i) {
            ring[i] = reinterpret_cast<float*>(ws + B->off_ring[i]);
            nsl[i] = B->nslots[i];
        }
        if ((e = h2d(ws + B->off_pring, ring.data(), ring.size() * sizeof(float*), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = h2d(ws + B->off_pstride, B->ring_stride.data(), B->ring_stride.size() * sizeof(int64_t),
                     hipMemcpyHostToDevice)) != hipSuccess ||
            (e = h2d(ws + B->off_pnsl, nsl.data(), nsl.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = h2d(ws + B->off_pwork, B->pwork.data(), B->pwork.size() * sizeof(BatchWork),
                     hipMemcpyHostToDevice)) != hipSuccess)
            return bhip(e, "hipMemcpy(persistent tables)");
    }
    return KM_OK;
}

km_status enqueue_batch(km_batch* B, int32_t iters, hipStream_t s)
{
    const unsigned char* ws = B->ws;
    const FinArgs* fa = reinterpret_cast<const FinArgs*>(ws + B->off_fa);
    const PassArgs* pa = reinterpret_cast<const PassArgs*>(ws + B->off_pa);
    const BatchWork* work = reinterpret_cast<const BatchWork*>(ws + B->off_work);
    const BatchFinWork* fwork = reinterpret_cast<const BatchFinWork*>(ws + B->off_fwork);
    const int m = (int)B->inst.size();
    hipError_t e = hipSuccess;
    // wide instances: all their iterations on the wide stream, forked from s
    // here and joined back at the end, overlapping the class launches
    if (!B->wide.empty()) {
        if ((e = hipEventRecord(B->ev_wfork, s)) != hipSuccess ||
            (e = hipStreamWaitEvent(B->wstream, B->ev_wfork, 0)) != hipSuccess)
            return bhip(e, "wide fork");
        for (size_t w = 0; w < B->wide.size(); ++w) {
            const km_instance& x = B->wide[w];
            const km_status st = plan_enqueue_fixed(B->wplan[w], x.X, x.C, x.labels, x.counts, x.obj_hist, iters,
                                                    B->wstream);
            if (st != KM_OK) return st;
        }
        if ((e = hipEventRecord(B->ev_wjoin, B->wstream)) != hipSuccess) return bhip(e, "wide join");
    }
    auto join_wide = [&]() -> km_status {
        if (!B->wide.empty() && (e = hipStreamWaitEvent(s, B->ev_wjoin, 0)) != hipSuccess) return bhip(e, "wide join");
        return KM_OK;
    };
    if (m == 0) return join_wide();
    if (B->persistent) {
        PersistArgs p;
        p.work = reinterpret_cast<const BatchWork*>(ws + B->off_pwork);
        p.nwork = (int32_t)B->pwork.size();
        p.insts = pa;
        p.fins = fa;
        p.ring = reinterpret_cast<float* const*>(ws + B->off_pring);
        p.ring_stride = reinterpret_cast<const int64_t*>(ws + B->off_pstride);
        p.nslots = reinterpret_cast<const int32_t*>(ws + B->off_pnsl);
        p.done = reinterpret_cast<int32_t*>(B->ws + B->off_pdone);
        p.ready = reinterpret_cast<int32_t*>(B->ws + B->off_pready);
        p.ctrl = reinterpret_cast<PersistCtrl*>(B->ws + B->off_pctrl);
        p.spin_limit = (int64_t)1 << 24;
        for (int32_t t0 = 0; t0 < iters; t0 += kPersistIters) {
            p.it0 = t0;
            p.iters = std::min(kPersistIters, iters - t0);
            if ((e = launch_persist_reset(p, m, s)) != hipSuccess) return bhip(e, "persistent reset launch");
            if ((e = launch_batch_persistent(p, B->p_grid, B->p_lds, s)) != hipSuccess)
                return bhip(e, "persistent launch");
        }
        return join_wide();
    }
    if ((e = launch_batch_pad(fa, nullptr, m, s)) != hipSuccess) return bhip(e, "batch pad launch");
    const BatchMix* bm = reinterpret_cast<const BatchMix*>(ws + B->off_bm);
    const BatchWork* mwork = reinterpret_cast<const BatchWork*>(ws + B->off_mwork);
    const BatchWork* rwork = reinterpret_cast<const BatchWork*>(ws + B->off_rwork);
    const BatchWork* xwork = reinterpret_cast<const BatchWork*>(ws + B->off_xwork);
    // one launch per shape class of a phase, spread over the side streams
    auto fork = [&](int nclass) -> hipError_t {
        hipError_t ee = hipEventRecord(B->ev_fork, s);
        for (int i = 0; ee == hipSuccess && i < std::min(nclass, km_batch::kSide); ++i)
            ee = hipStreamWaitEvent(B->side[i], B->ev_fork, 0);
        return ee;
    };
    auto join = [&](int nclass) -> hipError_t {
        hipError_t ee = hipSuccess;
        for (int i = 0; ee == hipSuccess && i < std::min(nclass, km_batch::kSide); ++i) {
            ee = hipEventRecord(B->ev_join[i], B->side[i]);
            if (ee == hipSuccess) ee = hipStreamWaitEvent(s, B->ev_join[i], 0);
        }
        return ee;
    };
    auto lane_of = [&](const Group& G) { return B->side[G.lane]; };
    if (B->mixed && (e = launch_batch_prep_x(xwork, (int)B->xwork.size(), bm, m, s)) != hipSuccess)
        return bhip(e, "batch prep_x launch");
    for (int32_t t = 0; t < iters; ++t) {
        if (B->mixed) {
            if ((e = launch_batch_prep_c(bm, m, s)) != hipSuccess) return bhip(e, "batch prep_c launch");
            const int nm = (int)B->mgroups.size(), nr = (int)B->rgroups.size();
            if ((e = fork(nm)) != hipSuccess) return bhip(e, "batch fork");
            for (int g = 0; g < nm; ++g) {
                const Group& G = B->mgroups[g];
                if ((e = launch_batch_mfma(G.D8, mwork + G.first, G.count, bm, t, lane_of(G))) != hipSuccess)
                    return bhip(e, "batch MFMA launch");
            }
            if ((e = join(nm)) != hipSuccess) return bhip(e, "batch join");
            if ((e = fork(nr)) != hipSuccess) return bhip(e, "batch fork");
            for (int g = 0; g < nr; ++g) {
                const Group& G = B->rgroups[g];
                if ((e = launch_batch_recheck(G.D8, rwork + G.first, G.count, bm, t, lane_of(G))) != hipSuccess)
                    return bhip(e, "batch recheck launch");
            }
            if ((e = join(nr)) != hipSuccess) return bhip(e, "batch join");
        }
        const int np = (int)B->groups.size();
        if ((e = fork(np)) != hipSuccess) return bhip(e, "batch fork");
        for (int g = 0; g < np; ++g) {
            const Group& G = B->groups[g];
            if ((e = launch_batch_pass(G.D8, B->mixed ? MODE_UPDATE : MODE_FUSED, work + G.first, G.count, pa, t,
                                       G.lds, lane_of(G))) != hipSuccess)
                return bhip(e, "batch pass launch");
        }
        if ((e = join(np)) != hipSuccess) return bhip(e, "batch join");
        if ((e = launch_batch_finalize(fwork, (int)B->fwork.size(), fa, t, s)) != hipSuccess)
            return bhip(e, "batch finalize launch");
        if (B->mixed && (e = launch_batch_objective(fa, m, t, s)) != hipSuccess)
            return bhip(e, "batch objective launch");
    }
    return join_wide();
}

}  // namespace

extern "C" {

km_status km_batch_create(const km_instance* inst, int32_t count, km_precision prec, km_batch** out)
{
    km_set_error(KM_OK, "");
    if (!out) return berr(KM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!inst || count < 1) return berr(KM_EINVAL, "need at least one instance");
    if (prec != KM_FP32 && prec != KM_BF16 && prec != KM_FP8_E4M3) return berr(KM_EINVAL, "unknown precision %d", (int)prec);
    // FP8 batches run every instance through its own FP8 plan (the FP8 screen
    // needs a BF16 screen and refine of its open samples; there are no
    // batched FP8 kernels)
    const bool via_plans = prec == KM_FP8_E4M3;
    for (int32_t i = 0; i < count; ++i) {
        const km_instance& x = inst[i];
        if (x.n < 1 || x.n >= ((int64_t)1 << 31)) return berr(KM_EINVAL, "instance %d: n outside [1, 2^31)", i);
        if (x.d < 1 || x.d > 1024) return berr(KM_EINVAL, "instance %d: d outside [1, 1024]", i);
        if (x.k < 1 || (int64_t)x.k > x.n) return berr(KM_EINVAL, "instance %d: k outside [1, n]", i);
        if (!x.X || !x.C || !x.labels) return berr(KM_EINVAL, "instance %d: X, C and labels must be non-NULL", i);
        if ((reinterpret_cast<uintptr_t>(x.X) | reinterpret_cast<uintptr_t>(x.C)) & 15u)
            return berr(KM_EINVAL, "instance %d: X and C must be 16-byte aligned", i);
        if (via_plans || x.d > 8 * kMaxD8Plain) continue;   // checked by its plan
        if (plain_lds_bytes(x.k, x.d, MODE_FUSED) > 80 * 1024)
            return berr(KM_ENOTSUP, "instance %d: k*d too large for a batched per-label record", i);
        if (prec == KM_BF16 && kpad_of(x.k) > 16384)
            return berr(KM_ENOTSUP, "instance %d: BF16 distances support k <= 16384", i);
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return bhip(e, "hipGetDevice");
    km_batch* B = new (std::nothrow) km_batch();
    if (!B) return berr(KM_EINVAL, "out of host memory");
    B->device = dev;
    B->mixed = prec == KM_BF16;
    for (int32_t i = 0; i < count; ++i) {
        if (!via_plans && inst[i].d <= 8 * kMaxD8Plain) {
            B->inst.push_back(inst[i]);
            continue;
        }
        km_plan* p = nullptr;
        const km_status st = km_plan_create(inst[i].n, inst[i].d, inst[i].k, prec, &p);
        if (st != KM_OK) {
            const std::string why = km_last_error();
            delete B;
            return berr(st, "instance %d (d = %d): %s", i, inst[i].d, why.c_str());
        }
        B->wide.push_back(inst[i]);
        B->wplan.push_back(p);
    }
    if (!B->wide.empty() &&
        ((e = hipStreamCreateWithFlags(&B->wstream, hipStreamNonBlocking)) != hipSuccess ||
         (e = hipEventCreateWithFlags(&B->ev_wfork, hipEventDisableTiming)) != hipSuccess ||
         (e = hipEventCreateWithFlags(&B->ev_wjoin, hipEventDisableTiming)) != hipSuccess)) {
        delete B;
        return bhip(e, "wide stream / event creation");
    }
    for (int i = 0; i < km_batch::kSide; ++i) {
        if ((e = hipStreamCreateWithFlags(&B->side[i], hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&B->ev_join[i], hipEventDisableTiming)) != hipSuccess) {
            delete B;
            return bhip(e, "side stream / event creation");
        }
    }
    if ((e = hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming)) != hipSuccess) {
        delete B;
        return bhip(e, "event creation");
    }
    layout(B);
    *out = B;
    return KM_OK;
}

size_t km_batch_workspace_bytes(const km_batch* batch) { return batch ? batch->total : 0; }

km_status km_batch_set_workspace(km_batch* batch, void* ws, size_t bytes)
{
    km_set_error(KM_OK, "");
    if (!batch) return berr(KM_EINVAL, "batch is NULL");
    if (!ws) return berr(KM_EWORKSPACE, "workspace pointer is NULL");
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return berr(KM_EWORKSPACE, "workspace must be 256-byte aligned");
    if (bytes < batch->total)
        return berr(KM_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu the batch needs", bytes, batch->total);
    batch->ws = static_cast<unsigned char*>(ws);
    batch->drop_graph();
    return upload(batch);
}

km_status km_batch_set_schedule(km_batch* batch, int32_t tiles_per_block, int32_t order)
{
    km_set_error(KM_OK, "");
    if (!batch) return berr(KM_EINVAL, "batch is NULL");
    if (tiles_per_block < 1 || tiles_per_block > kMaxTilesPerBlock || (order != 0 && order != 1))
        return berr(KM_EINVAL, "bad schedule (tiles per block in [1, %d], order 0 or 1)", kMaxTilesPerBlock);
    batch->tpb = tiles_per_block;
    batch->order = order;
    batch->drop_graph();
    batch->ws = nullptr;   // layout changes: a workspace must be bound again
    layout(batch);
    return KM_OK;
}

int32_t km_batch_num_classes(const km_batch* batch)
{
    return batch ? (int32_t)batch->classes.size() : 0;
}

km_status km_batch_class_info(const km_batch* batch, int32_t cls, int32_t* d8, int32_t* lds_bytes,
                              int32_t* instances, int32_t* tiles_per_block)
{
    km_set_error(KM_OK, "");
    if (!batch) return berr(KM_EINVAL, "batch is NULL");
    if (cls < 0 || cls >= (int32_t)batch->classes.size()) return berr(KM_EINVAL, "class %d out of range", cls);
    const auto key = batch->classes[cls];
    int cnt = 0, tpb = batch->tpb;
    for (size_t i = 0; i < batch->inst.size(); ++i)
        if (class_of(batch, batch->inst[i]) == key) { ++cnt; tpb = batch->tpb_inst[i]; }
    if (d8) *d8 = key.first;
    if (lds_bytes) *lds_bytes = (int32_t)key.second;
    if (instances) *instances = cnt;
    if (tiles_per_block) *tiles_per_block = tpb;
    return KM_OK;
}

km_status km_batch_set_class_schedule(km_batch* batch, int32_t cls, int32_t tiles_per_block)
{
    km_set_error(KM_OK, "");
    if (!batch) return berr(KM_EINVAL, "batch is NULL");
    if (cls < 0 || cls >= (int32_t)batch->classes.size()) return berr(KM_EINVAL, "class %d out of range", cls);
    if (tiles_per_block < 0 || tiles_per_block > kMaxTilesPerBlock)
        return berr(KM_EINVAL, "bad tiles_per_block %d (0, or 1 to %d)", tiles_per_block, kMaxTilesPerBlock);
    batch->class_tpb[batch->classes[cls]] = tiles_per_block;
    batch->drop_graph();
    batch->ws = nullptr;   // layout changes: a workspace must be bound again
    layout(batch);
    return KM_OK;
}

km_status km_batch_use_persistent(km_batch* batch, int32_t enable)
{
    km_set_error(KM_OK, "");
    if (!batch) return berr(KM_EINVAL, "batch is NULL");
    if (enable) {
        if (batch->mixed || batch->inst.empty() && batch->wide.empty())
            return berr(KM_ENOTSUP, "the persistent launch runs FP32 batches");
        for (const km_instance& x : batch->inst)
            if (d8_of(x.d) > 8) return berr(KM_ENOTSUP, "the persistent launch takes instances of d <= 64");
        if (!batch->wplan.empty() && batch->inst.empty())
            return berr(KM_ENOTSUP, "the persistent launch needs instances of d <= 64");
    }
    batch->persistent = enable != 0;
    batch->drop_graph();
    batch->ws = nullptr;   // layout changes: a workspace must be bound again
    layout(batch);
    if (batch->persistent) {
        const int per_cu = persistent_blocks_per_cu(batch->p_lds);
        if (per_cu < 1) {
            batch->persistent = false;
            layout(batch);
            return berr(KM_EHIP, "occupancy query for the persistent launch failed");
        }
        int ncu = 0;
        hipError_t e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, batch->device);
        if (e != hipSuccess) return bhip(e, "hipDeviceGetAttribute");
        batch->p_grid = std::max(1, ncu * per_cu);
    }
    return KM_OK;
}

km_status km_batch_persistent_status(km_batch* batch, int32_t* aborted)
{
    km_set_error(KM_OK, "");
    if (!batch || !aborted) return berr(KM_EINVAL, "batch and aborted must be non-NULL");
    *aborted = 0;
    if (!batch->persistent || !batch->ws) return KM_OK;
    PersistCtrl c;
    hipError_t e = hipMemcpy(&c, batch->ws + batch->off_pctrl, sizeof c, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return bhip(e, "hipMemcpy(persistent control)");
    *aborted = c.abort;
    return KM_OK;
}

km_status km_batch_use_graphs(km_batch* batch, int32_t enable)
{
    km_set_error(KM_OK, "");
    if (!batch) return berr(KM_EINVAL, "batch is NULL");
    batch->use_graph = enable != 0;
    batch->drop_graph();
    return KM_OK;
}

void km_batch_destroy(km_batch* batch) { delete batch; }

km_status kmeans_lloyd_batched(km_batch* B, int32_t iters, hipStream_t stream)
{
    km_set_error(KM_OK, "");
    if (!B) return berr(KM_EINVAL, "batch is NULL");
    if (!B->ws) return berr(KM_EWORKSPACE, "no workspace bound to the batch (km_batch_set_workspace)");
    if (iters < 1) return berr(KM_EINVAL, "iterations = %d must be >= 1", iters);
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return bhip(e, "hipGetDevice");
    if (cur != B->device) return berr(KM_EINVAL, "batch was created on device %d but device %d is current", B->device, cur);
    if (!B->use_graph) return enqueue_batch(B, iters, stream);
    if (!B->gexec || B->g_iters != iters) {
        B->drop_graph();
        if (!B->cap_stream && (e = hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking)) != hipSuccess)
            return bhip(e, "hipStreamCreateWithFlags");
        if ((e = hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return bhip(e, "hipStreamBeginCapture");
        km_status cs = enqueue_batch(B, iters, B->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t ee = hipStreamEndCapture(B->cap_stream, &g);
        if (cs != KM_OK) { if (g) (void)hipGraphDestroy(g); return cs; }
        if (ee != hipSuccess) return bhip(ee, "hipStreamEndCapture");
        ee = hipGraphInstantiate(&B->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ee != hipSuccess) { B->gexec = nullptr; return bhip(ee, "hipGraphInstantiate"); }
        B->g_iters = iters;
    }
    if ((e = hipGraphLaunch(B->gexec, stream)) != hipSuccess) return bhip(e, "hipGraphLaunch");
    return KM_OK;
}

}  // extern "C"
