// Serving loop: entropy queries on registered graphs, admitted by an HBM
// budget, run with continuous batching.
//
// A query is split into slot tasks of at most max_cols probe columns.  An
// admitted task gets a slot (two or four 16-column FP32 tasks of one graph
// that wait together may share a group slot): its matrix stays the
// registered graph's,
// its vectors and Lanczos state live in the server's arena.  One tick
// advances every active slot by one Lanczos step in a few launches
// (normalize, SpMM + recurrence, long rows, finalize) whatever graphs the
// slots belong to; a task that reaches its step count gets its quadrature
// and leaves, and waiting tasks are admitted between ticks as mailbox
// entries and arena space free up.  A task's arithmetic depends only on its
// own graph, probes and step count (in a group slot too), so a query gives
// the same bits alone and in any mix.
//
// With rel_eps > 0 a query first runs a pilot of pilot_probes columns; the
// step cap comes from the a-priori bound of Proposition 4.4 with Remark 2.3
// (lambda_max from a Gershgorin bound, S(A) from below by -log tr(A^2)), the
// probe count from the pilot's sample standard deviation (Remarks 5.1, 5.2:
// half of the relative budget each).  A task stops earlier at the first
// checked step at which the a-posteriori upper bound of Theorem 4.8 meets the
// same per-form target for all its probes; the device records that step and
// the quadrature uses it, whenever the host learns of it.
//
// The scheduling (tickets, queue, admission, ticks, stages, completion) is
// the host-only ServeCore (serve_core.cpp); this file is its executor on the
// GPU: slot state carved from the arena, probe blocks, the step launches of
// a tick, quadrature and the copies of results to pinned host buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ctx_internal.h"
#include "serve_core.h"
#include "serve_host.h"

using namespace vne;
using namespace vne::rt;

namespace {

size_t rnd(size_t b) { return (b + 255) / 256 * 256; }

// Device pointers of a slot's state, carved from its arena block.
struct DevTask {
    char *P[2] = {nullptr, nullptr}, *V[2] = {nullptr, nullptr};
    double *alpha = nullptr, *beta = nullptr, *st_alpha = nullptr, *st_inv = nullptr, *st_coup = nullptr;
    double *norm2 = nullptr, *mean = nullptr, *partials = nullptr, *probe_part = nullptr;
    double *seg_acc = nullptr, *long_part = nullptr, *level2 = nullptr;
    int32_t *k_eff = nullptr;
    double *b_lo = nullptr, *b_hi = nullptr;
    int2 *d_state = nullptr;         // [n_mem] {uid, first step within tol}
};

// Arena bytes of a task of width m_pad and k steps on a graph.
size_t task_bytes_of(const GraphSet *set, int m_pad, int k, bool fp64) {
    const size_t es = fp64 ? 8 : 4;
    const size_t blk = rnd((size_t)set->n * m_pad * es);
    const Schedule &sc = set->sched;
    size_t b = 4 * blk;
    b += 2 * rnd((size_t)m_pad * k * 8);
    b += 5 * rnd((size_t)m_pad * 8) + rnd((size_t)m_pad * 4);
    b += rnd((size_t)sc.n_blocks() * 3 * m_pad * 8);
    b += rnd((size_t)set->probe_blocks * m_pad * 8);
    b += rnd((size_t)std::max(1, sc.n_seg) * m_pad * 8);
    b += rnd((size_t)std::max(1, sc.n_long) * 3 * m_pad * 8);
    b += rnd((size_t)kSlotLevel2 * 3 * m_pad * 8);
    b += 2 * rnd((size_t)m_pad * 8) + 256;
    return b;
}

DevTask carve(const ServeTask &t, char *base, const GraphSet *set, bool fp64) {
    DevTask d;
    const size_t es = fp64 ? 8 : 4;
    const Schedule &sc = set->sched;
    char *p = base;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += rnd(bytes);
        return r;
    };
    const size_t blk = (size_t)set->n * t.m_pad * es;
    d.P[0] = take(blk);
    d.P[1] = take(blk);
    d.V[0] = take(blk);
    d.V[1] = take(blk);
    d.alpha = (double *)take((size_t)t.m_pad * t.k * 8);
    d.beta = (double *)take((size_t)t.m_pad * t.k * 8);
    d.st_alpha = (double *)take((size_t)t.m_pad * 8);
    d.st_inv = (double *)take((size_t)t.m_pad * 8);
    d.st_coup = (double *)take((size_t)t.m_pad * 8);
    d.norm2 = (double *)take((size_t)t.m_pad * 8);
    d.mean = (double *)take((size_t)t.m_pad * 8);
    d.k_eff = (int32_t *)take((size_t)t.m_pad * 4);
    d.partials = (double *)take((size_t)sc.n_blocks() * 3 * t.m_pad * 8);
    d.probe_part = (double *)take((size_t)set->probe_blocks * t.m_pad * 8);
    d.seg_acc = (double *)take((size_t)std::max(1, sc.n_seg) * t.m_pad * 8);
    d.long_part = (double *)take((size_t)std::max(1, sc.n_long) * 3 * t.m_pad * 8);
    d.level2 = (double *)take((size_t)kSlotLevel2 * 3 * t.m_pad * 8);
    d.b_lo = (double *)take((size_t)t.m_pad * 8);
    d.b_hi = (double *)take((size_t)t.m_pad * 8);
    d.d_state = (int2 *)take(256);
    return d;
}

bool all_adaptive(const ServeTask &t) {
    for (int i = 0; i < t.n_mem; ++i)
        if (!t.mem[i].adaptive) return false;
    return true;
}

// The executor's state of a query: its graph, pinned result buffer
// (forms [psi_cap], estimate, flags) and completion event.
struct GpuQuery {
    Graph *g = nullptr;
    GraphSet *set = nullptr;
    double *h_buf = nullptr;
    hipEvent_t ev = nullptr;
};

GpuQuery *gq(ServeQuery &q) { return static_cast<GpuQuery *>(q.x); }
const GpuQuery *gq(const ServeQuery &q) { return static_cast<const GpuQuery *>(q.x); }

class GpuExec final : public ServeExec {
public:
    vne_ctx *ctx = nullptr;
    bool fp64 = false, desing = false;
    int psi_cap = 0;
    int stop_rule = VNE_STOP_BOUND;  // what a task's check compares with its tolerance
    hipStream_t stream = nullptr;
    // the width classes of a tick (each its normalize, step and long-row
    // launches) touch disjoint tasks: they run on the stream and up to kSide
    // side streams, forked after the tick's descriptor copy and joined before
    // its finalize
    // (two side streams measured best: 486 and 520 queries/s at 1000 and
    // 2000 req/s against 447 and 479 on one stream, 485 and 510 with one
    // side stream, 475 and 493 with three)
    static constexpr int kSide = 3;
    hipStream_t side[kSide] = {};
    hipEvent_t fork_ev = nullptr, join_ev[kSide] = {};
    int n_side = 2;
    DevBuf arena_mem;
    std::vector<double *> pinned_pool;
    std::vector<hipEvent_t> event_pool;
    static constexpr int kRing = 4;
    char *stage[kRing] = {};
    size_t stage_cap[kRing] = {};
    hipEvent_t ring_ev[kRing] = {};
    bool ring_used[kRing] = {};
    int ring_pos = 0;
    char *d_desc = nullptr;
    size_t d_desc_cap = 0;
    int2 *mailbox = nullptr;         // pinned [max_slots]: stop records
    // [max_slots] on the device: each check's record at its mailbox entry,
    // the whole array copied to the pinned mailbox once per checking tick
    DevBuf mail;
    int max_slots = 0;
    // flags word of the columns of a group slot's member that has ended (its
    // query's block may belong to another query by now)
    DevBuf sink;
    std::mutex err_mu;
    std::string err;

    vne_status hip_err(hipError_t e, const char *what) {
        if (e == hipSuccess) return VNE_OK;
        std::lock_guard<std::mutex> lk(err_mu);
        err = std::string(what) + ": " + hipGetErrorString(e);
        return VNE_EDEVICE;
    }

    char *arena_base() const { return (char *)arena_mem.p; }
    double *d_psi(const ServeQuery &q) const { return (double *)(arena_base() + q.off); }
    double *d_est(const ServeQuery &q) const { return (double *)(arena_base() + q.off + rnd((size_t)psi_cap * 8)); }
    int32_t *d_flags(const ServeQuery &q) const {
        return (int32_t *)(arena_base() + q.off + rnd((size_t)psi_cap * 8) + 256);
    }
    // the most steps a quadrature of the query took (the word after the flags)
    int32_t *d_steps(const ServeQuery &q) const { return d_flags(q) + 1; }
    DevTask dev(const ServeTask &t, const ServeQuery &q) const {
        return carve(t, arena_base() + t.off, gq(q)->set, fp64);
    }

    void thread_init() override { (void)hipSetDevice(ctx->device); }

    uint64_t task_bytes(const ServeQuery &q, int m_pad, int k) override {
        return task_bytes_of(gq(q)->set, m_pad, k, fp64);
    }

    void tile(int m, int *mt, int *m_pad) override {
        *mt = choose_tile(m, fp64, 0);
        *m_pad = pad_columns(m, *mt);
    }

    double *get_pinned() {
        if (!pinned_pool.empty()) {
            double *p = pinned_pool.back();
            pinned_pool.pop_back();
            return p;
        }
        void *p = nullptr;
        if (hipHostMalloc(&p, (size_t)(psi_cap + 2) * 8, hipHostMallocDefault) != hipSuccess) return nullptr;
        return (double *)p;
    }

    hipEvent_t get_event() {
        if (!event_pool.empty()) {
            hipEvent_t e = event_pool.back();
            event_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }

    vne_status open_query(ServeQuery &q) override {
        GpuQuery *x = gq(q);
        x->h_buf = get_pinned();
        x->ev = get_event();
        if (!x->h_buf || !x->ev) return hip_err(hipErrorOutOfMemory, "pinned buffer or event");
        return hip_err(hipMemsetAsync(d_flags(q), 0, 8, stream), "hipMemsetAsync");   // flags and steps
    }

    // Probe block of member i (the query's hash columns col0.., eq. (3.8))
    // into its columns of the slot.
    vne_status member_probes(const ServeTask &t, const DevTask &d, int i, const ServeQuery &q) {
        const ServeMember &u = t.mem[i];
        const GraphSet *set = gq(q)->set;
        const size_t es = fp64 ? 8 : 4;
        ProbeArgs pa{};
        pa.gen = GEN_RADEMACHER;
        pa.n = (int32_t)set->n;
        pa.m = u.m;
        pa.m_pad = t.group() ? t.mt : t.m_pad;
        pa.mt = t.mt;
        pa.ld_out = t.m_pad;
        pa.col_offset = u.col0;
        pa.seed = q.q.seed;
        pa.keys = (const int64_t *)set->keys.p;
        pa.desing = desing ? 1 : 0;
        pa.P_out = d.P[0] + (size_t)u.c_off * es;
        pa.partials = d.probe_part;
        pa.n_blocks = set->probe_blocks;
        pa.mean = d.mean + u.c_off;
        pa.norm2 = d.norm2 + u.c_off;
        pa.st_alpha = d.st_alpha + u.c_off;
        pa.st_inv = d.st_inv + u.c_off;
        pa.st_coup = d.st_coup + u.c_off;
        pa.k_eff = d.k_eff + u.c_off;
        pa.k = t.k;
        pa.block_row_begin = (const int32_t *)set->probe_rows.p;
        pa.block_graph = (const int32_t *)set->probe_block_graph.p;
        pa.graph_block_begin = (const int32_t *)set->probe_graph_begin.p;
        pa.graph_row_begin = (const int64_t *)set->graph_row_begin.p;
        pa.n_graphs = 1;
        return hip_err(launch_probe(pa, fp64, stream), "launch_probe");
    }

    vne_status start_task(ServeTask &t, ServeQuery *const *qm) override {
        const DevTask d = dev(t, *qm[0]);
        VNE_TRY(hip_err(hipMemsetAsync(d.d_state, 0, sizeof(int2) * t.n_mem, stream), "hipMemsetAsync"));
        for (int i = 0; i < t.n_mem; ++i) VNE_TRY(member_probes(t, d, i, *qm[i]));
        // zero v_0
        return hip_err(hipMemsetAsync(d.V[1], 0, (size_t)gq(*qm[0])->set->n * t.m_pad * (fp64 ? 8 : 4), stream),
                       "hipMemsetAsync");
    }

    StepArgs step_args(const ServeTask &t, const DevTask &d, const GraphSet *set) const {
        StepArgs a{};
        const int j = t.j + 1;
        a.row_ptr = set->d_row_ptr;
        a.col = set->d_col;
        a.val = fp64 ? set->val64.p : set->val32.p;
        a.scale = set->scale;
        a.n = (int32_t)set->n;
        a.m_pad = t.m_pad;
        a.mt = t.mt;
        a.n_tiles = t.m_pad / t.mt;
        a.P_in = d.P[(j - 1) & 1];
        a.P_out = d.P[j & 1];
        a.V_out = d.V[(j - 1) & 1];
        a.V_prev = d.V[j & 1];
        a.V_cur = a.V_out;
        a.two_pass = 1;
        a.st_alpha = d.st_alpha;
        a.st_inv = d.st_inv;
        a.st_coup = d.st_coup;
        a.segs = (const SegItem *)set->segs.p;
        a.n_seg = set->sched.n_seg;
        a.seg_len = set->sched.seg_len;
        a.block_ranges = (const int4 *)set->block_ranges.p;
        a.n_blocks = set->sched.n_blocks();
        a.seg_acc = d.seg_acc;
        a.n_long = set->sched.n_long;
        a.long_first = (const int32_t *)set->long_first.p;
        a.long_nseg = (const int32_t *)set->long_nseg.p;
        a.long_part = d.long_part;
        a.partials = d.partials;
        a.stop_state = all_adaptive(t) ? d.d_state : nullptr;
        a.stop_uid = t.mem[0].uid;
        a.stop_count = t.n_mem;
        return a;
    }

    // flags_m[i]: the flags word of member i's query
    FinalizeArgs fin_args(const ServeTask &t, const DevTask &d, const GraphSet *set, int32_t *const *flags_m) const {
        FinalizeArgs f{};
        f.partials = d.partials;
        f.long_part = d.long_part;
        f.level2 = d.level2;
        f.n_level2 = kSlotLevel2;
        f.n_blocks = set->sched.n_blocks();
        f.n_long = set->sched.n_long;
        f.mt = t.mt;
        f.m_pad = t.m_pad;
        f.m = t.m;
        f.step = t.j + 1;
        f.k = t.k;
        f.tau = fp64 ? std::ldexp(1.0, -23) : std::ldexp(1.0, -18);
        f.st_alpha = d.st_alpha;
        f.st_inv = d.st_inv;
        f.st_coup = d.st_coup;
        f.alpha = d.alpha;
        f.beta = d.beta;
        f.k_eff = d.k_eff;
        f.flags = flags_m[0];
        f.n_graphs = 1;
        f.stop_state = all_adaptive(t) ? d.d_state : nullptr;
        f.stop_uid = t.mem[0].uid;
        f.stop_count = t.n_mem;
        if (t.group()) {
            for (int i = 0; i < t.n_mem; ++i) f.flags_mem[i] = flags_m[i];
            f.mem_cols = t.mt;
        }
        return f;
    }

    // One Lanczos step of every active slot.
    vne_status tick(const std::vector<ServeTask> &active, const std::vector<ServeQuery *> &qs) override {
        const int A = (int)active.size();
        // descriptors: StepArgs[A], FinalizeArgs[A], then per tile width the
        // step and long-row maps (and per group size those of the group
        // slots), then the finalize map
        std::vector<DevTask> dt(A);
        std::vector<StepArgs> sa(A);
        std::vector<FinalizeArgs> fa(A);
        std::map<int, std::vector<int4>> smap, lmap, gmap, glmap;
        std::vector<int2> fmap;
        auto flags_of = [&](const ServeQuery *q) { return q ? d_flags(*q) : (int32_t *)sink.p; };
        for (int i = 0; i < A; ++i) {
            const ServeTask &t = active[i];
            ServeQuery *const *qi = qs.data() + (size_t)kMaxMembers * i;
            // a running member's query (the members of a group share the graph)
            const ServeQuery *q0 = nullptr;
            for (int mi = 0; mi < t.n_mem && !q0; ++mi) q0 = qi[mi];
            const GraphSet *set = gq(*q0)->set;
            dt[i] = dev(t, *q0);
            sa[i] = step_args(t, dt[i], set);
            int32_t *flags_m[kMaxMembers] = {};
            for (int mi = 0; mi < t.n_mem; ++mi) flags_m[mi] = flags_of(qi[mi]);
            fa[i] = fin_args(t, dt[i], set, flags_m);
            const int nt = t.m_pad / t.mt, nb = set->sched.n_blocks();
            if (t.group()) {
                auto &gm = gmap[t.n_mem];
                for (int b = 0; b < nb; ++b) gm.push_back(make_int4(i, b, 0, 0));
            } else {
                auto &sm = smap[t.mt];
                for (int tile = 0; tile < nt; ++tile)
                    for (int b = 0; b < nb; ++b) sm.push_back(make_int4(i, b, tile, 0));
            }
            if (set->sched.n_long > 0) {
                const int per = long_rows_per_group(t.mt, fp64);
                auto &lm = t.group() ? glmap[t.n_mem] : lmap[t.mt];
                for (int tile = 0; tile < nt; ++tile)
                    for (int gi = 0; gi < (set->sched.n_long + per - 1) / per; ++gi)
                        lm.push_back(make_int4(i, gi, tile, 0));
            }
            for (int ch = 0; ch < (t.m_pad + kFinalizeCols - 1) / kFinalizeCols; ++ch) fmap.push_back(make_int2(i, ch));
        }
        // a-posteriori checks (Theorem 4.8) of adaptive members after this
        // step: from step 3 on, every other step
        std::vector<BoundArgs> ba;
        std::vector<StopArgs> sta;
        std::vector<int2> bmap;
        for (int i = 0; i < A; ++i) {
            const ServeTask &t = active[i];
            const DevTask &d = dt[i];
            const int j = t.j + 1;
            if (j < 3 || j % 2 == 0 || j >= t.k) continue;
            for (int mi = 0; mi < t.n_mem; ++mi) {
                const ServeMember &u = t.mem[mi];
                if (!u.adaptive || u.ended) continue;
                const ServeQuery *q = qs[(size_t)kMaxMembers * i + mi];
                const Graph *g = gq(*q)->g;
                const int64_t co = u.c_off;
                BoundArgs b{};
                b.alpha = d.alpha + co * t.k;
                b.beta = d.beta + co * t.k;
                b.k_eff = d.k_eff + co;
                b.norm2 = d.norm2 + co;
                b.k = t.k;
                b.m = u.m;
                b.steps = j;
                b.lam_hi = g->lambda_ub;
                b.lam_lo = g->lambda_ub * kLamLoFraction;
                b.n_grid = kBoundGrid;
                b.lo = d.b_lo + co;
                b.hi = d.b_hi + co;
                b.flags = d_flags(*q);
                b.stop_state = d.d_state + mi;
                b.stop_uid = u.uid;
                b.stop_count = 1;
                for (int grp = 0; grp < (u.m + 3) / 4; ++grp) bmap.push_back(make_int2((int)ba.size(), grp));
                ba.push_back(b);
                StopArgs sc{};
                sc.lo = d.b_lo + co;
                sc.hi = d.b_hi + co;
                sc.estimate = stop_rule == VNE_STOP_ESTIMATE ? 1 : 0;
                sc.m = u.m;
                sc.tol = u.tol;
                sc.step = j;
                sc.uid = u.uid;
                sc.state = d.d_state + mi;
                sc.mail = (int2 *)mail.p + u.slot;
                sta.push_back(sc);
            }
        }
        size_t bytes = rnd(sizeof(StepArgs) * A) + rnd(sizeof(FinalizeArgs) * A) + rnd(sizeof(int2) * fmap.size());
        bytes += rnd(sizeof(BoundArgs) * ba.size()) + rnd(sizeof(int2) * bmap.size()) + rnd(sizeof(StopArgs) * sta.size());
        for (auto &kv : smap) bytes += rnd(sizeof(int4) * kv.second.size());
        for (auto &kv : lmap) bytes += rnd(sizeof(int4) * kv.second.size());
        for (auto &kv : gmap) bytes += rnd(sizeof(int4) * kv.second.size());
        for (auto &kv : glmap) bytes += rnd(sizeof(int4) * kv.second.size());
        // staging ring: wait until the copy that last used this slot has run
        const int r = ring_pos;
        ring_pos = (r + 1) % kRing;
        if (ring_used[r]) VNE_TRY(hip_err(hipEventSynchronize(ring_ev[r]), "hipEventSynchronize"));
        if (stage_cap[r] < bytes) {
            if (stage[r]) VNE_TRY(hip_err(hipHostFree(stage[r]), "hipHostFree"));
            stage[r] = nullptr;
            const size_t cap = std::max(bytes, 2 * stage_cap[r]);
            VNE_TRY(hip_err(hipHostMalloc((void **)&stage[r], cap, hipHostMallocDefault), "hipHostMalloc"));
            stage_cap[r] = cap;
        }
        if (d_desc_cap < bytes) {
            // kernels of earlier ticks may still read the old buffer
            VNE_TRY(hip_err(hipStreamSynchronize(stream), "hipStreamSynchronize"));
            if (d_desc) VNE_TRY(hip_err(hipFree(d_desc), "hipFree"));
            d_desc = nullptr;
            const size_t cap = std::max(bytes, 2 * d_desc_cap);
            VNE_TRY(hip_err(hipMalloc((void **)&d_desc, cap), "hipMalloc"));
            d_desc_cap = cap;
        }
        char *h = stage[r];
        size_t off = 0;
        auto put = [&](const void *src, size_t n) {
            std::memcpy(h + off, src, n);
            const size_t o = off;
            off += rnd(n);
            return d_desc + o;
        };
        const StepArgs *d_sa = (const StepArgs *)put(sa.data(), sizeof(StepArgs) * A);
        const FinalizeArgs *d_fa = (const FinalizeArgs *)put(fa.data(), sizeof(FinalizeArgs) * A);
        const int2 *d_fm = (const int2 *)put(fmap.data(), sizeof(int2) * fmap.size());
        std::map<int, const int4 *> d_sm, d_lm;
        for (auto &kv : smap) d_sm[kv.first] = (const int4 *)put(kv.second.data(), sizeof(int4) * kv.second.size());
        for (auto &kv : lmap) d_lm[kv.first] = (const int4 *)put(kv.second.data(), sizeof(int4) * kv.second.size());
        std::map<int, const int4 *> d_gm, d_glm;
        for (auto &kv : gmap) d_gm[kv.first] = (const int4 *)put(kv.second.data(), sizeof(int4) * kv.second.size());
        for (auto &kv : glmap) d_glm[kv.first] = (const int4 *)put(kv.second.data(), sizeof(int4) * kv.second.size());
        const BoundArgs *d_ba = (const BoundArgs *)put(ba.data(), sizeof(BoundArgs) * ba.size());
        const int2 *d_bm = (const int2 *)put(bmap.data(), sizeof(int2) * bmap.size());
        const StopArgs *d_st = (const StopArgs *)put(sta.data(), sizeof(StopArgs) * sta.size());
        VNE_TRY(hip_err(hipMemcpyAsync(d_desc, h, off, hipMemcpyHostToDevice, stream), "hipMemcpyAsync"));
        VNE_TRY(hip_err(hipEventRecord(ring_ev[r], stream), "hipEventRecord"));
        ring_used[r] = true;
        // class 0 (the group slots when there are any, which carry most of
        // the work at saturation) on the tick's own stream, class i >= 1 on
        // side stream (i - 1) mod (the side streams this tick uses: at most
        // n_side, and no more than the classes after the first)
        const int n_cls = (int)gmap.size() + (int)smap.size();
        const int n_str = std::min(n_cls, n_side + 1);
        if (n_str > 1) VNE_TRY(hip_err(hipEventRecord(fork_ev, stream), "hipEventRecord"));
        for (int j = 1; j < n_str; ++j)
            VNE_TRY(hip_err(hipStreamWaitEvent(side[j - 1], fork_ev, 0), "hipStreamWaitEvent"));
        int cls = 0;
        auto class_stream = [&]() {
            const int i = cls++;
            return i == 0 || n_str == 1 ? stream : side[(i - 1) % (n_str - 1)];
        };
        for (auto &kv : gmap) {
            const int members = kv.first;
            const auto lit = glmap.find(members);
            const int n_long = lit == glmap.end() ? 0 : (int)lit->second.size();
            VNE_TRY(hip_err(launch_step_groups(d_sa, d_gm[members], (int32_t)kv.second.size(),
                                               n_long ? d_glm[members] : nullptr, n_long, members, class_stream()),
                            "launch_step_groups"));
        }
        for (auto &kv : smap) {
            const int mt = kv.first;
            const auto lit = lmap.find(mt);
            const int n_long = lit == lmap.end() ? 0 : (int)lit->second.size();
            VNE_TRY(hip_err(launch_step_slots(d_sa, d_sm[mt], (int32_t)kv.second.size(), n_long ? d_lm[mt] : nullptr,
                                              n_long, mt, fp64, class_stream()),
                            "launch_step_slots"));
        }
        for (int j = 1; j < n_str; ++j) {
            VNE_TRY(hip_err(hipEventRecord(join_ev[j - 1], side[j - 1]), "hipEventRecord"));
            VNE_TRY(hip_err(hipStreamWaitEvent(stream, join_ev[j - 1], 0), "hipStreamWaitEvent"));
        }
        VNE_TRY(hip_err(launch_finalize_slots(d_fa, d_fm, (int32_t)fmap.size(), stream), "launch_finalize_slots"));
        if (!sta.empty()) {
            VNE_TRY(hip_err(launch_error_bound(d_ba, d_bm, (int32_t)bmap.size(), stream), "launch_error_bound"));
            VNE_TRY(hip_err(launch_stop_check(d_st, (int32_t)sta.size(), stream), "launch_stop_check"));
            // an entry of a slot's earlier owner carries another uid: the
            // host passes over it
            VNE_TRY(hip_err(hipMemcpyAsync(mailbox, mail.p, sizeof(int2) * max_slots, hipMemcpyDeviceToHost, stream),
                            "hipMemcpyAsync"));
        }
        return VNE_OK;
    }

    void stop_record(int slot, int32_t *uid, int32_t *step) override {
        const volatile int2 *mb = mailbox + slot;
        *uid = mb->x;
        *step = mb->y;
    }

    vne_status quadrature(const ServeTask &t, int i, ServeQuery &q, int steps) override {
        const ServeMember &u = t.mem[i];
        const DevTask d = dev(t, q);
        // an adaptive task's own stop record (if the device made one) decides
        // the step count, whenever the host noticed it (a task can reach its
        // cap before the record reaches the host: the device's count of the
        // steps taken is the one reported)
        const int64_t co = u.c_off;
        return hip_err(launch_quadrature(d.alpha + co * t.k, d.beta + co * t.k, d.k_eff + co, d.norm2 + co, t.k,
                                         steps, u.m, d_psi(q) + u.col0, d_flags(q), stream, fp64,
                                         u.adaptive ? d.d_state + i : nullptr, u.uid, nullptr, d_steps(q)),
                       "launch_quadrature");
    }

    vne_status issue_stage(ServeQuery &q) override {
        GpuQuery *x = gq(q);
        VNE_TRY(hip_err(hipMemcpyAsync(x->h_buf, d_psi(q), (size_t)q.cols_issued * 8, hipMemcpyDeviceToHost, stream),
                        "hipMemcpyAsync"));
        VNE_TRY(hip_err(hipMemcpyAsync(x->h_buf + psi_cap + 1, d_flags(q), 4, hipMemcpyDeviceToHost, stream),
                        "hipMemcpyAsync"));
        return hip_err(hipEventRecord(x->ev, stream), "hipEventRecord");
    }

    // estimator combine (eq. (3.8)) on the device and the copy of psi,
    // estimate and flags to the host
    vne_status issue_final(ServeQuery &q) override {
        GpuQuery *x = gq(q);
        VNE_TRY(hip_err(launch_combine(d_psi(q), q.N, 0, 0, d_est(q), stream), "launch_combine"));
        VNE_TRY(hip_err(hipMemcpyAsync(x->h_buf, d_psi(q), (size_t)q.N * 8, hipMemcpyDeviceToHost, stream),
                        "hipMemcpyAsync"));
        VNE_TRY(hip_err(hipMemcpyAsync(x->h_buf + q.N, d_est(q), 8, hipMemcpyDeviceToHost, stream), "hipMemcpyAsync"));
        // flags and the step count, adjacent words
        VNE_TRY(hip_err(hipMemcpyAsync(x->h_buf + q.N + 1, d_flags(q), 8, hipMemcpyDeviceToHost, stream),
                        "hipMemcpyAsync"));
        return hip_err(hipEventRecord(x->ev, stream), "hipEventRecord");
    }

    vne_status ready(ServeQuery &q, bool block, bool *done) override {
        hipError_t e = hipEventQuery(gq(q)->ev);
        if (e == hipErrorNotReady && block) e = hipEventSynchronize(gq(q)->ev);
        *done = e == hipSuccess;
        return e == hipErrorNotReady ? VNE_OK : hip_err(e, "hipEventQuery");
    }

    const double *forms(ServeQuery &q) override { return q.x ? gq(q)->h_buf : nullptr; }
    double estimate(ServeQuery &q) override { return gq(q)->h_buf[q.N]; }
    int32_t flags(ServeQuery &q, bool final) override {
        int32_t fl = 0;
        std::memcpy(&fl, gq(q)->h_buf + (final ? q.N + 1 : psi_cap + 1), 4);
        return fl;
    }
    int32_t steps_taken(ServeQuery &q) override {
        int32_t st = 0;
        std::memcpy(&st, reinterpret_cast<const char *>(gq(q)->h_buf + q.N + 1) + 4, 4);
        return st;
    }

    void close_query(ServeQuery &q) override {
        GpuQuery *x = gq(q);
        if (!x) return;
        if (x->h_buf) pinned_pool.push_back(x->h_buf);
        if (x->ev) event_pool.push_back(x->ev);
        delete x;
        q.x = nullptr;
    }

    void release_graph(ServeQuery &q) override {
        GpuQuery *x = gq(q);
        if (!x || !x->g) return;
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        x->g->in_use--;
        x->g = nullptr;
    }

    std::string error_text() override {
        std::lock_guard<std::mutex> lk(err_mu);
        return err;
    }
};

}  // namespace

struct vne_server {
    GpuExec exec;
    std::unique_ptr<ServeCore> core;
    std::thread worker;
};

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" vne_status vne_server_start(vne_ctx *c, const vne_server_cfg *cfg, vne_server **out) {
    if (!c) return VNE_EINVAL;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    c->err.clear();
    if (!cfg || !out) return fail(c, VNE_EINVAL, "NULL argument");
    *out = nullptr;
    vne_server_cfg k = *cfg;
    // (measured on a 24-graph pool at saturation under the eq. (4.10) rule:
    // 64, 128, 256, 512 tasks at once gave 512, 544, 592, 626 queries/s; 256
    // keeps the median latency of a saturated queue lower than 512 does)
    if (k.max_slots <= 0) k.max_slots = 256;
    if (k.max_cols <= 0) k.max_cols = 256;
    if (k.pilot_probes <= 0) k.pilot_probes = 16;
    if (k.max_probes <= 0) k.max_probes = 4096;
    if (k.max_steps <= 0) k.max_steps = 100;
    if (!(k.z > 0.0)) k.z = 2.576;
    if (k.max_group == 0) k.max_group = 2;
    if (k.stop != VNE_STOP_BOUND && k.stop != VNE_STOP_ESTIMATE)
        return fail(c, VNE_EINVAL, "stop must be VNE_STOP_BOUND or VNE_STOP_ESTIMATE");
    if (k.max_group != 1 && k.max_group != 2 && k.max_group != 4)
        return fail(c, VNE_EINVAL, "max_group must be 0, 1, 2 or 4");
    if (k.mode & ~(uint32_t)(VNE_MODE_F64 | VNE_MODE_DESING)) return fail(c, VNE_EINVAL, "unknown mode bits");
    if (k.max_steps > kMaxSteps || k.max_cols > 4096 || k.pilot_probes > k.max_probes)
        return fail(c, VNE_EINVAL, "bad server limits");
    HIP_TRY(c, hipSetDevice(c->device));
    auto s = std::make_unique<vne_server>();
    GpuExec &x = s->exec;
    x.ctx = c;
    x.fp64 = (k.mode & VNE_MODE_F64) != 0;
    x.desing = (k.mode & VNE_MODE_DESING) != 0;
    x.psi_cap = k.max_probes;
    x.stop_rule = k.stop;
    uint64_t bytes = k.arena_bytes;
    if (bytes == 0) {
        size_t fr = 0, tot = 0;
        HIP_TRY(c, hipMemGetInfo(&fr, &tot));
        bytes = fr / 4;
    }
    VNE_TRY(dev_alloc(c, &x.arena_mem, bytes));
    if (vne_status st0 = dev_alloc(c, &x.sink, 256); st0 != VNE_OK) {
        dev_free(c, &x.arena_mem);
        return st0;
    }
    auto undo = [&](vne_status st) {
        for (int r = 0; r < GpuExec::kRing; ++r)
            if (x.ring_ev[r]) (void)hipEventDestroy(x.ring_ev[r]);
        if (x.mailbox) (void)hipHostFree(x.mailbox);
        for (int j = 0; j < GpuExec::kSide; ++j) {
            if (x.side[j]) (void)hipStreamDestroy(x.side[j]);
            if (x.join_ev[j]) (void)hipEventDestroy(x.join_ev[j]);
        }
        if (x.fork_ev) (void)hipEventDestroy(x.fork_ev);
        if (x.stream) (void)hipStreamDestroy(x.stream);
        dev_free(c, &x.mail);
        dev_free(c, &x.sink);
        dev_free(c, &x.arena_mem);
        return st;
    };
    hipError_t e = hipStreamCreate(&x.stream);
    if (e != hipSuccess) return undo(hip_fail(c, e, "hipStreamCreate"));
    x.n_side = std::max(0, std::min(GpuExec::kSide, env_int("VNE_SERVE_STREAMS", 3) - 1));
    for (int j = 0; j < GpuExec::kSide; ++j) {
        e = hipStreamCreate(&x.side[j]);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&x.join_ev[j], hipEventDisableTiming);
        if (e != hipSuccess) return undo(hip_fail(c, e, "hipStreamCreate"));
    }
    e = hipEventCreateWithFlags(&x.fork_ev, hipEventDisableTiming);
    if (e != hipSuccess) return undo(hip_fail(c, e, "hipEventCreate"));
    for (int r = 0; r < GpuExec::kRing; ++r) {
        e = hipEventCreateWithFlags(&x.ring_ev[r], hipEventDisableTiming);
        if (e != hipSuccess) return undo(hip_fail(c, e, "hipEventCreate"));
    }
    e = hipHostMalloc((void **)&x.mailbox, sizeof(int2) * k.max_slots, hipHostMallocDefault);
    if (e != hipSuccess) return undo(hip_fail(c, e, "hipHostMalloc"));
    std::memset(x.mailbox, 0, sizeof(int2) * k.max_slots);
    x.max_slots = k.max_slots;
    if (vne_status st1 = dev_alloc(c, &x.mail, sizeof(int2) * k.max_slots); st1 != VNE_OK) return undo(st1);
    e = hipMemsetAsync(x.mail.p, 0, sizeof(int2) * k.max_slots, x.stream);
    if (e != hipSuccess) return undo(hip_fail(c, e, "hipMemsetAsync"));
    ServeConfig sc;
    sc.max_slots = k.max_slots;
    sc.max_cols = k.max_cols;
    sc.pilot_probes = k.pilot_probes;
    sc.psi_cap = k.max_probes;
    sc.max_steps = k.max_steps;
    sc.z = k.z;
    sc.fp64 = x.fp64;
    sc.arena_bytes = bytes;
    sc.query_bytes = rnd((size_t)x.psi_cap * 8) + 512;
    sc.skip_blocked = env_int("VNE_SERVE_SKIP_BLOCKED", 0) != 0;
    sc.max_group = k.max_group;
    s->core = std::make_unique<ServeCore>(sc, &s->exec);
    vne_server *raw = s.release();
    raw->worker = std::thread([raw] { raw->core->run(); });
    *out = raw;
    return VNE_OK;
}

extern "C" vne_status vne_server_submit(vne_server *s, const vne_query *q, uint64_t *ticket) {
    if (!s || !q || !ticket) return VNE_EINVAL;
    if (s->core->stopping()) return VNE_EBUSY;
    auto sq = std::make_unique<ServeQuery>();
    sq->q = *q;
    auto x = std::make_unique<GpuQuery>();
    {
        vne_ctx *c = s->exec.ctx;
        std::lock_guard<std::recursive_mutex> lock(c->mu);
        Graph *g = get_graph(c, q->graph_id);
        if (!g) return fail(c, VNE_EINVAL, "unknown graph id");
        if (!(q->rel_eps >= 0.0)) return fail(c, VNE_EINVAL, "rel_eps must be >= 0");
        if (q->rel_eps == 0.0) {
            if (q->m < 1 || q->m > s->exec.psi_cap) return fail(c, VNE_EINVAL, "m must be in [1, max_probes]");
            if (q->k_steps < 1 || q->k_steps > kMaxSteps) return fail(c, VNE_EINVAL, "k_steps must be in [1, 128]");
        }
        if (s->exec.desing && !g->zero_rowsum)
            return fail(c, VNE_EINVAL, "VNE_MODE_DESING needs a matrix whose rows sum to zero (A 1 = 0)");
        GraphSet *set = nullptr;
        VNE_TRY(get_set(c, {q->graph_id}, &set));
        x->g = g;
        x->set = set;
        sq->n = g->n;
        sq->lambda_ub = g->lambda_ub;
        sq->fro2 = g->fro2;
        sq->trace = g->trace;
        g->in_use++;
    }
    sq->x = x.get();
    const vne_status st = s->core->submit(std::move(sq), ticket);
    if (st != VNE_OK) {   // stop began meanwhile: the query was not taken
        std::lock_guard<std::recursive_mutex> lock(s->exec.ctx->mu);
        x->g->in_use--;
        return st;
    }
    x.release();          // the core's query owns it now
    return VNE_OK;
}

extern "C" vne_status vne_server_poll(vne_server *s, uint64_t ticket, int32_t timeout_ms, vne_query_result *res,
                                      double *quad, int32_t quad_cap) {
    if (!s || !res) return VNE_EINVAL;
    return s->core->poll(ticket, timeout_ms, res, quad, quad_cap);
}

extern "C" vne_status vne_server_stats(vne_server *s, vne_server_info *st) {
    if (!s || !st) return VNE_EINVAL;
    s->core->stats(st);
    return VNE_OK;
}

extern "C" vne_status vne_server_stop(vne_server *s) {
    if (!s) return VNE_EINVAL;
    s->core->request_stop();
    if (s->worker.joinable()) s->worker.join();
    GpuExec &x = s->exec;
    vne_ctx *c = x.ctx;
    (void)hipSetDevice(c->device);
    for (int j = 0; j < GpuExec::kSide; ++j) (void)hipStreamSynchronize(x.side[j]);
    (void)hipStreamSynchronize(x.stream);
    for (ServeQuery *q : s->core->unfinished()) {
        x.release_graph(*q);
        x.close_query(*q);
    }
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    for (double *p : x.pinned_pool) (void)hipHostFree(p);
    for (hipEvent_t e : x.event_pool) (void)hipEventDestroy(e);
    for (int r = 0; r < GpuExec::kRing; ++r) {
        if (x.stage[r]) (void)hipHostFree(x.stage[r]);
        if (x.ring_ev[r]) (void)hipEventDestroy(x.ring_ev[r]);
    }
    if (x.d_desc) (void)hipFree(x.d_desc);
    if (x.mailbox) (void)hipHostFree(x.mailbox);
    dev_free(c, &x.mail);
    dev_free(c, &x.sink);
    dev_free(c, &x.arena_mem);
    for (int j = 0; j < GpuExec::kSide; ++j) {
        (void)hipStreamDestroy(x.side[j]);
        (void)hipEventDestroy(x.join_ev[j]);
    }
    (void)hipEventDestroy(x.fork_ev);
    (void)hipStreamDestroy(x.stream);
    delete s;
    return VNE_OK;
}
