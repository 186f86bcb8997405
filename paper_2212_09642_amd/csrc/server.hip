// Serving loop: entropy queries on registered graphs, admitted by an HBM
// budget, run with continuous batching.
//
// A query is split into slot tasks of at most max_cols probe columns.  An
// admitted task gets a slot (two 16-column FP32 tasks of one graph that wait
// together may share a pair slot): its matrix stays the registered graph's,
// its vectors and Lanczos state live in the server's arena.  One tick
// advances every active slot by one Lanczos step in a few launches
// (normalize, SpMM + recurrence, long rows, finalize) whatever graphs the
// slots belong to; a task that reaches its step count gets its quadrature
// and leaves, and waiting tasks are admitted between ticks as mailbox
// entries and arena space free up.  A task's arithmetic depends only on its
// own graph, probes and step count (in a pair slot too), so a query gives
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
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ctx_internal.h"
#include "serve_host.h"

using namespace vne;
using namespace vne::rt;

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// One query's share of a slot: its columns, stopping rule and mailbox entry.
struct SrvMember {
    uint64_t ticket = 0;
    int m = 0;                       // probe columns
    int col0 = 0;                    // first column of the query's probe set
    int c_off = 0;                   // first column within the slot
    bool pilot = false;
    bool adaptive = false;           // a-posteriori stopping (rel_eps > 0)
    double tol = 0.0;                // per quadratic form
    int32_t uid = 0, slot = -1;      // stop record id, mailbox entry while running
    bool ended = false;
};

// A slot: one task of a query, or two 16-column FP32 tasks of two queries on
// the same graph with the same step cap (pair slot, m_pad = 32, mt = 16),
// whose two column tiles share one workgroup per work block.  Members keep
// their own probes, stop records and results; every column gets the
// arithmetic it gets alone.
struct SrvTask {
    int m = 0, m_pad = 0, mt = 0, k = 0;
    int j = 0;                       // steps done
    uint64_t off = 0, bytes = 0;
    char *P[2] = {nullptr, nullptr}, *V[2] = {nullptr, nullptr};
    double *alpha = nullptr, *beta = nullptr, *st_alpha = nullptr, *st_inv = nullptr, *st_coup = nullptr;
    double *norm2 = nullptr, *mean = nullptr, *partials = nullptr, *probe_part = nullptr;
    double *seg_acc = nullptr, *long_part = nullptr, *level2 = nullptr;
    int32_t *k_eff = nullptr;
    double *b_lo = nullptr, *b_hi = nullptr;
    int2 *d_state = nullptr;         // [n_mem] {uid, first step within tol}
    int n_mem = 1;
    SrvMember mem[2];
    bool pair() const { return n_mem == 2; }
};

struct SrvQuery {
    uint64_t ticket = 0;
    vne_query q{};
    Graph *g = nullptr;
    GraphSet *set = nullptr;
    int N = 0, k = 0;                // planned probes and steps
    int cols_issued = 0, tasks_open = 0;
    bool planned = false, started = false;
    bool stage_wait = false, final_wait = false, done = false;
    double s_lower = 0.0, bound = 0.0;
    int steps_used = 0;              // largest step count a task of the query used
    int rounds = 0;                  // probe-count plans made (rel_eps > 0)
    uint64_t off = 0;                // arena block: psi [cap], estimate, flags
    double *d_psi = nullptr, *d_est = nullptr;
    int32_t *d_flags = nullptr;
    double *h_buf = nullptr;         // pinned: psi [cap], estimate, flags
    hipEvent_t ev = nullptr;
    Clock::time_point t_submit, t_admit, t_done;
    vne_query_result res{};
    std::vector<double> quad;
};

}  // namespace

struct vne_server {
    vne_ctx *ctx = nullptr;
    vne_server_cfg cfg{};
    bool fp64 = false, desing = false;
    hipStream_t stream = nullptr;
    DevBuf arena_mem;
    Arena arena;
    uint64_t arena_peak = 0;
    int psi_cap = 0;
    size_t query_bytes = 0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stopping = false, broken = false;
    std::string broken_msg;
    uint64_t next_ticket = 1;
    std::deque<uint64_t> incoming;                  // submitted, not yet split into tasks
    std::map<uint64_t, std::unique_ptr<SrvQuery>> queries;

    // worker-owned state
    std::deque<SrvTask> pending;                     // in ticket order
    std::vector<SrvTask> active;
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
    int2 *mailbox = nullptr;                         // pinned [max_slots]: stop records
    std::vector<int> free_slots;
    int32_t next_uid = 1;

    // statistics (worker-owned; snap is the copy readers see)
    int64_t ticks = 0, tasks_admitted = 0, queries_done = 0, pair_slots = 0;
    double occupancy_sum = 0.0;
    vne_server_info snap{};
};

namespace {

vne_status srv_hip(vne_server *s, hipError_t e, const char *what) {
    if (e == hipSuccess) return VNE_OK;
    std::lock_guard<std::mutex> lk(s->mu);
    s->broken = true;
    s->broken_msg = std::string(what) + ": " + hipGetErrorString(e);
    return VNE_EDEVICE;
}

#define SRV_HIP(s, expr)                                               \
    do {                                                               \
        hipError_t _e = (expr);                                        \
        if (_e != hipSuccess) return srv_hip((s), _e, #expr);          \
    } while (0)

size_t rnd(size_t b) { return (b + 255) / 256 * 256; }

constexpr int kPlanRounds = 4;   // probe-count plans of a rel_eps query (pilot included)

// Arena bytes of a task of width m_pad and k steps on a graph.
size_t task_bytes(const GraphSet *set, int m_pad, int k, bool fp64) {
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

void carve(SrvTask &t, char *base, const GraphSet *set, bool fp64) {
    const size_t es = fp64 ? 8 : 4;
    const Schedule &sc = set->sched;
    char *p = base;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += rnd(bytes);
        return r;
    };
    const size_t blk = (size_t)set->n * t.m_pad * es;
    t.P[0] = take(blk);
    t.P[1] = take(blk);
    t.V[0] = take(blk);
    t.V[1] = take(blk);
    t.alpha = (double *)take((size_t)t.m_pad * t.k * 8);
    t.beta = (double *)take((size_t)t.m_pad * t.k * 8);
    t.st_alpha = (double *)take((size_t)t.m_pad * 8);
    t.st_inv = (double *)take((size_t)t.m_pad * 8);
    t.st_coup = (double *)take((size_t)t.m_pad * 8);
    t.norm2 = (double *)take((size_t)t.m_pad * 8);
    t.mean = (double *)take((size_t)t.m_pad * 8);
    t.k_eff = (int32_t *)take((size_t)t.m_pad * 4);
    t.partials = (double *)take((size_t)sc.n_blocks() * 3 * t.m_pad * 8);
    t.probe_part = (double *)take((size_t)set->probe_blocks * t.m_pad * 8);
    t.seg_acc = (double *)take((size_t)std::max(1, sc.n_seg) * t.m_pad * 8);
    t.long_part = (double *)take((size_t)std::max(1, sc.n_long) * 3 * t.m_pad * 8);
    t.level2 = (double *)take((size_t)kSlotLevel2 * 3 * t.m_pad * 8);
    t.b_lo = (double *)take((size_t)t.m_pad * 8);
    t.b_hi = (double *)take((size_t)t.m_pad * 8);
    t.d_state = (int2 *)take(256);
}

// Tasks for columns [c0, c1) of a query, in the pending queue after every
// task of an earlier ticket.  Widths: max_cols while that much is left, then
// the largest power of two (at least 16) that fits, then the rest, so that a
// task's width is a whole number of column tiles wherever possible.
void add_tasks(vne_server *s, SrvQuery &q, int c0, int c1, bool pilot) {
    std::vector<SrvTask> ts;
    for (int c = c0; c < c1;) {
        const int rem = c1 - c;
        int w = rem;
        if (rem >= s->cfg.max_cols) {
            w = s->cfg.max_cols;
        } else if (rem >= 16) {
            w = 16;
            while (2 * w <= rem) w *= 2;
        }
        SrvTask t;
        t.m = w;
        t.mt = choose_tile(t.m, s->fp64, 0);
        t.m_pad = pad_columns(t.m, t.mt);
        t.k = q.k;
        SrvMember &u = t.mem[0];
        u.ticket = q.ticket;
        u.m = w;
        u.col0 = c;
        u.pilot = pilot;
        u.adaptive = q.q.rel_eps > 0.0 && q.s_lower > 0.0;
        u.tol = 0.5 * q.q.rel_eps * q.s_lower;
        t.bytes = task_bytes(q.set, t.m_pad, t.k, s->fp64);
        ts.push_back(t);
        c += w;
    }
    q.cols_issued = c1;
    q.tasks_open += (int)ts.size();
    auto pos = s->pending.begin();
    while (pos != s->pending.end() && pos->mem[0].ticket <= q.ticket) ++pos;
    s->pending.insert(pos, ts.begin(), ts.end());
}

double *get_pinned(vne_server *s) {
    if (!s->pinned_pool.empty()) {
        double *p = s->pinned_pool.back();
        s->pinned_pool.pop_back();
        return p;
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, (size_t)(s->psi_cap + 2) * 8, hipHostMallocDefault) != hipSuccess) return nullptr;
    return (double *)p;
}

hipEvent_t get_event(vne_server *s) {
    if (!s->event_pool.empty()) {
        hipEvent_t e = s->event_pool.back();
        s->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

// Completion bookkeeping of a query whose result has reached the host.
void finish_query(vne_server *s, SrvQuery &q, vne_status st, const std::string &msg) {
    q.t_done = Clock::now();
    if (q.h_buf && st == VNE_OK) {
        q.quad.assign(q.h_buf, q.h_buf + q.N);
        q.res.estimate = q.h_buf[q.N];
        double mean = 0.0;
        for (double v : q.quad) mean += v;
        mean /= std::max(1, q.N);
        double var = 0.0;
        for (double v : q.quad) var += (v - mean) * (v - mean);
        q.res.std_error = q.N > 1 ? std::sqrt(var / (q.N - 1) / q.N) : 0.0;
    }
    q.res.status = st;
    std::snprintf(q.res.message, sizeof(q.res.message), "%s", msg.c_str());
    q.res.probes = q.N;
    q.res.steps = q.steps_used > 0 ? q.steps_used : q.k;
    q.res.quad_bound = q.bound;
    q.res.queue_ms = q.started ? ms_between(q.t_submit, q.t_admit) : 0.0;
    q.res.latency_ms = ms_between(q.t_submit, q.t_done);
    if (q.h_buf) s->pinned_pool.push_back(q.h_buf);
    q.h_buf = nullptr;
    if (q.ev) s->event_pool.push_back(q.ev);
    q.ev = nullptr;
    if (q.started) s->arena.release(q.off);
    q.started = false;
    {
        std::lock_guard<std::recursive_mutex> lk(s->ctx->mu);
        q.g->in_use--;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    q.done = true;
    s->queries_done++;
    s->cv_done.notify_all();
}

// Drops the pending tasks of a query and reports the failure.
void fail_query(vne_server *s, SrvQuery &q, vne_status st, const std::string &msg) {
    s->pending.erase(std::remove_if(s->pending.begin(), s->pending.end(),
                                    [&](const SrvTask &t) { return t.mem[0].ticket == q.ticket; }),
                     s->pending.end());
    q.stage_wait = q.final_wait = false;
    finish_query(s, q, st, msg);
}

SrvQuery *query_of(vne_server *s, uint64_t ticket) {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->queries.find(ticket);
    return it == s->queries.end() ? nullptr : it->second.get();
}

// After the last task of a query: estimator combine (eq. (3.8)) on the
// device and the copy of psi, estimate and flags to the host.
vne_status issue_final(vne_server *s, SrvQuery &q) {
    SRV_HIP(s, launch_combine(q.d_psi, q.N, 0, 0, q.d_est, s->stream));
    SRV_HIP(s, hipMemcpyAsync(q.h_buf, q.d_psi, (size_t)q.N * 8, hipMemcpyDeviceToHost, s->stream));
    SRV_HIP(s, hipMemcpyAsync(q.h_buf + q.N, q.d_est, 8, hipMemcpyDeviceToHost, s->stream));
    SRV_HIP(s, hipMemcpyAsync(q.h_buf + q.N + 1, q.d_flags, 4, hipMemcpyDeviceToHost, s->stream));
    SRV_HIP(s, hipEventRecord(q.ev, s->stream));
    q.final_wait = true;
    return VNE_OK;
}

std::string flag_text(int32_t fl) {
    if (fl & 1) return "non-finite Lanczos coefficient";
    if (fl & 4) return "tridiagonal QR did not converge";
    if (fl & 8) return "tridiagonal QR rotation record overflowed";
    return "numerical failure";
}

// Pilot or final results that have reached the host.
vne_status poll_events(vne_server *s, bool block_one) {
    std::vector<SrvQuery *> waiting;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto &kv : s->queries)
            if (kv.second->stage_wait || kv.second->final_wait) waiting.push_back(kv.second.get());
    }
    bool blocked = false;
    for (SrvQuery *q : waiting) {
        hipError_t e = hipEventQuery(q->ev);
        if (e == hipErrorNotReady && block_one && !blocked) {
            blocked = true;
            e = hipEventSynchronize(q->ev);
        }
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return srv_hip(s, e, "hipEventQuery");
        int32_t fl = 0;
        if (q->stage_wait) {
            q->stage_wait = false;
            const int n0 = q->cols_issued;
            std::memcpy(&fl, q->h_buf + s->psi_cap + 1, 4);
            if (fl) {
                fail_query(s, *q, VNE_ENUMERIC, flag_text(fl));
                continue;
            }
            double mean = 0.0, var = 0.0;
            for (int i = 0; i < n0; ++i) mean += q->h_buf[i];
            mean /= n0;
            for (int i = 0; i < n0; ++i) var += (q->h_buf[i] - mean) * (q->h_buf[i] - mean);
            const double sd = n0 > 1 ? std::sqrt(var / (n0 - 1)) : 0.0;
            // the rule's N from every form so far (sequential sampling: the
            // count is planned again after each stage), rounded up to whole
            // 16-column groups: the extra columns would be computed as
            // padding anyway, and more probes only tighten the estimate
            int nn = plan_probes(mean, sd, q->q.rel_eps, 0.5, s->cfg.z, n0, s->psi_cap);
            if (nn > n0) nn = std::min(s->psi_cap, n0 + (nn - n0 + 15) / 16 * 16);
            q->rounds++;
            q->planned = true;
            q->N = nn;
            if (nn > n0) add_tasks(s, *q, n0, nn, false);
            else VNE_TRY(issue_final(s, *q));
        } else {
            q->final_wait = false;
            std::memcpy(&fl, q->h_buf + q->N + 1, 4);
            if (fl) finish_query(s, *q, VNE_ENUMERIC, flag_text(fl));
            else finish_query(s, *q, VNE_OK, "");
        }
    }
    return VNE_OK;
}

// The query's own arena block (psi, estimate, flags), pinned buffer and
// event, taken when its first task is admitted.  false: no room.
bool open_query(vne_server *s, SrvQuery *q, vne_status *st) {
    *st = VNE_OK;
    if (!s->arena.alloc(s->query_bytes, &q->off)) return false;
    char *qb = (char *)s->arena_mem.p + q->off;
    q->d_psi = (double *)qb;
    q->d_est = (double *)(qb + rnd((size_t)s->psi_cap * 8));
    q->d_flags = (int32_t *)(qb + rnd((size_t)s->psi_cap * 8) + 256);
    q->h_buf = get_pinned(s);
    q->ev = get_event(s);
    q->started = true;
    q->t_admit = Clock::now();
    if (!q->h_buf || !q->ev) {
        *st = srv_hip(s, hipErrorOutOfMemory, "pinned buffer or event");
        return true;
    }
    const hipError_t e = hipMemsetAsync(q->d_flags, 0, 4, s->stream);
    if (e != hipSuccess) *st = srv_hip(s, e, "hipMemsetAsync");
    return true;
}

// A task that can share a pair slot: 16 FP32 columns in one 16-column tile.
bool pairable(const vne_server *s, const SrvTask &t) {
    return !s->fp64 && t.n_mem == 1 && t.m == 16 && t.m_pad == 16 && t.mt == 16;
}

constexpr int kPairWindow = 256;   // pending tasks searched for a partner

// Probe block of member i (the query's hash columns col0.., eq. (3.8)) into
// its columns of the slot.
vne_status member_probes(vne_server *s, SrvTask &t, int i, const SrvQuery *q) {
    const SrvMember &u = t.mem[i];
    const GraphSet *set = q->set;
    const size_t es = s->fp64 ? 8 : 4;
    ProbeArgs pa{};
    pa.gen = GEN_RADEMACHER;
    pa.n = (int32_t)set->n;
    pa.m = u.m;
    pa.m_pad = t.pair() ? t.mt : t.m_pad;
    pa.mt = t.mt;
    pa.ld_out = t.m_pad;
    pa.col_offset = u.col0;
    pa.seed = q->q.seed;
    pa.keys = (const int64_t *)set->keys.p;
    pa.desing = s->desing ? 1 : 0;
    pa.P_out = t.P[0] + (size_t)u.c_off * es;
    pa.partials = t.probe_part;
    pa.n_blocks = set->probe_blocks;
    pa.mean = t.mean + u.c_off;
    pa.norm2 = t.norm2 + u.c_off;
    pa.st_alpha = t.st_alpha + u.c_off;
    pa.st_inv = t.st_inv + u.c_off;
    pa.st_coup = t.st_coup + u.c_off;
    pa.k_eff = t.k_eff + u.c_off;
    pa.k = t.k;
    pa.block_row_begin = (const int32_t *)set->probe_rows.p;
    pa.block_graph = (const int32_t *)set->probe_block_graph.p;
    pa.graph_block_begin = (const int32_t *)set->probe_graph_begin.p;
    pa.graph_row_begin = (const int64_t *)set->graph_row_begin.p;
    pa.n_graphs = 1;
    SRV_HIP(s, launch_probe(pa, s->fp64, s->stream));
    return VNE_OK;
}

// Starts waiting tasks while mailbox entries and arena space allow (first
// come, first served: a task that does not fit blocks the ones behind it).
// A 16-column FP32 task takes the first waiting 16-column task of the same
// graph with the same step cap and stopping mode as its partner in a pair
// slot, when the arena has room for it.
vne_status admit(vne_server *s) {
    while (!s->pending.empty() && !s->free_slots.empty()) {
        SrvTask t = s->pending.front();
        SrvQuery *q = query_of(s, t.mem[0].ticket);
        const size_t need = t.bytes + (q->started ? 0 : s->query_bytes);
        if (need > s->arena.size()) {
            fail_query(s, *q, VNE_ENOMEM,
                       "query needs " + std::to_string(need) + " bytes of slot state, the arena holds " +
                           std::to_string(s->arena.size()));
            continue;
        }
        // partner search
        int partner = -1;
        SrvQuery *pq = nullptr;
        size_t pair_bytes = 0;
        if (pairable(s, t) && s->free_slots.size() >= 2) {
            const int lim = std::min<int>((int)s->pending.size(), kPairWindow);
            for (int i = 1; i < lim; ++i) {
                const SrvTask &c = s->pending[i];
                if (!pairable(s, c) || c.k != t.k || c.mem[0].adaptive != t.mem[0].adaptive) continue;
                SrvQuery *cq = query_of(s, c.mem[0].ticket);
                if (!cq || cq->set != q->set) continue;
                partner = i;
                pq = cq;
                break;
            }
            if (partner > 0) {
                pair_bytes = task_bytes(q->set, 32, t.k, s->fp64);
                size_t room = s->arena.round(pair_bytes);
                if (!q->started) room += s->query_bytes;
                if (pq != q && !pq->started) room += s->query_bytes;
                if (s->arena.largest_free() < room) partner = -1;
            }
        }
        if (!q->started) {
            if (s->arena.largest_free() < s->query_bytes + s->arena.round(t.bytes)) break;
            vne_status st;
            if (!open_query(s, q, &st)) break;
            VNE_TRY(st);
        }
        if (partner > 0 && !pq->started) {
            vne_status st;
            if (!open_query(s, pq, &st)) partner = -1;
            VNE_TRY(st);
        }
        if (partner > 0) {
            t.mem[1] = s->pending[partner].mem[0];
            t.mem[1].c_off = 16;
            t.n_mem = 2;
            t.m = 32;
            t.m_pad = 32;
            t.bytes = pair_bytes;
        }
        if (!s->arena.alloc(t.bytes, &t.off)) {
            if (partner < 0) break;
            // no room for the pair after all: the task alone
            partner = -1;
            t.n_mem = 1;
            t.m = t.m_pad = 16;
            t.bytes = task_bytes(q->set, 16, t.k, s->fp64);
            if (!s->arena.alloc(t.bytes, &t.off)) break;
        }
        s->arena_peak = std::max(s->arena_peak, s->arena.in_use());
        if (partner > 0) s->pending.erase(s->pending.begin() + partner);
        s->pending.pop_front();
        carve(t, (char *)s->arena_mem.p + t.off, q->set, s->fp64);
        for (int i = 0; i < t.n_mem; ++i) {
            t.mem[i].uid = s->next_uid + i;
            t.mem[i].slot = s->free_slots.back();
            s->free_slots.pop_back();
        }
        s->next_uid += t.n_mem;
        SRV_HIP(s, hipMemsetAsync(t.d_state, 0, sizeof(int2) * t.n_mem, s->stream));
        VNE_TRY(member_probes(s, t, 0, q));
        if (t.pair()) VNE_TRY(member_probes(s, t, 1, pq));
        // zero v_0
        SRV_HIP(s, hipMemsetAsync(t.V[1], 0, (size_t)q->set->n * t.m_pad * (s->fp64 ? 8 : 4), s->stream));
        s->active.push_back(t);
        s->tasks_admitted += t.n_mem;
        s->pair_slots += t.pair() ? 1 : 0;
    }
    return VNE_OK;
}

bool all_adaptive(const SrvTask &t) {
    for (int i = 0; i < t.n_mem; ++i)
        if (!t.mem[i].adaptive) return false;
    return true;
}

StepArgs step_args(const vne_server *s, const SrvTask &t, const GraphSet *set) {
    StepArgs a{};
    const int j = t.j + 1;
    a.row_ptr = set->d_row_ptr;
    a.col = set->d_col;
    a.val = s->fp64 ? set->val64.p : set->val32.p;
    a.scale = set->scale;
    a.n = (int32_t)set->n;
    a.m_pad = t.m_pad;
    a.mt = t.mt;
    a.n_tiles = t.m_pad / t.mt;
    a.P_in = t.P[(j - 1) & 1];
    a.P_out = t.P[j & 1];
    a.V_out = t.V[(j - 1) & 1];
    a.V_prev = t.V[j & 1];
    a.V_cur = a.V_out;
    a.two_pass = 1;
    a.st_alpha = t.st_alpha;
    a.st_inv = t.st_inv;
    a.st_coup = t.st_coup;
    a.segs = (const SegItem *)set->segs.p;
    a.n_seg = set->sched.n_seg;
    a.seg_len = set->sched.seg_len;
    a.block_ranges = (const int4 *)set->block_ranges.p;
    a.n_blocks = set->sched.n_blocks();
    a.seg_acc = t.seg_acc;
    a.n_long = set->sched.n_long;
    a.long_first = (const int32_t *)set->long_first.p;
    a.long_nseg = (const int32_t *)set->long_nseg.p;
    a.long_part = t.long_part;
    a.partials = t.partials;
    a.stop_state = all_adaptive(t) ? t.d_state : nullptr;
    a.stop_uid = t.mem[0].uid;
    a.stop_count = t.n_mem;
    return a;
}

FinalizeArgs fin_args(const vne_server *s, const SrvTask &t, const GraphSet *set, int32_t *flags,
                      int32_t *flags_hi) {
    FinalizeArgs f{};
    f.partials = t.partials;
    f.long_part = t.long_part;
    f.level2 = t.level2;
    f.n_level2 = kSlotLevel2;
    f.n_blocks = set->sched.n_blocks();
    f.n_long = set->sched.n_long;
    f.mt = t.mt;
    f.m_pad = t.m_pad;
    f.m = t.m;
    f.step = t.j + 1;
    f.k = t.k;
    f.tau = s->fp64 ? std::ldexp(1.0, -23) : std::ldexp(1.0, -18);
    f.st_alpha = t.st_alpha;
    f.st_inv = t.st_inv;
    f.st_coup = t.st_coup;
    f.alpha = t.alpha;
    f.beta = t.beta;
    f.k_eff = t.k_eff;
    f.flags = flags;
    f.n_graphs = 1;
    f.stop_state = all_adaptive(t) ? t.d_state : nullptr;
    f.stop_uid = t.mem[0].uid;
    f.stop_count = t.n_mem;
    f.flags_hi = t.pair() ? flags_hi : nullptr;
    f.flag_split = t.pair() ? t.mem[1].c_off : t.m_pad;
    return f;
}

// Quadrature of member i of a slot after `steps` steps, its mailbox entry
// back, and the query's next stage when it was the query's last task.  The
// slot's memory goes back when its last member has ended.
vne_status end_member(vne_server *s, SrvTask &t, int i, SrvQuery &q, int steps) {
    SrvMember &u = t.mem[i];
    // an adaptive task's own stop record (if the device made one) decides the
    // step count, whenever the host noticed it
    const int64_t co = u.c_off;
    SRV_HIP(s, launch_quadrature(t.alpha + co * t.k, t.beta + co * t.k, t.k_eff + co, t.norm2 + co, t.k, steps, u.m,
                                 q.d_psi + u.col0, q.d_flags, s->stream, s->fp64,
                                 u.adaptive ? t.d_state + i : nullptr, u.uid));
    u.ended = true;
    s->free_slots.push_back(u.slot);
    q.steps_used = std::max(q.steps_used, steps);
    q.tasks_open--;
    if (q.tasks_open > 0) return VNE_OK;
    if (q.q.rel_eps > 0.0 && q.rounds < kPlanRounds && q.cols_issued < s->psi_cap) {
        // a stage of a rel_eps query done: its forms and the flags to the
        // host, which plans the probe count again from all forms so far
        SRV_HIP(s, hipMemcpyAsync(q.h_buf, q.d_psi, (size_t)q.cols_issued * 8, hipMemcpyDeviceToHost, s->stream));
        SRV_HIP(s, hipMemcpyAsync(q.h_buf + s->psi_cap + 1, q.d_flags, 4, hipMemcpyDeviceToHost, s->stream));
        SRV_HIP(s, hipEventRecord(q.ev, s->stream));
        q.stage_wait = true;
    } else {
        q.N = q.cols_issued;
        VNE_TRY(issue_final(s, q));
    }
    return VNE_OK;
}

// One Lanczos step of every active slot.
vne_status tick(vne_server *s) {
    const int A = (int)s->active.size();
    // queries of the members of each slot
    std::vector<SrvQuery *> qs(2 * A, nullptr);
    for (int i = 0; i < A; ++i)
        for (int mi = 0; mi < s->active[i].n_mem; ++mi) qs[2 * i + mi] = query_of(s, s->active[i].mem[mi].ticket);
    // descriptors: StepArgs[A], FinalizeArgs[A], then per tile width the step
    // and long-row maps (and those of the pair slots), then the finalize map
    std::vector<StepArgs> sa(A);
    std::vector<FinalizeArgs> fa(A);
    std::map<int, std::vector<int4>> smap, lmap;
    std::vector<int4> pmap, plmap;
    std::vector<int2> fmap;
    int running = 0;
    for (int i = 0; i < A; ++i) {
        const SrvTask &t = s->active[i];
        const GraphSet *set = qs[2 * i]->set;
        sa[i] = step_args(s, t, set);
        fa[i] = fin_args(s, t, set, qs[2 * i]->d_flags, t.pair() ? qs[2 * i + 1]->d_flags : nullptr);
        for (int mi = 0; mi < t.n_mem; ++mi) running += t.mem[mi].ended ? 0 : 1;
        const int nt = t.m_pad / t.mt, nb = set->sched.n_blocks();
        if (t.pair()) {
            for (int b = 0; b < nb; ++b) pmap.push_back(make_int4(i, b, 0, 0));
        } else {
            auto &sm = smap[t.mt];
            for (int tile = 0; tile < nt; ++tile)
                for (int b = 0; b < nb; ++b) sm.push_back(make_int4(i, b, tile, 0));
        }
        if (set->sched.n_long > 0) {
            const int per = long_rows_per_group(t.mt, s->fp64);
            auto &lm = t.pair() ? plmap : lmap[t.mt];
            for (int tile = 0; tile < nt; ++tile)
                for (int gi = 0; gi < (set->sched.n_long + per - 1) / per; ++gi) lm.push_back(make_int4(i, gi, tile, 0));
        }
        for (int ch = 0; ch < (t.m_pad + kFinalizeCols - 1) / kFinalizeCols; ++ch) fmap.push_back(make_int2(i, ch));
    }
    // a-posteriori checks (Theorem 4.8) of adaptive members after this step:
    // from step 3 on, every other step
    std::vector<BoundArgs> ba;
    std::vector<StopArgs> sta;
    std::vector<int2> bmap;
    std::vector<int2> checked;       // {slot, member}
    for (int i = 0; i < A; ++i) {
        const SrvTask &t = s->active[i];
        const int j = t.j + 1;
        if (j < 3 || j % 2 == 0 || j >= t.k) continue;
        for (int mi = 0; mi < t.n_mem; ++mi) {
            const SrvMember &u = t.mem[mi];
            if (!u.adaptive || u.ended) continue;
            const SrvQuery *q = qs[2 * i + mi];
            const Graph *g = q->g;
            const int64_t co = u.c_off;
            BoundArgs b{};
            b.alpha = t.alpha + co * t.k;
            b.beta = t.beta + co * t.k;
            b.k_eff = t.k_eff + co;
            b.norm2 = t.norm2 + co;
            b.k = t.k;
            b.m = u.m;
            b.steps = j;
            b.lam_hi = g->lambda_ub;
            b.lam_lo = g->lambda_ub * kLamLoFraction;
            b.n_grid = kBoundGrid;
            b.lo = t.b_lo + co;
            b.hi = t.b_hi + co;
            b.flags = q->d_flags;
            b.stop_state = t.d_state + mi;
            b.stop_uid = u.uid;
            b.stop_count = 1;
            for (int grp = 0; grp < (u.m + 3) / 4; ++grp) bmap.push_back(make_int2((int)ba.size(), grp));
            ba.push_back(b);
            StopArgs sc{};
            sc.hi = t.b_hi + co;
            sc.m = u.m;
            sc.tol = u.tol;
            sc.step = j;
            sc.uid = u.uid;
            sc.state = t.d_state + mi;
            sta.push_back(sc);
            checked.push_back(make_int2(i, mi));
        }
    }
    size_t bytes = rnd(sizeof(StepArgs) * A) + rnd(sizeof(FinalizeArgs) * A) + rnd(sizeof(int2) * fmap.size());
    bytes += rnd(sizeof(BoundArgs) * ba.size()) + rnd(sizeof(int2) * bmap.size()) + rnd(sizeof(StopArgs) * sta.size());
    for (auto &kv : smap) bytes += rnd(sizeof(int4) * kv.second.size());
    for (auto &kv : lmap) bytes += rnd(sizeof(int4) * kv.second.size());
    bytes += rnd(sizeof(int4) * pmap.size()) + rnd(sizeof(int4) * plmap.size());
    // staging ring: wait until the copy that last used this slot has run
    const int r = s->ring_pos;
    s->ring_pos = (r + 1) % vne_server::kRing;
    if (s->ring_used[r]) SRV_HIP(s, hipEventSynchronize(s->ring_ev[r]));
    if (s->stage_cap[r] < bytes) {
        if (s->stage[r]) SRV_HIP(s, hipHostFree(s->stage[r]));
        s->stage[r] = nullptr;
        const size_t cap = std::max(bytes, 2 * s->stage_cap[r]);
        SRV_HIP(s, hipHostMalloc((void **)&s->stage[r], cap, hipHostMallocDefault));
        s->stage_cap[r] = cap;
    }
    if (s->d_desc_cap < bytes) {
        // kernels of earlier ticks may still read the old buffer
        SRV_HIP(s, hipStreamSynchronize(s->stream));
        if (s->d_desc) SRV_HIP(s, hipFree(s->d_desc));
        s->d_desc = nullptr;
        const size_t cap = std::max(bytes, 2 * s->d_desc_cap);
        SRV_HIP(s, hipMalloc((void **)&s->d_desc, cap));
        s->d_desc_cap = cap;
    }
    char *h = s->stage[r];
    size_t off = 0;
    auto put = [&](const void *src, size_t n) {
        std::memcpy(h + off, src, n);
        const size_t o = off;
        off += rnd(n);
        return s->d_desc + o;
    };
    const StepArgs *d_sa = (const StepArgs *)put(sa.data(), sizeof(StepArgs) * A);
    const FinalizeArgs *d_fa = (const FinalizeArgs *)put(fa.data(), sizeof(FinalizeArgs) * A);
    const int2 *d_fm = (const int2 *)put(fmap.data(), sizeof(int2) * fmap.size());
    std::map<int, const int4 *> d_sm, d_lm;
    for (auto &kv : smap) d_sm[kv.first] = (const int4 *)put(kv.second.data(), sizeof(int4) * kv.second.size());
    for (auto &kv : lmap) d_lm[kv.first] = (const int4 *)put(kv.second.data(), sizeof(int4) * kv.second.size());
    const int4 *d_pm = (const int4 *)put(pmap.data(), sizeof(int4) * pmap.size());
    const int4 *d_plm = (const int4 *)put(plmap.data(), sizeof(int4) * plmap.size());
    const BoundArgs *d_ba = (const BoundArgs *)put(ba.data(), sizeof(BoundArgs) * ba.size());
    const int2 *d_bm = (const int2 *)put(bmap.data(), sizeof(int2) * bmap.size());
    const StopArgs *d_st = (const StopArgs *)put(sta.data(), sizeof(StopArgs) * sta.size());
    SRV_HIP(s, hipMemcpyAsync(s->d_desc, h, off, hipMemcpyHostToDevice, s->stream));
    SRV_HIP(s, hipEventRecord(s->ring_ev[r], s->stream));
    s->ring_used[r] = true;
    for (auto &kv : smap) {
        const int mt = kv.first;
        const auto lit = lmap.find(mt);
        const int n_long = lit == lmap.end() ? 0 : (int)lit->second.size();
        SRV_HIP(s, launch_step_slots(d_sa, d_sm[mt], (int32_t)kv.second.size(), n_long ? d_lm[mt] : nullptr, n_long,
                                     mt, s->fp64, s->stream));
    }
    if (!pmap.empty())
        SRV_HIP(s, launch_step_pairs(d_sa, d_pm, (int32_t)pmap.size(), plmap.empty() ? nullptr : d_plm,
                                     (int32_t)plmap.size(), s->stream));
    SRV_HIP(s, launch_finalize_slots(d_fa, d_fm, (int32_t)fmap.size(), s->stream));
    if (!sta.empty()) {
        SRV_HIP(s, launch_error_bound(d_ba, d_bm, (int32_t)bmap.size(), s->stream));
        SRV_HIP(s, launch_stop_check(d_st, (int32_t)sta.size(), s->stream));
        for (const int2 &c : checked) {
            const SrvTask &t = s->active[c.x];
            SRV_HIP(s, hipMemcpyAsync(s->mailbox + t.mem[c.y].slot, t.d_state + c.y, sizeof(int2),
                                      hipMemcpyDeviceToHost, s->stream));
        }
    }
    s->ticks++;
    s->occupancy_sum += running;
    // members at the step cap, and adaptive members whose recorded stop step
    // has reached the host, end: quadrature (eq. (4.2)) into the query's psi
    std::vector<SrvTask> keep;
    for (int i = 0; i < A; ++i) {
        SrvTask &t = s->active[i];
        t.j++;
        bool open = false;
        for (int mi = 0; mi < t.n_mem; ++mi) {
            SrvMember &u = t.mem[mi];
            if (u.ended) continue;
            int use = t.j >= t.k ? t.k : 0;
            if (!use && u.adaptive) {
                const volatile int2 *mb = s->mailbox + u.slot;
                const int id = mb->x, st = mb->y;
                if (id == u.uid && st > 0) use = st;
            }
            if (!use) {
                open = true;
                continue;
            }
            VNE_TRY(end_member(s, t, mi, *qs[2 * i + mi], use));
        }
        if (open) keep.push_back(t);
        else s->arena.release(t.off);
    }
    s->active.swap(keep);
    return VNE_OK;
}

bool has_waits(vne_server *s) {
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto &kv : s->queries)
        if (kv.second->stage_wait || kv.second->final_wait) return true;
    return false;
}

// Turns a submitted query into tasks (explicit probe count, or the pilot).
void start_query(vne_server *s, SrvQuery &q) {
    if (q.q.rel_eps > 0.0) {
        // Proposition 4.4 with Remark 2.3: ||c||^2 <= n for +-1 probes;
        // S(A) >= -log tr(A^2) for a unit-trace PSD matrix
        const Graph *g = q.g;
        const bool density = std::fabs(g->trace - 1.0) < 1e-9 && g->fro2 > 0.0 && g->fro2 < 1.0;
        q.s_lower = density ? -std::log(g->fro2) : 0.0;
        q.k = density ? plan_steps((double)g->n, g->lambda_ub, q.s_lower, q.q.rel_eps, 0.5, s->cfg.max_steps)
                      : s->cfg.max_steps;
        // per-form target: the a-priori bound at k meets it, and adaptive
        // tasks stop once the a-posteriori bound does
        q.bound = density ? 0.5 * q.q.rel_eps * q.s_lower : 0.0;
        q.N = std::min(s->cfg.pilot_probes, s->psi_cap);
        add_tasks(s, q, 0, q.N, true);
    } else {
        q.k = q.q.k_steps;
        q.N = q.q.m;
        q.planned = true;
        add_tasks(s, q, 0, q.N, false);
    }
}

// Snapshot of the worker-owned counters for vne_server_stats.
void publish(vne_server *s) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->snap.ticks = s->ticks;
    s->snap.tasks = s->tasks_admitted;
    s->snap.pair_slots = s->pair_slots;
    s->snap.slot_occupancy = s->ticks ? s->occupancy_sum / (double)s->ticks : 0.0;
    s->snap.arena_bytes = s->arena.size();
    s->snap.arena_in_use = s->arena.in_use();
    s->snap.arena_peak = s->arena_peak;
    int running = 0;
    for (const SrvTask &t : s->active)
        for (int i = 0; i < t.n_mem; ++i) running += t.mem[i].ended ? 0 : 1;
    s->snap.active = running;
    s->snap.pending = (int32_t)s->pending.size();
}

void worker_loop(vne_server *s) {
    (void)hipSetDevice(s->ctx->device);
    for (;;) {
        std::vector<uint64_t> fresh;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            const bool idle = s->incoming.empty() && s->pending.empty() && s->active.empty();
            bool waits = false;
            for (auto &kv : s->queries) waits = waits || kv.second->stage_wait || kv.second->final_wait;
            if (idle && !waits) {
                if (s->stopping) break;
                s->cv_work.wait(lk);
                continue;
            }
            fresh.assign(s->incoming.begin(), s->incoming.end());
            s->incoming.clear();
            if (s->broken) {
                // fail everything still open (open queries are never erased)
                std::vector<SrvQuery *> open;
                for (auto &kv : s->queries)
                    if (!kv.second->done) open.push_back(kv.second.get());
                const std::string msg = s->broken_msg;
                lk.unlock();
                for (SrvQuery *q : open) {
                    q->stage_wait = q->final_wait = false;
                    q->started = false;
                    finish_query(s, *q, VNE_EDEVICE, msg);
                }
                s->pending.clear();
                s->active.clear();
                publish(s);
                continue;
            }
        }
        for (uint64_t tk : fresh) start_query(s, *query_of(s, tk));
        vne_status st = poll_events(s, false);
        if (st == VNE_OK) st = admit(s);
        if (st == VNE_OK && !s->active.empty()) {
            st = tick(s);
        } else if (st == VNE_OK && has_waits(s)) {
            st = poll_events(s, true);
        } else if (st == VNE_OK) {
            // nothing runs and nothing can start: wait for a submission
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait_for(lk, std::chrono::milliseconds(1));
        }
        if (st != VNE_OK) {
            std::lock_guard<std::mutex> lk(s->mu);
            if (!s->broken) {
                s->broken = true;
                s->broken_msg = "server loop failed";
            }
        }
        publish(s);
    }
    publish(s);
}

}  // namespace

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
    if (k.max_slots <= 0) k.max_slots = 64;
    if (k.max_cols <= 0) k.max_cols = 256;
    if (k.pilot_probes <= 0) k.pilot_probes = 16;
    if (k.max_probes <= 0) k.max_probes = 4096;
    if (k.max_steps <= 0) k.max_steps = 100;
    if (!(k.z > 0.0)) k.z = 2.576;
    if (k.mode & ~(uint32_t)(VNE_MODE_F64 | VNE_MODE_DESING)) return fail(c, VNE_EINVAL, "unknown mode bits");
    if (k.max_steps > kMaxSteps || k.max_cols > 4096 || k.pilot_probes > k.max_probes)
        return fail(c, VNE_EINVAL, "bad server limits");
    HIP_TRY(c, hipSetDevice(c->device));
    auto s = std::make_unique<vne_server>();
    s->ctx = c;
    s->cfg = k;
    s->fp64 = (k.mode & VNE_MODE_F64) != 0;
    s->desing = (k.mode & VNE_MODE_DESING) != 0;
    s->psi_cap = k.max_probes;
    s->query_bytes = rnd((size_t)s->psi_cap * 8) + 512;
    uint64_t bytes = k.arena_bytes;
    if (bytes == 0) {
        size_t fr = 0, tot = 0;
        HIP_TRY(c, hipMemGetInfo(&fr, &tot));
        bytes = fr / 4;
    }
    VNE_TRY(dev_alloc(c, &s->arena_mem, bytes));
    s->arena.reset(bytes);
    hipError_t e = hipStreamCreate(&s->stream);
    if (e != hipSuccess) {
        dev_free(c, &s->arena_mem);
        return hip_fail(c, e, "hipStreamCreate");
    }
    for (int r = 0; r < vne_server::kRing; ++r) {
        e = hipEventCreateWithFlags(&s->ring_ev[r], hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(c, e, "hipEventCreate");
    }
    e = hipHostMalloc((void **)&s->mailbox, sizeof(int2) * k.max_slots, hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(c, e, "hipHostMalloc");
    std::memset(s->mailbox, 0, sizeof(int2) * k.max_slots);
    for (int i = k.max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
    vne_server *raw = s.release();
    raw->worker = std::thread(worker_loop, raw);
    *out = raw;
    return VNE_OK;
}

extern "C" vne_status vne_server_submit(vne_server *s, const vne_query *q, uint64_t *ticket) {
    if (!s || !q || !ticket) return VNE_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) return VNE_EBUSY;
    }
    auto sq = std::make_unique<SrvQuery>();
    sq->q = *q;
    sq->t_submit = Clock::now();
    {
        vne_ctx *c = s->ctx;
        std::lock_guard<std::recursive_mutex> lock(c->mu);
        Graph *g = get_graph(c, q->graph_id);
        if (!g) return fail(c, VNE_EINVAL, "unknown graph id");
        if (!(q->rel_eps >= 0.0)) return fail(c, VNE_EINVAL, "rel_eps must be >= 0");
        if (q->rel_eps == 0.0) {
            if (q->m < 1 || q->m > s->psi_cap) return fail(c, VNE_EINVAL, "m must be in [1, max_probes]");
            if (q->k_steps < 1 || q->k_steps > kMaxSteps) return fail(c, VNE_EINVAL, "k_steps must be in [1, 128]");
        }
        if (s->desing && !g->zero_rowsum)
            return fail(c, VNE_EINVAL, "VNE_MODE_DESING needs a matrix whose rows sum to zero (A 1 = 0)");
        GraphSet *set = nullptr;
        VNE_TRY(get_set(c, {q->graph_id}, &set));
        sq->g = g;
        sq->set = set;
        g->in_use++;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->stopping) {   // stop began meanwhile
        lk.unlock();
        std::lock_guard<std::recursive_mutex> lock(s->ctx->mu);
        sq->g->in_use--;
        return VNE_EBUSY;
    }
    sq->ticket = s->next_ticket++;
    *ticket = sq->ticket;
    s->incoming.push_back(sq->ticket);
    s->queries[sq->ticket] = std::move(sq);
    s->cv_work.notify_one();
    return VNE_OK;
}

extern "C" vne_status vne_server_poll(vne_server *s, uint64_t ticket, int32_t timeout_ms, vne_query_result *res,
                                      double *quad, int32_t quad_cap) {
    if (!s || !res) return VNE_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->queries.find(ticket);
    if (it == s->queries.end()) return VNE_EINVAL;
    SrvQuery *q = it->second.get();
    auto ready = [&] { return q->done; };
    if (timeout_ms < 0) s->cv_done.wait(lk, ready);
    else if (timeout_ms > 0) s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
    if (!q->done) return VNE_EBUSY;
    *res = q->res;
    if (quad && quad_cap > 0)
        std::memcpy(quad, q->quad.data(), sizeof(double) * std::min<size_t>(quad_cap, q->quad.size()));
    s->queries.erase(it);
    return VNE_OK;
}

extern "C" vne_status vne_server_stats(vne_server *s, vne_server_info *st) {
    if (!s || !st) return VNE_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *st = s->snap;
    st->queries_done = s->queries_done;
    return VNE_OK;
}

extern "C" vne_status vne_server_stop(vne_server *s) {
    if (!s) return VNE_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    vne_ctx *c = s->ctx;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(s->stream);
    for (auto &kv : s->queries)
        if (!kv.second->done && kv.second->g) kv.second->g->in_use--;
    for (double *p : s->pinned_pool) (void)hipHostFree(p);
    for (auto &kv : s->queries)
        if (kv.second->h_buf) (void)hipHostFree(kv.second->h_buf);
    for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
    for (int r = 0; r < vne_server::kRing; ++r) {
        if (s->stage[r]) (void)hipHostFree(s->stage[r]);
        if (s->ring_ev[r]) (void)hipEventDestroy(s->ring_ev[r]);
    }
    if (s->d_desc) (void)hipFree(s->d_desc);
    if (s->mailbox) (void)hipHostFree(s->mailbox);
    dev_free(c, &s->arena_mem);
    (void)hipStreamDestroy(s->stream);
    delete s;
    return VNE_OK;
}
