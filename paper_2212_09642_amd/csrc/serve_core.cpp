// Scheduling core of the serving loop (host only); see serve_core.h.
#include "serve_core.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace vne {

namespace {

#define SC_TRY(expr)                           \
    do {                                       \
        const vne_status _s = (expr);          \
        if (_s != VNE_OK) return _s;           \
    } while (0)

constexpr int kPlanRounds = 4;     // probe-count plans of a rel_eps query (pilot included)
constexpr int kGroupWindow = 256;  // pending tasks searched for partners

double steady_ms() {
    using C = std::chrono::steady_clock;
    return std::chrono::duration<double, std::milli>(C::now().time_since_epoch()).count();
}

}  // namespace

ServeCore::ServeCore(const ServeConfig &cfg, ServeExec *exec, ClockMs clock)
    : cfg_(cfg), exec_(exec), clock_(clock ? clock : ClockMs(steady_ms)) {
    arena_.reset(cfg_.arena_bytes);
    for (int i = cfg_.max_slots - 1; i >= 0; --i) free_slots_.push_back(i);
}

ServeQuery *ServeCore::query_of(uint64_t ticket) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = queries_.find(ticket);
    return it == queries_.end() ? nullptr : it->second.get();
}

// Tasks for columns [c0, c1) of a query, in the pending queue after every
// task of an earlier ticket.  Widths: max_cols while that much is left, then
// the largest power of two (at least 16) that fits, then the rest, so that a
// task's width is a whole number of column tiles wherever possible.
void ServeCore::add_tasks(ServeQuery &q, int c0, int c1, bool pilot) {
    std::vector<ServeTask> ts;
    for (int c = c0; c < c1;) {
        const int rem = c1 - c;
        int w = rem;
        if (rem >= cfg_.max_cols) {
            w = cfg_.max_cols;
        } else if (rem >= 16) {
            w = 16;
            while (2 * w <= rem) w *= 2;
        }
        ServeTask t;
        t.m = w;
        exec_->tile(t.m, &t.mt, &t.m_pad);
        t.k = q.k;
        ServeMember &u = t.mem[0];
        u.ticket = q.ticket;
        u.m = w;
        u.col0 = c;
        u.pilot = pilot;
        u.adaptive = q.q.rel_eps > 0.0 && q.s_lower > 0.0;
        u.tol = 0.5 * q.q.rel_eps * q.s_lower;
        t.bytes = exec_->task_bytes(q, t.m_pad, t.k);
        ts.push_back(t);
        c += w;
    }
    q.cols_issued = c1;
    q.tasks_open += (int)ts.size();
    auto pos = pending_.begin();
    while (pos != pending_.end() && pos->mem[0].ticket <= q.ticket) ++pos;
    pending_.insert(pos, ts.begin(), ts.end());
}

// Turns a submitted query into tasks (explicit probe count, or the pilot).
void ServeCore::start_query(ServeQuery &q) {
    if (q.q.rel_eps > 0.0) {
        // Proposition 4.4 with Remark 2.3: ||c||^2 <= n for +-1 probes;
        // S(A) >= -log tr(A^2) for a unit-trace PSD matrix
        const bool density = std::fabs(q.trace - 1.0) < 1e-9 && q.fro2 > 0.0 && q.fro2 < 1.0;
        q.s_lower = density ? -std::log(q.fro2) : 0.0;
        q.k = density ? plan_steps((double)q.n, q.lambda_ub, q.s_lower, q.q.rel_eps, 0.5, cfg_.max_steps)
                      : cfg_.max_steps;
        // per-form target: the a-priori bound at k meets it, and adaptive
        // tasks stop once the a-posteriori bound does
        q.bound = density ? 0.5 * q.q.rel_eps * q.s_lower : 0.0;
        q.N = std::min(cfg_.pilot_probes, cfg_.psi_cap);
        add_tasks(q, 0, q.N, true);
    } else {
        q.k = q.q.k_steps;
        q.N = q.q.m;
        q.planned = true;
        add_tasks(q, 0, q.N, false);
    }
}

// Completion bookkeeping of a query whose result has reached the host (or
// that failed).  After done is set the query belongs to the caller of poll.
void ServeCore::finish_query(ServeQuery &q, vne_status st, const std::string &msg) {
    q.t_done = now();
    const double *f = exec_->forms(q);
    if (f && st == VNE_OK) {
        q.quad.assign(f, f + q.N);
        q.res.estimate = exec_->estimate(q);
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
    // the device's count when the final copy came back (a stop recorded on
    // the device can reach the host only after the task's cap), else the
    // host's
    const int32_t dev_steps = f && st == VNE_OK ? exec_->steps_taken(q) : 0;
    q.res.steps = dev_steps > 0 ? dev_steps : (q.steps_used > 0 ? q.steps_used : q.k);
    q.res.quad_bound = q.bound;
    q.res.queue_ms = q.started ? q.t_admit - q.t_submit : 0.0;
    q.res.latency_ms = q.t_done - q.t_submit;
    exec_->release_graph(q);
    exec_->close_query(q);
    if (q.started) arena_.release(q.off);
    q.started = false;
    std::lock_guard<std::mutex> lk(mu_);
    q.done = true;
    queries_done_++;
    cv_done_.notify_all();
}

// Drops the pending tasks of a query and reports the failure.
void ServeCore::fail_query(ServeQuery &q, vne_status st, const std::string &msg) {
    pending_.erase(std::remove_if(pending_.begin(), pending_.end(),
                                  [&](const ServeTask &t) { return t.mem[0].ticket == q.ticket; }),
                   pending_.end());
    q.stage_wait = q.final_wait = false;
    finish_query(q, st, msg);
}

static std::string flag_text(int32_t fl) {
    if (fl & 1) return "non-finite Lanczos coefficient";
    if (fl & 4) return "tridiagonal QR did not converge";
    if (fl & 8) return "tridiagonal QR rotation record overflowed";
    return "numerical failure";
}

// Pilot or final results that have reached the host.
vne_status ServeCore::poll_events(bool block_one) {
    std::vector<ServeQuery *> waiting;
    {
        std::lock_guard<std::mutex> lk(mu_);
        for (auto &kv : queries_)
            if (kv.second->stage_wait || kv.second->final_wait) waiting.push_back(kv.second.get());
    }
    bool blocked = false;
    for (ServeQuery *q : waiting) {
        bool done = false;
        SC_TRY(exec_->ready(*q, false, &done));
        if (!done && block_one && !blocked) {
            // nothing else to do: wait for the first copy still in flight
            blocked = true;
            SC_TRY(exec_->ready(*q, true, &done));
        }
        if (!done) continue;
        if (q->stage_wait) {
            q->stage_wait = false;
            const int n0 = q->cols_issued;
            const int32_t fl = exec_->flags(*q, false);
            if (fl) {
                fail_query(*q, VNE_ENUMERIC, flag_text(fl));
                continue;
            }
            const double *f = exec_->forms(*q);
            double mean = 0.0, var = 0.0;
            for (int i = 0; i < n0; ++i) mean += f[i];
            mean /= n0;
            for (int i = 0; i < n0; ++i) var += (f[i] - mean) * (f[i] - mean);
            const double sd = n0 > 1 ? std::sqrt(var / (n0 - 1)) : 0.0;
            // the rule's N from every form so far (sequential sampling: the
            // count is planned again after each stage), rounded up to whole
            // 16-column groups: the extra columns would be computed as
            // padding anyway, and more probes only tighten the estimate
            int nn = plan_probes(mean, sd, q->q.rel_eps, 0.5, cfg_.z, n0, cfg_.psi_cap);
            if (nn > n0) nn = std::min(cfg_.psi_cap, n0 + (nn - n0 + 15) / 16 * 16);
            q->rounds++;
            q->planned = true;
            q->N = nn;
            if (nn > n0) {
                add_tasks(*q, n0, nn, false);
            } else {
                SC_TRY(exec_->issue_final(*q));
                q->final_wait = true;
            }
        } else {
            q->final_wait = false;
            const int32_t fl = exec_->flags(*q, true);
            if (fl) finish_query(*q, VNE_ENUMERIC, flag_text(fl));
            else finish_query(*q, VNE_OK, "");
        }
    }
    return VNE_OK;
}

// The query's own arena block, taken when its first task is admitted.
// false: no room (nothing taken).
bool ServeCore::open_query(ServeQuery &q, vne_status *st) {
    *st = VNE_OK;
    if (!arena_.alloc(cfg_.query_bytes, &q.off)) return false;
    q.started = true;
    q.t_admit = now();
    *st = exec_->open_query(q);
    return true;
}

// A task that can join a group slot: 16 FP32 columns in one 16-column tile.
bool ServeCore::groupable(const ServeTask &t) const {
    return !cfg_.fp64 && cfg_.max_group > 1 && t.n_mem == 1 && t.m == 16 && t.m_pad == 16 && t.mt == 16;
}

// Starts waiting tasks while mailbox entries and arena space allow.  First
// come, first served: a task that does not fit blocks the ones behind it
// (with skip_blocked, later tasks that fit start meanwhile).  A 16-column
// FP32 task takes the first waiting 16-column tasks of the same graph with
// the same step cap and stopping mode as its partners in a group slot of
// two or four tasks (at most max_group), as far as mailbox entries and the
// arena allow.
vne_status ServeCore::admit() {
    size_t head = 0;   // index in pending_ of the task considered
    while (head < pending_.size() && !free_slots_.empty()) {
        ServeTask t = pending_[head];
        ServeQuery *q = query_of(t.mem[0].ticket);
        const uint64_t need = t.bytes + (q->started ? 0 : cfg_.query_bytes);
        if (need > arena_.size()) {
            fail_query(*q, VNE_ENOMEM,
                       "query needs " + std::to_string(need) + " bytes of slot state, the arena holds " +
                           std::to_string(arena_.size()));
            head = 0;   // the query's tasks left the queue, wherever they were
            continue;
        }
        auto blocked = [&]() {
            if (!cfg_.skip_blocked) return false;
            ++head;
            return true;
        };
        // partner search: pending indices of the partners, in queue order
        std::vector<size_t> partners;
        if (groupable(t) && free_slots_.size() >= 2) {
            const size_t lim = std::min(pending_.size(), head + (size_t)kGroupWindow);
            for (size_t i = head + 1; i < lim && (int)partners.size() + 1 < cfg_.max_group; ++i) {
                const ServeTask &c = pending_[i];
                if (!groupable(c) || c.k != t.k || c.mem[0].adaptive != t.mem[0].adaptive) continue;
                ServeQuery *cq = query_of(c.mem[0].ticket);
                if (!cq || cq->q.graph_id != q->q.graph_id) continue;
                partners.push_back(i);
            }
        }
        // the group: the largest power of two of the members found that
        // fits the free mailbox entries and the arena (with the blocks of the
        // queries that have not started yet)
        auto fits = [&](int g) {
            if (g > (int)free_slots_.size()) return false;
            uint64_t room = arena_.round(exec_->task_bytes(*q, 16 * g, t.k));
            std::vector<ServeQuery *> seen;
            for (int i = 0; i < g; ++i) {
                ServeQuery *mq = i == 0 ? q : query_of(pending_[partners[i - 1]].mem[0].ticket);
                if (mq->started || std::find(seen.begin(), seen.end(), mq) != seen.end()) continue;
                seen.push_back(mq);
                room += cfg_.query_bytes;
            }
            return arena_.largest_free() >= room;
        };
        int g = 1;
        while (2 * g <= 1 + (int)partners.size() && 2 * g <= cfg_.max_group) g *= 2;
        while (g > 1 && !fits(g)) g /= 2;
        partners.resize(g - 1);
        if (!q->started) {
            if (arena_.largest_free() < cfg_.query_bytes + arena_.round(t.bytes)) {
                if (blocked()) continue;
                break;
            }
            vne_status st;
            if (!open_query(*q, &st)) {
                if (blocked()) continue;
                break;
            }
            SC_TRY(st);
        }
        for (size_t pi = 0; pi < partners.size(); ++pi) {
            ServeQuery *cq = query_of(pending_[partners[pi]].mem[0].ticket);
            if (cq->started) continue;
            vne_status st;
            if (!open_query(*cq, &st)) {
                partners.resize(pi);
                SC_TRY(st);
                break;
            }
            SC_TRY(st);
        }
        // a group cut short by a query that could not open: the largest
        // power of two that remains
        g = 1;
        while (2 * g <= 1 + (int)partners.size()) g *= 2;
        partners.resize(g - 1);
        if (g > 1) {
            for (int i = 1; i < g; ++i) {
                t.mem[i] = pending_[partners[i - 1]].mem[0];
                t.mem[i].c_off = 16 * i;
            }
            t.n_mem = g;
            t.m = t.m_pad = 16 * g;
            t.bytes = exec_->task_bytes(*q, 16 * g, t.k);
        }
        if (!arena_.alloc(t.bytes, &t.off)) {
            if (g == 1) {
                if (blocked()) continue;
                break;
            }
            // no room for the group after all: the task alone
            g = 1;
            partners.clear();
            t.n_mem = 1;
            t.m = t.m_pad = 16;
            t.bytes = exec_->task_bytes(*q, 16, t.k);
            if (!arena_.alloc(t.bytes, &t.off)) {
                if (blocked()) continue;
                break;
            }
        }
        arena_peak_ = std::max(arena_peak_, arena_.in_use());
        for (size_t pi = partners.size(); pi-- > 0;) pending_.erase(pending_.begin() + partners[pi]);
        pending_.erase(pending_.begin() + head);
        ServeQuery *qm[kMaxMembers] = {};
        for (int i = 0; i < t.n_mem; ++i) {
            t.mem[i].uid = next_uid_ + i;
            t.mem[i].slot = free_slots_.back();
            free_slots_.pop_back();
            qm[i] = i == 0 ? q : query_of(t.mem[i].ticket);
        }
        next_uid_ += t.n_mem;
        SC_TRY(exec_->start_task(t, qm));
        active_.push_back(t);
        tasks_admitted_ += t.n_mem;
        pair_slots_ += t.n_mem == 2 ? 1 : 0;
        group_tasks_ += t.n_mem > 1 ? t.n_mem : 0;
    }
    return VNE_OK;
}

// Quadrature of member i of a slot after `steps` steps, its mailbox entry
// back, and the query's next stage when it was the query's last task.
vne_status ServeCore::end_member(ServeTask &t, int i, ServeQuery &q, int steps) {
    ServeMember &u = t.mem[i];
    SC_TRY(exec_->quadrature(t, i, q, steps));
    u.ended = true;
    free_slots_.push_back(u.slot);
    q.steps_used = std::max(q.steps_used, steps);
    q.tasks_open--;
    if (q.tasks_open > 0) return VNE_OK;
    if (q.q.rel_eps > 0.0 && q.rounds < kPlanRounds && q.cols_issued < cfg_.psi_cap) {
        // a stage of a rel_eps query done: its forms and the flags to the
        // host, which plans the probe count again from all forms so far
        SC_TRY(exec_->issue_stage(q));
        q.stage_wait = true;
    } else {
        q.N = q.cols_issued;
        SC_TRY(exec_->issue_final(q));
        q.final_wait = true;
    }
    return VNE_OK;
}

// One Lanczos step of every active slot; members at their step cap, and
// adaptive members whose recorded stop step has reached the host, end.
vne_status ServeCore::tick() {
    const int A = (int)active_.size();
    std::vector<ServeQuery *> qs((size_t)kMaxMembers * A, nullptr);
    int running = 0;
    for (int i = 0; i < A; ++i)
        for (int mi = 0; mi < active_[i].n_mem; ++mi) {
            // a member that ended may belong to a query that has finished
            // (and whose result the caller may have taken already)
            if (active_[i].mem[mi].ended) continue;
            qs[(size_t)kMaxMembers * i + mi] = query_of(active_[i].mem[mi].ticket);
            running++;
        }
    SC_TRY(exec_->tick(active_, qs));
    ticks_++;
    occupancy_sum_ += running;
    std::vector<ServeTask> keep;
    for (int i = 0; i < A; ++i) {
        ServeTask &t = active_[i];
        t.j++;
        bool open = false;
        for (int mi = 0; mi < t.n_mem; ++mi) {
            ServeMember &u = t.mem[mi];
            if (u.ended) continue;
            int use = t.j >= t.k ? t.k : 0;
            if (!use && u.adaptive) {
                int32_t id = 0, st = 0;
                exec_->stop_record(u.slot, &id, &st);
                if (id == u.uid && st > 0) use = st;
            }
            if (!use) {
                open = true;
                continue;
            }
            SC_TRY(end_member(t, mi, *qs[(size_t)kMaxMembers * i + mi], use));
        }
        if (open) keep.push_back(t);
        else arena_.release(t.off);
    }
    active_.swap(keep);
    return VNE_OK;
}

bool ServeCore::has_waits() {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto &kv : queries_)
        if (kv.second->stage_wait || kv.second->final_wait) return true;
    return false;
}

// Snapshot of the worker-owned counters for stats().
void ServeCore::publish() {
    std::lock_guard<std::mutex> lk(mu_);
    snap_.ticks = ticks_;
    snap_.tasks = tasks_admitted_;
    snap_.pair_slots = pair_slots_;
    snap_.group_tasks = group_tasks_;
    snap_.slot_occupancy = ticks_ ? occupancy_sum_ / (double)ticks_ : 0.0;
    snap_.arena_bytes = arena_.size();
    snap_.arena_in_use = arena_.in_use();
    snap_.arena_peak = arena_peak_;
    int running = 0;
    for (const ServeTask &t : active_)
        for (int i = 0; i < t.n_mem; ++i) running += t.mem[i].ended ? 0 : 1;
    snap_.active = running;
    snap_.pending = (int32_t)pending_.size();
}

// After a failure of the device: every query still open ends with it.
void ServeCore::fail_all(const std::string &msg) {
    std::vector<ServeQuery *> open;
    {
        std::lock_guard<std::mutex> lk(mu_);
        for (auto &kv : queries_)
            if (!kv.second->done) open.push_back(kv.second.get());
    }
    for (ServeQuery *q : open) {
        q->stage_wait = q->final_wait = false;
        q->started = false;
        finish_query(*q, VNE_EDEVICE, msg);
    }
    pending_.clear();
    active_.clear();
}

void ServeCore::run() {
    exec_->thread_init();
    for (;;) {
        std::vector<uint64_t> fresh;
        bool broken = false;
        std::string msg;
        {
            std::unique_lock<std::mutex> lk(mu_);
            const bool idle = incoming_.empty() && pending_.empty() && active_.empty();
            bool waits = false;
            for (auto &kv : queries_) waits = waits || kv.second->stage_wait || kv.second->final_wait;
            if (idle && !waits) {
                if (stopping_) break;
                cv_work_.wait(lk);
                continue;
            }
            fresh.assign(incoming_.begin(), incoming_.end());
            incoming_.clear();
            broken = broken_;
            msg = broken_msg_;
        }
        if (broken) {
            fail_all(msg);
            publish();
            continue;
        }
        for (uint64_t tk : fresh) start_query(*query_of(tk));
        vne_status st = poll_events(false);
        if (st == VNE_OK) st = admit();
        if (st == VNE_OK && !active_.empty()) {
            st = tick();
        } else if (st == VNE_OK && has_waits()) {
            st = poll_events(true);
        } else if (st == VNE_OK) {
            // nothing runs and nothing can start: wait for a submission
            std::unique_lock<std::mutex> lk(mu_);
            cv_work_.wait_for(lk, std::chrono::milliseconds(1));
        }
        if (st != VNE_OK) {
            const std::string why = exec_->error_text();
            std::lock_guard<std::mutex> lk(mu_);
            if (!broken_) {
                broken_ = true;
                broken_msg_ = why.empty() ? "server loop failed" : why;
            }
        }
        publish();
    }
    publish();
}

vne_status ServeCore::submit(std::unique_ptr<ServeQuery> q, uint64_t *ticket) {
    std::lock_guard<std::mutex> lk(mu_);
    if (stopping_) return VNE_EBUSY;
    q->ticket = next_ticket_++;
    q->t_submit = now();
    *ticket = q->ticket;
    incoming_.push_back(q->ticket);
    queries_[q->ticket] = std::move(q);
    cv_work_.notify_one();
    return VNE_OK;
}

vne_status ServeCore::poll(uint64_t ticket, int32_t timeout_ms, vne_query_result *res, double *quad,
                           int32_t quad_cap) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = queries_.find(ticket);
    if (it == queries_.end()) return VNE_EINVAL;
    ServeQuery *q = it->second.get();
    auto ready = [&] { return q->done; };
    if (timeout_ms < 0) cv_done_.wait(lk, ready);
    else if (timeout_ms > 0) cv_done_.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
    if (!q->done) return VNE_EBUSY;
    *res = q->res;
    if (quad && quad_cap > 0 && !q->quad.empty())
        std::memcpy(quad, q->quad.data(), sizeof(double) * std::min<size_t>(quad_cap, q->quad.size()));
    queries_.erase(it);
    return VNE_OK;
}

void ServeCore::stats(vne_server_info *st) {
    std::lock_guard<std::mutex> lk(mu_);
    *st = snap_;
    st->queries_done = queries_done_;
}

bool ServeCore::stopping() {
    std::lock_guard<std::mutex> lk(mu_);
    return stopping_;
}

void ServeCore::request_stop() {
    std::lock_guard<std::mutex> lk(mu_);
    stopping_ = true;
    cv_work_.notify_all();
}

std::vector<ServeQuery *> ServeCore::unfinished() {
    std::lock_guard<std::mutex> lk(mu_);
    std::vector<ServeQuery *> out;
    for (auto &kv : queries_)
        if (!kv.second->done) out.push_back(kv.second.get());
    return out;
}

}  // namespace vne
