// Host check of the serving loop's scheduling core (ServeCore) against a
// host-only executor: every device step is replaced by bookkeeping that
// checks the core's promises.
//  - Slot state never overlaps: every task's and query's arena range is
//    disjoint from every other live one and inside the arena; a mailbox entry
//    is held by one running member at a time.
//  - Each quadratic form reaches its own query's column: form c of a query
//    is a function of (seed, c) only, so a column routed to the wrong query
//    or the wrong place in a group slot shows.
//  - A member ends at its step cap, or (a-posteriori stopping) at the stop
//    step its device record holds, and never steps past its cap; the
//    records reach the host 0 to 3 ticks late, so a member can reach its cap
//    first, and the device's own record still decides its steps and the
//    query's reported step count.
//  - First come, first served: with one slot, tasks start in ticket order.
//  - Group slots: 16-column tasks of one graph queued together start in
//    groups of up to max_group, the largest power of two the free mailbox
//    entries and the arena allow.
//  - Arena peak within the arena; everything released at the end.
//  - Oversize queries fail with VNE_ENOMEM, a non-finite stage with
//    VNE_ENUMERIC, a device failure ends every open query with VNE_EDEVICE.
//  - Stop with queries in flight drains them; later submissions get
//    VNE_EBUSY.
// Clients submit and poll from several threads while the worker runs; the
// program is built with ThreadSanitizer and with AddressSanitizer (tests/
// test_serve_core.py).
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "serve_core.h"

using namespace vne;

static std::atomic<int> g_fail{0};
#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
            std::printf(__VA_ARGS__);                      \
            std::printf("\n");                             \
            g_fail++;                                      \
        }                                                  \
    } while (0)

// form c of a query with probe seed `seed`
static double form_of(uint64_t seed, int c) {
    uint64_t z = seed * 0x9E3779B97F4A7C15ull + (uint64_t)c * 0xBF58476D1CE4E5B9ull + 1;
    z ^= z >> 31;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 29;
    return 10.0 + ((double)(z >> 11) / 9007199254740992.0 - 0.5);
}

// the device's stop step of an adaptive member (a check step 3, 5, ..., 11)
static int stop_of(uint64_t ticket, int col0) { return 3 + 2 * (int)((ticket * 7 + (uint64_t)col0) % 5); }

struct I2 {
    int32_t x, y;
};

struct Graph {
    int64_t n;
    double lambda_ub, fro2, trace;
};

struct FakeQ {
    int graph = 0;
    std::vector<double> dev;         // the device's forms
    std::vector<double> host;        // forms, estimate, flags of the last copy
    std::vector<double> staged;      // copy in flight
    int countdown = -1;              // polls until the copy lands (-1: none)
    bool opened = false;
    bool numeric = false;            // the stage's flags report a failure
    int dev_steps = 0;               // the most steps a quadrature took (device side)
};

class FakeExec : public ServeExec {
public:
    uint64_t arena_bytes = 0, query_bytes = 0;
    int psi_cap = 0, max_slots = 0;
    std::vector<Graph> graphs;
    std::vector<int> in_use;
    std::mutex in_use_mu;                     // clients take a graph, the worker gives it back
    std::mt19937 rng{3};
    int fail_tick = -1;              // tick at which the device fails (-1: never)
    int ticks = 0;
    // while hold is set, a tick waits (and sets held): submissions then
    // queue up behind the running tasks
    std::atomic<bool> hold{false}, held{false};
    // checks
    std::map<uint64_t, uint64_t> live;        // arena offset -> end
    std::map<uint64_t, int> task_members;     // task offset -> members not ended
    std::set<int> busy_slots;
    std::vector<I2> mailbox;                // {uid, step} as the host sees it
    // stop records: on the device at once (by uid), in the host's mailbox
    // 0 to 3 ticks later, as over the real copy path
    std::map<int32_t, int> dev_stop;
    struct Post {
        int visible_at, slot;
        I2 rec;
    };
    std::vector<Post> posts;
    int cap_first = 0;                        // members that reached the cap before their record
    std::vector<uint64_t> start_order;        // ticket of each started task
    std::map<uint64_t, std::vector<std::pair<int, int>>> ended;   // ticket -> (col0, steps)
    std::mutex log_mu;                        // start_order / ended are read by the main thread at the end

    static FakeQ *fq(ServeQuery &q) { return static_cast<FakeQ *>(q.x); }

    void take(uint64_t off, uint64_t bytes) {
        CHECK(off + bytes <= arena_bytes, "range [%llu, %llu) outside the arena", (unsigned long long)off,
              (unsigned long long)(off + bytes));
        auto it = live.lower_bound(off);
        if (it != live.end()) CHECK(it->first >= off + bytes, "overlap with a later live range");
        if (it != live.begin()) {
            --it;
            CHECK(it->second <= off, "overlap with an earlier live range");
        }
        live[off] = off + bytes;
    }
    void drop(uint64_t off) {
        CHECK(live.count(off) == 1, "release of an unknown range");
        live.erase(off);
    }

    uint64_t task_bytes(const ServeQuery &q, int m_pad, int k) override {
        return (uint64_t)graphs[static_cast<FakeQ *>(q.x)->graph].n * m_pad / 4 + (uint64_t)m_pad * k * 16 + 4096;
    }
    void tile(int m, int *mt, int *m_pad) override {
        *mt = m <= 16 ? 16 : 64;
        *m_pad = (m + *mt - 1) / *mt * *mt;
    }
    vne_status open_query(ServeQuery &q) override {
        FakeQ *x = fq(q);
        CHECK(!x->opened, "query opened twice");
        x->opened = true;
        x->dev.assign(psi_cap, 0.0);
        x->host.assign(psi_cap + 2, 0.0);
        take(q.off, query_bytes);
        return VNE_OK;
    }
    vne_status start_task(ServeTask &t, ServeQuery *const *qm) override {
        CHECK(t.n_mem == 1 || t.n_mem == 2 || t.n_mem == 4, "group slot of %d tasks", t.n_mem);
        for (int i = 0; i < t.n_mem; ++i) {
            CHECK(qm[i] && fq(*qm[i])->opened, "member %d of a query that is not open", i);
            CHECK(qm[i]->ticket == t.mem[i].ticket, "member %d's query mismatch", i);
            if (t.group())
                CHECK(qm[i]->q.graph_id == qm[0]->q.graph_id && t.mem[i].c_off == 16 * i && t.mem[i].m == 16 &&
                          t.m == 16 * t.n_mem && t.m_pad == t.m && t.mt == 16,
                      "bad group slot");
        }
        take(t.off, t.bytes);
        task_members[t.off] = t.n_mem;
        for (int i = 0; i < t.n_mem; ++i) {
            CHECK(t.mem[i].slot >= 0 && t.mem[i].slot < max_slots, "mailbox entry out of range");
            CHECK(busy_slots.insert(t.mem[i].slot).second, "mailbox entry %d held twice", t.mem[i].slot);
            mailbox[t.mem[i].slot] = {0, 0};
            std::lock_guard<std::mutex> lk(log_mu);
            start_order.push_back(t.mem[i].ticket);
        }
        return VNE_OK;
    }
    vne_status tick(const std::vector<ServeTask> &active, const std::vector<ServeQuery *> &qs) override {
        if (ticks++ == fail_tick) return VNE_EDEVICE;
        if (hold.load()) {
            held.store(true);
            while (hold.load()) std::this_thread::yield();
        }
        for (size_t i = 0; i < active.size(); ++i) {
            const ServeTask &t = active[i];
            CHECK(t.j < t.k, "a slot stepped past its cap");
            CHECK(task_members.count(t.off) == 1, "tick of a slot that is not live");
            for (int mi = 0; mi < t.n_mem; ++mi) {
                const ServeMember &u = t.mem[mi];
                // a running member's query, and none for a member that ended
                // (its query may be gone)
                const ServeQuery *mq = qs[(size_t)kMaxMembers * i + mi];
                CHECK(u.ended ? mq == nullptr : (mq && mq->ticket == u.ticket), "member's query mismatch");
                if (u.ended || !u.adaptive) continue;
                const int j = t.j + 1, s = stop_of(u.ticket, u.col0);
                if (j >= 3 && j % 2 == 1 && j < t.k && j >= s && dev_stop.count(u.uid) == 0) {
                    dev_stop[u.uid] = s;
                    posts.push_back({ticks + (int)(rng() % 4), u.slot, {u.uid, s}});
                }
            }
        }
        return VNE_OK;
    }
    void stop_record(int slot, int32_t *uid, int32_t *step) override {
        for (size_t i = 0; i < posts.size();) {
            if (posts[i].visible_at <= ticks) {
                mailbox[posts[i].slot] = posts[i].rec;
                posts[i] = posts.back();
                posts.pop_back();
            } else {
                ++i;
            }
        }
        *uid = mailbox[slot].x;
        *step = mailbox[slot].y;
    }
    vne_status quadrature(const ServeTask &t, int i, ServeQuery &q, int steps) override {
        const ServeMember &u = t.mem[i];
        const int want = u.adaptive ? std::min(stop_of(u.ticket, u.col0), t.k) : t.k;
        // the host passes its step count (the cap when the record had not
        // reached it yet); the device takes its own record first
        int used = steps;
        if (u.adaptive && dev_stop.count(u.uid)) used = std::min(used, dev_stop[u.uid]);
        CHECK(used == want, "member of ticket %llu ended at %d steps (host %d), expected %d",
              (unsigned long long)u.ticket, used, steps, want);
        CHECK(steps == want || (steps == t.k && u.adaptive), "host ended member of ticket %llu at %d, not %d or the cap",
              (unsigned long long)u.ticket, steps, want);
        fq(q)->dev_steps = std::max(fq(q)->dev_steps, used);
        if (steps == t.k && used < t.k) cap_first++;
        CHECK(u.col0 + u.m <= psi_cap, "columns beyond the query's forms");
        for (int c = 0; c < u.m; ++c) fq(q)->dev[u.col0 + c] = form_of(q.q.seed, u.col0 + c);
        CHECK(busy_slots.erase(u.slot) == 1, "mailbox entry freed twice");
        {
            std::lock_guard<std::mutex> lk(log_mu);
            ended[q.ticket].push_back({u.col0, used});
        }
        if (--task_members[t.off] == 0) {
            task_members.erase(t.off);
            drop(t.off);
        }
        return VNE_OK;
    }
    vne_status issue_stage(ServeQuery &q) override {
        FakeQ *x = fq(q);
        x->staged.assign(x->dev.begin(), x->dev.begin() + q.cols_issued);
        x->staged.resize(psi_cap + 2, 0.0);
        x->staged[psi_cap + 1] = x->numeric ? 1.0 : 0.0;
        x->countdown = (int)(rng() % 3);
        return VNE_OK;
    }
    vne_status issue_final(ServeQuery &q) override {
        FakeQ *x = fq(q);
        double mean = 0.0;
        for (int c = 0; c < q.N; ++c) mean += x->dev[c];
        x->staged.assign(x->dev.begin(), x->dev.begin() + q.N);
        x->staged.push_back(mean / q.N);
        x->staged.push_back(0.0);
        x->staged.push_back((double)x->dev_steps);
        x->countdown = (int)(rng() % 3);
        return VNE_OK;
    }
    vne_status ready(ServeQuery &q, bool block, bool *done) override {
        FakeQ *x = fq(q);
        CHECK(x->countdown >= 0, "poll of a query with no copy in flight");
        if (x->countdown > 0 && !block) {
            x->countdown--;
            *done = false;
            return VNE_OK;
        }
        x->host = x->staged;
        x->countdown = -1;
        *done = true;
        return VNE_OK;
    }
    const double *forms(ServeQuery &q) override { return q.x && fq(q)->opened ? fq(q)->host.data() : nullptr; }
    double estimate(ServeQuery &q) override { return fq(q)->host[q.N]; }
    int32_t steps_taken(ServeQuery &q) override { return (int32_t)fq(q)->host[q.N + 2]; }
    // the most steps a member of the query ended at (device side), once done
    int max_steps_of(uint64_t ticket) {
        std::lock_guard<std::mutex> lk(log_mu);
        int m = 0;
        for (const auto &e : ended[ticket]) m = std::max(m, e.second);
        return m;
    }
    int32_t flags(ServeQuery &q, bool final) override {
        return fq(q)->host[final ? q.N + 1 : psi_cap + 1] != 0.0 ? 1 : 0;
    }
    void close_query(ServeQuery &q) override {
        FakeQ *x = fq(q);
        if (!x) return;
        if (x->opened && live.count(q.off)) drop(q.off);
        delete x;
        q.x = nullptr;
    }
    void release_graph(ServeQuery &q) override {
        FakeQ *x = fq(q);
        if (!x) return;
        std::lock_guard<std::mutex> lk(in_use_mu);
        in_use[x->graph]--;
        CHECK(in_use[x->graph] >= 0, "graph released more often than used");
    }
    std::string error_text() override { return "injected device failure"; }
};

struct Setup {
    FakeExec ex;
    std::unique_ptr<ServeCore> core;
    std::thread worker;
    std::atomic<int64_t> clock_ms{0};
    Setup(int max_slots, uint64_t arena, int psi_cap, bool skip, int fail_tick = -1, int max_group = 2) {
        ex.arena_bytes = arena;
        ex.query_bytes = (uint64_t)psi_cap * 8 + 512;
        ex.psi_cap = psi_cap;
        ex.max_slots = max_slots;
        ex.mailbox.assign(max_slots, {0, 0});
        ex.fail_tick = fail_tick;
        // density matrices (unit trace, tr(A^2) < 1) of several sizes, and
        // one too large for the arena
        ex.graphs = {{1000, 0.01, 0.002, 1.0}, {5000, 0.004, 4e-4, 1.0}, {20000, 1e-3, 1e-4, 1.0},
                     {300, 0.05, 0.01, 1.0}, {50000, 5e-4, 4e-5, 1.0}, {2000000000, 1e-9, 1e-9, 1.0}};
        ex.in_use.assign(ex.graphs.size(), 0);
        ServeConfig c;
        c.max_slots = max_slots;
        c.max_cols = 64;
        c.pilot_probes = 16;
        c.psi_cap = psi_cap;
        c.max_steps = 24;
        c.arena_bytes = arena;
        c.query_bytes = ex.query_bytes;
        c.skip_blocked = skip;
        c.max_group = max_group;
        core.reset(new ServeCore(c, &ex, [this] { return (double)clock_ms.fetch_add(1); }));
        worker = std::thread([this] { core->run(); });
    }
    vne_status submit(int graph, double rel_eps, int m, int k, uint64_t seed, uint64_t *ticket, bool numeric = false) {
        auto q = std::make_unique<ServeQuery>();
        q->q.graph_id = graph;
        q->q.rel_eps = rel_eps;
        q->q.m = m;
        q->q.k_steps = k;
        q->q.seed = seed;
        const Graph &g = ex.graphs[graph];
        q->n = g.n;
        q->lambda_ub = g.lambda_ub;
        q->fro2 = g.fro2;
        q->trace = g.trace;
        auto x = std::make_unique<FakeQ>();
        x->graph = graph;
        x->numeric = numeric;
        q->x = x.get();
        // the caller's side of a submission: the graph is in use from here
        {
            std::lock_guard<std::mutex> lk(ex.in_use_mu);
            ex.in_use[graph]++;
        }
        const vne_status st = core->submit(std::move(q), ticket);
        if (st == VNE_OK) {
            x.release();
        } else {
            std::lock_guard<std::mutex> lk(ex.in_use_mu);
            ex.in_use[graph]--;
        }
        return st;
    }
    void finish() {
        core->request_stop();
        worker.join();
        CHECK(core->unfinished().empty(), "queries left unfinished after stop");
    }
};

struct Want {
    uint64_t ticket;
    int graph;
    double rel_eps;
    int m, k;
    uint64_t seed;
    vne_status status;
};

static void check_result(const Want &w, const vne_query_result &r, const std::vector<double> &quad, int psi_cap,
                         FakeExec *ex = nullptr) {
    CHECK(r.status == w.status, "ticket %llu: status %d, expected %d (%s)", (unsigned long long)w.ticket, r.status,
          w.status, r.message);
    if (r.status != VNE_OK) return;
    // the reported steps are the device's: a task that reached its cap
    // before its stop record reached the host still reports its stop
    if (ex)
        CHECK(r.steps == ex->max_steps_of(w.ticket), "ticket %llu: %d steps reported, the tasks took %d",
              (unsigned long long)w.ticket, r.steps, ex->max_steps_of(w.ticket));
    if (w.rel_eps == 0.0) {
        CHECK(r.probes == w.m, "ticket %llu: %d probes, expected %d", (unsigned long long)w.ticket, r.probes, w.m);
        CHECK(r.steps == w.k, "ticket %llu: %d steps, expected %d", (unsigned long long)w.ticket, r.steps, w.k);
    } else {
        CHECK(r.probes >= 16 && r.probes <= psi_cap, "ticket %llu: %d probes", (unsigned long long)w.ticket, r.probes);
    }
    double mean = 0.0;
    for (int c = 0; c < r.probes; ++c) {
        CHECK(quad[c] == form_of(w.seed, c), "ticket %llu: form %d is another column's", (unsigned long long)w.ticket,
              c);
        mean += quad[c];
    }
    mean /= r.probes;
    CHECK(std::fabs(r.estimate - mean) <= 1e-12 * std::fabs(mean), "ticket %llu: estimate", (unsigned long long)w.ticket);
    CHECK(r.queue_ms >= 0.0 && r.latency_ms >= r.queue_ms, "ticket %llu: times", (unsigned long long)w.ticket);
}

// Several client threads submit and poll a mix of queries.
static void mixed_clients(bool skip, int group) {
    const int psi_cap = 512;
    Setup s(12, 24ull << 20, psi_cap, skip, -1, group);
    const int T = 4, Q = 30;
    std::vector<std::thread> clients;
    std::mutex want_mu;
    std::vector<Want> all;
    for (int th = 0; th < T; ++th)
        clients.emplace_back([&, th] {
            std::mt19937 r(100 + th);
            std::vector<Want> mine;
            for (int i = 0; i < Q; ++i) {
                Want w{};
                w.graph = (int)(r() % 5);
                w.seed = r();
                w.status = VNE_OK;
                const int kind = (int)(r() % 4);
                if (kind == 0) {
                    w.rel_eps = 1e-2;
                } else if (kind == 1) {
                    w.rel_eps = 2e-3;
                } else {
                    w.m = kind == 2 ? 16 : 1 + (int)(r() % 200);
                    w.k = 2 + (int)(r() % 20);
                }
                if (i == 7 && th == 0) {     // does not fit the arena
                    w.graph = 5;
                    w.rel_eps = 0.0;
                    w.m = 16;
                    w.k = 4;
                    w.status = VNE_ENOMEM;
                }
                const vne_status st = s.submit(w.graph, w.rel_eps, w.m, w.k, w.seed, &w.ticket);
                CHECK(st == VNE_OK, "submit failed");
                mine.push_back(w);
                if (r() % 3 == 0) std::this_thread::yield();
            }
            // poll: blocking for some, spinning for the others
            for (size_t i = 0; i < mine.size(); ++i) {
                vne_query_result res{};
                std::vector<double> quad(psi_cap);
                vne_status st;
                if (i % 2) {
                    st = s.core->poll(mine[i].ticket, -1, &res, quad.data(), psi_cap);
                } else {
                    while ((st = s.core->poll(mine[i].ticket, 0, &res, quad.data(), psi_cap)) == VNE_EBUSY)
                        std::this_thread::yield();
                }
                CHECK(st == VNE_OK, "poll failed");
                check_result(mine[i], res, quad, psi_cap, &s.ex);
                vne_query_result again{};
                CHECK(s.core->poll(mine[i].ticket, 0, &again, nullptr, 0) == VNE_EINVAL, "ticket kept after poll");
            }
            std::lock_guard<std::mutex> lk(want_mu);
            all.insert(all.end(), mine.begin(), mine.end());
        });
    for (auto &c : clients) c.join();
    // after the worker has stopped: its last snapshot (a client's poll can
    // return before the worker publishes the iteration that completed it)
    s.finish();
    vne_server_info info{};
    s.core->stats(&info);
    CHECK(info.queries_done == T * Q, "queries done %lld", (long long)info.queries_done);
    CHECK(info.arena_peak <= info.arena_bytes, "arena peak beyond the arena");
    CHECK(info.arena_in_use == 0 && info.active == 0 && info.pending == 0, "server not empty at the end");
    CHECK(s.ex.live.empty() && s.ex.busy_slots.empty() && s.ex.task_members.empty(), "state left behind");
    for (int v : s.ex.in_use) CHECK(v == 0, "graph still in use");
    if (!skip) CHECK(info.pair_slots > 0, "no pair slot was formed");
    if (group == 2) CHECK(info.group_tasks == 2 * info.pair_slots, "a group beyond two with max_group 2");
    std::printf("mixed clients (skip_blocked=%d, groups of up to %d): %lld queries, %lld tasks, %lld pair slots, "
                "%lld tasks in group slots, %d reached the cap before their stop record, arena peak %llu of %llu\n",
                (int)skip, group, (long long)info.queries_done, (long long)info.tasks, (long long)info.pair_slots,
                (long long)info.group_tasks, s.ex.cap_first, (unsigned long long)info.arena_peak,
                (unsigned long long)info.arena_bytes);
}

// One slot: tasks start in ticket order, each query's tasks in column order.
static void fcfs_order() {
    Setup s(1, 64ull << 20, 256, false);
    std::vector<Want> ws;
    for (int i = 0; i < 25; ++i) {
        Want w{};
        w.graph = i % 4;
        w.m = 1 + (i * 37) % 150;
        w.k = 3 + i % 7;
        w.seed = 1000 + i;
        w.status = VNE_OK;
        CHECK(s.submit(w.graph, 0.0, w.m, w.k, w.seed, &w.ticket) == VNE_OK, "submit");
        ws.push_back(w);
    }
    for (const Want &w : ws) {
        vne_query_result r{};
        std::vector<double> quad(256);
        CHECK(s.core->poll(w.ticket, -1, &r, quad.data(), 256) == VNE_OK, "poll");
        check_result(w, r, quad, 256);
    }
    s.finish();
    std::lock_guard<std::mutex> lk(s.ex.log_mu);
    for (size_t i = 1; i < s.ex.start_order.size(); ++i)
        CHECK(s.ex.start_order[i] >= s.ex.start_order[i - 1], "task of ticket %llu started after ticket %llu",
              (unsigned long long)s.ex.start_order[i - 1], (unsigned long long)s.ex.start_order[i]);
    for (auto &kv : s.ex.ended)
        for (size_t i = 1; i < kv.second.size(); ++i)
            CHECK(kv.second[i].first > kv.second[i - 1].first, "columns of a query out of order with one slot");
    std::printf("first come, first served: %zu tasks in ticket order\n", s.ex.start_order.size());
}

// Eight 16-column queries of one graph queue up while a one-column query
// holds the worker in a tick; then they start in group slots as large as
// max_group and the free mailbox entries allow.
static void group_slots(int slots, int group, int64_t want_group_tasks, int64_t want_pairs,
                        uint64_t arena = 32ull << 20) {
    const int psi_cap = 64;
    Setup s(slots, arena, psi_cap, false, -1, group);
    s.ex.hold.store(true);
    Want blocker{};
    blocker.graph = 0;
    blocker.m = 1;
    blocker.k = 24;
    blocker.seed = 99;
    blocker.status = VNE_OK;
    CHECK(s.submit(blocker.graph, 0.0, blocker.m, blocker.k, blocker.seed, &blocker.ticket) == VNE_OK, "submit");
    while (!s.ex.held.load()) std::this_thread::yield();
    std::vector<Want> ws(8);
    for (int i = 0; i < 8; ++i) {
        ws[i] = Want{};
        ws[i].graph = 1;
        ws[i].m = 16;
        ws[i].k = 8;
        ws[i].seed = 1000 + i;
        ws[i].status = VNE_OK;
        CHECK(s.submit(ws[i].graph, 0.0, ws[i].m, ws[i].k, ws[i].seed, &ws[i].ticket) == VNE_OK, "submit");
    }
    s.ex.hold.store(false);
    ws.push_back(blocker);
    for (Want &w : ws) {
        vne_query_result res{};
        std::vector<double> quad(psi_cap);
        CHECK(s.core->poll(w.ticket, -1, &res, quad.data(), psi_cap) == VNE_OK, "poll failed");
        check_result(w, res, quad, psi_cap, &s.ex);
    }
    s.finish();
    vne_server_info info{};
    s.core->stats(&info);
    CHECK(info.group_tasks == want_group_tasks && info.pair_slots == want_pairs,
          "%d mailbox entries, groups of up to %d: %lld tasks in group slots, %lld pair slots (expected %lld, %lld)",
          slots, group, (long long)info.group_tasks, (long long)info.pair_slots, (long long)want_group_tasks,
          (long long)want_pairs);
    std::printf("group slots (%d mailbox entries, up to %d, arena %llu): %lld tasks in group slots, %lld pair slots\n",
                slots, group, (unsigned long long)arena, (long long)info.group_tasks, (long long)info.pair_slots);
}

// A stage whose flags report a failure ends its query; the others complete.
static void numeric_stage() {
    Setup s(8, 32ull << 20, 256, false);
    uint64_t bad = 0, good = 0;
    CHECK(s.submit(1, 1e-2, 0, 0, 5, &bad, true) == VNE_OK, "submit");
    CHECK(s.submit(1, 1e-2, 0, 0, 6, &good) == VNE_OK, "submit");
    vne_query_result r{};
    CHECK(s.core->poll(bad, -1, &r, nullptr, 0) == VNE_OK && r.status == VNE_ENUMERIC, "numeric failure not reported");
    CHECK(s.core->poll(good, -1, &r, nullptr, 0) == VNE_OK && r.status == VNE_OK, "other query failed");
    s.finish();
    for (int v : s.ex.in_use) CHECK(v == 0, "graph still in use");
    std::printf("non-finite stage: reported, other query unaffected\n");
}

// Stop while queries are queued and running: they all complete, later
// submissions are refused.
static void stop_in_flight() {
    Setup s(6, 16ull << 20, 256, false);
    std::vector<Want> ws;
    for (int i = 0; i < 60; ++i) {
        Want w{};
        w.graph = i % 5;
        w.rel_eps = i % 3 == 0 ? 1e-2 : 0.0;
        w.m = 16 + (i % 5) * 24;
        w.k = 4 + i % 11;
        w.seed = 77 + i;
        w.status = VNE_OK;
        CHECK(s.submit(w.graph, w.rel_eps, w.m, w.k, w.seed, &w.ticket) == VNE_OK, "submit");
        ws.push_back(w);
    }
    std::thread stopper([&] { s.core->request_stop(); });
    stopper.join();
    uint64_t t = 0;
    CHECK(s.submit(0, 0.0, 16, 4, 1, &t) == VNE_EBUSY, "submission accepted after stop");
    std::thread pollers([&] {
        for (const Want &w : ws) {
            vne_query_result r{};
            std::vector<double> quad(256);
            CHECK(s.core->poll(w.ticket, -1, &r, quad.data(), 256) == VNE_OK, "poll");
            check_result(w, r, quad, 256);
        }
    });
    pollers.join();
    s.worker.join();
    CHECK(s.core->unfinished().empty(), "queries left unfinished");
    vne_server_info info{};
    s.core->stats(&info);
    CHECK(info.queries_done == 60 && info.arena_in_use == 0, "stop did not drain the server");
    for (int v : s.ex.in_use) CHECK(v == 0, "graph still in use");
    std::printf("stop with 60 queries in flight: all completed, later submission refused\n");
}

// A device failure ends every open query with VNE_EDEVICE; the server stays
// stoppable.
static void device_failure() {
    Setup s(4, 16ull << 20, 256, false, 9);
    std::vector<uint64_t> ts;
    for (int i = 0; i < 20; ++i) {
        uint64_t t = 0;
        CHECK(s.submit(i % 4, 0.0, 32, 12, 300 + i, &t) == VNE_OK, "submit");
        ts.push_back(t);
    }
    int failed = 0;
    for (uint64_t t : ts) {
        vne_query_result r{};
        CHECK(s.core->poll(t, -1, &r, nullptr, 0) == VNE_OK, "poll");
        CHECK(r.status == VNE_OK || r.status == VNE_EDEVICE, "status %d", r.status);
        if (r.status == VNE_EDEVICE) {
            failed++;
            CHECK(std::strstr(r.message, "injected") != nullptr, "message '%s'", r.message);
        }
    }
    CHECK(failed > 0, "the injected failure ended no query");
    s.finish();
    for (int v : s.ex.in_use) CHECK(v == 0, "graph still in use");
    std::printf("device failure: %d of 20 queries ended with VNE_EDEVICE\n", failed);
}

int main() {
    mixed_clients(false, 2);
    mixed_clients(true, 2);
    mixed_clients(false, 4);
    mixed_clients(true, 4);
    group_slots(9, 4, 8, 0);   // two groups of four
    group_slots(8, 4, 6, 1);   // seven free entries: four, two, one, then one
    group_slots(9, 2, 8, 4);   // four pairs
    group_slots(9, 1, 0, 0);   // no groups
    // an arena of 80000 bytes: with the one-column task running (15360),
    // a group of four (four query blocks of 1024 and a 64-column task of
    // 92416) does not fit, a pair (2 x 1024 + 48384) does: four pairs
    group_slots(9, 4, 8, 4, 80000);
    fcfs_order();
    numeric_stage();
    stop_in_flight();
    device_failure();
    if (g_fail) {
        std::printf("%d check(s) failed\n", g_fail.load());
        return 1;
    }
    std::printf("serve core ok\n");
    return 0;
}
