// Scheduling core of the serving loop, free of device code: tickets, the
// queue of slot tasks, admission into mailbox entries and arena space,
// continuous batching one step per tick, the pilot / planning stages of a
// relative-accuracy query and completion.  Everything that touches the
// device (slot state, probe blocks, the step launches, quadrature, copies
// to the host) goes through a ServeExec; the library's executor drives the
// GPU, and tests drive the same core with a host-only executor and clock.
//
// Threads: one worker runs run(); submit, poll, stats and request_stop may
// be called from any thread.  Worker-owned state (pending and active tasks,
// arena, mailbox entries) is touched by the worker only; the ticket table,
// the incoming list and the published statistics are guarded by the core's
// mutex.
#pragma once

#include <condition_variable>
#include <cstdint>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "serve_host.h"
#include "vne.h"

namespace vne {

// One query's share of a slot: its columns, stopping rule and mailbox entry.
struct ServeMember {
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

constexpr int kMaxMembers = 4;       // tasks of a group slot at most

// A slot: one task of a query, or a group of two or four 16-column FP32
// tasks of queries on the same graph with the same step cap and stopping
// mode (a group slot, m_pad = 16 * n_mem, mt = 16).  Its state lives in the
// arena at [off, off + bytes).
struct ServeTask {
    int m = 0, m_pad = 0, mt = 0, k = 0;
    int j = 0;                       // steps done
    uint64_t off = 0, bytes = 0;
    int n_mem = 1;
    ServeMember mem[kMaxMembers];
    bool group() const { return n_mem > 1; }
};

struct ServeQuery {
    uint64_t ticket = 0;
    vne_query q{};
    // facts of the query's graph for the error rule: rows, Gershgorin bound
    // of lambda_max, ||A||_F^2 and tr(A)
    int64_t n = 0;
    double lambda_ub = 0.0, fro2 = 0.0, trace = 0.0;
    int N = 0, k = 0;                // planned probes and steps
    int cols_issued = 0, tasks_open = 0;
    bool planned = false, started = false;
    bool stage_wait = false, final_wait = false, done = false;
    double s_lower = 0.0, bound = 0.0;
    int steps_used = 0;              // largest step count a task of the query used
    int rounds = 0;                  // probe-count plans made (rel_eps > 0)
    uint64_t off = 0;                // the query's arena block (forms, estimate, flags)
    double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;   // ms on the core's clock
    vne_query_result res{};
    std::vector<double> quad;
    void *x = nullptr;               // the executor's state of the query
};

class ServeExec {
public:
    virtual ~ServeExec() = default;
    // once, on the worker thread, before anything else
    virtual void thread_init() {}
    // arena bytes of a task of width m_pad and k steps on the query's graph
    virtual uint64_t task_bytes(const ServeQuery &q, int m_pad, int k) = 0;
    // column tile and padded width of a task of m columns
    virtual void tile(int m, int *mt, int *m_pad) = 0;
    // the query's first task is being admitted and its arena block is at
    // q.off: result buffers and the cleared flags
    virtual vne_status open_query(ServeQuery &q) = 0;
    // slot state at t.off (members' uids and mailbox entries assigned):
    // probe blocks of the members (qm[i]: the query of member i), cleared
    // stop records
    virtual vne_status start_task(ServeTask &t, ServeQuery *const *qm) = 0;
    // one Lanczos step of every active slot (qs[kMaxMembers i + mi]: the
    // query of member mi of slot i, null for a member that has ended: its
    // query may be gone), with the a-posteriori checks of adaptive members
    virtual vne_status tick(const std::vector<ServeTask> &active, const std::vector<ServeQuery *> &qs) = 0;
    // the stop record of a mailbox entry as the host sees it now
    virtual void stop_record(int slot, int32_t *uid, int32_t *step) = 0;
    // the quadrature of member i after `steps` steps into the query's forms
    virtual vne_status quadrature(const ServeTask &t, int i, ServeQuery &q, int steps) = 0;
    // forms [0, q.cols_issued) and the flags of a finished stage to the host
    virtual vne_status issue_stage(ServeQuery &q) = 0;
    // estimator combine over forms [0, q.N), then forms, estimate and flags to the host
    virtual vne_status issue_final(ServeQuery &q) = 0;
    // whether the query's last issued copy has reached the host (block: wait for it)
    virtual vne_status ready(ServeQuery &q, bool block, bool *done) = 0;
    // host copies of the forms, the estimate (final) and the flags of the last copy
    virtual const double *forms(ServeQuery &q) = 0;
    virtual double estimate(ServeQuery &q) = 0;
    virtual int32_t flags(ServeQuery &q, bool final) = 0;
    // after the final copy: the most steps a quadrature of the query took on
    // the device (0: not known)
    virtual int32_t steps_taken(ServeQuery &q) = 0;
    // the query ended: its executor state back
    virtual void close_query(ServeQuery &q) = 0;
    // the query no longer uses its graph
    virtual void release_graph(ServeQuery &q) = 0;
    // text of the last failure of a call that returned an error
    virtual std::string error_text() = 0;
};

struct ServeConfig {
    int max_slots = 64, max_cols = 256, pilot_probes = 16, psi_cap = 4096, max_steps = 100;
    double z = 2.576;
    bool fp64 = false;
    uint64_t arena_bytes = 0;
    uint64_t query_bytes = 0;        // arena block of a query's forms, estimate and flags
    // admission: a task that does not fit may let later tasks that do fit
    // start before it (false: first come, first served)
    bool skip_blocked = false;
    // largest group slot of 16-column FP32 tasks of one graph: 1 (none), 2
    // or 4
    int max_group = 2;
};

class ServeCore {
public:
    using ClockMs = std::function<double()>;
    ServeCore(const ServeConfig &cfg, ServeExec *exec, ClockMs clock = ClockMs());

    // the worker's loop; returns once stop was requested and no work is left
    void run();
    // queues a query whose graph facts are filled in; VNE_EBUSY once stop began
    vne_status submit(std::unique_ptr<ServeQuery> q, uint64_t *ticket);
    vne_status poll(uint64_t ticket, int32_t timeout_ms, vne_query_result *res, double *quad, int32_t quad_cap);
    void stats(vne_server_info *st);
    bool stopping();
    void request_stop();
    // after the worker ended: queries that never finished (for their graphs)
    std::vector<ServeQuery *> unfinished();

    const ServeConfig &config() const { return cfg_; }
    double now() const { return clock_(); }

private:
    void add_tasks(ServeQuery &q, int c0, int c1, bool pilot);
    void start_query(ServeQuery &q);
    void finish_query(ServeQuery &q, vne_status st, const std::string &msg);
    void fail_query(ServeQuery &q, vne_status st, const std::string &msg);
    ServeQuery *query_of(uint64_t ticket);
    vne_status end_member(ServeTask &t, int i, ServeQuery &q, int steps);
    vne_status poll_events(bool block_one);
    bool open_query(ServeQuery &q, vne_status *st);
    bool groupable(const ServeTask &t) const;
    vne_status admit();
    vne_status tick();
    bool has_waits();
    void publish();
    void fail_all(const std::string &msg);

    ServeConfig cfg_;
    ServeExec *exec_;
    ClockMs clock_;

    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    bool stopping_ = false, broken_ = false;
    std::string broken_msg_;
    uint64_t next_ticket_ = 1;
    std::deque<uint64_t> incoming_;                 // submitted, not yet split into tasks
    std::map<uint64_t, std::unique_ptr<ServeQuery>> queries_;
    int64_t queries_done_ = 0;
    vne_server_info snap_{};

    // worker-owned
    Arena arena_;
    uint64_t arena_peak_ = 0;
    std::deque<ServeTask> pending_;                  // in ticket order
    std::vector<ServeTask> active_;
    std::vector<int> free_slots_;
    int32_t next_uid_ = 1;
    int64_t ticks_ = 0, tasks_admitted_ = 0, pair_slots_ = 0, group_tasks_ = 0;
    double occupancy_sum_ = 0.0;
};

}  // namespace vne
