// Context internals shared by the runtime and the serving loop (host code
// of libvne; not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace vne {
namespace rt {

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct Plan {
    bool fp64 = false;
    int G = 1;                       // graphs in the set
    int m = 0, m_pad = 0, mt = 0, k = 0;
    bool store = false;              // keep every v_j (Hutch++ sketch)
    DevBuf P[2], V[2], Vstore;
    DevBuf alpha, beta, st_alpha, st_inv, st_coup, k_eff, norm2, mean, psi, estimate, flags;
    DevBuf partials, level2, probe_part, seg_acc, long_part, colors, dense;
    DevBuf graph_k, graph_m, seeds;  // per graph
    std::vector<int32_t> h_graph_k, h_graph_m;
    // Hutch++ extras (only in the quadratic-form plan of a Hutch++ run)
    DevBuf S, B, gram_part, gram, rinv, rot;
    // the k-step loop captured as one HIP graph, per (schedule, tile); with
    // kernel timing on the steps are launched directly with an event pair
    // around each step's Lanczos kernels (measured: 0.75 ms per large
    // estimate over the captured loop, against 2.8 ms for one graph per step
    // part with the events between graph launches)
    std::map<std::pair<int, int>, hipGraphExec_t> exec;
    std::vector<hipEvent_t> ev;      // 2k events
    // per-column stopping (allocated on first use): tolerances, recorded stop
    // steps, the bracket of the last check, per-check-step kernel arguments,
    // the running-column count and its pinned host copy; the step loop is
    // captured chunk by chunk (steps up to one check), keyed by (schedule,
    // tile, first step of the chunk)
    DevBuf col_tol, col_stop, bound_lo, bound_hi, adapt_args, remaining;
    int32_t *h_remaining = nullptr;
    std::vector<char> h_adapt;
    std::map<std::tuple<int, int, int>, hipGraphExec_t> chunk_exec;
    // the k-step loop of each concurrent tile chain, per (schedule, tile,
    // chains, chain)
    std::map<std::tuple<int, int, int, int>, hipGraphExec_t> chain_exec;
    int steps_run = 0;               // steps the block ran in the last run
    // values last uploaded to graph_k / graph_m / seeds (skipped when equal)
    std::vector<int32_t> up_graph_k, up_graph_m;
    std::vector<uint64_t> up_seeds;
    void *h_stage = nullptr;         // pinned staging of copy_out
    size_t h_stage_bytes = 0;
};

struct Graph {
    int64_t n = 0, nnz = 0;
    double scale = 1.0;
    std::vector<int32_t> h_row_ptr, h_col;   // host copies (schedules, stacking)
    std::vector<double> h_val;
    std::vector<int64_t> h_keys;
    DevBuf row_ptr, col;                     // owned device copies (host input)
    const int32_t *d_row_ptr = nullptr, *d_col = nullptr;
    Schedule sched;
    bool alive = false;
    bool zero_rowsum = false;                // A 1 = 0 exactly
    // spectral facts of A = scale * CSR for the serving error rule
    double lambda_ub = 0.0;                  // max_i sum_j |A_ij| >= lambda_max (Gershgorin)
    double fro2 = 0.0;                       // ||A||_F^2 = tr(A^2) for symmetric A
    double trace = 0.0;
    int in_use = 0;                          // queries of a running server on this graph
};

// Graphs stacked as one block-diagonal matrix: rows, entries, work blocks and
// probe blocks of graph q follow those of graphs 0..q-1.  A set of one graph
// uses the graph's own row_ptr / col_idx.
struct GraphSet {
    std::vector<int32_t> ids;
    int G = 1;
    int64_t n = 0, nnz = 0;
    double scale = 1.0;
    bool zero_rowsum = true;
    const int32_t *d_row_ptr = nullptr, *d_col = nullptr;
    DevBuf row_ptr, col, val32, val64, keys;
    DevBuf row_graph, long_graph, block_graph, graph_block_begin, graph_long_begin, graph_scale;
    DevBuf segs, block_ranges, long_first, long_nseg;
    DevBuf probe_rows, probe_block_graph, probe_graph_begin, graph_row_begin;
    Schedule sched;
    std::vector<int64_t> h_row_begin;                      // [G+1]
    int probe_blocks = 0;
    uint64_t last_use = 0;
    std::map<std::tuple<int, int, int, int, int>, std::unique_ptr<Plan>> plans;
};

}  // namespace rt
}  // namespace vne

struct vne_ctx {
    using Graph = vne::rt::Graph;
    using GraphSet = vne::rt::GraphSet;
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;    // used when the caller gives no stream
    uint64_t budget = 0, used = 0;
    std::string err;
    std::vector<std::unique_ptr<Graph>> graphs;
    std::map<std::vector<int32_t>, std::unique_ptr<GraphSet>> sets;
    uint64_t tick = 0;                   // set use counter (eviction order)
    bool timing = false;
    int64_t t_launches = 0;
    double t_ms = 0.0, t_bytes = 0.0;
    struct Pending {
        void *plan;
        double bytes;
        int steps;                       // step launches with recorded events
        bool loop = false;               // one event pair around the whole loop (tile chains)
    };
    std::vector<Pending> pending;        // timed step loops not yet collected
    std::map<std::string, int> tuned;    // autotuner: set signature -> column tile
    int32_t last_tile = 0, last_m_pad = 0;   // column tile and padded width of the last run
    std::string tune_file;
    // concurrent tile chains: their streams (default priority) and the
    // fork / join events, created on first use
    std::vector<hipStream_t> chain_streams;
    std::vector<hipEvent_t> chain_events;
    // serialises the registry (register, release, estimates) against the
    // worker thread of a server running on this context
    std::recursive_mutex mu;
};

namespace vne {
namespace rt {

#define HIP_TRY(ctx, expr)                                           \
    do {                                                             \
        hipError_t _e = (expr);                                      \
        if (_e != hipSuccess) return hip_fail((ctx), _e, #expr);     \
    } while (0)

#define VNE_TRY(expr)                       \
    do {                                    \
        vne_status _s = (expr);             \
        if (_s != VNE_OK) return _s;        \
    } while (0)

vne_status fail(vne_ctx *c, vne_status st, const std::string &m);
vne_status hip_fail(vne_ctx *c, hipError_t e, const char *what);
vne_status dev_alloc(vne_ctx *c, DevBuf *b, size_t bytes);
void dev_free(vne_ctx *c, DevBuf *b);
int env_int(const char *name, int dflt);
Graph *get_graph(vne_ctx *c, int32_t gid);
// the device arrays of one graph (a set of one), built on first use
vne_status get_set(vne_ctx *c, const std::vector<int32_t> &ids, GraphSet **out);
// buffers of an m-column, k-step problem on a set (cached per shape and tag)
vne_status get_plan(vne_ctx *c, GraphSet *set, int m, int k, bool fp64, bool store, int tag, Plan **out);
// tile and padded width of a plan (no buffers), and the list of its device
// buffers with their sizes in a fixed order
vne_status plan_shape(vne_ctx *c, const GraphSet *set, Plan *p, int m, int k, bool fp64, bool store);
void plan_buffers(const GraphSet *set, Plan *p, const std::function<void(DevBuf *, size_t)> &take);
void free_graph(vne_ctx *c, Graph *g);
// device address of the allocation-free estimate's static scratch array on
// `device` (the current device), resolved once per device
vne_status noalloc_attach(int device, std::string *err);

// Probe description for run_lanczos.
struct ProbeSpec {
    int gen = GEN_RADEMACHER;
    std::vector<uint64_t> seeds;       // per graph (Rademacher)
    int col_offset = 0;
    const int32_t *colors = nullptr;   // device, stacked rows
    const void *dense = nullptr;       // device, stacked rows
    int ld_dense = 0;
};

struct RunOpts {
    bool collect = true;               // record kernel timing for this run
    int steps = -1;                    // autotuner: only this many steps, no graph, no quadrature
    bool graph_trial = false;          // autotuner: the whole loop as the run would launch it (captured
                                       // graphs kept for later runs), no quadrature
    int tile = 0;                      // column tile (0: the plan's)
    // per-column a-posteriori stopping (one graph): the Theorem 4.8 upper
    // bound on [lam_lo, lam_hi] (n_grid points) is checked after steps 3, 5,
    // 7, ...; a column stops at the first check within p->col_tol[c], the
    // block when every column has stopped
    bool adaptive = false;
    double lam_lo = 0.0, lam_hi = 0.0;
    int n_grid = kBoundGrid;
    bool estimate = false;             // stop on the eq. (4.10) estimate instead of the upper bound
    bool direct = false;               // launch every step directly (no captured graph)
};

// Probe block, Lanczos steps, quadrature; leaves psi, coefficients, k_eff and
// norm2 in the plan (and col_stop, steps_run when adaptive).
vne_status run_lanczos(vne_ctx *c, GraphSet *set, Plan *p, const ProbeSpec &ps, bool desing,
                       const RunOpts &opt = RunOpts());
// column tile of the plan (timed choice, cached per set shape)
vne_status autotune(vne_ctx *c, GraphSet *set, Plan *p, const ProbeSpec &ps, bool desing);
vne_status check_flags(vne_ctx *c, int32_t fl);
// probe spec of a set's queries; colours / dense host blocks go to the plan
vne_status make_probe_spec(vne_ctx *c, GraphSet *set, Plan *p, const vne_probes *pr, int m_max, bool fp64,
                           ProbeSpec *ps, int *combine_kind);
vne_status collect_timing(vne_ctx *c);
// Hutch++ (eq. (3.9)) on one graph: sketch Omega = Rademacher hash columns
// [0, nr) of `seed`, nh Hutchinson vectors on hash columns [g_col0,
// g_col0 + nh).  Leaves the forms of [Q | G~] in (*q_out)->psi and their
// combination in (*q_out)->estimate on the context's stream (nothing is
// copied to the host); *sk_out (may be NULL) receives the sketch's plan
// (NULL with q_src).  q_src (device, may be NULL): the orthonormal Q of an
// earlier run of the same sketch (n x nr, leading dimension q_ld), used
// instead of sketching again.
vne_status hutchpp_run(vne_ctx *c, GraphSet *set, int nr, int nh, int g_col0, int k, uint64_t seed, bool fp64,
                       bool desing, Plan **sk_out, Plan **q_out, const void *q_src = nullptr, int q_ld = 0);
vne_status check_mode(vne_ctx *c, uint32_t mode);

}  // namespace rt
}  // namespace vne
