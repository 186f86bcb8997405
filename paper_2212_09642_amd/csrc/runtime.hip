// Host runtime of the entropy engine: context, graph registry, cached
// workspaces ("plans") and the estimate entry points of vne.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"
#include "kernels.h"

using namespace vne;

namespace {

std::string g_create_error;

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct Plan {
    bool fp64 = false;
    int m = 0, m_pad = 0, mt = 0, n_tiles = 0, k = 0;
    bool store = false;              // keep every v_j (Hutch++ sketch)
    int probe_blocks = 0;
    DevBuf P[2], V[2], Vstore;
    DevBuf alpha, beta, st_alpha, st_inv, st_coup, k_eff, norm2, mean, psi, estimate, flags;
    DevBuf partials, level2, probe_part, seg_acc, long_part, colors, dense;
    // Hutch++ extras (only in the quadratic-form plan of a Hutch++ run)
    DevBuf S, B, gram_part, gram, rinv, rot;
    // the k-step loop captured as one HIP graph, per two_pass schedule;
    // with kernel timing on, one graph per step part instead, so that event
    // pairs recorded between graph launches bracket the Lanczos step kernels
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    std::vector<hipGraphExec_t> part_exec[2];   // [2k]: step j, finalize j
    std::vector<hipEvent_t> ev;                 // 2k events
};

struct Graph {
    int64_t n = 0, nnz = 0;
    double scale = 1.0;
    DevBuf row_ptr, col, val32, val64, keys;         // owned copies
    const int32_t *d_row_ptr = nullptr, *d_col = nullptr;
    const float *d_val32 = nullptr;
    const double *d_val64 = nullptr;
    const int64_t *d_keys = nullptr;
    Schedule sched;
    DevBuf segs, block_begin, long_first, long_nseg;
    std::map<std::tuple<int, int, int, int, int>, std::unique_ptr<Plan>> plans;
    bool alive = false;
    bool zero_rowsum = false;            // A 1 = 0 exactly (checked at registration)
    double local_frac = 0.0;             // off-diagonal entries with |i - j| <= 256
};

}  // namespace

struct vne_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;    // used when the caller gives no stream
    uint64_t budget = 0, used = 0;
    std::string err;
    std::vector<std::unique_ptr<Graph>> graphs;
    bool timing = false;
    int64_t t_launches = 0;
    double t_ms = 0.0, t_bytes = 0.0;
    struct Pending {
        void *plan;
        double bytes;
    };
    std::vector<Pending> pending;        // timed step loops not yet collected
};

namespace {

vne_status fail(vne_ctx *c, vne_status st, const std::string &m) {
    c->err = m;
    return st;
}

vne_status hip_fail(vne_ctx *c, hipError_t e, const char *what) {
    c->err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? VNE_ENOMEM : VNE_EDEVICE;
}

#define HIP_TRY(ctx, expr)                                           \
    do {                                                             \
        hipError_t _e = (expr);                                      \
        if (_e != hipSuccess) return hip_fail((ctx), _e, #expr);     \
    } while (0)

vne_status dev_alloc(vne_ctx *c, DevBuf *b, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (c->budget && c->used + bytes > c->budget)
        return fail(c, VNE_ENOMEM, "HBM budget exceeded: need " + std::to_string(bytes) + " more bytes, " +
                                       std::to_string(c->budget - c->used) + " left");
    hipError_t e = hipMalloc(&b->p, bytes);
    if (e != hipSuccess) {
        b->p = nullptr;
        return hip_fail(c, e, "hipMalloc");
    }
    b->bytes = bytes;
    c->used += bytes;
    return VNE_OK;
}

void dev_free(vne_ctx *c, DevBuf *b) {
    if (b->p) {
        (void)hipFree(b->p);
        c->used -= b->bytes;
    }
    b->p = nullptr;
    b->bytes = 0;
}

void free_plan(vne_ctx *c, Plan *p) {
    for (auto &e : p->exec)
        if (e) {
            (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
    for (auto &v : p->part_exec) {
        for (auto &e : v)
            if (e) (void)hipGraphExecDestroy(e);
        v.clear();
    }
    for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
    p->ev.clear();
    DevBuf *all[] = {&p->P[0], &p->P[1], &p->V[0], &p->V[1], &p->Vstore, &p->alpha, &p->beta,
                     &p->st_alpha, &p->st_inv, &p->st_coup, &p->k_eff, &p->norm2, &p->mean, &p->psi,
                     &p->estimate, &p->flags, &p->partials, &p->level2, &p->probe_part, &p->seg_acc,
                     &p->long_part, &p->colors, &p->dense, &p->S, &p->B, &p->gram_part, &p->gram,
                     &p->rinv, &p->rot};
    for (DevBuf *b : all) dev_free(c, b);
}

void free_graph(vne_ctx *c, Graph *g) {
    for (auto &kv : g->plans) free_plan(c, kv.second.get());
    g->plans.clear();
    DevBuf *all[] = {&g->row_ptr, &g->col, &g->val32, &g->val64, &g->keys,
                     &g->segs, &g->block_begin, &g->long_first, &g->long_nseg};
    for (DevBuf *b : all) dev_free(c, b);
    g->alive = false;
}

// Allocates max(count, 1) elements and copies count elements (none if h is NULL).
template <typename T>
vne_status upload(vne_ctx *c, DevBuf *b, const T *h, size_t count) {
    vne_status st = dev_alloc(c, b, std::max<size_t>(count, 1) * sizeof(T));
    if (st != VNE_OK) return st;
    if (count && h) HIP_TRY(c, hipMemcpy(b->p, h, count * sizeof(T), hipMemcpyHostToDevice));
    return VNE_OK;
}

Graph *get_graph(vne_ctx *c, int32_t gid) {
    if (gid < 0 || gid >= (int32_t)c->graphs.size() || !c->graphs[gid] || !c->graphs[gid]->alive) return nullptr;
    return c->graphs[gid].get();
}

int env_int(const char *name, int dflt) {
    const char *v = getenv(name);
    return v ? atoi(v) : dflt;
}

// Workspace for a probe block of width m on graph g.
vne_status get_plan(vne_ctx *c, Graph *g, int m, int k, bool fp64, bool store, int tag, Plan **out) {
    auto key = std::make_tuple(m, k, (int)fp64, (int)store, tag);
    auto it = g->plans.find(key);
    if (it != g->plans.end()) {
        *out = it->second.get();
        return VNE_OK;
    }
    auto p = std::make_unique<Plan>();
    p->fp64 = fp64;
    p->m = m;
    p->k = k;
    p->store = store;
    p->mt = choose_tile(m, fp64, env_int("VNE_TILE", 0));
    p->m_pad = pad_columns(m, p->mt);
    p->n_tiles = p->m_pad / p->mt;
    const size_t es = fp64 ? 8 : 4;
    const size_t blk = (size_t)g->n * p->m_pad * es;
    const Schedule &s = g->sched;
    vne_status st = VNE_OK;
    auto A = [&](DevBuf *b, size_t bytes) {
        if (st == VNE_OK) st = dev_alloc(c, b, bytes);
    };
    A(&p->P[0], blk);
    A(&p->P[1], blk);
    if (store) {
        A(&p->Vstore, blk * (size_t)k);
    } else {
        A(&p->V[0], blk);
        A(&p->V[1], blk);
    }
    const size_t cols = (size_t)p->m_pad;
    A(&p->alpha, cols * k * 8);
    A(&p->beta, cols * k * 8);
    A(&p->st_alpha, cols * 8);
    A(&p->st_inv, cols * 8);
    A(&p->st_coup, cols * 8);
    A(&p->k_eff, cols * 4);
    A(&p->norm2, cols * 8);
    A(&p->mean, cols * 8);
    A(&p->psi, cols * 8);
    A(&p->estimate, 8);
    A(&p->flags, 4);
    A(&p->partials, (size_t)s.n_blocks() * 3 * cols * 8);
    A(&p->level2, (size_t)kLevel2 * 3 * cols * 8);
    p->probe_blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (g->n + 255) / 256));
    A(&p->probe_part, (size_t)p->probe_blocks * cols * 8);
    A(&p->seg_acc, (size_t)std::max(1, s.n_seg) * cols * 8);
    A(&p->long_part, (size_t)std::max(1, s.n_long) * 3 * cols * 8);
    if (st != VNE_OK) {
        free_plan(c, p.get());
        return st;
    }
    HIP_TRY(c, hipMemsetAsync(p->long_part.p, 0, p->long_part.bytes, c->stream));
    *out = p.get();
    g->plans[key] = std::move(p);
    return VNE_OK;
}

vne_status collect_timing(vne_ctx *c) {
    for (auto &pd : c->pending) {
        Plan *p = (Plan *)pd.plan;
        for (int j = 0; j < p->k; ++j) {
            float ms = 0.f;
            HIP_TRY(c, hipEventElapsedTime(&ms, p->ev[2 * j], p->ev[2 * j + 1]));
            c->t_ms += ms;
            c->t_bytes += pd.bytes;
            c->t_launches++;
        }
    }
    c->pending.clear();
    return VNE_OK;
}

struct ProbeSpec {
    int gen = GEN_RADEMACHER;
    uint64_t seed = 0;
    int col_offset = 0;
    const int32_t *colors = nullptr;   // device
    const void *dense = nullptr;       // device
    int ld_dense = 0;
};

// Probe block, k Lanczos steps, quadrature.  Leaves psi, coefficients,
// k_eff and norm2 in the plan.
vne_status run_lanczos(vne_ctx *c, Graph *g, Plan *p, const ProbeSpec &ps, bool desing) {
    const Schedule &s = g->sched;
    HIP_TRY(c, hipMemsetAsync(p->flags.p, 0, 4, c->stream));
    ProbeArgs pa{};
    pa.gen = ps.gen;
    pa.n = (int32_t)g->n;
    pa.m = p->m;
    pa.m_pad = p->m_pad;
    pa.mt = p->mt;
    pa.col_offset = ps.col_offset;
    pa.seed = ps.seed;
    pa.keys = g->d_keys;
    pa.colors = ps.colors;
    pa.dense = ps.dense;
    pa.ld_dense = ps.ld_dense;
    pa.desing = desing ? 1 : 0;
    pa.P_out = p->P[0].p;
    pa.partials = (double *)p->probe_part.p;
    pa.n_blocks = p->probe_blocks;
    pa.mean = (double *)p->mean.p;
    pa.norm2 = (double *)p->norm2.p;
    pa.st_alpha = (double *)p->st_alpha.p;
    pa.st_inv = (double *)p->st_inv.p;
    pa.st_coup = (double *)p->st_coup.p;
    pa.k_eff = (int32_t *)p->k_eff.p;
    pa.k = p->k;
    HIP_TRY(c, launch_probe(pa, p->fp64, c->stream));

    const size_t es = p->fp64 ? 8 : 4;
    const size_t blk_elems = (size_t)g->n * p->m_pad;
    const double bytes = 4.0 * (g->n + 1) + (double)g->nnz * (4.0 + es) + 3.0 * g->n * p->m * es;
    StepArgs a{};
    a.row_ptr = g->d_row_ptr;
    a.col = g->d_col;
    a.val = p->fp64 ? (const void *)g->d_val64 : (const void *)g->d_val32;
    a.scale = g->scale;
    a.n = (int32_t)g->n;
    a.m_pad = p->m_pad;
    a.mt = p->mt;
    a.n_tiles = p->n_tiles;
    a.st_alpha = (const double *)p->st_alpha.p;
    a.st_inv = (const double *)p->st_inv.p;
    a.st_coup = (const double *)p->st_coup.p;
    a.segs = (const SegItem *)g->segs.p;
    a.n_seg = s.n_seg;
    a.seg_len = s.seg_len;
    a.block_begin = (const int32_t *)g->block_begin.p;
    a.n_blocks = s.n_blocks();
    a.seg_acc = (double *)p->seg_acc.p;
    a.n_long = s.n_long;
    // schedule: normalize pass + single-stream SpMM by default (measured
    // faster on both random and ring-local graphs); the lazy one-pass
    // schedule (4 streams, two of them gathered) stays selectable
    {
        const int forced = env_int("VNE_SCHED", -1);
        a.two_pass = forced >= 0 ? forced : 1;
    }
    a.long_first = (const int32_t *)g->long_first.p;
    a.long_nseg = (const int32_t *)g->long_nseg.p;
    a.long_part = (double *)p->long_part.p;
    a.partials = (double *)p->partials.p;

    FinalizeArgs f{};
    f.partials = (const double *)p->partials.p;
    f.long_part = (const double *)p->long_part.p;
    f.level2 = (double *)p->level2.p;
    f.n_level2 = kLevel2;
    f.n_blocks = s.n_blocks();
    f.n_long = s.n_long;
    f.mt = p->mt;
    f.m_pad = p->m_pad;
    f.m = p->m;
    f.k = p->k;
    f.tau = p->fp64 ? std::ldexp(1.0, -23) : std::ldexp(1.0, -18);
    f.st_alpha = (double *)p->st_alpha.p;
    f.st_inv = (double *)p->st_inv.p;
    f.st_coup = (double *)p->st_coup.p;
    f.alpha = (double *)p->alpha.p;
    f.beta = (double *)p->beta.p;
    f.k_eff = (int32_t *)p->k_eff.p;
    f.flags = (int32_t *)p->flags.p;

    const bool use_graph = env_int("VNE_GRAPH", 1) != 0;
    const bool timing = c->timing;
    // part 0: the step kernels of step j; part 1: its reduction and finalize
    auto issue = [&](int j, int part) -> vne_status {
        char *Pb[2] = {(char *)p->P[0].p, (char *)p->P[1].p};
        a.P_in = Pb[(j - 1) & 1];
        a.P_out = Pb[j & 1];
        if (p->store) {
            char *base = (char *)p->Vstore.p;
            a.V_out = base + (size_t)(j - 1) * blk_elems * es;
            a.V_prev = j >= 2 ? base + (size_t)(j - 2) * blk_elems * es : nullptr;
        } else {
            a.V_out = p->V[(j - 1) & 1].p;
            a.V_prev = p->V[j & 1].p;
        }
        a.V_cur = a.V_out;
        if (part == 0) {
            HIP_TRY(c, launch_step(a, p->fp64, j == 1, c->stream));
        } else {
            f.step = j;
            HIP_TRY(c, launch_finalize(f, c->stream));
        }
        return VNE_OK;
    };
    auto capture = [&](hipGraphExec_t *ex, int j0, int j1, int part_only) -> vne_status {
        hipGraph_t graph = nullptr;
        HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
        vne_status st = VNE_OK;
        for (int j = j0; j <= j1 && st == VNE_OK; ++j)
            for (int part = 0; part < 2 && st == VNE_OK; ++part)
                if (part_only < 0 || part == part_only) st = issue(j, part);
        hipError_t e_end = hipStreamEndCapture(c->stream, &graph);
        if (st != VNE_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e_end != hipSuccess) return hip_fail(c, e_end, "hipStreamEndCapture");
        hipError_t e_inst = hipGraphInstantiate(ex, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e_inst != hipSuccess) {
            *ex = nullptr;
            return hip_fail(c, e_inst, "hipGraphInstantiate");
        }
        return VNE_OK;
    };
    if (timing && p->ev.size() < (size_t)(2 * p->k)) {
        while (p->ev.size() < (size_t)(2 * p->k)) {
            hipEvent_t e;
            HIP_TRY(c, hipEventCreate(&e));
            p->ev.push_back(e);
        }
    }
    const int sched = a.two_pass ? 1 : 0;
    vne_status st = VNE_OK;
    if (use_graph && !timing) {
        hipGraphExec_t &ex = p->exec[sched];
        if (!ex && (st = capture(&ex, 1, p->k, -1)) != VNE_OK) return st;
        HIP_TRY(c, hipGraphLaunch(ex, c->stream));
    } else if (use_graph) {
        auto &parts = p->part_exec[sched];
        if (parts.empty()) {
            parts.assign(2 * p->k, nullptr);
            for (int j = 1; j <= p->k; ++j)
                for (int part = 0; part < 2; ++part)
                    if ((st = capture(&parts[2 * (j - 1) + part], j, j, part)) != VNE_OK) return st;
        }
        for (int j = 1; j <= p->k; ++j) {
            HIP_TRY(c, hipEventRecord(p->ev[2 * (j - 1)], c->stream));
            HIP_TRY(c, hipGraphLaunch(parts[2 * (j - 1)], c->stream));
            HIP_TRY(c, hipEventRecord(p->ev[2 * (j - 1) + 1], c->stream));
            HIP_TRY(c, hipGraphLaunch(parts[2 * (j - 1) + 1], c->stream));
        }
    } else {
        for (int j = 1; j <= p->k; ++j) {
            if (timing) HIP_TRY(c, hipEventRecord(p->ev[2 * (j - 1)], c->stream));
            if ((st = issue(j, 0)) != VNE_OK) return st;
            if (timing) HIP_TRY(c, hipEventRecord(p->ev[2 * (j - 1) + 1], c->stream));
            if ((st = issue(j, 1)) != VNE_OK) return st;
        }
    }
    if (timing) {
        c->pending.push_back({p, bytes});
    }
    HIP_TRY(c, launch_quadrature((const double *)p->alpha.p, (const double *)p->beta.p,
                                 (const int32_t *)p->k_eff.p, (const double *)p->norm2.p, p->k, p->m,
                                 (double *)p->psi.p, (int32_t *)p->flags.p, c->stream));
    return VNE_OK;
}

vne_status copy_out(vne_ctx *c, Plan *p, vne_result *out, int32_t *flags_h) {
    const int m = p->m, k = p->k;
    hipStream_t s = c->stream;
    HIP_TRY(c, hipMemcpyAsync(&out->estimate, p->estimate.p, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(flags_h, p->flags.p, 4, hipMemcpyDeviceToHost, s));
    if (out->quad) HIP_TRY(c, hipMemcpyAsync(out->quad, p->psi.p, (size_t)m * 8, hipMemcpyDeviceToHost, s));
    if (out->alpha)
        HIP_TRY(c, hipMemcpyAsync(out->alpha, p->alpha.p, (size_t)m * k * 8, hipMemcpyDeviceToHost, s));
    if (out->beta) HIP_TRY(c, hipMemcpyAsync(out->beta, p->beta.p, (size_t)m * k * 8, hipMemcpyDeviceToHost, s));
    if (out->k_eff) HIP_TRY(c, hipMemcpyAsync(out->k_eff, p->k_eff.p, (size_t)m * 4, hipMemcpyDeviceToHost, s));
    if (out->norm2) HIP_TRY(c, hipMemcpyAsync(out->norm2, p->norm2.p, (size_t)m * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    return VNE_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" vne_status vne_ctx_create(int device, uint64_t hbm_budget_bytes, void *hip_stream, vne_ctx **out) {
    if (!out) {
        g_create_error = "out is NULL";
        return VNE_EINVAL;
    }
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) {
        g_create_error = std::string("no HIP device: ") + hipGetErrorString(e);
        return VNE_EDEVICE;
    }
    if (device < 0 || device >= ndev) {
        g_create_error = "device index out of range";
        return VNE_EINVAL;
    }
    e = hipSetDevice(device);
    if (e != hipSuccess) {
        g_create_error = std::string("hipSetDevice: ") + hipGetErrorString(e);
        return VNE_EDEVICE;
    }
    auto *c = new vne_ctx();
    c->device = device;
    c->budget = hbm_budget_bytes;
    // the legacy null stream cannot be captured into a graph: without a
    // caller stream the context runs on a stream of its own (blocking, so it
    // stays ordered with work on the null stream; default priority)
    e = hipStreamCreate(&c->own_stream);
    if (e != hipSuccess) {
        g_create_error = std::string("hipStreamCreate: ") + hipGetErrorString(e);
        delete c;
        return VNE_EDEVICE;
    }
    c->stream = hip_stream ? (hipStream_t)hip_stream : c->own_stream;
    *out = c;
    return VNE_OK;
}

extern "C" void vne_ctx_destroy(vne_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto &g : c->graphs)
        if (g) free_graph(c, g.get());
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    delete c;
}

extern "C" const char *vne_last_error(const vne_ctx *c) {
    return c ? c->err.c_str() : g_create_error.c_str();
}

extern "C" vne_status vne_ctx_set_stream(vne_ctx *c, void *hip_stream) {
    if (!c) return VNE_EINVAL;
    c->stream = hip_stream ? (hipStream_t)hip_stream : c->own_stream;
    return VNE_OK;
}

extern "C" vne_status vne_ctx_memory(const vne_ctx *c, uint64_t *bytes) {
    if (!c || !bytes) return VNE_EINVAL;
    *bytes = c->used;
    return VNE_OK;
}

extern "C" vne_status vne_graph_register(vne_ctx *c, const vne_csr *csr, uint32_t flags, int32_t *graph_id) {
    if (!c) return VNE_EINVAL;
    c->err.clear();
    if (!csr || !graph_id) return fail(c, VNE_EINVAL, "NULL argument");
    HIP_TRY(c, hipSetDevice(c->device));
    const int64_t n = csr->n, nnz = csr->nnz;
    if (n < 1 || nnz < 0 || nnz > INT32_MAX || n > INT32_MAX - 1) return fail(c, VNE_EINVAL, "bad sizes");
    if (csr->location != VNE_HOST && csr->location != VNE_DEVICE) return fail(c, VNE_EINVAL, "bad location");
    // host view of the three arrays (copied back for device input)
    std::vector<int32_t> h_rp, h_ci;
    std::vector<char> h_val;
    vne_csr hv = *csr;
    const size_t vs = csr->value_dtype == VNE_F64 ? 8 : 4;
    if (csr->location == VNE_DEVICE) {
        if (!csr->row_ptr || (nnz && (!csr->col_idx || !csr->values))) return fail(c, VNE_EINVAL, "NULL CSR array");
        h_rp.resize(n + 1);
        h_ci.resize(nnz);
        h_val.resize(nnz * vs);
        HIP_TRY(c, hipMemcpy(h_rp.data(), csr->row_ptr, (n + 1) * 4, hipMemcpyDeviceToHost));
        if (nnz) {
            HIP_TRY(c, hipMemcpy(h_ci.data(), csr->col_idx, nnz * 4, hipMemcpyDeviceToHost));
            HIP_TRY(c, hipMemcpy(h_val.data(), csr->values, nnz * vs, hipMemcpyDeviceToHost));
        }
        hv.row_ptr = h_rp.data();
        hv.col_idx = h_ci.data();
        hv.values = h_val.data();
        hv.location = VNE_HOST;
    }
    std::string msg;
    vne_status st = validate_host_csr(&hv, flags, &msg);
    if (st != VNE_OK) return fail(c, st, msg);

    auto g = std::make_unique<Graph>();
    g->n = n;
    g->nnz = nnz;
    g->scale = csr->scale;
    std::vector<float> v32(nnz);
    std::vector<double> v64(nnz);
    for (int64_t p = 0; p < nnz; ++p) {
        double v = csr->value_dtype == VNE_F64 ? ((const double *)hv.values)[p] : (double)((const float *)hv.values)[p];
        v64[p] = v;
        v32[p] = (float)v;
    }
    {
        int64_t off = 0, near = 0;
        for (int64_t i = 0; i < n; ++i)
            for (int32_t q = hv.row_ptr[i]; q < hv.row_ptr[i + 1]; ++q) {
                const int64_t j = hv.col_idx[q];
                if (j == i) continue;
                ++off;
                near += (j - i <= 256 && i - j <= 256);
            }
        g->local_frac = off ? (double)near / (double)off : 1.0;
    }
    g->zero_rowsum = true;
    for (int64_t i = 0; i < n && g->zero_rowsum; ++i) {
        double rs = 0.0;
        for (int32_t q = hv.row_ptr[i]; q < hv.row_ptr[i + 1]; ++q) rs += v64[q];
        g->zero_rowsum = rs == 0.0;
    }
    std::vector<int64_t> keys(n);
    for (int64_t i = 0; i < n; ++i) keys[i] = csr->node_keys ? csr->node_keys[i] : i;
    if (csr->location == VNE_DEVICE) {
        g->d_row_ptr = csr->row_ptr;
        g->d_col = csr->col_idx;
    } else {
        if ((st = upload(c, &g->row_ptr, hv.row_ptr, n + 1)) != VNE_OK) { free_graph(c, g.get()); return st; }
        if ((st = upload(c, &g->col, hv.col_idx, nnz)) != VNE_OK) { free_graph(c, g.get()); return st; }
        g->d_row_ptr = (const int32_t *)g->row_ptr.p;
        g->d_col = (const int32_t *)g->col.p;
    }
    if ((st = upload(c, &g->val32, v32.data(), nnz)) != VNE_OK ||
        (st = upload(c, &g->val64, v64.data(), nnz)) != VNE_OK ||
        (st = upload(c, &g->keys, keys.data(), n)) != VNE_OK) {
        free_graph(c, g.get());
        return st;
    }
    g->d_val32 = (const float *)g->val32.p;
    g->d_val64 = (const double *)g->val64.p;
    g->d_keys = (const int64_t *)g->keys.p;

    // work schedule: segments of long rows, cost-balanced blocks
    const int seg_len = std::max(1, env_int("VNE_SEG_LEN", 64));
    const int max_blocks = std::max(8, env_int("VNE_MAX_BLOCKS", 1024));
    int64_t total_cost = nnz + 4 * n;
    int64_t cpb = std::max<int64_t>(256, (total_cost + max_blocks - 1) / max_blocks);
    g->sched = build_schedule(hv.row_ptr, n, seg_len, cpb, max_blocks);
    const Schedule &s = g->sched;
    if ((st = upload(c, &g->segs, s.segs.data(), s.segs.size())) != VNE_OK ||
        (st = upload(c, &g->block_begin, s.block_begin.data(), s.block_begin.size())) != VNE_OK ||
        (st = upload(c, &g->long_first, s.long_first.data(), s.long_first.size())) != VNE_OK ||
        (st = upload(c, &g->long_nseg, s.long_nseg.data(), s.long_nseg.size())) != VNE_OK) {
        free_graph(c, g.get());
        return st;
    }
    g->alive = true;
    c->graphs.push_back(std::move(g));
    *graph_id = (int32_t)c->graphs.size() - 1;
    return VNE_OK;
}

extern "C" vne_status vne_graph_release(vne_ctx *c, int32_t gid) {
    if (!c) return VNE_EINVAL;
    Graph *g = get_graph(c, gid);
    if (!g) return fail(c, VNE_EINVAL, "unknown graph id");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    free_graph(c, g);
    return VNE_OK;
}

extern "C" vne_status vne_enable_kernel_timing(vne_ctx *c, int32_t enable) {
    if (!c) return VNE_EINVAL;
    c->timing = enable != 0;
    return VNE_OK;
}

extern "C" vne_status vne_kernel_timing(vne_ctx *c, int32_t reset, int64_t *launches, double *total_ms,
                                        double *bytes) {
    if (!c) return VNE_EINVAL;
    if (launches) *launches = c->t_launches;
    if (total_ms) *total_ms = c->t_ms;
    if (bytes) *bytes = c->t_bytes;
    if (reset) {
        c->t_launches = 0;
        c->t_ms = 0.0;
        c->t_bytes = 0.0;
    }
    return VNE_OK;
}

static vne_status estimate_hutchpp(vne_ctx *c, Graph *g, const vne_probes *pr, int k, bool fp64, bool desing,
                                   vne_result *out) {
    const int nr = pr->n_sketch, m = pr->m, nh = m - nr;
    if (nr < 1 || nh < 0 || nr > 128) return fail(c, VNE_ENOTSUP, "Hutch++ needs 1 <= n_sketch <= min(m, 128)");
    const size_t es = fp64 ? 8 : 4;
    Plan *sk = nullptr, *q = nullptr;
    vne_status st = get_plan(c, g, nr, k, fp64, true, 1, &sk);
    if (st != VNE_OK) return st;
    st = get_plan(c, g, m, k, fp64, false, 2, &q);
    if (st != VNE_OK) return st;
    if (!q->B.p) {
        auto A = [&](DevBuf *b, size_t bytes) {
            if (st == VNE_OK) st = dev_alloc(c, b, bytes);
        };
        A(&q->S, (size_t)nr * k * 8);
        A(&q->B, (size_t)g->n * m * es);
        const int64_t gd = std::max(gram_scratch_doubles((int32_t)g->n, nr, nr),
                                    gram_scratch_doubles((int32_t)g->n, nr, std::max(nh, 1)));
        A(&q->gram_part, (size_t)gd * 8);
        A(&q->gram, (size_t)nr * std::max(nr, nh) * 8);
        A(&q->rinv, (size_t)nr * nr * 8);
        A(&q->rot, (size_t)nr * rot_capacity(k) * kRotBytes);
        if (st != VNE_OK) return st;
    }
    hipStream_t s = c->stream;
    // 1. sketch: k Lanczos steps on Omega (kept basis), then Y = f(A) Omega by eq. (4.3)
    ProbeSpec ps;
    ps.gen = GEN_RADEMACHER;
    ps.seed = pr->seed;
    ps.col_offset = 0;
    if ((st = run_lanczos(c, g, sk, ps, desing)) != VNE_OK) return st;
    HIP_TRY(c, launch_fT_e1((const double *)sk->alpha.p, (const double *)sk->beta.p, (const int32_t *)sk->k_eff.p,
                            k, nr, (double *)q->S.p, q->rot.p, (int32_t *)sk->flags.p, s));
    const int64_t step_stride = (int64_t)g->n * sk->m_pad;
    HIP_TRY(c, launch_reconstruct(sk->Vstore.p, fp64, step_stride, sk->m_pad, (const double *)q->S.p,
                                  (const double *)sk->norm2.p, k, (int32_t)g->n, nr, q->B.p, m, s));
    // 2. G block, raw +-1 in the columns after the sketch
    if (nh > 0)
        HIP_TRY(c, launch_rademacher_fill(q->B.p, fp64, (int32_t)g->n, nh, m, nr, nr, pr->seed, g->d_keys, s));
    // 3. Q = orth(Y) by CholeskyQR (FP64 Gram and triangular factors), in
    // place; a second pass in FP64 mode (with FP32 storage the rounding of Q
    // itself bounds its orthogonality, so one pass suffices)
    for (int pass = 0; pass < (fp64 ? 2 : 1); ++pass) {
        HIP_TRY(c, launch_gram(q->B.p, m, q->B.p, m, fp64, (int32_t)g->n, nr, nr, (double *)q->gram_part.p,
                               (double *)q->gram.p, s));
        HIP_TRY(c, launch_cholinv((double *)q->gram.p, (double *)q->rinv.p, nr, (int32_t *)sk->flags.p, s));
        HIP_TRY(c, launch_apply(q->B.p, m, (const double *)q->rinv.p, nr, nr, q->B.p, m, fp64, (int32_t)g->n, 0, s));
    }
    // 4. G~ = G - Q (Q^T G)
    if (nh > 0) {
        char *Gp = (char *)q->B.p + (size_t)nr * es;
        HIP_TRY(c, launch_gram(q->B.p, m, Gp, m, fp64, (int32_t)g->n, nr, nh, (double *)q->gram_part.p,
                               (double *)q->gram.p, s));
        HIP_TRY(c, launch_apply(q->B.p, m, (const double *)q->gram.p, nr, nh, Gp, m, fp64, (int32_t)g->n, 1, s));
    }
    // 5. quadratic forms of [Q | G~] and the Hutch++ combination (3.9)
    ProbeSpec pq;
    pq.gen = GEN_DENSE;
    pq.dense = q->B.p;
    pq.ld_dense = m;
    if ((st = run_lanczos(c, g, q, pq, desing)) != VNE_OK) return st;
    HIP_TRY(c, launch_combine((const double *)q->psi.p, m, 2, nr, (double *)q->estimate.p, s));
    int32_t fl_q = 0, fl_s = 0;
    st = copy_out(c, q, out, &fl_q);
    if (st != VNE_OK) return st;
    HIP_TRY(c, hipMemcpy(&fl_s, sk->flags.p, 4, hipMemcpyDeviceToHost));
    if (c->timing && (st = collect_timing(c)) != VNE_OK) return st;
    if (fl_s & 2) return fail(c, VNE_ENUMERIC, "Cholesky of the sketch Gram matrix failed (rank-deficient sketch)");
    if ((fl_q | fl_s) & 1) return fail(c, VNE_ENUMERIC, "non-finite Lanczos coefficient");
    if ((fl_q | fl_s) & 4) return fail(c, VNE_ENUMERIC, "tridiagonal QR did not converge");
    if (fl_s & 8) return fail(c, VNE_ENUMERIC, "tridiagonal QR rotation record overflowed");
    return VNE_OK;
}

extern "C" vne_status vne_entropy_estimate(vne_ctx *c, int32_t gid, const vne_probes *pr, int32_t k,
                                           uint32_t mode, vne_result *out) {
    if (!c) return VNE_EINVAL;
    c->err.clear();
    if (!pr || !out) return fail(c, VNE_EINVAL, "NULL argument");
    Graph *g = get_graph(c, gid);
    if (!g) return fail(c, VNE_EINVAL, "unknown graph id");
    if (k < 1 || k > kMaxSteps) return fail(c, VNE_EINVAL, "k_steps must be in [1, 128]");
    if (pr->m < 1) return fail(c, VNE_EINVAL, "probe count m must be >= 1");
    if (pr->m > (1 << 20)) return fail(c, VNE_ENOTSUP, "probe count too large");
    if (mode & ~(uint32_t)(VNE_MODE_F64 | VNE_MODE_DESING)) return fail(c, VNE_EINVAL, "unknown mode bits");
    HIP_TRY(c, hipSetDevice(c->device));
    const bool fp64 = (mode & VNE_MODE_F64) != 0;
    const bool desing = (mode & VNE_MODE_DESING) != 0;
    if (desing && !g->zero_rowsum)
        return fail(c, VNE_EINVAL, "VNE_MODE_DESING needs a matrix whose rows sum to zero (A 1 = 0)");
    if (pr->kind == VNE_PROBE_HUTCHPP) return estimate_hutchpp(c, g, pr, k, fp64, desing, out);

    Plan *p = nullptr;
    vne_status st = get_plan(c, g, pr->m, k, fp64, false, 0, &p);
    if (st != VNE_OK) return st;
    ProbeSpec ps;
    int combine_kind = 0;
    const size_t es = fp64 ? 8 : 4;
    switch (pr->kind) {
        case VNE_PROBE_RADEMACHER:
            ps.gen = GEN_RADEMACHER;
            ps.seed = pr->seed;
            break;
        case VNE_PROBE_COLORING: {
            if (!pr->colors) return fail(c, VNE_EINVAL, "colors is NULL");
            ps.gen = GEN_COLORING;
            combine_kind = 1;
            if (pr->location == VNE_DEVICE) {
                ps.colors = pr->colors;
            } else {
                for (int64_t i = 0; i < g->n; ++i)
                    if (pr->colors[i] < 0 || pr->colors[i] >= pr->m)
                        return fail(c, VNE_EINVAL, "colour out of range at row " + std::to_string(i));
                if (!p->colors.p && (st = dev_alloc(c, &p->colors, (size_t)g->n * 4)) != VNE_OK) return st;
                HIP_TRY(c, hipMemcpyAsync(p->colors.p, pr->colors, (size_t)g->n * 4, hipMemcpyHostToDevice, c->stream));
                ps.colors = (const int32_t *)p->colors.p;
            }
            break;
        }
        case VNE_PROBE_DENSE: {
            if (!pr->dense) return fail(c, VNE_EINVAL, "dense is NULL");
            ps.gen = GEN_DENSE;
            ps.ld_dense = pr->m;
            if (pr->location == VNE_DEVICE) {
                ps.dense = pr->dense;
            } else {
                if (!p->dense.p && (st = dev_alloc(c, &p->dense, (size_t)g->n * pr->m * es)) != VNE_OK) return st;
                HIP_TRY(c, hipMemcpyAsync(p->dense.p, pr->dense, (size_t)g->n * pr->m * es, hipMemcpyHostToDevice,
                                          c->stream));
                ps.dense = p->dense.p;
            }
            break;
        }
        default:
            return fail(c, VNE_EINVAL, "unknown probe kind");
    }
    if ((st = run_lanczos(c, g, p, ps, desing)) != VNE_OK) return st;
    HIP_TRY(c, launch_combine((const double *)p->psi.p, p->m, combine_kind, 0, (double *)p->estimate.p, c->stream));
    int32_t fl = 0;
    if ((st = copy_out(c, p, out, &fl)) != VNE_OK) return st;
    if (c->timing && (st = collect_timing(c)) != VNE_OK) return st;
    if (fl & 1) return fail(c, VNE_ENUMERIC, "non-finite Lanczos coefficient");
    if (fl & 4) return fail(c, VNE_ENUMERIC, "tridiagonal QR did not converge");
    return VNE_OK;
}
