// Host runtime of the entropy engine: context, graph registry, graph sets
// (one graph, or several graphs stacked into one block-diagonal launch),
// cached workspaces ("plans"), the tile autotuner and the estimate entry
// points of vne.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "ctx_internal.h"
#include "internal.h"
#include "kernels.h"

using namespace vne;

namespace {

std::string g_create_error;

}  // namespace

namespace vne {
namespace rt {

vne_status fail(vne_ctx *c, vne_status st, const std::string &m) {
    c->err = m;
    return st;
}

vne_status hip_fail(vne_ctx *c, hipError_t e, const char *what) {
    c->err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? VNE_ENOMEM : VNE_EDEVICE;
}

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

// Allocates max(count, 1) elements and copies count elements (none if h is NULL).
template <typename T>
vne_status upload(vne_ctx *c, DevBuf *b, const T *h, size_t count) {
    VNE_TRY(dev_alloc(c, b, std::max<size_t>(count, 1) * sizeof(T)));
    if (count && h) HIP_TRY(c, hipMemcpy(b->p, h, count * sizeof(T), hipMemcpyHostToDevice));
    return VNE_OK;
}

int env_int(const char *name, int dflt) {
    const char *v = getenv(name);
    return v ? atoi(v) : dflt;
}

void free_plan(vne_ctx *c, Plan *p) {
    for (auto &kv : p->exec)
        if (kv.second) (void)hipGraphExecDestroy(kv.second);
    p->exec.clear();
    for (auto &kv : p->chunk_exec)
        if (kv.second) (void)hipGraphExecDestroy(kv.second);
    p->chunk_exec.clear();
    for (auto &kv : p->chain_exec)
        if (kv.second) (void)hipGraphExecDestroy(kv.second);
    p->chain_exec.clear();
    for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
    p->ev.clear();
    if (p->h_remaining) (void)hipHostFree(p->h_remaining);
    p->h_remaining = nullptr;
    if (p->h_stage) (void)hipHostFree(p->h_stage);
    p->h_stage = nullptr;
    p->h_stage_bytes = 0;
    DevBuf *all[] = {&p->P[0], &p->P[1], &p->V[0], &p->V[1], &p->Vstore, &p->alpha, &p->beta,
                     &p->st_alpha, &p->st_inv, &p->st_coup, &p->k_eff, &p->norm2, &p->mean, &p->psi,
                     &p->estimate, &p->flags, &p->partials, &p->level2, &p->probe_part, &p->seg_acc,
                     &p->long_part, &p->colors, &p->dense, &p->graph_k, &p->graph_m, &p->seeds,
                     &p->S, &p->B, &p->gram_part, &p->gram, &p->rinv, &p->rot, &p->col_tol, &p->col_stop,
                     &p->bound_lo, &p->bound_hi, &p->adapt_args, &p->remaining};
    for (DevBuf *b : all) dev_free(c, b);
}

void free_set(vne_ctx *c, GraphSet *s) {
    for (auto &kv : s->plans) free_plan(c, kv.second.get());
    s->plans.clear();
    DevBuf *all[] = {&s->row_ptr, &s->col, &s->val32, &s->val64, &s->keys, &s->row_graph, &s->long_graph,
                     &s->block_graph, &s->graph_block_begin, &s->graph_long_begin, &s->graph_scale,
                     &s->segs, &s->block_ranges, &s->long_first, &s->long_nseg, &s->probe_rows,
                     &s->probe_block_graph, &s->probe_graph_begin, &s->graph_row_begin};
    for (DevBuf *b : all) dev_free(c, b);
}

void free_graph(vne_ctx *c, Graph *g) {
    dev_free(c, &g->row_ptr);
    dev_free(c, &g->col);
    g->alive = false;
}

Graph *get_graph(vne_ctx *c, int32_t gid) {
    if (gid < 0 || gid >= (int32_t)c->graphs.size() || !c->graphs[gid] || !c->graphs[gid]->alive) return nullptr;
    return c->graphs[gid].get();
}


// Work blocks of a set of several graphs: each graph's own schedule, built
// with one cost per block for the whole set (so that a batch of many small
// graphs gets a few blocks per graph, not the padded count of a lone graph).
Schedule set_schedule(const std::vector<Graph *> &gs, const std::vector<int64_t> &row_begin,
                      const std::vector<int64_t> &nnz_begin, std::vector<int32_t> *gbb, std::vector<int32_t> *glb,
                      std::vector<int32_t> *bg) {
    int64_t total = 0;
    for (const Graph *g : gs) total += g->nnz + 4 * g->n;
    // 16384 blocks: on the 512-graph batch the step ran 12% faster than with
    // 4096 and 2% faster than with 65536 (measured)
    const int max_blocks = std::max(8, env_int("VNE_SET_MAX_BLOCKS", 16384));
    const int64_t cpb = std::max<int64_t>(256, (total + max_blocks - 1) / max_blocks);
    std::vector<Schedule> parts;
    for (const Graph *g : gs)
        parts.push_back(build_schedule(g->h_row_ptr.data(), g->n, g->sched.seg_len, cpb, max_blocks, false));
    return stack_schedules(parts, std::vector<int64_t>(row_begin.begin(), row_begin.end() - 1),
                           std::vector<int64_t>(nnz_begin.begin(), nnz_begin.end() - 1), gbb, glb, bg);
}

// The set of the given graphs (built and cached on first use).
vne_status get_set(vne_ctx *c, const std::vector<int32_t> &ids, GraphSet **out) {
    auto it = c->sets.find(ids);
    if (it != c->sets.end()) {
        it->second->last_use = ++c->tick;
        *out = it->second.get();
        return VNE_OK;
    }
    if (ids.size() > 1) {
        // keep at most VNE_MAX_SETS stacked sets (least recently used first out)
        const size_t cap = (size_t)std::max(1, env_int("VNE_MAX_SETS", 4));
        for (;;) {
            size_t multi = 0;
            auto victim = c->sets.end();
            for (auto jt = c->sets.begin(); jt != c->sets.end(); ++jt) {
                if (jt->second->G < 2) continue;
                ++multi;
                if (victim == c->sets.end() || jt->second->last_use < victim->second->last_use) victim = jt;
            }
            if (multi < cap) break;
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            free_set(c, victim->second.get());
            c->sets.erase(victim);
        }
    }
    auto s = std::make_unique<GraphSet>();
    s->last_use = ++c->tick;
    s->ids = ids;
    s->G = (int)ids.size();
    std::vector<Graph *> gs;
    for (int32_t id : ids) {
        Graph *g = get_graph(c, id);
        if (!g) return fail(c, VNE_EINVAL, "unknown graph id " + std::to_string(id));
        gs.push_back(g);
    }
    const int G = s->G;
    s->h_row_begin.assign(G + 1, 0);
    std::vector<int64_t> nnz_begin(G + 1, 0);
    for (int q = 0; q < G; ++q) {
        s->h_row_begin[q + 1] = s->h_row_begin[q] + gs[q]->n;
        nnz_begin[q + 1] = nnz_begin[q] + gs[q]->nnz;
        s->zero_rowsum = s->zero_rowsum && gs[q]->zero_rowsum;
    }
    s->n = s->h_row_begin[G];
    s->nnz = nnz_begin[G];
    if (s->n > INT32_MAX - 1 || s->nnz > INT32_MAX) return fail(c, VNE_ENOTSUP, "batch too large for int32 indices");
    s->scale = gs[0]->scale;
    vne_status st = VNE_OK;
    auto fin = [&](vne_status e) {
        free_set(c, s.get());
        return e;
    };
    // stacked matrix (for one graph: the graph's own index arrays)
    if (G == 1) {
        s->d_row_ptr = gs[0]->d_row_ptr;
        s->d_col = gs[0]->d_col;
    } else {
        std::vector<int32_t> rp(s->n + 1), ci(s->nnz), rg(s->n);
        for (int q = 0; q < G; ++q) {
            const Graph *g = gs[q];
            for (int64_t i = 0; i < g->n; ++i) {
                rp[s->h_row_begin[q] + i] = (int32_t)(g->h_row_ptr[i] + nnz_begin[q]);
                rg[s->h_row_begin[q] + i] = q;
            }
            for (int64_t p = 0; p < g->nnz; ++p) ci[nnz_begin[q] + p] = (int32_t)(g->h_col[p] + s->h_row_begin[q]);
        }
        rp[s->n] = (int32_t)s->nnz;
        std::vector<double> scales(G);
        for (int q = 0; q < G; ++q) scales[q] = gs[q]->scale;
        if ((st = upload(c, &s->row_ptr, rp.data(), rp.size())) != VNE_OK ||
            (st = upload(c, &s->col, ci.data(), ci.size())) != VNE_OK ||
            (st = upload(c, &s->row_graph, rg.data(), rg.size())) != VNE_OK ||
            (st = upload(c, &s->graph_scale, scales.data(), scales.size())) != VNE_OK)
            return fin(st);
        s->d_row_ptr = (const int32_t *)s->row_ptr.p;
        s->d_col = (const int32_t *)s->col.p;
    }
    {
        std::vector<float> v32(s->nnz);
        std::vector<double> v64(s->nnz);
        std::vector<int64_t> keys(s->n);
        for (int q = 0; q < G; ++q) {
            const Graph *g = gs[q];
            for (int64_t p = 0; p < g->nnz; ++p) {
                v64[nnz_begin[q] + p] = g->h_val[p];
                v32[nnz_begin[q] + p] = (float)g->h_val[p];
            }
            std::copy(g->h_keys.begin(), g->h_keys.end(), keys.begin() + s->h_row_begin[q]);
        }
        if ((st = upload(c, &s->val32, v32.data(), v32.size())) != VNE_OK ||
            (st = upload(c, &s->val64, v64.data(), v64.size())) != VNE_OK ||
            (st = upload(c, &s->keys, keys.data(), keys.size())) != VNE_OK)
            return fin(st);
    }
    // work schedule
    std::vector<int32_t> gbb, glb, bg;
    if (G == 1) {
        s->sched = gs[0]->sched;
        gbb = {0, s->sched.n_blocks()};
        glb = {0, s->sched.n_long};
    } else {
        s->sched = set_schedule(gs, s->h_row_begin, nnz_begin, &gbb, &glb, &bg);
        std::vector<int32_t> lg(s->sched.n_long);
        for (int q = 0; q < G; ++q)
            for (int L = glb[q]; L < glb[q + 1]; ++L) lg[L] = q;
        if ((st = upload(c, &s->long_graph, lg.data(), lg.size())) != VNE_OK ||
            (st = upload(c, &s->block_graph, bg.data(), bg.size())) != VNE_OK)
            return fin(st);
    }
    const Schedule &sc = s->sched;
    if ((st = upload(c, &s->segs, sc.segs.data(), sc.segs.size())) != VNE_OK ||
        (st = upload(c, &s->block_ranges, sc.block_ranges.data(), sc.block_ranges.size())) != VNE_OK ||
        (st = upload(c, &s->long_first, sc.long_first.data(), sc.long_first.size())) != VNE_OK ||
        (st = upload(c, &s->long_nseg, sc.long_nseg.data(), sc.long_nseg.size())) != VNE_OK ||
        (st = upload(c, &s->graph_block_begin, gbb.data(), gbb.size())) != VNE_OK ||
        (st = upload(c, &s->graph_long_begin, glb.data(), glb.size())) != VNE_OK)
        return fin(st);
    // probe blocks: row ranges inside one graph each, about 2048 blocks in all
    const int64_t probe_rows = std::min<int64_t>(2048, std::max<int64_t>(64, (s->n + 2047) / 2048));
    std::vector<int32_t> prows, pbg, pgb(G + 1, 0);
    for (int q = 0; q < G; ++q) {
        pgb[q] = (int32_t)pbg.size();
        for (int64_t r = s->h_row_begin[q]; r < s->h_row_begin[q + 1]; r += probe_rows) {
            prows.push_back((int32_t)r);
            pbg.push_back(q);
        }
    }
    pgb[G] = (int32_t)pbg.size();
    prows.push_back((int32_t)s->n);
    s->probe_blocks = (int)pbg.size();
    if ((st = upload(c, &s->probe_rows, prows.data(), prows.size())) != VNE_OK ||
        (st = upload(c, &s->probe_block_graph, pbg.data(), pbg.size())) != VNE_OK ||
        (st = upload(c, &s->probe_graph_begin, pgb.data(), pgb.size())) != VNE_OK ||
        (st = upload(c, &s->graph_row_begin, s->h_row_begin.data(), s->h_row_begin.size())) != VNE_OK)
        return fin(st);
    *out = s.get();
    c->sets[ids] = std::move(s);
    return VNE_OK;
}

// Shape of a plan (tile, padded width) for m columns per graph and k steps.
vne_status plan_shape(vne_ctx *c, const GraphSet *set, Plan *p, int m, int k, bool fp64, bool store) {
    p->fp64 = fp64;
    p->G = set->G;
    p->m = m;
    p->k = k;
    p->store = store;
    const int forced = env_int("VNE_TILE", 0);
    p->mt = forced > 0 || env_int("VNE_TILE3", 1) == 0 ? choose_tile(m, fp64, forced)
                                                       : choose_plan_tile(m, fp64, set->n, set->nnz);
    p->m_pad = pad_columns(m, p->mt);
    const size_t es = fp64 ? 8 : 4;
    // sizes far beyond any device (and beyond size_t arithmetic) fail here
    if ((double)set->n * p->m_pad * es * (store ? k : 1) > 0x1p56)
        return fail(c, VNE_ENOMEM, "probe block of " + std::to_string(m) + " columns on " +
                                       std::to_string(set->n) + " rows exceeds any device memory");
    return VNE_OK;
}

// Every device buffer of a shaped plan, in a fixed order: take(buffer, bytes).
void plan_buffers(const GraphSet *set, Plan *p, const std::function<void(DevBuf *, size_t)> &take) {
    const size_t es = p->fp64 ? 8 : 4;
    const size_t blk = (size_t)set->n * p->m_pad * es;
    const Schedule &s = set->sched;
    const size_t cols = (size_t)p->G * p->m_pad;      // (graph, column) pairs
    const size_t k = (size_t)p->k;
    take(&p->P[0], blk);
    take(&p->P[1], blk);
    if (p->store) {
        take(&p->Vstore, blk * k);
    } else {
        take(&p->V[0], blk);
        take(&p->V[1], blk);
    }
    take(&p->alpha, cols * k * 8);
    take(&p->beta, cols * k * 8);
    take(&p->st_alpha, cols * 8);
    take(&p->st_inv, cols * 8);
    take(&p->st_coup, cols * 8);
    take(&p->k_eff, cols * 4);
    take(&p->norm2, cols * 8);
    take(&p->mean, cols * 8);
    take(&p->psi, cols * 8);
    take(&p->estimate, (size_t)p->G * 8);
    take(&p->flags, 4);
    take(&p->partials, (size_t)s.n_blocks() * 3 * p->m_pad * 8);
    take(&p->level2, (size_t)kLevel2 * 3 * p->m_pad * 8);
    take(&p->probe_part, (size_t)set->probe_blocks * p->m_pad * 8);
    take(&p->seg_acc, (size_t)std::max(1, s.n_seg) * p->m_pad * 8);
    take(&p->long_part, (size_t)std::max(1, s.n_long) * 3 * p->m_pad * 8);
    take(&p->graph_k, (size_t)p->G * 4);
    take(&p->graph_m, (size_t)p->G * 4);
    take(&p->seeds, (size_t)p->G * 8);
}

// Workspace for probe blocks of width m (per graph) and k steps on a set.
vne_status get_plan(vne_ctx *c, GraphSet *set, int m, int k, bool fp64, bool store, int tag, Plan **out) {
    auto key = std::make_tuple(m, k, (int)fp64, (int)store, tag);
    auto it = set->plans.find(key);
    if (it != set->plans.end()) {
        *out = it->second.get();
        return VNE_OK;
    }
    auto p = std::make_unique<Plan>();
    VNE_TRY(plan_shape(c, set, p.get(), m, k, fp64, store));
    vne_status st = VNE_OK;
    plan_buffers(set, p.get(), [&](DevBuf *b, size_t bytes) {
        if (st == VNE_OK) st = dev_alloc(c, b, bytes);
    });
    if (st != VNE_OK) {
        free_plan(c, p.get());
        return st;
    }
    HIP_TRY(c, hipMemsetAsync(p->long_part.p, 0, p->long_part.bytes, c->stream));
    HIP_TRY(c, hipMemsetAsync(p->seeds.p, 0, p->seeds.bytes, c->stream));
    *out = p.get();
    set->plans[key] = std::move(p);
    return VNE_OK;
}

vne_status collect_timing(vne_ctx *c) {
    for (auto &pd : c->pending) {
        Plan *p = (Plan *)pd.plan;
        if (pd.loop) {
            // concurrent tile chains: the loop's span, every step counted once
            float ms = 0.f;
            HIP_TRY(c, hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
            c->t_ms += ms;
            c->t_bytes += pd.bytes * pd.steps;
            c->t_launches += pd.steps;
            continue;
        }
        for (int j = 0; j < pd.steps; ++j) {
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

// Probe block, Lanczos steps, quadrature (declared with RunOpts).
vne_status run_lanczos(vne_ctx *c, GraphSet *set, Plan *p, const ProbeSpec &ps, bool desing,
                       const RunOpts &opt) {
    const Schedule &s = set->sched;
    const int mt = opt.tile > 0 ? opt.tile : p->mt;
    if (opt.steps < 0) {                 // not an autotuner trial
        c->last_tile = mt;
        c->last_m_pad = p->m_pad;
    }
    HIP_TRY(c, hipMemsetAsync(p->flags.p, 0, 4, c->stream));
    // per-graph steps, widths and seeds: uploaded only when they change (a
    // copy from pageable memory waits for the stream, which would expose the
    // host's launch latency between the phases of one estimate)
    if (p->up_graph_k != p->h_graph_k) {
        HIP_TRY(c, hipMemcpyAsync(p->graph_k.p, p->h_graph_k.data(), p->G * 4, hipMemcpyHostToDevice, c->stream));
        p->up_graph_k = p->h_graph_k;
    }
    if (p->up_graph_m != p->h_graph_m) {
        HIP_TRY(c, hipMemcpyAsync(p->graph_m.p, p->h_graph_m.data(), p->G * 4, hipMemcpyHostToDevice, c->stream));
        p->up_graph_m = p->h_graph_m;
    }
    if (!ps.seeds.empty() && p->up_seeds != ps.seeds) {
        HIP_TRY(c, hipMemcpyAsync(p->seeds.p, ps.seeds.data(), p->G * 8, hipMemcpyHostToDevice, c->stream));
        p->up_seeds = ps.seeds;
    }
    ProbeArgs pa{};
    pa.gen = ps.gen;
    pa.n = (int32_t)set->n;
    pa.m = p->m;
    pa.m_pad = p->m_pad;
    pa.mt = mt;
    pa.col_offset = ps.col_offset;
    pa.seed = ps.seeds.empty() ? 0 : ps.seeds[0];
    pa.keys = (const int64_t *)set->keys.p;
    pa.colors = ps.colors;
    pa.dense = ps.dense;
    pa.ld_dense = ps.ld_dense;
    pa.desing = desing ? 1 : 0;
    pa.P_out = p->P[0].p;
    pa.partials = (double *)p->probe_part.p;
    pa.n_blocks = set->probe_blocks;
    pa.mean = (double *)p->mean.p;
    pa.norm2 = (double *)p->norm2.p;
    pa.st_alpha = (double *)p->st_alpha.p;
    pa.st_inv = (double *)p->st_inv.p;
    pa.st_coup = (double *)p->st_coup.p;
    pa.k_eff = (int32_t *)p->k_eff.p;
    pa.k = p->k;
    pa.block_row_begin = (const int32_t *)set->probe_rows.p;
    pa.block_graph = (const int32_t *)set->probe_block_graph.p;
    pa.graph_block_begin = (const int32_t *)set->probe_graph_begin.p;
    pa.graph_row_begin = (const int64_t *)set->graph_row_begin.p;
    pa.seeds = (const uint64_t *)p->seeds.p;
    pa.graph_k = (const int32_t *)p->graph_k.p;
    pa.graph_m = (const int32_t *)p->graph_m.p;
    pa.n_graphs = p->G;
    pa.flags = (int32_t *)p->flags.p;
    HIP_TRY(c, launch_probe(pa, p->fp64, c->stream));

    const size_t es = p->fp64 ? 8 : 4;
    const size_t blk_elems = (size_t)set->n * p->m_pad;
    // algorithmic bytes of one step launch: CSR once, v_j gathered once,
    // v_{j-1} read once, P_{j+1} written once (real columns only)
    int64_t m_sum = 0;
    for (int q = 0; q < p->G; ++q) m_sum += (int64_t)p->h_graph_m[q] * (set->h_row_begin[q + 1] - set->h_row_begin[q]);
    const double bytes = 4.0 * (set->n + 1) + (double)set->nnz * (4.0 + es) + 3.0 * (double)m_sum * es;
    StepArgs a{};
    a.row_ptr = set->d_row_ptr;
    a.col = set->d_col;
    a.val = p->fp64 ? set->val64.p : set->val32.p;
    a.scale = set->scale;
    a.n = (int32_t)set->n;
    a.m_pad = p->m_pad;
    a.mt = mt;
    a.n_tiles = p->m_pad / mt;
    a.st_alpha = (const double *)p->st_alpha.p;
    a.st_inv = (const double *)p->st_inv.p;
    a.st_coup = (const double *)p->st_coup.p;
    a.segs = (const SegItem *)set->segs.p;
    a.n_seg = s.n_seg;
    a.seg_len = s.seg_len;
    a.block_ranges = (const int4 *)set->block_ranges.p;
    a.n_blocks = s.n_blocks();
    a.seg_acc = (double *)p->seg_acc.p;
    a.n_long = s.n_long;
    a.long_first = (const int32_t *)set->long_first.p;
    a.long_nseg = (const int32_t *)set->long_nseg.p;
    a.long_part = (double *)p->long_part.p;
    a.partials = (double *)p->partials.p;
    if (set->G > 1) {
        a.block_graph = (const int32_t *)set->block_graph.p;
        a.row_graph = (const int32_t *)set->row_graph.p;
        a.long_graph = (const int32_t *)set->long_graph.p;
        a.graph_scale = (const double *)set->graph_scale.p;
    }
    // schedule: normalize pass + single-stream SpMM by default (measured
    // faster on both random and ring-local graphs); the lazy one-pass
    // schedule (4 streams, two of them gathered) stays selectable
    {
        const int forced = env_int("VNE_SCHED", -1);
        a.two_pass = forced >= 0 ? forced : 1;
    }

    FinalizeArgs f{};
    f.partials = (const double *)p->partials.p;
    f.long_part = (const double *)p->long_part.p;
    f.level2 = (double *)p->level2.p;
    f.n_level2 = kLevel2;
    f.n_blocks = s.n_blocks();
    f.n_long = s.n_long;
    f.mt = mt;
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
    f.n_graphs = p->G;
    f.segmented = p->G > 1 ? 1 : 0;
    f.graph_block_begin = (const int32_t *)set->graph_block_begin.p;
    f.graph_long_begin = (const int32_t *)set->graph_long_begin.p;
    f.graph_k = (const int32_t *)p->graph_k.p;
    f.graph_m = (const int32_t *)p->graph_m.p;

    const bool tuning = opt.steps > 0;
    const int nsteps = tuning ? std::min(opt.steps, p->k) : p->k;
    const bool use_graph = env_int("VNE_GRAPH", 1) != 0 && (!tuning || opt.graph_trial) && !opt.direct;
    const bool timing = c->timing && opt.collect;
    // part 0: the step kernels of step j; part 1: its reduction and finalize
    auto issue_on = [&](StepArgs &sa, FinalizeArgs &fa, int j, int part, hipStream_t st) -> vne_status {
        char *Pb[2] = {(char *)p->P[0].p, (char *)p->P[1].p};
        sa.P_in = Pb[(j - 1) & 1];
        sa.P_out = Pb[j & 1];
        if (p->store) {
            char *base = (char *)p->Vstore.p;
            sa.V_out = base + (size_t)(j - 1) * blk_elems * es;
            sa.V_prev = j >= 2 ? base + (size_t)(j - 2) * blk_elems * es : nullptr;
        } else {
            sa.V_out = p->V[(j - 1) & 1].p;
            sa.V_prev = p->V[j & 1].p;
        }
        sa.V_cur = sa.V_out;
        if (part == 0) {
            HIP_TRY(c, launch_step(sa, p->fp64, j == 1, st));
        } else {
            fa.step = j;
            HIP_TRY(c, launch_finalize(fa, st));
        }
        return VNE_OK;
    };
    auto issue = [&](int j, int part) -> vne_status { return issue_on(a, f, j, part, c->stream); };
    auto capture_on = [&](hipStream_t cs, hipGraphExec_t *ex, const std::function<vne_status()> &body) -> vne_status {
        hipGraph_t graph = nullptr;
        HIP_TRY(c, hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
        vne_status st = body();
        hipError_t e_end = hipStreamEndCapture(cs, &graph);
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
    auto capture_fn = [&](hipGraphExec_t *ex, const std::function<vne_status()> &body) -> vne_status {
        return capture_on(c->stream, ex, body);
    };
    auto capture = [&](hipGraphExec_t *ex, int j0, int j1, int part_only) -> vne_status {
        return capture_fn(ex, [&]() -> vne_status {
            for (int j = j0; j <= j1; ++j)
                for (int part = 0; part < 2; ++part)
                    if (part_only < 0 || part == part_only) VNE_TRY(issue(j, part));
            return VNE_OK;
        });
    };
    if (timing) {
        while (p->ev.size() < (size_t)(2 * p->k)) {
            hipEvent_t e;
            HIP_TRY(c, hipEventCreate(&e));
            p->ev.push_back(e);
        }
    }
    const auto key = std::make_pair(a.two_pass ? 1 : 0, mt);
    if (opt.adaptive && !tuning) {
        // Per-column stopping: the steps up to each check (3, 5, 7, ...) run
        // as one chunk, followed by the bracket of the running columns and
        // the stop record; the host reads the running count after each check
        // and launches no further chunk once it is zero.
        if (p->G != 1 || p->store) return fail(c, VNE_ENOTSUP, "per-column stopping runs on one graph");
        const int K = p->k, M = p->m;
        const size_t nb = (size_t)(K + 1) * (sizeof(BoundArgs) + sizeof(ColStopArgs));
        // each buffer on its own, so that a failed allocation leaves no half
        // set-up plan behind
        if (!p->col_stop.p) VNE_TRY(dev_alloc(c, &p->col_stop, (size_t)p->m_pad * 4));
        if (!p->bound_lo.p) VNE_TRY(dev_alloc(c, &p->bound_lo, (size_t)p->m_pad * 8));
        if (!p->bound_hi.p) VNE_TRY(dev_alloc(c, &p->bound_hi, (size_t)p->m_pad * 8));
        if (!p->adapt_args.p) VNE_TRY(dev_alloc(c, &p->adapt_args, nb));
        if (!p->remaining.p) VNE_TRY(dev_alloc(c, &p->remaining, 4));
        if (!p->col_tol.p) return fail(c, VNE_EINVAL, "per-column tolerances not set");
        if (!p->h_remaining) HIP_TRY(c, hipHostMalloc((void **)&p->h_remaining, 4, hipHostMallocDefault));
        p->h_adapt.assign(nb, 0);
        BoundArgs *hb = (BoundArgs *)p->h_adapt.data();
        ColStopArgs *hs = (ColStopArgs *)(hb + K + 1);
        BoundArgs *db = (BoundArgs *)p->adapt_args.p;
        ColStopArgs *ds = (ColStopArgs *)(db + K + 1);
        for (int j = 0; j <= K; ++j) {
            BoundArgs &b = hb[j];
            b.alpha = (const double *)p->alpha.p;
            b.beta = (const double *)p->beta.p;
            b.k_eff = (const int32_t *)p->k_eff.p;
            b.norm2 = (const double *)p->norm2.p;
            b.k = K;
            b.m = M;
            b.steps = std::max(j, 1);
            b.lam_lo = opt.lam_lo;
            b.lam_hi = opt.lam_hi;
            b.n_grid = opt.n_grid;
            b.lo = (double *)p->bound_lo.p;
            b.hi = (double *)p->bound_hi.p;
            b.flags = (int32_t *)p->flags.p;
            b.col_stop = (const int32_t *)p->col_stop.p;
            ColStopArgs &q = hs[j];
            q.lo = (const double *)p->bound_lo.p;
            q.estimate = opt.estimate ? 1 : 0;
            q.hi = (const double *)p->bound_hi.p;
            q.tol = (const double *)p->col_tol.p;
            q.col_stop = (int32_t *)p->col_stop.p;
            q.m = M;
            q.step = j;
            q.remaining = (int32_t *)p->remaining.p;
        }
        HIP_TRY(c, hipMemcpyAsync(p->adapt_args.p, p->h_adapt.data(), nb, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemsetAsync(p->col_stop.p, 0, (size_t)p->m_pad * 4, c->stream));
        // done columns: their tiles and normalize groups are skipped, their
        // coefficients kept (the quadrature takes the stop step's);
        // VNE_FREEZE=0 keeps computing them (for measurements)
        if (env_int("VNE_FREEZE", 1) != 0) {
            a.col_stop = (const int32_t *)p->col_stop.p;
            f.col_stop = (const int32_t *)p->col_stop.p;
        }
        struct Chunk {
            int j0, j1;
            bool check;
        };
        std::vector<Chunk> chunks;
        int j0 = 1;
        for (int sc = 3; sc <= K; sc += 2) {
            chunks.push_back({j0, sc, true});
            j0 = sc + 1;
        }
        if (j0 <= K) chunks.push_back({j0, K, false});
        auto body = [&](const Chunk &ch) -> vne_status {
            for (int j = ch.j0; j <= ch.j1; ++j) {
                if (timing) HIP_TRY(c, hipEventRecord(p->ev[2 * (j - 1)], c->stream));
                VNE_TRY(issue(j, 0));
                if (timing) HIP_TRY(c, hipEventRecord(p->ev[2 * (j - 1) + 1], c->stream));
                VNE_TRY(issue(j, 1));
            }
            if (ch.check) {
                HIP_TRY(c, launch_error_bound_cols(db + ch.j1, M, c->stream));
                HIP_TRY(c, launch_column_stop(ds + ch.j1, c->stream));
            }
            return VNE_OK;
        };
        int ran = 0;
        for (const Chunk &ch : chunks) {
            if (use_graph && !timing) {
                // (the captured launches hold the arguments: one graph per
                // schedule, tile, freezing and first step of the chunk)
                hipGraphExec_t &ex =
                    p->chunk_exec[std::make_tuple(key.first | (a.col_stop ? 2 : 0), key.second, ch.j0)];
                if (!ex) VNE_TRY(capture_fn(&ex, [&]() { return body(ch); }));
                HIP_TRY(c, hipGraphLaunch(ex, c->stream));
            } else {
                VNE_TRY(body(ch));
            }
            ran = ch.j1;
            if (ch.check) {
                HIP_TRY(c, hipMemcpyAsync(p->h_remaining, p->remaining.p, 4, hipMemcpyDeviceToHost, c->stream));
                HIP_TRY(c, hipStreamSynchronize(c->stream));
                if (*p->h_remaining == 0) break;
            }
        }
        p->steps_run = ran;
        if (timing) c->pending.push_back({p, bytes, ran});
        HIP_TRY(c, launch_quadrature((const double *)p->alpha.p, (const double *)p->beta.p,
                                     (const int32_t *)p->k_eff.p, (const double *)p->norm2.p, K, K, p->m_pad,
                                     (double *)p->psi.p, (int32_t *)p->flags.p, c->stream, p->fp64, nullptr, 0,
                                     (const int32_t *)p->col_stop.p));
        return VNE_OK;
    }
    // Concurrent tile chains (one graph, two-pass schedule, two or more
    // tiles): the tiles of the block are split into up to VNE_CHAINS groups
    // (default 2), each with its whole k-step loop on a stream of its own
    // after a fork from the caller's stream and joined back at the end.
    // Columns never meet across tiles, so each chain's kernels touch only
    // their own columns of the shared buffers and the results are the same
    // bits; the chains overlap one tile's streaming pass with another's
    // gathers.  Kernel timing then records the loop's span once.
    // (2 chains: BA n = 2e5 Hutch++ 128 + 128 at tile 64, 35.9 ms per
    // estimate against 38.1 ms with one chain and 37.7 ms with 4)
    const int max_chains = std::min(env_int("VNE_CHAINS", 2), 8);
    const int chains = (a.two_pass && set->G == 1 && a.n_tiles >= 2 && !opt.direct && max_chains >= 2)
                           ? std::min(a.n_tiles, max_chains)
                           : 1;
    if (chains > 1) {
        while ((int)c->chain_streams.size() < chains) {
            hipStream_t cs = nullptr;
            HIP_TRY(c, hipStreamCreate(&cs));
            c->chain_streams.push_back(cs);
        }
        while ((int)c->chain_events.size() < chains + 1) {
            hipEvent_t e = nullptr;
            HIP_TRY(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
            c->chain_events.push_back(e);
        }
        std::vector<StepArgs> ca(chains, a);
        std::vector<FinalizeArgs> cf(chains, f);
        for (int i = 0, t0 = 0; i < chains; ++i) {
            const int cnt = a.n_tiles / chains + (i < a.n_tiles % chains ? 1 : 0);
            ca[i].tile_base = t0;
            ca[i].n_tiles = cnt;
            ca[i].col_base = t0 * mt;
            ca[i].col_count = cnt * mt;
            cf[i].col_base = t0 * mt;
            cf[i].col_count = cnt * mt;
            t0 += cnt;
        }
        const bool chain_graphs = use_graph;
        if (timing) HIP_TRY(c, hipEventRecord(p->ev[0], c->stream));
        HIP_TRY(c, hipEventRecord(c->chain_events[0], c->stream));
        for (int i = 0; i < chains; ++i) {
            hipStream_t cs = c->chain_streams[i];
            HIP_TRY(c, hipStreamWaitEvent(cs, c->chain_events[0], 0));
            if (chain_graphs) {
                hipGraphExec_t &ex = p->chain_exec[std::make_tuple(key.first, key.second, chains, i)];
                if (!ex) {
                    VNE_TRY(capture_on(cs, &ex, [&]() -> vne_status {
                        for (int j = 1; j <= p->k; ++j)
                            for (int part = 0; part < 2; ++part) VNE_TRY(issue_on(ca[i], cf[i], j, part, cs));
                        return VNE_OK;
                    }));
                }
                HIP_TRY(c, hipGraphLaunch(ex, cs));
            } else {
                for (int j = 1; j <= nsteps; ++j)
                    for (int part = 0; part < 2; ++part) VNE_TRY(issue_on(ca[i], cf[i], j, part, cs));
            }
            HIP_TRY(c, hipEventRecord(c->chain_events[1 + i], cs));
            HIP_TRY(c, hipStreamWaitEvent(c->stream, c->chain_events[1 + i], 0));
        }
        if (timing) HIP_TRY(c, hipEventRecord(p->ev[1], c->stream));
        if (tuning) return VNE_OK;
        if (timing) c->pending.push_back({p, bytes, p->k, true});
        if (p->store) return VNE_OK;
        HIP_TRY(c, launch_quadrature((const double *)p->alpha.p, (const double *)p->beta.p,
                                     (const int32_t *)p->k_eff.p, (const double *)p->norm2.p, p->k, p->k,
                                     p->G * p->m_pad, (double *)p->psi.p, (int32_t *)p->flags.p, c->stream, p->fp64));
        return VNE_OK;
    }
    if (use_graph && (!timing || tuning)) {
        hipGraphExec_t &ex = p->exec[key];
        if (!ex) VNE_TRY(capture(&ex, 1, p->k, -1));
        HIP_TRY(c, hipGraphLaunch(ex, c->stream));
    } else {
        for (int j = 1; j <= nsteps; ++j) {
            if (timing) HIP_TRY(c, hipEventRecord(p->ev[2 * (j - 1)], c->stream));
            VNE_TRY(issue(j, 0));
            if (timing) HIP_TRY(c, hipEventRecord(p->ev[2 * (j - 1) + 1], c->stream));
            VNE_TRY(issue(j, 1));
        }
    }
    if (tuning) return VNE_OK;
    if (timing) c->pending.push_back({p, bytes, p->k});
    if (p->store) return VNE_OK;   // the Hutch++ sketch needs f(T) e1 (k_fT_e1), not psi
    HIP_TRY(c, launch_quadrature((const double *)p->alpha.p, (const double *)p->beta.p, (const int32_t *)p->k_eff.p,
                                 (const double *)p->norm2.p, p->k, p->k, p->G * p->m_pad, (double *)p->psi.p,
                                 (int32_t *)p->flags.p, c->stream, p->fp64));
    return VNE_OK;
}

// Column tile of a plan, chosen by timing a few steps of every tile that
// divides the padded width; cached per set shape.  VNE_AUTOTUNE=0 (or a
// forced VNE_TILE) keeps the default rule; VNE_AUTOTUNE_CACHE names a file
// that keeps the choices across processes.
vne_status autotune(vne_ctx *c, GraphSet *set, Plan *p, const ProbeSpec &ps, bool desing) {
    if (const int forced = env_int("VNE_TILE", 0); forced > 0) {
        const int t = choose_tile(p->m, p->fp64, forced);
        if (p->m_pad % t == 0) p->mt = t;
        return VNE_OK;
    }
    if (env_int("VNE_AUTOTUNE", 1) == 0) return VNE_OK;
    std::ostringstream sig;
    sig << "G" << set->G << "_n" << set->n << "_nnz" << set->nnz << "_m" << p->m_pad << (p->fp64 ? "_f64" : "_f32")
        << "_s" << set->sched.seg_len << "_b" << set->sched.n_blocks();
    auto it = c->tuned.find(sig.str());
    if (it != c->tuned.end()) {
        if (p->m_pad % it->second == 0) p->mt = it->second;
        return VNE_OK;
    }
    const int cpl = p->fp64 ? 2 : 4;
    std::vector<int> cands;
    // the narrow tiles (one or two lanes per row) only for narrow blocks
    for (int t = p->m_pad <= cpl * 4 ? cpl : cpl * 4; t <= cpl * 64; t *= 2)
        if (t <= p->m_pad && p->m_pad % t == 0) cands.push_back(t);
    if (std::find(cands.begin(), cands.end(), p->mt) == cands.end()) cands.push_back(p->mt);
    int best = p->mt;
    if (cands.size() > 1) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIP_TRY(c, hipEventCreate(&e0));
        HIP_TRY(c, hipEventCreate(&e1));
        float best_ms = 1e30f;
        vne_status st = VNE_OK;
        for (int t : cands) {
            // each candidate runs the whole loop the way the estimate will
            // (captured graphs, concurrent tile chains), the first time to
            // capture and warm up, the second timed; the graphs stay for
            // later runs (VNE_TUNE_GRAPH=0: a few direct-launched steps)
            RunOpts o;
            o.collect = false;
            o.graph_trial = env_int("VNE_TUNE_GRAPH", 1) != 0;
            o.steps = o.graph_trial ? p->k : std::min(3, p->k);
            o.tile = t;
            if ((st = run_lanczos(c, set, p, ps, desing, o)) != VNE_OK) break;   // warm-up
            hipError_t e = hipEventRecord(e0, c->stream);
            if (e == hipSuccess && (st = run_lanczos(c, set, p, ps, desing, o)) != VNE_OK) break;
            if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                st = hip_fail(c, e, "autotune timing");
                break;
            }
            if (ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        VNE_TRY(st);
    }
    p->mt = best;
    c->tuned[sig.str()] = best;
    if (!c->tune_file.empty()) {
        std::ofstream f(c->tune_file, std::ios::app);
        if (f) f << sig.str() << " " << best << "\n";
    }
    return VNE_OK;
}

vne_status check_flags(vne_ctx *c, int32_t fl) {
    if (fl & 2) return fail(c, VNE_ENUMERIC, "Cholesky of the sketch Gram matrix failed (rank-deficient sketch)");
    if (fl & 1) return fail(c, VNE_ENUMERIC, "non-finite start vector or Lanczos coefficient");
    if (fl & 4) return fail(c, VNE_ENUMERIC, "tridiagonal QR did not converge");
    if (fl & 8) return fail(c, VNE_ENUMERIC, "tridiagonal QR rotation record overflowed");
    return VNE_OK;
}

// Results of every graph of the plan: one device-to-host copy per array,
// then scattered into out[q] (m[q] columns, k[q] steps).  Also reads the
// flag word of the plan (and of extra, if given) and synchronises.
vne_status copy_out(vne_ctx *c, Plan *p, const int32_t *m, const int32_t *k, vne_result *out, Plan *extra) {
    hipStream_t s = c->stream;
    const int G = p->G;
    const size_t cols = (size_t)G * p->m_pad;
    bool any_quad = false, any_alpha = false, any_beta = false, any_keff = false, any_norm = false;
    for (int q = 0; q < G; ++q) {
        any_quad |= out[q].quad != nullptr;
        any_alpha |= out[q].alpha != nullptr;
        any_beta |= out[q].beta != nullptr;
        any_keff |= out[q].k_eff != nullptr;
        any_norm |= out[q].norm2 != nullptr;
    }
    // every array goes into one pinned staging buffer of the plan, so the
    // copies queue without waiting and the call synchronises once
    const size_t n_est = (size_t)G, n_psi = any_quad ? cols : 0, n_nrm = any_norm ? cols : 0;
    const size_t n_al = any_alpha ? cols * p->k : 0, n_be = any_beta ? cols * p->k : 0;
    const size_t n_ke = any_keff ? cols : 0;
    const size_t need = 8 * (n_est + n_psi + n_nrm + n_al + n_be) + 4 * n_ke + 8;
    if (p->h_stage_bytes < need) {
        if (p->h_stage) HIP_TRY(c, hipHostFree(p->h_stage));
        p->h_stage = nullptr;
        p->h_stage_bytes = 0;
        HIP_TRY(c, hipHostMalloc(&p->h_stage, need, hipHostMallocDefault));
        p->h_stage_bytes = need;
    }
    double *est = (double *)p->h_stage;
    double *psi = est + n_est, *nrm = psi + n_psi, *al = nrm + n_nrm, *be = al + n_al;
    int32_t *ke = (int32_t *)(be + n_be);
    int32_t *fl = ke + n_ke;
    fl[0] = fl[1] = 0;
    HIP_TRY(c, hipMemcpyAsync(est, p->estimate.p, n_est * 8, hipMemcpyDeviceToHost, s));
    if (n_psi) HIP_TRY(c, hipMemcpyAsync(psi, p->psi.p, n_psi * 8, hipMemcpyDeviceToHost, s));
    if (n_nrm) HIP_TRY(c, hipMemcpyAsync(nrm, p->norm2.p, n_nrm * 8, hipMemcpyDeviceToHost, s));
    if (n_ke) HIP_TRY(c, hipMemcpyAsync(ke, p->k_eff.p, n_ke * 4, hipMemcpyDeviceToHost, s));
    if (n_al) HIP_TRY(c, hipMemcpyAsync(al, p->alpha.p, n_al * 8, hipMemcpyDeviceToHost, s));
    if (n_be) HIP_TRY(c, hipMemcpyAsync(be, p->beta.p, n_be * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(&fl[0], p->flags.p, 4, hipMemcpyDeviceToHost, s));
    if (extra) HIP_TRY(c, hipMemcpyAsync(&fl[1], extra->flags.p, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    if (c->timing) VNE_TRY(collect_timing(c));
    for (int q = 0; q < G; ++q) {
        const size_t c0 = (size_t)q * p->m_pad;
        vne_result &o = out[q];
        o.estimate = est[q];
        if (o.quad) std::memcpy(o.quad, psi + c0, (size_t)m[q] * 8);
        if (o.norm2) std::memcpy(o.norm2, nrm + c0, (size_t)m[q] * 8);
        if (o.k_eff) std::memcpy(o.k_eff, ke + c0, (size_t)m[q] * 4);
        for (int col = 0; col < m[q]; ++col) {
            if (o.alpha) std::memcpy(o.alpha + (size_t)col * k[q], al + (c0 + col) * p->k, (size_t)k[q] * 8);
            if (o.beta) std::memcpy(o.beta + (size_t)col * k[q], be + (c0 + col) * p->k, (size_t)k[q] * 8);
        }
    }
    return check_flags(c, fl[0] | fl[1]);
}

vne_status hutchpp_run(vne_ctx *c, GraphSet *set, int nr, int nh, int g_col0, int k, uint64_t seed, bool fp64,
                       bool desing, Plan **sk_out, Plan **q_out, const void *q_src, int q_ld) {
    const int m = nr + nh;
    if (nr < 1 || nh < 0 || nr > 128) return fail(c, VNE_ENOTSUP, "Hutch++ needs 1 <= n_sketch <= min(m, 128)");
    const size_t es = fp64 ? 8 : 4;
    Plan *sk = nullptr, *q = nullptr;
    if (!q_src) VNE_TRY(get_plan(c, set, nr, k, fp64, true, 1, &sk));
    VNE_TRY(get_plan(c, set, m, k, fp64, false, 2, &q));
    const int64_t n = set->n;
    // the Hutch++ workspace of the quadratic-form plan depends on N_r, which
    // the plan's key (m, k) does not fix: every buffer is checked against
    // this call's size and replaced when too small
    auto ensure = [&](DevBuf *b, size_t bytes) -> vne_status {
        if (b->p && b->bytes >= bytes) return VNE_OK;
        dev_free(c, b);
        return dev_alloc(c, b, bytes);
    };
    {
        const int64_t gd = std::max(gram_scratch_doubles((int32_t)n, nr, nr),
                                    gram_scratch_doubles((int32_t)n, nr, std::max(nh, 1)));
        VNE_TRY(ensure(&q->S, (size_t)nr * k * 8));
        VNE_TRY(ensure(&q->B, (size_t)n * m * es));
        VNE_TRY(ensure(&q->gram_part, (size_t)gd * 8));
        VNE_TRY(ensure(&q->gram, (size_t)nr * std::max(nr, nh) * 8));
        VNE_TRY(ensure(&q->rinv, (size_t)nr * nr * 8));
        VNE_TRY(ensure(&q->rot, (size_t)nr * rot_capacity(k) * kRotBytes));
    }
    q->h_graph_k = {k};
    q->h_graph_m = {m};
    hipStream_t s = c->stream;
    const int64_t *keys = (const int64_t *)set->keys.p;
    ProbeSpec ps;
    ps.gen = GEN_RADEMACHER;
    ps.seeds = {seed};
    // column tiles of the Lanczos runs, timed on Rademacher blocks of their
    // widths (the speed of a step does not depend on the values; the runs
    // below probe their own blocks again)
    VNE_TRY(autotune(c, set, q, ps, desing));
    if (q_src) {
        // Q of an earlier run of the same sketch (n x nr, leading dimension
        // q_ld, another plan's buffer): copied into the first nr columns
        if (q_src != q->B.p || q_ld != m)
            HIP_TRY(c, hipMemcpy2DAsync(q->B.p, (size_t)m * es, q_src, (size_t)q_ld * es, (size_t)nr * es,
                                        (size_t)n, hipMemcpyDeviceToDevice, s));
        if (nh > 0) HIP_TRY(c, launch_rademacher_fill(q->B.p, fp64, (int32_t)n, nh, m, nr, g_col0, seed, keys, s));
    } else {
        sk->h_graph_k = {k};
        sk->h_graph_m = {nr};
        VNE_TRY(autotune(c, set, sk, ps, desing));
        // 1. sketch: k Lanczos steps on Omega (kept basis), then Y = f(A) Omega by eq. (4.3)
        VNE_TRY(run_lanczos(c, set, sk, ps, desing));
        HIP_TRY(c, launch_fT_e1((const double *)sk->alpha.p, (const double *)sk->beta.p,
                                (const int32_t *)sk->k_eff.p, k, nr, (double *)q->S.p, q->rot.p,
                                (int32_t *)sk->flags.p, s, fp64));
        const int64_t step_stride = n * sk->m_pad;
        HIP_TRY(c, launch_reconstruct(sk->Vstore.p, fp64, step_stride, sk->m_pad, (const double *)q->S.p,
                                      (const double *)sk->norm2.p, k, (int32_t)n, nr, q->B.p, m, s));
        // 2. G block, raw +-1 in the columns after the sketch (hash columns
        // g_col0, g_col0 + 1, ...)
        if (nh > 0) HIP_TRY(c, launch_rademacher_fill(q->B.p, fp64, (int32_t)n, nh, m, nr, g_col0, seed, keys, s));
        // 3. Q = orth(Y) by CholeskyQR2 (FP64 Gram and triangular factors,
        // two passes, in place): the first pass leaves an orthogonality
        // error of about u cond(Y)^2, the second brings it to the rounding
        // of Q's storage
        for (int pass = 0; pass < 2; ++pass) {
            HIP_TRY(c, launch_gram(q->B.p, m, q->B.p, m, fp64, (int32_t)n, nr, nr, (double *)q->gram_part.p,
                                   (double *)q->gram.p, s));
            HIP_TRY(c, launch_cholinv((double *)q->gram.p, (double *)q->rinv.p, nr, (int32_t *)sk->flags.p, s));
            HIP_TRY(c, launch_apply(q->B.p, m, (const double *)q->rinv.p, nr, nr, q->B.p, m, fp64, (int32_t)n, 0,
                                    s));
        }
    }
    // 4. G~ = G - Q (Q^T G)
    if (nh > 0) {
        char *Gp = (char *)q->B.p + (size_t)nr * es;
        HIP_TRY(c, launch_gram(q->B.p, m, Gp, m, fp64, (int32_t)n, nr, nh, (double *)q->gram_part.p,
                               (double *)q->gram.p, s));
        HIP_TRY(c, launch_apply(q->B.p, m, (const double *)q->gram.p, nr, nh, Gp, m, fp64, (int32_t)n, 1, s));
    }
    // 5. quadratic forms of [Q | G~] and the Hutch++ combination (3.9)
    ProbeSpec pq;
    pq.gen = GEN_DENSE;
    pq.dense = q->B.p;
    pq.ld_dense = m;
    VNE_TRY(run_lanczos(c, set, q, pq, desing));
    HIP_TRY(c, launch_combine((const double *)q->psi.p, m, 2, nr, (double *)q->estimate.p, s));
    if (sk_out) *sk_out = sk;
    *q_out = q;
    return VNE_OK;
}

vne_status estimate_hutchpp(vne_ctx *c, GraphSet *set, const vne_probes *pr, int k, bool fp64, bool desing,
                            vne_result *out) {
    const int nr = pr->n_sketch, m = pr->m;
    if (nr < 1 || m < nr || nr > 128) return fail(c, VNE_ENOTSUP, "Hutch++ needs 1 <= n_sketch <= min(m, 128)");
    Plan *sk = nullptr, *q = nullptr;
    // the Hutchinson columns follow the sketch's in the hash (columns nr .. m - 1)
    VNE_TRY(hutchpp_run(c, set, nr, m - nr, nr, k, pr->seed, fp64, desing, &sk, &q));
    const int32_t mm = m, kk = k;
    return copy_out(c, q, &mm, &kk, out, sk);
}

// Probe spec of a set's queries (one probe kind): Rademacher seeds, or the
// colours / dense blocks copied into the plan's buffers in stacked row order
// (a single graph's device arrays are used in place).
vne_status make_probe_spec(vne_ctx *c, GraphSet *set, Plan *p, const vne_probes *pr, int m_max, bool fp64,
                           ProbeSpec *ps, int *combine_kind) {
    const int G = set->G;
    const int kind = pr[0].kind;
    const size_t es = fp64 ? 8 : 4;
    *combine_kind = 0;
    switch (kind) {
        case VNE_PROBE_RADEMACHER:
            ps->gen = GEN_RADEMACHER;
            for (int q = 0; q < G; ++q) ps->seeds.push_back(pr[q].seed);
            break;
        case VNE_PROBE_COLORING: {
            ps->gen = GEN_COLORING;
            *combine_kind = 1;
            if (G == 1 && pr[0].location == VNE_DEVICE) {
                if (!pr[0].colors) return fail(c, VNE_EINVAL, "colors is NULL");
                ps->colors = pr[0].colors;
                break;
            }
            std::vector<int32_t> col(set->n);
            for (int q = 0; q < G; ++q) {
                if (!pr[q].colors || pr[q].location != VNE_HOST)
                    return fail(c, VNE_EINVAL, "colors must be host arrays in a batch");
                const int64_t r0 = set->h_row_begin[q], nq = set->h_row_begin[q + 1] - r0;
                for (int64_t i = 0; i < nq; ++i) {
                    const int32_t v = pr[q].colors[i];
                    if (v < 0 || v >= pr[q].m)
                        return fail(c, VNE_EINVAL, "colour out of range at row " + std::to_string(i));
                    col[r0 + i] = v;
                }
            }
            if (!p->colors.p) VNE_TRY(dev_alloc(c, &p->colors, (size_t)set->n * 4));
            HIP_TRY(c, hipMemcpyAsync(p->colors.p, col.data(), (size_t)set->n * 4, hipMemcpyHostToDevice, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            ps->colors = (const int32_t *)p->colors.p;
            break;
        }
        case VNE_PROBE_DENSE: {
            ps->gen = GEN_DENSE;
            if (G == 1 && pr[0].location == VNE_DEVICE) {
                if (!pr[0].dense) return fail(c, VNE_EINVAL, "dense is NULL");
                ps->dense = pr[0].dense;
                ps->ld_dense = pr[0].m;
                break;
            }
            std::vector<char> buf((size_t)set->n * m_max * es, 0);
            for (int q = 0; q < G; ++q) {
                if (!pr[q].dense || pr[q].location != VNE_HOST)
                    return fail(c, VNE_EINVAL, "dense blocks must be host arrays in a batch");
                const int64_t r0 = set->h_row_begin[q], nq = set->h_row_begin[q + 1] - r0;
                for (int64_t i = 0; i < nq; ++i)
                    std::memcpy(buf.data() + (size_t)(r0 + i) * m_max * es,
                                (const char *)pr[q].dense + (size_t)i * pr[q].m * es, (size_t)pr[q].m * es);
            }
            if (!p->dense.p) VNE_TRY(dev_alloc(c, &p->dense, buf.size()));
            HIP_TRY(c, hipMemcpyAsync(p->dense.p, buf.data(), buf.size(), hipMemcpyHostToDevice, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            ps->dense = p->dense.p;
            ps->ld_dense = m_max;
            break;
        }
        default:
            return fail(c, VNE_EINVAL, "unknown probe kind");
    }
    return VNE_OK;
}

// One query per graph of the set, all graphs in one stacked launch per step.
vne_status estimate_set(vne_ctx *c, GraphSet *set, const vne_probes *pr, const int32_t *k_steps, bool fp64,
                        bool desing, vne_result *out) {
    const int G = set->G;
    const int kind = pr[0].kind;
    int k_max = 0, m_max = 0;
    std::vector<int32_t> ms(G);
    for (int q = 0; q < G; ++q) {
        if (pr[q].kind != kind) return fail(c, VNE_ENOTSUP, "a batch takes one probe kind");
        if (pr[q].m < 1) return fail(c, VNE_EINVAL, "probe count m must be >= 1");
        if (k_steps[q] < 1 || k_steps[q] > kMaxSteps) return fail(c, VNE_EINVAL, "k_steps must be in [1, 128]");
        k_max = std::max(k_max, (int)k_steps[q]);
        m_max = std::max(m_max, (int)pr[q].m);
        ms[q] = pr[q].m;
    }
    if (m_max > (1 << 20)) return fail(c, VNE_ENOTSUP, "probe count too large");
    Plan *p = nullptr;
    VNE_TRY(get_plan(c, set, m_max, k_max, fp64, false, 0, &p));
    p->h_graph_k.assign(k_steps, k_steps + G);
    p->h_graph_m = ms;
    ProbeSpec ps;
    int combine_kind = 0;
    VNE_TRY(make_probe_spec(c, set, p, pr, m_max, fp64, &ps, &combine_kind));
    VNE_TRY(autotune(c, set, p, ps, desing));
    VNE_TRY(run_lanczos(c, set, p, ps, desing));
    HIP_TRY(c, launch_combine_graphs((const double *)p->psi.p, p->m_pad, (const int32_t *)p->graph_m.p, G,
                                     combine_kind, (double *)p->estimate.p, c->stream));
    return copy_out(c, p, ms.data(), k_steps, out, nullptr);
}

vne_status check_mode(vne_ctx *c, uint32_t mode) {
    if (mode & ~(uint32_t)(VNE_MODE_F64 | VNE_MODE_DESING)) return fail(c, VNE_EINVAL, "unknown mode bits");
    return VNE_OK;
}

}  // namespace rt
}  // namespace vne

using namespace vne::rt;

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
    {
        std::string err;
        if (noalloc_attach(device, &err) != VNE_OK) {
            g_create_error = err;
            return VNE_EDEVICE;
        }
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
    if (const char *tf = getenv("VNE_AUTOTUNE_CACHE")) {
        c->tune_file = tf;
        std::ifstream f(tf);
        std::string sig;
        int t;
        while (f >> sig >> t)
            if (t > 0) c->tuned[sig] = t;
    }
    *out = c;
    return VNE_OK;
}

extern "C" void vne_ctx_destroy(vne_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto &kv : c->sets) free_set(c, kv.second.get());
    c->sets.clear();
    for (auto &g : c->graphs)
        if (g) free_graph(c, g.get());
    for (hipStream_t cs : c->chain_streams) (void)hipStreamDestroy(cs);
    for (hipEvent_t e : c->chain_events) (void)hipEventDestroy(e);
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
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    c->err.clear();
    if (!csr || !graph_id) return fail(c, VNE_EINVAL, "NULL argument");
    HIP_TRY(c, hipSetDevice(c->device));
    const int64_t n = csr->n, nnz = csr->nnz;
    if (n < 1 || nnz < 0 || nnz > INT32_MAX || n > INT32_MAX - 1) return fail(c, VNE_EINVAL, "bad sizes");
    if (csr->location != VNE_HOST && csr->location != VNE_DEVICE) return fail(c, VNE_EINVAL, "bad location");
    if (csr->value_dtype != VNE_F32 && csr->value_dtype != VNE_F64) return fail(c, VNE_EINVAL, "bad value dtype");
    auto g = std::make_unique<Graph>();
    // host view of the three arrays (copied back for device input)
    const size_t vs = csr->value_dtype == VNE_F64 ? 8 : 4;
    std::vector<char> h_val;
    vne_csr hv = *csr;
    if (csr->location == VNE_DEVICE) {
        if (!csr->row_ptr || (nnz && (!csr->col_idx || !csr->values))) return fail(c, VNE_EINVAL, "NULL CSR array");
        g->h_row_ptr.resize(n + 1);
        g->h_col.resize(nnz);
        h_val.resize(nnz * vs);
        HIP_TRY(c, hipMemcpy(g->h_row_ptr.data(), csr->row_ptr, (n + 1) * 4, hipMemcpyDeviceToHost));
        if (nnz) {
            HIP_TRY(c, hipMemcpy(g->h_col.data(), csr->col_idx, nnz * 4, hipMemcpyDeviceToHost));
            HIP_TRY(c, hipMemcpy(h_val.data(), csr->values, nnz * vs, hipMemcpyDeviceToHost));
        }
        hv.row_ptr = g->h_row_ptr.data();
        hv.col_idx = g->h_col.data();
        hv.values = h_val.data();
        hv.location = VNE_HOST;
    }
    std::string msg;
    vne_status st = validate_host_csr(&hv, flags, &msg);
    if (st != VNE_OK) return fail(c, st, msg);
    if (csr->location == VNE_HOST) {
        g->h_row_ptr.assign(hv.row_ptr, hv.row_ptr + n + 1);
        g->h_col.assign(hv.col_idx, hv.col_idx + nnz);
    }
    g->n = n;
    g->nnz = nnz;
    g->scale = csr->scale;
    g->h_val.resize(nnz);
    for (int64_t p = 0; p < nnz; ++p)
        g->h_val[p] = csr->value_dtype == VNE_F64 ? ((const double *)hv.values)[p] : (double)((const float *)hv.values)[p];
    g->zero_rowsum = true;
    double amax = 0.0, fro2 = 0.0, tr = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double rs = 0.0, ra = 0.0;
        for (int32_t q = g->h_row_ptr[i]; q < g->h_row_ptr[i + 1]; ++q) {
            const double v = g->h_val[q];
            rs += v;
            ra += std::fabs(v);
            fro2 += v * v;
            if (g->h_col[q] == i) tr += v;
        }
        g->zero_rowsum = g->zero_rowsum && rs == 0.0;
        amax = std::max(amax, ra);
    }
    g->lambda_ub = std::fabs(g->scale) * amax;
    g->fro2 = g->scale * g->scale * fro2;
    g->trace = g->scale * tr;
    g->h_keys.resize(n);
    for (int64_t i = 0; i < n; ++i) g->h_keys[i] = csr->node_keys ? csr->node_keys[i] : i;
    if (csr->location == VNE_DEVICE) {
        g->d_row_ptr = csr->row_ptr;
        g->d_col = csr->col_idx;
    } else {
        if ((st = upload(c, &g->row_ptr, g->h_row_ptr.data(), n + 1)) != VNE_OK ||
            (st = upload(c, &g->col, g->h_col.data(), nnz)) != VNE_OK) {
            free_graph(c, g.get());
            return st;
        }
        g->d_row_ptr = (const int32_t *)g->row_ptr.p;
        g->d_col = (const int32_t *)g->col.p;
    }
    // work schedule: segments of long rows, cost-balanced blocks
    const int seg_len = std::max(1, env_int("VNE_SEG_LEN", 64));
    const int max_blocks = std::max(8, env_int("VNE_MAX_BLOCKS", 1024));
    const int64_t total_cost = nnz + 4 * n;
    const int64_t cpb = std::max<int64_t>(256, (total_cost + max_blocks - 1) / max_blocks);
    g->sched = build_schedule(g->h_row_ptr.data(), n, seg_len, cpb, max_blocks);
    g->alive = true;
    c->graphs.push_back(std::move(g));
    const int32_t gid = (int32_t)c->graphs.size() - 1;
    // the device arrays of the graph alone (values, keys, work schedule) are
    // built here, so that later estimates on it allocate only workspaces
    GraphSet *set = nullptr;
    if ((st = get_set(c, {gid}, &set)) != VNE_OK) {
        free_graph(c, c->graphs[gid].get());
        return st;
    }
    *graph_id = gid;
    return VNE_OK;
}

extern "C" vne_status vne_graph_release(vne_ctx *c, int32_t gid) {
    if (!c) return VNE_EINVAL;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    c->err.clear();
    Graph *g = get_graph(c, gid);
    if (!g) return fail(c, VNE_EINVAL, "unknown graph id");
    if (g->in_use > 0) return fail(c, VNE_EBUSY, "graph has queries in a running server");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (auto it = c->sets.begin(); it != c->sets.end();) {
        if (std::find(it->first.begin(), it->first.end(), gid) != it->first.end()) {
            free_set(c, it->second.get());
            it = c->sets.erase(it);
        } else {
            ++it;
        }
    }
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

extern "C" vne_status vne_entropy_estimate(vne_ctx *c, int32_t gid, const vne_probes *pr, int32_t k,
                                           uint32_t mode, vne_result *out) {
    if (!c) return VNE_EINVAL;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    c->err.clear();
    if (!pr || !out) return fail(c, VNE_EINVAL, "NULL argument");
    if (!get_graph(c, gid)) return fail(c, VNE_EINVAL, "unknown graph id");
    if (k < 1 || k > kMaxSteps) return fail(c, VNE_EINVAL, "k_steps must be in [1, 128]");
    if (pr->m < 1) return fail(c, VNE_EINVAL, "probe count m must be >= 1");
    VNE_TRY(check_mode(c, mode));
    HIP_TRY(c, hipSetDevice(c->device));
    GraphSet *set = nullptr;
    VNE_TRY(get_set(c, {gid}, &set));
    const bool fp64 = (mode & VNE_MODE_F64) != 0;
    const bool desing = (mode & VNE_MODE_DESING) != 0;
    if (desing && !set->zero_rowsum)
        return fail(c, VNE_EINVAL, "VNE_MODE_DESING needs a matrix whose rows sum to zero (A 1 = 0)");
    if (pr->kind == VNE_PROBE_HUTCHPP) return estimate_hutchpp(c, set, pr, k, fp64, desing, out);
    return estimate_set(c, set, pr, &k, fp64, desing, out);
}

extern "C" vne_status vne_last_plan(const vne_ctx *c, int32_t *tile, int32_t *m_pad) {
    if (!c || !tile || !m_pad) return VNE_EINVAL;
    std::lock_guard<std::recursive_mutex> lock(const_cast<vne_ctx *>(c)->mu);
    *tile = c->last_tile;
    *m_pad = c->last_m_pad;
    return VNE_OK;
}

extern "C" vne_status vne_error_bounds(vne_ctx *c, int32_t m, int32_t k, const double *alpha, const double *beta,
                                       const int32_t *k_eff, const double *norm2, int32_t steps, double lam_lo,
                                       double lam_hi, int32_t n_grid, double *lo, double *hi) {
    if (!c) return VNE_EINVAL;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    c->err.clear();
    if (!alpha || !beta || !k_eff || !norm2 || !lo || !hi) return fail(c, VNE_EINVAL, "NULL argument");
    if (m < 1 || k < 1 || k > kMaxSteps || steps < 1 || steps > k)
        return fail(c, VNE_EINVAL, "need m >= 1, 1 <= steps <= k <= 128");
    if (!(lam_lo > 0.0) || !(lam_hi > lam_lo) || !std::isfinite(lam_hi))
        return fail(c, VNE_EINVAL, "need 0 < lam_lo < lam_hi");
    if (n_grid < 2 || n_grid > (1 << 16)) return fail(c, VNE_EINVAL, "n_grid must be in [2, 65536]");
    HIP_TRY(c, hipSetDevice(c->device));
    DevBuf d_al, d_be, d_ke, d_nr, d_lo, d_hi, d_args, d_map, d_fl;
    auto fin = [&](vne_status st) {
        DevBuf *all[] = {&d_al, &d_be, &d_ke, &d_nr, &d_lo, &d_hi, &d_args, &d_map, &d_fl};
        for (DevBuf *b : all) dev_free(c, b);
        return st;
    };
    const int ng = (m + 3) / 4;
    std::vector<int2> map(ng);
    for (int i = 0; i < ng; ++i) map[i] = make_int2(0, i);
    vne_status st = VNE_OK;
    if ((st = upload(c, &d_al, alpha, (size_t)m * k)) != VNE_OK || (st = upload(c, &d_be, beta, (size_t)m * k)) != VNE_OK ||
        (st = upload(c, &d_ke, k_eff, (size_t)m)) != VNE_OK || (st = upload(c, &d_nr, norm2, (size_t)m)) != VNE_OK ||
        (st = dev_alloc(c, &d_lo, (size_t)m * 8)) != VNE_OK || (st = dev_alloc(c, &d_hi, (size_t)m * 8)) != VNE_OK ||
        (st = upload(c, &d_map, map.data(), map.size())) != VNE_OK || (st = dev_alloc(c, &d_fl, 4)) != VNE_OK)
        return fin(st);
    BoundArgs a{};
    a.alpha = (const double *)d_al.p;
    a.beta = (const double *)d_be.p;
    a.k_eff = (const int32_t *)d_ke.p;
    a.norm2 = (const double *)d_nr.p;
    a.k = k;
    a.m = m;
    a.steps = steps;
    a.lam_lo = lam_lo;
    a.lam_hi = lam_hi;
    a.n_grid = n_grid;
    a.lo = (double *)d_lo.p;
    a.hi = (double *)d_hi.p;
    a.flags = (int32_t *)d_fl.p;
    if ((st = upload(c, &d_args, &a, 1)) != VNE_OK) return fin(st);
    int32_t fl = 0;
    hipError_t e = hipMemsetAsync(d_fl.p, 0, 4, c->stream);
    if (e == hipSuccess) e = launch_error_bound((const BoundArgs *)d_args.p, (const int2 *)d_map.p, ng, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(lo, d_lo.p, (size_t)m * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(hi, d_hi.p, (size_t)m * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&fl, d_fl.p, 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fin(hip_fail(c, e, "error bound kernel"));
    fin(VNE_OK);
    return check_flags(c, fl);
}

extern "C" vne_status vne_entropy_estimate_batch(vne_ctx *c, int32_t n_queries, const int32_t *graph_ids,
                                                 const vne_probes *probes, const int32_t *k_steps, uint32_t mode,
                                                 vne_result *out) {
    if (!c) return VNE_EINVAL;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    c->err.clear();
    if (n_queries < 1 || !graph_ids || !probes || !k_steps || !out)
        return fail(c, VNE_EINVAL, "NULL argument or empty batch");
    VNE_TRY(check_mode(c, mode));
    HIP_TRY(c, hipSetDevice(c->device));
    std::vector<int32_t> ids(graph_ids, graph_ids + n_queries);
    for (int q = 0; q < n_queries; ++q) {
        if (!get_graph(c, ids[q])) return fail(c, VNE_EINVAL, "unknown graph id " + std::to_string(ids[q]));
        if (probes[q].kind == VNE_PROBE_HUTCHPP) return fail(c, VNE_ENOTSUP, "Hutch++ queries are not batched");
    }
    GraphSet *set = nullptr;
    VNE_TRY(get_set(c, ids, &set));
    const bool fp64 = (mode & VNE_MODE_F64) != 0;
    const bool desing = (mode & VNE_MODE_DESING) != 0;
    if (desing && !set->zero_rowsum)
        return fail(c, VNE_EINVAL, "VNE_MODE_DESING needs matrices whose rows sum to zero (A 1 = 0)");
    return estimate_set(c, set, probes, k_steps, fp64, desing, out);
}
