// Quadratic forms with per-vector a-posteriori stopping (Theorem 4.8 as the
// stopping rule of step 3 of Algorithm 2), and the probing method with a
// relative accuracy target (Section 5, probing method implementation;
// Algorithm 2).  Host code: colourings run on the host (Algorithm 1), every
// Lanczos pass runs through run_lanczos on the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ctx_internal.h"
#include "internal.h"
#include "kernels.h"
#include "probing_host.h"

using namespace vne;
using namespace vne::rt;

namespace {

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

struct PassOut {
    double estimate = 0.0;
    std::vector<double> psi;
    std::vector<int32_t> steps;    // stop step per vector (0: never met its tolerance, ran k_max steps)
    int steps_run = 0;             // steps the block ran
    int unconverged = 0;
};

// One run with per-vector stopping on a set of one graph; tol is host [m].
// out (may be NULL) receives quad / alpha / beta / k_eff / norm2 when asked.
vne_status adaptive_run(vne_ctx *c, GraphSet *set, const vne_probes *pr, int k_max, bool fp64, bool desing,
                        const double *tol, double lam_lo, double lam_hi, int n_grid, bool estimate, vne_result *out,
                        PassOut *po) {
    const int m = pr->m;
    Plan *p = nullptr;
    VNE_TRY(get_plan(c, set, m, k_max, fp64, false, 0, &p));
    p->h_graph_k.assign(1, k_max);
    p->h_graph_m.assign(1, m);
    ProbeSpec ps;
    int combine_kind = 0;
    VNE_TRY(make_probe_spec(c, set, p, pr, m, fp64, &ps, &combine_kind));
    if (!p->col_tol.p) VNE_TRY(dev_alloc(c, &p->col_tol, (size_t)p->m_pad * 8));
    HIP_TRY(c, hipMemcpyAsync(p->col_tol.p, tol, (size_t)m * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    VNE_TRY(autotune(c, set, p, ps, desing));
    RunOpts o;
    o.adaptive = true;
    o.lam_lo = lam_lo;
    o.lam_hi = lam_hi;
    o.n_grid = n_grid;
    o.estimate = estimate;
    VNE_TRY(run_lanczos(c, set, p, ps, desing, o));
    HIP_TRY(c, launch_combine_graphs((const double *)p->psi.p, p->m_pad, (const int32_t *)p->graph_m.p, 1,
                                     combine_kind, (double *)p->estimate.p, c->stream));
    hipStream_t s = c->stream;
    po->psi.assign(m, 0.0);
    po->steps.assign(m, 0);
    int32_t fl = 0;
    HIP_TRY(c, hipMemcpyAsync(&po->estimate, p->estimate.p, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(po->psi.data(), p->psi.p, (size_t)m * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(po->steps.data(), p->col_stop.p, (size_t)m * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(&fl, p->flags.p, 4, hipMemcpyDeviceToHost, s));
    if (out) {
        const size_t mk = (size_t)m * p->k * 8;
        if (out->alpha) HIP_TRY(c, hipMemcpyAsync(out->alpha, p->alpha.p, mk, hipMemcpyDeviceToHost, s));
        if (out->beta) HIP_TRY(c, hipMemcpyAsync(out->beta, p->beta.p, mk, hipMemcpyDeviceToHost, s));
        if (out->k_eff) HIP_TRY(c, hipMemcpyAsync(out->k_eff, p->k_eff.p, (size_t)m * 4, hipMemcpyDeviceToHost, s));
        if (out->norm2) HIP_TRY(c, hipMemcpyAsync(out->norm2, p->norm2.p, (size_t)m * 8, hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(c, hipStreamSynchronize(s));
    if (c->timing) VNE_TRY(collect_timing(c));
    VNE_TRY(check_flags(c, fl));
    po->steps_run = p->steps_run;
    po->unconverged = 0;
    for (int j = 0; j < m; ++j) po->unconverged += po->steps[j] == 0;
    if (out) {
        out->estimate = po->estimate;
        if (out->quad) std::memcpy(out->quad, po->psi.data(), (size_t)m * 8);
    }
    return VNE_OK;
}

struct Pass {
    int d = 0, n_colors = 0;
    std::vector<int32_t> colors;
    PassOut out;
};

}  // namespace

extern "C" vne_status vne_entropy_estimate_adaptive(vne_ctx *c, int32_t gid, const vne_probes *pr, int32_t k_max,
                                                    uint32_t mode, const vne_stop_rule *rule, vne_result *out,
                                                    int32_t *steps_out) {
    if (!c) return VNE_EINVAL;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    c->err.clear();
    if (!pr || !out || !rule || !rule->tol) return fail(c, VNE_EINVAL, "NULL argument");
    if (!get_graph(c, gid)) return fail(c, VNE_EINVAL, "unknown graph id");
    if (k_max < 3 || k_max > kMaxSteps) return fail(c, VNE_EINVAL, "k_max must be in [3, 128]");
    if (pr->m < 1 || pr->m > (1 << 20)) return fail(c, VNE_EINVAL, "probe count m must be in [1, 2^20]");
    if (pr->kind == VNE_PROBE_HUTCHPP)
        return fail(c, VNE_ENOTSUP, "per-vector stopping takes RADEMACHER, COLORING or DENSE probes");
    const int n_grid = rule->n_grid == 0 ? kBoundGrid : rule->n_grid;
    if (n_grid < 2 || n_grid > 65536) return fail(c, VNE_EINVAL, "n_grid must be in [2, 65536]");
    if (!(rule->lam_lo > 0.0) || !(rule->lam_hi > rule->lam_lo) || !std::isfinite(rule->lam_hi))
        return fail(c, VNE_EINVAL, "need 0 < lam_lo < lam_hi");
    if (rule->stop != VNE_STOP_BOUND && rule->stop != VNE_STOP_ESTIMATE)
        return fail(c, VNE_EINVAL, "stop must be VNE_STOP_BOUND or VNE_STOP_ESTIMATE");
    for (int j = 0; j < pr->m; ++j)
        if (!(rule->tol[j] >= 0.0) || !std::isfinite(rule->tol[j]))
            return fail(c, VNE_EINVAL, "tolerance " + std::to_string(j) + " is negative or not finite");
    VNE_TRY(check_mode(c, mode));
    HIP_TRY(c, hipSetDevice(c->device));
    GraphSet *set = nullptr;
    VNE_TRY(get_set(c, {gid}, &set));
    const bool fp64 = (mode & VNE_MODE_F64) != 0;
    const bool desing = (mode & VNE_MODE_DESING) != 0;
    if (desing && !set->zero_rowsum)
        return fail(c, VNE_EINVAL, "VNE_MODE_DESING needs a matrix whose rows sum to zero (A 1 = 0)");
    PassOut po;
    VNE_TRY(adaptive_run(c, set, pr, k_max, fp64, desing, rule->tol, rule->lam_lo, rule->lam_hi, n_grid,
                         rule->stop == VNE_STOP_ESTIMATE, out, &po));
    if (steps_out) std::memcpy(steps_out, po.steps.data(), (size_t)pr->m * 4);
    return VNE_OK;
}

extern "C" vne_status vne_entropy_probing(vne_ctx *c, int32_t gid, const vne_probing_cfg *cfg,
                                          vne_probing_result *res) {
    if (!c) return VNE_EINVAL;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    c->err.clear();
    if (!cfg || !res) return fail(c, VNE_EINVAL, "NULL argument");
    Graph *g = get_graph(c, gid);
    if (!g) return fail(c, VNE_EINVAL, "unknown graph id");
    if (!(cfg->rel_eps > 0.0 && cfg->rel_eps < 1.0)) return fail(c, VNE_EINVAL, "rel_eps must be in (0, 1)");
    if (cfg->select != VNE_SELECT_HEURISTIC && cfg->select != VNE_SELECT_BOUND)
        return fail(c, VNE_EINVAL, "select must be VNE_SELECT_HEURISTIC or VNE_SELECT_BOUND");
    const int d_max = cfg->d_max == 0 ? 16 : cfg->d_max;
    const int k_max = cfg->k_max == 0 ? kMaxSteps : cfg->k_max;
    const double frac = cfg->lam_lo_fraction == 0.0 ? kLamLoFraction : cfg->lam_lo_fraction;
    const int n_grid = cfg->n_grid == 0 ? kBoundGrid : cfg->n_grid;
    if (d_max < 1 || d_max > 64) return fail(c, VNE_EINVAL, "d_max must be in [1, 64]");
    if (k_max < 3 || k_max > kMaxSteps) return fail(c, VNE_EINVAL, "k_max must be in [3, 128]");
    if (!(frac > 0.0 && frac < 1.0)) return fail(c, VNE_EINVAL, "lam_lo_fraction must be in (0, 1)");
    if (n_grid < 2 || n_grid > 65536) return fail(c, VNE_EINVAL, "n_grid must be in [2, 65536]");
    if (cfg->stop != VNE_STOP_BOUND && cfg->stop != VNE_STOP_ESTIMATE)
        return fail(c, VNE_EINVAL, "stop must be VNE_STOP_BOUND or VNE_STOP_ESTIMATE");
    VNE_TRY(check_mode(c, cfg->mode));
    if (!(std::fabs(g->trace - 1.0) < 1e-9 && g->fro2 > 0.0 && g->fro2 < 1.0))
        return fail(c, VNE_EINVAL, "the probing method with a target needs a unit-trace matrix (a density matrix)");
    HIP_TRY(c, hipSetDevice(c->device));
    GraphSet *set = nullptr;
    VNE_TRY(get_set(c, {gid}, &set));
    const bool fp64 = (cfg->mode & VNE_MODE_F64) != 0;
    const bool desing = (cfg->mode & VNE_MODE_DESING) != 0;
    if (desing && !set->zero_rowsum)
        return fail(c, VNE_EINVAL, "VNE_MODE_DESING needs a matrix whose rows sum to zero (A 1 = 0)");

    // scalar results start from zero; the caller's output arrays are kept
    int32_t *colors_out = res->colors, *steps_out = res->steps;
    double *quad_out = res->quad;
    const int32_t quad_cap = res->quad_cap;
    std::memset(res, 0, sizeof(*res));
    res->colors = colors_out;
    res->steps = steps_out;
    res->quad = quad_out;
    res->quad_cap = quad_cap;

    const int64_t n = g->n;
    const double lam_hi = g->lambda_ub, lam_lo = frac * lam_hi;
    const double s_lower = -std::log(g->fro2);
    res->s_lower = s_lower;

    // one distance-d pass: colouring (Algorithm 1, unless given), tolerances
    // of eq. (5.3), Lanczos with per-colour stopping
    auto run_pass = [&](int d, double eps_hat, Pass *ps) -> vne_status {
        auto t0 = Clock::now();
        if (ps->d != d) {
            ps->d = d;
            ps->colors.assign(n, 0);
            ps->n_colors = greedy_color(n, g->h_row_ptr.data(), g->h_col.data(), d, ps->colors.data());
            res->color_ms += ms_since(t0);
        }
        std::vector<double> size(ps->n_colors, 0.0);
        for (int64_t i = 0; i < n; ++i) size[ps->colors[i]] += 1.0;
        std::vector<double> tol(ps->n_colors);
        for (int l = 0; l < ps->n_colors; ++l) tol[l] = eps_hat * size[l] / (double)n;
        vne_probes pr{};
        pr.kind = VNE_PROBE_COLORING;
        pr.m = ps->n_colors;
        pr.location = VNE_HOST;
        pr.colors = ps->colors.data();
        t0 = Clock::now();
        VNE_TRY(adaptive_run(c, set, &pr, k_max, fp64, desing, tol.data(), lam_lo, lam_hi, n_grid,
                             cfg->stop == VNE_STOP_ESTIMATE, nullptr, &ps->out));
        res->lanczos_ms += ms_since(t0);
        res->passes++;
        for (int32_t st : ps->out.steps) res->vector_steps += st > 0 ? st : k_max;
        res->block_steps += ps->out.steps_run;
        return VNE_OK;
    };

    Pass pre[3];
    Pass main_pass;
    const Pass *final_pass = nullptr;
    DistanceChoice ch;
    const double eps_hat0 = 0.5 * cfg->rel_eps * s_lower;
    if (cfg->select == VNE_SELECT_HEURISTIC) {
        {
            // the three colourings from one neighbourhood search
            auto t0 = Clock::now();
            const int32_t ds[3] = {1, 2, 3};
            int32_t *outs[3];
            int32_t nc[3];
            for (int q = 0; q < 3; ++q) {
                pre[q].colors.assign(n, 0);
                outs[q] = pre[q].colors.data();
            }
            greedy_color_multi(n, g->h_row_ptr.data(), g->h_col.data(), ds, 3, outs, nc);
            for (int q = 0; q < 3; ++q) {
                pre[q].d = ds[q];
                pre[q].n_colors = nc[q];
            }
            res->color_ms += ms_since(t0);
        }
        for (int d = 1; d <= 3; ++d) VNE_TRY(run_pass(d, eps_hat0, &pre[d - 1]));
        const double T[3] = {pre[0].out.estimate, pre[1].out.estimate, pre[2].out.estimate};
        for (int i = 0; i < 3; ++i) res->t_pre[i] = T[i];
        res->s_hat = std::max(s_lower, std::max(T[0], std::max(T[1], T[2])));
        res->eps_hat = 0.5 * cfg->rel_eps * res->s_hat;
        ch = probing_heuristic_distance(T, (double)n, lam_hi, res->eps_hat, d_max);
    } else {
        res->s_hat = s_lower;
        res->eps_hat = eps_hat0;
        ch = probing_bound_distance((double)n, lam_hi, res->eps_hat, d_max);
    }
    res->d = ch.d;
    res->fallback = ch.fallback;
    res->capped = ch.capped;
    res->e1 = ch.e1;
    res->q[0] = ch.q[0];
    res->q[1] = ch.q[1];
    if (cfg->select == VNE_SELECT_HEURISTIC && ch.d <= 3) {
        final_pass = &pre[ch.d - 1];
    } else {
        VNE_TRY(run_pass(ch.d, res->eps_hat, &main_pass));
        final_pass = &main_pass;
    }
    res->estimate = final_pass->out.estimate;
    res->n_colors = final_pass->n_colors;
    res->unconverged = final_pass->out.unconverged;
    if (colors_out) std::memcpy(colors_out, final_pass->colors.data(), (size_t)n * 4);
    const int w = std::min<int>(std::max<int32_t>(quad_cap, 0), final_pass->n_colors);
    if (quad_out && w > 0) std::memcpy(quad_out, final_pass->out.psi.data(), (size_t)w * 8);
    if (steps_out && w > 0) std::memcpy(steps_out, final_pass->out.steps.data(), (size_t)w * 4);
    return VNE_OK;
}
