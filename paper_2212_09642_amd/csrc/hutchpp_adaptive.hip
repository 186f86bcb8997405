// Adaptive Hutch++ (Section 3.2, the tail bound eq. (3.10); the adaptive
// Hutch++ implementation of Section 5).  Host code: every round is a
// Hutch++ run of the device path (sketch Lanczos with a kept basis, f(A)
// Omega by eq. (4.3), CholeskyQR2, projection, quadratic forms of
// [Q | G~]); the rule that picks the sketch width and the Hutchinson count
// (hutchpp_rule.h, host only) reads the round's forms on the host.  The
// rule is stated with its declaration in vne.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "ctx_internal.h"
#include "hutchpp_rule.h"
#include "internal.h"
#include "kernels.h"

using namespace vne;
using namespace vne::rt;

namespace {

// hash column of the first deflated (Hutchinson) vector: past every sketch
// width, so the deflated vectors do not depend on N_r
constexpr int kGCol0 = 128;

struct RoundOut {
    double estimate = 0.0;
    std::vector<double> psi;
    const Plan *q = nullptr;         // the run's plan: its B holds [Q | G~]
};

// one Hutch++ run (a round, or the final run on the Q of `from`) and its
// results on the host
vne_status round_run(vne_ctx *c, GraphSet *set, int nr, int nh, int k, uint64_t seed, bool fp64, bool desing,
                     const RoundOut *from, RoundOut *ro) {
    Plan *sk = nullptr, *q = nullptr;
    if (from)
        VNE_TRY(hutchpp_run(c, set, nr, nh, kGCol0, k, seed, fp64, desing, nullptr, &q, from->q->B.p,
                            from->q->m));
    else
        VNE_TRY(hutchpp_run(c, set, nr, nh, kGCol0, k, seed, fp64, desing, &sk, &q));
    hipStream_t s = c->stream;
    const int m = nr + nh;
    ro->psi.assign(m, 0.0);
    ro->q = q;
    int32_t fl[2] = {0, 0};
    HIP_TRY(c, hipMemcpyAsync(&ro->estimate, q->estimate.p, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(ro->psi.data(), q->psi.p, (size_t)m * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(&fl[0], q->flags.p, 4, hipMemcpyDeviceToHost, s));
    if (sk) HIP_TRY(c, hipMemcpyAsync(&fl[1], sk->flags.p, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    return check_flags(c, fl[0] | fl[1]);
}

}  // namespace

extern "C" vne_status vne_hutchpp_adaptive(vne_ctx *c, int32_t gid, const vne_hutchpp_cfg *cfg,
                                           vne_hutchpp_result *res, double *quad, int32_t quad_cap) {
    if (!c) return VNE_EINVAL;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    c->err.clear();
    if (!cfg || !res) return fail(c, VNE_EINVAL, "NULL argument");
    if (!get_graph(c, gid)) return fail(c, VNE_EINVAL, "unknown graph id");
    const int k = cfg->k_steps;
    const int n_pilot = cfg->n_pilot == 0 ? 16 : cfg->n_pilot;
    const int r_first = cfg->r_first == 0 ? 3 : cfg->r_first;
    const int r_max = cfg->r_max == 0 ? std::max(96, r_first) : cfg->r_max;
    const int n_h_max = cfg->n_h_max == 0 ? 4096 : cfg->n_h_max;
    if (k < 1 || k > kMaxSteps) return fail(c, VNE_EINVAL, "k_steps must be in [1, 128]");
    if (!(cfg->delta > 0.0 && cfg->delta < 1.0)) return fail(c, VNE_EINVAL, "delta must be in (0, 1)");
    if (!(cfg->abs_eps >= 0.0) || !std::isfinite(cfg->abs_eps))
        return fail(c, VNE_EINVAL, "abs_eps must be finite and >= 0");
    if (cfg->abs_eps == 0.0 && !(cfg->rel_eps > 0.0 && cfg->rel_eps < 1.0))
        return fail(c, VNE_EINVAL, "rel_eps must be in (0, 1) when abs_eps is 0");
    if (n_pilot < 2 || n_pilot > 1024) return fail(c, VNE_EINVAL, "n_pilot must be in [2, 1024]");
    if (r_first < 1 || r_first > 128) return fail(c, VNE_EINVAL, "r_first must be in [1, 128]");
    if (r_max < r_first || r_max > 128) return fail(c, VNE_EINVAL, "r_max must be in [r_first, 128]");
    if (n_h_max < n_pilot || n_h_max > (1 << 20)) return fail(c, VNE_EINVAL, "n_h_max must be in [n_pilot, 2^20]");
    if (quad_cap < 0 || (quad_cap > 0 && !quad)) return fail(c, VNE_EINVAL, "quad_cap > 0 needs a quad buffer");
    VNE_TRY(check_mode(c, cfg->mode));
    HIP_TRY(c, hipSetDevice(c->device));
    GraphSet *set = nullptr;
    VNE_TRY(get_set(c, {gid}, &set));
    const bool fp64 = (cfg->mode & VNE_MODE_F64) != 0;
    const bool desing = (cfg->mode & VNE_MODE_DESING) != 0;
    if (desing && !set->zero_rowsum)
        return fail(c, VNE_EINVAL, "VNE_MODE_DESING needs a matrix whose rows sum to zero (A 1 = 0)");
    const auto t0 = std::chrono::steady_clock::now();
    std::memset(res, 0, sizeof(*res));
    HutchppRule rule(cfg->rel_eps, cfg->abs_eps, cfg->delta, n_pilot, r_first, r_max, n_h_max);
    std::vector<RoundOut> outs;
    while (const int nr = rule.next()) {
        outs.emplace_back();
        VNE_TRY(round_run(c, set, nr, n_pilot, k, cfg->seed, fp64, desing, nullptr, &outs.back()));
        rule.record(outs.back().estimate, hpp_sample_sd(outs.back().psi.data() + nr, n_pilot));
    }
    const HutchppRound &kb = rule.rounds()[rule.kept()];
    const int nh_final = rule.final_nh();
    // a kept round with the pilot's count is the final run itself (same
    // columns: the device would repeat it bit for bit); otherwise the final
    // run takes the kept round's Q (the rounds have distinct widths, so no
    // later round's plan holds it) and new deflated columns
    RoundOut fin;
    const RoundOut &ro = rule.reuse() ? outs[rule.kept()] : fin;
    if (!rule.reuse())
        VNE_TRY(round_run(c, set, kb.nr, nh_final, k, cfg->seed, fp64, desing, &outs[rule.kept()], &fin));

    res->estimate = ro.estimate;
    res->std_error = hpp_sample_sd(ro.psi.data() + kb.nr, nh_final) / std::sqrt((double)nh_final);
    res->eps_hat = kb.eps_hat;
    res->n_sketch = kb.nr;
    res->n_hutch = nh_final;
    res->capped = rule.capped() ? 1 : 0;
    res->rounds = (int32_t)rule.rounds().size();
    for (size_t i = 0; i < rule.rounds().size() && i < VNE_HUTCHPP_MAX_ROUNDS; ++i) {
        const HutchppRound &r = rule.rounds()[i];
        res->round_nr[i] = r.nr;
        res->round_nh[i] = (int32_t)std::min<int64_t>(r.nh, INT32_MAX);
        res->round_estimate[i] = r.estimate;
        res->round_sd[i] = r.sd;
    }
    res->krylov_runs = rule.krylov_runs();
    if (quad && quad_cap > 0)
        std::memcpy(quad, ro.psi.data(), (size_t)std::min<int64_t>(quad_cap, (int64_t)ro.psi.size()) * 8);
    res->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return VNE_OK;
}
