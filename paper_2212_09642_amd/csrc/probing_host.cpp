// Choice of the colouring distance d (Section 5, probing method
// implementation: the heuristic of eq. (5.1) and the bound of Corollary 3.2).
#include "probing_host.h"

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace vne {

DistanceChoice probing_bound_distance(double n, double b, double eps_hat, int32_t d_max) {
    DistanceChoice r;
    r.fallback = 1;
    r.d = d_max;
    r.model = INFINITY;                  // Corollary 3.2 covers d >= 2 only
    for (int32_t d = 2; d <= d_max; ++d) {
        const double v = n * b / (2.0 * ((double)d * d - 1.0));
        r.d = d;
        r.model = v;
        if (v <= eps_hat) return r;
    }
    r.capped = 1;
    return r;
}

static double model_value(const DistanceChoice &c, int32_t d) {
    double v = 0.0;
    for (int t = 0; t < 2; ++t) {
        const double kappa = 2.0 + t;
        v = std::max(v, c.e1 * std::pow(c.q[t], d - 1) / std::pow((double)d, kappa));
    }
    return v;
}

DistanceChoice probing_heuristic_distance(const double T[3], double n, double b, double eps_hat, int32_t d_max) {
    DistanceChoice r;
    const double e1 = std::fabs(T[1] - T[0]);
    const double e2 = std::fabs(T[2] - T[1]);
    r.e1 = e1;
    if (e1 > 0.0) {
        r.q[0] = 4.0 * e2 / e1;
        r.q[1] = 8.0 * e2 / e1;
    }
    if (e1 == 0.0 && e2 == 0.0) {
        r.d = 1;
        return r;
    }
    if (e1 == 0.0 || r.q[0] >= 1.0 || r.q[1] >= 1.0) {
        DistanceChoice f = probing_bound_distance(n, b, eps_hat, d_max);
        f.e1 = r.e1;
        f.q[0] = r.q[0];
        f.q[1] = r.q[1];
        return f;
    }
    for (int32_t d = 1; d <= std::max<int32_t>(d_max, 1); ++d) {
        r.d = d;
        r.model = model_value(r, d);
        if (r.model <= eps_hat) return r;
    }
    r.capped = 1;
    return r;
}

}  // namespace vne

extern "C" vne_status vne_probing_select(const double *T, double eps_hat, double n, double lambda_ub,
                                         int32_t d_max, int32_t use_bound, vne_distance_choice *out) {
    if (!out || (!use_bound && !T)) return VNE_EINVAL;
    if (!(eps_hat > 0.0) || !(n > 0.0) || !(lambda_ub > 0.0) || d_max < 1 || d_max > 64) return VNE_EINVAL;
    const vne::DistanceChoice c = use_bound ? vne::probing_bound_distance(n, lambda_ub, eps_hat, d_max)
                                            : vne::probing_heuristic_distance(T, n, lambda_ub, eps_hat, d_max);
    out->d = c.d;
    out->fallback = c.fallback;
    out->capped = c.capped;
    out->e1 = c.e1;
    out->q[0] = c.q[0];
    out->q[1] = c.q[1];
    out->model = c.model;
    return VNE_OK;
}
