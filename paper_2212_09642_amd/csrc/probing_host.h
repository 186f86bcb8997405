// Host-side choice of the colouring distance for the probing method with an
// accuracy target (Section 5, probing method implementation), free of device
// code so that it can be tested on its own.
#pragma once

#include <cstdint>

namespace vne {

struct DistanceChoice {
    int32_t d = 1;
    int32_t fallback = 0;   // 1: Corollary 3.2 chose d (the fit of eq. (5.1) had no decay, or was not asked for)
    int32_t capped = 0;     // 1: no d <= d_max met the target; d = d_max
    double e1 = 0.0;        // |T_2 - T_1|
    double q[2] = {0, 0};   // fitted ratio for kappa = 2 and kappa = 3 (0 when e1 = 0)
    double model = 0.0;     // error the chosen rule predicts at d
};

// Corollary 3.2 with a = 0: the smallest d in [2, d_max] with
// n b / (2 (d^2 - 1)) <= eps_hat, else d_max flagged capped (d_max = 1: the
// corollary covers no allowed d; d = 1, capped).
DistanceChoice probing_bound_distance(double n, double b, double eps_hat, int32_t d_max);

// Eq. (5.1): |tr f(A) - T_d| ~ C q^d / d^kappa, fitted for kappa = 2 and 3
// from e1 = |T_2 - T_1| = C q and e2 = |T_3 - T_2| = C q^2 / 2^kappa; the
// model value at d is e1 q^(d-1) / d^kappa, the larger of the two counts.
// d is the smallest in [1, d_max] whose value is within eps_hat.  Both
// differences zero: d = 1.  e1 = 0 < e2, or q >= 1 for either kappa: the
// bound's choice.
DistanceChoice probing_heuristic_distance(const double T[3], double n, double b, double eps_hat, int32_t d_max);

}  // namespace vne
