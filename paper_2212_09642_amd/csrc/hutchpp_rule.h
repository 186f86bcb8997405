// The rule of adaptive Hutch++ (vne_hutchpp_adaptive; the target of eq.
// (3.10) and the adaptive Hutch++ implementation of Section 5, in the
// reading stated with the declaration in vne.h): which sketch width to run
// next, when to stop, which round to keep and how many deflated forms its
// final run takes.  Host only, no device code: vne_hutchpp_adaptive feeds
// it each round's estimate and the sample standard deviation of its pilot
// forms.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace vne {

// z with P(|N(0, 1)| >= z) = delta: the root of erfc(z / sqrt 2) = delta on
// [0, 40], by bisection (erfc decreases; the halvings end at the double
// spacing)
inline double hpp_normal_quantile_two_sided(double delta) {
    double lo = 0.0, hi = 40.0;
    for (int i = 0; i < 200; ++i) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (std::erfc(mid / std::sqrt(2.0)) > delta)
            lo = mid;
        else
            hi = mid;
    }
    return 0.5 * (lo + hi);
}

// deflated forms a round asks for: ceil((z s / eps_hat)^2), the square
// capped at 1e15, at least n_pilot
inline int64_t hpp_hutch_count(double s, double eps_hat, double z, int n_pilot) {
    if (!(s > 0.0)) return n_pilot;
    double x = eps_hat > 0.0 ? (z * s / eps_hat) * (z * s / eps_hat) : 1e15;
    x = std::min(x, 1e15);
    return std::max<int64_t>((int64_t)std::ceil(x), n_pilot);
}

// sample standard deviation (n - 1 in the denominator), two passes
inline double hpp_sample_sd(const double *x, int n) {
    double mean = 0.0;
    for (int i = 0; i < n; ++i) mean += x[i];
    mean /= n;
    double ss = 0.0;
    for (int i = 0; i < n; ++i) ss += (x[i] - mean) * (x[i] - mean);
    return std::sqrt(ss / (n - 1));
}

struct HutchppRound {
    int nr = 0;                      // sketch width
    int64_t nh = 0, effort = 0;      // Hutchinson count asked for, 2 nr + nh
    double estimate = 0.0, sd = 0.0, eps_hat = 0.0;
};

class HutchppRule {
public:
    HutchppRule(double rel_eps, double abs_eps, double delta, int n_pilot, int r_first, int r_max, int n_h_max)
        : rel_eps_(rel_eps), abs_eps_(abs_eps), n_pilot_(n_pilot), r_max_(r_max), n_h_max_(n_h_max),
          z_(hpp_normal_quantile_two_sided(delta)), nr_(r_first) {}

    // sketch width of the next round (0 once the rounds are over)
    int next() const { return done_ ? 0 : nr_; }

    // the round of width next() ran: its estimate and its pilot forms' sd
    void record(double estimate, double sd) {
        HutchppRound r;
        r.nr = nr_;
        r.estimate = estimate;
        r.sd = sd;
        r.eps_hat = abs_eps_ > 0.0 ? abs_eps_ : 0.5 * rel_eps_ * std::fabs(estimate);
        r.nh = hpp_hutch_count(sd, r.eps_hat, z_, n_pilot_);
        r.effort = 2 * (int64_t)r.nr + r.nh;
        rounds_.push_back(r);
        int64_t least = rounds_[0].effort;
        for (const HutchppRound &q : rounds_) least = std::min(least, q.effort);
        // a wider round runs only while its effort could still be below the
        // least so far: it is at least 2 N_r' + n_pilot
        const int nxt = std::min(2 * nr_, r_max_);
        if (nr_ >= r_max_ || 2 * (int64_t)nxt + n_pilot_ >= least)
            done_ = true;
        else
            nr_ = nxt;
    }

    bool done() const { return done_; }
    double z() const { return z_; }
    const std::vector<HutchppRound> &rounds() const { return rounds_; }

    // the round of least effort (the earlier on ties)
    size_t kept() const {
        size_t b = 0;
        for (size_t i = 1; i < rounds_.size(); ++i)
            if (rounds_[i].effort < rounds_[b].effort) b = i;
        return b;
    }
    int final_nh() const { return (int)std::min<int64_t>(rounds_[kept()].nh, n_h_max_); }
    bool capped() const { return rounds_[kept()].nh > n_h_max_; }
    // a kept round that asks for the pilot's count is the final run itself;
    // otherwise the final run takes the kept round's Q and new deflated forms
    bool reuse() const { return final_nh() == n_pilot_; }
    // Krylov runs: 2 N_r + n_pilot per round (N_r products, N_r + n_pilot
    // forms), and N_r + N_H forms for a final run (its Q is the kept round's)
    int64_t krylov_runs() const {
        int64_t r = 0;
        for (const HutchppRound &q : rounds_) r += 2 * (int64_t)q.nr + n_pilot_;
        if (!reuse()) r += (int64_t)rounds_[kept()].nr + final_nh();
        return r;
    }

private:
    double rel_eps_, abs_eps_;
    int n_pilot_, r_max_, n_h_max_;
    double z_;
    int nr_;
    bool done_ = false;
    std::vector<HutchppRound> rounds_;
};

}  // namespace vne
