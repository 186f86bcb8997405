// Host test of the adaptive Hutch++ rule (paper_2212_09642_amd/csrc/
// hutchpp_rule.h), built by tests/test_hutchpp_rule.py with AddressSanitizer
// and UndefinedBehaviorSanitizer.
//
// Without arguments: textbook normal quantiles, hand-worked counts and
// standard deviations, and one hand-worked sequence of rounds.
// With "cases": reads cases from stdin and prints the rule's decisions, one
// line per case, for the Python side to compare with the oracle's rule:
//   input:  ncases, then per case
//           rel_eps abs_eps delta n_pilot r_first r_max n_h_max ntab
//           and ntab lines "nr estimate sd" (the statistics of the round of
//           sketch width nr)
//   output: "rounds R  nr nh eps_hat ... kept K nh F capped C reuse U runs X"
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>

#include "hutchpp_rule.h"

using namespace vne;

static int failures = 0;
#define CHECK(cond)                                                   \
    do {                                                              \
        if (!(cond)) {                                                \
            std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                               \
        }                                                             \
    } while (0)

static void self_checks() {
    // two-sided tails of the standard normal: 1%, 5% and the one-sigma tail
    CHECK(std::fabs(hpp_normal_quantile_two_sided(0.01) - 2.5758293035489004) < 1e-12);
    CHECK(std::fabs(hpp_normal_quantile_two_sided(0.05) - 1.959963984540054) < 1e-12);
    CHECK(std::fabs(hpp_normal_quantile_two_sided(0.31731050786291415) - 1.0) < 1e-12);
    // (2 * 1 / 0.1)^2 = 400 exactly; just above 401: 402
    CHECK(hpp_hutch_count(1.0, 0.1, 2.0, 16) == 400);
    CHECK(hpp_hutch_count(1.0, 0.1, 2.0 * std::sqrt(401.0001 / 400.0), 16) == 402);
    CHECK(hpp_hutch_count(0.0, 0.1, 2.0, 16) == 16);
    CHECK(hpp_hutch_count(1e-3, 1.0, 2.576, 16) == 16);
    CHECK(hpp_hutch_count(1.0, 1e-30, 2.576, 16) == 1000000000000000LL);
    CHECK(hpp_hutch_count(1.0, 0.0, 2.576, 16) == 1000000000000000LL);
    const double x[4] = {1.0, 2.0, 3.0, 4.0};
    CHECK(std::fabs(hpp_sample_sd(x, 4) - 1.2909944487358056) < 1e-15);
    // a rank-10 like sequence: widths 3 and 6 ask for ~1e6 forms, 12 for the
    // pilot's 16 (effort 40); 24 could not do better (2 * 24 + 16 = 64)
    HutchppRule r(1e-3, 0.0, 1e-2, 16, 3, 96, 4096);
    CHECK(r.next() == 3);
    r.record(3.68, 0.65);
    CHECK(r.next() == 6);
    r.record(3.68, 0.71);
    CHECK(r.next() == 12);
    r.record(3.68, 1e-5);
    CHECK(r.done() && r.next() == 0 && r.rounds().size() == 3);
    CHECK(r.kept() == 2 && r.final_nh() == 16 && !r.capped() && r.reuse());
    CHECK(r.krylov_runs() == 2 * (3 + 6 + 12) + 3 * 16);
    // one round at r_max, capped
    HutchppRule c(1e-4, 0.0, 1e-2, 16, 3, 3, 32);
    c.record(10.0, 1.0);
    CHECK(c.done() && c.capped() && c.final_nh() == 32 && !c.reuse());
    CHECK(c.krylov_runs() == (6 + 16) + (3 + 32));
    // a round that asks for the pilot's count ends the rounds (the next
    // width costs at least 2 * 6 + 16 = 28 > 22) and is the final run itself
    HutchppRule e(1e-2, 0.0, 1e-2, 16, 3, 96, 4096);
    e.record(10.0, 1e-6);
    CHECK(e.done() && e.rounds().size() == 1 && e.reuse() && e.krylov_runs() == 22);
}

static int run_cases() {
    int ncases = 0;
    if (std::scanf("%d", &ncases) != 1) return 1;
    for (int ci = 0; ci < ncases; ++ci) {
        double rel, abs_eps, delta;
        int n_pilot, r_first, r_max, n_h_max, ntab;
        if (std::scanf("%lf %lf %lf %d %d %d %d %d", &rel, &abs_eps, &delta, &n_pilot, &r_first, &r_max, &n_h_max,
                       &ntab) != 8)
            return 1;
        std::map<int, std::pair<double, double>> tab;
        for (int t = 0; t < ntab; ++t) {
            int nr;
            double est, sd;
            if (std::scanf("%d %lf %lf", &nr, &est, &sd) != 3) return 1;
            tab[nr] = {est, sd};
        }
        HutchppRule rule(rel, abs_eps, delta, n_pilot, r_first, r_max, n_h_max);
        while (const int nr = rule.next()) {
            auto it = tab.find(nr);
            if (it == tab.end()) {
                std::printf("case %d: no statistics for width %d\n", ci, nr);
                return 1;
            }
            rule.record(it->second.first, it->second.second);
        }
        std::printf("rounds %zu", rule.rounds().size());
        for (const HutchppRound &r : rule.rounds())
            std::printf("  %d %lld %.17g", r.nr, (long long)r.nh, r.eps_hat);
        std::printf(" kept %zu nh %d capped %d reuse %d runs %lld\n", rule.kept(), rule.final_nh(),
                    rule.capped() ? 1 : 0, rule.reuse() ? 1 : 0, (long long)rule.krylov_runs());
    }
    return 0;
}

int main(int argc, char **argv) {
    if (argc > 1 && std::strcmp(argv[1], "cases") == 0) return run_cases();
    self_checks();
    if (failures) return 1;
    std::printf("hutchpp rule ok\n");
    return 0;
}
