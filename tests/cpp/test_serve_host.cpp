// Host check of the serving loop's arena allocator and error rule.
// The arena is compared with a byte-map model under random alloc/release
// sequences: live ranges never overlap, stay inside the arena, are aligned,
// the first fit is the lowest free offset that holds the request, and
// releasing everything leaves one free range.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "serve_host.h"

static int fail(const char *m) {
    std::printf("FAIL: %s\n", m);
    return 1;
}

int main() {
    std::mt19937_64 rng(11);
    for (int trial = 0; trial < 200; ++trial) {
        const uint64_t align = 1ull << (rng() % 9);          // 1 .. 256
        const uint64_t size = align * (1 + rng() % 400);
        vne::Arena a(size, align);
        std::vector<int> used(size, 0);
        std::vector<std::pair<uint64_t, uint64_t>> live;   // off, rounded len
        for (int op = 0; op < 400; ++op) {
            if (!live.empty() && rng() % 3 == 0) {
                const size_t i = rng() % live.size();
                if (!a.release(live[i].first)) return fail("release of a live range");
                for (uint64_t b = live[i].first; b < live[i].first + live[i].second; ++b) used[b] = 0;
                live.erase(live.begin() + i);
                continue;
            }
            const uint64_t want = 1 + rng() % (size / 3 + 1);
            const uint64_t len = (want + align - 1) / align * align;
            // model: lowest aligned offset with len free bytes
            int64_t expect = -1;
            for (uint64_t o = 0; o + len <= size && expect < 0; o += align) {
                bool ok = true;
                for (uint64_t b = o; b < o + len && ok; ++b) ok = !used[b];
                if (ok) expect = (int64_t)o;
            }
            uint64_t off = 0;
            const bool got = a.alloc(want, &off);
            if (got != (expect >= 0)) return fail("alloc success differs from the model");
            if (!got) continue;
            if ((int64_t)off != expect) return fail("not the lowest fit");
            if (off % align) return fail("misaligned");
            for (uint64_t b = off; b < off + len; ++b) {
                if (used[b]) return fail("overlap");
                used[b] = 1;
            }
            live.push_back({off, len});
        }
        uint64_t in_use = 0;
        for (auto &l : live) in_use += l.second;
        if (a.in_use() != in_use) return fail("in_use");
        if (a.release(size + 1)) return fail("release of an unknown offset");
        for (auto &l : live)
            if (!a.release(l.first)) return fail("final release");
        if (a.in_use() != 0 || a.free_ranges() != 1 || a.largest_free() != a.size()) return fail("coalescing");
    }
    // error rule
    for (int trial = 0; trial < 2000; ++trial) {
        const double n = std::exp(std::uniform_real_distribution<double>(std::log(10.0), std::log(1e7))(rng));
        const double lam = std::exp(std::uniform_real_distribution<double>(std::log(1e-8), std::log(1.0))(rng));
        const double s = std::uniform_real_distribution<double>(0.1, 16.0)(rng);
        const double eps = std::exp(std::uniform_real_distribution<double>(std::log(1e-5), std::log(1e-1))(rng));
        const int kmax = 2 + (int)(rng() % 127);
        const int k = vne::plan_steps(n, lam, s, eps, 0.5, kmax);
        auto bound = [&](int kk) { const double d = 2.0 * kk - 1; return 2 * n * lam / (4 * (d * d - 1)); };
        const double target = 0.5 * eps * s;
        if (k < 2 || k > kmax) return fail("steps out of range");
        if (k < kmax && bound(k) > target) return fail("bound not met");
        if (k > 2 && bound(k - 1) <= target) return fail("not the smallest k");
    }
    if (vne::plan_steps(100, 1, 0.0, 1e-3, 0.5, 77) != 77) return fail("no target gives k_max");
    if (vne::plan_probes(10.0, 0.0, 1e-3, 0.5, 2.576, 16, 4096) != 16) return fail("zero spread gives n_min");
    if (vne::plan_probes(10.0, 1e3, 1e-3, 0.5, 2.576, 16, 4096) != 4096) return fail("cap");
    // (2.576 * 0.01 / (0.5e-3 * 10))^2 = 26.54... -> 27
    if (vne::plan_probes(10.0, 0.01, 1e-3, 0.5, 2.576, 16, 4096) != 27) return fail("closed form");
    std::printf("serve host ok\n");
    return 0;
}
