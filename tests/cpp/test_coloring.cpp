// Host check of the threaded greedy distance-d colouring (Algorithm 1): on
// random graphs large enough for the chunked, threaded path, the colouring
// equals a plain sequential first-fit with a breadth-first search per node,
// for 1 and several worker threads, for several distances from one shared
// search, and with bitset memory caps that send some or all distances to
// the earlier-neighbour route; and no two nodes within distance d share a
// colour.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <random>
#include <set>
#include <vector>

#include "internal.h"

struct Csr {
    int n;
    std::vector<int32_t> rp, ci;
};

static Csr from_edges(int n, const std::vector<std::pair<int, int>> &e) {
    std::vector<std::set<int>> adj(n);
    for (auto &p : e) {
        if (p.first == p.second) continue;
        adj[p.first].insert(p.second);
        adj[p.second].insert(p.first);
    }
    Csr c;
    c.n = n;
    c.rp.assign(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        adj[i].insert(i);                       // diagonal, as in a Laplacian
        c.rp[i + 1] = c.rp[i] + (int)adj[i].size();
        for (int j : adj[i]) c.ci.push_back(j);
    }
    return c;
}

static Csr ring(int n, int k, double p, std::mt19937_64 &rng) {
    std::vector<std::pair<int, int>> e;
    std::uniform_real_distribution<double> u(0.0, 1.0);
    for (int i = 0; i < n; ++i)
        for (int r = 1; r <= k / 2; ++r) {
            int j = (i + r) % n;
            if (u(rng) < p) j = (int)(rng() % n);
            e.push_back({i, j});
        }
    return from_edges(n, e);
}

static Csr random_graph(int n, double deg, std::mt19937_64 &rng) {
    std::vector<std::pair<int, int>> e;
    const long m = (long)(n * deg / 2);
    for (long t = 0; t < m; ++t) e.push_back({(int)(rng() % n), (int)(rng() % n)});
    for (int h = 0; h < 5; ++h)                 // a few hubs
        for (int t = 0; t < 300; ++t) e.push_back({h, (int)(rng() % n)});
    return from_edges(n, e);
}

// plain sequential reference: order by (degree desc, index asc), first fit
// over the already coloured nodes within distance d (BFS per node)
static std::vector<int32_t> reference(const Csr &c, int d) {
    const int n = c.n;
    std::vector<int> deg(n), order(n);
    for (int i = 0; i < n; ++i) {
        deg[i] = 0;
        for (int p = c.rp[i]; p < c.rp[i + 1]; ++p) deg[i] += c.ci[p] != i;
    }
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return deg[a] > deg[b]; });
    std::vector<int32_t> col(n, -1);
    std::vector<int> dist(n, -1);
    for (int i : order) {
        std::vector<int> q{i}, seen{i};
        dist[i] = 0;
        std::vector<char> used(n + 1, 0);
        for (size_t h = 0; h < q.size(); ++h) {
            const int x = q[h];
            if (col[x] >= 0) used[col[x]] = 1;
            if (dist[x] == d) continue;
            for (int p = c.rp[x]; p < c.rp[x + 1]; ++p) {
                const int y = c.ci[p];
                if (dist[y] >= 0) continue;
                dist[y] = dist[x] + 1;
                q.push_back(y);
                seen.push_back(y);
            }
        }
        for (int y : seen) dist[y] = -1;
        int k = 0;
        while (used[k]) ++k;
        col[i] = k;
    }
    return col;
}

static bool valid(const Csr &c, const std::vector<int32_t> &col, int d) {
    std::vector<int> dist(c.n, -1);
    for (int i = 0; i < c.n; ++i) {
        std::vector<int> q{i};
        dist[i] = 0;
        bool ok = true;
        for (size_t h = 0; h < q.size(); ++h) {
            const int x = q[h];
            if (x != i && col[x] == col[i]) ok = false;
            if (dist[x] == d) continue;
            for (int p = c.rp[x]; p < c.rp[x + 1]; ++p)
                if (dist[c.ci[p]] < 0) {
                    dist[c.ci[p]] = dist[x] + 1;
                    q.push_back(c.ci[p]);
                }
        }
        for (int y : q) dist[y] = -1;
        if (!ok) return false;
    }
    return true;
}

int main() {
    std::mt19937_64 rng(2212);
    std::vector<Csr> graphs;
    graphs.push_back(ring(6000, 10, 0.1, rng));
    graphs.push_back(random_graph(9000, 5.0, rng));
    graphs.push_back(ring(5000, 6, 0.0, rng));
    const int ds[3] = {1, 2, 3};
    for (size_t gi = 0; gi < graphs.size(); ++gi) {
        const Csr &c = graphs[gi];
        std::vector<std::vector<int32_t>> ref(3);
        for (int q = 0; q < 3; ++q) {
            ref[q] = reference(c, ds[q]);
            if (!valid(c, ref[q], ds[q])) {
                std::printf("FAIL: reference colouring invalid (graph %zu, d %d)\n", gi, ds[q]);
                return 1;
            }
        }
        // the bitset route alone, then caps that send the distances whose
        // colours outgrow them (some or all) to the earlier-neighbour route
        for (const char *cap : {"268435456", "200000", "8"})
        for (const char *th : {"1", "3", "8"}) {
            setenv("VNE_COLOR_BITSET_BYTES", cap, 1);
            setenv("VNE_COLOR_THREADS", th, 1);
            for (int q = 0; q < 3; ++q) {
                std::vector<int32_t> col(c.n, -7);
                const int s = vne::greedy_color(c.n, c.rp.data(), c.ci.data(), ds[q], col.data());
                if (col != ref[q] || s != *std::max_element(col.begin(), col.end()) + 1) {
                    std::printf("FAIL: graph %zu d %d threads %s cap %s differs from the sequential reference\n",
                                gi, ds[q], th, cap);
                    return 1;
                }
            }
            std::vector<std::vector<int32_t>> multi(3, std::vector<int32_t>(c.n, -7));
            int32_t *outs[3] = {multi[0].data(), multi[1].data(), multi[2].data()};
            int32_t counts[3];
            vne::greedy_color_multi(c.n, c.rp.data(), c.ci.data(), ds, 3, outs, counts);
            for (int q = 0; q < 3; ++q)
                if (multi[q] != ref[q]) {
                    std::printf("FAIL: graph %zu shared search d %d threads %s cap %s\n", gi, ds[q], th, cap);
                    return 1;
                }
        }
    }
    std::printf("colouring ok\n");
    return 0;
}
