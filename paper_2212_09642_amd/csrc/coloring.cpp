// Greedy distance-d colouring (Section 3.1, Algorithm 1) on the host.
//
// The paper builds the distance-d neighbourhoods from the pattern of A^d;
// here each node's neighbourhood is found by a breadth-first search cut at
// depth d, which visits the same node set (O(n Delta^d) work, as the paper
// notes for the graph-traversal route).  Visiting order: descending degree
// (number of off-diagonal entries), ties by increasing row index.  Each node
// takes the smallest colour, counting from 0, that no already coloured node
// of its neighbourhood carries.
//
// The neighbourhoods do not depend on the colours, only the first-fit scan
// does.  Nodes are therefore taken in chunks of the visiting order: worker
// threads list, for every node of the next chunk, the neighbours that come
// earlier in the order (the only ones coloured when the node's turn comes),
// while the calling thread runs the first-fit scan over the current chunk in
// order.  The result is the sequential algorithm's colouring exactly.  Several
// distances share one search to the largest of them: every listed neighbour
// carries its distance, and each distance's scan skips the farther ones.
#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <memory>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

using namespace vne;

namespace {

// Neighbour lists of one chunk: node t0 + j lists its earlier neighbours in
// items[begin[j] .. begin[j + 1]) (per worker, nodes interleaved by worker).
struct ChunkLists {
    int64_t t0 = 0, t1 = 0;
    int nw = 1;
    std::vector<std::vector<int32_t>> items;     // per worker
    std::vector<std::vector<uint8_t>> depth;     // per worker: distance of each listed neighbour
    std::vector<std::vector<int64_t>> begin;     // per worker, per owned node + 1
};

// one per worker thread, on cache lines of its own (the frontier vectors
// change size on every push)
class alignas(128) Searcher {
public:
    Searcher(int64_t n, const int32_t *rp, const int32_t *ci, int32_t d, const std::vector<int32_t> &pos)
        : rp_(rp), ci_(ci), d_(d), pos_(pos), seen_(n, -1) {}

    // earlier neighbours (position < pos of i) of node i within distance d,
    // with their distance
    void list(int32_t i, int32_t stamp, std::vector<int32_t> *out, std::vector<uint8_t> *dist) {
        frontier_.clear();
        frontier_.push_back(i);
        seen_[i] = stamp;
        const int32_t pi = pos_[i];
        for (int32_t depth = 0; depth < d_ && !frontier_.empty(); ++depth) {
            next_.clear();
            for (int32_t x : frontier_) {
                for (int32_t p = rp_[x]; p < rp_[x + 1]; ++p) {
                    const int32_t y = ci_[p];
                    if (seen_[y] == stamp) continue;
                    seen_[y] = stamp;
                    next_.push_back(y);
                    if (pos_[y] < pi) {
                        out->push_back(y);
                        dist->push_back((uint8_t)(depth + 1));
                    }
                }
            }
            frontier_.swap(next_);
        }
    }

private:
    const int32_t *rp_, *ci_;
    int32_t d_;
    const std::vector<int32_t> &pos_;
    std::vector<int32_t> seen_;
    std::vector<int32_t> frontier_, next_;
};

void build_lists(ChunkLists *cl, std::vector<std::unique_ptr<Searcher>> &srch, const std::vector<int32_t> &order) {
    const int nw = cl->nw;
    auto work = [&](int w) {
        // fill vectors local to the thread, hand them over at the end
        std::vector<int32_t> it;
        std::vector<uint8_t> dp;
        std::vector<int64_t> bg;
        it.swap(cl->items[w]);
        dp.swap(cl->depth[w]);
        bg.swap(cl->begin[w]);
        it.clear();
        dp.clear();
        bg.clear();
        bg.push_back(0);
        for (int64_t t = cl->t0 + w; t < cl->t1; t += nw) {
            srch[w]->list(order[t], (int32_t)t, &it, &dp);
            bg.push_back((int64_t)it.size());
        }
        cl->items[w].swap(it);
        cl->depth[w].swap(dp);
        cl->begin[w].swap(bg);
    };
    if (nw == 1) {
        work(0);
        return;
    }
    std::vector<std::thread> th;
    for (int w = 1; w < nw; ++w) th.emplace_back(work, w);
    work(0);
    for (auto &x : th) x.join();
}

}  // namespace

// First-fit state of one distance.
struct FirstFit {
    int32_t d = 1;
    std::vector<int32_t> color;
    std::vector<int64_t> banned;                 // stamp per colour
    int32_t ncol = 0;

    void scan(const ChunkLists &cl, const std::vector<int32_t> &order) {
        const int nw = cl.nw;
        const bool all = d >= 255;
        for (int64_t t = cl.t0; t < cl.t1; ++t) {
            const int64_t r = t - cl.t0;
            const int w = (int)(r % nw);
            const int64_t slot = r / nw;
            const auto &it = cl.items[w];
            const auto &dp = cl.depth[w];
            // the search lists a node's neighbours by increasing distance
            for (int64_t q = cl.begin[w][slot]; q < cl.begin[w][slot + 1]; ++q) {
                if (!all && dp[q] > d) break;
                banned[color[it[q]]] = t;
            }
            int32_t c = 0;
            while (c < ncol && banned[c] == t) ++c;
            if (c == ncol) {
                ncol++;
                banned.push_back(-1);
            }
            color[order[t]] = c;
        }
    }
};

void vne::greedy_color_multi(int64_t n, const int32_t *rp, const int32_t *ci, const int32_t *ds, int nd,
                             int32_t *const *colors_out, int32_t *n_colors) {
    std::vector<int32_t> deg(n);
    for (int64_t i = 0; i < n; ++i) {
        int32_t c = 0;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) c += (ci[p] != i);
        deg[i] = c;
    }
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return deg[a] > deg[b]; });
    std::vector<int32_t> pos(n);
    for (int64_t t = 0; t < n; ++t) pos[order[t]] = (int32_t)t;
    int32_t dmax = 1;
    for (int q = 0; q < nd; ++q) dmax = std::max(dmax, ds[q]);

    int nw = (int)std::thread::hardware_concurrency();
    if (const char *e = std::getenv("VNE_COLOR_THREADS")) nw = std::atoi(e);
    nw = std::max(1, std::min(nw, 16));
    if (n < 4096) nw = 1;
    std::vector<std::unique_ptr<Searcher>> srch;
    for (int w = 0; w < nw; ++w) srch.emplace_back(new Searcher(n, rp, ci, dmax, pos));

    std::vector<FirstFit> ff(nd);
    for (int q = 0; q < nd; ++q) {
        ff[q].d = ds[q];
        ff[q].color.assign(n, -1);
    }
    // chunk sizes: aim at about 2^24 listed neighbours per chunk
    const int64_t kBudget = int64_t(1) << 24;
    int64_t chunk = std::min<int64_t>(n, 1024);
    ChunkLists cur, nxt;
    for (ChunkLists *cl : {&cur, &nxt}) {
        cl->nw = nw;
        cl->items.resize(nw);
        cl->depth.resize(nw);
        cl->begin.resize(nw);
    }
    cur.t0 = 0;
    cur.t1 = chunk;
    build_lists(&cur, srch, order);
    while (cur.t0 < n) {
        // size the next chunk from this one's mean list length
        int64_t total = 0;
        for (int w = 0; w < nw; ++w) total += (int64_t)cur.items[w].size();
        const double mean = std::max(1.0, (double)total / (double)std::max<int64_t>(1, cur.t1 - cur.t0));
        chunk = std::max<int64_t>(256, std::min<int64_t>(1 << 16, (int64_t)(kBudget / mean)));
        nxt.t0 = cur.t1;
        nxt.t1 = std::min<int64_t>(n, cur.t1 + chunk);
        std::thread lister;
        if (nxt.t0 < n) lister = std::thread([&]() { build_lists(&nxt, srch, order); });
        // first-fit scans of the current chunk, one distance per thread
        std::vector<std::thread> scanners;
        for (int q = 1; q < nd; ++q) scanners.emplace_back([&, q]() { ff[q].scan(cur, order); });
        ff[0].scan(cur, order);
        for (auto &x : scanners) x.join();
        if (lister.joinable()) lister.join();
        std::swap(cur, nxt);
        if (cur.t0 >= n) break;
    }
    for (int q = 0; q < nd; ++q) {
        std::copy(ff[q].color.begin(), ff[q].color.end(), colors_out[q]);
        n_colors[q] = ff[q].ncol;
    }
}

int32_t vne::greedy_color(int64_t n, const int32_t *rp, const int32_t *ci, int32_t d, int32_t *colors_out) {
    int32_t ncol = 0;
    int32_t *out[1] = {colors_out};
    greedy_color_multi(n, rp, ci, &d, 1, out, &ncol);
    return ncol;
}

extern "C" vne_status vne_color_greedy(const vne_csr *csr, int32_t d, int32_t *colors_out,
                                       int32_t *n_colors, char *msg, int64_t msg_len) {
    if (!csr || csr->location != VNE_HOST) {
        set_msg(msg, msg_len, "vne_color_greedy needs a host CSR");
        return VNE_EINVAL;
    }
    if (d < 1) { set_msg(msg, msg_len, "distance d must be >= 1"); return VNE_EINVAL; }
    if (!colors_out || !n_colors) { set_msg(msg, msg_len, "NULL output"); return VNE_EINVAL; }
    std::string m;
    vne_status st = validate_host_csr(csr, 0, &m);
    if (st != VNE_OK) { set_msg(msg, msg_len, m); return st; }
    *n_colors = greedy_color(csr->n, csr->row_ptr, csr->col_idx, d, colors_out);
    set_msg(msg, msg_len, "");
    return VNE_OK;
}
