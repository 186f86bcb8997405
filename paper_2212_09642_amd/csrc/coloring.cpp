// Greedy distance-d colouring (Section 3.1, Algorithm 1) on the host.
//
// Visiting order: descending degree (number of off-diagonal entries), ties
// by increasing row index.  Each node takes the smallest colour, counting
// from 0, that no already coloured node within distance d carries (distance
// in the graph of the off-diagonal pattern; the paper forms the same
// neighbourhoods from the pattern of A^d).
//
// The colours within distance d of node i are the union, over the nodes y
// within distance a of i, of the colours within distance b of y, for any
// a + b = d: a shortest path from i to a node z at distance t <= d passes
// through a node y at distance min(a, t) from i, which is within distance
// t - min(a, t) <= b of z.  Each distance therefore keeps, per node y, a
// bitset of the colours found within distance b of y among the nodes
// coloured so far (b = floor(d / 2), a = d - b).  Node i takes the first
// colour missing from the union over its distance-a ball, then sets that
// colour's bit in the sets of its distance-b ball.  The balls (to depth
// ceil(d_max / 2), with each node's distance) do not depend on the colours:
// worker threads list them for the next chunk of the visiting order while
// the calling thread runs the first-fit scans of the current chunk, one
// thread per distance.  The result is the sequential algorithm's colouring
// exactly, at the cost of searches to half the depth.
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

// Balls of one chunk: node t0 + j lists its ball in
// items[begin[j] .. begin[j + 1]) (per worker, nodes interleaved by worker),
// by nondecreasing distance, the node itself first.
struct ChunkLists {
    int64_t t0 = 0, t1 = 0;
    int nw = 1;
    std::vector<std::vector<int32_t>> items;     // per worker
    std::vector<std::vector<uint8_t>> depth;     // per worker: distance of each listed node
    std::vector<std::vector<int64_t>> begin;     // per worker, per owned node + 1
};

// one per worker thread, on cache lines of its own (the frontier vectors
// change size on every push)
class alignas(128) Searcher {
public:
    Searcher(int64_t n, const int32_t *rp, const int32_t *ci, int32_t depth)
        : rp_(rp), ci_(ci), d_(depth), seen_(n, -1) {}

    // the nodes within distance d_ of node i, breadth first, with their distance
    void list(int32_t i, int32_t stamp, std::vector<int32_t> *out, std::vector<uint8_t> *dist) {
        frontier_.clear();
        frontier_.push_back(i);
        seen_[i] = stamp;
        out->push_back(i);
        dist->push_back(0);
        for (int32_t depth = 0; depth < d_ && !frontier_.empty(); ++depth) {
            next_.clear();
            const bool last = depth + 1 == d_;     // the last level is not expanded
            const uint8_t dd = (uint8_t)(depth + 1);
            for (int32_t x : frontier_) {
                for (int32_t p = rp_[x]; p < rp_[x + 1]; ++p) {
                    const int32_t y = ci_[p];
                    if (seen_[y] == stamp) continue;
                    seen_[y] = stamp;
                    if (!last) next_.push_back(y);
                    out->push_back(y);
                    dist->push_back(dd);
                }
            }
            frontier_.swap(next_);
        }
    }

private:
    const int32_t *rp_, *ci_;
    int32_t d_;
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

// First-fit state of one distance d: per node, the colours within distance
// b of it among the coloured nodes, as W 64-bit words.
struct FirstFit {
    int32_t d = 1, a = 1, b = 0;
    int64_t n = 0;
    int W = 1;
    std::vector<uint64_t> bits;                  // [n][W]
    std::vector<int32_t> color;
    int32_t ncol = 0;

    void init(int64_t nn, int32_t dist) {
        n = nn;
        d = dist;
        b = d / 2;
        a = d - b;
        W = 1;
        bits.assign((size_t)n * W, 0);
        color.assign((size_t)n, -1);
        ncol = 0;
    }

    void widen() {
        std::vector<uint64_t> nb((size_t)n * (W + 1), 0);
        for (int64_t y = 0; y < n; ++y)
            for (int w = 0; w < W; ++w) nb[(size_t)y * (W + 1) + w] = bits[(size_t)y * W + w];
        bits.swap(nb);
        W++;
    }

    // WW: the word count W as a compile-time constant (0: any)
    template <int WW>
    void scan_w(const ChunkLists &cl, const std::vector<int32_t> &order, int64_t *t_next) {
        const int nw = cl.nw;
        const int Wn = WW > 0 ? WW : W;
        std::vector<uint64_t> forb(Wn);
        for (int64_t t = *t_next; t < cl.t1; ++t) {
            const int64_t r = t - cl.t0;
            const int wk = (int)(r % nw);
            const int64_t slot = r / nw;
            const auto &it = cl.items[wk];
            const auto &dp = cl.depth[wk];
            const int64_t q0 = cl.begin[wk][slot], q1 = cl.begin[wk][slot + 1];
            // union over the distance-a ball (listed by distance)
            for (int w = 0; w < Wn; ++w) forb[w] = 0;
            for (int64_t q = q0; q < q1 && dp[q] <= a; ++q) {
                const uint64_t *src = &bits[(size_t)it[q] * Wn];
                for (int w = 0; w < Wn; ++w) forb[w] |= src[w];
            }
            int w = 0;
            while (w < Wn && forb[w] == ~0ull) ++w;
            const int32_t c = w * 64 + (w < Wn ? __builtin_ctzll(~forb[w]) : 0);
            if (c >= 64 * Wn) {
                // every colour of the W words is taken: one more word, and
                // the rest of the chunk with the new width
                widen();
                *t_next = t;
                return;
            }
            const int32_t i = order[t];
            color[i] = c;
            ncol = std::max(ncol, c + 1);
            // mark c in the sets of the distance-b ball
            const uint64_t m = 1ull << (c & 63);
            for (int64_t q = q0; q < q1 && dp[q] <= b; ++q) bits[(size_t)it[q] * Wn + w] |= m;
        }
        *t_next = cl.t1;
    }

    void scan(const ChunkLists &cl, const std::vector<int32_t> &order) {
        int64_t t = cl.t0;
        while (t < cl.t1) {
            switch (W) {
                case 1: scan_w<1>(cl, order, &t); break;
                case 2: scan_w<2>(cl, order, &t); break;
                case 3: scan_w<3>(cl, order, &t); break;
                case 4: scan_w<4>(cl, order, &t); break;
                default: scan_w<0>(cl, order, &t); break;
            }
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
    int32_t depth = 1;                         // the deepest ball any distance needs
    for (int q = 0; q < nd; ++q) depth = std::max(depth, ds[q] - ds[q] / 2);

    int nw = (int)std::thread::hardware_concurrency();
    if (const char *e = std::getenv("VNE_COLOR_THREADS")) nw = std::atoi(e);
    nw = std::max(1, std::min(nw, 16));
    if (n < 4096) nw = 1;
    std::vector<std::unique_ptr<Searcher>> srch;
    for (int w = 0; w < nw; ++w) srch.emplace_back(new Searcher(n, rp, ci, depth));

    std::vector<FirstFit> ff(nd);
    for (int q = 0; q < nd; ++q) ff[q].init(n, ds[q]);
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
