// Greedy distance-d colouring (Section 3.1, Algorithm 1) on the host.
//
// Visiting order: descending degree (number of off-diagonal entries), ties
// by increasing row index.  Each node takes the smallest colour, counting
// from 0, that no already coloured node within distance d carries (distance
// in the graph of the off-diagonal pattern; the paper forms the same
// neighbourhoods from the pattern of A^d).
//
// Two routes give this colouring exactly.
//
// Half-depth balls (first choice): the colours within distance d of node i
// are the union, over the nodes y within distance a of i, of the colours
// within distance b of y, for any a + b = d: a shortest path from i to a
// node z at distance t <= d passes through a node y at distance min(a, t)
// from i, which is within distance t - min(a, t) <= b of z.  Each distance
// keeps, per node y, a bitset of the colours found within distance b of y
// among the nodes coloured so far (b = floor(d / 2), a = d - b).  Node i
// takes the first colour missing from the union over its distance-a ball,
// then sets that colour's bit in the sets of its distance-b ball.  The
// bitsets take n * ceil(colours / 64) words; a distance whose colours
// outgrow 256 (or a memory cap of 256 MB per distance; scale-free graphs
// can need colours in the order of n) is coloured again by the second
// route, which is faster there.
//
// Earlier neighbours (fallback): each node lists the nodes within distance
// d that come earlier in the visiting order, and the first-fit scan marks
// their colours in a per-colour stamp array.
//
// Either way the lists do not depend on the colours: worker threads list
// them for the next chunk of the visiting order while the calling thread
// runs the first-fit scans of the current chunk, one thread per distance.
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

// Past 4 words per node (256 colours) the unions cost more than the
// earlier-neighbour route's stamps (measured: BA graphs with n = 2e5 need
// 1259 colours at d = 2 and 3975 at d = 3, and take 3.5x as long with
// bitsets; a ring lattice at d = 16 with 136 colours is faster with them).
constexpr int kMaxWords = 4;

// bitset memory per distance before the earlier-neighbour route takes over
// (VNE_COLOR_BITSET_BYTES overrides it)
int64_t bitset_cap() {
    if (const char *e = std::getenv("VNE_COLOR_BITSET_BYTES")) return std::max<int64_t>(8, std::atoll(e));
    return int64_t(256) << 20;
}

// Lists of one chunk: node t0 + j lists its nodes in
// items[begin[j] .. begin[j + 1]) (per worker, nodes interleaved by worker),
// by nondecreasing distance.
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
    // pos == nullptr: list the whole ball (the node itself first, at
    // distance 0); else only the nodes earlier than the node in the order
    Searcher(int64_t n, const int32_t *rp, const int32_t *ci, int32_t depth, const int32_t *pos)
        : rp_(rp), ci_(ci), d_(depth), pos_(pos), seen_(n, -1) {}

    // the nodes within distance d_ of node i, breadth first, with their distance
    void list(int32_t i, int32_t stamp, std::vector<int32_t> *out, std::vector<uint8_t> *dist) {
        frontier_.clear();
        frontier_.push_back(i);
        seen_[i] = stamp;
        const int32_t pi = pos_ ? pos_[i] : 0;
        if (!pos_) {
            out->push_back(i);
            dist->push_back(0);
        }
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
                    if (!pos_ || pos_[y] < pi) {
                        out->push_back(y);
                        dist->push_back(dd);
                    }
                }
            }
            frontier_.swap(next_);
        }
    }

private:
    const int32_t *rp_, *ci_;
    int32_t d_;
    const int32_t *pos_;
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

// the lists of node t of a chunk: [*q0, *q1) in the worker's arrays
inline void node_range(const ChunkLists &cl, int64_t t, int *wk, int64_t *q0, int64_t *q1) {
    const int64_t r = t - cl.t0;
    *wk = (int)(r % cl.nw);
    const int64_t slot = r / cl.nw;
    *q0 = cl.begin[*wk][slot];
    *q1 = cl.begin[*wk][slot + 1];
}

// First-fit state of one distance d, half-depth route: per node, the
// colours within distance b of it among the coloured nodes, as W 64-bit words.
struct BallFit {
    int32_t d = 1, a = 1, b = 0;
    int64_t n = 0;
    int W = 1;
    int64_t cap = 0;                             // bytes allowed for bits
    bool overflow = false;                       // colours outgrew cap
    std::vector<uint64_t> bits;                  // [n][W]
    std::vector<int32_t> color;
    int32_t ncol = 0;

    void init(int64_t nn, int32_t dist) {
        n = nn;
        d = dist;
        b = d / 2;
        a = d - b;
        W = 1;
        cap = bitset_cap();
        overflow = (int64_t)n * 8 > cap;
        if (!overflow) bits.assign((size_t)n * W, 0);
        color.assign((size_t)n, -1);
        ncol = 0;
    }

    // one more word per node; false (and overflow) past kMaxWords or the
    // memory cap
    bool widen() {
        if (W + 1 > kMaxWords || (int64_t)n * (W + 1) * 8 > cap) {
            overflow = true;
            std::vector<uint64_t>().swap(bits);
            return false;
        }
        std::vector<uint64_t> nb((size_t)n * (W + 1), 0);
        for (int64_t y = 0; y < n; ++y)
            for (int w = 0; w < W; ++w) nb[(size_t)y * (W + 1) + w] = bits[(size_t)y * W + w];
        bits.swap(nb);
        W++;
        return true;
    }

    // WW: the word count W as a compile-time constant (0: any)
    template <int WW>
    void scan_w(const ChunkLists &cl, const std::vector<int32_t> &order, int64_t *t_next) {
        const int Wn = WW > 0 ? WW : W;
        std::vector<uint64_t> forb(Wn);
        for (int64_t t = *t_next; t < cl.t1; ++t) {
            int wk;
            int64_t q0, q1;
            node_range(cl, t, &wk, &q0, &q1);
            const auto &it = cl.items[wk];
            const auto &dp = cl.depth[wk];
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
                *t_next = widen() ? t : cl.t1;
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

    bool finished() const { return overflow; }

    void scan(const ChunkLists &cl, const std::vector<int32_t> &order) {
        int64_t t = cl.t0;
        while (t < cl.t1 && !overflow) {
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

// First-fit state of one distance d, earlier-neighbour route.
struct DirectFit {
    int32_t d = 1;
    std::vector<int32_t> color;
    std::vector<int64_t> banned;                 // stamp per colour
    int32_t ncol = 0;

    void init(int64_t n, int32_t dist) {
        d = dist;
        color.assign((size_t)n, -1);
        banned.clear();
        ncol = 0;
    }

    bool finished() const { return false; }

    void scan(const ChunkLists &cl, const std::vector<int32_t> &order) {
        for (int64_t t = cl.t0; t < cl.t1; ++t) {
            int wk;
            int64_t q0, q1;
            node_range(cl, t, &wk, &q0, &q1);
            const auto &it = cl.items[wk];
            const auto &dp = cl.depth[wk];
            for (int64_t q = q0; q < q1 && dp[q] <= d; ++q) banned[color[it[q]]] = t;
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

int color_threads(int64_t n) {
    int nw = (int)std::thread::hardware_concurrency();
    if (const char *e = std::getenv("VNE_COLOR_THREADS")) nw = std::atoi(e);
    nw = std::max(1, std::min(nw, 16));
    return n < 4096 ? 1 : nw;
}

// Lists to `depth` (whole balls, or earlier nodes when pos is given) chunk by
// chunk, each chunk scanned by every fit of `fits` (one thread per fit)
// while the next chunk is listed; stops early once every fit has given up.
template <class Fit>
void run_pipeline(int64_t n, const int32_t *rp, const int32_t *ci, const std::vector<int32_t> &order,
                  int32_t depth, const int32_t *pos, std::vector<Fit *> &fits) {
    const int nw = color_threads(n);
    std::vector<std::unique_ptr<Searcher>> srch;
    for (int w = 0; w < nw; ++w) srch.emplace_back(new Searcher(n, rp, ci, depth, pos));
    // chunk sizes: aim at about 2^24 listed nodes per chunk
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
    const int nf = (int)fits.size();
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
        std::vector<std::thread> scanners;
        for (int q = 1; q < nf; ++q) scanners.emplace_back([&, q]() { fits[q]->scan(cur, order); });
        if (nf > 0) fits[0]->scan(cur, order);
        for (auto &x : scanners) x.join();
        if (lister.joinable()) lister.join();
        std::swap(cur, nxt);
        if (cur.t0 >= n) break;
        bool all = true;
        for (Fit *f : fits) all = all && f->finished();
        if (all) break;
    }
}

}  // namespace

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

    // half-depth balls for every distance
    std::vector<BallFit> ball(nd);
    std::vector<BallFit *> bp;
    int32_t depth = 1;                         // the deepest ball any distance needs
    for (int q = 0; q < nd; ++q) {
        ball[q].init(n, ds[q]);
        bp.push_back(&ball[q]);
        depth = std::max(depth, ds[q] - ds[q] / 2);
    }
    run_pipeline(n, rp, ci, order, depth, nullptr, bp);

    // distances whose colours outgrew the bitsets: earlier neighbours
    std::vector<DirectFit> direct;
    std::vector<int> redo;
    int32_t dmax = 1;
    for (int q = 0; q < nd; ++q)
        if (ball[q].overflow) {
            redo.push_back(q);
            dmax = std::max(dmax, ds[q]);
        }
    if (!redo.empty()) {
        std::vector<int32_t> pos(n);
        for (int64_t t = 0; t < n; ++t) pos[order[t]] = (int32_t)t;
        direct.resize(redo.size());
        std::vector<DirectFit *> dp;
        for (size_t r = 0; r < redo.size(); ++r) {
            direct[r].init(n, ds[redo[r]]);
            dp.push_back(&direct[r]);
        }
        run_pipeline(n, rp, ci, order, dmax, pos.data(), dp);
    }
    size_t r = 0;
    for (int q = 0; q < nd; ++q) {
        if (ball[q].overflow) {
            std::copy(direct[r].color.begin(), direct[r].color.end(), colors_out[q]);
            n_colors[q] = direct[r].ncol;
            ++r;
        } else {
            std::copy(ball[q].color.begin(), ball[q].color.end(), colors_out[q]);
            n_colors[q] = ball[q].ncol;
        }
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
    // distances are kept in one byte per listed node
    if (d < 1 || d > 254) { set_msg(msg, msg_len, "distance d must be in [1, 254]"); return VNE_EINVAL; }
    if (!colors_out || !n_colors) { set_msg(msg, msg_len, "NULL output"); return VNE_EINVAL; }
    std::string m;
    vne_status st = validate_host_csr(csr, 0, &m);
    if (st != VNE_OK) { set_msg(msg, msg_len, m); return st; }
    *n_colors = greedy_color(csr->n, csr->row_ptr, csr->col_idx, d, colors_out);
    set_msg(msg, msg_len, "");
    return VNE_OK;
}
