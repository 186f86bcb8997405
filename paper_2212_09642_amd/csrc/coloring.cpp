// Greedy distance-d colouring (Section 3.1, Algorithm 1) on the host.
//
// The paper builds the distance-d neighbourhoods from the pattern of A^d;
// here each node's neighbourhood is found by a breadth-first search cut at
// depth d, which visits the same node set (O(n Delta^d) work, as the paper
// notes for the graph-traversal route).  Visiting order: descending degree
// (number of off-diagonal entries), ties by increasing row index.  Each node
// takes the smallest colour, counting from 0, that no already coloured node
// of its neighbourhood carries.
#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"

using namespace vne;

int32_t vne::greedy_color(int64_t n, const int32_t *rp, const int32_t *ci, int32_t d, int32_t *colors_out) {
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

    std::vector<int32_t> color(n, -1);
    std::vector<int64_t> seen(n, -1);         // stamp: last search that reached the node
    std::vector<int64_t> banned;               // stamp per colour
    std::vector<int32_t> frontier, next;
    int32_t ncol = 0;
    for (int64_t t = 0; t < n; ++t) {
        const int32_t i = order[t];
        frontier.clear();
        frontier.push_back(i);
        seen[i] = t;
        for (int32_t depth = 0; depth < d && !frontier.empty(); ++depth) {
            next.clear();
            for (int32_t x : frontier) {
                for (int32_t p = rp[x]; p < rp[x + 1]; ++p) {
                    int32_t y = ci[p];
                    if (seen[y] == t) continue;
                    seen[y] = t;
                    next.push_back(y);
                    int32_t c = color[y];
                    if (c >= 0) banned[c] = t;
                }
            }
            frontier.swap(next);
        }
        int32_t c = 0;
        while (c < ncol && banned[c] == t) ++c;
        if (c == ncol) { ncol++; banned.push_back(-1); }
        color[i] = c;
    }
    std::copy(color.begin(), color.end(), colors_out);
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
