// Host-side matrix ingest: graph Laplacian of the largest connected component
// (eq. (2.3); preprocessing of Section 6.1), CSR validation and the work
// schedule of the Lanczos step kernel.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"

namespace vne {

void set_msg(char *msg, int64_t msg_len, const std::string &s) {
    if (!msg || msg_len <= 0) return;
    size_t k = std::min<size_t>(s.size(), (size_t)msg_len - 1);
    std::memcpy(msg, s.data(), k);
    msg[k] = '\0';
}

vne_status validate_host_csr(const vne_csr *csr, uint32_t flags, std::string *msg) {
    if (!csr) { *msg = "csr is NULL"; return VNE_EINVAL; }
    const int64_t n = csr->n, nnz = csr->nnz;
    if (n < 1) { *msg = "n must be >= 1"; return VNE_EINVAL; }
    if (nnz < 0 || nnz > INT32_MAX) { *msg = "nnz out of range"; return VNE_EINVAL; }
    if (n > INT32_MAX - 1) { *msg = "n out of range"; return VNE_EINVAL; }
    if (!csr->row_ptr || (nnz > 0 && (!csr->col_idx || !csr->values))) {
        *msg = "NULL CSR array"; return VNE_EINVAL;
    }
    if (csr->value_dtype != VNE_F32 && csr->value_dtype != VNE_F64) {
        *msg = "value_dtype must be VNE_F32 or VNE_F64"; return VNE_EINVAL;
    }
    if (!(std::isfinite(csr->scale) && csr->scale > 0)) {
        *msg = "scale must be finite and > 0"; return VNE_EINVAL;
    }
    const int32_t *rp = csr->row_ptr, *ci = csr->col_idx;
    if (rp[0] != 0 || rp[n] != nnz) { *msg = "row_ptr[0] must be 0 and row_ptr[n] == nnz"; return VNE_EINVAL; }
    auto val = [&](int64_t p) -> double {
        return csr->value_dtype == VNE_F32 ? (double)((const float *)csr->values)[p]
                                           : ((const double *)csr->values)[p];
    };
    for (int64_t i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) { *msg = "row_ptr not monotone at row " + std::to_string(i); return VNE_EINVAL; }
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (ci[p] < 0 || ci[p] >= n) { *msg = "column out of range in row " + std::to_string(i); return VNE_EINVAL; }
            if (p > rp[i] && ci[p] <= ci[p - 1]) {
                *msg = "columns not sorted/unique in row " + std::to_string(i); return VNE_EINVAL;
            }
            if (!std::isfinite(val(p))) { *msg = "non-finite value in row " + std::to_string(i); return VNE_EINVAL; }
        }
    }
    if (flags & VNE_VALIDATE_ZERO_ROWSUM) {
        for (int64_t i = 0; i < n; ++i) {
            double s = 0;
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) s += val(p);
            if (s != 0.0) { *msg = "row " + std::to_string(i) + " does not sum to zero"; return VNE_EINVAL; }
        }
    }
    if (flags & VNE_VALIDATE_SYMMETRIC) {
        for (int64_t i = 0; i < n; ++i) {
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                int32_t j = ci[p];
                const int32_t *b = ci + rp[j], *e = ci + rp[j + 1];
                const int32_t *q = std::lower_bound(b, e, (int32_t)i);
                if (q == e || *q != i || val(q - ci) != val(p)) {
                    *msg = "matrix not symmetric at (" + std::to_string(i) + "," + std::to_string(j) + ")";
                    return VNE_EINVAL;
                }
            }
        }
    }
    return VNE_OK;
}

static void ranges_from_items(Schedule &s) {
    const int32_t nb = (int32_t)s.block_begin.size() - 1;
    s.block_ranges.assign(4 * (size_t)nb, 0);
    for (int32_t b = 0; b < nb; ++b) {
        const int64_t ib = s.block_begin[b], ie = s.block_begin[b + 1];
        const int64_t sb = std::min<int64_t>(ib, s.n_seg), se = std::min<int64_t>(ie, s.n_seg);
        const int64_t rb = std::max<int64_t>(ib, s.n_seg) - s.n_seg, re = std::max<int64_t>(ie, s.n_seg) - s.n_seg;
        s.block_ranges[4 * b + 0] = (int32_t)sb;
        s.block_ranges[4 * b + 1] = (int32_t)se;
        s.block_ranges[4 * b + 2] = (int32_t)rb;
        s.block_ranges[4 * b + 3] = (int32_t)re;
    }
}

Schedule build_schedule(const int32_t *row_ptr, int64_t n, int32_t seg_len, int64_t cost_per_block,
                        int32_t max_blocks, bool pad8) {
    Schedule s;
    s.seg_len = seg_len;
    s.n_rows = n;
    const int64_t row_overhead = 4;   // loads and stores of the row's own vectors
    for (int64_t i = 0; i < n; ++i) {
        int32_t deg = row_ptr[i + 1] - row_ptr[i];
        if (deg > seg_len) {
            int32_t L = s.n_long++;
            s.long_first.push_back((int32_t)s.segs.size());
            int32_t nseg = (deg + seg_len - 1) / seg_len;
            s.long_nseg.push_back(nseg);
            for (int32_t k = 0; k < nseg; ++k) {
                int32_t p0 = row_ptr[i] + k * seg_len;
                int32_t p1 = std::min(p0 + seg_len, row_ptr[i + 1]);
                s.segs.push_back({(int32_t)i, p0, p1, L});
            }
        }
    }
    s.n_seg = (int32_t)s.segs.size();
    const int64_t n_items = s.n_items();
    // cost of every item, then cut into blocks of about cost_per_block
    std::vector<int64_t> cost(n_items);
    for (int64_t t = 0; t < s.n_seg; ++t) cost[t] = (s.segs[t].p1 - s.segs[t].p0) + row_overhead;
    for (int64_t i = 0; i < n; ++i) {
        int32_t deg = row_ptr[i + 1] - row_ptr[i];
        cost[s.n_seg + i] = deg > seg_len ? 1 : deg + row_overhead;
    }
    int64_t total = 0;
    for (int64_t c : cost) total += c;
    int64_t nb = std::max<int64_t>(1, (total + cost_per_block - 1) / cost_per_block);
    nb = std::min<int64_t>(nb, std::max<int32_t>(1, max_blocks));
    nb = std::min<int64_t>(nb, std::max<int64_t>(1, n_items));
    // a multiple of 8 (the 8 XCDs each take a contiguous range); blocks past
    // the cost-balanced ones are empty
    const int64_t nb_work = nb;
    if (pad8) nb = (nb + 7) / 8 * 8;
    s.block_begin.assign(nb + 1, 0);
    int64_t acc = 0, b = 1;
    for (int64_t t = 0; t < n_items && b < nb_work; ++t) {
        acc += cost[t];
        while (b < nb_work && acc * nb_work >= b * total) s.block_begin[b++] = (int32_t)(t + 1);
    }
    while (b < nb) s.block_begin[b++] = (int32_t)n_items;
    s.block_begin[nb] = (int32_t)n_items;
    ranges_from_items(s);
    return s;
}

Schedule stack_schedules(const std::vector<Schedule> &parts, const std::vector<int64_t> &row_offset,
                         const std::vector<int64_t> &nnz_offset, std::vector<int32_t> *graph_block_begin,
                         std::vector<int32_t> *graph_long_begin, std::vector<int32_t> *block_graph) {
    Schedule s;
    const size_t G = parts.size();
    graph_block_begin->assign(G + 1, 0);
    graph_long_begin->assign(G + 1, 0);
    block_graph->clear();
    s.seg_len = G ? parts[0].seg_len : 0;
    for (size_t q = 0; q < G; ++q) {
        const Schedule &p = parts[q];
        const int32_t seg0 = (int32_t)s.segs.size(), long0 = s.n_long;
        (*graph_block_begin)[q] = s.n_blocks();
        (*graph_long_begin)[q] = s.n_long;
        for (const SegItem &it : p.segs)
            s.segs.push_back({(int32_t)(it.row + row_offset[q]), (int32_t)(it.p0 + nnz_offset[q]),
                              (int32_t)(it.p1 + nnz_offset[q]), it.lrow + long0});
        for (int32_t L = 0; L < p.n_long; ++L) {
            s.long_first.push_back(p.long_first[L] + seg0);
            s.long_nseg.push_back(p.long_nseg[L]);
        }
        s.n_long += p.n_long;
        for (int32_t b = 0; b < p.n_blocks(); ++b) {
            s.block_ranges.push_back(p.block_ranges[4 * b + 0] + seg0);
            s.block_ranges.push_back(p.block_ranges[4 * b + 1] + seg0);
            s.block_ranges.push_back((int32_t)(p.block_ranges[4 * b + 2] + row_offset[q]));
            s.block_ranges.push_back((int32_t)(p.block_ranges[4 * b + 3] + row_offset[q]));
            block_graph->push_back((int32_t)q);
        }
        s.n_rows += p.n_rows;
    }
    (*graph_block_begin)[G] = s.n_blocks();
    (*graph_long_begin)[G] = s.n_long;
    s.n_seg = (int32_t)s.segs.size();
    while (s.n_blocks() % 8) {   // empty blocks
        for (int q = 0; q < 4; ++q) s.block_ranges.push_back(0);
        block_graph->push_back(G ? (int32_t)G - 1 : 0);
    }
    return s;
}

}  // namespace vne

using namespace vne;

extern "C" const char *vne_version(void) { return "vne 0.1 (gfx950)"; }

extern "C" vne_status vne_csr_validate(const vne_csr *csr, uint32_t flags, char *msg, int64_t msg_len) {
    std::string m;
    if (csr && csr->location != VNE_HOST) {
        set_msg(msg, msg_len, "vne_csr_validate needs host arrays");
        return VNE_EINVAL;
    }
    vne_status st = validate_host_csr(csr, flags, &m);
    set_msg(msg, msg_len, m);
    return st;
}

extern "C" vne_status vne_laplacian_from_edges(int64_t n_nodes, int64_t n_edges, const int64_t *edges,
                                               int64_t *n_out, int64_t *nnz_out, int32_t *row_ptr,
                                               int32_t *col_idx, void *values, int32_t value_dtype,
                                               int64_t *node_ids, double *scale, char *msg,
                                               int64_t msg_len) {
    if (n_nodes < 1 || n_nodes > INT32_MAX - 1) { set_msg(msg, msg_len, "n_nodes out of range"); return VNE_EINVAL; }
    if (n_edges < 0 || (n_edges > 0 && !edges)) { set_msg(msg, msg_len, "bad edge array"); return VNE_EINVAL; }
    if (!n_out || !nnz_out) { set_msg(msg, msg_len, "n_out and nnz_out are required"); return VNE_EINVAL; }
    if (row_ptr && value_dtype != VNE_F32 && value_dtype != VNE_F64) {
        set_msg(msg, msg_len, "value_dtype must be VNE_F32 or VNE_F64"); return VNE_EINVAL;
    }
    const int64_t n = n_nodes;
    // adjacency by counting sort, both directions, self loops dropped
    std::vector<int64_t> cnt(n + 1, 0);
    for (int64_t e = 0; e < n_edges; ++e) {
        int64_t u = edges[2 * e], v = edges[2 * e + 1];
        if (u < 0 || v < 0 || u >= n || v >= n) { set_msg(msg, msg_len, "edge endpoint out of range"); return VNE_EINVAL; }
        if (u == v) continue;
        cnt[u + 1]++;
        cnt[v + 1]++;
    }
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    std::vector<int32_t> adj(cnt[n]);
    {
        std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
        for (int64_t e = 0; e < n_edges; ++e) {
            int64_t u = edges[2 * e], v = edges[2 * e + 1];
            if (u == v) continue;
            adj[pos[u]++] = (int32_t)v;
            adj[pos[v]++] = (int32_t)u;
        }
    }
    // sort and deduplicate every neighbour list (binary weights)
    std::vector<int64_t> start(n + 1, 0);
    {
        int64_t w = 0;
        for (int64_t i = 0; i < n; ++i) {
            int32_t *b = adj.data() + cnt[i], *e = adj.data() + cnt[i + 1];
            std::sort(b, e);
            int32_t *last = std::unique(b, e);
            start[i] = w;
            for (int32_t *q = b; q < last; ++q) adj[w++] = *q;
        }
        start[n] = w;
        adj.resize(w);
    }
    // connected components by breadth-first search, in increasing start node
    std::vector<int32_t> comp(n, -1), queue(n);
    int32_t best = -1;
    int64_t best_size = 0;
    int32_t nc = 0;
    for (int64_t s = 0; s < n; ++s) {
        if (comp[s] >= 0) continue;
        int64_t qh = 0, qt = 0;
        queue[qt++] = (int32_t)s;
        comp[s] = nc;
        while (qh < qt) {
            int32_t x = queue[qh++];
            for (int64_t p = start[x]; p < start[x + 1]; ++p) {
                int32_t y = adj[p];
                if (comp[y] < 0) { comp[y] = nc; queue[qt++] = y; }
            }
        }
        // components are discovered in increasing order of their smallest
        // node, so a strict '>' keeps the one with the smallest id on ties
        if (qt > best_size) { best_size = qt; best = nc; }
        nc++;
    }
    std::vector<int32_t> newid(n, -1);
    int64_t m = 0, nnz = 0;
    for (int64_t i = 0; i < n; ++i)
        if (comp[i] == best) {
            newid[i] = (int32_t)m++;
            nnz += (start[i + 1] - start[i]) + 1;
        }
    if (nnz > INT32_MAX) { set_msg(msg, msg_len, "component too large for int32 indices"); return VNE_ENOTSUP; }
    *n_out = m;
    *nnz_out = nnz;
    int64_t trace = nnz - m;  // sum of degrees
    if (trace == 0) { set_msg(msg, msg_len, "largest component has no edge (tr(L) = 0)"); return VNE_EINVAL; }
    if (!row_ptr) { set_msg(msg, msg_len, ""); return VNE_OK; }
    if (!col_idx || !values) { set_msg(msg, msg_len, "col_idx and values are required"); return VNE_EINVAL; }
    int64_t w = 0;
    int64_t r = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (comp[i] != best) continue;
        row_ptr[r] = (int32_t)w;
        const int64_t deg = start[i + 1] - start[i];
        bool diag_done = false;
        auto put = [&](int32_t c, double v) {
            col_idx[w] = c;
            if (value_dtype == VNE_F32) ((float *)values)[w] = (float)v;
            else ((double *)values)[w] = v;
            ++w;
        };
        for (int64_t p = start[i]; p < start[i + 1]; ++p) {
            int32_t c = newid[adj[p]];   // renumbering is monotone: order kept
            if (!diag_done && c > r) { put((int32_t)r, (double)deg); diag_done = true; }
            put(c, -1.0);
        }
        if (!diag_done) put((int32_t)r, (double)deg);
        if (node_ids) node_ids[r] = i;
        ++r;
    }
    row_ptr[m] = (int32_t)w;
    if (scale) *scale = 1.0 / (double)trace;
    set_msg(msg, msg_len, "");
    return VNE_OK;
}
