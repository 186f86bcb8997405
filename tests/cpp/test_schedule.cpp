// Host check of the Lanczos step kernel's work schedule, as the kernel reads
// it: walking every block's segment range and row range covers every stored
// entry exactly once (short rows whole, long rows through their segments),
// segments stay inside their row, and the block count is a multiple of 8.
// Also checks schedules of several matrices stacked block-diagonally.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "internal.h"

static int fail(const char *m) {
    std::printf("FAIL: %s\n", m);
    return 1;
}

static std::vector<int32_t> random_rows(std::mt19937_64 &rng, int n) {
    std::vector<int32_t> rp(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        int deg = (int)(rng() % 12);
        if (rng() % 50 == 0) deg += (int)(rng() % 700);   // hubs
        rp[i + 1] = rp[i] + deg;
    }
    return rp;
}

// Checks s against row_ptr rp (n rows); rows [r_lo, r_hi) and blocks
// [b_lo, b_hi) may restrict the check to one graph of a stack.
static const char *check(const vne::Schedule &s, const std::vector<int32_t> &rp, int n, int seg) {
    if ((int)s.segs.size() != s.n_seg) return "n_seg";
    if ((int)s.long_first.size() != s.n_long || (int)s.long_nseg.size() != s.n_long) return "long sizes";
    std::vector<int> cover(rp[n], 0), long_row(n, 0);
    for (int L = 0; L < s.n_long; ++L) {
        const int f = s.long_first[L], k = s.long_nseg[L];
        if (f < 0 || k < 1 || f + k > s.n_seg) return "long table";
        const int row = s.segs[f].row;
        if (row < 0 || row >= n) return "long row index";
        if (rp[row + 1] - rp[row] <= seg) return "short row split";
        long_row[row] = 1;
        for (int q = 0; q < k; ++q) {
            const vne::SegItem &it = s.segs[f + q];
            if (it.row != row || it.lrow != L) return "segment row";
            if (it.p0 < rp[row] || it.p1 > rp[row + 1] || it.p1 <= it.p0 || it.p1 - it.p0 > seg)
                return "segment bounds";
            if (q > 0 && it.p0 != s.segs[f + q - 1].p1) return "segments not contiguous";
        }
        if (s.segs[f].p0 != rp[row] || s.segs[f + k - 1].p1 != rp[row + 1]) return "segment span";
    }
    for (int i = 0; i < n; ++i)
        if (!long_row[i] && rp[i + 1] - rp[i] > seg) return "long row not split";
    const int nb = s.n_blocks();
    if (nb < 1 || nb % 8) return "block count";
    std::vector<int> seen_seg(s.n_seg, 0), seen_row(n, 0);
    for (int b = 0; b < nb; ++b) {
        const int32_t *r = &s.block_ranges[4 * (size_t)b];
        if (r[0] < 0 || r[1] < r[0] || r[1] > s.n_seg) return "block segment range";
        if (r[2] < 0 || r[3] < r[2] || r[3] > n) return "block row range";
        for (int t = r[0]; t < r[1]; ++t) {
            seen_seg[t]++;
            for (int p = s.segs[t].p0; p < s.segs[t].p1; ++p) cover[p]++;
        }
        for (int i = r[2]; i < r[3]; ++i) {
            seen_row[i]++;
            if (!long_row[i])
                for (int p = rp[i]; p < rp[i + 1]; ++p) cover[p]++;
        }
    }
    for (int t = 0; t < s.n_seg; ++t)
        if (seen_seg[t] != 1) return "segment not in exactly one block";
    for (int i = 0; i < n; ++i)
        if (seen_row[i] != 1) return "row not in exactly one block";
    for (int p = 0; p < rp[n]; ++p)
        if (cover[p] != 1) return "entry coverage";
    return nullptr;
}

int main() {
    std::mt19937_64 rng(7);
    for (int trial = 0; trial < 300; ++trial) {
        const int n = 1 + (int)(rng() % 3000);
        const std::vector<int32_t> rp = random_rows(rng, n);
        const int seg = 1 + (int)(rng() % 64);
        const int maxb = 1 + (int)(rng() % 3000);
        const int64_t cpb = 1 + (int64_t)(rng() % 4000);
        vne::Schedule s = vne::build_schedule(rp.data(), n, seg, cpb, maxb);
        if (const char *e = check(s, rp, n, seg)) return fail(e);
        if (s.n_blocks() > (maxb + 7) / 8 * 8) return fail("block cap");
        if (s.block_begin[0] != 0 || s.block_begin[s.n_blocks()] != s.n_items()) return fail("block ends");
    }
    // stacks of graphs: the stacked schedule is a valid schedule of the
    // block-diagonal matrix, blocks never straddle graphs, tables line up
    for (int trial = 0; trial < 100; ++trial) {
        const int G = 1 + (int)(rng() % 12);
        const int seg = 1 + (int)(rng() % 64);
        const int64_t cpb = 1 + (int64_t)(rng() % 4000);
        std::vector<vne::Schedule> parts;
        std::vector<int64_t> roff, eoff;
        std::vector<int32_t> all(1, 0), graph_of_row;
        for (int q = 0; q < G; ++q) {
            const int n = 1 + (int)(rng() % 800);
            const std::vector<int32_t> rp = random_rows(rng, n);
            roff.push_back((int64_t)all.size() - 1);
            eoff.push_back(all.back());
            parts.push_back(vne::build_schedule(rp.data(), n, seg, cpb, 4096, false));
            for (int i = 0; i < n; ++i) {
                all.push_back(all.back() + rp[i + 1] - rp[i]);
                graph_of_row.push_back(q);
            }
        }
        const int N = (int)all.size() - 1;
        std::vector<int32_t> gbb, glb, bg;
        vne::Schedule s = vne::stack_schedules(parts, roff, eoff, &gbb, &glb, &bg);
        if (const char *e = check(s, all, N, seg)) return fail(e);
        if ((int)bg.size() != s.n_blocks() || (int)gbb.size() != G + 1 || (int)glb.size() != G + 1)
            return fail("stack table sizes");
        if (gbb[0] != 0 || glb[0] != 0 || glb[G] != s.n_long) return fail("stack table ends");
        for (int q = 0; q < G; ++q) {
            if (gbb[q + 1] < gbb[q] || glb[q + 1] < glb[q]) return fail("stack tables not monotone");
            for (int b = gbb[q]; b < gbb[q + 1]; ++b) {
                if (bg[b] != q) return fail("block_graph");
                const int32_t *r = &s.block_ranges[4 * (size_t)b];
                for (int i = r[2]; i < r[3]; ++i)
                    if (graph_of_row[i] != q) return fail("block straddles graphs (rows)");
                for (int t = r[0]; t < r[1]; ++t)
                    if (graph_of_row[s.segs[t].row] != q) return fail("block straddles graphs (segments)");
            }
            for (int L = glb[q]; L < glb[q + 1]; ++L)
                if (graph_of_row[s.segs[s.long_first[L]].row] != q) return fail("long row graph");
        }
        for (int b = gbb[G]; b < s.n_blocks(); ++b) {   // padding blocks are empty
            const int32_t *r = &s.block_ranges[4 * (size_t)b];
            if (r[0] != r[1] || r[2] != r[3]) return fail("padding block not empty");
        }
    }
    std::printf("schedule ok\n");
    return 0;
}
