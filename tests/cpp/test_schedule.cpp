// Host check of the Lanczos step kernel's work schedule: every stored entry
// of every row is covered exactly once (whole rows or segments), segments stay
// inside their row, and the block ranges tile the item list.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "internal.h"

static int fail(const char *m) {
    std::printf("FAIL: %s\n", m);
    return 1;
}

int main() {
    std::mt19937_64 rng(7);
    for (int trial = 0; trial < 300; ++trial) {
        const int n = 1 + (int)(rng() % 3000);
        std::vector<int32_t> rp(n + 1, 0);
        for (int i = 0; i < n; ++i) {
            int deg = (int)(rng() % 12);
            if (rng() % 50 == 0) deg += (int)(rng() % 700);   // hubs
            rp[i + 1] = rp[i] + deg;
        }
        const int seg = 1 + (int)(rng() % 64);
        const int maxb = 1 + (int)(rng() % 3000);
        const int64_t cpb = 1 + (int64_t)(rng() % 4000);
        vne::Schedule s = vne::build_schedule(rp.data(), n, seg, cpb, maxb);
        std::vector<int> cover(rp[n], 0);
        for (int i = 0; i < n; ++i)
            if (rp[i + 1] - rp[i] <= seg)
                for (int p = rp[i]; p < rp[i + 1]; ++p) cover[p]++;
        if ((int)s.segs.size() != s.n_seg) return fail("n_seg");
        for (int L = 0; L < s.n_long; ++L) {
            int f = s.long_first[L], k = s.long_nseg[L];
            if (f < 0 || f + k > s.n_seg) return fail("long table");
            int row = s.segs[f].row;
            if (rp[row + 1] - rp[row] <= seg) return fail("short row split");
            for (int q = 0; q < k; ++q) {
                const vne::SegItem &it = s.segs[f + q];
                if (it.row != row || it.lrow != L) return fail("segment row");
                if (it.p0 < rp[row] || it.p1 > rp[row + 1] || it.p1 <= it.p0 || it.p1 - it.p0 > seg)
                    return fail("segment bounds");
                if (q > 0 && it.p0 != s.segs[f + q - 1].p1) return fail("segments not contiguous");
                for (int p = it.p0; p < it.p1; ++p) cover[p]++;
            }
            if (s.segs[f].p0 != rp[row] || s.segs[f + k - 1].p1 != rp[row + 1]) return fail("segment span");
        }
        for (int p = 0; p < rp[n]; ++p)
            if (cover[p] != 1) return fail("coverage");
        const int nb = s.n_blocks();
        if (nb < 1 || nb > (maxb + 7) / 8 * 8 || nb % 8) return fail("block count");
        if (s.block_begin[0] != 0 || s.block_begin[nb] != s.n_items()) return fail("block ends");
        for (int b = 0; b < nb; ++b)
            if (s.block_begin[b + 1] < s.block_begin[b]) return fail("block order");
    }
    std::printf("schedule ok\n");
    return 0;
}
