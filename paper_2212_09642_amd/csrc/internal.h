// Internal declarations shared by the host-side C++ (graph ingest, validation,
// colouring, work schedule) and the HIP runtime.  Not part of the C ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "vne.h"

namespace vne {

// Segment of a long CSR row, processed by one lane group of the Lanczos
// step kernel.  Segments of one long row are consecutive in the item list.
struct SegItem {
    int32_t row;
    int32_t p0;      // first entry (absolute index into col_idx)
    int32_t p1;      // one past the last entry
    int32_t lrow;    // index of the long row in the long-row tables
};

// Work schedule of the Lanczos step kernel for one matrix (or for a
// block-diagonal stack of matrices).
//   items [0, n_seg)        : segments of rows with more than seg_len entries
//   items [n_seg, n_seg+n)  : row (item - n_seg); skipped if it is long
// Blocks take contiguous item ranges of roughly equal cost; block_ranges
// holds, per block, its segment range and its row range:
// {seg_begin, seg_end, row_begin, row_end}.
struct Schedule {
    int32_t seg_len = 0;
    int32_t n_seg = 0;                    // segment items
    int32_t n_long = 0;                   // rows split into segments
    std::vector<SegItem> segs;            // [n_seg]
    std::vector<int32_t> long_first;      // [n_long] first segment item
    std::vector<int32_t> long_nseg;       // [n_long]
    std::vector<int32_t> block_begin;     // [n_blocks + 1] item ranges
    std::vector<int32_t> block_ranges;    // [4 * n_blocks]
    int64_t n_items() const { return (int64_t)n_seg + n_rows; }
    int64_t n_rows = 0;
    int32_t n_blocks() const { return (int32_t)block_ranges.size() / 4; }
};

// Builds the schedule from a host row_ptr.  seg_len >= 1, cost_per_block >= 1.
// pad8: round the block count up to a multiple of 8 with empty blocks.
Schedule build_schedule(const int32_t *row_ptr, int64_t n, int32_t seg_len,
                        int64_t cost_per_block, int32_t max_blocks, bool pad8 = true);

// Stacks per-graph schedules (rows and entries offset by the graphs before
// them); blocks never straddle two graphs.  graph_block_begin[G+1],
// graph_long_begin[G+1] and block_graph[n_blocks] describe the stacking; the
// block count is padded to a multiple of 8 with empty blocks.
Schedule stack_schedules(const std::vector<Schedule> &parts, const std::vector<int64_t> &row_offset,
                         const std::vector<int64_t> &nnz_offset, std::vector<int32_t> *graph_block_begin,
                         std::vector<int32_t> *graph_long_begin, std::vector<int32_t> *block_graph);

// Validation shared by vne_csr_validate and vne_graph_register (host arrays).
vne_status validate_host_csr(const vne_csr *csr, uint32_t flags, std::string *msg);

void set_msg(char *msg, int64_t msg_len, const std::string &s);

// Greedy distance-d colouring (Algorithm 1) of the pattern of a validated
// CSR with n rows; colors[n] receives colours from 0; returns the count.
int32_t greedy_color(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t d, int32_t *colors);
// The colourings of nd distances ds[q] (1..254) at once, from one search to
// the largest: colors_out[q][n], n_colors[q].
void greedy_color_multi(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const int32_t *ds, int nd,
                        int32_t *const *colors_out, int32_t *n_colors);

}  // namespace vne
