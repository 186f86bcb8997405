// Launch wrappers of the gfx950 kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace vne {

constexpr int kMaxSteps = 128;     // largest k_steps the quadrature kernels accept
constexpr int kBlock = 256;        // threads per block of the streaming kernels
constexpr int kStepThreads = 256;  // threads per block of the Lanczos step kernel

enum ProbeGen { GEN_RADEMACHER = 0, GEN_COLORING = 1, GEN_DENSE = 2 };

// Everything the Lanczos step kernel reads or writes, for one matrix and one
// probe block of width m_pad (a multiple of the column tile mt).
struct StepArgs {
    const int32_t *row_ptr;
    const int32_t *col;
    const void *val;            // float (FP32 mode) or double (FP64 mode)
    double scale;
    int32_t n;
    int32_t m_pad;
    int32_t mt;                 // column tile of the launch
    int32_t n_tiles;
    const void *P_in;           // raw vector P_j (n x m_pad)
    const void *V_prev;         // v_{j-1} (ignored on the first step)
    void *V_out;                // v_j, written
    const void *V_cur;          // two-pass schedule: v_j as written by the normalize pass
    int32_t two_pass;           // 0: lazy schedule, 1: normalize pass + single-stream SpMM
    void *P_out;                // P_{j+1} = A v_j - beta_{j-1} v_{j-1}, written
    const double *st_alpha;     // per column alpha_{j-1}
    const double *st_inv;       // per column 1/beta_{j-1} (1/||c|| at j = 1; 0 frozen)
    const double *st_coup;      // per column beta_{j-1} (0 at j = 1)
    const SegItem *segs;
    int32_t n_seg;
    int32_t seg_len;
    const int4 *block_ranges;   // [n_blocks] {seg_begin, seg_end, row_begin, row_end}
    int32_t n_blocks;
    double *seg_acc;            // [n_seg][m_pad]
    int32_t n_long;             // rows split into segments
    const int32_t *long_first;
    const int32_t *long_nseg;
    double *long_part;          // [n_long][3][m_pad]
    double *partials;           // [n_blocks][3][m_pad]
    // several graphs in one launch (block-diagonal matrix, rows stacked by
    // graph; work blocks never straddle two graphs).  Per-column state is
    // indexed graph * m_pad + column.  nullptr arrays mean one graph.
    const int32_t *block_graph; // [n_blocks]
    const int32_t *row_graph;   // [n]
    const int32_t *long_graph;  // [n_long]
    const double *graph_scale;  // [G]
    // serving slots: records {stop_uid + i, j > 0} at stop_state[i] for every
    // i < stop_count (nullptr: none) mean that every task sharing the slot
    // has met its stopping rule; the slot's kernels then return at once
    const int2 *stop_state;
    int32_t stop_uid;
    int32_t stop_count;
    // per-column stopping (one graph): col_stop[c] > 0 is the step at which
    // column c met its tolerance; such a column is done (nullptr: none).  A
    // work block whose tile holds only done or frozen columns returns at
    // once, and the normalize pass skips groups of done columns.
    const int32_t *col_stop;
    // a launch over part of the block: its tiles start at tile_base (grid y
    // counts from there) and the normalize pass covers columns [col_base,
    // col_base + col_count) (col_count 0: every column)
    int32_t tile_base;
    int32_t col_base, col_count;
};

constexpr int kLevel2 = 32;       // first-level reduction rows of the step partials

struct FinalizeArgs {
    const double *partials;
    const double *long_part;
    double *level2;             // [n_level2][3][m_pad]
    int32_t n_level2;
    int32_t n_blocks;
    int32_t n_long;
    int32_t mt;
    int32_t m_pad;
    int32_t m;                  // real columns (pad columns stay frozen)
    int32_t step;               // 1-based step just taken
    int32_t k;                  // steps of the run (row stride of alpha/beta)
    double tau;
    double *st_alpha, *st_inv, *st_coup;
    double *alpha, *beta;       // [G * m_pad][k]
    int32_t *k_eff;
    int32_t *flags;             // bit 0: non-finite coefficient
    // several graphs: per-graph single-level reduction over the graph's own
    // blocks and long rows (in order); per-graph step counts and widths
    int32_t n_graphs;
    int32_t segmented;
    const int32_t *graph_block_begin;  // [G+1]
    const int32_t *graph_long_begin;   // [G+1]
    const int32_t *graph_k;            // [G] (nullptr: k)
    const int32_t *graph_m;            // [G] (nullptr: m)
    const int2 *stop_state;            // slots: as in StepArgs
    int32_t stop_uid;
    int32_t stop_count;
    int32_t *flags_mem[4];             // group slots: flags of member c / mem_cols (nullptr: flags)
    int32_t mem_cols;                  // columns per member of a group slot (0: one query)
    const int32_t *col_stop;           // as in StepArgs: done columns keep their coefficients
    // one graph: the reduction and update of columns [col_base, col_base +
    // col_count) only (col_count 0: every column)
    int32_t col_base, col_count;
};

// Returns the column tile width the step kernel uses for this probe width;
// three: FP32 widths 3 * 2^j (12 .. 192) may take a tile of three columns per
// lane (launch_step only; the slot kernels have four per lane).
int choose_tile(int m, bool fp64, int requested, bool three = false);
int pad_columns(int m, int mt);
// The tile of a plan for an n-row matrix with nnz entries (launch_step
// widths: 4 columns per lane, or 3 for FP32 widths 3 * 2^j): the one whose
// padding, CSR passes and gathers move the fewest bytes per step.
int choose_plan_tile(int m, bool fp64, int64_t n, int64_t nnz);

// [normalize pass,] step kernel, then (if the matrix has long rows) the long-row kernel
hipError_t launch_step(const StepArgs &a, bool fp64, bool first, hipStream_t s);
hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t s);

// Several independent problems ("slots") per launch, two-pass schedule, one
// column tile mt for all of them.  args: device array of per-slot StepArgs
// (graph fields unused: one matrix per slot).  step_map entries {slot, work
// block, tile, 0} cover every block (padding blocks included) and tile of
// each slot; long_map entries {slot, group, tile, 0} cover the long rows in
// groups of long_rows_per_group(mt, fp64).  The first step of a slot needs
// its v_{j-1} buffer zeroed.  Then launch_finalize_slots with map entries
// {slot, column chunk of kFinalizeCols}; each slot's FinalizeArgs carries
// n_level2 = kSlotLevel2 and a level2 scratch of kSlotLevel2 * 3 * m_pad
// doubles.
hipError_t launch_step_slots(const StepArgs *args, const int4 *step_map, int32_t n_step, const int4 *long_map,
                             int32_t n_long, int32_t mt, bool fp64, hipStream_t s);
int long_rows_per_group(int mt, bool fp64);
// Group slots of `members` (2 or 4) 16-column FP32 tiles (m_pad = 16 *
// members, mt = 16), every tile of a work block in one workgroup: group_map
// entries {slot, work block, 0, 0}; long_map entries {slot, group, tile, 0}
// as for mt = 16.  Every column gets the same arithmetic, in the same order,
// as in a 16-column slot.
hipError_t launch_step_groups(const StepArgs *args, const int4 *group_map, int32_t n_group, const int4 *long_map,
                              int32_t n_long, int32_t members, hipStream_t s);
constexpr int kFinalizeCols = 16;
constexpr int kSlotLevel2 = 16;   // first-level parts of a slot's reduction (FinalizeArgs.n_level2)
hipError_t launch_finalize_slots(const FinalizeArgs *fargs, const int2 *map, int32_t n_entries, hipStream_t s);

// probe block: sums, centring, norms; P_1 written with element type of the mode
struct ProbeArgs {
    int32_t gen;                // ProbeGen
    int32_t n, m, m_pad, mt;
    int32_t col_offset;         // first hash column (Hutch++ G block)
    uint64_t seed;
    const int64_t *keys;        // [n] row keys (Rademacher)
    const int32_t *colors;      // [n] (colouring)
    const void *dense;          // [n][ld_dense] (dense), element type of the mode
    int32_t ld_dense;
    int32_t desing;
    void *P_out;                // [n][ld_out]
    int32_t ld_out;             // row stride of P_out (0: m_pad)
    double *partials;           // scratch [n_blocks][m_pad]
    int32_t n_blocks;
    double *mean;               // [m_pad]
    double *norm2;              // [m_pad]
    double *st_alpha, *st_inv, *st_coup;
    int32_t *k_eff;
    int32_t k;
    // blocks own row ranges of one graph each; per-graph seed, width, steps
    const int32_t *block_row_begin;    // [n_blocks+1]
    const int32_t *block_graph;        // [n_blocks]
    const int32_t *graph_block_begin;  // [G+1]
    const int64_t *graph_row_begin;    // [G+1]
    const uint64_t *seeds;             // [G]
    const int32_t *graph_k;            // [G]
    const int32_t *graph_m;            // [G]
    int32_t n_graphs;
    int32_t *flags;                    // bit 0 set for a start vector whose norm is not finite
};
hipError_t launch_probe(const ProbeArgs &a, bool fp64, hipStream_t s);

// raw +-1 Rademacher block into out[i*ld + off + c], c < m (no centring)
hipError_t launch_rademacher_fill(void *out, bool fp64, int32_t n, int32_t m, int32_t ld, int32_t off,
                                  int32_t col_offset, uint64_t seed, const int64_t *keys,
                                  hipStream_t s);

// Gauss quadrature of every column after min(k_eff[c], steps) steps:
// psi[c] = norm2[c] e1^T f(T) e1 (1 <= steps <= k).  With `stop` given, a
// record {uid, j > 0} there lowers steps to j (a-posteriori stopping); with
// col_stop given, col_stop[c] > 0 lowers column c's steps to it.  fp64: the
// coefficients come from FP64 vectors (tighter limit on the shift of the
// integral route, see kernels.hip).
hipError_t launch_quadrature(const double *alpha, const double *beta, const int32_t *k_eff,
                             const double *norm2, int32_t k, int32_t steps, int32_t m, double *psi,
                             int32_t *flags, hipStream_t s, bool fp64, const int2 *stop = nullptr,
                             int32_t uid = 0, const int32_t *col_stop = nullptr, int32_t *steps_out = nullptr);
// f(T) e1 for every column (rows >= k_eff are 0), step-major: S[r*m + c]; rot_scratch
// holds rot_capacity(k) recorded rotations (24 bytes each) per column
__host__ __device__ int64_t rot_capacity(int32_t k);
constexpr int64_t kRotBytes = 24;
hipError_t launch_fT_e1(const double *alpha, const double *beta, const int32_t *k_eff,
                        int32_t k, int32_t m, double *S, void *rot_scratch, int32_t *flags,
                        hipStream_t s, bool fp64);

// Theorem 4.8 bracket per column (see kernels.hip): one problem = m columns
// of Lanczos coefficients (layout [m][k]) after `steps` steps
struct BoundArgs {
    const double *alpha, *beta;
    const int32_t *k_eff;
    const double *norm2;
    int32_t k, m, steps;
    double lam_lo, lam_hi;      // 0 < lam_lo < lam_hi
    int32_t n_grid;             // >= 2
    double *lo, *hi;            // [m]
    int32_t *flags;             // QR status bits
    const int32_t *col_stop;    // [m] or NULL: columns with a recorded stop step are skipped
    const int2 *stop_state;     // slots: as in StepArgs (the whole problem is skipped)
    int32_t stop_uid;
    int32_t stop_count;
};
// map entries {problem, group of 4 columns}
hipError_t launch_error_bound(const BoundArgs *args, const int2 *map, int32_t n_entries, hipStream_t s);

struct StopArgs {
    const double *lo, *hi;
    int32_t estimate;           // 0: every hi <= tol (eq. (4.9)); 1: every sqrt(lo hi) <= tol (eq. (4.10))
    int32_t m;
    double tol;
    int32_t step;
    int32_t uid;
    int2 *state;                // {uid, first step with every hi <= tol, or 0}
    int2 *mail;                 // a copy of *state in an array copied to the host at once (or NULL)
};
hipError_t launch_stop_check(const StopArgs *args, int32_t n, hipStream_t s);
// the bracket for the m columns of one problem (args in device memory)
hipError_t launch_error_bound_cols(const BoundArgs *args, int32_t m, hipStream_t s);

// Per-column stopping: a running column (col_stop[c] == 0) whose upper bound
// hi[c] is within tol[c] records `step` in col_stop[c]; *remaining receives
// the number of columns still running.  One block, any m.
struct ColStopArgs {
    const double *lo, *hi, *tol;
    int32_t *col_stop;
    int32_t m, step;
    int32_t *remaining;
    int32_t estimate;           // 0: stop on hi <= tol (eq. (4.9)); 1: on sqrt(lo hi) <= tol (eq. (4.10))
};
hipError_t launch_column_stop(const ColStopArgs *args, hipStream_t s);
constexpr int kBoundGrid = 256;            // grid points of the serving loop's checks
constexpr double kLamLoFraction = 1e-12;   // serving: lower end of the bound interval / lambda_ub

// estimate from psi: kind 0 mean, 1 sum, 2 Hutch++ (first n_sketch summed,
// rest averaged); one estimate per graph from psi[g * ld + c], c < graph_m[g]
hipError_t launch_combine(const double *psi, int32_t m, int32_t kind, int32_t n_sketch,
                          double *estimate, hipStream_t s);
hipError_t launch_combine_graphs(const double *psi, int32_t ld, const int32_t *graph_m, int32_t n_graphs,
                                 int32_t kind, double *estimates, hipStream_t s);

// Y[i*ldy + c] = sqrt(norm2[c]) * sum_j S[j*m + c] Vstore[j][i*ldv + c]  (m <= 128)
hipError_t launch_reconstruct(const void *Vstore, bool fp64, int64_t step_stride, int32_t ldv,
                              const double *S, const double *norm2, int32_t k, int32_t n,
                              int32_t m, void *Y, int32_t ldy, hipStream_t s);

// out[a*nb + b] = sum_i X[i*ldx + a] * Y[i*ldy + b] (FP64 accumulation),
// na <= 128, any nb; uses part (scratch, [chunks][na][nb] doubles, see
// gram_scratch_doubles)
int64_t gram_scratch_doubles(int32_t n, int32_t na, int32_t nb);
hipError_t launch_gram(const void *X, int32_t ldx, const void *Y, int32_t ldy, bool fp64,
                       int32_t n, int32_t na, int32_t nb, double *part, double *out,
                       hipStream_t s);
// upper Cholesky factor of G (na x na, FP64, na <= 128) and its inverse Rinv;
// flags bit 1 when a pivot is not positive
hipError_t launch_cholinv(double *G, double *Rinv, int32_t na, int32_t *flags, hipStream_t s);
// Z[i*ldz + b] = (sub ? Z[i*ldz + b] - s : s), s = sum_a X[i*ldx + a] * M[a*nb + b],
// na <= 128; row-local: Z may alias X only for sub == 0, which needs nb <= 128
hipError_t launch_apply(const void *X, int32_t ldx, const double *M, int32_t na, int32_t nb,
                        void *Z, int32_t ldz, bool fp64, int32_t n, int32_t sub,
                        hipStream_t s);

}  // namespace vne
