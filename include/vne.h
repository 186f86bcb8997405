/*
 * vne.h -- C ABI of the MI355X Lanczos-quadrature engine for the von Neumann
 * entropy S(rho) = tr(-rho log rho) of a sparse symmetric positive
 * semidefinite matrix rho (Benzi, Rinelli, Simunec, "Computation of the von
 * Neumann entropy of large matrices via trace estimators and rational Krylov
 * methods").
 *
 * The engine computes quadratic forms psi = b^T f(A) b, f(x) = -x log x, by
 * the polynomial Krylov (Lanczos) method with Gauss quadrature, eq. (4.2):
 * psi_k = ||b||^2 e_1^T f(T_k) e_1, for a whole block of probe vectors at
 * once, and combines them into a trace estimate: Hutchinson, eq. (3.8);
 * probing with a distance-d colouring, eq. (3.1)-(3.2) and Algorithm 1;
 * Hutch++, eq. (3.9) with f(A) Omega from eq. (4.3).
 *
 * Conventions shared by every entry point
 *  - Every function returns a vne_status; nothing throws or aborts across the
 *    ABI.  After a failure vne_last_error(ctx) describes it (per context; the
 *    context-free helpers write into the caller's msg buffer when given one).
 *  - The caller owns every array it passes.  The library never frees caller
 *    memory.  Arrays marked "host" are plain CPU memory; arrays with a
 *    `location` field may live on the device (VNE_DEVICE: a pointer returned
 *    by hipMalloc or a torch tensor's data_ptr on the context's device).
 *  - Sizes are int64 element counts; index arrays are int32.
 *  - Calls on one context are serialised by a lock of the context.  All
 *    device work of a context's own calls runs on its stream; every call
 *    returns only after its results are in the caller's buffers (the call
 *    synchronizes that stream).  A server (vne_server_*) runs on a stream and
 *    a worker thread of its own.
 *  - Matrix layout: compressed sparse rows with sorted, unique column indices
 *    in [0, n), row_ptr[0] = 0, row_ptr[n] = nnz.  The represented matrix is
 *    A = scale * CSR.  For graph density matrices the CSR holds the exact
 *    integers of the Laplacian L = D - Adj (eq. (2.3)) and scale = 1 / tr(L),
 *    so A = rho exactly and the null vector 1 stays exact (eq. (2.2)).
 *  - Probe blocks on the device are n x m_pad row-major (probe index fastest),
 *    m_pad = m rounded up to the kernel's column tile.
 */
#ifndef VNE_H
#define VNE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VNE_OK = 0,
    VNE_EINVAL = -1,    /* malformed argument or matrix                        */
    VNE_ENOMEM = -2,    /* device allocation failed or the HBM budget is spent */
    VNE_EDEVICE = -3,   /* a HIP runtime call failed                           */
    VNE_ENOTSUP = -4,   /* valid request outside what the library supports     */
    VNE_EBUSY = -5,     /* resource in use (e.g. releasing a graph in a plan)  */
    VNE_ENUMERIC = -6   /* NaN or Inf in a start vector or the coefficients,
                           or a failed factorisation of the Hutch++ sketch  */
} vne_status;

enum { VNE_F32 = 0, VNE_F64 = 1 };          /* element type of values / dense blocks */
enum { VNE_HOST = 0, VNE_DEVICE = 1 };      /* where a caller array lives            */

/* mode bits of an estimate */
enum {
    VNE_MODE_F64 = 1u << 0,     /* FP64 Lanczos vectors (default: FP32 vectors;
                                   alpha/beta sums, coefficients and the
                                   quadrature are FP64 in both modes)          */
    VNE_MODE_DESING = 1u << 1   /* implicit desingularization (Remark 4.6):
                                   start from c = b - (1^T b / n) 1; requires
                                   zero row sums (A 1 = 0)                     */
};

/* probe kinds */
enum {
    VNE_PROBE_RADEMACHER = 0,   /* m Rademacher vectors, estimate = mean (3.8) */
    VNE_PROBE_HUTCHPP = 1,      /* n_sketch + (m - n_sketch) Rademacher vectors,
                                   estimate by Hutch++ (3.9)                   */
    VNE_PROBE_COLORING = 2,     /* indicator vector per colour (3.1),
                                   estimate = sum (3.2)                        */
    VNE_PROBE_DENSE = 3         /* caller-supplied n x m block, estimate = mean */
};

/* validation flags of vne_csr_validate / vne_graph_register */
enum {
    VNE_VALIDATE_SYMMETRIC = 1u << 0,  /* check A = A^T (O(nnz log deg))       */
    VNE_VALIDATE_ZERO_ROWSUM = 1u << 1 /* check every row sums to zero         */
};

typedef struct vne_ctx vne_ctx;

typedef struct {
    int64_t n;                /* rows = columns, n >= 1                          */
    int64_t nnz;              /* stored entries                                  */
    const int32_t *row_ptr;   /* [n+1]                                           */
    const int32_t *col_idx;   /* [nnz]                                           */
    const void *values;       /* [nnz], element type value_dtype                 */
    int32_t value_dtype;      /* VNE_F32 or VNE_F64                              */
    int32_t location;         /* VNE_HOST or VNE_DEVICE, for the three arrays    */
    const int64_t *node_keys; /* host [n] or NULL: key of each row in the probe
                                 hash (the original node id); NULL = row index  */
    double scale;             /* A = scale * CSR, finite and > 0                 */
} vne_csr;

typedef struct {
    int32_t kind;             /* VNE_PROBE_*                                     */
    int32_t m;                /* probe vectors in the block, 1 <= m             */
    uint64_t seed;            /* RADEMACHER / HUTCHPP: hash seed                 */
    int32_t n_sketch;         /* HUTCHPP: N_r = columns of Omega (the first
                                 n_sketch hash columns); G uses the next m-N_r */
    int32_t location;         /* DENSE / COLORING arrays: VNE_HOST/VNE_DEVICE    */
    const int32_t *colors;    /* COLORING: [n] colour of each row in [0, m);
                                 host arrays are checked (VNE_EINVAL), device
                                 arrays are not: a row with a colour outside
                                 [0, m) belongs to no probe vector             */
    const void *dense;        /* DENSE: n x m row-major, FP32 (default mode) or
                                 FP64 (VNE_MODE_F64)                             */
} vne_probes;

typedef struct {
    double estimate;          /* out: trace estimate for this probe kind          */
    double *quad;             /* host [m] or NULL: psi of every quadratic form   */
    double *alpha;            /* host [m*k] or NULL: column c, step j at c*k+j   */
    double *beta;             /* host [m*k] or NULL: same layout; beta_j couples
                                 v_j and v_{j+1}; 0 after a breakdown            */
    int32_t *k_eff;           /* host [m] or NULL: Krylov dimension used         */
    double *norm2;            /* host [m] or NULL: ||c||^2 of the start vector   */
} vne_result;

/* ----------------------------------------------------------------------------
 * Context-free host helpers (no GPU needed).
 * ------------------------------------------------------------------------- */

/* Library version string (static storage). */
const char *vne_version(void);

/* Graph density matrix, eq. (2.3) with the preprocessing of Section 6.1.
 * Input: n_nodes >= 1 and n_edges pairs edges[2*e], edges[2*e+1] in
 * [0, n_nodes) (host).  Self loops are dropped, repeated edges count once
 * (binary weights), and only the largest connected component is kept (ties:
 * the component holding the smallest node id); kept nodes are renumbered in
 * increasing original id.  Output: the Laplacian L = D - Adj of that
 * component in CSR with every diagonal entry stored, values as exact
 * integers in value_dtype, node_ids[i] = original id of row i, and
 * *scale = 1 / tr(L).  Call once with row_ptr == NULL to get *n_out and
 * *nnz_out, then again with arrays of those sizes.  EINVAL on bad input or a
 * component with no edge (tr(L) = 0).  msg (may be NULL) receives a message. */
vne_status vne_laplacian_from_edges(int64_t n_nodes, int64_t n_edges, const int64_t *edges,
                                    int64_t *n_out, int64_t *nnz_out, int32_t *row_ptr,
                                    int32_t *col_idx, void *values, int32_t value_dtype,
                                    int64_t *node_ids, double *scale, char *msg, int64_t msg_len);

/* Structural and numerical checks of a host CSR: sizes, monotone row_ptr,
 * sorted unique in-range columns, finite values, finite positive scale, plus
 * the checks selected by flags (VNE_VALIDATE_*).  EINVAL with a message on
 * the first violation. */
vne_status vne_csr_validate(const vne_csr *csr, uint32_t flags, char *msg, int64_t msg_len);

/* Greedy distance-d colouring, Algorithm 1 of Section 3.1: nodes in order of
 * descending degree (number of off-diagonal entries; ties by increasing row
 * index), each taking the smallest colour (from 0) not used by an earlier
 * node within geodesic distance d in the graph of the matrix.  Host CSR only.
 * colors_out: host [n]; *n_colors = number of colours used.  1 <= d <= 254
 * (VNE_EINVAL otherwise). */
vne_status vne_color_greedy(const vne_csr *csr, int32_t d, int32_t *colors_out,
                            int32_t *n_colors, char *msg, int64_t msg_len);

/* ----------------------------------------------------------------------------
 * Device context and graph registry.
 * ------------------------------------------------------------------------- */

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * memory the context allocates for graphs and workspaces (0 = no cap).
 * hip_stream: a hipStream_t to run on (borrowed), or NULL for the null
 * stream.  *out receives the context. */
vne_status vne_ctx_create(int device, uint64_t hbm_budget_bytes, void *hip_stream, vne_ctx **out);

/* Release every device allocation of the context and the context itself. */
void vne_ctx_destroy(vne_ctx *ctx);

/* Message of the last failed call on ctx ("" if none); static until the next
 * call on ctx.  NULL ctx gives the message of the last failed vne_ctx_create. */
const char *vne_last_error(const vne_ctx *ctx);

/* Replace the stream (hipStream_t, borrowed; NULL = null stream). */
vne_status vne_ctx_set_stream(vne_ctx *ctx, void *hip_stream);

/* Device bytes currently held by the context. */
vne_status vne_ctx_memory(const vne_ctx *ctx, uint64_t *bytes_in_use);

/* Register a matrix.  HOST arrays are copied into device memory owned by the
 * context until vne_graph_release; DEVICE arrays are borrowed and must stay
 * valid and unchanged until release.  The structure is validated (see
 * vne_csr_validate; DEVICE arrays are copied back for the checks).  The work
 * schedule of the Lanczos kernels (row segments of long rows, cost-balanced
 * blocks) is built here.  *graph_id receives a handle >= 0. */
vne_status vne_graph_register(vne_ctx *ctx, const vne_csr *csr, uint32_t validate_flags,
                              int32_t *graph_id);

/* Free a registered matrix and every cached workspace built for it. */
vne_status vne_graph_release(vne_ctx *ctx, int32_t graph_id);

/* ----------------------------------------------------------------------------
 * Estimates.
 * ------------------------------------------------------------------------- */

/* k_steps Lanczos steps on every probe vector of `probes` for the matrix
 * `graph_id`, Gauss quadrature of each quadratic form (eq. (4.2)) and the
 * estimator of the probe kind.  1 <= k_steps <= 128.  With VNE_MODE_DESING
 * each start vector b is replaced by c = b - (1^T b / n) 1 (Remark 4.6).
 * Breakdown: a column stops after step j when beta_j <= tau (|alpha_j| +
 * beta_{j-1}), tau = 2^-18 for FP32 vectors and 2^-23 for FP64 vectors;
 * k_eff records j.  Results go to the caller's host buffers in *out (each may
 * be NULL except `out` itself).  For HUTCHPP, quad/alpha/beta/k_eff/norm2
 * describe the final block [Q | G~] of m quadratic forms (the sketch's own
 * coefficients are not returned).  Workspaces are cached per (graph, probe
 * width, k, mode, kind) and reused by later calls.  The column tile of a
 * workspace is picked on its first use by timing each admissible tile's
 * whole step loop (see vne_last_plan).  When the block spans two or more
 * tiles, its tiles run as up to two concurrent chains, each chain's step
 * loop on a stream the context owns (VNE_CHAINS, default 2, 1 disables); the
 * context's stream waits for them, and the results are bitwise those of one
 * chain. */
vne_status vne_entropy_estimate(vne_ctx *ctx, int32_t graph_id, const vne_probes *probes,
                                int32_t k_steps, uint32_t mode, vne_result *out);

/* n_queries independent estimates in one stacked launch per Lanczos step:
 * the matrices are placed as the diagonal blocks of one block-diagonal
 * matrix (rows, work blocks and probe blocks of query q after those of
 * queries 0..q-1), so that every step is one SpMM + recurrence launch over
 * all of them.  Query q runs k_steps[q] steps on probes[q] for
 * graph_ids[q] and writes out[q]; each result is the one vne_entropy_estimate
 * gives for that query alone, up to the order of the FP64 reductions (the
 * per-graph sums add the same partials in the same order; only the first
 * level of the reduction differs).  All queries take one probe kind, one of
 * RADEMACHER, COLORING or DENSE (HUTCHPP is not batched: VNE_ENOTSUP);
 * COLORING and DENSE probes must be HOST arrays here.  A graph id may appear
 * more than once.  The stacked copy of the matrices is cached for the exact
 * id sequence (at most VNE_MAX_SETS such sets, default 4, least recently
 * used freed first); the column tile of the launch is picked on first use by
 * timing each admissible tile's whole captured step loop (VNE_AUTOTUNE=0
 * disables; VNE_AUTOTUNE_CACHE=<file> keeps the choices).  Errors: VNE_EINVAL for bad
 * ids, sizes or mode bits; VNE_ENOMEM when the HBM budget is exceeded. */
vne_status vne_entropy_estimate_batch(vne_ctx *ctx, int32_t n_queries, const int32_t *graph_ids,
                                      const vne_probes *probes, const int32_t *k_steps,
                                      uint32_t mode, vne_result *out);

/* Per-vector stopping rule of vne_entropy_estimate_adaptive. */
enum { VNE_STOP_BOUND = 0, VNE_STOP_ESTIMATE = 1 };

typedef struct {
    const double *tol;          /* host [m]: tolerance of each quadratic form (> 0)        */
    double lam_lo, lam_hi;      /* interval of the Theorem 4.8 bound, 0 < lam_lo < lam_hi  */
    int32_t n_grid;             /* log-spaced points of the interval, 2..65536 (0: 256)    */
    int32_t stop;               /* VNE_STOP_BOUND: stop when the upper bound hi of the
                                   bracket (eq. (4.9)) is within tol; VNE_STOP_ESTIMATE:
                                   when the geometric mean sqrt(lo hi) of the bracket
                                   (eq. (4.10)) is (no guarantee: Remark 4.11)             */
} vne_stop_rule;

/* Quadratic forms with an a-posteriori stopping rule (Theorem 4.8, used as
 * in step 3 of Algorithm 2): Lanczos on every probe vector as in
 * vne_entropy_estimate, with the bracket (the one vne_error_bounds returns,
 * on [rule->lam_lo, rule->lam_hi] with rule->n_grid points) evaluated for
 * every running vector after steps 3, 5, 7, ... (at most k_max).  Vector c
 * stops at the first such step s with hi <= rule->tol[c] (rule->stop =
 * VNE_STOP_BOUND) or sqrt(lo hi) <= rule->tol[c] (VNE_STOP_ESTIMATE); its
 * psi is the Gauss quadrature after min(k_eff, s) steps.  A stopped vector
 * is not computed further: a column tile of the step kernels whose vectors
 * have all stopped (or broken down) is skipped, and so are groups of
 * stopped vectors in the normalize pass.  A vector that never meets its
 * tolerance ends at k_max.  The block stops when every vector has stopped
 * (the call synchronises its stream after each check to read the running
 * count).  steps_out (host [m], may be
 * NULL) receives each vector's stop step, or 0 for a vector that never met
 * its tolerance (its psi is the quadrature after k_max steps).  out->alpha /
 * out->beta entries past a vector's stop step are unspecified.  Probe kinds RADEMACHER, COLORING and DENSE on one graph;
 * 3 <= k_max <= 128.  The interval must contain the spectrum the start
 * vectors see for hi to bound the error (see vne_error_bounds). */
vne_status vne_entropy_estimate_adaptive(vne_ctx *ctx, int32_t graph_id, const vne_probes *probes,
                                         int32_t k_max, uint32_t mode, const vne_stop_rule *rule,
                                         vne_result *out, int32_t *steps_out);

/* Probing method with a relative accuracy target: Algorithm 2 of Section 5. */
enum { VNE_SELECT_HEURISTIC = 0, VNE_SELECT_BOUND = 1 };

typedef struct {
    double rel_eps;             /* target relative error epsilon, 0 < rel_eps < 1          */
    int32_t select;             /* VNE_SELECT_HEURISTIC: eq. (5.1) from T_1..T_3;
                                   VNE_SELECT_BOUND: Corollary 3.2 with a = 0               */
    int32_t d_max;              /* largest distance considered, 1..64 (0: 16)              */
    int32_t k_max;              /* step cap per quadratic form, 3..128 (0: 128)            */
    uint32_t mode;              /* VNE_MODE_* bits of the Lanczos runs                     */
    double lam_lo_fraction;     /* lower end of the bound interval / lambda_ub (0: 1e-12)  */
    int32_t n_grid;             /* bound grid points (0: 256)                              */
    int32_t stop;               /* VNE_STOP_BOUND or VNE_STOP_ESTIMATE (vne_stop_rule)     */
} vne_probing_cfg;

typedef struct {
    double estimate;            /* T_d: sum of the psi of the final pass                   */
    int32_t d, n_colors;        /* selected distance and its colour count                  */
    int32_t fallback;           /* 1: Corollary 3.2 chose d                                */
    int32_t capped;             /* 1: no d <= d_max met the target (d = d_max)             */
    int32_t unconverged;        /* colours of the final pass that ended at k_max           */
    int32_t passes;             /* distance-d passes run (colouring + Lanczos)             */
    double t_pre[3];            /* T_1, T_2, T_3 of the heuristic (0 with the bound)       */
    double e1, q[2];            /* fit: |T_2 - T_1|, q for kappa = 2 and 3                 */
    double s_lower;             /* -log tr(A^2)                                            */
    double s_hat;               /* rough entropy behind eps_hat                            */
    double eps_hat;             /* absolute target for d and for the Krylov part           */
    int64_t vector_steps;       /* sum over passes and colours of the steps used           */
    int64_t block_steps;        /* sum over passes of the steps the block ran              */
    double color_ms, lanczos_ms;/* host colouring time; Lanczos passes (wall, synchronised) */
    int32_t *colors;            /* host [n] or NULL: colouring of the final pass           */
    double *quad;               /* host [quad_cap] or NULL: psi of the final pass          */
    int32_t *steps;             /* host [quad_cap] or NULL: stop step per colour (0: k_max
                                   reached without meeting the tolerance)                   */
    int32_t quad_cap;           /* the first min(quad_cap, n_colors) entries are written  */
} vne_probing_result;

/* Algorithm 2 for a unit-trace matrix (a density matrix; EINVAL otherwise).
 * With S_lower = -log tr(A^2) <= S(A), lambda_ub = max_i sum_j |A_ij|:
 *  1. select = HEURISTIC: distance-d passes for d = 1, 2, 3 with
 *     eps_hat0 = rel_eps S_lower / 2; then s_hat = max(S_lower, T_1, T_2, T_3)
 *     (every T_d is a lower bound of S for an M-matrix, Proposition 3.6),
 *     eps_hat = rel_eps s_hat / 2 and d from the fit of eq. (5.1) (the larger
 *     of the kappa = 2 and kappa = 3 models; Corollary 3.2 when the fit has no
 *     decay).  select = BOUND: s_hat = S_lower and the smallest d >= 2 with
 *     n lambda_ub / (2 (d^2 - 1)) <= eps_hat.
 *  2. a greedy distance-d colouring (Algorithm 1, as vne_color_greedy);
 *  3. psi of each colour indicator v_l with the stopping rule of
 *     vne_entropy_estimate_adaptive (cfg->stop), tolerance eps_hat |V_l| / n
 *     (eq. (5.3)), on [lam_lo_fraction lambda_ub, lambda_ub];
 *  4. estimate = sum of psi.
 * A selected d of 1, 2 or 3 reuses that preprocessing pass.  The colourings
 * run on the host; the passes on the context's stream. */
vne_status vne_entropy_probing(vne_ctx *ctx, int32_t graph_id, const vne_probing_cfg *cfg,
                               vne_probing_result *res);

/* The distance choice of step 1, for callers that plan on their own (host
 * only): the eq. (5.1) fit from T[3] = {T_1, T_2, T_3} (use_bound = 0) or
 * Corollary 3.2 alone (use_bound = 1, T may be NULL), for a target eps_hat,
 * size n and lambda_ub.  1 <= d_max <= 64. */
typedef struct {
    int32_t d, fallback, capped;
    double e1, q[2];
    double model;               /* the chosen rule's error value at d                      */
} vne_distance_choice;
vne_status vne_probing_select(const double *T, double eps_hat, double n, double lambda_ub, int32_t d_max,
                              int32_t use_bound, vne_distance_choice *out);

/* Adaptive Hutch++: Hutch++ (eq. (3.9)) with the sketch width N_r and the
 * Hutchinson count N_H chosen for a target of the form of eq. (3.10),
 * P[|estimate - tr f(A)| >= eps_hat] <= delta (Section 3.2; the adaptive
 * Hutch++ implementation of Section 5).  The paper takes this algorithm
 * from elsewhere without stating it; the rule below is this library's
 * reading of what the paper fixes (eps_hat = eps/2 tr f(A) for a relative
 * target, at least three products with f(A), N_r and N_H chosen for the
 * least effort N_r + (N_r + N_H)):
 *  - rounds of sketch width N_r = r_first, 2 r_first, 4 r_first, ... (at
 *    most r_max): Omega = the first N_r Rademacher hash columns of `seed`
 *    (the same columns in every round), Q an orthonormal basis of
 *    f(A) Omega (eq. (4.3)), n_pilot deflated forms on the Rademacher
 *    hash columns 128, 129, ... of `seed`;
 *  - round estimate t = sum of the Q forms + mean of the deflated forms;
 *    eps_hat = abs_eps, or rel_eps / 2 |t|;
 *  - N_H = max(n_pilot, ceil(min((z s / eps_hat)^2, 1e15))), s the sample
 *    standard deviation of the deflated forms, z the two-sided normal
 *    quantile of delta; effort 2 N_r + N_H;
 *  - a next round runs only while its effort could still be below the least
 *    so far (2 N_r' + n_pilot < least effort); the round of least effort is
 *    kept (the earlier on ties);
 *  - final: Hutch++ with the kept N_r and min(N_H, n_h_max) deflated forms
 *    (their first n_pilot columns are the pilot's): the kept round itself
 *    when it asked for the pilot's count, else a run on the kept round's Q
 *    (kept on the device, not sketched again) with new deflated columns.
 * Every Krylov run takes k_steps Lanczos steps (the caller picks k_steps
 * for the Krylov share of the error, e.g. with vne_plan_steps).  The round
 * statistics (mean, standard deviation, counts) are computed on the host
 * from the device forms.  quad (host [quad_cap], may be NULL) receives the
 * final forms, the N_r Q forms first.  Errors: VNE_EINVAL for bad
 * arguments, VNE_ENOMEM when a round's workspace exceeds the budget,
 * VNE_ENUMERIC as for vne_entropy_estimate. */
typedef struct {
    double rel_eps;             /* relative target, 0 < rel_eps < 1 (used when abs_eps == 0) */
    double abs_eps;             /* absolute tolerance eps_hat (> 0: overrides rel_eps)       */
    double delta;               /* failure probability, 0 < delta < 1                        */
    int32_t k_steps;            /* Lanczos steps of every Krylov run, 1..128                 */
    int32_t n_pilot;            /* deflated forms per round, 2..1024 (0: 16)                 */
    int32_t r_first;            /* first sketch width, 1..128 (0: 3)                         */
    int32_t r_max;              /* widest sketch, r_first..128 (0: max(96, r_first))         */
    int32_t n_h_max;            /* most deflated forms of the final run, n_pilot..2^20
                                   (0: 4096)                                                 */
    uint32_t mode;              /* VNE_MODE_* bits                                           */
    uint64_t seed;
} vne_hutchpp_cfg;

#define VNE_HUTCHPP_MAX_ROUNDS 8
typedef struct {
    double estimate;            /* final Hutch++ estimate                                    */
    double std_error;           /* s / sqrt(N_H) of the final deflated forms                 */
    double eps_hat;             /* tolerance of the kept round                               */
    int32_t n_sketch, n_hutch;  /* kept N_r; N_H of the final run                            */
    int32_t capped;             /* 1: n_h_max cut the kept round's N_H                       */
    int32_t rounds;             /* rounds run                                                */
    int32_t round_nr[VNE_HUTCHPP_MAX_ROUNDS], round_nh[VNE_HUTCHPP_MAX_ROUNDS];
    double round_estimate[VNE_HUTCHPP_MAX_ROUNDS], round_sd[VNE_HUTCHPP_MAX_ROUNDS];
    int64_t krylov_runs;        /* Lanczos runs: 2 N_r + n_pilot per round, N_r + N_H for a
                                   final run on a kept Q                                     */
    double ms;                  /* wall time of the call                                     */
} vne_hutchpp_result;
vne_status vne_hutchpp_adaptive(vne_ctx *ctx, int32_t graph_id, const vne_hutchpp_cfg *cfg,
                                vne_hutchpp_result *res, double *quad, int32_t quad_cap);

/* A-posteriori error bracket of Theorem 4.8 for the polynomial Krylov
 * method, per column of a result (host arrays laid out as in vne_result:
 * alpha, beta [m*k], k_eff, norm2 [m]) after min(k_eff[c], steps) steps:
 * lo[c] <= |psi - psi_m| <= hi[c] with lo, hi = ||c||^2 min, max |g_m(z)| of
 * eq. (4.8) for f = -x log x over [lam_lo, lam_hi].  g_m is evaluated in
 * its residue form -int_0^inf t (beta_m e1^T (T_m + tI)^{-1} e_m)^2 / (t + z)
 * dt, in which |g_m| decreases in z, so hi and lo are its values at lam_lo
 * and lam_hi; a column whose T_m has a Ritz value below -5e-16 of its scale
 * (rounding) is evaluated term by term over n_grid log-spaced points plus
 * the Ritz values inside the interval instead.  The interval
 * must contain the spectrum of A seen by the start vectors (for a Laplacian
 * density matrix with VNE_MODE_DESING: [lambda_2, lambda_n]; any
 * 0 < lam_lo <= lambda_2 and lam_hi >= lambda_n, e.g. a Gershgorin bound,
 * keep hi an upper bound).  Ritz values below lam_lo are raised to it.  A
 * column whose recurrence stopped on beta = 0 gets lo = hi = 0.  Needs
 * 1 <= steps <= k <= 128, 0 < lam_lo < lam_hi, 2 <= n_grid <= 65536. */
vne_status vne_error_bounds(vne_ctx *ctx, int32_t m, int32_t k, const double *alpha, const double *beta,
                            const int32_t *k_eff, const double *norm2, int32_t steps, double lam_lo,
                            double lam_hi, int32_t n_grid, double *lo, double *hi);

/* Kernel timing for measurement: when enabled, the context records a HIP
 * event pair on its stream around every launch of the Lanczos step kernel
 * and accumulates their durations.  vne_kernel_timing returns (and with
 * reset != 0 clears) the number of timed launches, their total milliseconds
 * and the algorithmic bytes those launches were due to move (CSR once, the
 * gathered block once, the previous block once, the new block once per
 * step).  Timing adds one event pair per launch and no synchronization
 * inside a call. */
vne_status vne_enable_kernel_timing(vne_ctx *ctx, int32_t enable);
vne_status vne_kernel_timing(vne_ctx *ctx, int32_t reset, int64_t *launches, double *total_ms,
                             double *algorithmic_bytes);

/* Rational Krylov cross-check of the polynomial path (Section 4: the
 * rational Krylov space q_{m-1}(A)^{-1} K_m(A, b) of eq. (4.1) and the
 * form psi_m = ||b||^2 e_1^T f(A_m) e_1 of eq. (4.2) with A_m = V_m^T A V_m;
 * rational Arnoldi with full orthogonalization, Remark 4.2).  FP64 only
 * (VNE_MODE_F64, else VNE_ENOTSUP); RADEMACHER, COLORING or DENSE probes,
 * 1 <= m <= 128; start vectors as in vne_entropy_estimate (VNE_MODE_DESING
 * centres them).  Step j applies A to v_j, adds column j of A_m, evaluates
 * psi_j, and (j < steps) takes w = A v_j for a pole at infinity or solves
 * (I - A / xi) w = A v_j for a finite pole xi < 0 (symmetric positive
 * definite; conjugate gradients on the sparse product until the residual
 * is within cg_tol of the right-hand side, at most cg_max iterations), then
 * orthogonalizes w twice against v_1..v_j (v_{j+1} = w / ||w||; a column
 * whose w vanishes in the orthogonalization, an invariant subspace, stops
 * growing).  Poles: `poles` [steps - 1] gives the pole of every step
 * (+INFINITY or < 0) for all columns; with poles == NULL each column starts
 * with poles at infinity and switches to `finite_poles` (in order; past the
 * list, infinity again) after the first step j >= ell + 2 at which its error
 * bound err_j has not dropped by c^ell since step j - ell - 1,
 * err_j >= c^ell err_{j-ell-1} (the switch rule of the Krylov method
 * implementation of Section 5; the paper's choice is ell = 3, c = 0.75).
 * err_j is the a-posteriori upper bound of Theorem 4.8, eq. (4.9), or with
 * estimate != 0 the geometric mean of eq. (4.10), for the polynomial Krylov
 * space of step j over [lam_lo, lam_hi] (0 < lam_lo < lam_hi: an interval
 * that holds the spectrum of A on the Krylov space, e.g. [lambda_2,
 * lambda_max] for centred vectors of a connected graph's Laplacian).
 * Results: psi after the last step, psi after every step, the applications
 * of A behind each (one per basis vector plus every conjugate-gradient
 * iteration), the switch step per column and the basis size.  The call
 * allocates its workspace (steps + 6 blocks of n x m_pad FP64) and frees it
 * before returning. */
typedef struct {
    int32_t steps;              /* basis vectors per column (Krylov dimension), 1..64     */
    const double *poles;        /* host [steps - 1] or NULL (switch rule)                 */
    const double *finite_poles; /* switch rule: host [n_finite] negative poles, in order   */
    int32_t n_finite;
    int32_t ell;                /* switch rule: window (>= 1)                             */
    double c;                   /* switch rule: factor, 0 < c < 1                          */
    double cg_tol;              /* relative residual of a shifted solve (0: 1e-10)        */
    int32_t cg_max;             /* iteration cap of one solve (0: 20000)                  */
    double lam_lo, lam_hi;      /* switch rule: interval of the error bound               */
    int32_t estimate;           /* switch rule: 0 upper bound (4.9), 1 estimate (4.10)    */
} vne_rational_cfg;

typedef struct {
    double *quad;               /* host [m] or NULL: psi after the last step              */
    double *psi_steps;          /* host [m*steps] or NULL: psi_j at c*steps + j - 1        */
    int64_t *apps_steps;        /* host [m*steps] or NULL: applications of A behind psi_j  */
    int32_t *switch_step;       /* host [m] or NULL: step of the switch (0: none)         */
    int32_t *basis;             /* host [m] or NULL: basis vectors built                  */
    double *norm2;              /* host [m] or NULL: ||c||^2 of the start vector          */
    double *err_steps;          /* host [m*steps] or NULL: switch rule's err_j up to the
                                   switch (0 after it, and with explicit poles)           */
    int64_t cg_iterations;      /* out: conjugate-gradient iterations, all columns        */
    double ms;                  /* out: wall time of the call                             */
} vne_rational_out;

vne_status vne_rational_quadforms(vne_ctx *ctx, int32_t graph_id, const vne_probes *probes, uint32_t mode,
                                  const vne_rational_cfg *cfg, vne_rational_out *out);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the estimate of
 * vne_entropy_estimate for RADEMACHER, COLORING or DENSE probes (HUTCHPP:
 * VNE_ENOTSUP), with the same arguments and results, that calls no
 * allocating routine.  Its whole workspace (probe and Lanczos blocks,
 * coefficients, reduction partials, results) is carved from one static
 * device array of VNE_NOALLOC_SCRATCH_BYTES per GPU, which the library holds
 * from its first context on that GPU until the process ends; host colour or
 * dense arrays are staged in it too.  A request whose workspace does not
 * fit fails with VNE_ENOMEM (the message gives the bytes it needed); about
 * 16 n m_pad bytes of FP32 vectors (32 for FP64) plus coefficients and
 * partials, e.g. n = 1e5 rows and 32 probes.  The graph's device arrays are
 * built by vne_graph_register.  Steps are launched one by one (no captured
 * graph, no autotuner: the column tile of the byte model, or VNE_TILE) and
 * results go straight to the caller's host buffers; the call synchronizes
 * the context's stream.  Every call on a GPU shares that GPU's array and
 * leaves its contents behind (what must start at zero is cleared by each
 * call): calls that overlap on one GPU, from different contexts or
 * processes' threads, race and must be serialized by the caller.  Results
 * are bitwise those of vne_entropy_estimate with the same column tile. */
#define VNE_NOALLOC_SCRATCH_BYTES (64ull << 20)
vne_status vne_entropy_estimate_noalloc(vne_ctx *ctx, int32_t graph_id, const vne_probes *probes,
                                        int32_t k_steps, uint32_t mode, vne_result *out);

/* Diagnostics: the column tile (columns per work block of the Lanczos step
 * kernels) and the padded block width m_pad of the Lanczos run of the last
 * estimate on ctx (for Hutch++, its quadratic-form block; 0, 0 before any
 * estimate).  The tile comes from the autotuner on a plan's first use (it
 * times the whole step loop of every tile that divides the padded width,
 * concurrent chains included, and keeps the fastest); VNE_AUTOTUNE=0 keeps
 * the byte model's tile of plan creation, VNE_TILE forces one. */
vne_status vne_last_plan(const vne_ctx *ctx, int32_t *tile, int32_t *m_pad);

/* ----------------------------------------------------------------------------
 * Serving loop (continuous batching).
 *
 * A server owns a worker thread, a HIP stream (default priority) and an
 * arena of device memory for the state of running queries.  A query asks for
 * the entropy estimate of a registered graph with Rademacher probes (eq.
 * (3.8)).  It is split into slot tasks of at most max_cols probe columns;
 * tasks wait in arrival order and are admitted while fewer than max_slots
 * run and the arena has room for their vectors and coefficients (a task that
 * does not fit waits, and the ones behind it wait too; a task larger than the
 * whole arena fails its query with VNE_ENOMEM).  Every tick advances all
 * running tasks by one Lanczos step, whatever their graphs, in one set of
 * launches; a task that reaches its step count gets its Gauss quadrature and
 * frees its slot at once, and the query's estimate is combined on the device
 * when its last task ends.  A task's arithmetic depends only on its own graph,
 * probes and step count, so a query's result is bitwise the same alone and
 * among any other queries (for the same server mode).  Two or four
 * 16-column tasks (FP32 mode) of the same graph with the same step cap and
 * stopping rule may share a group slot, admitted together: the 16-column
 * tiles of a work block run in one workgroup and read each neighbour's 32 or
 * 64 columns as one run of 128 or 256 bytes, where one task alone would use
 * half of every cache line it fetches.  The configuration's
 * max_group (1, 2 or 4; default 2) sets the largest group; a group is
 * the largest power of two of the waiting partners that the free mailbox
 * entries and the arena allow.  Each task keeps its own probes, stop record
 * and results, with the arithmetic it has alone; a group slot's step kernels
 * stop running once every task has met its stopping rule.
 *
 * rel_eps == 0: the query gives m (<= max_probes) and k_steps (<= 128).
 * rel_eps > 0: half of the relative error budget goes to the quadrature and
 * half to sampling (Remarks 5.1, 5.2).  Steps: at most the smallest k with
 * 2 n lambda_ub / (4 ((2k-1)^2 - 1)) <= (rel_eps / 2) S_lower (Proposition 4.4
 * with the gamma = 0 bound of Remark 2.3, ||c||^2 <= n), where lambda_ub is
 * the Gershgorin bound max_i sum_j |A_ij| and S_lower = -log tr(A^2) <= S(A)
 * for a unit-trace PSD matrix (otherwise k = max_steps, no early stop).  A
 * task stops earlier at the first of steps 3, 5, 7, ... at which the Theorem
 * 4.8 upper bound (vne_error_bounds over [1e-12 lambda_ub, lambda_ub], 256
 * grid points) is within (rel_eps / 2) S_lower for each of its probes; the
 * step is recorded on the device, so the result does not depend on when the
 * worker notices it.  Probes: a pilot of
 * pilot_probes columns runs first; N = ceil((z sd / ((rel_eps / 2) mean))^2)
 * over its quadratic forms, clamped to [pilot_probes, max_probes] and, when
 * above the pilot, rounded up to whole groups of 16 columns; the pilot's
 * forms are kept and columns pilot_probes..N-1 follow.  After each stage the
 * count is planned again from all forms so far (up to 4 plans), so that the
 * realized spread, not only the pilot's, meets the target.  Tasks are max_cols
 * wide while that much is left, then powers of two of at least 16 columns.
 *
 * Thread safety: submit, poll and stats may be called from any thread.
 * While a server runs, its context may still register graphs and run
 * estimates (they take the context lock); a graph with queries in the server
 * cannot be released (VNE_EBUSY).  Stop every server of a context before
 * destroying it.  The first query on a graph builds the graph's device arrays
 * if no estimate has done so.
 * ------------------------------------------------------------------------- */

typedef struct vne_server vne_server;

typedef struct {
    int32_t max_slots;          /* tasks running at once (0: 256) */
    uint64_t arena_bytes;       /* device memory for running tasks (0: a quarter of free memory) */
    int32_t max_cols;           /* probe columns per task (0: 256; at most 4096) */
    int32_t pilot_probes;       /* pilot width (0: 16) */
    int32_t max_probes;         /* cap on a query's probe count (0: 4096) */
    int32_t max_steps;          /* cap on the planned step count (0: 100; at most 128) */
    double z;                   /* standard errors of the sampling bound (0: 2.576, delta = 1e-2) */
    uint32_t mode;              /* VNE_MODE_* bits of every query of the server */
    int32_t max_group;          /* largest group slot of 16-column FP32 tasks: 1 (none), 2 or 4
                                   (0: 2); other values fail with VNE_EINVAL */
    int32_t stop;               /* check of a rel_eps query's tasks: VNE_STOP_BOUND (0) stops a
                                   task when the upper bound of every column's bracket
                                   (eq. (4.9)) is within tol; VNE_STOP_ESTIMATE when the
                                   geometric mean sqrt(lo hi) of every bracket (eq. (4.10)) is
                                   (no guarantee: Remark 4.11); other values: VNE_EINVAL */
} vne_server_cfg;

typedef struct {
    int32_t graph_id;
    double rel_eps;             /* > 0: probes and steps from the error rule above */
    int32_t m;                  /* rel_eps == 0: probe count */
    int32_t k_steps;            /* rel_eps == 0: Lanczos steps */
    uint64_t seed;              /* probe seed; query columns are hash columns 0..N-1 */
} vne_query;

typedef struct {
    vne_status status;          /* of the query itself */
    char message[128];          /* "" on success */
    double estimate;            /* eq. (3.8) over the N quadratic forms */
    double std_error;           /* sample standard deviation of the forms / sqrt(N) */
    double quad_bound;          /* rel_eps > 0: the per-form quadrature error target */
    int32_t probes, steps;      /* N, and the most Lanczos steps a task of the query used */
    double queue_ms;            /* submit -> first task admitted */
    double latency_ms;          /* submit -> result ready on the host */
} vne_query_result;

typedef struct {
    int64_t ticks, tasks, queries_done;
    double slot_occupancy;      /* mean running tasks per tick */
    uint64_t arena_bytes, arena_in_use, arena_peak;
    int32_t active, pending;    /* running and waiting tasks */
    int64_t pair_slots;         /* group slots admitted with two tasks */
    int64_t group_tasks;        /* tasks admitted into group slots (two or four 16-column
                                   tasks of one graph) */
} vne_server_info;

/* Start a server on ctx.  cfg is copied.  Fails with VNE_ENOMEM when the
 * arena does not fit the context's budget or the device. */
vne_status vne_server_start(vne_ctx *ctx, const vne_server_cfg *cfg, vne_server **out);

/* Queue a query; *ticket identifies it.  VNE_EINVAL for a bad graph id or
 * bad sizes (message in vne_last_error(ctx)); VNE_EBUSY once stop began. */
vne_status vne_server_submit(vne_server *srv, const vne_query *query, uint64_t *ticket);

/* Wait up to timeout_ms (-1: no limit, 0: do not wait) for a query.  On
 * VNE_OK *res holds the result (res->status is the query's own status) and
 * quad (may be NULL) receives min(N, quad_cap) quadratic forms; the ticket is
 * then forgotten.  VNE_EBUSY: not finished yet.  VNE_EINVAL: unknown ticket. */
vne_status vne_server_poll(vne_server *srv, uint64_t ticket, int32_t timeout_ms, vne_query_result *res,
                           double *quad, int32_t quad_cap);

vne_status vne_server_stats(vne_server *srv, vne_server_info *stats);

/* Finish every queued and running query, stop the worker and free the
 * server's memory.  srv is invalid afterwards. */
vne_status vne_server_stop(vne_server *srv);

/* The error rule of the serving loop, for callers that plan on their own:
 * smallest k >= 2 (at most k_max) with 2 norm2 lambda_max / (4 ((2k-1)^2-1))
 * <= share * rel_eps * s_lower; and ceil((z sigma / (share rel_eps s_hat))^2)
 * clamped to [n_min, n_max]. */
int32_t vne_plan_steps(double norm2, double lambda_max, double s_lower, double rel_eps, double share,
                       int32_t k_max);
int32_t vne_plan_probes(double s_hat, double sigma, double rel_eps, double share, double z, int32_t n_min,
                        int32_t n_max);

#ifdef __cplusplus
}
#endif

#endif /* VNE_H */
