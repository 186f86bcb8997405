// gfx950 kernels of the Lanczos-quadrature entropy engine.
//
// Layout: probe blocks are n x m_pad row-major (probe index fastest), so the
// SpMM gathers one contiguous m-vector per stored entry.  Lanczos vectors are
// FP32 (FP64 in FP64 mode); every dot product, the alpha/beta coefficients
// and the quadrature are FP64.  Reductions are two-stage with a fixed
// summation order (no floating-point atomics), so results are bitwise
// reproducible for a given launch shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "kernels.h"

namespace vne {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

template <typename T, int N> struct VecOf;
template <> struct VecOf<float, 4> { using type = float4; };
template <> struct VecOf<double, 2> { using type = double2; };

template <typename T, int N>
__device__ __forceinline__ void load_vec(const T *p, T (&out)[N]) {
    using V = typename VecOf<T, N>::type;
    V v = *reinterpret_cast<const V *>(p);
    const T *q = reinterpret_cast<const T *>(&v);
#pragma unroll
    for (int k = 0; k < N; ++k) out[k] = q[k];
}

template <typename T, int N>
__device__ __forceinline__ void store_vec(T *p, const T (&in)[N]) {
    using V = typename VecOf<T, N>::type;
    V v;
    T *q = reinterpret_cast<T *>(&v);
#pragma unroll
    for (int k = 0; k < N; ++k) q[k] = in[k];
    *reinterpret_cast<V *>(p) = v;
}

// Streaming accesses (read or written once per step) carry the non-temporal
// hint so that the caches keep the gathered block instead.
typedef float nf4 __attribute__((ext_vector_type(4)));
typedef double nd2 __attribute__((ext_vector_type(2)));
template <typename T, int N> struct NVecOf;
template <> struct NVecOf<float, 4> { using type = nf4; };
template <> struct NVecOf<double, 2> { using type = nd2; };

template <typename T, int N>
__device__ __forceinline__ void load_vec_nt(const T *p, T (&out)[N]) {
    using V = typename NVecOf<T, N>::type;
    V v = __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
    const T *q = reinterpret_cast<const T *>(&v);
#pragma unroll
    for (int k = 0; k < N; ++k) out[k] = q[k];
}

template <typename T, int N>
__device__ __forceinline__ void store_vec_nt(T *p, const T (&in)[N]) {
    using V = typename NVecOf<T, N>::type;
    V v;
    T *q = reinterpret_cast<T *>(&v);
#pragma unroll
    for (int k = 0; k < N; ++k) q[k] = in[k];
    __builtin_nontemporal_store(v, reinterpret_cast<V *>(p));
}

// three FP32 columns per lane (tiles of 3 * 2^j columns): 12-byte runs, one
// three-dword access each (a 3-wide vector type with 4-byte alignment; the
// default alignment of a 3-wide vector is 16 bytes)
typedef float f3v __attribute__((ext_vector_type(3)));
typedef f3v __attribute__((aligned(4))) f3u;
template <>
__device__ __forceinline__ void load_vec<float, 3>(const float *p, float (&out)[3]) {
    const f3v v = *reinterpret_cast<const f3u *>(p);
    out[0] = v.x;
    out[1] = v.y;
    out[2] = v.z;
}
template <>
__device__ __forceinline__ void store_vec<float, 3>(float *p, const float (&in)[3]) {
    f3v v;
    v.x = in[0];
    v.y = in[1];
    v.z = in[2];
    *reinterpret_cast<f3u *>(p) = v;
}
template <>
__device__ __forceinline__ void load_vec_nt<float, 3>(const float *p, float (&out)[3]) {
    const f3v v = __builtin_nontemporal_load(reinterpret_cast<const f3u *>(p));
    out[0] = v.x;
    out[1] = v.y;
    out[2] = v.z;
}
template <>
__device__ __forceinline__ void store_vec_nt<float, 3>(float *p, const float (&in)[3]) {
    f3v v;
    v.x = in[0];
    v.y = in[1];
    v.z = in[2];
    __builtin_nontemporal_store(v, reinterpret_cast<f3u *>(p));
}

template <bool NT, typename T, int N>
__device__ __forceinline__ void load_s(const T *p, T (&out)[N]) {
    if (NT) load_vec_nt<T, N>(p, out);
    else load_vec<T, N>(p, out);
}
template <bool NT, typename T, int N>
__device__ __forceinline__ void store_s(T *p, const T (&in)[N]) {
    if (NT) store_vec_nt<T, N>(p, in);
    else store_vec<T, N>(p, in);
}

#ifndef VNE_STREAM_NT
#define VNE_STREAM_NT 1
#endif
constexpr bool kNT = VNE_STREAM_NT != 0;

// entries of a CSR row whose gathers are issued together: 16 when a row's
// lane group is wide (16 or more lanes, so few rows share a wave and each
// needs more loads in flight), else 8 (measured); VNE_GATHER_U forces one
#ifndef VNE_GATHER_U
#define VNE_GATHER_U 0
#endif
template <int LPR>
constexpr int gather_batch() { return VNE_GATHER_U > 0 ? VNE_GATHER_U : (LPR >= 16 ? 16 : 8); }

// slots of a gather batch skipped together when no row of the wave needs
// them (0: the default of the step core)
#ifndef VNE_SLOT_RUN
#define VNE_SLOT_RUN 0
#endif

// basis steps of k_reconstruct in flight per thread (2 measured faster than 4:
// at 4 the register count halves the waves per SIMD)
#ifndef VNE_RECON_UJ
#define VNE_RECON_UJ 2
#endif
// rows per thread of k_reconstruct
#ifndef VNE_RECON_RPT
#define VNE_RECON_RPT 4
#endif

// minimum waves per SIMD requested for the step kernels (0: compiler's choice)
#ifndef VNE_STEP_WAVES
#define VNE_STEP_WAVES 0
#endif
#if VNE_STEP_WAVES > 0
#define VNE_STEP_OCCUPANCY __attribute__((amdgpu_waves_per_eu(VNE_STEP_WAVES)))
#else
#define VNE_STEP_OCCUPANCY
#endif

// Lazily normalised Lanczos vector: v_j = (P_j - alpha_{j-1} v_{j-1}) / beta_{j-1},
// evaluated identically wherever an entry of v_j is needed.
__device__ __forceinline__ float materialize(float p, float vp, float a, float inv) {
    return __fmul_rn(__fmaf_rn(-a, vp, p), inv);
}
__device__ __forceinline__ double materialize(double p, double vp, double a, double inv) {
    return __dmul_rn(__fma_rn(-a, vp, p), inv);
}

// Logical block index such that each XCD (blocks are dealt round-robin to
// the 8 XCDs) receives one contiguous range of logical blocks.
__device__ __forceinline__ int xcd_remap(int p, int total) {
    constexpr int kXcd = 8;
    const int q = total / kXcd, r = total % kXcd;
    const int x = p % kXcd, i = p / kXcd;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// SplitMix64 output function (Steele, Lea, Flood 2014).
__device__ __forceinline__ uint64_t splitmix64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Rademacher entry for (row key, hash column): sign of the top bit of
// mix(seed + (key * 2^32 + col + 1) * 0x9E3779B97F4A7C15).
__device__ __forceinline__ double rademacher(uint64_t seed, int64_t key, int64_t col) {
    const uint64_t ctr = ((uint64_t)key << 32) + (uint64_t)col + 1ull;
    const uint64_t h = splitmix64_mix(seed + ctr * 0x9E3779B97F4A7C15ull);
    return (h >> 63) ? -1.0 : 1.0;
}

__device__ __forceinline__ double f_entropy(double x) { return x > 0.0 ? -x * log(x) : 0.0; }

// fixed-order tree sum over the 256 threads of a block (result in thread 0)
__device__ __forceinline__ double block_sum_256(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// Lanczos step: u = A v_j on the CSR (gathering m-vectors), recurrence
// w = u - beta_{j-1} v_{j-1}, and the FP64 partial sums v.w, w.w, v.v per
// column; v_j is materialised on the fly from (P_j, v_{j-1}) and written.
// A lane group of LPR lanes owns one row (or row segment) and MT = CPL * LPR
// columns of the tile; each lane holds CPL consecutive columns.
// ---------------------------------------------------------------------------

// TWO = false (lazy schedule): v_j is never stored before the SpMM; every
// entry of it, at a neighbour or at the row itself, is evaluated from P_j and
// v_{j-1}, and the step also writes v_j.  TWO = true (two-pass schedule): a
// streaming pass has already written v_j (k_normalize), and the SpMM gathers
// v_j alone.  Both evaluate every entry of v_j with the same expression, so
// the two schedules give bitwise identical results.
template <typename T, int CPL, int LPR, bool FIRST, bool TWO>
struct StepCore {
    static constexpr int MT = CPL * LPR;
    const StepArgs &a;
    int c0;
    int64_t ld;
    const T *P_in, *V_prev, *V_cur, *val;
    T *V_out, *P_out;
    T al[CPL], inv[CPL];
    double coup[CPL];

    double scale;

    __device__ __forceinline__ StepCore(const StepArgs &args, int tile, int gl, int g) : a(args) {
        c0 = tile * MT + gl * CPL;
        ld = a.m_pad;
        scale = a.graph_scale ? a.graph_scale[g] : a.scale;
        const int64_t s0 = (int64_t)g * a.m_pad + c0;   // per-column state of this graph
        P_in = static_cast<const T *>(a.P_in);
        V_prev = static_cast<const T *>(a.V_prev);
        V_cur = static_cast<const T *>(a.V_cur);
        V_out = static_cast<T *>(a.V_out);
        P_out = static_cast<T *>(a.P_out);
        val = static_cast<const T *>(a.val);
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            al[k] = (T)a.st_alpha[s0 + k];
            inv[k] = (T)a.st_inv[s0 + k];
            coup[k] = a.st_coup[s0 + k];
        }
    }

    static constexpr int U = gather_batch<LPR>();

    // Column indices and weights of a batch of UB entries [p, p + UB) of a
    // row, held spread over the lane group: lane gl keeps entries
    // p + gl + r LPR (r < R).  One coalesced load per array and round r
    // replaces UB same-address loads per lane: the step kernels are bound by
    // the vector-memory pipeline (address and data paths), in which every
    // load instruction costs its 64 lanes whatever their addresses.  Slots
    // past p1 hold the row itself with a zero weight.
    template <int UB>
    struct Idx {
        static constexpr int R = (UB + LPR - 1) / LPR;
        int j[R];
        T v[R];
    };

    template <int UB>
    __device__ __forceinline__ void batch_fetch(int row, int p, int p1, Idx<UB> &x) const {
        const int gl = (int)(threadIdx.x & 63) % LPR;
#pragma unroll
        for (int r = 0; r < Idx<UB>::R; ++r) {
            const int s = gl + r * LPR, e = p + s;
            const bool ok = s < UB && e < p1;
            x.j[r] = ok ? a.col[e] : row;
            x.v[r] = ok ? val[e] : (T)0;
        }
    }

    // the value of slot u for every lane of the group: from lane u % LPR of
    // the group, round u / LPR (a wave-wide group reads it as a scalar)
    template <typename V>
    static __device__ __forceinline__ V from_lane(V x, int src) {
        if constexpr (sizeof(V) == 8) {
            const int64_t b = __builtin_bit_cast(int64_t, x);
            const int lo = from_lane<int>((int)(b & 0xffffffff), src), hi = from_lane<int>((int)(b >> 32), src);
            return __builtin_bit_cast(V, (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
        } else {
            const int b = __builtin_bit_cast(int, x);
            int r;
            if constexpr (LPR == 1) return x;       // the lane is the group
            if constexpr (LPR == 64) r = __builtin_amdgcn_readlane(b, src);
            else r = __builtin_amdgcn_ds_bpermute(4 * (((int)(threadIdx.x & 63) & ~(LPR - 1)) + src), b);
            return __builtin_bit_cast(V, r);
        }
    }

    template <int UB>
    __device__ __forceinline__ void batch_spread(const Idx<UB> &x, int (&jj)[UB], T (&vv)[UB]) const {
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            jj[u] = from_lane<int>(x.j[u / LPR], u % LPR);
            vv[u] = from_lane<T>(x.v[u / LPR], u % LPR);
        }
    }

    // Slots of a batch in runs of kSlotRun: a run that no lane group of the
    // wave needs (every row of the wave has fewer entries left) is neither
    // loaded nor added (a wave-uniform branch; its slots would have added
    // val 0 times the row's own entry, exactly nothing).
    static constexpr int kSlotRun = VNE_SLOT_RUN > 0 ? VNE_SLOT_RUN : (U >= 16 ? 8 : U);

    // the gathered entries of v_j (lazy: P_j and v_{j-1}) of a batch whose
    // first cnt slots are entries of the row
    template <int UB>
    __device__ __forceinline__ void batch_load(const int (&jj)[UB], int cnt, T (&pv)[UB][CPL],
                                               T (&qv)[UB][CPL]) const {
#pragma unroll
        for (int c = 0; c < UB; c += kSlotRun) {
            if (c == 0 || __any(cnt > c)) {
#pragma unroll
                for (int u = c; u < c + kSlotRun && u < UB; ++u) {
                    if (TWO) {
                        load_vec<T, CPL>(V_cur + (int64_t)jj[u] * ld + c0, pv[u]);
                    } else {
                        load_vec<T, CPL>(P_in + (int64_t)jj[u] * ld + c0, pv[u]);
                        if (!FIRST) load_vec<T, CPL>(V_prev + (int64_t)jj[u] * ld + c0, qv[u]);
                    }
                }
            }
        }
    }

    template <int UB>
    __device__ __forceinline__ void batch_acc(const T (&vv)[UB], int cnt, const T (&pv)[UB][CPL],
                                              const T (&qv)[UB][CPL], double (&acc)[CPL]) const {
#pragma unroll
        for (int c = 0; c < UB; c += kSlotRun) {
            if (c == 0 || __any(cnt > c)) {
#pragma unroll
                for (int u = c; u < c + kSlotRun && u < UB; ++u) {
#pragma unroll
                    for (int k = 0; k < CPL; ++k) {
                        const T v = TWO ? pv[u][k] : materialize(pv[u][k], FIRST ? (T)0 : qv[u][k], al[k], inv[k]);
                        acc[k] = fma((double)vv[u], (double)v, acc[k]);
                    }
                }
            }
        }
    }

    // acc += sum over entries p in [p0, p1) of val[p] * v_j[col[p], cols],
    // in batches of UB entries whose loads are all in flight together
    template <int UB = U>
    __device__ __forceinline__ void gather_from(int row, int p0, int p1, double (&acc)[CPL]) const {
        for (int p = p0; p < p1; p += UB) {
            Idx<UB> x;
            int jj[UB];
            T vv[UB], pv[UB][CPL], qv[UB][CPL];
            const int cnt = min(UB, p1 - p);
            batch_fetch<UB>(row, p, p1, x);
            batch_spread<UB>(x, jj, vv);
            batch_load<UB>(jj, cnt, pv, qv);
            batch_acc<UB>(vv, cnt, pv, qv, acc);
        }
    }

    // the row's own entries: pv = P_j (lazy) or v_j (two-pass), qv = v_{j-1}
    __device__ __forceinline__ void load_self(int row, T (&pv)[CPL], T (&qv)[CPL]) const {
        load_vec<T, CPL>((TWO ? V_cur : P_in) + (int64_t)row * ld + c0, pv);
        if (!FIRST) load_s<kNT && TWO, T, CPL>(V_prev + (int64_t)row * ld + c0, qv);
        else
#pragma unroll
            for (int k = 0; k < CPL; ++k) qv[k] = (T)0;
    }

    // w = scale*acc - beta_{j-1} v_{j-1}; store P_{j+1} (and v_j, lazy); the
    // row's contributions to v.w, w.w, v.v
    __device__ __forceinline__ void finish(int row, const T (&pv)[CPL], const T (&qv)[CPL],
                                           const double (&acc)[CPL], double (&dvw)[CPL],
                                           double (&dww)[CPL], double (&dvv)[CPL]) const {
        T v[CPL], wr[CPL];
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            v[k] = TWO ? pv[k] : materialize(pv[k], qv[k], al[k], inv[k]);
            const double w = fma(-coup[k], (double)qv[k], scale * acc[k]);
            wr[k] = (T)w;
            const double vd = (double)v[k], wd = (double)wr[k];
            dvw[k] = vd * wd;
            dww[k] = wd * wd;
            dvv[k] = vd * vd;
        }
        store_s<kNT, T, CPL>(P_out + (int64_t)row * ld + c0, wr);
        if (!TWO) store_s<kNT, T, CPL>(V_out + (int64_t)row * ld + c0, v);
    }
};

// Two-pass schedule, first pass: v_j = (P_j - alpha_{j-1} v_{j-1}) / beta_{j-1}
// for every entry, streaming, CPL consecutive columns per thread.
template <typename T, int CPL, bool FIRST>
__global__ void __launch_bounds__(256) k_normalize(StepArgs a) {
    const T *P = static_cast<const T *>(a.P_in);
    const T *Vp = static_cast<const T *>(a.V_prev);
    T *Vo = static_cast<T *>(a.V_out);
    const int width = a.col_count > 0 ? a.col_count : a.m_pad;
    const int64_t groups = (int64_t)a.n * (width / CPL);
    const int cg = width / CPL;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < groups; t += (int64_t)gridDim.x * 256) {
        const int64_t i = t / cg;
        const int c0 = a.col_base + (int)(t % cg) * CPL;
        const int64_t s0 = (a.row_graph ? (int64_t)a.row_graph[i] * a.m_pad : 0) + c0;
        if (a.col_stop) {
            bool done = true;
#pragma unroll
            for (int k = 0; k < CPL; ++k) done = done && a.col_stop[s0 + k] > 0;
            if (done) continue;
        }
        T pv[CPL], qv[CPL], v[CPL];
        load_s<kNT, T, CPL>(P + i * a.m_pad + c0, pv);
        if (!FIRST) load_s<kNT, T, CPL>(Vp + i * a.m_pad + c0, qv);
#pragma unroll
        for (int k = 0; k < CPL; ++k)
            v[k] = materialize(pv[k], FIRST ? (T)0 : qv[k], (T)a.st_alpha[s0 + k], (T)a.st_inv[s0 + k]);
        store_vec<T, CPL>(Vo + i * a.m_pad + c0, v);
    }
}

// Whether any column of tiles tile0 .. tile0 + ntile - 1 (mt columns each)
// still runs: not stopped by its a-posteriori rule and not frozen.  The same
// answer for every thread of the block (a barrier inside).
__device__ __forceinline__ bool tile_live(const StepArgs &a, int tile0, int ntile, int mt) {
    bool live = false;
    for (int t = threadIdx.x; t < ntile * mt; t += blockDim.x) {
        const int c = tile0 * mt + t;
        live = live || (c < a.m_pad && a.col_stop[c] == 0 && a.st_inv[c] != 0.0);
    }
    return __syncthreads_or(live) != 0;
}

// One work block b of the schedule, column tiles tile0 .. tile0 + JT - 1:
// its segments, then its rows, and the block's partial sums (red: shared
// scratch of the block, 3 rows per tile).  Each tile has NG lane groups that
// take the block's items round robin, whatever JT is, so a tile's arithmetic
// (and its order) is the same in a JT-tile block of JT * kStepThreads
// threads as alone.  With JT > 1 the lane groups of the JT tiles of one item
// sit side by side in a wave: their gathers of one neighbour row are one
// contiguous run of JT * MT columns (narrow tiles fill whole cache lines).
template <typename T, int CPL, int LPR, bool FIRST, bool TWO, int JT = 1>
__device__ __forceinline__ void step_block(const StepArgs &a, int b, int tile0,
                                           double (*red)[(kStepThreads / 64) * (64 / LPR) * CPL * LPR]) {
    static_assert(JT == 1 || LPR * JT <= 64, "the tiles of an item share a wave");
    using Core = StepCore<T, CPL, LPR, FIRST, TWO>;
    constexpr int MT = Core::MT;
    constexpr int GPW = 64 / LPR;                    // lane groups per wave
    constexpr int NG = (kStepThreads / 64) * GPW;    // lane groups per block and tile
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int sub = lane / LPR;
    const int gl = lane % LPR;
    const int jt = JT == 1 ? 0 : sub % JT;
    const int gid = wave * (GPW / JT) + sub / JT;
    const int g = a.block_graph ? a.block_graph[b] : 0;
    const Core core(a, tile0 + jt, gl, g);

    // the lane group's running sums of v.w, w.w, v.v live in its own slots
    // of red (fixed order within the group)
    double *my0 = &red[3 * jt + 0][gid * MT + gl * CPL];
    double *my1 = &red[3 * jt + 1][gid * MT + gl * CPL];
    double *my2 = &red[3 * jt + 2][gid * MT + gl * CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) my0[k] = my1[k] = my2[k] = 0.0;

    // the block's items: its segments, then its rows.  Software pipeline
    // over the items of a lane group: while the gathers of item t are in
    // flight, the first column/weight batch of item t + NG and the location
    // (row_ptr or segment record) of item t + 2 NG are loaded.
    const int4 rg = a.block_ranges[b];
    const int n_sb = rg.y - rg.x;
    const int total = n_sb + (rg.w - rg.z);
    constexpr int U = Core::U;
    struct Item {
        int row, p0, p1, it;
        bool seg;
    };
    auto locate = [&](int t) {
        Item x{0, 0, 0, 0, false};
        if (t < total) {
            x.seg = t < n_sb;
            if (x.seg) {
                x.it = rg.x + t;
                const SegItem sg = a.segs[x.it];
                x.row = sg.row;
                x.p0 = sg.p0;
                x.p1 = sg.p1;
            } else {
                x.row = rg.z + (t - n_sb);
                x.p0 = a.row_ptr[x.row];
                x.p1 = a.row_ptr[x.row + 1];
            }
        }
        return x;
    };
    // a long row is done by its segments: no entries here, no result
    auto settle = [&](Item &x, bool &skip, int t) {
        skip = t >= total || (!x.seg && x.p1 - x.p0 > a.seg_len);
        if (skip) x.p1 = x.p0;
        if (LPR == 64) {
            x.row = __builtin_amdgcn_readfirstlane(x.row);
            x.p0 = __builtin_amdgcn_readfirstlane(x.p0);
            x.p1 = __builtin_amdgcn_readfirstlane(x.p1);
        }
    };
    Item cur = locate(gid);
    bool cur_skip;
    settle(cur, cur_skip, gid);
    typename Core::template Idx<U> ix;
    core.template batch_fetch<U>(cur.row, cur.p0, cur.p1, ix);
    Item nxt = locate(gid + NG);
    for (int t = gid; t < total; t += NG) {
        int jj[U];
        T vv[U], pv[U][CPL], qv[U][CPL];
        const int cnt = min(U, cur.p1 - cur.p0);
        core.template batch_spread<U>(ix, jj, vv);
        core.template batch_load<U>(jj, cnt, pv, qv);
        T sp[CPL], sq[CPL];
        if (!cur.seg) core.load_self(cur.row, sp, sq);
        bool nxt_skip;
        settle(nxt, nxt_skip, t + NG);
        core.template batch_fetch<U>(nxt.row, nxt.p0, nxt.p1, ix);
        const Item nn = locate(t + 2 * NG);
        double acc[CPL];
#pragma unroll
        for (int k = 0; k < CPL; ++k) acc[k] = 0.0;
        core.template batch_acc<U>(vv, cnt, pv, qv, acc);
        if (cur.p1 - cur.p0 > U) core.template gather_from<(U > 1 ? U / 2 : 1)>(cur.row, cur.p0 + U, cur.p1, acc);
        if (!cur_skip) {
            if (!cur.seg) {
                double dvw[CPL], dww[CPL], dvv[CPL];
                core.finish(cur.row, sp, sq, acc, dvw, dww, dvv);
#pragma unroll
                for (int k = 0; k < CPL; ++k) {
                    my0[k] += dvw[k];
                    my1[k] += dww[k];
                    my2[k] += dvv[k];
                }
            } else {
                // segment of a long row: its partial product is finished by
                // k_long_rows after this kernel (the kernel boundary orders it)
                double *dst = a.seg_acc + (int64_t)cur.it * core.ld + core.c0;
#pragma unroll
                for (int k = 0; k < CPL; ++k) dst[k] = acc[k];
            }
        }
        cur = nxt;
        cur_skip = nxt_skip;
        nxt = nn;
    }

    // block reduction over the lane groups that share columns (fixed order)
    __syncthreads();
    // partials layout [n_blocks][3][m_pad]: the finalize reads whole rows
    double *out = a.partials + (int64_t)b * 3 * a.m_pad + tile0 * MT;
    for (int t = threadIdx.x; t < JT * 3 * MT; t += JT * kStepThreads) {
        const int row = t / MT, cc = t % MT;         // row = 3 * tile + sum index
        const int tj = row / 3, sidx = row % 3;
        double sum = 0.0;
#pragma unroll 4
        for (int g = 0; g < NG; ++g) sum += red[row][g * MT + cc];
        out[(int64_t)tj * MT + (int64_t)sidx * a.m_pad + cc] = sum;
    }
}

template <typename T, int CPL, int LPR, bool FIRST, bool TWO>
__global__ void __launch_bounds__(kStepThreads) VNE_STEP_OCCUPANCY k_lanczos_step(StepArgs a) {
    constexpr int NG = (kStepThreads / 64) * (64 / LPR);
    __shared__ double red[3][NG * CPL * LPR];
    // column tiles are dispatched one after the other (tile-major grid), so
    // the gathered block of one tile stays resident in the last-level cache;
    // within a tile each XCD takes one contiguous range of row blocks
    // (n_blocks is a multiple of 8)
    const int tile = a.tile_base + (int)blockIdx.y;
    if (a.col_stop && !tile_live(a, tile, 1, CPL * LPR)) return;
    step_block<T, CPL, LPR, FIRST, TWO>(a, xcd_remap(blockIdx.x, a.n_blocks), tile, red);
}

// Several independent problems ("slots") in one launch: entry e = {slot,
// work block, column tile} of map runs block e.y, tile e.z of slot e.x, whose
// matrix, vectors and state args[e.x] describes.  Two-pass schedule; the
// first step of a slot runs as a later step whose v_{j-1} is zero and whose
// alpha_{j-1}, beta_{j-1} are zero, which gives the same values.
// A slot whose stopping rule was met at an earlier step: the quadrature
// takes that step's coefficients, so later steps are skipped (the host learns
// of the stop a few ticks after the device).  The record is written by a
// kernel of an earlier tick, so every kernel of a tick sees the same value.
__device__ __forceinline__ bool slot_stopped(const int2 *state, int32_t uid, int32_t count) {
    if (!state) return false;
    for (int i = 0; i < count; ++i) {
        const int2 st = state[i];
        if (st.x != uid + i || st.y <= 0) return false;
    }
    return true;
}

template <typename T, int CPL, int LPR>
__global__ void __launch_bounds__(kStepThreads) VNE_STEP_OCCUPANCY k_lanczos_step_slots(const StepArgs *args, const int4 *map,
                                                                     int32_t n_entries) {
    constexpr int NG = (kStepThreads / 64) * (64 / LPR);
    __shared__ double red[3][NG * CPL * LPR];
    const int4 e = map[xcd_remap(blockIdx.x, n_entries)];
    const StepArgs a = args[e.x];
    if (slot_stopped(a.stop_state, a.stop_uid, a.stop_count)) return;
    step_block<T, CPL, LPR, false, true>(a, e.y, e.z, red);
}

// JT column tiles of one slot per block (JT * kStepThreads threads): entry
// {slot, work block, first tile}.  For group slots of narrow tiles, whose
// single-tile blocks would each gather a part of every cache line they
// fetch; each tile keeps the arithmetic and order it has alone.
template <typename T, int CPL, int LPR, int JT>
__global__ void __launch_bounds__(JT * kStepThreads) k_lanczos_step_groups(const StepArgs *args, const int4 *map,
                                                                            int32_t n_entries) {
    constexpr int NG = (kStepThreads / 64) * (64 / LPR);
    __shared__ double red[JT * 3][NG * CPL * LPR];
    const int4 e = map[xcd_remap(blockIdx.x, n_entries)];
    const StepArgs a = args[e.x];
    if (slot_stopped(a.stop_state, a.stop_uid, a.stop_count)) return;
    step_block<T, CPL, LPR, false, true, JT>(a, e.y, e.z, red);
}

// Normalize pass of the slots: entry {slot, work block, tile} writes v_j on
// the block's row range, tile columns.
template <typename T, int CPL, int LPR>
__global__ void __launch_bounds__(256) k_normalize_slots(const StepArgs *args, const int4 *map, int32_t n_entries) {
    constexpr int MT = CPL * LPR;
    constexpr int RP = 256 / LPR;                    // rows per pass
    const int4 e = map[xcd_remap(blockIdx.x, n_entries)];
    const StepArgs a = args[e.x];
    if (slot_stopped(a.stop_state, a.stop_uid, a.stop_count)) return;
    const int4 rg = a.block_ranges[e.y];
    const int c0 = e.z * MT + (int)(threadIdx.x % LPR) * CPL;
    const T *P = static_cast<const T *>(a.P_in);
    const T *Vp = static_cast<const T *>(a.V_prev);
    T *Vo = static_cast<T *>(a.V_out);
    T al[CPL], inv[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        al[k] = (T)a.st_alpha[c0 + k];
        inv[k] = (T)a.st_inv[c0 + k];
    }
    for (int64_t i = rg.z + (int)(threadIdx.x / LPR); i < rg.w; i += RP) {
        T pv[CPL], qv[CPL], v[CPL];
        load_s<kNT, T, CPL>(P + i * a.m_pad + c0, pv);
        load_s<kNT, T, CPL>(Vp + i * a.m_pad + c0, qv);
#pragma unroll
        for (int k = 0; k < CPL; ++k) v[k] = materialize(pv[k], qv[k], al[k], inv[k]);
        store_vec<T, CPL>(Vo + i * a.m_pad + c0, v);
    }
}

// Long rows: add the segment partial products in segment order and finish
// the row; its dot-product contributions go to a slot of its own.
template <typename T, int CPL, int LPR, bool FIRST, bool TWO>
__device__ __forceinline__ void long_rows_group(const StepArgs &a, int group, int tile) {
    using Core = StepCore<T, CPL, LPR, FIRST, TWO>;
    constexpr int GPW = 64 / LPR;
    constexpr int NG = 4 * GPW;
    const int lane = threadIdx.x & 63;
    const int grp = lane / LPR;
    const int gl = lane % LPR;
    const int L = group * NG + (threadIdx.x >> 6) * GPW + grp;
    if (L >= a.n_long) return;
    const Core core(a, tile, gl, a.long_graph ? a.long_graph[L] : 0);
    const int first = a.long_first[L], nseg = a.long_nseg[L];
    const int row = a.segs[first].row;
    double tot[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) tot[k] = 0.0;
    constexpr int UQ = 8;
    int q = 0;
    for (; q + UQ <= nseg; q += UQ) {
        double buf[UQ][CPL];
#pragma unroll
        for (int u = 0; u < UQ; ++u) {
            const double *src = a.seg_acc + (int64_t)(first + q + u) * core.ld + core.c0;
#pragma unroll
            for (int k = 0; k < CPL; ++k) buf[u][k] = src[k];
        }
#pragma unroll
        for (int u = 0; u < UQ; ++u)
#pragma unroll
            for (int k = 0; k < CPL; ++k) tot[k] += buf[u][k];
    }
    for (; q < nseg; ++q) {
        const double *src = a.seg_acc + (int64_t)(first + q) * core.ld + core.c0;
#pragma unroll
        for (int k = 0; k < CPL; ++k) tot[k] += src[k];
    }
    T pv[CPL], qv[CPL];
    core.load_self(row, pv, qv);
    double dvw[CPL], dww[CPL], dvv[CPL];
    core.finish(row, pv, qv, tot, dvw, dww, dvv);
    double *lp = a.long_part + (int64_t)L * 3 * core.ld + core.c0;
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        lp[k] = dvw[k];
        lp[core.ld + k] = dww[k];
        lp[2 * core.ld + k] = dvv[k];
    }
}

template <typename T, int CPL, int LPR, bool FIRST, bool TWO>
__global__ void __launch_bounds__(256) k_long_rows(StepArgs a) {
    const int tile = a.tile_base + (int)blockIdx.y;
    if (a.col_stop && !tile_live(a, tile, 1, CPL * LPR)) return;
    long_rows_group<T, CPL, LPR, FIRST, TWO>(a, blockIdx.x, tile);
}

// entry {slot, group of long rows, tile}
template <typename T, int CPL, int LPR>
__global__ void __launch_bounds__(256) k_long_rows_slots(const StepArgs *args, const int4 *map) {
    const int4 e = map[blockIdx.x];
    const StepArgs a = args[e.x];
    if (slot_stopped(a.stop_state, a.stop_uid, a.stop_count)) return;
    long_rows_group<T, CPL, LPR, false, true>(a, e.y, e.z);
}

int choose_tile(int m, bool fp64, int requested, bool three) {
    // FP32 widths 3 * 2^j (12 .. 192) as one tile of three columns per lane,
    // without padding to the next power of two
    if (three && !fp64 && requested <= 0 && m % 3 == 0) {
        const int q = m / 3;
        if (q >= 4 && q <= 64 && (q & (q - 1)) == 0) return m;
    }
    // column tile = CPL * LPR; by default at most 128 FP32 (64 FP64) columns,
    // the widest tile whose gathered block stays cache friendly on large graphs;
    // a requested tile may also be one of the narrow ones (one or two lanes
    // per row)
    const int cpl = fp64 ? 2 : 4;
    const int maxt = cpl * 64, mint = requested > 0 ? cpl : cpl * 4;
    const int cap = requested > 0 ? maxt : (fp64 ? 64 : 128);
    const int want = requested > 0 ? requested : m;
    int t = mint;
    while (t < want && t < cap) t *= 2;
    return t;
}

int pad_columns(int m, int mt) { return ((m + mt - 1) / mt) * mt; }

int choose_plan_tile(int m, bool fp64, int64_t n, int64_t nnz) {
    // Bytes of one step by a simple model: six streams of the padded block,
    // and per column tile the CSR (8 B per entry) and one gather per entry
    // of at least a 128-byte line.  The cheapest tile wins (ties: the wider).
    // The narrow tiles (one or two lanes per row: 4 and 8 FP32 columns, 2 and
    // 4 FP64) win only for blocks of a few columns, where padding to the
    // next wide tile would multiply the streams.
    const int es = fp64 ? 8 : 4, cpl = fp64 ? 2 : 4;
    std::vector<int> cands;
    for (int t = cpl; t <= (fp64 ? 64 : 128); t *= 2) cands.push_back(t);
    if (!fp64) {
        for (int t = 12; t <= 96; t *= 2) cands.push_back(t);
        if (m == 192) cands.push_back(192);
    }
    int best = 0;
    double best_cost = 0.0;
    for (int t : cands) {
        const int mp = pad_columns(m, t), tiles = mp / t;
        const double cost = 6.0 * (double)n * mp * es + (double)tiles * (double)nnz * (8.0 + std::max(t * es, 128));
        if (best == 0 || cost < best_cost || (cost == best_cost && t > best)) {
            best = t;
            best_cost = cost;
        }
    }
    return best;
}

template <typename T, int CPL, int LPR, bool FIRST, bool TWO>
static void launch_step_k(const StepArgs &a, hipStream_t s) {
    if (TWO) {
        const int64_t groups = (int64_t)a.n * ((a.col_count > 0 ? a.col_count : a.m_pad) / CPL);
        const unsigned nb = (unsigned)std::min<int64_t>((groups + 255) / 256, 8192);
        hipLaunchKernelGGL((k_normalize<T, CPL, FIRST>), dim3(nb), dim3(256), 0, s, a);
    }
    dim3 grid(a.n_blocks, a.n_tiles);
    hipLaunchKernelGGL((k_lanczos_step<T, CPL, LPR, FIRST, TWO>), grid, dim3(kStepThreads), 0, s, a);
    if (a.n_long > 0) {
        constexpr int NG = 4 * (64 / LPR);
        dim3 lg((a.n_long + NG - 1) / NG, a.n_tiles);
        hipLaunchKernelGGL((k_long_rows<T, CPL, LPR, FIRST, TWO>), lg, dim3(256), 0, s, a);
    }
}

template <typename T, int CPL, int LPR>
static hipError_t launch_step_t(const StepArgs &a, bool first, hipStream_t s) {
    if (a.two_pass) {
        if (first) launch_step_k<T, CPL, LPR, true, true>(a, s);
        else launch_step_k<T, CPL, LPR, false, true>(a, s);
    } else {
        if (first) launch_step_k<T, CPL, LPR, true, false>(a, s);
        else launch_step_k<T, CPL, LPR, false, false>(a, s);
    }
    return hipGetLastError();
}

template <typename T, int CPL, int LPR>
static hipError_t launch_slots_t(const StepArgs *args, const int4 *step_map, int32_t n_step,
                                 const int4 *long_map, int32_t n_long, hipStream_t s) {
    if (n_step > 0) {
        hipLaunchKernelGGL((k_normalize_slots<T, CPL, LPR>), dim3(n_step), dim3(256), 0, s, args, step_map, n_step);
        hipLaunchKernelGGL((k_lanczos_step_slots<T, CPL, LPR>), dim3(n_step), dim3(kStepThreads), 0, s, args,
                           step_map, n_step);
    }
    if (n_long > 0) hipLaunchKernelGGL((k_long_rows_slots<T, CPL, LPR>), dim3(n_long), dim3(256), 0, s, args, long_map);
    return hipGetLastError();
}

int long_rows_per_group(int mt, bool fp64) { return 4 * (64 / (mt / (fp64 ? 2 : 4))); }

hipError_t launch_step_slots(const StepArgs *args, const int4 *step_map, int32_t n_step, const int4 *long_map,
                             int32_t n_long, int32_t mt, bool fp64, hipStream_t s) {
    if (!fp64) {
        switch (mt) {
            case 16: return launch_slots_t<float, 4, 4>(args, step_map, n_step, long_map, n_long, s);
            case 32: return launch_slots_t<float, 4, 8>(args, step_map, n_step, long_map, n_long, s);
            case 64: return launch_slots_t<float, 4, 16>(args, step_map, n_step, long_map, n_long, s);
            case 128: return launch_slots_t<float, 4, 32>(args, step_map, n_step, long_map, n_long, s);
            case 256: return launch_slots_t<float, 4, 64>(args, step_map, n_step, long_map, n_long, s);
        }
    } else {
        switch (mt) {
            case 8: return launch_slots_t<double, 2, 4>(args, step_map, n_step, long_map, n_long, s);
            case 16: return launch_slots_t<double, 2, 8>(args, step_map, n_step, long_map, n_long, s);
            case 32: return launch_slots_t<double, 2, 16>(args, step_map, n_step, long_map, n_long, s);
            case 64: return launch_slots_t<double, 2, 32>(args, step_map, n_step, long_map, n_long, s);
            case 128: return launch_slots_t<double, 2, 64>(args, step_map, n_step, long_map, n_long, s);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_step_groups(const StepArgs *args, const int4 *group_map, int32_t n_group, const int4 *long_map,
                              int32_t n_long, int32_t members, hipStream_t s) {
    if (members != 2 && members != 4) return hipErrorInvalidValue;
    if (n_group > 0) {
        // the normalize pass is elementwise: the members' tiles as one tile
        // of 16 * members columns
        if (members == 2) {
            hipLaunchKernelGGL((k_normalize_slots<float, 4, 8>), dim3(n_group), dim3(256), 0, s, args, group_map,
                               n_group);
            hipLaunchKernelGGL((k_lanczos_step_groups<float, 4, 4, 2>), dim3(n_group), dim3(2 * kStepThreads), 0, s,
                               args, group_map, n_group);
        } else {
            hipLaunchKernelGGL((k_normalize_slots<float, 4, 16>), dim3(n_group), dim3(256), 0, s, args, group_map,
                               n_group);
            hipLaunchKernelGGL((k_lanczos_step_groups<float, 4, 4, 4>), dim3(n_group), dim3(4 * kStepThreads), 0, s,
                               args, group_map, n_group);
        }
    }
    if (n_long > 0) hipLaunchKernelGGL((k_long_rows_slots<float, 4, 4>), dim3(n_long), dim3(256), 0, s, args, long_map);
    return hipGetLastError();
}

hipError_t launch_step(const StepArgs &a, bool fp64, bool first, hipStream_t s) {
    if (!fp64) {
        switch (a.mt) {
            case 4: return launch_step_t<float, 4, 1>(a, first, s);
            case 8: return launch_step_t<float, 4, 2>(a, first, s);
            case 16: return launch_step_t<float, 4, 4>(a, first, s);
            case 32: return launch_step_t<float, 4, 8>(a, first, s);
            case 64: return launch_step_t<float, 4, 16>(a, first, s);
            case 128: return launch_step_t<float, 4, 32>(a, first, s);
            case 256: return launch_step_t<float, 4, 64>(a, first, s);
            case 12: return launch_step_t<float, 3, 4>(a, first, s);
            case 24: return launch_step_t<float, 3, 8>(a, first, s);
            case 48: return launch_step_t<float, 3, 16>(a, first, s);
            case 96: return launch_step_t<float, 3, 32>(a, first, s);
            case 192: return launch_step_t<float, 3, 64>(a, first, s);
        }
    } else {
        switch (a.mt) {
            case 2: return launch_step_t<double, 2, 1>(a, first, s);
            case 4: return launch_step_t<double, 2, 2>(a, first, s);
            case 8: return launch_step_t<double, 2, 4>(a, first, s);
            case 16: return launch_step_t<double, 2, 8>(a, first, s);
            case 32: return launch_step_t<double, 2, 16>(a, first, s);
            case 64: return launch_step_t<double, 2, 32>(a, first, s);
            case 128: return launch_step_t<double, 2, 64>(a, first, s);
        }
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Finalize a step: fixed-order sum of the block and long-row partials, then
// alpha_j = (v.w)/(v.v), beta_j^2 = w.w - alpha_j (v.w) = ||w - alpha_j v||^2,
// breakdown test and the scalars of the next lazy normalisation.
// ---------------------------------------------------------------------------

// First level: block (x, r) adds, for 64 columns, the partial rows
// r, r + R, r + 2R, ... of the step blocks (then of the long rows) in fixed
// order; the result goes to level2[r][3][m_pad].
__global__ void __launch_bounds__(256) k_reduce_partials(FinalizeArgs a) {
    __shared__ double sh[3][4][64];
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int c = a.col_base + (int)blockIdx.x * 64 + lane;
    const int c_end = a.col_count > 0 ? a.col_base + a.col_count : a.m_pad;
    const int r = blockIdx.y, R = gridDim.y;
    double s3[3] = {0.0, 0.0, 0.0};
    if (c < c_end) {
        constexpr int UB = 4;
        const int stride = 4 * R;
        int bb = r + grp * R;
        for (; bb + stride * (UB - 1) < a.n_blocks; bb += stride * UB) {
            double buf[UB][3];
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                const double *p = a.partials + (int64_t)(bb + stride * u) * 3 * a.m_pad + c;
                buf[u][0] = p[0];
                buf[u][1] = p[a.m_pad];
                buf[u][2] = p[2 * a.m_pad];
            }
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                s3[0] += buf[u][0];
                s3[1] += buf[u][1];
                s3[2] += buf[u][2];
            }
        }
        for (; bb < a.n_blocks; bb += stride) {
            const double *p = a.partials + (int64_t)bb * 3 * a.m_pad + c;
            s3[0] += p[0];
            s3[1] += p[a.m_pad];
            s3[2] += p[2 * a.m_pad];
        }
        for (int L = r + grp * R; L < a.n_long; L += stride) {
            const double *p = a.long_part + (int64_t)L * 3 * a.m_pad + c;
            s3[0] += p[0];
            s3[1] += p[a.m_pad];
            s3[2] += p[2 * a.m_pad];
        }
    }
    sh[0][grp][lane] = s3[0];
    sh[1][grp][lane] = s3[1];
    sh[2][grp][lane] = s3[2];
    __syncthreads();
    if (grp != 0 || c >= c_end) return;
    double* out = a.level2 + (int64_t)r * 3 * a.m_pad + c;
#pragma unroll
    for (int q = 0; q < 3; ++q) out[(int64_t)q * a.m_pad] = sh[q][0][lane] + sh[q][1][lane] + sh[q][2][lane] + sh[q][3][lane];
}

// alpha_j = (v.w)/(v.v), beta_j^2 = w.w - alpha_j (v.w) = ||w - alpha_j v||^2,
// breakdown test and the scalars of the next normalisation, for the column
// c of graph g (state index gc = g * m_pad + c).  A graph with fewer steps
// than the launch keeps its last beta and stops.
__device__ __forceinline__ void update_coefficients(const FinalizeArgs &a, int g, int c, double svw, double sww,
                                                    double svv) {
    const int64_t gc = (int64_t)g * a.m_pad + c;
    if (a.col_stop && a.col_stop[gc] > 0) return;      // met its tolerance: done
    const int j = a.step - 1;
    const int kg = a.graph_k ? a.graph_k[g] : a.k;
    const int mg = a.graph_m ? a.graph_m[g] : a.m;
    const double inv_prev = a.st_inv[gc];
    if (inv_prev == 0.0 || c >= mg || a.step > kg) {   // frozen, empty, pad column or done
        a.alpha[gc * a.k + j] = 0.0;
        a.beta[gc * a.k + j] = 0.0;
        a.st_inv[gc] = 0.0;
        a.st_alpha[gc] = 0.0;
        a.st_coup[gc] = 0.0;
        return;
    }
    const double coup_prev = a.st_coup[gc];
    const double alpha = svw / svv;
    double b2 = sww - alpha * svw;
    b2 = b2 > 0.0 ? b2 : 0.0;
    const double beta = sqrt(b2);
    a.alpha[gc * a.k + j] = alpha;
    const bool finite = isfinite(alpha) && isfinite(beta);
    if (!finite) {
        // a group slot's column reports to its member's query
        int32_t *fl = a.flags;
        if (a.mem_cols > 0 && a.flags_mem[c / a.mem_cols]) fl = a.flags_mem[c / a.mem_cols];
        atomicOr(fl, 1);
    }
    if (!finite || beta <= a.tau * (fabs(alpha) + coup_prev)) {
        a.k_eff[gc] = a.step;
        a.beta[gc * a.k + j] = 0.0;
        a.st_inv[gc] = 0.0;
        a.st_alpha[gc] = 0.0;
        a.st_coup[gc] = 0.0;
    } else {
        a.beta[gc * a.k + j] = beta;
        const bool last = a.step == kg;
        a.st_alpha[gc] = last ? 0.0 : alpha;
        a.st_inv[gc] = last ? 0.0 : 1.0 / beta;
        a.st_coup[gc] = last ? 0.0 : beta;
    }
}

// Second level (one graph): sum the R first-level rows in order, update.
// With R = kLevel2 every row is loaded before the first add, so the loads
// overlap instead of forming a chain of dependent round trips; the sums keep
// the same order.
__global__ void __launch_bounds__(64) k_finalize(FinalizeArgs a) {
    const int c = a.col_base + (int)blockIdx.x * 64 + (int)threadIdx.x;
    if (c >= (a.col_count > 0 ? a.col_base + a.col_count : a.m_pad)) return;
    double svw = 0.0, sww = 0.0, svv = 0.0;
    if (a.n_level2 == kLevel2) {
        double v[kLevel2][3];
#pragma unroll
        for (int r = 0; r < kLevel2; ++r) {
            const double *p = a.level2 + (int64_t)r * 3 * a.m_pad + c;
            v[r][0] = p[0];
            v[r][1] = p[a.m_pad];
            v[r][2] = p[2 * a.m_pad];
        }
#pragma unroll
        for (int r = 0; r < kLevel2; ++r) {
            svw += v[r][0];
            sww += v[r][1];
            svv += v[r][2];
        }
    } else {
        for (int r = 0; r < a.n_level2; ++r) {
            const double *p = a.level2 + (int64_t)r * 3 * a.m_pad + c;
            svw += p[0];
            sww += p[a.m_pad];
            svv += p[2 * a.m_pad];
        }
    }
    update_coefficients(a, 0, c, svw, sww, svv);
}

// Several graphs: thread (g, c) adds graph g's block partials, then its long
// rows, in order, and updates.
__global__ void __launch_bounds__(256) k_finalize_graphs(FinalizeArgs a) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)a.n_graphs * a.m_pad) return;
    const int g = (int)(t / a.m_pad), c = (int)(t % a.m_pad);
    double svw = 0.0, sww = 0.0, svv = 0.0;
    // the graph's block partials, then its long-row partials, in order; in
    // batches of UB whose loads are all issued before the adds (same order)
    const int b0 = a.graph_block_begin[g], nb = a.graph_block_begin[g + 1] - b0;
    const int L0 = a.graph_long_begin[g], total = nb + (a.graph_long_begin[g + 1] - L0);
    auto src = [&](int i) -> const double * {
        return i < nb ? a.partials + (int64_t)(b0 + i) * 3 * a.m_pad + c
                      : a.long_part + (int64_t)(L0 + i - nb) * 3 * a.m_pad + c;
    };
    constexpr int UB = 8;
    int i = 0;
    for (; i + UB <= total; i += UB) {
        double v[UB][3];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const double *p = src(i + u);
            v[u][0] = p[0];
            v[u][1] = p[a.m_pad];
            v[u][2] = p[2 * a.m_pad];
        }
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            svw += v[u][0];
            sww += v[u][1];
            svv += v[u][2];
        }
    }
    for (; i < total; ++i) {
        const double *p = src(i);
        svw += p[0];
        sww += p[a.m_pad];
        svv += p[2 * a.m_pad];
    }
    update_coefficients(a, g, c, svw, sww, svv);
}

// Slots, first level: block (slot e.x, columns e.y * C .., part blockIdx.y)
// of 16 groups of C threads.  The slot's items (its work blocks, then its
// long rows) are cut into n_level2 * G contiguous ranges; group q of part r
// adds range r * G + q in order, and the block writes the G group sums, added
// in order, to level2[r][3][m_pad] of the slot.  The order depends only on
// the slot's own shape.
__global__ void __launch_bounds__(256) k_reduce_slots(const FinalizeArgs *fargs, const int2 *map) {
    constexpr int C = kFinalizeCols, G = 256 / C;
    __shared__ double sh[3][G][C];
    const int2 e = map[blockIdx.x];
    const FinalizeArgs a = fargs[e.x];
    if (slot_stopped(a.stop_state, a.stop_uid, a.stop_count)) return;
    const int r = blockIdx.y;
    const int cc = threadIdx.x % C, grp = threadIdx.x / C;
    const int c = e.y * C + cc;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (c < a.m_pad && r < a.n_level2) {
        const int total = a.n_blocks + a.n_long;
        const int ranges = a.n_level2 * G;
        const int per = (total + ranges - 1) / ranges;
        const int i0 = min(total, (r * G + grp) * per), i1 = min(total, i0 + per);
        const int b1 = min(i1, a.n_blocks);
        for (int i = i0; i < b1; ++i) {
            const double *p = a.partials + (int64_t)i * 3 * a.m_pad + c;
            s0 += p[0];
            s1 += p[a.m_pad];
            s2 += p[2 * a.m_pad];
        }
        for (int i = max(i0, a.n_blocks); i < i1; ++i) {
            const double *p = a.long_part + (int64_t)(i - a.n_blocks) * 3 * a.m_pad + c;
            s0 += p[0];
            s1 += p[a.m_pad];
            s2 += p[2 * a.m_pad];
        }
    }
    sh[0][grp][cc] = s0;
    sh[1][grp][cc] = s1;
    sh[2][grp][cc] = s2;
    __syncthreads();
    if (grp != 0 || c >= a.m_pad || r >= a.n_level2) return;
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    for (int q = 0; q < G; ++q) {
        t0 += sh[0][q][cc];
        t1 += sh[1][q][cc];
        t2 += sh[2][q][cc];
    }
    double *out = a.level2 + (int64_t)r * 3 * a.m_pad + c;
    out[0] = t0;
    out[a.m_pad] = t1;
    out[2 * a.m_pad] = t2;
}

// Slots, second level: thread (slot, column) adds the n_level2 rows in order
// and updates.
__global__ void __launch_bounds__(kFinalizeCols) k_finalize_slots(const FinalizeArgs *fargs, const int2 *map) {
    const int2 e = map[blockIdx.x];
    const FinalizeArgs a = fargs[e.x];
    if (slot_stopped(a.stop_state, a.stop_uid, a.stop_count)) return;
    const int c = e.y * kFinalizeCols + threadIdx.x;
    if (c >= a.m_pad) return;
    double svw = 0.0, sww = 0.0, svv = 0.0;
    if (a.n_level2 == kSlotLevel2) {
        double v[kSlotLevel2][3];
#pragma unroll
        for (int r = 0; r < kSlotLevel2; ++r) {
            const double *p = a.level2 + (int64_t)r * 3 * a.m_pad + c;
            v[r][0] = p[0];
            v[r][1] = p[a.m_pad];
            v[r][2] = p[2 * a.m_pad];
        }
#pragma unroll
        for (int r = 0; r < kSlotLevel2; ++r) {
            svw += v[r][0];
            sww += v[r][1];
            svv += v[r][2];
        }
    } else {
        for (int r = 0; r < a.n_level2; ++r) {
            const double *p = a.level2 + (int64_t)r * 3 * a.m_pad + c;
            svw += p[0];
            sww += p[a.m_pad];
            svv += p[2 * a.m_pad];
        }
    }
    update_coefficients(a, 0, c, svw, sww, svv);
}

hipError_t launch_finalize_slots(const FinalizeArgs *fargs, const int2 *map, int32_t n_entries, hipStream_t s) {
    if (n_entries > 0) {
        hipLaunchKernelGGL(k_reduce_slots, dim3(n_entries, kSlotLevel2), dim3(256), 0, s, fargs, map);
        hipLaunchKernelGGL(k_finalize_slots, dim3(n_entries), dim3(kFinalizeCols), 0, s, fargs, map);
    }
    return hipGetLastError();
}

hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t s) {
    if (a.segmented) {
        const int64_t t = (int64_t)a.n_graphs * a.m_pad;
        hipLaunchKernelGGL(k_finalize_graphs, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    const int width = a.col_count > 0 ? a.col_count : a.m_pad;
    hipLaunchKernelGGL(k_reduce_partials, dim3((width + 63) / 64, a.n_level2), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_finalize, dim3((width + 63) / 64), dim3(64), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Probe block.  Thread layout: columns of one tile fastest, 256 / mt rows per
// pass (integer division).  Pass 1 sums every column (for the centring of
// Remark 4.6), pass 2 writes P_1 = c (element type of the mode) and sums c^2
// of the stored values.
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ double probe_value(const ProbeArgs &a, int g, int64_t i, int c) {
    const int mg = a.graph_m ? a.graph_m[g] : a.m;
    if (c >= mg) return 0.0;
    if (a.gen == GEN_RADEMACHER)
        return rademacher(a.seeds ? a.seeds[g] : a.seed, a.keys[i], (int64_t)a.col_offset + c);
    if (a.gen == GEN_COLORING) return a.colors[i] == c ? 1.0 : 0.0;
    return (double)static_cast<const T *>(a.dense)[i * a.ld_dense + c];
}

// Block b owns rows [block_row_begin[b], block_row_begin[b+1]) of one graph.
// Pass 1 sums every column; pass 2 writes P_1 = b - mean (element type of the
// mode) and sums the squares of the stored values.
template <typename T, int PASS>
__global__ void __launch_bounds__(256) k_probe(ProbeArgs a) {
    __shared__ double sh[256];
    const int rows_per = 256 / a.mt;
    const int cc = threadIdx.x % a.mt, rr = threadIdx.x / a.mt;
    // a tile width that does not divide 256 leaves the last threads idle
    const bool active = rr < rows_per;
    const int b = blockIdx.x;
    const int g = a.block_graph ? a.block_graph[b] : 0;
    const int64_t r0 = a.block_row_begin[b], r1 = a.block_row_begin[b + 1];
    T *P = static_cast<T *>(a.P_out);
    const int64_t ld = a.ld_out > 0 ? a.ld_out : a.m_pad;
    for (int t0 = 0; t0 < a.m_pad; t0 += a.mt) {
        const int c = t0 + cc;
        double acc = 0.0;
        const double mu = PASS == 2 ? a.mean[(int64_t)g * a.m_pad + c] : 0.0;
        for (int64_t i = r0 + rr; active && i < r1; i += rows_per) {
            const double v = probe_value<T>(a, g, i, c);
            if (PASS == 1) {
                acc += v;
            } else {
                const T cv = (T)(v - mu);
                P[i * ld + c] = cv;
                acc += (double)cv * (double)cv;
            }
        }
        // fixed-order sum over the rows_per threads of this column
        sh[threadIdx.x] = acc;
        __syncthreads();
        if (rr == 0) {
            double sum = 0.0;
            for (int q = 0; q < rows_per; ++q) sum += sh[q * a.mt + cc];
            a.partials[(int64_t)b * a.m_pad + c] = sum;
        }
        __syncthreads();
    }
}

// (g, c) per block: adds graph g's probe-block partials in order.
template <int PASS>
__global__ void __launch_bounds__(256) k_probe_reduce(ProbeArgs a) {
    __shared__ double sh[256];
    const int g = blockIdx.x / a.m_pad, c = blockIdx.x % a.m_pad;
    const int64_t gc = (int64_t)g * a.m_pad + c;
    double sum = 0.0;
    for (int bb = a.graph_block_begin[g] + threadIdx.x; bb < a.graph_block_begin[g + 1]; bb += 256)
        sum += a.partials[(int64_t)bb * a.m_pad + c];
    sum = block_sum_256(sum, sh);
    if (threadIdx.x != 0) return;
    const int mg = a.graph_m ? a.graph_m[g] : a.m;
    const int kg = a.graph_k ? a.graph_k[g] : a.k;
    if (PASS == 1) {
        const double ng = (double)(a.graph_row_begin[g + 1] - a.graph_row_begin[g]);
        a.mean[gc] = a.desing ? sum / ng : 0.0;
    } else {
        a.norm2[gc] = sum;
        a.st_alpha[gc] = 0.0;
        a.st_coup[gc] = 0.0;
        // a NaN or Inf in a caller's probe block: reported, the column frozen
        if (!isfinite(sum) && c < mg && a.flags) atomicOr(a.flags, 1);
        if (sum > 0.0 && isfinite(sum) && c < mg) {
            a.st_inv[gc] = 1.0 / sqrt(sum);
            a.k_eff[gc] = kg;
        } else {
            a.st_inv[gc] = 0.0;
            a.k_eff[gc] = 0;
        }
    }
}

hipError_t launch_probe(const ProbeArgs &a, bool fp64, hipStream_t s) {
    dim3 g(a.n_blocks), r((unsigned)((int64_t)a.n_graphs * a.m_pad));
    if (fp64) {
        hipLaunchKernelGGL((k_probe<double, 1>), g, dim3(256), 0, s, a);
        hipLaunchKernelGGL((k_probe_reduce<1>), r, dim3(256), 0, s, a);
        hipLaunchKernelGGL((k_probe<double, 2>), g, dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_probe<float, 1>), g, dim3(256), 0, s, a);
        hipLaunchKernelGGL((k_probe_reduce<1>), r, dim3(256), 0, s, a);
        hipLaunchKernelGGL((k_probe<float, 2>), g, dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL((k_probe_reduce<2>), r, dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(256) k_rademacher_fill(T *out, int32_t n, int32_t m, int32_t ld,
                                                         int32_t off, int32_t col_offset, uint64_t seed,
                                                         const int64_t *keys) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)n * m) return;
    const int64_t i = t / m;
    const int c = (int)(t % m);
    out[i * ld + off + c] = (T)rademacher(seed, keys[i], (int64_t)col_offset + c);
}

hipError_t launch_rademacher_fill(void *out, bool fp64, int32_t n, int32_t m, int32_t ld, int32_t off,
                                  int32_t col_offset, uint64_t seed, const int64_t *keys,
                                  hipStream_t s) {
    const int64_t total = (int64_t)n * m;
    dim3 g((unsigned)((total + 255) / 256));
    if (fp64)
        hipLaunchKernelGGL(k_rademacher_fill<double>, g, dim3(256), 0, s, (double *)out, n, m, ld, off,
                           col_offset, seed, keys);
    else
        hipLaunchKernelGGL(k_rademacher_fill<float>, g, dim3(256), 0, s, (float *)out, n, m, ld, off,
                           col_offset, seed, keys);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Symmetric tridiagonal eigenproblem T = Z diag(theta) Z^T by implicit QR
// steps with Wilkinson shifts (Golub & Van Loan, implicit symmetric QR step),
// one wavefront per column.  Lane l keeps rows l and l + 64 of T (diagonal
// d, off-diagonal e, e[i] coupling i and i+1) and of the tracked first row z
// of Z in registers; the bulge chase runs wave-uniformly, reading the rows it
// needs with readlane and writing them back with a lane select.  Deflation is
// found for all indices at once with a ballot.
// ---------------------------------------------------------------------------

struct Rot {
    double c, s;
    int32_t i, pad;
};

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// element i (wave-uniform, < 128) of a two-register lane-resident vector;
// both halves are read and the choice is a scalar select (no branch)
template <int NH = 2>
__device__ __forceinline__ double get_row(double lo, double hi, int i) {
    if (NH == 1) return readlane_d(lo, i & 63);
    const double a = readlane_d(lo, i & 63), b = readlane_d(hi, i & 63);
    return i < 64 ? a : b;
}
// writes x into element i; any i outside [0, 64 * NH) (e.g. -1) writes nothing
template <int NH = 2>
__device__ __forceinline__ void set_row(double &lo, double &hi, int i, double x, int lane) {
    lo = (lane == i) ? x : lo;
    if (NH == 2) hi = (lane + 64 == i) ? x : hi;
}

// Givens rotation [c s; -s c] taking (x, y) to (r, 0): 1/r from the
// hardware reciprocal square root and one Newton step (c^2 + s^2 = 1 to a
// few units of rounding, which keeps the QR sweep backward stable).
__device__ __forceinline__ void givens(double x, double y, double &c, double &s, double &r) {
    const double a = fma(x, x, y * y);
    double q = __builtin_amdgcn_rsq(a);
    q = q * fma(-0.5 * a, q * q, 1.5);
    const bool nz = a > 0.0;
    c = nz ? x * q : 1.0;
    s = nz ? y * q : 0.0;
    r = nz ? a * q : 0.0;
}

struct LaneTri {
    double d0, d1, e0, e1, z0, z1;
    double w0 = 0.0, w1 = 0.0;   // last row of the eigenvector matrix (LAST)
};

// Runs the QR iteration on the first n (<= 128) rows.  With RECORD, every
// rotation goes to rot[0..cap), 64 at a time from lane-resident chunks.
// Returns 0 on success, bit 2 if an eigenvalue needed more than 60 sweeps,
// bit 3 if the record overflowed.  The chase body has no branch: the rows
// two ahead of the bulge (untouched by the sweep so far) are read while the
// rotation is computed.
template <bool RECORD, int NH, bool LAST = false>
__device__ int lane_tridiag_qr(LaneTri &t, int n, int lane, Rot *rot, int cap, int *nrot) {
    const double eps = 1.1102230246251565e-16;   // 2^-53
    int status = 0, cnt = 0;
    double rc = 1.0, rs = 0.0;
    int ri = 0;
    int hi = n - 1, sweeps = 0;
    while (hi > 0) {
        // negligible off-diagonals, all indices at once
        double dn0 = __shfl_down(t.d0, 1, 64);
        const double d64 = readlane_d(t.d1, 0);
        if (lane == 63) dn0 = d64;
        const double dn1 = __shfl_down(t.d1, 1, 64);
        const bool p0 = (lane >= n - 1) || fabs(t.e0) <= eps * (fabs(t.d0) + fabs(dn0)) || fabs(t.e0) < 1e-300;
        const bool p1 = (lane + 64 >= n - 1) || fabs(t.e1) <= eps * (fabs(t.d1) + fabs(dn1)) ||
                        fabs(t.e1) < 1e-300;
        const uint64_t m0 = __ballot(p0), m1 = __ballot(p1);
        const int b = hi - 1;
        const bool negl = b < 64 ? ((m0 >> b) & 1ull) : ((m1 >> (b - 64)) & 1ull);
        if (negl) {
            set_row<NH>(t.e0, t.e1, b, 0.0, lane);
            --hi;
            sweeps = 0;
            continue;
        }
        // lo = 1 + largest negligible index below hi - 1 (0 if none)
        int lo = 0;
        {
            uint64_t h1 = b > 64 ? (m1 & ((b - 64 >= 64) ? ~0ull : ((1ull << (b - 64)) - 1ull))) : 0ull;
            uint64_t h0 = b >= 64 ? m0 : (m0 & ((1ull << b) - 1ull));
            if (h1) lo = 64 + (63 - __builtin_clzll(h1)) + 1;
            else if (h0) lo = (63 - __builtin_clzll(h0)) + 1;
        }
        if (lo > 0) set_row<NH>(t.e0, t.e1, lo - 1, 0.0, lane);
        if (++sweeps > 60) {
            status |= 4;
            break;
        }
        // Wilkinson shift from the trailing 2x2 block
        const double dh1 = get_row<NH>(t.d0, t.d1, hi - 1), dh = get_row<NH>(t.d0, t.d1, hi);
        const double bh = get_row<NH>(t.e0, t.e1, hi - 1);
        const double dl = 0.5 * (dh1 - dh);
        const double rt = sqrt(fma(dl, dl, bh * bh));
        const double den = dl + (dl < 0.0 ? -rt : rt);
        const double mu = dh - bh * (bh / den);
        // bulge chase with the active rows carried in registers
        double di = get_row<NH>(t.d0, t.d1, lo), dj = get_row<NH>(t.d0, t.d1, lo + 1);
        double ei = get_row<NH>(t.e0, t.e1, lo);
        const double e_lo1 = get_row<NH>(t.e0, t.e1, lo + 1);
        double enx = lo + 1 < hi ? e_lo1 : 0.0;
        double zi = get_row<NH>(t.z0, t.z1, lo), zj = get_row<NH>(t.z0, t.z1, lo + 1);
        double wi = 0.0, wj = 0.0;
        if (LAST) {
            wi = get_row<NH>(t.w0, t.w1, lo);
            wj = get_row<NH>(t.w0, t.w1, lo + 1);
        }
        double x = di - mu, y = ei;
        for (int i = lo; i < hi; ++i) {
            const int i2 = min(i + 2, 64 * NH - 1);
            const double dn = get_row<NH>(t.d0, t.d1, i2), en = get_row<NH>(t.e0, t.e1, i2);
            const double zn = get_row<NH>(t.z0, t.z1, i2);
            const double wn = LAST ? get_row<NH>(t.w0, t.w1, i2) : 0.0;
            double c, sn, r;
            givens(x, y, c, sn, r);
            set_row<NH>(t.e0, t.e1, i > lo ? i - 1 : -1, r, lane);
            const double cs = c * sn, cc = c * c, ss = sn * sn;
            const double ndi = fma(cc, di, fma(2.0 * cs, ei, ss * dj));
            const double ndj = fma(ss, di, fma(-2.0 * cs, ei, cc * dj));
            const double nei = fma(cs, dj - di, (cc - ss) * ei);
            const double nzi = fma(c, zi, sn * zj);
            const double nzj = fma(-sn, zi, c * zj);
            const double nwi = fma(c, wi, sn * wj);
            const double nwj = fma(-sn, wi, c * wj);
            set_row<NH>(t.d0, t.d1, i, ndi, lane);
            set_row<NH>(t.z0, t.z1, i, nzi, lane);
            if (LAST) set_row<NH>(t.w0, t.w1, i, nwi, lane);
            if (RECORD) {
                const int slot = cnt & 63;
                rc = lane == slot ? c : rc;
                rs = lane == slot ? sn : rs;
                ri = lane == slot ? i : ri;
                ++cnt;
                if ((cnt & 63) == 0) {
                    if (cnt <= cap) rot[cnt - 64 + lane] = Rot{rc, rs, ri, 0};
                    else status |= 8;
                }
            }
            // carried rows for the next rotation (after the last one they
            // hold rows hi - 1 and hi of the sweep's result)
            y = sn * enx;
            ei = c * enx;
            x = nei;
            di = ndj;
            dj = dn;
            enx = i + 2 < hi ? en : 0.0;
            zi = nzj;
            zj = zn;
            wi = nwj;
            wj = wn;
        }
        set_row<NH>(t.d0, t.d1, hi, di, lane);
        set_row<NH>(t.e0, t.e1, hi - 1, x, lane);
        set_row<NH>(t.z0, t.z1, hi, zi, lane);
        if (LAST) set_row<NH>(t.w0, t.w1, hi, wi, lane);
    }
    if (RECORD) {
        const int part = cnt & 63;
        if (part) {
            if (cnt <= cap) {
                if (lane < part) rot[cnt - part + lane] = Rot{rc, rs, ri, 0};
            } else {
                status |= 8;
            }
        }
        if (nrot) *nrot = min(cnt, cap);
    }
    return status;
}

__device__ __forceinline__ void load_tri(LaneTri &t, const double *alpha, const double *beta, int ke, int lane) {
    t.d0 = lane < ke ? alpha[lane] : 0.0;
    t.d1 = lane + 64 < ke ? alpha[lane + 64] : 0.0;
    t.e0 = lane + 1 < ke ? beta[lane] : 0.0;
    t.e1 = lane + 65 < ke ? beta[lane + 64] : 0.0;
    t.z0 = lane == 0 ? 1.0 : 0.0;
    t.z1 = 0.0;
}

// fixed-order sum over the 64 lanes (butterfly; every lane gets the result)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// e1^T f(T) e1 for f = -x log x (the value of the Gauss rule of eq. (4.2))
// without diagonalising T.  With sigma >= lambda_max(T) (Gershgorin) and
// T~ = T / sigma, f(T) = sigma f(T~) - sigma log(sigma) T~; for 0 <= x <= 1,
// -x log x = x (1 - x) int_0^inf dt / ((x + t)(1 + t)), so
// e1^T f(T~) e1 = int_0^inf u^T (T~ + t I)^{-1} e1 dt / (1 + t) with
// u = T~ (I - T~) e1, whose only nonzero entries are the first three.  The
// first three entries of (T~ + t I)^{-1} e1 follow from the pivots of the
// bottom-up elimination d_k = a_k + t, d_j = a_j + t - b_j^2 / d_{j+1}, all
// positive while T~ + t I is positive definite.
//
// The integral runs from t0 = 2 c, c the smallest of 5e-16, 5e-14, ...,
// 5e-8 (at most shift_max + 1 of them) at which T~ + c I is positive
// definite (checked by the same elimination), so every eigenvalue of
// T~ + t I at the nodes is at least t / 2.  c is 5e-16 unless T has negative
// Ritz values beyond rounding of the coefficients (with FP32 vectors a
// component along a null vector can give -1e-8 sigma); the eigen route
// gives such values f = 0, and the integral differs from it by about c
// relative.  The part
// below t0 is t0 (1 - a_1) to first order (the integrand tends to
// e1^T (I - T~) e1 as t -> 0), added as is.  With t = e^s the rule is the
// trapezoidal one in s on [ln t0, 37] with kQuadNodes points (three per
// lane): the integrand is analytic in a strip of half-width pi about the
// real axis, so the error falls geometrically with the spacing (below 1e-14
// relative against diagonalisation at t0 = 1e-15, on Lanczos matrices of
// graphs and on a spectrum spanning 1e-3..1e3).  Returns false, for the
// whole wave, if no allowed shift makes T~ positive definite: the caller
// then diagonalises.
constexpr int kQuadNodes = 192;

template <int NH>
__device__ bool e1_fT_e1_integral(const LaneTri &t, int ke, int lane, int shift_max, double &out) {
    // Gershgorin bound of T: |alpha_r| + |beta_{r-1}| + |beta_r| over the rows
    const double up0 = __shfl_up(t.e0, 1, 64);
    const double prev0 = lane == 0 ? 0.0 : up0;
    double g = lane < ke ? fabs(t.d0) + fabs(t.e0) + fabs(prev0) : 0.0;
    if (NH == 2) {
        const double up1 = __shfl_up(t.e1, 1, 64);
        const double e63 = readlane_d(t.e0, 63);
        const double prev1 = lane == 0 ? e63 : up1;
        g = fmax(g, lane + 64 < ke ? fabs(t.d1) + fabs(t.e1) + fabs(prev1) : 0.0);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) g = fmax(g, __shfl_xor(g, o, 64));
    const double sigma = g;
    if (!(sigma > 0.0)) {
        out = 0.0;                       // T = 0: f(0) = 0
        return true;
    }
    const double is = 1.0 / sigma;
    // 1. positive definiteness of T~ + c I for the candidate shifts
    constexpr int NC = 5;
    const double shift[NC] = {5e-16, 5e-14, 5e-12, 5e-10, 5e-8};
    double ic[NC];
    bool pc[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        ic[q] = 0.0;
        pc[q] = true;
    }
    for (int j = ke - 1; j >= 0; --j) {
        const double aj = get_row<NH>(t.d0, t.d1, j) * is;
        const double bj = j < ke - 1 ? get_row<NH>(t.e0, t.e1, j) * is : 0.0;
        const double bj2 = bj * bj;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const double d = fma(-bj2, ic[q], aj + shift[q]);
            pc[q] = pc[q] && d > 0.0;
            ic[q] = 1.0 / d;
        }
    }
    double c0 = -1.0;
#pragma unroll
    for (int q = NC - 1; q >= 0; --q) c0 = (pc[q] && q <= shift_max) ? shift[q] : c0;
    // wave-uniform data: every lane took the same decisions
    c0 = readlane_d(c0, 0);
    if (c0 < 0.0) return false;
    // 2. the trapezoidal rule on [ln t0, 37]
    const double t0 = 2.0 * c0;
    const double s_lo = log(t0);
    const double s_hi = 37.0;
    const double h = (s_hi - s_lo) / (double)(kQuadNodes - 1);
    double tt[3], inv[3], inv1[3], inv2[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        tt[q] = exp(s_lo + h * (double)(lane + 64 * q));
        inv[q] = 0.0;
        inv1[q] = inv2[q] = 0.0;
    }
    for (int j = ke - 1; j >= 0; --j) {
        const double aj = get_row<NH>(t.d0, t.d1, j) * is;
        const double bj = j < ke - 1 ? get_row<NH>(t.e0, t.e1, j) * is : 0.0;
        const double bj2 = bj * bj;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double d = fma(-bj2, inv[q], aj + tt[q]);
            inv[q] = 1.0 / d;
            if (j == 2) inv2[q] = inv[q];
            if (j == 1) inv1[q] = inv[q];
        }
    }
    const double a0 = get_row<NH>(t.d0, t.d1, 0) * is;
    const double a1 = ke > 1 ? get_row<NH>(t.d0, t.d1, 1) * is : 0.0;
    const double b0 = ke > 1 ? get_row<NH>(t.e0, t.e1, 0) * is : 0.0;
    const double b1 = ke > 2 ? get_row<NH>(t.e0, t.e1, 1) * is : 0.0;
    const double u1 = a0 - a0 * a0 - b0 * b0;
    const double u2 = b0 * (1.0 - a0 - a1);
    const double u3 = -b0 * b1;
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int n = lane + 64 * q;
        const double y1 = inv[q];
        const double y2 = ke > 1 ? -b0 * y1 * inv1[q] : 0.0;
        const double y3 = ke > 2 ? -b1 * y2 * inv2[q] : 0.0;
        const double w = (n == 0 || n == kQuadNodes - 1) ? 0.5 * h : h;
        part += w * (u1 * y1 + u2 * y2 + u3 * y3) * (tt[q] / (1.0 + tt[q]));
    }
    const double integral = wave_sum(part) + t0 * (1.0 - a0);
    out = sigma * integral - log(sigma) * (a0 * sigma);
    return true;
}

__global__ void __launch_bounds__(256) k_quadrature(const double *alpha, const double *beta,
                                                    const int32_t *k_eff, const double *norm2, int32_t k,
                                                    int32_t steps, int32_t m, double *psi, int32_t *flags,
                                                    const int2 *stop, int32_t uid, const int32_t *col_stop,
                                                    int32_t shift_max, int32_t *steps_out) {
    const int c = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (c >= m) return;
    if (stop) {
        const int2 st = *stop;
        if (st.x == uid && st.y > 0) steps = min(steps, st.y);
    }
    // the steps the problem's quadrature takes (the same for every column
    // before per-column stops), kept as the largest over the problems that
    // share the word
    if (steps_out && c == 0 && lane == 0) atomicMax(steps_out, steps);
    if (col_stop) {
        const int cs = __builtin_amdgcn_readfirstlane(col_stop[c]);
        if (cs > 0) steps = min(steps, cs);
    }
    const int ke = __builtin_amdgcn_readfirstlane(min(k_eff[c], steps));
    if (ke <= 0) {
        if (lane == 0) psi[c] = 0.0;
        return;
    }
    LaneTri t;
    load_tri(t, alpha + (int64_t)c * k, beta + (int64_t)c * k, ke, lane);
    double val = 0.0;
    const bool done = ke <= 64 ? e1_fT_e1_integral<1>(t, ke, lane, shift_max, val)
                               : e1_fT_e1_integral<2>(t, ke, lane, shift_max, val);
    if (done) {
        if (lane == 0) psi[c] = norm2[c] * val;
        return;
    }
    const int st = ke <= 64 ? lane_tridiag_qr<false, 1>(t, ke, lane, nullptr, 0, nullptr)
                            : lane_tridiag_qr<false, 2>(t, ke, lane, nullptr, 0, nullptr);
    double part = 0.0;
    if (lane < ke) part += t.z0 * t.z0 * f_entropy(t.d0);
    if (lane + 64 < ke) part += t.z1 * t.z1 * f_entropy(t.d1);
    const double tot = wave_sum(part);
    if (lane == 0) {
        psi[c] = norm2[c] * tot;
        if (st) atomicOr(flags, st);
    }
}

// ---------------------------------------------------------------------------
// A-posteriori error bracket of Theorem 4.8 for the polynomial Krylov method
// (K_m = I, h_{m+1} = beta_m e_m): with T_m = U diag(theta) U^T,
// a_j = beta_m U[m-1, j], b_j = U[0, j], c_j = sum_{l != j} a_l b_l / (theta_j -
// theta_l), eq. (4.8) is g_m(z) = sum_j (a_j b_j)^2 D2(z, theta_j) +
// 2 a_j b_j c_j D1(z, theta_j) with the divided differences of f = -x log x
// D1 = (f(z) - f(theta)) / (z - theta), D2 = (D1 - f'(theta)) / (z - theta).
// With r = z / theta, t = r - 1: D1 = -log theta - (1 + t) log1p(t) / t and
// D2 = q(t) / theta, q(t) = (t - (1 + t) log1p(t)) / t^2, by their Taylor
// series for |t| < 1e-3 (the limits at z = theta are the ones eq. (4.8)
// gives).  lo, hi = ||c||^2 min, max |g_m| over [lam_lo, lam_hi].  The
// columns are evaluated in the residue form of eq. (4.8) (bound_integral
// below), which gives the extremes at the ends of the interval; a column
// with a Ritz value below -5e-16 of its scale is evaluated term by term over
// n_grid log-spaced points and the Ritz values inside the interval, Ritz
// values below lam_lo raised to it.  A column whose recurrence stopped on a
// zero beta has an invariant Krylov space and zero error.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void entropy_dd(double z, double th, double log_th, double inv_th, double &d1,
                                           double &d2) {
    const double t = fma(z, inv_th, -1.0);
    double h, q;
    if (fabs(t) < 1e-3) {
        h = 1.0 + t * (0.5 + t * (-1.0 / 6.0 + t * (1.0 / 12.0 + t * (-1.0 / 20.0))));
        q = -0.5 + t * (1.0 / 6.0 + t * (-1.0 / 12.0 + t * (1.0 / 20.0 + t * (-1.0 / 30.0))));
    } else {
        const double l1 = log1p(t);
        const double it = 1.0 / t;
        h = (1.0 + t) * l1 * it;
        q = (t - (1.0 + t) * l1) * it * it;
    }
    d1 = -log_th - h;
    d2 = q * inv_th;
}

// The bracket without diagonalising T_m.  With h(w) = sum_j a_j b_j / (w -
// theta_j) = beta_m e1^T (w I - T_m)^{-1} e_m, eq. (4.8) is the sum of the
// residues of f(w) h(w)^2 / (w - z) at the Ritz values and at z (double poles
// at theta_j give the D2 terms, the cross terms of h^2 the c_j D1 terms).  For
// f = -x log x on the scaled problem (T~ = T_m / sigma, spectrum in [0, 1];
// g_m scales as sigma g~_m(z / sigma), the linear part of f contributing
// nothing) the representation -x log x = int_0^inf x (1 - x) / ((x + t)(1 + t))
// dt turns every residue sum into minus the residue at w = -t, so
//     g~_m(z) = - int_0^inf t h~(-t)^2 / (t + z) dt,
//     h~(-t)^2 = beta~_m^2 (e1^T (T~ + t I)^{-1} e_m)^2
//              = beta~_m^2 prod_{i < m} (beta~_i / p_i)^2 / p_m^2
// with the top-down pivots p_1 = a_1 + t, p_{i+1} = a_{i+1} + t - b_i^2 / p_i.
// g is negative and |g| decreases in z, so the extremes over [lam_lo, lam_hi]
// are its values at the ends: hi = ||c||^2 |g(lam_lo)|, lo = ||c||^2
// |g(lam_hi)|.  (Against a 50-digit evaluation of eq. (4.8) this agrees to
// 3e-15; eq. (4.8) in double precision loses up to 4e-8 to cancellation at
// m = 20.)  Same trapezoidal rule in ln t as the quadrature, from t0 = 1e-15
// (the part below t0 is O(t0^2)); the running product is renormalised with
// frexp.  Returns false when T~ + 5e-16 I is not positive definite (a
// Ritz value below -5e-16 sigma), for the QR route with its floor.
template <int NH>
__device__ bool bound_integral(const LaneTri &t, int mm, double beta_m, double lam_lo, double lam_hi, int lane,
                               double &g_lo, double &g_hi) {
    const double up0 = __shfl_up(t.e0, 1, 64);
    const double prev0 = lane == 0 ? 0.0 : up0;
    double g = lane < mm ? fabs(t.d0) + fabs(t.e0) + fabs(prev0) : 0.0;
    if (NH == 2) {
        const double up1 = __shfl_up(t.e1, 1, 64);
        const double e63 = readlane_d(t.e0, 63);
        const double prev1 = lane == 0 ? e63 : up1;
        g = fmax(g, lane + 64 < mm ? fabs(t.d1) + fabs(t.e1) + fabs(prev1) : 0.0);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) g = fmax(g, __shfl_xor(g, o, 64));
    const double sigma = g;
    if (!(sigma > 0.0)) return false;
    const double is = 1.0 / sigma;
    // positive definiteness of T~ + 5e-16 I (bottom-up, as in the quadrature),
    // so that T~ + t I has every eigenvalue at least t / 2 at the nodes
    {
        double ic = 0.0;
        bool pd = true;
        for (int j = mm - 1; j >= 0; --j) {
            const double aj = get_row<NH>(t.d0, t.d1, j) * is;
            const double bj = j < mm - 1 ? get_row<NH>(t.e0, t.e1, j) * is : 0.0;
            const double d = fma(-bj * bj, ic, aj + 5e-16);
            pd = pd && d > 0.0;
            ic = 1.0 / d;
        }
        if (__builtin_amdgcn_readfirstlane(pd ? 1 : 0) == 0) return false;
    }
    const double bm = beta_m * is;
    const double zl = lam_lo * is, zh = lam_hi * is;
    const double s_lo = -34.538776394910684;          // ln 1e-15
    const double h = (37.0 - s_lo) / (double)(kQuadNodes - 1);
    double part_l = 0.0, part_h = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int n = lane + 64 * q;
        const double tt = exp(s_lo + h * (double)n);
        double p = 0.0, prod = 1.0;
        int ex = 0;
        for (int j = 0; j < mm; ++j) {
            const double aj = get_row<NH>(t.d0, t.d1, j) * is;
            const double bprev = j > 0 ? get_row<NH>(t.e0, t.e1, j - 1) * is : 0.0;
            p = j > 0 ? aj + tt - bprev * bprev / p : aj + tt;
            if (j < mm - 1) {
                const double bj = get_row<NH>(t.e0, t.e1, j) * is;
                const double r = bj / p;
                prod *= r * r;
            } else {
                prod /= p * p;
            }
            int e;
            prod = frexp(prod, &e);
            ex += e;
        }
        const double h2 = ldexp(prod, ex) * bm * bm;           // h~(-t)^2 (0 on underflow)
        const double w = (n == 0 || n == kQuadNodes - 1) ? 0.5 * h : h;
        const double tw = w * tt * tt * h2;                    // dt = t ds
        part_l += tw / (tt + zl);
        part_h += tw / (tt + zh);
    }
    g_lo = sigma * wave_sum(part_l);     // |g| at lam_lo (the maximum)
    g_hi = sigma * wave_sum(part_h);     // |g| at lam_hi (the minimum)
    return true;
}

template <int NH>
__device__ void bound_column(const BoundArgs &a, int c, int lane) {
    if (a.col_stop && __builtin_amdgcn_readfirstlane(a.col_stop[c]) > 0) return;   // stopped earlier
    const int64_t base = (int64_t)c * a.k;
    const int ke = __builtin_amdgcn_readfirstlane(a.k_eff[c]);
    const int mm = min(ke, a.steps);
    const double beta_m = mm > 0 ? a.beta[base + mm - 1] : 0.0;
    if (mm <= 0 || beta_m == 0.0) {
        if (lane == 0) {
            a.lo[c] = 0.0;
            a.hi[c] = 0.0;
        }
        return;
    }
    LaneTri t;
    load_tri(t, a.alpha + base, a.beta + base, mm, lane);
    {
        double gmax = 0.0, gmin = 0.0;
        if (bound_integral<NH>(t, mm, beta_m, a.lam_lo, a.lam_hi, lane, gmax, gmin)) {
            if (lane == 0) {
                const double nb = a.norm2[c];
                a.lo[c] = nb * gmin;
                a.hi[c] = nb * gmax;
            }
            return;
        }
    }
    t.w0 = lane == mm - 1 ? 1.0 : 0.0;
    t.w1 = lane + 64 == mm - 1 ? 1.0 : 0.0;
    const int st = lane_tridiag_qr<false, NH, true>(t, mm, lane, nullptr, 0, nullptr);
    if (st && lane == 0) atomicOr(a.flags, st);
    // per Ritz value (lane j, and j + 64): a_j b_j, c_j, the raised theta
    double ab0 = lane < mm ? beta_m * t.w0 * t.z0 : 0.0;
    double ab1 = lane + 64 < mm ? beta_m * t.w1 * t.z1 : 0.0;
    double c0 = 0.0, c1 = 0.0;
    for (int l = 0; l < mm; ++l) {
        const double thl = get_row<NH>(t.d0, t.d1, l), abl = get_row<NH>(ab0, ab1, l);
        if (l != lane) c0 += abl / (t.d0 - thl);
        if (NH == 2 && l != lane + 64) c1 += abl / (t.d1 - thl);
    }
    const double th0 = fmax(t.d0, a.lam_lo), th1 = fmax(t.d1, a.lam_lo);
    const double lg0 = log(th0), lg1 = log(th1), iv0 = 1.0 / th0, iv1 = 1.0 / th1;
    const double ratio = log(a.lam_hi / a.lam_lo) / (double)max(a.n_grid - 1, 1);
    double gmax = 0.0, gmin = INFINITY;
    const int npts = a.n_grid + mm;
    for (int p0 = 0; p0 < npts; p0 += 64) {
        const int p = p0 + lane;
        // grid point, or the Ritz value p - n_grid if it lies inside the interval
        const int j = max(p - a.n_grid, 0);
        const double s0 = __shfl(t.d0, j & 63, 64), s1 = __shfl(t.d1, j & 63, 64);
        const double th = j < 64 ? s0 : s1;
        const bool grid_pt = p < a.n_grid;
        const double z = grid_pt ? (p == a.n_grid - 1 ? a.lam_hi : a.lam_lo * exp(ratio * (double)p)) : th;
        const bool use = p < npts && (grid_pt || (th > a.lam_lo && th < a.lam_hi));
        double g = 0.0;
        for (int j = 0; j < mm; ++j) {
            const double thj = get_row<NH>(th0, th1, j), lgj = get_row<NH>(lg0, lg1, j);
            const double ivj = get_row<NH>(iv0, iv1, j), abj = get_row<NH>(ab0, ab1, j);
            const double cj = get_row<NH>(c0, c1, j);
            (void)thj;
            double d1, d2;
            entropy_dd(z, thj, lgj, ivj, d1, d2);
            g = fma(abj * abj, d2, fma(2.0 * abj * cj, d1, g));
        }
        if (use) {
            gmax = fmax(gmax, fabs(g));
            gmin = fmin(gmin, fabs(g));
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        gmax = fmax(gmax, __shfl_xor(gmax, o, 64));
        gmin = fmin(gmin, __shfl_xor(gmin, o, 64));
    }
    if (lane == 0) {
        const double nb = a.norm2[c];
        a.lo[c] = nb * gmin;
        a.hi[c] = nb * gmax;
    }
}

// entry e = {problem, column group}: columns 4 e.y .. 4 e.y + 3 of args[e.x]
__global__ void __launch_bounds__(256) k_error_bound(const BoundArgs *args, const int2 *map) {
    const int2 e = map[blockIdx.x];
    const BoundArgs a = args[e.x];
    if (slot_stopped(a.stop_state, a.stop_uid, a.stop_count)) return;
    const int c = __builtin_amdgcn_readfirstlane(e.y * 4 + (int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (c >= a.m) return;
    const int ke = __builtin_amdgcn_readfirstlane(min(a.k_eff[c], a.steps));
    if (ke <= 64) bound_column<1>(a, c, lane);
    else bound_column<2>(a, c, lane);
}

hipError_t launch_error_bound(const BoundArgs *args, const int2 *map, int32_t n_entries, hipStream_t s) {
    if (n_entries > 0) hipLaunchKernelGGL(k_error_bound, dim3(n_entries), dim3(256), 0, s, args, map);
    return hipGetLastError();
}

// One block per problem: if every column's upper bound (or, with estimate,
// the geometric mean of its bracket) is within tol, the first such step is
// recorded in state = {uid, stop step} (a state left by an earlier owner of
// the memory, with another uid, is reset first).
__global__ void __launch_bounds__(64) k_stop_check(const StopArgs *args) {
    const StopArgs a = args[blockIdx.x];
    bool ok = true;
    for (int c = threadIdx.x; c < a.m; c += 64) {
        const double e = a.estimate ? sqrt(a.lo[c] * a.hi[c]) : a.hi[c];
        ok = ok && e <= a.tol;
    }
    const bool all = __all(ok);
    if (threadIdx.x != 0) return;
    int2 st = *a.state;
    if (st.x != a.uid) st = make_int2(a.uid, 0);
    if (all && st.y == 0) st.y = a.step;
    *a.state = st;
    if (a.mail) *a.mail = st;
}

hipError_t launch_stop_check(const StopArgs *args, int32_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_stop_check, dim3(n), dim3(64), 0, s, args);
    return hipGetLastError();
}

// Columns [4 b, 4 b + 4) of the one problem *args per block (b = blockIdx.x).
__global__ void __launch_bounds__(256) k_error_bound_cols(const BoundArgs *args) {
    const BoundArgs a = *args;
    const int c = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + (int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (c >= a.m) return;
    const int ke = __builtin_amdgcn_readfirstlane(min(a.k_eff[c], a.steps));
    if (ke <= 64) bound_column<1>(a, c, lane);
    else bound_column<2>(a, c, lane);
}

hipError_t launch_error_bound_cols(const BoundArgs *args, int32_t m, hipStream_t s) {
    if (m > 0) hipLaunchKernelGGL(k_error_bound_cols, dim3((m + 3) / 4), dim3(256), 0, s, args);
    return hipGetLastError();
}

// One block: every running column whose upper bound is within its tolerance
// records the step; the count of columns still running goes to *remaining.
__global__ void __launch_bounds__(256) k_column_stop(const ColStopArgs *args) {
    const ColStopArgs a = *args;
    __shared__ int part[4];
    int run = 0;
    for (int c = threadIdx.x; c < a.m; c += 256) {
        int cs = a.col_stop[c];
        const double e = a.estimate ? sqrt(a.lo[c] * a.hi[c]) : a.hi[c];
        if (cs == 0 && e <= a.tol[c]) {
            cs = a.step;
            a.col_stop[c] = cs;
        }
        run += cs == 0;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) run += __shfl_xor(run, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = run;
    __syncthreads();
    if (threadIdx.x == 0) *a.remaining = part[0] + part[1] + part[2] + part[3];
}

hipError_t launch_column_stop(const ColStopArgs *args, hipStream_t s) {
    hipLaunchKernelGGL(k_column_stop, dim3(1), dim3(256), 0, s, args);
    return hipGetLastError();
}

hipError_t launch_quadrature(const double *alpha, const double *beta, const int32_t *k_eff,
                             const double *norm2, int32_t k, int32_t steps, int32_t m, double *psi,
                             int32_t *flags, hipStream_t s, bool fp64, const int2 *stop, int32_t uid,
                             const int32_t *col_stop, int32_t *steps_out) {
    if (k > kMaxSteps || steps < 1 || steps > k) return hipErrorInvalidValue;
    // FP64 vectors: shifts up to 5e-14 (below 1e-13 relative); FP32: up to 5e-8
    const int32_t shift_max = fp64 ? 1 : 4;
    hipLaunchKernelGGL(k_quadrature, dim3((m + 3) / 4), dim3(256), 0, s, alpha, beta, k_eff, norm2, k, steps, m,
                       psi, flags, stop, uid, col_stop, shift_max, steps_out);
    return hipGetLastError();
}

__host__ __device__ int64_t rot_capacity(int32_t k) { return 4 * (int64_t)k * k + 64; }

// f(T) e1 = Z f(theta) Z^T e1: QR with the rotations recorded, then the
// rotations are applied in reverse order to w = f(theta) .* z.  Rows of the
// result come back lane-resident in w0 (rows 0..63) and w1 (64..127).
template <int NH>
__device__ int fT_e1_qr(LaneTri t, int ke, int lane, Rot *rot, int cap, double &w0, double &w1) {
    int nrot = 0;
    const int st = lane_tridiag_qr<true, NH>(t, ke, lane, rot, cap, &nrot);
    w0 = lane < ke ? f_entropy(t.d0) * t.z0 : 0.0;
    w1 = lane + 64 < ke ? f_entropy(t.d1) * t.z1 : 0.0;
    // the wave's own record, read back in reverse order in chunks of 64 (lane
    // j of a chunk holds rotation top - 64 + j); the next chunk is in flight
    // while the current one is applied
    __threadfence_block();
    auto fetch = [&](int top, double &cr, double &sr, int &ir) {
        const int idx = top - 64 + lane;
        if (idx >= 0) {
            const Rot r = rot[idx];
            cr = r.c;
            sr = r.s;
            ir = r.i;
        } else {
            cr = 1.0;
            sr = 0.0;
            ir = 0;
        }
    };
    double cr = 1.0, sr = 0.0;
    int ir = 0;
    if (nrot > 0) fetch(nrot, cr, sr, ir);
    for (int top = nrot; top > 0; top -= 64) {
        double ncr = 1.0, nsr = 0.0;
        int nir = 0;
        if (top > 64) fetch(top - 64, ncr, nsr, nir);
        const int j_end = top >= 64 ? 0 : 64 - top;
        for (int j = 63; j >= j_end; --j) {
            const double c = readlane_d(cr, j), sn = readlane_d(sr, j);
            const int i = __builtin_amdgcn_readlane(ir, j);
            const double a = get_row(w0, w1, i), b = get_row(w0, w1, i + 1);
            set_row(w0, w1, i, fma(c, a, -sn * b), lane);
            set_row(w0, w1, i + 1, fma(sn, a, c * b), lane);
        }
        cr = ncr;
        sr = nsr;
        ir = nir;
    }
    return st;
}

// y = M x for the symmetric tridiagonal M with diagonal d and off-diagonal e
// (e couples rows r and r + 1), all lane-resident (rows r and r + 64).
template <int NH>
__device__ __forceinline__ void tri_mul(double d0, double d1, double e0, double e1, double x0, double x1,
                                        int lane, double &y0, double &y1) {
    // every cross-lane read runs on all lanes; the row ends are selected after
    const double up_x0 = __shfl_up(x0, 1, 64), up_e0 = __shfl_up(e0, 1, 64), dn_x0 = __shfl_down(x0, 1, 64);
    const double x64 = NH == 2 ? readlane_d(x1, 0) : 0.0;
    const double xm0 = lane == 0 ? 0.0 : up_x0;
    const double em0 = lane == 0 ? 0.0 : up_e0;
    const double xp0 = lane == 63 ? x64 : dn_x0;
    y0 = fma(d0, x0, fma(em0, xm0, e0 * xp0));
    y1 = 0.0;
    if (NH == 2) {
        const double x63 = readlane_d(x0, 63), e63 = readlane_d(e0, 63);
        const double up_x1 = __shfl_up(x1, 1, 64), up_e1 = __shfl_up(e1, 1, 64), dn_x1 = __shfl_down(x1, 1, 64);
        const double xm1 = lane == 0 ? x63 : up_x1;
        const double em1 = lane == 0 ? e63 : up_e1;
        const double xp1 = lane == 63 ? 0.0 : dn_x1;
        y1 = fma(d1, x1, fma(em1, xm1, e1 * xp1));
    }
}

// f(T) e1 by the integral representation of the quadrature kernel: with
// z(t) = (T~ + t I)^{-1} e1 and Z = int z(t) dt / (1 + t) over [t0, inf),
// f(T~) e1 = T~ (I - T~) Z + t0 (I - T~) e1 (the part below t0 to first
// order) and f(T) e1 = sigma f(T~) e1 - log(sigma) T e1.  For each node, the
// bottom-up elimination stores the inverse pivots of the lane's node in LDS,
// then z_1 = 1/d_1, z_{j+1} = -b_j z_j / d_{j+1} runs forward and every
// entry is summed over the lanes' nodes (fixed butterfly order) into the
// lane-resident Z.  Returns false when no allowed shift makes T~ positive
// definite (the caller takes the QR route).
template <int NH>
__device__ bool fT_e1_integral(const LaneTri &t, int ke, int lane, int shift_max, double *piv, double &r0,
                               double &r1) {
    const double up0 = __shfl_up(t.e0, 1, 64);
    const double prev0 = lane == 0 ? 0.0 : up0;
    double g = lane < ke ? fabs(t.d0) + fabs(t.e0) + fabs(prev0) : 0.0;
    if (NH == 2) {
        const double up1 = __shfl_up(t.e1, 1, 64);
        const double e63 = readlane_d(t.e0, 63);
        const double prev1 = lane == 0 ? e63 : up1;
        g = fmax(g, lane + 64 < ke ? fabs(t.d1) + fabs(t.e1) + fabs(prev1) : 0.0);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) g = fmax(g, __shfl_xor(g, o, 64));
    const double sigma = g;
    r0 = r1 = 0.0;
    if (!(sigma > 0.0)) return true;     // T = 0: f(T) e1 = 0
    const double is = 1.0 / sigma;
    constexpr int NC = 5;
    const double shift[NC] = {5e-16, 5e-14, 5e-12, 5e-10, 5e-8};
    double ic[NC];
    bool pc[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        ic[q] = 0.0;
        pc[q] = true;
    }
    for (int j = ke - 1; j >= 0; --j) {
        const double aj = get_row<NH>(t.d0, t.d1, j) * is;
        const double bj = j < ke - 1 ? get_row<NH>(t.e0, t.e1, j) * is : 0.0;
        const double bj2 = bj * bj;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const double d = fma(-bj2, ic[q], aj + shift[q]);
            pc[q] = pc[q] && d > 0.0;
            ic[q] = 1.0 / d;
        }
    }
    double c0 = -1.0;
#pragma unroll
    for (int q = NC - 1; q >= 0; --q) c0 = (pc[q] && q <= shift_max) ? shift[q] : c0;
    c0 = readlane_d(c0, 0);
    if (c0 < 0.0) return false;
    const double t0 = 2.0 * c0;
    const double s_lo = log(t0);
    const double h = (37.0 - s_lo) / (double)(kQuadNodes - 1);
    double Z0 = 0.0, Z1 = 0.0;
    for (int q = 0; q < 3; ++q) {
        const int n = lane + 64 * q;
        const double tt = exp(s_lo + h * (double)n);
        const double w = ((n == 0 || n == kQuadNodes - 1) ? 0.5 * h : h) * (tt / (1.0 + tt));
        double inv = 0.0;
        for (int j = ke - 1; j >= 0; --j) {
            const double aj = get_row<NH>(t.d0, t.d1, j) * is;
            const double bj = j < ke - 1 ? get_row<NH>(t.e0, t.e1, j) * is : 0.0;
            inv = 1.0 / fma(-bj * bj, inv, aj + tt);
            piv[j * 64 + lane] = inv;
        }
        double z = piv[lane];
        for (int j = 0; j < ke; ++j) {
            const double sj = wave_sum(w * z);
            if (j < 64) Z0 += lane == j ? sj : 0.0;
            else Z1 += lane == j - 64 ? sj : 0.0;
            if (j + 1 < ke) z = -(get_row<NH>(t.e0, t.e1, j) * is) * z * piv[(j + 1) * 64 + lane];
        }
    }
    // f(T~) e1 = T~ (Z - T~ Z) + t0 (e1 - T~ e1), T~ = T / sigma
    const double a0 = t.d0 * is, a1 = t.d1 * is, b0 = t.e0 * is, b1 = t.e1 * is;
    double y0, y1, v0, v1;
    tri_mul<NH>(a0, a1, b0, b1, Z0, Z1, lane, y0, y1);
    tri_mul<NH>(a0, a1, b0, b1, Z0 - y0, Z1 - y1, lane, v0, v1);
    const double e1_0 = lane == 0 ? 1.0 : 0.0;
    double te0, te1;
    tri_mul<NH>(a0, a1, b0, b1, e1_0, 0.0, lane, te0, te1);
    const double f0 = v0 + t0 * (e1_0 - te0), f1 = v1 - t0 * te1;
    // f(T) e1 = sigma f(T~) e1 - log(sigma) T e1, T e1 = sigma T~ e1
    const double ls = log(sigma);
    r0 = lane < ke ? sigma * (f0 - ls * te0) : 0.0;
    r1 = lane + 64 < ke ? sigma * (f1 - ls * te1) : 0.0;
    return true;
}

// One column per 64-thread block: the integral route, or the QR route when
// T~ has a negative eigenvalue beyond the allowed shift.
__global__ void __launch_bounds__(64) k_fT_e1(const double *alpha, const double *beta, const int32_t *k_eff,
                                              int32_t k, int32_t m, double *S, Rot *rot_buf, int32_t *flags,
                                              int32_t shift_max) {
    __shared__ double piv[kMaxSteps * 64];
    const int c = blockIdx.x;
    const int lane = threadIdx.x;
    if (c >= m) return;
    const int ke = __builtin_amdgcn_readfirstlane(k_eff[c]);
    // S is stored step-major: S[r * m + c]
    if (lane < k) S[(int64_t)lane * m + c] = 0.0;
    if (lane + 64 < k) S[(int64_t)(lane + 64) * m + c] = 0.0;
    if (ke <= 0) return;
    LaneTri t;
    load_tri(t, alpha + (int64_t)c * k, beta + (int64_t)c * k, ke, lane);
    double w0 = 0.0, w1 = 0.0;
    int st = 0;
    const bool done = ke <= 64 ? fT_e1_integral<1>(t, ke, lane, shift_max, piv, w0, w1)
                               : fT_e1_integral<2>(t, ke, lane, shift_max, piv, w0, w1);
    if (!done) {
        const int cap = (int)rot_capacity(k);
        Rot *rot = rot_buf + (int64_t)c * cap;
        st = ke <= 64 ? fT_e1_qr<1>(t, ke, lane, rot, cap, w0, w1) : fT_e1_qr<2>(t, ke, lane, rot, cap, w0, w1);
    }
    if (lane < ke) S[(int64_t)lane * m + c] = w0;
    if (lane + 64 < ke) S[(int64_t)(lane + 64) * m + c] = w1;
    if (lane == 0 && st) atomicOr(flags, st);
}

hipError_t launch_fT_e1(const double *alpha, const double *beta, const int32_t *k_eff, int32_t k, int32_t m,
                        double *S, void *rot_scratch, int32_t *flags, hipStream_t s, bool fp64) {
    if (k > kMaxSteps) return hipErrorInvalidValue;
    if (m > 0)
        hipLaunchKernelGGL(k_fT_e1, dim3(m), dim3(64), 0, s, alpha, beta, k_eff, k, m, S, (Rot *)rot_scratch, flags,
                           fp64 ? 1 : 4);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// estimator combine (one block, fixed order)
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_combine(const double *psi, int32_t m, int32_t kind,
                                                 int32_t n_sketch, double *estimate) {
    __shared__ double sh[256];
    double a = 0.0, b = 0.0;
    for (int c = threadIdx.x; c < m; c += 256) {
        if (kind == 2 && c < n_sketch) a += psi[c];
        else b += psi[c];
    }
    a = block_sum_256(a, sh);
    b = block_sum_256(b, sh);
    if (threadIdx.x == 0) {
        if (kind == 0) *estimate = b / (double)m;
        else if (kind == 1) *estimate = b;
        else *estimate = a + (m > n_sketch ? b / (double)(m - n_sketch) : 0.0);
    }
}

__global__ void __launch_bounds__(256) k_combine_graphs(const double *psi, int32_t ld, const int32_t *graph_m,
                                                        int32_t kind, double *estimates) {
    __shared__ double sh[256];
    const int g = blockIdx.x;
    const int mg = graph_m[g];
    double b = 0.0;
    for (int c = threadIdx.x; c < mg; c += 256) b += psi[(int64_t)g * ld + c];
    b = block_sum_256(b, sh);
    if (threadIdx.x == 0) estimates[g] = kind == 1 ? b : (mg > 0 ? b / (double)mg : 0.0);
}

hipError_t launch_combine_graphs(const double *psi, int32_t ld, const int32_t *graph_m, int32_t n_graphs,
                                 int32_t kind, double *estimates, hipStream_t s) {
    hipLaunchKernelGGL(k_combine_graphs, dim3(n_graphs), dim3(256), 0, s, psi, ld, graph_m, kind, estimates);
    return hipGetLastError();
}

hipError_t launch_combine(const double *psi, int32_t m, int32_t kind, int32_t n_sketch, double *estimate,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_combine, dim3(1), dim3(256), 0, s, psi, m, kind, n_sketch, estimate);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Hutch++ pieces
// ---------------------------------------------------------------------------

// Y[i, c] = ||c_c|| sum_j S[j, c] v_j[i, c] (eq. (4.3)).  Thread layout: CPL
// consecutive columns of RPT rows; a block covers 256 / (m_pad / CPL) * RPT
// rows and streams the stored basis (read once: non-temporal) a few steps at
// a time.
template <typename T, int CPL>
__global__ void __launch_bounds__(256) k_reconstruct(const T *V, int64_t stride, int32_t ldv,
                                                     const double *S, const double *norm2,
                                                     int32_t k, int32_t n, int32_t m, T *Y, int32_t ldy) {
    constexpr int RPT = VNE_RECON_RPT, UJ = VNE_RECON_UJ;
    const int groups = (m + CPL - 1) / CPL;            // column groups per row
    const int rows_per_pass = 256 / groups;
    if ((int)threadIdx.x >= rows_per_pass * groups) return;
    const int cg = threadIdx.x % groups, ro = threadIdx.x / groups;
    const int c0 = cg * CPL;
    const int64_t rbase = (int64_t)blockIdx.x * rows_per_pass * RPT + ro;
    double acc[RPT][CPL];
    bool ok[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        ok[q] = rbase + (int64_t)q * rows_per_pass < n;
#pragma unroll
        for (int u = 0; u < CPL; ++u) acc[q][u] = 0.0;
    }
    for (int j = 0; j < k; j += UJ) {
        T vb[UJ][RPT][CPL];
        double sb[UJ][CPL];
#pragma unroll
        for (int t = 0; t < UJ; ++t) {
            const bool jok = j + t < k;
#pragma unroll
            for (int u = 0; u < CPL; ++u) sb[t][u] = (jok && c0 + u < m) ? S[(int64_t)(j + t) * m + c0 + u] : 0.0;
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int64_t r = rbase + (int64_t)q * rows_per_pass;
                if (jok && ok[q]) load_vec_nt<T, CPL>(V + (int64_t)(j + t) * stride + r * ldv + c0, vb[t][q]);
                else
#pragma unroll
                    for (int u = 0; u < CPL; ++u) vb[t][q][u] = (T)0;
            }
        }
#pragma unroll
        for (int t = 0; t < UJ; ++t)
#pragma unroll
            for (int q = 0; q < RPT; ++q)
#pragma unroll
                for (int u = 0; u < CPL; ++u) acc[q][u] = fma(sb[t][u], (double)vb[t][q][u], acc[q][u]);
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        if (!ok[q]) continue;
        const int64_t r = rbase + (int64_t)q * rows_per_pass;
#pragma unroll
        for (int u = 0; u < CPL; ++u)
            if (c0 + u < m) Y[r * ldy + c0 + u] = (T)(sqrt(norm2[c0 + u]) * acc[q][u]);
    }
}

hipError_t launch_reconstruct(const void *Vstore, bool fp64, int64_t step_stride, int32_t ldv,
                              const double *S, const double *norm2, int32_t k, int32_t n, int32_t m,
                              void *Y, int32_t ldy, hipStream_t s) {
    // ldv (the sketch plan's padded width) is a multiple of the vector width
    const int cpl = fp64 ? 2 : 4;
    const int groups = (m + cpl - 1) / cpl;
    if (groups > 256 || ldv % cpl) return hipErrorInvalidValue;
    const int rows_per_block = (256 / groups) * VNE_RECON_RPT;
    dim3 g((unsigned)((n + rows_per_block - 1) / rows_per_block));
    if (fp64)
        hipLaunchKernelGGL((k_reconstruct<double, 2>), g, dim3(256), 0, s, (const double *)Vstore, step_stride,
                           ldv, S, norm2, k, n, m, (double *)Y, ldy);
    else
        hipLaunchKernelGGL((k_reconstruct<float, 4>), g, dim3(256), 0, s, (const float *)Vstore, step_stride, ldv,
                           S, norm2, k, n, m, (float *)Y, ldy);
    return hipGetLastError();
}

// Gram X^T Y (na, nb <= 128): a block computes the whole na x nb product over
// a chunk of rows; each thread owns an 8 x 8 sub-tile; 32 rows at a time are
// staged through LDS in FP64.  Products of FP32 inputs are exact in FP64;
// accumulation is FP64; the chunk partials are added in chunk order.
constexpr int kGramRows = 512;   // rows per chunk

int64_t gram_scratch_doubles(int32_t n, int32_t na, int32_t nb) {
    const int64_t chunks = (n + kGramRows - 1) / kGramRows;
    return chunks * (int64_t)na * nb;
}

template <typename T>
__global__ void __launch_bounds__(256) k_gram(const T *X, int32_t ldx, const T *Y, int32_t ldy, int32_t n,
                                              int32_t na, int32_t nb, double *part, int64_t part_stride,
                                              int32_t ldo) {
    constexpr int RS = 32;
    __shared__ double xs[RS][128];
    __shared__ double ys[RS][128];
    const int chunk = blockIdx.x;
    const int64_t r0 = (int64_t)chunk * kGramRows;
    const int64_t r1 = min((int64_t)n, r0 + kGramRows);
    // thread (ta, tb) owns rows ta + 16 u and columns tb + 16 v of the output:
    // the 16 threads of a quarter-wave read 16 consecutive doubles of a staged
    // row (no LDS bank conflicts), the 4 quarter-waves read 4 broadcast rows
    const int ta = threadIdx.x / 16, tb = threadIdx.x % 16;
    double acc[8][8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int v = 0; v < 8; ++v) acc[u][v] = 0.0;
    // staging: thread t moves column t % 128 of rows t / 128 + 2 i; the next
    // round's values are loaded into registers while this round computes
    constexpr int PER = RS * 128 / 256;
    const int scol = threadIdx.x % 128, srow = threadIdx.x / 128;
    T xr[PER], yr[PER];
    auto fetch = [&](int64_t rs) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int64_t r = rs + srow + 2 * i;
            xr[i] = (r < r1 && scol < na) ? X[r * ldx + scol] : (T)0;
            yr[i] = (r < r1 && scol < nb) ? Y[r * ldy + scol] : (T)0;
        }
    };
    fetch(r0);
    for (int64_t rs = r0; rs < r1; rs += RS) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            xs[srow + 2 * i][scol] = (double)xr[i];
            ys[srow + 2 * i][scol] = (double)yr[i];
        }
        __syncthreads();
        if (rs + RS < r1) fetch(rs + RS);
        for (int rr = 0; rr < RS; ++rr) {
            double xa[8], yb[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                xa[u] = xs[rr][ta + 16 * u];
                yb[u] = ys[rr][tb + 16 * u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int v = 0; v < 8; ++v) acc[u][v] = fma(xa[u], yb[v], acc[u][v]);
        }
        __syncthreads();
    }
    double *out = part + (int64_t)chunk * part_stride;
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int a = ta + 16 * u, b = tb + 16 * v;
            if (a < na && b < nb) out[(int64_t)a * ldo + b] = acc[u][v];
        }
}

__global__ void __launch_bounds__(256) k_gram_reduce(const double *part, int64_t chunks, int64_t total,
                                                     double *out) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= total) return;
    // chunk partials in order, in batches whose loads are issued before the adds
    constexpr int UB = 16;
    double s = 0.0;
    int64_t q = 0;
    for (; q + UB <= chunks; q += UB) {
        double v[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) v[u] = part[(q + u) * total + t];
#pragma unroll
        for (int u = 0; u < UB; ++u) s += v[u];
    }
    for (; q < chunks; ++q) s += part[q * total + t];
    out[t] = s;
}

hipError_t launch_gram(const void *X, int32_t ldx, const void *Y, int32_t ldy, bool fp64, int32_t n,
                       int32_t na, int32_t nb, double *part, double *out, hipStream_t s) {
    if (na > 128) return hipErrorInvalidValue;
    const int64_t chunks = (n + kGramRows - 1) / kGramRows;
    const int64_t total = (int64_t)na * nb;
    dim3 g((unsigned)chunks);
    // 128-column slices of Y, each writing its columns of the [na][nb] partials
    for (int b = 0; b < nb; b += 128) {
        const int w = min(128, nb - b);
        if (fp64)
            hipLaunchKernelGGL(k_gram<double>, g, dim3(256), 0, s, (const double *)X, ldx, (const double *)Y + b,
                               ldy, n, na, w, part + b, total, nb);
        else
            hipLaunchKernelGGL(k_gram<float>, g, dim3(256), 0, s, (const float *)X, ldx, (const float *)Y + b,
                               ldy, n, na, w, part + b, total, nb);
    }
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, part, chunks,
                       total, out);
    return hipGetLastError();
}

// Upper Cholesky G = R^T R (na <= 128), one block, G staged in LDS (128 KB
// of the 160 KB of a gfx950 CU); R overwrites G's upper triangle in memory.
// A pivot that is not positive sets flags bit 1 (and is replaced by 1).
__global__ void __launch_bounds__(256) k_chol(double *G_io, int32_t na, int32_t *flags) {
    __shared__ double G[128 * 128];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    for (int t = threadIdx.x; t < na * na; t += 256) G[t] = G_io[t];
    __syncthreads();
    for (int j = 0; j < na; ++j) {
        if (threadIdx.x == 0) {
            const double djj = G[j * na + j];
            if (!(djj > 0.0)) bad = 1;
            G[j * na + j] = djj > 0.0 ? sqrt(djj) : 1.0;
        }
        __syncthreads();
        const double rjj = G[j * na + j];
        for (int q = j + 1 + threadIdx.x; q < na; q += 256) G[j * na + q] /= rjj;
        __syncthreads();
        // trailing update of the upper triangle, 16 x 16 threads
        const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
        for (int p = j + 1 + ty; p < na; p += 16) {
            const double gjp = G[j * na + p];
            for (int q = p + tx; q < na; q += 16) G[p * na + q] -= gjp * G[j * na + q];
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < na * na; t += 256) G_io[t] = G[t];
    if (threadIdx.x == 0 && bad) atomicOr(flags, 2);
}

// R^{-1} (upper) of the upper triangle of R, one wavefront per column: column
// col solves x_col = 1 / R[col][col], then for p = col - 1 .. 0
// x_p = -(sum_{q = p+1 .. col} R[p][q] x_q) / R[p][p], the sum formed across
// the lanes (lane q holds x_q; fixed-order butterfly).
__global__ void __launch_bounds__(256) k_trinv(const double *R_in, double *Rinv, int32_t na) {
    __shared__ double R[128 * 128];
    for (int t = threadIdx.x; t < na * na; t += 256) R[t] = R_in[t];
    __syncthreads();
    const int col = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (col >= na) return;
    const double xc = 1.0 / R[col * na + col];
    double x0 = lane == col ? xc : 0.0;
    double x1 = lane + 64 == col ? xc : 0.0;
    for (int p = col - 1; p >= 0; --p) {
        double part = 0.0;
        if (lane > p && lane <= col) part = R[p * na + lane] * x0;
        if (lane + 64 > p && lane + 64 <= col) part = fma(R[p * na + lane + 64], x1, part);
        const double xp = -wave_sum(part) / R[p * na + p];
        x0 = lane == p ? xp : x0;
        x1 = lane + 64 == p ? xp : x1;
    }
    for (int p = lane; p < na; p += 64) {
        const double v = p < 64 ? x0 : x1;
        Rinv[(int64_t)p * na + col] = p <= col ? v : 0.0;
    }
}

hipError_t launch_cholinv(double *G, double *Rinv, int32_t na, int32_t *flags, hipStream_t s) {
    if (na > 128) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_chol, dim3(1), dim3(256), 0, s, G, na, flags);
    hipLaunchKernelGGL(k_trinv, dim3((na + 3) / 4), dim3(256), 0, s, G, Rinv, na);
    return hipGetLastError();
}

// Z = (sub ? Z - X M : X M) (na, nb <= 128), row-local: a block owns 128
// rows; each thread owns an 8 x 8 sub-tile (8 rows, 8 columns); the inner
// dimension is staged through LDS 32 at a time (X transposed, FP64).  Every
// row of X a block reads is read before the block writes Z, so Z may alias
// X (sub == 0) or hold other columns of the same rows (sub == 1).
template <typename T>
__global__ void __launch_bounds__(256) k_apply(const T *X, int32_t ldx, const double *M, int32_t ldm, int32_t na,
                                               int32_t nb, T *Z, int32_t ldz, int32_t n, int32_t sub) {
    constexpr int TS = 32;
    __shared__ double xt[128][TS + 1];   // xt[row][t]; the pad spreads the rows over the banks
    __shared__ double ms[TS][128];       // ms[t][col]
    const int64_t r0 = (int64_t)blockIdx.x * 128;
    // thread (i0, tb) owns rows i0 .. i0 + 7 and columns tb + 16 v: the 16
    // threads of a quarter-wave read 16 consecutive doubles of a row of ms
    const int i0 = (threadIdx.x / 16) * 8, tb = threadIdx.x % 16;
    double acc[8][8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int v = 0; v < 8; ++v) acc[u][v] = 0.0;
    // staging: thread t moves X[r0 + t / TS + 8 i][t0 + t % TS] (consecutive
    // threads read consecutive inner indices) and M[t0 + t / 128 + 2 i][t % 128];
    // the next step's values are loaded into registers while this one computes
    constexpr int PER = TS * 128 / 256;
    const int xc = threadIdx.x % TS, xr0 = threadIdx.x / TS;
    const int mc = threadIdx.x % 128, mr0 = threadIdx.x / 128;
    T xv[PER];
    double mv[PER];
    auto fetch = [&](int t0) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int64_t r = r0 + xr0 + 8 * i;
            xv[i] = (r < n && t0 + xc < na) ? X[r * ldx + t0 + xc] : (T)0;
            const int mt = t0 + mr0 + 2 * i;
            mv[i] = (mt < na && mc < nb) ? M[(int64_t)mt * ldm + mc] : 0.0;
        }
    };
    fetch(0);
    for (int t0 = 0; t0 < na; t0 += TS) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            xt[xr0 + 8 * i][xc] = (double)xv[i];
            ms[mr0 + 2 * i][mc] = mv[i];
        }
        __syncthreads();
        if (t0 + TS < na) fetch(t0 + TS);
        for (int tt = 0; tt < TS; ++tt) {
            double xa[8], mb[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                xa[u] = xt[i0 + u][tt];
                mb[u] = ms[tt][tb + 16 * u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int v = 0; v < 8; ++v) acc[u][v] = fma(xa[u], mb[v], acc[u][v]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int64_t r = r0 + i0 + u;
        if (r >= n) continue;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int cc = tb + 16 * v;
            if (cc >= nb) continue;
            if (sub) Z[r * ldz + cc] = (T)((double)Z[r * ldz + cc] - acc[u][v]);
            else Z[r * ldz + cc] = (T)acc[u][v];
        }
    }
}

hipError_t launch_apply(const void *X, int32_t ldx, const double *M, int32_t na, int32_t nb, void *Z,
                        int32_t ldz, bool fp64, int32_t n, int32_t sub, hipStream_t s) {
    if (na > 128) return hipErrorInvalidValue;
    // Z aliasing X (sub == 0) needs one pass over all columns
    if (sub == 0 && nb > 128) return hipErrorInvalidValue;
    dim3 g((unsigned)((n + 127) / 128));
    for (int b = 0; b < nb; b += 128) {
        const int w = min(128, nb - b);
        if (fp64)
            hipLaunchKernelGGL(k_apply<double>, g, dim3(256), 0, s, (const double *)X, ldx, M + b, nb, na, w,
                               (double *)Z + b, ldz, n, sub);
        else
            hipLaunchKernelGGL(k_apply<float>, g, dim3(256), 0, s, (const float *)X, ldx, M + b, nb, na, w,
                               (float *)Z + b, ldz, n, sub);
    }
    return hipGetLastError();
}

}  // namespace vne
