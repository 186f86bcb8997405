// gfx950 kernels of the Lanczos-quadrature entropy engine.
//
// Layout: probe blocks are n x m_pad row-major (probe index fastest), so the
// SpMM gathers one contiguous m-vector per stored entry.  Lanczos vectors are
// FP32 (FP64 in FP64 mode); every dot product, the alpha/beta coefficients
// and the quadrature are FP64.  Reductions are two-stage with a fixed
// summation order (no floating-point atomics), so results are bitwise
// reproducible for a given launch shape.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

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
// ---------------------------------------------------------------------------

template <typename T, int CPL, int LPR, bool FIRST>
__global__ void __launch_bounds__(256) k_lanczos_step(StepArgs a) {
    constexpr int MT = CPL * LPR;
    constexpr int GPW = 64 / LPR;        // lane groups per wave
    constexpr int NG = 4 * GPW;          // lane groups per block
    constexpr int U = (CPL == 4) ? 4 : 4;
    __shared__ double red[3][NG * MT];

    const int nb_total = gridDim.x * gridDim.y;
    const int lin = xcd_remap(blockIdx.y * gridDim.x + blockIdx.x, nb_total);
    const int tile = lin / a.n_blocks;
    const int b = lin % a.n_blocks;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int grp = lane / LPR;
    const int gl = lane % LPR;
    const int gid = wave * GPW + grp;
    const int c0 = tile * MT + gl * CPL;
    const int64_t ld = a.m_pad;

    const T *P_in = static_cast<const T *>(a.P_in);
    const T *V_prev = static_cast<const T *>(a.V_prev);
    T *V_out = static_cast<T *>(a.V_out);
    T *P_out = static_cast<T *>(a.P_out);
    const T *val = static_cast<const T *>(a.val);

    T al[CPL], inv[CPL];
    double coup[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        al[k] = (T)a.st_alpha[c0 + k];
        inv[k] = (T)a.st_inv[c0 + k];
        coup[k] = a.st_coup[c0 + k];
    }
    double s_vw[CPL], s_ww[CPL], s_vv[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) s_vw[k] = s_ww[k] = s_vv[k] = 0.0;

    // one row (or row segment): acc = sum_p val[p] * v_j[col[p], cols]
    auto gather = [&](int p0, int p1, double (&acc)[CPL]) {
#pragma unroll
        for (int k = 0; k < CPL; ++k) acc[k] = 0.0;
        int p = p0;
        for (; p + U <= p1; p += U) {
            int jj[U];
            T vv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                jj[u] = a.col[p + u];
                vv[u] = val[p + u];
            }
            T pv[U][CPL], qv[U][CPL];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                load_vec<T, CPL>(P_in + (int64_t)jj[u] * ld + c0, pv[u]);
                if (!FIRST) load_vec<T, CPL>(V_prev + (int64_t)jj[u] * ld + c0, qv[u]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int k = 0; k < CPL; ++k) {
                    T v = materialize(pv[u][k], FIRST ? (T)0 : qv[u][k], al[k], inv[k]);
                    acc[k] = fma((double)vv[u], (double)v, acc[k]);
                }
            }
        }
        for (; p < p1; ++p) {
            const int j = a.col[p];
            const T vv = val[p];
            T pv[CPL], qv[CPL];
            load_vec<T, CPL>(P_in + (int64_t)j * ld + c0, pv);
            if (!FIRST) load_vec<T, CPL>(V_prev + (int64_t)j * ld + c0, qv);
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                T v = materialize(pv[k], FIRST ? (T)0 : qv[k], al[k], inv[k]);
                acc[k] = fma((double)vv, (double)v, acc[k]);
            }
        }
    };

    // finish a row: w = scale*acc - beta_{j-1} v_{j-1}; store P_{j+1}, v_j;
    // return the row's contributions to v.w, w.w, v.v
    auto finish = [&](int row, const double (&acc)[CPL], double (&dvw)[CPL], double (&dww)[CPL],
                      double (&dvv)[CPL]) {
        T pv[CPL], qv[CPL], v[CPL], wr[CPL];
        load_vec<T, CPL>(P_in + (int64_t)row * ld + c0, pv);
        if (!FIRST) load_vec<T, CPL>(V_prev + (int64_t)row * ld + c0, qv);
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            const T q = FIRST ? (T)0 : qv[k];
            v[k] = materialize(pv[k], q, al[k], inv[k]);
            const double w = fma(-coup[k], (double)q, a.scale * acc[k]);
            wr[k] = (T)w;
            const double vd = (double)v[k], wd = (double)wr[k];
            dvw[k] = vd * wd;
            dww[k] = wd * wd;
            dvv[k] = vd * vd;
        }
        store_vec<T, CPL>(P_out + (int64_t)row * ld + c0, wr);
        store_vec<T, CPL>(V_out + (int64_t)row * ld + c0, v);
    };

    const int ib = a.block_begin[b], ie = a.block_begin[b + 1];
    for (int it = ib + gid; it < ie; it += NG) {
        int row, p0, p1, lrow = -1;
        if (it < a.n_seg) {
            const SegItem s = a.segs[it];
            row = s.row;
            p0 = s.p0;
            p1 = s.p1;
            lrow = s.lrow;
        } else {
            row = it - a.n_seg;
            p0 = a.row_ptr[row];
            p1 = a.row_ptr[row + 1];
            if (p1 - p0 > a.seg_len) continue;
        }
        if (LPR == 64) {
            row = __builtin_amdgcn_readfirstlane(row);
            p0 = __builtin_amdgcn_readfirstlane(p0);
            p1 = __builtin_amdgcn_readfirstlane(p1);
            lrow = __builtin_amdgcn_readfirstlane(lrow);
        }
        double acc[CPL];
        gather(p0, p1, acc);
        if (lrow < 0) {
            double dvw[CPL], dww[CPL], dvv[CPL];
            finish(row, acc, dvw, dww, dvv);
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                s_vw[k] += dvw[k];
                s_ww[k] += dww[k];
                s_vv[k] += dvv[k];
            }
        } else {
            // long row: publish this segment's partial product; the last
            // segment to arrive adds all segments in order and finishes the row
            double *dst = a.seg_acc + (int64_t)it * ld + c0;
#pragma unroll
            for (int k = 0; k < CPL; ++k) dst[k] = acc[k];
            __threadfence();
            int old = 0;
            if (gl == 0) old = atomicAdd(&a.tickets[lrow * a.n_tiles + tile], 1);
            old = __shfl(old, grp * LPR, 64);
            const int nseg = a.long_nseg[lrow];
            if (old == nseg - 1) {
                __threadfence();
                const int first = a.long_first[lrow];
                double tot[CPL];
#pragma unroll
                for (int k = 0; k < CPL; ++k) tot[k] = 0.0;
                for (int sgi = 0; sgi < nseg; ++sgi) {
                    const volatile double *src = a.seg_acc + (int64_t)(first + sgi) * ld + c0;
#pragma unroll
                    for (int k = 0; k < CPL; ++k) tot[k] += src[k];
                }
                double dvw[CPL], dww[CPL], dvv[CPL];
                finish(row, tot, dvw, dww, dvv);
                double *lp = a.long_part + (int64_t)lrow * 3 * ld + c0;
#pragma unroll
                for (int k = 0; k < CPL; ++k) {
                    lp[k] = dvw[k];
                    lp[ld + k] = dww[k];
                    lp[2 * ld + k] = dvv[k];
                }
                if (gl == 0) a.tickets[lrow * a.n_tiles + tile] = 0;
            }
        }
    }

    // block reduction over the lane groups that share columns (fixed order)
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        red[0][gid * MT + gl * CPL + k] = s_vw[k];
        red[1][gid * MT + gl * CPL + k] = s_ww[k];
        red[2][gid * MT + gl * CPL + k] = s_vv[k];
    }
    __syncthreads();
    double *out = a.partials + ((int64_t)tile * a.n_blocks + b) * 3 * MT;
    for (int t = threadIdx.x; t < 3 * MT; t += 256) {
        const int sidx = t / MT, cc = t % MT;
        double sum = 0.0;
#pragma unroll 4
        for (int g = 0; g < NG; ++g) sum += red[sidx][g * MT + cc];
        out[t] = sum;
    }
}

int choose_tile(int m, bool fp64, int requested) {
    const int cpl = fp64 ? 2 : 4;
    const int maxt = cpl * 64, mint = cpl * 4;
    if (requested > 0) {
        int t = mint;
        while (t < requested && t < maxt) t *= 2;
        return t;
    }
    int t = mint;
    while (t < m && t < maxt) t *= 2;
    return t;
}

int pad_columns(int m, int mt) { return ((m + mt - 1) / mt) * mt; }

template <typename T, int CPL, int LPR>
static hipError_t launch_step_t(const StepArgs &a, bool first, hipStream_t s) {
    dim3 grid(a.n_blocks, a.n_tiles);
    if (first)
        hipLaunchKernelGGL((k_lanczos_step<T, CPL, LPR, true>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_lanczos_step<T, CPL, LPR, false>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_step(const StepArgs &a, bool fp64, bool first, hipStream_t s) {
    if (!fp64) {
        switch (a.mt) {
            case 16: return launch_step_t<float, 4, 4>(a, first, s);
            case 32: return launch_step_t<float, 4, 8>(a, first, s);
            case 64: return launch_step_t<float, 4, 16>(a, first, s);
            case 128: return launch_step_t<float, 4, 32>(a, first, s);
            case 256: return launch_step_t<float, 4, 64>(a, first, s);
        }
    } else {
        switch (a.mt) {
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

__global__ void __launch_bounds__(256) k_finalize(FinalizeArgs a) {
    __shared__ double sh[256];
    const int c = blockIdx.x;
    const int tile = c / a.mt, cc = c % a.mt;
    double s3[3] = {0.0, 0.0, 0.0};
    for (int bb = threadIdx.x; bb < a.n_blocks; bb += 256) {
        const double *p = a.partials + ((int64_t)tile * a.n_blocks + bb) * 3 * a.mt + cc;
        s3[0] += p[0];
        s3[1] += p[a.mt];
        s3[2] += p[2 * a.mt];
    }
    for (int L = threadIdx.x; L < a.n_long; L += 256) {
        const double *p = a.long_part + (int64_t)L * 3 * a.m_pad + c;
        s3[0] += p[0];
        s3[1] += p[a.m_pad];
        s3[2] += p[2 * a.m_pad];
    }
    const double svw = block_sum_256(s3[0], sh);
    const double sww = block_sum_256(s3[1], sh);
    const double svv = block_sum_256(s3[2], sh);
    if (threadIdx.x != 0) return;
    const int j = a.step - 1;
    const double inv_prev = a.st_inv[c];
    if (inv_prev == 0.0 || c >= a.m) {      // frozen earlier, empty or pad column
        a.alpha[(int64_t)c * a.k + j] = 0.0;
        a.beta[(int64_t)c * a.k + j] = 0.0;
        a.st_inv[c] = 0.0;
        a.st_alpha[c] = 0.0;
        a.st_coup[c] = 0.0;
        return;
    }
    const double coup_prev = a.st_coup[c];
    const double alpha = svw / svv;
    double b2 = sww - alpha * svw;
    b2 = b2 > 0.0 ? b2 : 0.0;
    const double beta = sqrt(b2);
    a.alpha[(int64_t)c * a.k + j] = alpha;
    const bool finite = isfinite(alpha) && isfinite(beta);
    if (!finite) atomicOr(a.flags, 1);
    if (!finite || beta <= a.tau * (fabs(alpha) + coup_prev)) {
        a.k_eff[c] = a.step;
        a.beta[(int64_t)c * a.k + j] = 0.0;
        a.st_inv[c] = 0.0;
        a.st_alpha[c] = 0.0;
        a.st_coup[c] = 0.0;
    } else {
        a.beta[(int64_t)c * a.k + j] = beta;
        a.st_alpha[c] = alpha;
        a.st_inv[c] = 1.0 / beta;
        a.st_coup[c] = beta;
    }
}

hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(a.m_pad), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Probe block.  Thread layout: columns of one tile fastest, 256 / mt rows per
// pass.  Pass 1 sums every column (for the centring of Remark 4.6), pass 2
// writes P_1 = c (element type of the mode) and sums c^2 of the stored values.
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ double probe_value(const ProbeArgs &a, int64_t i, int c) {
    if (c >= a.m) return 0.0;
    if (a.gen == GEN_RADEMACHER) return rademacher(a.seed, a.keys[i], (int64_t)a.col_offset + c);
    if (a.gen == GEN_COLORING) return a.colors[i] == c ? 1.0 : 0.0;
    return (double)static_cast<const T *>(a.dense)[i * a.ld_dense + c];
}

template <typename T, int PASS>
__global__ void __launch_bounds__(256) k_probe(ProbeArgs a) {
    __shared__ double sh[256];
    const int rows_per = 256 / a.mt;
    const int cc = threadIdx.x % a.mt, rr = threadIdx.x / a.mt;
    const int64_t per_block = ((int64_t)a.n + a.n_blocks - 1) / a.n_blocks;
    const int64_t r0 = (int64_t)blockIdx.x * per_block;
    const int64_t r1 = min((int64_t)a.n, r0 + per_block);
    T *P = static_cast<T *>(a.P_out);
    for (int t0 = 0; t0 < a.m_pad; t0 += a.mt) {
        const int c = t0 + cc;
        double acc = 0.0;
        const double mu = PASS == 2 ? a.mean[c] : 0.0;
        for (int64_t i = r0 + rr; i < r1; i += rows_per) {
            const double b = probe_value<T>(a, i, c);
            if (PASS == 1) {
                acc += b;
            } else {
                const T cv = (T)(b - mu);
                P[i * a.m_pad + c] = cv;
                acc += (double)cv * (double)cv;
            }
        }
        // fixed-order sum over the rows_per threads of this column
        sh[threadIdx.x] = acc;
        __syncthreads();
        if (rr == 0) {
            double s = 0.0;
            for (int q = 0; q < rows_per; ++q) s += sh[q * a.mt + cc];
            a.partials[(int64_t)blockIdx.x * a.m_pad + c] = s;
        }
        __syncthreads();
    }
}

template <int PASS>
__global__ void __launch_bounds__(256) k_probe_reduce(ProbeArgs a) {
    __shared__ double sh[256];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int bb = threadIdx.x; bb < a.n_blocks; bb += 256) s += a.partials[(int64_t)bb * a.m_pad + c];
    s = block_sum_256(s, sh);
    if (threadIdx.x != 0) return;
    if (PASS == 1) {
        a.mean[c] = a.desing ? s / (double)a.n : 0.0;
    } else {
        a.norm2[c] = s;
        a.st_alpha[c] = 0.0;
        a.st_coup[c] = 0.0;
        if (s > 0.0 && c < a.m) {
            a.st_inv[c] = 1.0 / sqrt(s);
            a.k_eff[c] = a.k;
        } else {
            a.st_inv[c] = 0.0;
            a.k_eff[c] = 0;
        }
    }
}

hipError_t launch_probe(const ProbeArgs &a, bool fp64, hipStream_t s) {
    dim3 g(a.n_blocks), r(a.m_pad);
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
// Symmetric tridiagonal eigenproblem by implicit QR steps with Wilkinson
// shifts (Golub & Van Loan, implicit symmetric QR step), tracking selected
// rows of the eigenvector matrix Z (T = Z diag(d) Z^T).  d: diagonal, e:
// off-diagonal (e[i] couples i and i+1).  NR rows of Z are tracked, row
// indices rows[0..NR); z[r][*] starts as the unit row e_{rows[r]}^T.
// Returns false if an eigenvalue needed more than 60 sweeps.
// ---------------------------------------------------------------------------

template <int NR>
__device__ bool tridiag_qr(double *d, double *e, int n, double (*z)[kMaxSteps]) {
    const double eps = 1.1102230246251565e-16;   // 2^-53
    int hi = n - 1;
    int sweeps = 0;
    while (hi > 0) {
        if (fabs(e[hi - 1]) <= eps * (fabs(d[hi - 1]) + fabs(d[hi]))) {
            e[hi - 1] = 0.0;
            --hi;
            sweeps = 0;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && fabs(e[lo - 1]) > eps * (fabs(d[lo - 1]) + fabs(d[lo]))) --lo;
        if (lo > 0) e[lo - 1] = 0.0;
        if (++sweeps > 60) return false;
        // Wilkinson shift from the trailing 2x2 block
        const double dl = 0.5 * (d[hi - 1] - d[hi]);
        const double bh = e[hi - 1];
        const double den = dl + copysign(hypot(dl, bh), dl == 0.0 ? 1.0 : dl);
        const double mu = d[hi] - bh * (bh / den);
        double x = d[lo] - mu, y = e[lo];
        for (int i = lo; i < hi; ++i) {
            const double r = hypot(x, y);
            const double c = r == 0.0 ? 1.0 : x / r;
            const double s = r == 0.0 ? 0.0 : y / r;
            if (i > lo) e[i - 1] = r;
            const double ai = d[i], aj = d[i + 1], bb = e[i];
            const double cs = c * s, cc = c * c, ss = s * s;
            d[i] = cc * ai + 2.0 * cs * bb + ss * aj;
            d[i + 1] = ss * ai - 2.0 * cs * bb + cc * aj;
            e[i] = cs * (aj - ai) + (cc - ss) * bb;
            if (i + 1 < hi) {
                y = s * e[i + 1];
                e[i + 1] = c * e[i + 1];
                x = e[i];
            }
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                const double zi = z[q][i], zj = z[q][i + 1];
                z[q][i] = c * zi + s * zj;
                z[q][i + 1] = -s * zi + c * zj;
            }
        }
    }
    return true;
}

__global__ void __launch_bounds__(64) k_quadrature(const double *alpha, const double *beta,
                                                   const int32_t *k_eff, const double *norm2, int32_t k,
                                                   int32_t m, double *psi, int32_t *flags) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m) return;
    const int ke = k_eff[c];
    if (ke <= 0) {
        psi[c] = 0.0;
        return;
    }
    double d[kMaxSteps], e[kMaxSteps];
    double z[1][kMaxSteps];
    for (int i = 0; i < ke; ++i) {
        d[i] = alpha[(int64_t)c * k + i];
        e[i] = i + 1 < ke ? beta[(int64_t)c * k + i] : 0.0;
        z[0][i] = i == 0 ? 1.0 : 0.0;
    }
    if (!tridiag_qr<1>(d, e, ke, z)) atomicOr(flags, 4);
    double s = 0.0;
    for (int i = 0; i < ke; ++i) s += z[0][i] * z[0][i] * f_entropy(d[i]);
    psi[c] = norm2[c] * s;
}

hipError_t launch_quadrature(const double *alpha, const double *beta, const int32_t *k_eff,
                             const double *norm2, int32_t k, int32_t m, double *psi, int32_t *flags,
                             hipStream_t s) {
    if (k > kMaxSteps) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_quadrature, dim3((m + 63) / 64), dim3(64), 0, s, alpha, beta, k_eff, norm2, k, m,
                       psi, flags);
    return hipGetLastError();
}

// f(T) e1: one wave per column; lane l tracks rows 0, l and l + 64 of Z
// (every lane repeats the same QR on its own copy of d, e).
__global__ void __launch_bounds__(64) k_fT_e1(const double *alpha, const double *beta,
                                              const int32_t *k_eff, int32_t k, int32_t m, double *S,
                                              int32_t *flags) {
    const int c = blockIdx.x;
    const int l = threadIdx.x;
    const int ke = k_eff[c];
    double *out = S + (int64_t)c * k;
    for (int r = l; r < k; r += 64) out[r] = 0.0;
    if (ke <= 0) return;
    double d[kMaxSteps], e[kMaxSteps];
    double z[3][kMaxSteps];
    for (int i = 0; i < ke; ++i) {
        d[i] = alpha[(int64_t)c * k + i];
        e[i] = i + 1 < ke ? beta[(int64_t)c * k + i] : 0.0;
        z[0][i] = i == 0 ? 1.0 : 0.0;
        z[1][i] = i == l ? 1.0 : 0.0;
        z[2][i] = i == l + 64 ? 1.0 : 0.0;
    }
    if (!tridiag_qr<3>(d, e, ke, z) && l == 0) atomicOr(flags, 4);
    double s1 = 0.0, s2 = 0.0;
    for (int i = 0; i < ke; ++i) {
        const double w = f_entropy(d[i]) * z[0][i];
        s1 += z[1][i] * w;
        s2 += z[2][i] * w;
    }
    if (l < ke) out[l] = s1;
    if (l + 64 < ke) out[l + 64] = s2;
}

hipError_t launch_fT_e1(const double *alpha, const double *beta, const int32_t *k_eff, int32_t k,
                        int32_t m, double *S, int32_t *flags, hipStream_t s) {
    if (k > kMaxSteps) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fT_e1, dim3(m), dim3(64), 0, s, alpha, beta, k_eff, k, m, S, flags);
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

hipError_t launch_combine(const double *psi, int32_t m, int32_t kind, int32_t n_sketch, double *estimate,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_combine, dim3(1), dim3(256), 0, s, psi, m, kind, n_sketch, estimate);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Hutch++ pieces
// ---------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(256) k_reconstruct(const T *V, int64_t stride, int32_t ldv,
                                                     const double *S, const double *norm2,
                                                     const int32_t *k_eff, int32_t k, int32_t n,
                                                     int32_t m, T *Y, int32_t ldy) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)n * m) return;
    const int64_t i = t / m;
    const int c = (int)(t % m);
    const int ke = k_eff[c];
    double acc = 0.0;
    for (int j = 0; j < ke; ++j) acc = fma(S[(int64_t)c * k + j], (double)V[j * stride + i * ldv + c], acc);
    Y[i * ldy + c] = (T)(sqrt(norm2[c]) * acc);
}

hipError_t launch_reconstruct(const void *Vstore, bool fp64, int64_t step_stride, int32_t ldv,
                              const double *S, const double *norm2, const int32_t *k_eff, int32_t k,
                              int32_t n, int32_t m, void *Y, int32_t ldy, hipStream_t s) {
    const int64_t total = (int64_t)n * m;
    dim3 g((unsigned)((total + 255) / 256));
    if (fp64)
        hipLaunchKernelGGL(k_reconstruct<double>, g, dim3(256), 0, s, (const double *)Vstore, step_stride,
                           ldv, S, norm2, k_eff, k, n, m, (double *)Y, ldy);
    else
        hipLaunchKernelGGL(k_reconstruct<float>, g, dim3(256), 0, s, (const float *)Vstore, step_stride, ldv,
                           S, norm2, k_eff, k, n, m, (float *)Y, ldy);
    return hipGetLastError();
}

// Gram X^T Y: block (tile of 32 x 32 outputs, chunk of rows); each thread
// owns 4 outputs; rows are staged through LDS 64 at a time.
constexpr int kGramTile = 32;
constexpr int kGramChunk = 2048;

int64_t gram_scratch_doubles(int32_t n, int32_t na, int32_t nb) {
    const int64_t chunks = (n + kGramChunk - 1) / kGramChunk;
    return chunks * (int64_t)na * nb;
}

template <typename T>
__global__ void __launch_bounds__(256) k_gram(const T *X, int32_t ldx, const T *Y, int32_t ldy, int32_t n,
                                              int32_t na, int32_t nb, double *part) {
    __shared__ double xs[64][kGramTile + 1];
    __shared__ double ys[64][kGramTile + 1];
    const int ta = blockIdx.x * kGramTile, tb = blockIdx.y * kGramTile;
    const int chunk = blockIdx.z;
    const int64_t r0 = (int64_t)chunk * kGramChunk;
    const int64_t r1 = min((int64_t)n, r0 + kGramChunk);
    const int oa = threadIdx.x / 8;           // 0..31
    const int ob = (threadIdx.x % 8) * 4;     // 0..28
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t rs = r0; rs < r1; rs += 64) {
        for (int q = threadIdx.x; q < 64 * kGramTile; q += 256) {
            const int rr = q / kGramTile, cc = q % kGramTile;
            const int64_t r = rs + rr;
            xs[rr][cc] = (r < r1 && ta + cc < na) ? (double)X[r * ldx + ta + cc] : 0.0;
            ys[rr][cc] = (r < r1 && tb + cc < nb) ? (double)Y[r * ldy + tb + cc] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int rr = 0; rr < 64; ++rr) {
            const double xa = xs[rr][oa];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = fma(xa, ys[rr][ob + q], acc[q]);
        }
        __syncthreads();
    }
    double *out = part + (int64_t)chunk * na * nb;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (ta + oa < na && tb + ob + q < nb) out[(int64_t)(ta + oa) * nb + tb + ob + q] = acc[q];
}

__global__ void __launch_bounds__(256) k_gram_reduce(const double *part, int64_t chunks, int64_t total,
                                                     double *out) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= total) return;
    double s = 0.0;
    for (int64_t q = 0; q < chunks; ++q) s += part[q * total + t];
    out[t] = s;
}

hipError_t launch_gram(const void *X, int32_t ldx, const void *Y, int32_t ldy, bool fp64, int32_t n,
                       int32_t na, int32_t nb, double *part, double *out, hipStream_t s) {
    const int64_t chunks = (n + kGramChunk - 1) / kGramChunk;
    dim3 g((na + kGramTile - 1) / kGramTile, (nb + kGramTile - 1) / kGramTile, (unsigned)chunks);
    if (fp64)
        hipLaunchKernelGGL(k_gram<double>, g, dim3(256), 0, s, (const double *)X, ldx, (const double *)Y, ldy,
                           n, na, nb, part);
    else
        hipLaunchKernelGGL(k_gram<float>, g, dim3(256), 0, s, (const float *)X, ldx, (const float *)Y, ldy, n,
                           na, nb, part);
    const int64_t total = (int64_t)na * nb;
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, part, chunks,
                       total, out);
    return hipGetLastError();
}

// Upper Cholesky G = R^T R (in place, one block) and R^{-1} (upper).
__global__ void __launch_bounds__(256) k_cholinv(double *G, double *Rinv, int32_t na, int32_t *flags) {
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < na; ++j) {
        // R[j][j] and row j of R: G[j][q] for q >= j hold the trailing update
        __syncthreads();
        if (threadIdx.x == 0) {
            const double djj = G[(int64_t)j * na + j];
            if (!(djj > 0.0)) bad = 1;
            G[(int64_t)j * na + j] = djj > 0.0 ? sqrt(djj) : 1.0;
        }
        __syncthreads();
        const double rjj = G[(int64_t)j * na + j];
        for (int q = j + 1 + threadIdx.x; q < na; q += 256) G[(int64_t)j * na + q] /= rjj;
        __syncthreads();
        // trailing update G[p][q] -= R[j][p] R[j][q], p, q > j (upper part)
        const int rem = na - j - 1;
        for (int t = threadIdx.x; t < rem * rem; t += 256) {
            const int p = j + 1 + t / rem, q = j + 1 + t % rem;
            if (q >= p) G[(int64_t)p * na + q] -= G[(int64_t)j * na + p] * G[(int64_t)j * na + q];
        }
    }
    __syncthreads();
    // zero the strict lower part so G holds R
    for (int t = threadIdx.x; t < na * na; t += 256) {
        const int p = t / na, q = t % na;
        if (q < p) G[t] = 0.0;
    }
    __syncthreads();
    // Rinv column by column: R x = e_col, back substitution
    for (int col = threadIdx.x; col < na; col += 256) {
        for (int p = na - 1; p >= 0; --p) {
            double s = (p == col) ? 1.0 : 0.0;
            for (int q = p + 1; q <= col; ++q) s -= G[(int64_t)p * na + q] * Rinv[(int64_t)q * na + col];
            Rinv[(int64_t)p * na + col] = p <= col ? s / G[(int64_t)p * na + p] : 0.0;
        }
    }
    if (threadIdx.x == 0 && bad) atomicOr(flags, 2);
}

hipError_t launch_cholinv(double *G, double *Rinv, int32_t na, int32_t *flags, hipStream_t s) {
    hipLaunchKernelGGL(k_cholinv, dim3(1), dim3(256), 0, s, G, Rinv, na, flags);
    return hipGetLastError();
}

// Z = (sub ? Z : 0) + sgn * X M, row-local: a block owns 32 rows, stages its
// X rows in LDS (FP64) before writing, so Z may alias X when sub == 0.
template <typename T>
__global__ void __launch_bounds__(256) k_apply(const T *X, int32_t ldx, const double *M, int32_t na,
                                               int32_t nb, T *Z, int32_t ldz, int32_t n, int32_t sub) {
    extern __shared__ double xs[];   // [32][na]
    const int64_t r0 = (int64_t)blockIdx.x * 32;
    for (int q = threadIdx.x; q < 32 * na; q += 256) {
        const int rr = q / na, cc = q % na;
        const int64_t r = r0 + rr;
        xs[q] = r < n ? (double)X[r * ldx + cc] : 0.0;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 32 * nb; q += 256) {
        const int rr = q / nb, cc = q % nb;
        const int64_t r = r0 + rr;
        if (r >= n) continue;
        double acc = 0.0;
        for (int t = 0; t < na; ++t) acc = fma(xs[rr * na + t], M[(int64_t)t * nb + cc], acc);
        if (sub) Z[r * ldz + cc] = (T)((double)Z[r * ldz + cc] - acc);
        else Z[r * ldz + cc] = (T)acc;
    }
}

hipError_t launch_apply(const void *X, int32_t ldx, const double *M, int32_t na, int32_t nb, void *Z,
                        int32_t ldz, bool fp64, int32_t n, int32_t sub, hipStream_t s) {
    dim3 g((unsigned)((n + 31) / 32));
    const size_t shm = (size_t)32 * na * sizeof(double);
    if (fp64)
        hipLaunchKernelGGL(k_apply<double>, g, dim3(256), shm, s, (const double *)X, ldx, M, na, nb,
                           (double *)Z, ldz, n, sub);
    else
        hipLaunchKernelGGL(k_apply<float>, g, dim3(256), shm, s, (const float *)X, ldx, M, na, nb, (float *)Z,
                           ldz, n, sub);
    return hipGetLastError();
}

}  // namespace vne
