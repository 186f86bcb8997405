// Rational Krylov cross-check of the polynomial path (Section 4: the
// rational Krylov space of eq. (4.1), the Rayleigh-Ritz form of eq. (4.2);
// rational Arnoldi with full orthogonalization, Remark 4.2; the switch from
// poles at infinity to finite poles of the Krylov method implementation of
// Section 5, on the a-posteriori bound of Theorem 4.8).  FP64 blocks of n x mp (probe index fastest, mp a power of two
// up to 128), one independent basis per column:
//   v_1 = c / ||c||;  for j = 1, 2, ...:  u_j = A v_j,
//   H(1:j, j) = V_j^T u_j,  psi_j = ||c||^2 e_1^T f(H_j) e_1,
//   w = u_j (pole at infinity) or the solution of (I - A / xi) w = u_j (a
//   finite pole xi < 0: a symmetric positive definite system, solved by
//   conjugate gradients on the same sparse product), orthogonalized twice
//   against v_1..v_j (classical Gram-Schmidt), v_{j+1} = w / ||w||.
// e_1^T f(H_j) e_1 is evaluated from the tridiagonal matrix of a Householder
// reduction of H_j whose reflectors leave e_1 fixed, by the Gauss quadrature
// kernel of the polynomial path.  Every reduction over rows is two-level in
// a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ctx_internal.h"
#include "internal.h"
#include "kernels.h"

using namespace vne;
using namespace vne::rt;

namespace {

constexpr int kRThreads = 256;
constexpr int kRBlocks = 512;          // grid of the row kernels (fixed: the reduction order)
constexpr int kRMaxCols = 128;
constexpr int kRMaxBasis = 64;

struct RMat {
    const int32_t *rp, *ci;
    const double *val;
    double scale;
    int32_t n, mp;
};

// lane group of LPR = mp / 2 lanes per row, two columns per lane
__device__ __forceinline__ void r_lanes(int mp, int &lpr, int &gl, int &grp, int &gpb) {
    lpr = mp / 2;
    const int lane = threadIdx.x & 63;
    gl = lane % lpr;
    grp = (threadIdx.x >> 6) * (64 / lpr) + lane / lpr;
    gpb = kRThreads / lpr;
}

// per-block column sums of the threads' values (fixed order over the
// block's lane groups) into part[blockIdx.x][col]
__device__ __forceinline__ void r_block_sums(double *sh, int mp, int gl, int grp, int gpb, const double (&v)[2],
                                             double *part) {
    sh[grp * mp + 2 * gl] = v[0];
    sh[grp * mp + 2 * gl + 1] = v[1];
    __syncthreads();
    for (int c = threadIdx.x; c < mp; c += kRThreads) {
        double s = 0.0;
        for (int g = 0; g < gpb; ++g) s += sh[g * mp + c];
        part[(int64_t)blockIdx.x * mp + c] = s;
    }
}

// Y = scale A X on the columns (mode 0), or, for the conjugate-gradient
// product, Y = X - (scale A X) / xi_c on live columns with the partial sums
// of x . y (mode 1).
__global__ void __launch_bounds__(kRThreads) k_r_apply(RMat a, const double *X, double *Y, const double *xi,
                                                       const int32_t *live, double *part) {
    __shared__ double sh[kRThreads * 2];
    int lpr, gl, grp, gpb;
    r_lanes(a.mp, lpr, gl, grp, gpb);
    const int c0 = 2 * gl;
    double dot[2] = {0.0, 0.0};
    const bool cg = part != nullptr;
    bool on[2] = {true, true};
    double inv[2] = {0.0, 0.0};
    if (cg) {
        for (int k = 0; k < 2; ++k) {
            on[k] = live[c0 + k] != 0;
            inv[k] = on[k] ? 1.0 / xi[c0 + k] : 0.0;
        }
    }
    for (int64_t i = (int64_t)blockIdx.x * gpb + grp; i < a.n; i += (int64_t)gridDim.x * gpb) {
        double acc[2] = {0.0, 0.0};
        for (int p = a.rp[i]; p < a.rp[i + 1]; ++p) {
            const double w = a.val[p];
            const double2 x = *reinterpret_cast<const double2 *>(X + (int64_t)a.ci[p] * a.mp + c0);
            acc[0] = fma(w, x.x, acc[0]);
            acc[1] = fma(w, x.y, acc[1]);
        }
        double2 out;
        if (!cg) {
            out.x = a.scale * acc[0];
            out.y = a.scale * acc[1];
        } else {
            const double2 x = *reinterpret_cast<const double2 *>(X + i * a.mp + c0);
            out.x = on[0] ? fma(-a.scale * acc[0], inv[0], x.x) : 0.0;
            out.y = on[1] ? fma(-a.scale * acc[1], inv[1], x.y) : 0.0;
            dot[0] = fma(x.x, out.x, dot[0]);
            dot[1] = fma(x.y, out.y, dot[1]);
        }
        *reinterpret_cast<double2 *>(Y + i * a.mp + c0) = out;
    }
    if (cg) r_block_sums(sh, a.mp, gl, grp, gpb, dot, part);
}

// partial sums of x . y per column (y = x: squared norms)
__global__ void __launch_bounds__(kRThreads) k_r_dot(int32_t n, int32_t mp, const double *X, const double *Y,
                                                     double *part) {
    __shared__ double sh[kRThreads * 2];
    int lpr, gl, grp, gpb;
    r_lanes(mp, lpr, gl, grp, gpb);
    const int c0 = 2 * gl;
    double dot[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * gpb + grp; i < n; i += (int64_t)gridDim.x * gpb) {
        const double2 x = *reinterpret_cast<const double2 *>(X + i * mp + c0);
        const double2 y = *reinterpret_cast<const double2 *>(Y + i * mp + c0);
        dot[0] = fma(x.x, y.x, dot[0]);
        dot[1] = fma(x.y, y.y, dot[1]);
    }
    r_block_sums(sh, mp, gl, grp, gpb, dot, part);
}

// partial sums of v_i . w for the basis vectors i < nb (V: nb blocks of n x mp)
__global__ void __launch_bounds__(kRThreads) k_r_basis_dots(int32_t n, int32_t mp, const double *V, int32_t nb,
                                                            const double *W, double *part) {
    __shared__ double sh[kRThreads * 2];
    int lpr, gl, grp, gpb;
    r_lanes(mp, lpr, gl, grp, gpb);
    const int c0 = 2 * gl;
    const int64_t blk = (int64_t)n * mp;
    for (int b = 0; b < nb; ++b) {
        double dot[2] = {0.0, 0.0};
        for (int64_t i = (int64_t)blockIdx.x * gpb + grp; i < n; i += (int64_t)gridDim.x * gpb) {
            const double2 v = *reinterpret_cast<const double2 *>(V + b * blk + i * mp + c0);
            const double2 w = *reinterpret_cast<const double2 *>(W + i * mp + c0);
            dot[0] = fma(v.x, w.x, dot[0]);
            dot[1] = fma(v.y, w.y, dot[1]);
        }
        r_block_sums(sh, mp, gl, grp, gpb, dot, part + (int64_t)b * gridDim.x * mp);
        __syncthreads();
    }
}

// out[r * mp + c] = sum over blocks of part[r][block][c] (fixed order), r < rows
__global__ void __launch_bounds__(256) k_r_reduce(const double *part, int32_t nblk, int32_t mp, int32_t rows,
                                                  double *out) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= rows * mp) return;
    const int r = t / mp, c = t % mp;
    const double *p = part + (int64_t)r * nblk * mp + c;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += p[(int64_t)b * mp];
    out[t] = s;
}

// W -= sum_i h[i][c] v_i (i < nb)
__global__ void __launch_bounds__(kRThreads) k_r_basis_axpy(int32_t n, int32_t mp, const double *V, int32_t nb,
                                                            const double *h, double *W) {
    const int64_t total = (int64_t)n * mp;
    for (int64_t t = (int64_t)blockIdx.x * kRThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kRThreads) {
        const int c = (int)(t % mp);
        double w = W[t];
        for (int b = 0; b < nb; ++b) w = fma(-h[b * mp + c], V[b * total + t], w);
        W[t] = w;
    }
}

// v = w / ||w|| per column; a column whose w lost all but 1e-12 of its norm
// to the orthogonalization (an invariant subspace) gets v = 0 and ends
__global__ void __launch_bounds__(kRThreads) k_r_normalize(int32_t n, int32_t mp, const double *W, const double *ww,
                                                           const double *ww0, double *Vout) {
    const int64_t total = (int64_t)n * mp;
    for (int64_t t = (int64_t)blockIdx.x * kRThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kRThreads) {
        const int c = (int)(t % mp);
        const double s = ww[c];
        Vout[t] = (s > 1e-24 * ww0[c] && s > 0.0) ? W[t] / sqrt(s) : 0.0;
    }
}

// conjugate gradients: x = 0, r = p = b on live columns; x = b elsewhere
__global__ void __launch_bounds__(kRThreads) k_r_cg_init(int32_t n, int32_t mp, const double *B, const int32_t *live,
                                                         double *X, double *R, double *P) {
    const int64_t total = (int64_t)n * mp;
    for (int64_t t = (int64_t)blockIdx.x * kRThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kRThreads) {
        const int c = (int)(t % mp);
        const double b = B[t];
        const bool on = live[c] != 0;
        X[t] = on ? 0.0 : b;
        R[t] = on ? b : 0.0;
        P[t] = on ? b : 0.0;
    }
}

// x += alpha p, r -= alpha q (alpha = rr / pq on live columns) and the
// partial sums of r . r
__global__ void __launch_bounds__(kRThreads) k_r_cg_update(int32_t n, int32_t mp, const double *rr, const double *pq,
                                                           const int32_t *live, const double *P, const double *Q,
                                                           double *X, double *R, double *part) {
    __shared__ double sh[kRThreads * 2];
    int lpr, gl, grp, gpb;
    r_lanes(mp, lpr, gl, grp, gpb);
    const int c0 = 2 * gl;
    double al[2];
    for (int k = 0; k < 2; ++k) al[k] = live[c0 + k] && pq[c0 + k] != 0.0 ? rr[c0 + k] / pq[c0 + k] : 0.0;
    double dot[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * gpb + grp; i < n; i += (int64_t)gridDim.x * gpb) {
        const int64_t o = i * mp + c0;
        const double2 p = *reinterpret_cast<const double2 *>(P + o);
        const double2 q = *reinterpret_cast<const double2 *>(Q + o);
        double2 x = *reinterpret_cast<const double2 *>(X + o);
        double2 r = *reinterpret_cast<const double2 *>(R + o);
        x.x = fma(al[0], p.x, x.x);
        x.y = fma(al[1], p.y, x.y);
        r.x = fma(-al[0], q.x, r.x);
        r.y = fma(-al[1], q.y, r.y);
        *reinterpret_cast<double2 *>(X + o) = x;
        *reinterpret_cast<double2 *>(R + o) = r;
        dot[0] = fma(r.x, r.x, dot[0]);
        dot[1] = fma(r.y, r.y, dot[1]);
    }
    r_block_sums(sh, mp, gl, grp, gpb, dot, part);
}

// per column: beta = rr_new / rr; a column ends when ||r|| <= tol ||b|| or
// after cg_max iterations; remaining = live columns left.  A zero right-hand
// side (a column whose basis stopped growing) is solved by x = 0 and counts
// no iteration.
__global__ void __launch_bounds__(256) k_r_cg_scalars(int32_t mp, double *rr, const double *rr_new, const double *rr0,
                                                      double tol2, int32_t cg_max, int32_t *live, int32_t *iters,
                                                      int64_t *apps, double *beta, int32_t *remaining) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int c = threadIdx.x; c < mp; c += 256) {
        double b = 0.0;
        if (live[c] && rr0[c] == 0.0) {
            live[c] = 0;
        } else if (live[c]) {
            iters[c] += 1;
            apps[c] += 1;
            const double rn = rr_new[c];
            b = rr[c] > 0.0 ? rn / rr[c] : 0.0;
            rr[c] = rn;
            if (!(rn > tol2 * rr0[c]) || iters[c] >= cg_max) live[c] = 0;
            else atomicAdd(&cnt, 1);
        }
        beta[c] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) *remaining = cnt;
}

// p = r + beta p on live columns
__global__ void __launch_bounds__(kRThreads) k_r_cg_dir(int32_t n, int32_t mp, const double *beta, const int32_t *live,
                                                        const double *R, double *P) {
    const int64_t total = (int64_t)n * mp;
    for (int64_t t = (int64_t)blockIdx.x * kRThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kRThreads) {
        const int c = (int)(t % mp);
        if (live[c]) P[t] = fma(beta[c], P[t], R[t]);
    }
}

// Per column: the leading j x j block of H (symmetric, H[c][a][b] at
// (c * kb + a) * kb + b), reduced to tridiagonal form by Householder
// reflectors on rows and columns 1.. (e_1 stays fixed), so that
// e_1^T f(H_j) e_1 = e_1^T f(T) e_1; T's diagonal and off-diagonal go to
// alpha / beta (row stride kb), k_eff[c] = the basis size (ke[c] capped at j).
__global__ void __launch_bounds__(64) k_r_tridiag(const double *H, int32_t kb, int32_t j, const int32_t *ke,
                                                  double *alpha, double *beta, int32_t *k_eff) {
    __shared__ double M[kRMaxBasis * kRMaxBasis];
    __shared__ double v[kRMaxBasis], p[kRMaxBasis], w[kRMaxBasis];
    __shared__ double sc[2];
    const int c = blockIdx.x, t = threadIdx.x;
    const int nn = min(j, ke[c]);
    for (int e = t; e < nn * nn; e += 64) M[e] = H[((int64_t)c * kb + e / nn) * kb + e % nn];
    __syncthreads();
    for (int k = 0; k + 2 < nn; ++k) {
        // x = M[k+1 .. nn-1][k]; v = x + sign(x0) ||x|| e_1, reflector I - 2 v v^T / v^T v
        if (t == 0) {
            double s = 0.0;
            for (int i = k + 1; i < nn; ++i) s += M[i * nn + k] * M[i * nn + k];
            const double nx = sqrt(s), x0 = M[(k + 1) * nn + k];
            sc[0] = nx;
            sc[1] = x0 >= 0.0 ? x0 + nx : x0 - nx;
        }
        __syncthreads();
        const double nx = sc[0], v0 = sc[1];
        if (nx == 0.0 || v0 == 0.0) {     // column already reduced
            __syncthreads();
            continue;
        }
        for (int i = k + 1 + t; i < nn; i += 64) v[i] = i == k + 1 ? v0 : M[i * nn + k];
        __syncthreads();
        double vv = 0.0;
        for (int i = k + 1; i < nn; ++i) vv += v[i] * v[i];
        const double tau = 2.0 / vv;
        // p = tau M v (trailing block), w = p - (tau / 2) (p^T v) v
        for (int i = k + 1 + t; i < nn; i += 64) {
            double s = 0.0;
            for (int l = k + 1; l < nn; ++l) s += M[i * nn + l] * v[l];
            p[i] = tau * s;
        }
        __syncthreads();
        double pv = 0.0;
        for (int i = k + 1; i < nn; ++i) pv += p[i] * v[i];
        for (int i = k + 1 + t; i < nn; i += 64) w[i] = p[i] - 0.5 * tau * pv * v[i];
        __syncthreads();
        for (int e = t; e < (nn - k - 1) * (nn - k - 1); e += 64) {
            const int i = k + 1 + e / (nn - k - 1), l = k + 1 + e % (nn - k - 1);
            M[i * nn + l] -= v[i] * w[l] + w[i] * v[l];
        }
        // column k: M[k+1][k] = -sign(x0) ||x||, the rest 0
        if (t == 0) {
            const double d = v0 > 0.0 ? -nx : nx;
            M[(k + 1) * nn + k] = M[k * nn + k + 1] = d;
            for (int i = k + 2; i < nn; ++i) M[i * nn + k] = M[k * nn + i] = 0.0;
        }
        __syncthreads();
    }
    for (int i = t; i < kb; i += 64) {
        alpha[(int64_t)c * kb + i] = i < nn ? M[i * nn + i] : 0.0;
        beta[(int64_t)c * kb + i] = i + 1 < nn ? fabs(M[(i + 1) * nn + i]) : 0.0;
    }
    if (t == 0) k_eff[c] = nn;
}

// H[c][i][j-1] = H[c][j-1][i] = h[i][c] for i < j (the new column of the
// symmetric projected matrix)
__global__ void __launch_bounds__(256) k_r_store_h(const double *h, int32_t j, int32_t mp, int32_t kb, double *H) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= j * mp) return;
    const int i = t / mp, c = t % mp;
    const double v = h[t];
    H[((int64_t)c * kb + i) * kb + (j - 1)] = v;
    H[((int64_t)c * kb + (j - 1)) * kb + i] = v;
}

// basis sizes: ke[c] = 1 for a nonzero start vector (c < m), else 0
__global__ void __launch_bounds__(256) k_r_init_ke(const double *norm2, int32_t m, int32_t mp, int32_t *ke) {
    for (int c = threadIdx.x; c < mp; c += 256) ke[c] = c < m && norm2[c] > 0.0 ? 1 : 0;
}

// after step j: apps[c] += 1 for u_j of a column whose basis has j vectors;
// apps_hist[j-1][c] = apps[c] (the applications of A behind psi_j)
__global__ void __launch_bounds__(256) k_r_count(const int32_t *ke, int32_t j, int32_t mp, int64_t *apps,
                                                 int64_t *apps_hist) {
    for (int c = threadIdx.x; c < mp; c += 256) {
        apps[c] += ke[c] >= j ? 1 : 0;
        apps_hist[(int64_t)(j - 1) * mp + c] = apps[c];
    }
}

// a column whose basis has j vectors takes v_{j+1} unless w vanished in the
// orthogonalization (the criterion of k_r_normalize)
__global__ void __launch_bounds__(256) k_r_grow(const double *ww, const double *ww0, int32_t j, int32_t mp,
                                                int32_t *ke) {
    for (int c = threadIdx.x; c < mp; c += 256)
        if (ke[c] == j && ww[c] > 1e-24 * ww0[c] && ww[c] > 0.0) ke[c] = j + 1;
}

// beta_j of the polynomial phase: the norm of A v_j orthogonalized against
// v_1..v_j (ww), for a column whose basis has j vectors and whose direction
// passes the invariant-subspace test of k_r_normalize; else 0.  Row c of beta
// at c * kb, entry j - 1.
__global__ void __launch_bounds__(256) k_r_beta_next(const double *ww, const double *ww0, const int32_t *ke,
                                                     int32_t j, int32_t mp, int32_t kb, double *beta) {
    for (int c = threadIdx.x; c < mp; c += 256) {
        const bool keep = ke[c] == j && ww[c] > 1e-24 * ww0[c] && ww[c] > 0.0;
        beta[(int64_t)c * kb + j - 1] = keep ? sqrt(ww[c]) : 0.0;
    }
}

// The switch rule (Section 5, Krylov method implementation): after
// polynomial step j, a column still on poles at infinity records its error
// bound err_j (Theorem 4.8's upper bound hi, or the estimate sqrt(lo hi) of
// eq. (4.10)) and switches to finite poles when err_j >= c^ell err_{j-ell-1}
// (j >= ell + 2); it then takes the finite poles in order.  xi[c] is the
// pole of step j (0: infinity).
__global__ void __launch_bounds__(256) k_r_switch(int32_t mp, int32_t m, const double *lo, const double *hi,
                                                  int32_t estimate, double *errs, int32_t kb, int32_t j, int32_t ell,
                                                  double c_ell, const double *finite, int32_t n_finite,
                                                  int32_t *switched, double *xi) {
    for (int c = threadIdx.x; c < mp; c += 256) {
        if (c >= m) {
            xi[c] = 0.0;
            continue;
        }
        double *e = errs + (int64_t)c * kb;
        int s = switched[c];
        if (s == 0) {
            e[j - 1] = estimate ? sqrt(lo[c] * hi[c]) : hi[c];
            if (j - ell - 1 >= 1 && e[j - 1] >= c_ell * e[j - ell - 2]) s = j;
        }
        switched[c] = s;
        const int t = s > 0 ? j - s : -1;
        xi[c] = t >= 0 && t < n_finite ? finite[t] : 0.0;
    }
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

extern "C" vne_status vne_rational_quadforms(vne_ctx *c, int32_t gid, const vne_probes *pr, uint32_t mode,
                                             const vne_rational_cfg *cfg, vne_rational_out *out) {
    if (!c) return VNE_EINVAL;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    c->err.clear();
    if (!pr || !cfg || !out) return fail(c, VNE_EINVAL, "NULL argument");
    if (!get_graph(c, gid)) return fail(c, VNE_EINVAL, "unknown graph id");
    VNE_TRY(check_mode(c, mode));
    if (!(mode & VNE_MODE_F64)) return fail(c, VNE_ENOTSUP, "the rational Krylov cross-check runs in FP64 (VNE_MODE_F64)");
    if (pr->kind == VNE_PROBE_HUTCHPP) return fail(c, VNE_ENOTSUP, "rational Krylov takes RADEMACHER, COLORING or DENSE probes");
    const int m = pr->m;
    if (m < 1 || m > kRMaxCols) return fail(c, VNE_EINVAL, "probe count m must be in [1, 128]");
    const int kb = cfg->steps;
    if (kb < 1 || kb > kRMaxBasis) return fail(c, VNE_EINVAL, "steps must be in [1, 64]");
    const bool switching = cfg->poles == nullptr;
    if (switching && (cfg->ell < 1 || !(cfg->c > 0.0 && cfg->c < 1.0)))
        return fail(c, VNE_EINVAL, "the switch rule needs ell >= 1 and 0 < c < 1");
    if (switching && !(cfg->lam_lo > 0.0 && cfg->lam_hi > cfg->lam_lo && std::isfinite(cfg->lam_hi)))
        return fail(c, VNE_EINVAL, "the switch rule's bound needs 0 < lam_lo < lam_hi");
    const int n_fin = switching ? cfg->n_finite : kb - 1;
    const double *fin = switching ? cfg->finite_poles : cfg->poles;
    if (n_fin < 0 || (n_fin > 0 && !fin)) return fail(c, VNE_EINVAL, "pole list missing");
    for (int i = 0; i < n_fin; ++i)
        if (!(fin[i] < 0.0) && !(switching ? false : std::isinf(fin[i]) && fin[i] > 0))
            return fail(c, VNE_EINVAL, "poles must be negative (or +INFINITY in an explicit list)");
    const double tol = cfg->cg_tol > 0.0 ? cfg->cg_tol : 1e-10;
    const int cg_max = cfg->cg_max > 0 ? cfg->cg_max : 20000;
    HIP_TRY(c, hipSetDevice(c->device));
    GraphSet *set = nullptr;
    VNE_TRY(get_set(c, {gid}, &set));
    const bool desing = (mode & VNE_MODE_DESING) != 0;
    if (desing && !set->zero_rowsum)
        return fail(c, VNE_EINVAL, "VNE_MODE_DESING needs a matrix whose rows sum to zero (A 1 = 0)");
    const auto t0 = std::chrono::steady_clock::now();
    int mp = 2;
    while (mp < m) mp *= 2;
    const int64_t n = set->n;
    const size_t blk = (size_t)n * mp * 8;
    hipStream_t s = c->stream;

    // device memory of the call: basis, work blocks, small per-column arrays
    DevBuf dV, dU, dW, dX, dR, dP, dQ, dPart, dH, dSmall, dAl, dBe, dKe, dPsi, dHist, dNorm, dMean, dFlags, dInt, dApps,
        dXi, dFin, dProbePart, dStA, dStI, dStC, dErr, dLo, dHi, dBa;
    auto all = {&dV, &dU, &dW, &dX, &dR, &dP, &dQ, &dPart, &dH, &dSmall, &dAl, &dBe, &dKe, &dPsi, &dHist, &dNorm,
                &dMean, &dFlags, &dInt, &dApps, &dXi, &dFin, &dProbePart, &dStA, &dStI, &dStC, &dErr, &dLo, &dHi, &dBa};
    auto fin_all = [&](vne_status st) {
        for (DevBuf *b : all) dev_free(c, b);
        return st;
    };
    vne_status st = VNE_OK;
    auto A = [&](DevBuf *b, size_t bytes) {
        if (st == VNE_OK) st = dev_alloc(c, b, bytes);
    };
    A(&dV, blk * kb);
    A(&dU, blk);
    A(&dW, blk);
    A(&dX, blk);
    A(&dR, blk);
    A(&dP, blk);
    A(&dQ, blk);
    A(&dPart, (size_t)kRBlocks * kb * mp * 8);
    A(&dH, (size_t)mp * kb * kb * 8);
    A(&dSmall, (size_t)8 * kb * mp * 8);     // h, rr, rr0, pq, rr_new, ww, ww0, beta
    A(&dAl, (size_t)mp * kb * 8);
    A(&dBe, (size_t)mp * kb * 8);
    A(&dKe, (size_t)mp * 4 * 2);            // k_eff, basis size
    A(&dPsi, (size_t)mp * 8);
    A(&dHist, (size_t)mp * kb * 8);
    A(&dNorm, (size_t)mp * 8);
    A(&dMean, (size_t)mp * 8);
    A(&dFlags, 4);
    A(&dInt, (size_t)mp * 4 * 3 + 64);      // live, iters, switched, remaining
    A(&dApps, (size_t)mp * 8 * (kb + 1));   // per column cumulative applications of A, and after each step
    A(&dXi, (size_t)mp * 8);
    A(&dFin, (size_t)std::max(1, n_fin) * 8);
    A(&dProbePart, (size_t)set->probe_blocks * mp * 8);
    A(&dStA, (size_t)mp * 8);
    A(&dStI, (size_t)mp * 8);
    A(&dStC, (size_t)mp * 8);
    A(&dErr, (size_t)mp * kb * 8);          // error bounds of the polynomial steps (switch rule)
    A(&dLo, (size_t)mp * 8);
    A(&dHi, (size_t)mp * 8);
    A(&dBa, sizeof(BoundArgs) * kb);
    if (st != VNE_OK) return fin_all(st);
    double *V = (double *)dV.p, *U = (double *)dU.p, *W = (double *)dW.p, *X = (double *)dX.p, *R = (double *)dR.p,
           *P = (double *)dP.p, *Q = (double *)dQ.p, *part = (double *)dPart.p, *H = (double *)dH.p;
    double *sm = (double *)dSmall.p;
    double *h = sm, *rr = sm + (size_t)kb * mp, *rr0 = rr + mp, *pq = rr0 + mp, *rrn = pq + mp, *ww = rrn + mp,
           *ww0 = ww + mp, *cgb = ww0 + mp;
    int32_t *live = (int32_t *)dInt.p, *iters = live + mp, *switched = iters + mp, *remaining = switched + mp;
    int64_t *apps = (int64_t *)dApps.p, *apps_hist = apps + mp;
    int32_t *ke = (int32_t *)dKe.p + mp;
    auto E = [&](hipError_t e, const char *w) -> vne_status { return e == hipSuccess ? VNE_OK : hip_fail(c, e, w); };
#define R_TRY(expr)                                       \
    do {                                                  \
        vne_status _s = E((expr), #expr);                 \
        if (_s != VNE_OK) return fin_all(_s);             \
    } while (0)
    R_TRY(hipMemsetAsync(dH.p, 0, dH.bytes, s));
    R_TRY(hipMemsetAsync(dInt.p, 0, dInt.bytes, s));
    R_TRY(hipMemsetAsync(dApps.p, 0, dApps.bytes, s));
    R_TRY(hipMemsetAsync(dHist.p, 0, dHist.bytes, s));
    R_TRY(hipMemsetAsync(dFlags.p, 0, 4, s));
    R_TRY(hipMemsetAsync(dErr.p, 0, dErr.bytes, s));
    if (switching) {
        // the bound of each polynomial step j (steps = j) over the caller's
        // interval; switched columns are skipped
        std::vector<BoundArgs> hb(kb);
        for (int jj = 1; jj <= kb; ++jj) {
            BoundArgs &b = hb[jj - 1];
            b.alpha = (const double *)dAl.p;
            b.beta = (const double *)dBe.p;
            b.k_eff = (const int32_t *)dKe.p;
            b.norm2 = (const double *)dNorm.p;
            b.k = kb;
            b.m = m;
            b.steps = jj;
            b.lam_lo = cfg->lam_lo;
            b.lam_hi = cfg->lam_hi;
            b.n_grid = kBoundGrid;
            b.lo = (double *)dLo.p;
            b.hi = (double *)dHi.p;
            b.flags = (int32_t *)dFlags.p;
            b.col_stop = switched;
            b.stop_state = nullptr;
        }
        R_TRY(hipMemcpyAsync(dBa.p, hb.data(), sizeof(BoundArgs) * kb, hipMemcpyHostToDevice, s));
        R_TRY(hipStreamSynchronize(s));     // hb leaves scope
    }
    if (n_fin > 0) R_TRY(hipMemcpyAsync(dFin.p, fin, (size_t)n_fin * 8, hipMemcpyHostToDevice, s));
    // start vectors c = b - mean (desingularized) into V_1 via the probe
    // kernels of the polynomial path (which also give ||c||^2)
    {
        Plan p;
        p.fp64 = true;
        p.G = 1;
        p.m = m;
        p.m_pad = mp;
        p.mt = mp;
        p.k = kb;
        p.h_graph_k = {kb};
        p.h_graph_m = {m};
        ProbeSpec ps;
        int combine_kind = 0;
        if (pr->kind == VNE_PROBE_COLORING && pr->location == VNE_HOST) A(&p.colors, (size_t)n * 4);
        if (pr->kind == VNE_PROBE_DENSE && pr->location == VNE_HOST) A(&p.dense, (size_t)n * m * 8);
        if (st != VNE_OK) return fin_all(st);
        vne_status ps_st = make_probe_spec(c, set, &p, pr, m, true, &ps, &combine_kind);
        if (ps_st != VNE_OK) {
            dev_free(c, &p.colors);
            dev_free(c, &p.dense);
            return fin_all(ps_st);
        }
        ProbeArgs pa{};
        pa.gen = ps.gen;
        pa.n = (int32_t)n;
        pa.m = m;
        pa.m_pad = mp;
        pa.mt = mp;
        pa.ld_out = mp;
        pa.seed = ps.seeds.empty() ? 0 : ps.seeds[0];
        pa.keys = (const int64_t *)set->keys.p;
        pa.colors = ps.colors;
        pa.dense = ps.dense;
        pa.ld_dense = ps.ld_dense;
        pa.desing = desing ? 1 : 0;
        pa.P_out = W;
        pa.partials = (double *)dProbePart.p;
        pa.n_blocks = set->probe_blocks;
        pa.mean = (double *)dMean.p;
        pa.norm2 = (double *)dNorm.p;
        pa.st_alpha = (double *)dStA.p;
        pa.st_inv = (double *)dStI.p;
        pa.st_coup = (double *)dStC.p;
        pa.k_eff = (int32_t *)dKe.p;
        pa.k = kb;
        pa.block_row_begin = (const int32_t *)set->probe_rows.p;
        pa.block_graph = (const int32_t *)set->probe_block_graph.p;
        pa.graph_block_begin = (const int32_t *)set->probe_graph_begin.p;
        pa.graph_row_begin = (const int64_t *)set->graph_row_begin.p;
        pa.n_graphs = 1;
        pa.flags = (int32_t *)dFlags.p;
        vne_status lst = E(launch_probe(pa, true, s), "launch_probe");
        if (lst == VNE_OK) lst = E(hipStreamSynchronize(s), "hipStreamSynchronize");
        dev_free(c, &p.colors);
        dev_free(c, &p.dense);
        if (lst != VNE_OK) return fin_all(lst);
    }
    // v_1 = c / ||c|| (ww = ww0 = ||c||^2); columns past m are zero
    R_TRY(hipMemcpyAsync(ww, dNorm.p, (size_t)mp * 8, hipMemcpyDeviceToDevice, s));
    R_TRY(hipMemcpyAsync(ww0, dNorm.p, (size_t)mp * 8, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_r_normalize, dim3(kRBlocks), dim3(kRThreads), 0, s, (int32_t)n, mp, W, ww, ww0, V);
    hipLaunchKernelGGL(k_r_init_ke, dim3(1), dim3(256), 0, s, (const double *)dNorm.p, m, mp, ke);
    RMat am{set->d_row_ptr, set->d_col, (const double *)set->val64.p, set->scale, (int32_t)n, mp};
    std::vector<double> h_xi(mp, 0.0);
    std::vector<int32_t> h_live(mp, 0), h_sw(mp, 0);
    bool all_switched = false;
    int64_t total_cg = 0;
    int steps_done = 0;
    for (int j = 1; j <= kb; ++j) {
        const double *vj = V + (size_t)(j - 1) * n * mp;
        // u_j = A v_j, H(1:j, j) = V_j^T u_j
        hipLaunchKernelGGL(k_r_apply, dim3(kRBlocks), dim3(kRThreads), 0, s, am, vj, U, (const double *)nullptr,
                           (const int32_t *)nullptr, (double *)nullptr);
        hipLaunchKernelGGL(k_r_basis_dots, dim3(kRBlocks), dim3(kRThreads), 0, s, (int32_t)n, mp, V, j, U, part);
        hipLaunchKernelGGL(k_r_reduce, dim3((j * mp + 255) / 256), dim3(256), 0, s, part, kRBlocks, mp, j, h);
        hipLaunchKernelGGL(k_r_store_h, dim3((j * mp + 255) / 256), dim3(256), 0, s, (const double *)h, j, mp, kb, H);
        // psi_j from H_j
        hipLaunchKernelGGL(k_r_tridiag, dim3(mp), dim3(64), 0, s, H, kb, j, ke, (double *)dAl.p, (double *)dBe.p,
                           (int32_t *)dKe.p);
        R_TRY(launch_quadrature((const double *)dAl.p, (const double *)dBe.p, (const int32_t *)dKe.p,
                                (const double *)dNorm.p, kb, j, mp, (double *)dPsi.p, (int32_t *)dFlags.p, s, true));
        R_TRY(hipMemcpy2DAsync((double *)dHist.p + (j - 1), (size_t)kb * 8, dPsi.p, 8, 8, mp, hipMemcpyDeviceToDevice,
                               s));
        steps_done = j;
        // cumulative applications of A per column: one for u_j
        hipLaunchKernelGGL(k_r_count, dim3(1), dim3(256), 0, s, (const int32_t *)ke, j, mp, apps, apps_hist);
        if (j == kb) break;
        // w_j orthogonalized twice against v_1..v_j (classical Gram-Schmidt),
        // with ||w||^2 before (ww0) and after (ww)
        auto orthogonalize = [&]() {
            hipLaunchKernelGGL(k_r_dot, dim3(kRBlocks), dim3(kRThreads), 0, s, (int32_t)n, mp, (const double *)W,
                               (const double *)W, part);
            hipLaunchKernelGGL(k_r_reduce, dim3((mp + 255) / 256), dim3(256), 0, s, part, kRBlocks, mp, 1, ww0);
            for (int pass = 0; pass < 2; ++pass) {
                hipLaunchKernelGGL(k_r_basis_dots, dim3(kRBlocks), dim3(kRThreads), 0, s, (int32_t)n, mp, V, j,
                                   (const double *)W, part);
                hipLaunchKernelGGL(k_r_reduce, dim3((j * mp + 255) / 256), dim3(256), 0, s, part, kRBlocks, mp, j, h);
                hipLaunchKernelGGL(k_r_basis_axpy, dim3(kRBlocks), dim3(kRThreads), 0, s, (int32_t)n, mp, V, j,
                                   (const double *)h, W);
            }
            hipLaunchKernelGGL(k_r_dot, dim3(kRBlocks), dim3(kRThreads), 0, s, (int32_t)n, mp, (const double *)W,
                               (const double *)W, part);
            hipLaunchKernelGGL(k_r_reduce, dim3((mp + 255) / 256), dim3(256), 0, s, part, kRBlocks, mp, 1, ww);
        };
        bool w_ready = false;    // W holds the orthogonalized polynomial direction
        // the pole of step j
        if (switching) {
            if (!all_switched) {
                // the polynomial direction of every column first: beta_j of
                // the bound (Theorem 4.8) that the switch rule reads
                R_TRY(hipMemcpyAsync(W, U, blk, hipMemcpyDeviceToDevice, s));
                orthogonalize();
                w_ready = true;
                hipLaunchKernelGGL(k_r_beta_next, dim3(1), dim3(256), 0, s, (const double *)ww, (const double *)ww0,
                                   (const int32_t *)ke, j, mp, kb, (double *)dBe.p);
                R_TRY(launch_error_bound_cols((const BoundArgs *)dBa.p + (j - 1), m, s));
            }
            hipLaunchKernelGGL(k_r_switch, dim3(1), dim3(256), 0, s, mp, m, (const double *)dLo.p,
                               (const double *)dHi.p, cfg->estimate ? 1 : 0, (double *)dErr.p, kb, j, cfg->ell,
                               std::pow(cfg->c, cfg->ell), (const double *)dFin.p, n_fin, switched, (double *)dXi.p);
            R_TRY(hipMemcpyAsync(h_xi.data(), dXi.p, (size_t)mp * 8, hipMemcpyDeviceToHost, s));
            R_TRY(hipMemcpyAsync(h_sw.data(), switched, (size_t)mp * 4, hipMemcpyDeviceToHost, s));
            R_TRY(hipStreamSynchronize(s));
            all_switched = true;
            for (int cc = 0; cc < m; ++cc) all_switched = all_switched && h_sw[cc] > 0;
        } else {
            const double xi = fin[j - 1];
            for (int cc = 0; cc < mp; ++cc) h_xi[cc] = cc < m && std::isfinite(xi) ? xi : 0.0;
            R_TRY(hipMemcpyAsync(dXi.p, h_xi.data(), (size_t)mp * 8, hipMemcpyHostToDevice, s));
        }
        // w = u_j, or the solution of (I - A / xi) w = u_j by conjugate gradients
        bool any = false;
        for (int cc = 0; cc < mp; ++cc) {
            h_live[cc] = h_xi[cc] != 0.0 ? 1 : 0;
            any = any || h_live[cc];
        }
        if (!any) {
            if (!w_ready) R_TRY(hipMemcpyAsync(W, U, blk, hipMemcpyDeviceToDevice, s));
        } else {
            w_ready = false;
            R_TRY(hipMemcpyAsync(live, h_live.data(), (size_t)mp * 4, hipMemcpyHostToDevice, s));
            R_TRY(hipMemsetAsync(iters, 0, (size_t)mp * 4, s));
            hipLaunchKernelGGL(k_r_cg_init, dim3(kRBlocks), dim3(kRThreads), 0, s, (int32_t)n, mp, (const double *)U,
                               (const int32_t *)live, W, R, P);
            hipLaunchKernelGGL(k_r_dot, dim3(kRBlocks), dim3(kRThreads), 0, s, (int32_t)n, mp, (const double *)R,
                               (const double *)R, part);
            hipLaunchKernelGGL(k_r_reduce, dim3((mp + 255) / 256), dim3(256), 0, s, part, kRBlocks, mp, 1, rr);
            R_TRY(hipMemcpyAsync(rr0, rr, (size_t)mp * 8, hipMemcpyDeviceToDevice, s));
            for (int it = 0; it < cg_max; ++it) {
                hipLaunchKernelGGL(k_r_apply, dim3(kRBlocks), dim3(kRThreads), 0, s, am, (const double *)P, Q,
                                   (const double *)dXi.p, (const int32_t *)live, part);
                hipLaunchKernelGGL(k_r_reduce, dim3((mp + 255) / 256), dim3(256), 0, s, part, kRBlocks, mp, 1, pq);
                hipLaunchKernelGGL(k_r_cg_update, dim3(kRBlocks), dim3(kRThreads), 0, s, (int32_t)n, mp,
                                   (const double *)rr, (const double *)pq, (const int32_t *)live, (const double *)P,
                                   (const double *)Q, W, R, part);
                hipLaunchKernelGGL(k_r_reduce, dim3((mp + 255) / 256), dim3(256), 0, s, part, kRBlocks, mp, 1, rrn);
                hipLaunchKernelGGL(k_r_cg_scalars, dim3(1), dim3(256), 0, s, mp, rr, (const double *)rrn,
                                   (const double *)rr0, tol * tol, cg_max, live, iters, apps, cgb, remaining);
                hipLaunchKernelGGL(k_r_cg_dir, dim3(kRBlocks), dim3(kRThreads), 0, s, (int32_t)n, mp,
                                   (const double *)cgb, (const int32_t *)live, (const double *)R, P);
                if ((it & 7) == 7 || it + 1 == cg_max) {
                    int32_t rem = 0;
                    R_TRY(hipMemcpyAsync(&rem, remaining, 4, hipMemcpyDeviceToHost, s));
                    R_TRY(hipStreamSynchronize(s));
                    if (rem == 0) break;
                }
            }
            std::vector<int32_t> hi(mp);
            R_TRY(hipMemcpyAsync(hi.data(), iters, (size_t)mp * 4, hipMemcpyDeviceToHost, s));
            R_TRY(hipStreamSynchronize(s));
            for (int cc = 0; cc < m; ++cc) total_cg += hi[cc];
        }
        if (!w_ready) orthogonalize();
        hipLaunchKernelGGL(k_r_normalize, dim3(kRBlocks), dim3(kRThreads), 0, s, (int32_t)n, mp, (const double *)W,
                           (const double *)ww, (const double *)ww0, V + (size_t)j * n * mp);
        // basis size: a column grows while its new vector is not zero
        hipLaunchKernelGGL(k_r_grow, dim3(1), dim3(256), 0, s, (const double *)ww, (const double *)ww0, j, mp, ke);
    }
    // results
    std::vector<double> hist((size_t)mp * kb);
    std::vector<int64_t> ah((size_t)kb * mp);
    std::vector<double> eh((size_t)mp * kb);
    std::vector<int32_t> sw(mp), kk(mp);
    int32_t fl = 0;
    R_TRY(hipMemcpyAsync(hist.data(), dHist.p, hist.size() * 8, hipMemcpyDeviceToHost, s));
    R_TRY(hipMemcpyAsync(eh.data(), dErr.p, eh.size() * 8, hipMemcpyDeviceToHost, s));
    R_TRY(hipMemcpyAsync(ah.data(), apps_hist, ah.size() * 8, hipMemcpyDeviceToHost, s));
    R_TRY(hipMemcpyAsync(sw.data(), switched, (size_t)mp * 4, hipMemcpyDeviceToHost, s));
    R_TRY(hipMemcpyAsync(kk.data(), ke, (size_t)mp * 4, hipMemcpyDeviceToHost, s));
    R_TRY(hipMemcpyAsync(&fl, dFlags.p, 4, hipMemcpyDeviceToHost, s));
    if (out->norm2) R_TRY(hipMemcpyAsync(out->norm2, dNorm.p, (size_t)m * 8, hipMemcpyDeviceToHost, s));
    R_TRY(hipStreamSynchronize(s));
#undef R_TRY
    for (int cc = 0; cc < m; ++cc) {
        if (out->quad) out->quad[cc] = hist[(size_t)cc * kb + steps_done - 1];
        for (int j = 0; j < kb; ++j) {
            if (out->psi_steps) out->psi_steps[(size_t)cc * kb + j] = j < steps_done ? hist[(size_t)cc * kb + j] : 0.0;
            if (out->apps_steps) out->apps_steps[(size_t)cc * kb + j] = j < steps_done ? ah[(size_t)j * mp + cc] : 0;
            if (out->err_steps) out->err_steps[(size_t)cc * kb + j] = eh[(size_t)cc * kb + j];
        }
        if (out->switch_step) out->switch_step[cc] = sw[cc];
        if (out->basis) out->basis[cc] = kk[cc];
    }
    out->cg_iterations = total_cg;
    out->ms = ms_since(t0);
    fin_all(VNE_OK);
    return check_flags(c, fl);
}
