// Condition-number estimate of a sparsifier (Eq. 2) and sigma-driven stopping.
//
// Alg. 1 takes the similarity target sigma but the paper's method never uses
// it; stopping when kappa(L_G, L_P) <= sigma^2 needs an estimate of kappa.
// P keeps G's weights on a subset of G's edges, so L_P <= L_G and the
// smallest eigenvalue of the pencil (L_G, L_P) is at least 1: kappa is at
// most lambda_max.  The estimate is the largest Ritz value of the pencil on
// the subspace reached by `steps` steps of Y <- L_P^+ L_G Y (subspace
// iteration with Rayleigh-Ritz after each step).  A Ritz value never exceeds
// lambda_max whatever the subspace (Courant-Fischer), so inexact inner solves
// only slow the approach from below.
//
// Inner solves L_P Y = Z: conjugate gradients on all k columns at once
// (per-column scalars in device memory, columns frozen once converged),
// preconditioned by the exact solve with P's spanning tree (tree.hip), each
// solve after the first started from the Ritz pairs (X = Y diag(theta)).
// Every block lives in the tree's preorder: G and P are relabelled once, so
// the tree solve needs no gathers and tree neighbours sit in nearby rows.
// HBM-bound: per iteration one Laplacian product on P (with p . Ap fused),
// the CG update (with r . r fused) and the tree solve (two block prefix sums,
// with r . z fused).
#include <algorithm>
#include <chrono>
#include <cmath>

#include "common.hpp"

namespace sfg {

size_t csr_workspace_bytes(int64_t n, int64_t m);
void build_csr(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
               const uint8_t *mask, int32_t *rowptr, int32_t *col, void *val, int32_t *eid, void *deg, void *ws,
               size_t ws_bytes, hipStream_t s);
void random_block(int64_t n, int32_t k, uint64_t seed, uint32_t block, double *x, hipStream_t s);
size_t tree_order_workspace_bytes(int64_t n, int64_t m);
void tree_order(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
                const uint8_t *keep, int32_t *order, int32_t *parent, int32_t *size, double *pw, int32_t *tdown,
                int32_t *tup, void *ws, size_t ws_bytes, hipStream_t s);
size_t tree_solve_workspace_bytes(int64_t n, int32_t k);
void tree_solve(const sfg_tree *T, int32_t k, const double *b, double *x, void *ws, size_t ws_bytes, hipStream_t s);
void block_dot(int64_t rows, int32_t k, const double *x, const double *y, double *out, double *scratch,
               hipStream_t s);
size_t colsum_scratch_doubles(int32_t k);
void block_colsum(int64_t rows, int32_t k, const double *x, double scale, double *out, double *scratch,
                  hipStream_t s);
size_t gram_scratch_doubles(int32_t k);
void block_gram(int64_t rows, int32_t k, const double *x, const double *y, double *out, double *scratch,
                hipStream_t s);
void convert_weights(const void *w, sfg_dtype wt, sfg_dtype want, int64_t m, void *out, hipStream_t s);
uint32_t lane_grid(int64_t rows, int32_t k);
size_t lane_partial_doubles(int32_t k);
void finish_partials(int32_t nb, int32_t k, const double *partial, double *out, hipStream_t s);
size_t tree_precond_workspace_bytes(int64_t n, int32_t k);
void tree_precond_pre(const sfg_tree *T, int32_t k, const double *r, double *z, double *rz, void *ws, hipStream_t s);

namespace {

constexpr int kB = 256;

// y = L_H x for an n x k block (Sec. 2.1): y_p = deg_p x_p - sum_q w_pq x_q
__global__ void k_lap(int64_t n, int32_t k, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                      const double *__restrict__ val, const double *__restrict__ deg, const double *__restrict__ x,
                      double *__restrict__ y) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int64_t p = t / k;
    const int c = (int)(t - p * k);
    double acc = 0.0;
    for (int32_t j = rowptr[p], e = rowptr[p + 1]; j < e; ++j) acc += val[j] * x[(int64_t)col[j] * k + c];
    y[t] = deg[p] * x[t] - acc;
}

__device__ __forceinline__ double safe_div(double a, double b) { return b != 0.0 ? a / b : 0.0; }

// p = z + beta p with beta_c = rz_new_c / rz_c on active columns (the mask
// `active`, or *dmask when the device keeps it)
__global__ void k_cg_dir(int64_t n, int32_t k, uint32_t active, const uint32_t *__restrict__ dmask,
                         const double *__restrict__ rz_new, const double *__restrict__ rz,
                         const double *__restrict__ z, double *__restrict__ p) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int c = (int)(t % k);
    const uint32_t act = dmask ? *dmask : active;
    if (!((act >> c) & 1u)) return;
    p[t] = z[t] + safe_div(rz_new[c], rz[c]) * p[t];
}

// Convergence test on the device, after each iteration: a column whose
// ||r||^2 is no longer above tol^2 ||z||^2 leaves the mask (the same test, on
// the same values, as the host makes otherwise); *dit counts the iterations
// that had an active column.
__global__ void k_cg_check(int32_t k, const double *__restrict__ rr, const double *__restrict__ zz, double tol2,
                           uint32_t *dmask, int64_t *dit) {
    if (threadIdx.x != 0) return;
    uint32_t m = *dmask;
    if (m) ++*dit;
    for (int c = 0; c < k; ++c)
        if (((m >> c) & 1u) && !(rr[c] > tol2 * zz[c])) m &= ~(1u << c);
    *dmask = m;
}

// Iterations between the host's reads of a device-kept convergence mask
// (after the first few, which are read at 1, 2, 4 and 8).
constexpr int kPoll = 16;

__global__ void k_cg_mask_init(uint32_t active, uint32_t *dmask, int64_t *dit) {
    if (threadIdx.x == 0) {
        *dmask = active;
        *dit = 0;
    }
}

__global__ void k_zero(int64_t cnt, double *__restrict__ x) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < cnt) x[t] = 0.0;
}

// ---- preorder relabelling: row i of the new CSR is row order[i] of the old
// one, entries in the same order with columns renamed; sums per row keep
// their order

__global__ void k_inverse(int64_t n, const int32_t *__restrict__ order, int32_t *__restrict__ inv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) inv[order[i]] = (int32_t)i;
}

__global__ void k_perm_len(int64_t n, const int32_t *__restrict__ order, const int32_t *__restrict__ rowptr,
                           int32_t *__restrict__ len) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t p = order[i];
    len[i] = rowptr[p + 1] - rowptr[p];
}

__global__ void k_perm_fill(int64_t n, const int32_t *__restrict__ order, const int32_t *__restrict__ inv,
                            const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                            const double *__restrict__ val, const double *__restrict__ deg,
                            const int32_t *__restrict__ nrowptr, int32_t *__restrict__ ncol,
                            double *__restrict__ nval, double *__restrict__ ndeg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t p = order[i];
    const int32_t a = rowptr[p], e = rowptr[p + 1], b = nrowptr[i];
    for (int32_t j = a; j < e; ++j) {
        ncol[b + (j - a)] = inv[col[j]];
        nval[b + (j - a)] = val[j];
    }
    ndeg[i] = deg[p];
}

__global__ void k_gather_rows(int64_t n, int32_t k, const int32_t *__restrict__ order, const double *__restrict__ src,
                              double *__restrict__ dst) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int64_t i = t / k;
    const int c = (int)(t - i * k);
    dst[t] = src[(int64_t)order[i] * k + c];
}

// ---- conjugate-gradient kernels in the row-lane layout: a workgroup is
// G x k threads (G = 256 / k), thread (g, c) owns column c of rows
// blockIdx * G + g + j * gridDim * G; per-workgroup column partial sums of a
// product go to partial[blockIdx][c] (reduced in a fixed order afterwards)

__device__ __forceinline__ void lane_reduce(double acc, int32_t k, double *sh, double *partial) {
    sh[threadIdx.x] = acc;
    __syncthreads();
    if ((int)threadIdx.x < k) {
        const int G = kB / k;
        double t = 0.0;
        for (int g = 0; g < G; ++g) t += sh[g * k + threadIdx.x];
        partial[(int64_t)blockIdx.x * k + threadIdx.x] = t;
    }
}

// y = L_H x and partial sums of x . y
__global__ __launch_bounds__(kB) void k_lap_dot(int64_t n, int32_t k, const int32_t *__restrict__ rowptr,
                                                const int32_t *__restrict__ col, const double *__restrict__ val,
                                                const double *__restrict__ deg, const double *__restrict__ x,
                                                double *__restrict__ y, double *__restrict__ partial) {
    __shared__ double sh[kB];
    const int G = kB / k;
    const int g = threadIdx.x / k, c = threadIdx.x % k;
    double acc = 0.0;
    if (g < G)
        for (int64_t p = (int64_t)blockIdx.x * G + g; p < n; p += (int64_t)gridDim.x * G) {
            double a = 0.0;
            for (int32_t j = rowptr[p], e = rowptr[p + 1]; j < e; ++j) a += val[j] * x[(int64_t)col[j] * k + c];
            const double xp = x[p * k + c];
            const double yp = deg[p] * xp - a;
            y[p * k + c] = yp;
            acc += xp * yp;
        }
    lane_reduce(acc, k, sh, partial);
}

// Same for even k, two adjacent columns per thread (16-byte loads and stores);
// the sums are added in the same order as k_lap_dot's
__global__ __launch_bounds__(kB) void k_lap_dot2(int64_t n, int32_t k, const int32_t *__restrict__ rowptr,
                                                 const int32_t *__restrict__ col, const double *__restrict__ val,
                                                 const double *__restrict__ deg, const double *__restrict__ x,
                                                 double *__restrict__ y, double *__restrict__ partial) {
    __shared__ double sh[2 * kB];
    const int kv = k >> 1;
    const int G = kB / kv;
    const int g = threadIdx.x / kv, c2 = threadIdx.x % kv;
    double acc0 = 0.0, acc1 = 0.0;
    if (g < G)
        for (int64_t p = (int64_t)blockIdx.x * G + g; p < n; p += (int64_t)gridDim.x * G) {
            double a0 = 0.0, a1 = 0.0;
            for (int32_t j = rowptr[p], e = rowptr[p + 1]; j < e; ++j) {
                const double w = val[j];
                const double2 xv = *reinterpret_cast<const double2 *>(x + (int64_t)col[j] * k + 2 * c2);
                a0 += w * xv.x;
                a1 += w * xv.y;
            }
            const double2 xp = *reinterpret_cast<const double2 *>(x + p * k + 2 * c2);
            const double d = deg[p];
            double2 yp;
            yp.x = d * xp.x - a0;
            yp.y = d * xp.y - a1;
            *reinterpret_cast<double2 *>(y + p * k + 2 * c2) = yp;
            acc0 += xp.x * yp.x;
            acc1 += xp.y * yp.y;
        }
    sh[2 * threadIdx.x] = acc0;
    sh[2 * threadIdx.x + 1] = acc1;
    __syncthreads();
    if ((int)threadIdx.x < k) {
        const int cc = threadIdx.x >> 1, half = threadIdx.x & 1;
        double t = 0.0;
        for (int gg = 0; gg < G; ++gg) t += sh[2 * (gg * kv + cc) + half];
        partial[(int64_t)blockIdx.x * k + threadIdx.x] = t;
    }
}

// r = z - L_H x
__global__ void k_lap_resid(int64_t n, int32_t k, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                            const double *__restrict__ val, const double *__restrict__ deg,
                            const double *__restrict__ x, const double *__restrict__ z, double *__restrict__ r) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int64_t p = t / k;
    const int c = (int)(t - p * k);
    double a = 0.0;
    for (int32_t j = rowptr[p], e = rowptr[p + 1]; j < e; ++j) a += val[j] * x[(int64_t)col[j] * k + c];
    r[t] = z[t] - (deg[p] * x[t] - a);
}

// x += alpha p, r -= alpha Ap (alpha_c = rz_c / pAp_c on active columns) and partial sums of r . r
__global__ __launch_bounds__(kB) void k_cg_step_rr(int64_t n, int32_t k, uint32_t active,
                                                   const uint32_t *__restrict__ dmask,
                                                   const double *__restrict__ rz, const double *__restrict__ pap,
                                                   const double *__restrict__ p, const double *__restrict__ ap,
                                                   double *__restrict__ x, double *__restrict__ r,
                                                   double *__restrict__ partial) {
    __shared__ double sh[kB];
    const int G = kB / k;
    const int g = threadIdx.x / k, c = threadIdx.x % k;
    const bool on = ((dmask ? *dmask : active) >> c) & 1u;
    const double a = on ? safe_div(rz[c], pap[c]) : 0.0;
    double acc = 0.0;
    if (g < G)
        for (int64_t i = (int64_t)blockIdx.x * G + g; i < n; i += (int64_t)gridDim.x * G) {
            const int64_t t = i * k + c;
            double ri = r[t];
            if (on) {
                x[t] += a * p[t];
                ri -= a * ap[t];
                r[t] = ri;
            }
            acc += ri * ri;
        }
    lane_reduce(acc, k, sh, partial);
}

// x = y diag(theta): the Ritz pairs' image under L_P^+ L_G, a warm start
__global__ void k_scale_cols(int64_t n, int32_t k, const double *__restrict__ y, const double *__restrict__ theta,
                             double *__restrict__ x) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    x[t] = y[t] * theta[t % k];
}

// out = X V for an n x k block and a k x k matrix V (row-major)
__global__ __launch_bounds__(kB) void k_rotate(int64_t n, int32_t k, const double *__restrict__ x,
                                               const double *__restrict__ V, double *__restrict__ out) {
    __shared__ double sv[32 * 32];
    for (int e = threadIdx.x; e < k * k; e += kB) sv[e] = V[e];
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int64_t p = t / k;
    const int j = (int)(t - p * k);
    double acc = 0.0;
    for (int i = 0; i < k; ++i) acc += x[p * k + i] * sv[i * k + j];
    out[t] = acc;
}

// ------------------------------------------------------------------ host: small generalized eigenproblem

// A v = theta B v for symmetric A and positive definite B (k x k, row-major):
// Cholesky B = L L^T, cyclic Jacobi on C = L^-1 A L^-T, V = L^-T Q so that
// V^T B V = I.  Returns false when B is not numerically positive definite.
bool gen_eig(int k, std::vector<double> A, std::vector<double> B, std::vector<double> &theta,
             std::vector<double> &V) {
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < i; ++j) {
            const double a = 0.5 * (A[i * k + j] + A[j * k + i]), b = 0.5 * (B[i * k + j] + B[j * k + i]);
            A[i * k + j] = A[j * k + i] = a;
            B[i * k + j] = B[j * k + i] = b;
        }
    std::vector<double> L(k * k, 0.0);
    double bmax = 0.0;
    for (int i = 0; i < k; ++i) bmax = std::max(bmax, std::fabs(B[i * k + i]));
    for (int j = 0; j < k; ++j) {
        double d = B[j * k + j];
        for (int t = 0; t < j; ++t) d -= L[j * k + t] * L[j * k + t];
        if (!(d > 1e-14 * bmax)) return false;
        L[j * k + j] = std::sqrt(d);
        for (int i = j + 1; i < k; ++i) {
            double x = B[i * k + j];
            for (int t = 0; t < j; ++t) x -= L[i * k + t] * L[j * k + t];
            L[i * k + j] = x / L[j * k + j];
        }
    }
    // X = L^-1 A, then C = L^-1 X^T (= L^-1 A L^-T)
    auto lsolve = [&](std::vector<double> &M) {   // in place, column by column
        for (int c = 0; c < k; ++c)
            for (int i = 0; i < k; ++i) {
                double x = M[i * k + c];
                for (int t = 0; t < i; ++t) x -= L[i * k + t] * M[t * k + c];
                M[i * k + c] = x / L[i * k + i];
            }
    };
    std::vector<double> X = A;
    lsolve(X);
    std::vector<double> C(k * k);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) C[i * k + j] = X[j * k + i];
    lsolve(C);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < i; ++j) C[i * k + j] = C[j * k + i] = 0.5 * (C[i * k + j] + C[j * k + i]);
    std::vector<double> Q(k * k, 0.0);
    for (int i = 0; i < k; ++i) Q[i * k + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int i = 0; i < k; ++i) {
            dia += C[i * k + i] * C[i * k + i];
            for (int j = i + 1; j < k; ++j) off += C[i * k + j] * C[i * k + j];
        }
        if (off <= 1e-30 * dia || off == 0.0) break;
        for (int p = 0; p < k; ++p)
            for (int q = p + 1; q < k; ++q) {
                const double apq = C[p * k + q];
                if (apq == 0.0) continue;
                const double th = (C[q * k + q] - C[p * k + p]) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int r = 0; r < k; ++r) {   // columns p, q
                    const double a = C[r * k + p], b = C[r * k + q];
                    C[r * k + p] = cs * a - sn * b;
                    C[r * k + q] = sn * a + cs * b;
                }
                for (int r = 0; r < k; ++r) {   // rows p, q
                    const double a = C[p * k + r], b = C[q * k + r];
                    C[p * k + r] = cs * a - sn * b;
                    C[q * k + r] = sn * a + cs * b;
                }
                for (int r = 0; r < k; ++r) {
                    const double a = Q[r * k + p], b = Q[r * k + q];
                    Q[r * k + p] = cs * a - sn * b;
                    Q[r * k + q] = sn * a + cs * b;
                }
            }
    }
    theta.assign(k, 0.0);
    for (int i = 0; i < k; ++i) theta[i] = C[i * k + i];
    // V = L^-T Q: back substitution per column
    V = Q;
    for (int c = 0; c < k; ++c)
        for (int i = k - 1; i >= 0; --i) {
            double x = V[i * k + c];
            for (int t = i + 1; t < k; ++t) x -= L[t * k + i] * V[t * k + c];
            V[i * k + c] = x / L[i * k + i];
        }
    return true;
}

}  // namespace

// ------------------------------------------------------------------ estimator

// Preorder CSR (F64) of one graph.
struct PreCsr {
    int32_t *rowptr, *col, *len;
    double *val, *deg;
};

struct KappaEstimator {
    int64_t n, m;
    int32_t k;
    const int32_t *u, *v;
    const double *w64;
    hipStream_t s;
    // CSR in node order (build target) and in the tree's preorder
    int32_t *o_rowptr, *o_col, *o_eid;
    double *o_val, *o_deg;
    PreCsr G, P;
    int32_t *scan_scr;
    int32_t *t_order, *t_parent, *t_size, *t_tdown, *t_tup, *inv;
    double *t_pw;
    sfg_tree T;
    void *csr_ws, *pre_ws;
    size_t csr_wsb;
    // n x k blocks in preorder
    double *Y, *Z, *X, *R, *Zp, *Pd, *AP, *W, *VP;
    double *small, *part, *gram_scr;

    PreCsr alloc_pre(DevArena &A) {
        PreCsr c;
        c.rowptr = A.alloc<int32_t>(n + 1);
        c.len = A.alloc<int32_t>(n + 1);
        c.col = A.alloc<int32_t>(2 * m + 1);
        c.val = A.alloc<double>(2 * m + 1);
        c.deg = A.alloc<double>(n + 1);
        return c;
    }

    // node-order CSR of the edges with mask != 0 (NULL = all), relabelled into preorder
    void build_pre(const uint8_t *mask, PreCsr &c) {
        build_csr(n, m, u, v, w64, SFG_F64, mask, o_rowptr, o_col, o_val, o_eid, o_deg, csr_ws, csr_wsb, s);
        const dim3 gn(grid_for(n, kB)), b(kB);
        hipLaunchKernelGGL(k_perm_len, gn, b, 0, s, n, t_order, o_rowptr, c.len);
        SFG_LAUNCH_CHECK();
        exclusive_scan_i32(c.len, c.rowptr, n, scan_scr, s);
        hipLaunchKernelGGL(k_perm_fill, gn, b, 0, s, n, t_order, inv, o_rowptr, o_col, o_val, o_deg, c.rowptr,
                           c.col, c.val, c.deg);
        SFG_LAUNCH_CHECK();
    }

    KappaEstimator(int64_t n_, int64_t m_, const int32_t *u_, const int32_t *v_, const double *w64_,
                   const uint8_t *tree_marks, int32_t k_, DevArena &A, hipStream_t s_)
        : n(n_), m(m_), k(k_), u(u_), v(v_), w64(w64_), s(s_) {
        const size_t nk = (size_t)n * k;
        csr_wsb = csr_workspace_bytes(n, m);
        csr_ws = A.raw(csr_wsb);
        o_rowptr = A.alloc<int32_t>(n + 1);
        o_col = A.alloc<int32_t>(2 * m + 1);
        o_eid = A.alloc<int32_t>(2 * m + 1);
        o_val = A.alloc<double>(2 * m + 1);
        o_deg = A.alloc<double>(n + 1);
        scan_scr = A.alloc<int32_t>(scan_scratch_ints(n + 1));
        t_order = A.alloc<int32_t>(n + 1);
        t_parent = A.alloc<int32_t>(n + 1);
        t_size = A.alloc<int32_t>(n + 1);
        t_tdown = A.alloc<int32_t>(n + 1);
        t_tup = A.alloc<int32_t>(n + 1);
        t_pw = A.alloc<double>(n + 1);
        inv = A.alloc<int32_t>(n + 1);
        {
            const size_t b = tree_order_workspace_bytes(n, m);
            tree_order(n, m, u, v, w64, SFG_F64, tree_marks, t_order, t_parent, t_size, t_pw, t_tdown, t_tup,
                       A.raw(b), b, s);
        }
        T = sfg_tree{n, t_order, t_parent, t_size, t_pw, t_tdown, t_tup};
        hipLaunchKernelGGL(k_inverse, dim3(grid_for(n, kB)), dim3(kB), 0, s, n, t_order, inv);
        SFG_LAUNCH_CHECK();
        G = alloc_pre(A);
        P = alloc_pre(A);
        build_pre(nullptr, G);
        pre_ws = A.raw(tree_precond_workspace_bytes(n, k));
        double **blocks[] = {&Y, &Z, &X, &R, &Zp, &Pd, &AP, &W, &VP};
        for (double **bl : blocks) *bl = A.alloc<double>(nk + 1);
        small = A.alloc<double>(16 * 64 + 3 * 32 * 32);
        part = A.alloc<double>(lane_partial_doubles(k));
        gram_scr = A.alloc<double>(gram_scratch_doubles(k));
    }

    void lap(const PreCsr &c, const double *x, double *y) {
        hipLaunchKernelGGL(k_lap, dim3(grid_for(n * k, kB)), dim3(kB), 0, s, n, k, c.rowptr, c.col, c.val, c.deg, x,
                           y);
        SFG_LAUNCH_CHECK();
    }

    std::vector<double> to_host(const double *d, int cnt) {
        std::vector<double> h(cnt);
        SFG_HIP(hipMemcpyAsync(h.data(), d, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
        SFG_HIP(hipStreamSynchronize(s));
        return h;
    }

    // X = L_P^+ Z (up to constants) by tree-preconditioned CG on all columns,
    // from X = Y diag(theta) when theta is given, else from 0.  A column stops
    // when ||r|| <= tol ||Z||.  Returns the iterations; *hit_cap at the cap.
    // check_every: convergence test every so many iterations (each costs a wait
    // for the host); an exact preconditioner (P = its tree) converges in one.
    // check_every = 0: the test runs on the device after every iteration (a
    // converged column stops changing at once, as with a host test every
    // iteration) and the host only polls the mask every kPoll iterations.
    int64_t solve(double tol, int32_t max_iter, const double *theta, bool *hit_cap, int check_every = 4) {
        double *rz0 = small, *rz1 = small + 64, *pap = small + 128, *rr = small + 192, *zz = small + 256;
        const dim3 g(grid_for(n * k, kB)), b(kB);
        const uint32_t lg = lane_grid(n, k);
        const uint32_t lg2 = k % 2 == 0 ? lane_grid(n, k / 2) : lg;   // two columns per thread
        block_dot(n, k, Z, Z, zz, part, s);
        if (theta) {
            hipLaunchKernelGGL(k_scale_cols, g, b, 0, s, n, k, Y, theta, X);
            SFG_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_lap_resid, g, b, 0, s, n, k, P.rowptr, P.col, P.val, P.deg, X, Z, R);
            SFG_LAUNCH_CHECK();
        } else {
            hipLaunchKernelGGL(k_zero, g, b, 0, s, n * k, X);
            SFG_LAUNCH_CHECK();
            SFG_HIP(hipMemcpyAsync(R, Z, (size_t)n * k * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
        block_dot(n, k, R, R, rr, part, s);
        const std::vector<double> hz = to_host(zz, k), h0 = to_host(rr, k);
        uint32_t active = 0;
        for (int c = 0; c < k; ++c)
            if (h0[c] > tol * tol * hz[c]) active |= 1u << c;
        *hit_cap = false;
        if (!active) return 0;
        tree_precond_pre(&T, k, R, Zp, rz0, pre_ws, s);
        SFG_HIP(hipMemcpyAsync(Pd, Zp, (size_t)n * k * sizeof(double), hipMemcpyDeviceToDevice, s));
        const bool dev_check = check_every == 0;
        const int kCheck = dev_check ? kPoll : (check_every < 1 ? 1 : check_every);
        uint32_t *dmask = nullptr;
        int64_t *dit = nullptr;
        if (dev_check) {
            dmask = reinterpret_cast<uint32_t *>(small + 320 + 64);
            dit = reinterpret_cast<int64_t *>(small + 320 + 65);
            hipLaunchKernelGGL(k_cg_mask_init, dim3(1), dim3(64), 0, s, active, dmask, dit);
            SFG_LAUNCH_CHECK();
        }
        const double tol2 = tol * tol;
        int64_t it = 0;
        while (active) {
            if (it == max_iter) {
                *hit_cap = true;
                break;
            }
            ++it;
            if (k % 2 == 0)
                hipLaunchKernelGGL(k_lap_dot2, dim3(lg2), dim3(kB), 0, s, n, k, P.rowptr, P.col, P.val, P.deg, Pd, AP,
                                   part);
            else
                hipLaunchKernelGGL(k_lap_dot, dim3(lg), dim3(kB), 0, s, n, k, P.rowptr, P.col, P.val, P.deg, Pd, AP,
                                   part);
            SFG_LAUNCH_CHECK();
            finish_partials((int32_t)(k % 2 == 0 ? lg2 : lg), k, part, pap, s);
            hipLaunchKernelGGL(k_cg_step_rr, dim3(lg), dim3(kB), 0, s, n, k, active, dmask, rz0, pap, Pd, AP, X, R,
                               part);
            SFG_LAUNCH_CHECK();
            finish_partials((int32_t)lg, k, part, rr, s);
            tree_precond_pre(&T, k, R, Zp, rz1, pre_ws, s);
            hipLaunchKernelGGL(k_cg_dir, g, b, 0, s, n, k, active, dmask, rz1, rz0, Zp, Pd);
            SFG_LAUNCH_CHECK();
            std::swap(rz0, rz1);
            if (dev_check) {
                hipLaunchKernelGGL(k_cg_check, dim3(1), dim3(64), 0, s, k, rr, zz, tol2, dmask, dit);
                SFG_LAUNCH_CHECK();
                // polls after iterations 1, 2, 4, 8, then every kPoll: a solve that converges at once (an
                // exact preconditioner) is not run on for kPoll iterations
                const bool poll = (it < kPoll && (it & (it - 1)) == 0) || it % kCheck == 0 || it == max_iter;
                if (poll) {
                    uint32_t hm = 0;
                    SFG_HIP(hipMemcpyAsync(&hm, dmask, sizeof(hm), hipMemcpyDeviceToHost, s));
                    SFG_HIP(hipStreamSynchronize(s));
                    active = hm;
                }
            } else if (it % kCheck == 0 || it == max_iter) {
                const std::vector<double> h = to_host(rr, k);
                for (int c = 0; c < k; ++c)
                    if (((active >> c) & 1u) && !(h[c] > tol2 * hz[c])) active &= ~(1u << c);
            }
        }
        if (dev_check) {
            // iterations after every column had converged changed nothing: count the ones that did
            int64_t hit = 0;
            SFG_HIP(hipMemcpyAsync(&hit, dit, sizeof(hit), hipMemcpyDeviceToHost, s));
            SFG_HIP(hipStreamSynchronize(s));
            return hit;
        }
        return it;
    }

    // one estimate for the sparsifier keep != 0 (its edges marked 1 must be
    // the tree this estimator was built with); y0 in node order or NULL
    double run(const uint8_t *keep, const sfg_kappa_params &kp, const double *y0, uint64_t seed, uint32_t block,
               sfg_kappa_report *rep) {
        const auto t0 = std::chrono::steady_clock::now();
        build_pre(keep, P);
        const dim3 g(grid_for(n * k, kB)), b(kB);
        // starting block (node order) into preorder; constants need no removal: they
        // are in the kernel of both Laplacians
        if (y0) {
            hipLaunchKernelGGL(k_gather_rows, g, b, 0, s, n, k, t_order, y0, Y);
        } else {
            random_block(n, k, seed, block, W, s);
            hipLaunchKernelGGL(k_gather_rows, g, b, 0, s, n, k, t_order, W, Y);
        }
        SFG_LAUNCH_CHECK();
        lap(G, Y, Z);
        double *Ad = small + 16 * 64, *Bd = Ad + 32 * 32, *Vd = Bd + 32 * 32, *thd = small + 320;
        double est = 0.0;
        int64_t iters = 0;
        int32_t max_inner = 0, uncon = 0;
        bool warm = false;
        for (int32_t t = 0; t < kp.steps; ++t) {
            bool cap = false;
            const int64_t it = solve(kp.tol, kp.max_iter, warm ? thd : nullptr, &cap);
            iters += it;
            max_inner = std::max<int32_t>(max_inner, (int32_t)it);
            uncon += cap ? 1 : 0;
            lap(G, X, W);
            lap(P, X, VP);
            block_gram(n, k, X, W, Ad, gram_scr, s);
            block_gram(n, k, X, VP, Bd, gram_scr, s);
            const std::vector<double> Ah = to_host(Ad, k * k), Bh = to_host(Bd, k * k);
            std::vector<double> theta, V;
            if (!gen_eig(k, Ah, Bh, theta, V))
                fail(SFG_ENUMERIC, "kappa_estimate: the block lost rank (k too large for the graph?)");
            est = *std::max_element(theta.begin(), theta.end());
            if (!(est == est) || std::isinf(est)) fail(SFG_ENUMERIC, "kappa_estimate: NaN or Inf Ritz value");
            if (rep && t < 64) rep->ritz[t] = est;
            SFG_HIP(hipMemcpyAsync(Vd, V.data(), k * k * sizeof(double), hipMemcpyHostToDevice, s));
            SFG_HIP(hipMemcpyAsync(thd, theta.data(), k * sizeof(double), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_rotate, g, b, 0, s, n, k, X, Vd, Y);
            SFG_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_rotate, g, b, 0, s, n, k, W, Vd, Z);
            SFG_LAUNCH_CHECK();
            SFG_HIP(hipStreamSynchronize(s));   // V and theta live on the host stack
            warm = true;
        }
        if (rep) {
            rep->kappa = est;
            rep->steps = kp.steps;
            rep->inner_iters = iters;
            rep->max_inner = max_inner;
            rep->unconverged = uncon;
            rep->ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        return est;
    }
};

sfg_kappa_params kappa_defaults(const sfg_kappa_params *in) {
    sfg_kappa_params p{};
    if (in) p = *in;
    if (p.k == 0) p.k = 8;
    if (p.steps == 0) p.steps = 6;
    if (p.tol == 0.0) p.tol = 1e-1;
    if (p.max_iter == 0) p.max_iter = 20000;
    return p;
}

void check_kappa_params(const sfg_kappa_params &p, int64_t n) {
    SFG_REQUIRE(p.k >= 1 && p.k <= 32, SFG_EINVAL, "kappa_estimate: k must be in 1..32");
    SFG_REQUIRE(p.k <= n - 1, SFG_EINVAL, "kappa_estimate: k must be at most n - 1");
    SFG_REQUIRE(p.steps >= 1 && p.steps <= 64, SFG_EINVAL, "kappa_estimate: steps must be in 1..64");
    SFG_REQUIRE(p.tol > 0.0 && p.tol < 1.0, SFG_EINVAL, "kappa_estimate: tol must be in (0, 1)");
    SFG_REQUIRE(p.max_iter >= 1, SFG_EINVAL, "kappa_estimate: max_iter must be >= 1");
}

// Estimator bound to one graph and one spanning tree (reused over the
// batches of sigma-driven stopping).
KappaEstimator *make_kappa_estimator(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const double *w64,
                                     const uint8_t *tree_marks, int32_t k, DevArena &A, hipStream_t s) {
    return new KappaEstimator(n, m, u, v, w64, tree_marks, k, A, s);
}

double run_kappa_estimator(KappaEstimator *e, const uint8_t *keep, const sfg_kappa_params &kp, uint64_t seed,
                           uint32_t block, sfg_kappa_report *rep) {
    return e->run(keep, kp, nullptr, seed, block, rep);
}

void free_kappa_estimator(KappaEstimator *e) { delete e; }

}  // namespace sfg

// ------------------------------------------------------------------ downstream PCG (Sec. 4)

namespace sfg {

namespace {

// grounded right-hand side for the preconditioner: the consistent singular
// system L_P z = rt with rt = r off node 0 and rt_0 = -sum(r) (r_0 = 0)
__global__ void k_ground_rhs(int64_t n, const double *__restrict__ r, const double *__restrict__ sum,
                             double *__restrict__ rt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) rt[i] = i == 0 ? -sum[0] : r[i];
}

// z = x - x_0: the solution grounded at node 0 (preorder position 0)
__global__ void k_shift0(int64_t n, const double *__restrict__ x, double *__restrict__ z) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = x[i] - x[0];
}

__global__ void k_zero_first(double *a) { a[0] = 0.0; }

// x += alpha p, r -= alpha q with alpha = rz / pq
__global__ void k_pcg_step(int64_t n, const double *__restrict__ rz, const double *__restrict__ pq,
                           const double *__restrict__ p, const double *__restrict__ q, double *__restrict__ x,
                           double *__restrict__ r) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double alpha = rz[0] / pq[0];
    x[i] += alpha * p[i];
    r[i] -= alpha * q[i];
}

// p = z + (rz_new / rz) p
__global__ void k_pcg_dir(int64_t n, const double *__restrict__ rzn, const double *__restrict__ rz,
                          const double *__restrict__ z, double *__restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = z[i] + (rzn[0] / rz[0]) * p[i];
}

}  // namespace

// Conjugate gradients on L_G x = b grounded at node 0 (row and column 0
// removed; x_0 = 0), preconditioned by solves with the sparsifier's grounded
// Laplacian, each done by the tree-preconditioned CG of the estimate to a
// relative residual inner_tol: the downstream use of the sparsifier in the
// paper's evaluation.  Stops when ||r|| <= tol ||b|| (b_0 ignored).
int64_t run_pcg(KappaEstimator &e, const uint8_t *keep, const double *b, double *x_out, double tol,
                int32_t max_iter, double inner_tol, int32_t inner_max, sfg_pcg_report *rep, DevArena &A) {
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = e.s;
    const int64_t n = e.n;
    e.build_pre(keep, e.P);
    double *bx = A.alloc<double>(n + 1), *x = A.alloc<double>(n + 1), *r = A.alloc<double>(n + 1);
    double *z = A.alloc<double>(n + 1), *pv = A.alloc<double>(n + 1), *q = A.alloc<double>(n + 1);
    double *sc = A.alloc<double>(16);   // rz, rz_new, pq, rr, bb, sum
    double *scr = A.alloc<double>(colsum_scratch_doubles(1) + 64);
    double *rz = sc, *rzn = sc + 1, *pq = sc + 2, *rr = sc + 3, *bb = sc + 4, *sum = sc + 5;
    const dim3 g(grid_for(n, kB)), blk(kB);
    hipLaunchKernelGGL(k_gather_rows, g, blk, 0, s, n, 1, e.t_order, b, bx);   // node order -> preorder
    SFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_zero_first, dim3(1), dim3(1), 0, s, bx);               // node 0 is preorder position 0
    SFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_zero, g, blk, 0, s, n, x);
    SFG_LAUNCH_CHECK();
    SFG_HIP(hipMemcpyAsync(r, bx, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    block_dot(n, 1, bx, bx, bb, scr, s);
    const double nb = std::sqrt(e.to_host(bb, 1)[0]);
    int64_t inner = 0;
    bool capped = false;
    auto precond = [&](const double *rin, double *zout) {
        block_colsum(n, 1, rin, 1.0, sum, scr, s);
        hipLaunchKernelGGL(k_ground_rhs, g, blk, 0, s, n, rin, sum, e.Z);
        SFG_LAUNCH_CHECK();
        bool cap = false;
        // tested after every iteration, on the device: iterations past
        // convergence would only add rounding noise, which the tree solve
        // amplifies, to the preconditioner
        inner += e.solve(inner_tol, inner_max, nullptr, &cap, 0);
        capped = capped || cap;
        hipLaunchKernelGGL(k_shift0, g, blk, 0, s, n, e.X, zout);
        SFG_LAUNCH_CHECK();
    };
    int64_t it = 0;
    double relres = nb > 0 ? 1.0 : 0.0;
    bool converged = nb == 0.0;
    if (!converged) {
        precond(r, z);
        SFG_HIP(hipMemcpyAsync(pv, z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        block_dot(n, 1, r, z, rz, scr, s);
        while (it < max_iter) {
            ++it;
            e.lap(e.G, pv, q);
            hipLaunchKernelGGL(k_zero_first, dim3(1), dim3(1), 0, s, q);       // row 0 removed
            SFG_LAUNCH_CHECK();
            block_dot(n, 1, pv, q, pq, scr, s);
            hipLaunchKernelGGL(k_pcg_step, g, blk, 0, s, n, rz, pq, pv, q, x, r);
            SFG_LAUNCH_CHECK();
            block_dot(n, 1, r, r, rr, scr, s);
            relres = std::sqrt(e.to_host(rr, 1)[0]) / nb;
            if (relres <= tol) {
                converged = true;
                break;
            }
            precond(r, z);
            block_dot(n, 1, r, z, rzn, scr, s);
            hipLaunchKernelGGL(k_pcg_dir, g, blk, 0, s, n, rzn, rz, z, pv);
            SFG_LAUNCH_CHECK();
            std::swap(rz, rzn);
        }
    }
    if (x_out) {
        hipLaunchKernelGGL(k_gather_rows, g, blk, 0, s, n, 1, e.inv, x, x_out);   // preorder -> node order
        SFG_LAUNCH_CHECK();
    }
    SFG_HIP(hipStreamSynchronize(s));
    if (rep) {
        rep->iters = it;
        rep->inner_iters = inner;
        rep->relres = relres;
        rep->converged = converged ? 1 : 0;
        rep->inner_capped = capped ? 1 : 0;
        rep->ms = (float)std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return it;
}

}  // namespace sfg

extern "C" sfg_status sfg_pcg(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
                              const uint8_t *keep, const double *b, double *x, double tol, int32_t max_iter,
                              sfg_pcg_report *rep, void *stream) {
    return sfg::guard([&] {
        hipStream_t s = sfg::as_stream(stream);
        SFG_REQUIRE(n >= 2 && m >= 1, SFG_EINVAL, "pcg: need n >= 2 and m >= 1");
        SFG_REQUIRE(2 * m < (int64_t(1) << 31), SFG_EUNSUPPORTED, "pcg: 2*m must be < 2^31");
        SFG_REQUIRE(wt == SFG_F64 || wt == SFG_F32, SFG_EINVAL, "pcg: weights must be F64 or F32");
        SFG_REQUIRE(u && v && w && keep && b, SFG_EINVAL, "pcg: null pointer");
        SFG_REQUIRE(tol > 0.0 && tol < 1.0, SFG_EINVAL, "pcg: tol must be in (0, 1)");
        SFG_REQUIRE(max_iter >= 1, SFG_EINVAL, "pcg: max_iter must be >= 1");
        if (rep) std::memset(rep, 0, sizeof(*rep));
        sfg::DevArena A(s);
        double *w64 = A.alloc<double>(m + 1);
        sfg::convert_weights(w, wt, SFG_F64, m, w64, s);
        sfg::KappaEstimator e(n, m, u, v, w64, keep, 1, A, s);
        sfg::run_pcg(e, keep, b, x, tol, max_iter, 1e-6, 20000, rep, A);
        A.finish();
    });
}

extern "C" sfg_status sfg_kappa_estimate(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w,
                                         sfg_dtype wt, const uint8_t *keep, const sfg_kappa_params *kp,
                                         const double *y0, double *kappa, sfg_kappa_report *rep, void *stream) {
    return sfg::guard([&] {
        hipStream_t s = sfg::as_stream(stream);
        SFG_REQUIRE(n >= 2 && m >= 1, SFG_EINVAL, "kappa_estimate: need n >= 2 and m >= 1");
        SFG_REQUIRE(2 * m < (int64_t(1) << 31), SFG_EUNSUPPORTED, "kappa_estimate: 2*m must be < 2^31");
        SFG_REQUIRE(wt == SFG_F64 || wt == SFG_F32, SFG_EINVAL, "kappa_estimate: weights must be F64 or F32");
        SFG_REQUIRE(u && v && w && keep && kappa, SFG_EINVAL, "kappa_estimate: null pointer");
        const sfg_kappa_params p = sfg::kappa_defaults(kp);
        sfg::check_kappa_params(p, n);
        if (rep) std::memset(rep, 0, sizeof(*rep));
        sfg::DevArena A(s);
        double *w64 = A.alloc<double>(m + 1);
        sfg::convert_weights(w, wt, SFG_F64, m, w64, s);
        sfg::KappaEstimator e(n, m, u, v, w64, keep, p.k, A, s);
        *kappa = e.run(keep, p, y0, p.seed, p.block, rep);
        A.finish();
    });
}
