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
// preconditioned by the exact solve with P's spanning tree (tree.hip).
// HBM-bound: per iteration one Laplacian product on P, one tree solve and
// three column reductions over n x k FP64 blocks.
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
size_t colsum_scratch_doubles(int32_t k);
void block_colsum(int64_t rows, int32_t k, const double *x, double scale, double *out, double *scratch,
                  hipStream_t s);
void block_dot(int64_t rows, int32_t k, const double *x, const double *y, double *out, double *scratch,
               hipStream_t s);
size_t gram_scratch_doubles(int32_t k);
void block_gram(int64_t rows, int32_t k, const double *x, const double *y, double *out, double *scratch,
                hipStream_t s);
void convert_weights(const void *w, sfg_dtype wt, sfg_dtype want, int64_t m, void *out, hipStream_t s);

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

// x += alpha p, r -= alpha Ap with alpha_c = rz_c / pAp_c on active columns
__global__ void k_cg_step(int64_t n, int32_t k, uint32_t active, const double *__restrict__ rz,
                          const double *__restrict__ pap, const double *__restrict__ p, const double *__restrict__ ap,
                          double *__restrict__ x, double *__restrict__ r) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int c = (int)(t % k);
    if (!((active >> c) & 1u)) return;
    const double a = safe_div(rz[c], pap[c]);
    x[t] += a * p[t];
    r[t] -= a * ap[t];
}

// p = z + beta p with beta_c = rz_new_c / rz_c on active columns
__global__ void k_cg_dir(int64_t n, int32_t k, uint32_t active, const double *__restrict__ rz_new,
                         const double *__restrict__ rz, const double *__restrict__ z, double *__restrict__ p) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int c = (int)(t % k);
    if (!((active >> c) & 1u)) return;
    p[t] = z[t] + safe_div(rz_new[c], rz[c]) * p[t];
}

__global__ void k_zero(int64_t cnt, double *__restrict__ x) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < cnt) x[t] = 0.0;
}

__global__ void k_subtract_mean(int64_t n, int32_t k, const double *__restrict__ mean, double *__restrict__ x) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    x[t] -= mean[t % k];
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

struct KappaEstimator {
    int64_t n, m;
    int32_t k;
    const int32_t *u, *v;
    const double *w64;
    hipStream_t s;
    // G and P (F64 CSR), the tree
    int32_t *g_rowptr, *g_col, *g_eid, *p_rowptr, *p_col, *p_eid;
    double *g_val, *g_deg, *p_val, *p_deg;
    int32_t *t_order, *t_parent, *t_size, *t_tdown, *t_tup;
    double *t_pw;
    sfg_tree T;
    void *csr_ws;
    size_t csr_wsb;
    void *ts_ws;
    size_t ts_wsb;
    // n x k blocks
    double *Y, *Z, *X, *R, *Zp, *Pd, *AP, *W, *VP;
    double *dev_small;   // rz (2 x 64), pap, rr, rr0, means, A, B, V
    double *red_scr, *gram_scr;

    KappaEstimator(int64_t n_, int64_t m_, const int32_t *u_, const int32_t *v_, const double *w64_,
                   const uint8_t *tree_marks, int32_t k_, DevArena &A, hipStream_t s_)
        : n(n_), m(m_), k(k_), u(u_), v(v_), w64(w64_), s(s_) {
        const size_t nk = (size_t)n * k;
        csr_wsb = csr_workspace_bytes(n, m);
        csr_ws = A.raw(csr_wsb);
        g_rowptr = A.alloc<int32_t>(n + 1);
        g_col = A.alloc<int32_t>(2 * m + 1);
        g_eid = A.alloc<int32_t>(2 * m + 1);
        g_val = A.alloc<double>(2 * m + 1);
        g_deg = A.alloc<double>(n + 1);
        p_rowptr = A.alloc<int32_t>(n + 1);
        p_col = A.alloc<int32_t>(2 * m + 1);
        p_eid = A.alloc<int32_t>(2 * m + 1);
        p_val = A.alloc<double>(2 * m + 1);
        p_deg = A.alloc<double>(n + 1);
        build_csr(n, m, u, v, w64, SFG_F64, nullptr, g_rowptr, g_col, g_val, g_eid, g_deg, csr_ws, csr_wsb, s);
        t_order = A.alloc<int32_t>(n + 1);
        t_parent = A.alloc<int32_t>(n + 1);
        t_size = A.alloc<int32_t>(n + 1);
        t_tdown = A.alloc<int32_t>(n + 1);
        t_tup = A.alloc<int32_t>(n + 1);
        t_pw = A.alloc<double>(n + 1);
        {
            const size_t b = tree_order_workspace_bytes(n, m);
            tree_order(n, m, u, v, w64, SFG_F64, tree_marks, t_order, t_parent, t_size, t_pw, t_tdown, t_tup,
                       A.raw(b), b, s);
        }
        T = sfg_tree{n, t_order, t_parent, t_size, t_pw, t_tdown, t_tup};
        ts_wsb = tree_solve_workspace_bytes(n, k);
        ts_ws = A.raw(ts_wsb);
        double **blocks[] = {&Y, &Z, &X, &R, &Zp, &Pd, &AP, &W, &VP};
        for (double **b : blocks) *b = A.alloc<double>(nk + 1);
        dev_small = A.alloc<double>(16 * 64 + 3 * 32 * 32);
        red_scr = A.alloc<double>(colsum_scratch_doubles(k));
        gram_scr = A.alloc<double>(gram_scratch_doubles(k));
    }

    void lap(bool on_g, const double *x, double *y) {
        hipLaunchKernelGGL(k_lap, dim3(grid_for(n * k, kB)), dim3(kB), 0, s, n, k, on_g ? g_rowptr : p_rowptr,
                           on_g ? g_col : p_col, on_g ? g_val : p_val, on_g ? g_deg : p_deg, x, y);
        SFG_LAUNCH_CHECK();
    }

    std::vector<double> to_host(const double *d, int cnt) {
        std::vector<double> h(cnt);
        SFG_HIP(hipMemcpyAsync(h.data(), d, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
        SFG_HIP(hipStreamSynchronize(s));
        return h;
    }

    // X = L_P^+ Z by tree-preconditioned CG, all columns at once.  Returns
    // the iterations taken; *hit_cap set when the cap was reached.
    int64_t solve(double tol, int32_t max_iter, bool *hit_cap) {
        double *rz0 = dev_small, *rz1 = dev_small + 64, *pap = dev_small + 128, *rr = dev_small + 192,
               *rr0 = dev_small + 256;
        const dim3 g(grid_for(n * k, kB)), b(kB);
        hipLaunchKernelGGL(k_zero, g, b, 0, s, n * k, X);
        SFG_LAUNCH_CHECK();
        SFG_HIP(hipMemcpyAsync(R, Z, (size_t)n * k * sizeof(double), hipMemcpyDeviceToDevice, s));
        block_dot(n, k, R, R, rr0, red_scr, s);
        const std::vector<double> h0 = to_host(rr0, k);
        uint32_t active = 0;
        for (int c = 0; c < k; ++c)
            if (h0[c] > 0.0) active |= 1u << c;
        *hit_cap = false;
        if (!active) return 0;
        tree_solve(&T, k, R, Zp, ts_ws, ts_wsb, s);
        SFG_HIP(hipMemcpyAsync(Pd, Zp, (size_t)n * k * sizeof(double), hipMemcpyDeviceToDevice, s));
        block_dot(n, k, R, Zp, rz0, red_scr, s);
        const int kCheck = 4;
        int64_t it = 0;
        while (active) {
            if (it == max_iter) {
                *hit_cap = true;
                break;
            }
            ++it;
            lap(false, Pd, AP);
            block_dot(n, k, Pd, AP, pap, red_scr, s);
            hipLaunchKernelGGL(k_cg_step, g, b, 0, s, n, k, active, rz0, pap, Pd, AP, X, R);
            SFG_LAUNCH_CHECK();
            tree_solve(&T, k, R, Zp, ts_ws, ts_wsb, s);
            block_dot(n, k, R, Zp, rz1, red_scr, s);
            hipLaunchKernelGGL(k_cg_dir, g, b, 0, s, n, k, active, rz1, rz0, Zp, Pd);
            SFG_LAUNCH_CHECK();
            std::swap(rz0, rz1);
            if (it % kCheck == 0 || it == max_iter) {
                block_dot(n, k, R, R, rr, red_scr, s);
                const std::vector<double> h = to_host(rr, k);
                for (int c = 0; c < k; ++c)
                    if (((active >> c) & 1u) && !(h[c] > tol * tol * h0[c])) active &= ~(1u << c);
            }
        }
        return it;
    }

    // one estimate for the sparsifier keep != 0 (its edges marked 1 must be
    // the tree this estimator was built with)
    double run(const uint8_t *keep, const sfg_kappa_params &kp, const double *y0, uint64_t seed, uint32_t block,
               sfg_kappa_report *rep) {
        const auto t0 = std::chrono::steady_clock::now();
        build_csr(n, m, u, v, w64, SFG_F64, keep, p_rowptr, p_col, p_val, p_eid, p_deg, csr_ws, csr_wsb, s);
        const size_t nk = (size_t)n * k;
        if (y0)
            SFG_HIP(hipMemcpyAsync(Y, y0, nk * sizeof(double), hipMemcpyDeviceToDevice, s));
        else
            random_block(n, k, seed, block, Y, s);
        double *mean = dev_small + 320, *Ad = dev_small + 16 * 64, *Bd = Ad + 32 * 32, *Vd = Bd + 32 * 32;
        const dim3 g(grid_for(n * k, kB)), b(kB);
        block_colsum(n, k, Y, 1.0 / (double)n, mean, red_scr, s);
        hipLaunchKernelGGL(k_subtract_mean, g, b, 0, s, n, k, mean, Y);
        SFG_LAUNCH_CHECK();
        lap(true, Y, Z);
        double est = 0.0;
        int64_t iters = 0;
        int32_t max_inner = 0, uncon = 0;
        for (int32_t t = 0; t < kp.steps; ++t) {
            bool cap = false;
            const int64_t it = solve(kp.tol, kp.max_iter, &cap);
            iters += it;
            max_inner = std::max<int32_t>(max_inner, (int32_t)it);
            uncon += cap ? 1 : 0;
            lap(true, X, W);
            lap(false, X, VP);
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
            hipLaunchKernelGGL(k_rotate, g, b, 0, s, n, k, X, Vd, Y);
            SFG_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_rotate, g, b, 0, s, n, k, W, Vd, Z);
            SFG_LAUNCH_CHECK();
            SFG_HIP(hipStreamSynchronize(s));   // V lives on the host stack
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
    if (p.tol == 0.0) p.tol = 1e-2;
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
        SFG_HIP(hipStreamSynchronize(s));
    });
}
