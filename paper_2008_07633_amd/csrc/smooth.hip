// Local spectral embedding (Sec. 3.2 of the paper): k random vectors made
// orthogonal to the all-one vector, then low-pass filtered by damped Jacobi
// relaxations of L x = 0.  One sweep is
//     y_p = (1 - omega) x_p + omega * (sum_q A_pq x_q) / D_pp .
//
// Sweep kernel layout (HBM-bound SpMM, no MFMA):
//   - the block X is node-major, so the k values of one neighbour are one
//     contiguous k*elt-byte run;
//   - a row is served by k/VPL lanes, each owning VPL consecutive columns
//     (one 8- or 16-byte load per neighbour), so one pass over the row's
//     col/val entries feeds all k vectors and a wavefront covers
//     64*VPL/k rows;
//   - each lane sums its row in ascending column order (no cross-lane
//     reduction, no atomics), which makes the FP64 result identical to the
//     plain sequential definition;
//   - workgroups are remapped so every XCD sweeps one contiguous row range
//     and neighbour rows tend to hit its own L2.
#include "common.hpp"

namespace sfg {

namespace {

// ------------------------------------------------------------------ double-double column sums
struct DD {
    double hi, lo;
};

__device__ __forceinline__ DD two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}
__device__ __forceinline__ DD quick_two_sum(double a, double b) {
    double s = a + b;
    double e = b - (s - a);
    return {s, e};
}
__device__ __forceinline__ DD dd_add(DD a, DD b) {
    DD s = two_sum(a.hi, b.hi);
    DD t = two_sum(a.lo, b.lo);
    double lo = s.lo + t.hi;
    DD r = quick_two_sum(s.hi, lo);
    lo = r.lo + t.lo;
    return quick_two_sum(r.hi, lo);
}
__device__ __forceinline__ DD dd_add1(DD a, double b) {
    DD s = two_sum(a.hi, b);
    double lo = s.lo + a.lo;
    return quick_two_sum(s.hi, lo);
}

constexpr int kSumThreads = 256;
constexpr int kSumMaxBlocks = 1024;

template <typename TIN>
__global__ __launch_bounds__(kSumThreads) void k_colsum_partial(int64_t n, int32_t k, const TIN *__restrict__ x,
                                                                int64_t rows_per_block, DD *partial) {
    __shared__ double shi[kSumThreads], slo[kSumThreads];
    const int rpi = kSumThreads / k;
    const int c = threadIdx.x % k, r0 = threadIdx.x / k;
    DD acc{0.0, 0.0};
    const int64_t start = (int64_t)blockIdx.x * rows_per_block;
    const int64_t end = start + rows_per_block < n ? start + rows_per_block : n;
    if (r0 < rpi)
        for (int64_t row = start + r0; row < end; row += rpi) acc = dd_add1(acc, cvt<double>(x[row * k + c]));
    shi[threadIdx.x] = acc.hi;
    slo[threadIdx.x] = acc.lo;
    __syncthreads();
    if ((int)threadIdx.x < k) {
        DD s{0.0, 0.0};
        for (int rr = 0; rr < rpi; ++rr) s = dd_add(s, DD{shi[rr * k + threadIdx.x], slo[rr * k + threadIdx.x]});
        partial[(int64_t)blockIdx.x * k + threadIdx.x] = s;
    }
}

__global__ void k_colsum_final(int32_t nb, int32_t k, const DD *partial, int64_t n, double *mean) {
    const int c = threadIdx.x;
    if (c >= k) return;
    DD s{0.0, 0.0};
    for (int b = 0; b < nb; ++b) s = dd_add(s, partial[(int64_t)b * k + c]);
    // s.hi is s.hi + s.lo rounded to nearest (quick_two_sum leaves it normalised)
    mean[c] = s.hi / (double)n;
}

template <typename TO>
__global__ void k_center_convert(int64_t total, int32_t k, const double *__restrict__ x0,
                                 const double *__restrict__ mean, TO *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    double d = x0[i] - mean[i % k];
    out[i] = cvt<TO>(d);
}

// ------------------------------------------------------------------ sweep

template <typename T, int N>
struct alignas(sizeof(T) * N) Vec {
    T v[N];
};

__device__ __forceinline__ double madd(double acc, double w, double x) { return acc + w * x; }
__device__ __forceinline__ float madd(float acc, float w, float x) { return __builtin_fmaf(w, x, acc); }

template <typename TX, typename TO, typename TW, typename TA, int VPL>
__global__ __launch_bounds__(256) void k_sweep(int64_t nthreads, int32_t lpr_log2, int32_t k,
                                               const int32_t *__restrict__ rowptr,
                                               const int32_t *__restrict__ col, const TW *__restrict__ val,
                                               const TW *__restrict__ deg, const TX *__restrict__ x,
                                               TO *__restrict__ y, TA keep, TA omega) {
    const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t t = (int64_t)b * 256 + threadIdx.x;
    if (t >= nthreads) return;
    const int64_t row = t >> lpr_log2;
    const int32_t off = (int32_t)(t & ((1 << lpr_log2) - 1)) * VPL;
    const int32_t j0 = rowptr[row], j1 = rowptr[row + 1];
    TA acc[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) acc[i] = TA(0);
    for (int32_t j = j0; j < j1; ++j) {
        const int64_t c = col[j];
        const TA wv = cvt<TA>(val[j]);
        const Vec<TX, VPL> xv = *reinterpret_cast<const Vec<TX, VPL> *>(x + c * k + off);
#pragma unroll
        for (int i = 0; i < VPL; ++i) acc[i] = madd(acc[i], wv, cvt<TA>(xv.v[i]));
    }
    const TA d = cvt<TA>(deg[row]);
    const Vec<TX, VPL> self = *reinterpret_cast<const Vec<TX, VPL> *>(x + row * k + off);
    Vec<TO, VPL> out;
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
        const TA a = keep * cvt<TA>(self.v[i]);
        const TA q = acc[i] / d;
        const TA bo = omega * q;
        out.v[i] = cvt<TO>(a + bo);
    }
    *reinterpret_cast<Vec<TO, VPL> *>(y + row * k + off) = out;
}

int ilog2(int x) {
    int r = 0;
    while ((1 << r) < x) ++r;
    return r;
}

template <typename TX, typename TO, typename TW, typename TA, int VPL>
void launch_sweep_v(const sfg_csr *H, int32_t k, const TX *x, TO *y, double omega, hipStream_t s) {
    const int lpr = k / VPL;
    const int64_t nthreads = H->n * (int64_t)lpr;
    hipLaunchKernelGGL((k_sweep<TX, TO, TW, TA, VPL>), dim3(grid_for(nthreads, 256)), dim3(256), 0, s, nthreads,
                       ilog2(lpr), k, H->rowptr, H->col, (const TW *)H->val, (const TW *)H->deg, x, y,
                       (TA)(1.0 - omega), (TA)omega);
    SFG_LAUNCH_CHECK();
}

// Columns per lane: the widest of 16 bytes that divides k into a power-of-two
// lane count (overridable with SFG_VPL for tuning).
template <typename TX>
int pick_vpl(int32_t k) {
    int best = 1;
    const int maxv = 16 / (int)sizeof(TX);
    static int forced = [] {
        const char *e = getenv("SFG_VPL");
        return e ? atoi(e) : 0;
    }();
    for (int v = 1; v <= maxv; v <<= 1) {
        if (k % v) continue;
        int lpr = k / v;
        if ((lpr & (lpr - 1)) != 0) continue;
        if (forced && v == forced) return v;
        best = v;
    }
    return best;
}

template <typename TX, typename TO, typename TW, typename TA>
void launch_sweep(const sfg_csr *H, int32_t k, const TX *x, TO *y, double omega, hipStream_t s) {
    const int vpl = pick_vpl<TX>(k);
    constexpr int maxv = 16 / (int)sizeof(TX);
    switch (vpl) {
        case 1: launch_sweep_v<TX, TO, TW, TA, 1>(H, k, x, y, omega, s); break;
        case 2: if constexpr (maxv >= 2) { launch_sweep_v<TX, TO, TW, TA, 2>(H, k, x, y, omega, s); break; } [[fallthrough]];
        case 4: if constexpr (maxv >= 4) { launch_sweep_v<TX, TO, TW, TA, 4>(H, k, x, y, omega, s); break; } [[fallthrough]];
        case 8: if constexpr (maxv >= 8) { launch_sweep_v<TX, TO, TW, TA, 8>(H, k, x, y, omega, s); break; } [[fallthrough]];
        default: fail(SFG_EUNSUPPORTED, "smooth: no kernel for this lane split");
    }
}

struct SmoothPlan {
    DD *partial;
    double *mean;
    void *buf0, *buf1;
};

int colsum_blocks(int64_t n) {
    int64_t nb = (n + kSumThreads - 1) / kSumThreads;
    if (nb > kSumMaxBlocks) nb = kSumMaxBlocks;
    return (int)(nb < 1 ? 1 : nb);
}

SmoothPlan plan_smooth(Carver &c, int64_t n, int32_t k, sfg_dtype storage) {
    SmoothPlan p;
    p.partial = c.take<DD>((size_t)colsum_blocks(n) * k);
    p.mean = c.take<double>(k);
    p.buf0 = c.take<char>((size_t)n * k * dtype_size(storage));
    p.buf1 = c.take<char>((size_t)n * k * dtype_size(storage));
    return p;
}

template <typename TX, typename TW, typename TA>
void run_smooth(const sfg_csr *H, int32_t k, int32_t sweeps, double omega, const double *x0, bool final_f32,
                void *xout, const SmoothPlan &p, hipStream_t s) {
    const int64_t n = H->n;
    const int64_t total = n * (int64_t)k;
    // a2: column means and centring (the block becomes orthogonal to 1)
    const int nb = colsum_blocks(n);
    const int64_t rpb = (n + nb - 1) / nb;
    hipLaunchKernelGGL(k_colsum_partial<double>, dim3(nb), dim3(kSumThreads), 0, s, n, k, x0, rpb, p.partial);
    SFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_colsum_final, dim3(1), dim3(64), 0, s, nb, k, p.partial, n, p.mean);
    SFG_LAUNCH_CHECK();
    if (sweeps == 0) {
        if (final_f32)
            hipLaunchKernelGGL(k_center_convert<float>, dim3(grid_for(total, 256)), dim3(256), 0, s, total, k, x0,
                               p.mean, (float *)xout);
        else
            hipLaunchKernelGGL(k_center_convert<TX>, dim3(grid_for(total, 256)), dim3(256), 0, s, total, k, x0,
                               p.mean, (TX *)xout);
        SFG_LAUNCH_CHECK();
        return;
    }
    TX *b0 = (TX *)p.buf0, *b1 = (TX *)p.buf1;
    hipLaunchKernelGGL(k_center_convert<TX>, dim3(grid_for(total, 256)), dim3(256), 0, s, total, k, x0, p.mean, b0);
    SFG_LAUNCH_CHECK();
    // a3: sweeps, ping-pong through the workspace, the last one into xout
    for (int32_t t = 0; t < sweeps; ++t) {
        const TX *src = (t % 2 == 0) ? b0 : b1;
        if (t == sweeps - 1) {
            if (final_f32)
                launch_sweep<TX, float, TW, TA>(H, k, src, (float *)xout, omega, s);
            else
                launch_sweep<TX, TX, TW, TA>(H, k, src, (TX *)xout, omega, s);
        } else {
            TX *dst = (t % 2 == 0) ? b1 : b0;
            launch_sweep<TX, TX, TW, TA>(H, k, src, dst, omega, s);
        }
    }
}

}  // namespace

size_t smooth_workspace_bytes(int64_t n, int32_t k, sfg_dtype storage) {
    Carver c(nullptr);
    plan_smooth(c, n, k, storage);
    return c.used + 256;
}

void smooth(const sfg_csr *H, int32_t k, int32_t sweeps, double omega, const double *x0, sfg_dtype storage,
            int32_t final_f32, void *x, void *ws, size_t ws_bytes, hipStream_t s) {
    SFG_REQUIRE(H && H->rowptr && H->deg && x0 && x, SFG_EINVAL, "smooth: null pointer");
    SFG_REQUIRE(H->n >= 1, SFG_EINVAL, "smooth: empty graph");
    SFG_REQUIRE(k >= 1, SFG_EINVAL, "smooth: k must be >= 1");
    SFG_REQUIRE(k <= 64, SFG_EUNSUPPORTED, "smooth: k > 64 is not supported");
    SFG_REQUIRE(sweeps >= 0, SFG_EINVAL, "smooth: sweeps must be >= 0");
    SFG_REQUIRE(omega > 0.0 && omega <= 1.0, SFG_EINVAL, "smooth: omega must be in (0, 1]");
    SFG_REQUIRE(valid_dtype(storage), SFG_EINVAL, "smooth: bad storage dtype");
    SFG_REQUIRE(H->n * (int64_t)k < (int64_t(1) << 40), SFG_EUNSUPPORTED, "smooth: block too large");
    SFG_REQUIRE(ws_bytes >= smooth_workspace_bytes(H->n, k, storage), SFG_EWORKSPACE, "smooth: workspace too small");
    const bool f32last = final_f32 && (storage == SFG_F16 || storage == SFG_BF16);
    Carver c(ws);
    SmoothPlan p = plan_smooth(c, H->n, k, storage);
    switch (storage) {
        case SFG_F64:
            SFG_REQUIRE(H->vt == SFG_F64, SFG_EUNSUPPORTED, "smooth: F64 storage needs an F64 graph");
            run_smooth<double, double, double>(H, k, sweeps, omega, x0, false, x, p, s);
            break;
        case SFG_F32:
            SFG_REQUIRE(H->vt == SFG_F32, SFG_EUNSUPPORTED, "smooth: F32 storage needs an F32 graph");
            run_smooth<float, float, float>(H, k, sweeps, omega, x0, false, x, p, s);
            break;
        case SFG_F16:
            SFG_REQUIRE(H->vt == SFG_F32, SFG_EUNSUPPORTED, "smooth: F16 storage needs an F32 graph");
            run_smooth<__half, float, float>(H, k, sweeps, omega, x0, f32last, x, p, s);
            break;
        case SFG_BF16:
            SFG_REQUIRE(H->vt == SFG_F32, SFG_EUNSUPPORTED, "smooth: BF16 storage needs an F32 graph");
            run_smooth<__hip_bfloat16, float, float>(H, k, sweeps, omega, x0, f32last, x, p, s);
            break;
    }
}

// Column means of a block (exact to double-double before one rounding);
// used for the affinity's centring.
void column_means(const void *x, sfg_dtype xt, int64_t n, int32_t k, double *mean, void *partial_ws,
                  hipStream_t s) {
    const int nb = colsum_blocks(n);
    const int64_t rpb = (n + nb - 1) / nb;
    DD *partial = (DD *)partial_ws;
    if (xt == SFG_F64)
        hipLaunchKernelGGL(k_colsum_partial<double>, dim3(nb), dim3(kSumThreads), 0, s, n, k, (const double *)x, rpb,
                           partial);
    else if (xt == SFG_F32)
        hipLaunchKernelGGL(k_colsum_partial<float>, dim3(nb), dim3(kSumThreads), 0, s, n, k, (const float *)x, rpb,
                           partial);
    else
        fail(SFG_EUNSUPPORTED, "column_means: F64 or F32 block required");
    SFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_colsum_final, dim3(1), dim3(64), 0, s, nb, k, partial, n, mean);
    SFG_LAUNCH_CHECK();
}

size_t column_means_partial_bytes(int64_t n, int32_t k) { return (size_t)colsum_blocks(n) * k * sizeof(DD); }

}  // namespace sfg

extern "C" sfg_status sfg_smooth(const sfg_csr *H, int32_t k, int32_t sweeps, double omega, const double *x0,
                                 sfg_dtype storage, int32_t final_f32, void *x, void *ws, size_t ws_bytes,
                                 void *stream) {
    return sfg::guard([&] {
        sfg::smooth(H, k, sweeps, omega, x0, storage, final_f32, x, ws, ws_bytes, sfg::as_stream(stream));
    });
}
