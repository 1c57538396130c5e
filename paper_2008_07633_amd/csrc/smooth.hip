// Local spectral embedding (Sec. 3.2 of the paper): k random vectors made
// orthogonal to the all-one vector, then low-pass filtered by damped Jacobi
// relaxations of L x = 0.  One sweep is
//     y_p = (1 - omega) x_p + omega * (sum_q A_pq x_q) / D_pp .
//
// Sweep kernel layout (HBM-bound SpMM, no MFMA):
//   - the block X is node-major, so the k values of one neighbour are one
//     contiguous k*elt-byte run;
//   - a row is served by k/VPL lanes, each owning VPL consecutive columns
//     (one wide load per neighbour), so one pass over the row's col/val
//     entries feeds all k vectors;
//   - the neighbour loop is unrolled by U with clamped indices: U col/val
//     loads, then U block-row gathers are in flight before any add, which
//     hides the dependent-load latency of short rows;
//   - each lane still adds its row in ascending column order (no cross-lane
//     reduction, no atomics), so the FP64 result equals the plain
//     sequential definition bit for bit;
//   - the first sweep reads the raw FP64 block and subtracts the column
//     means on the fly (centring costs no extra pass);
//   - workgroups are remapped so every XCD sweeps one contiguous row range
//     and neighbour rows tend to hit its own L2;
//   - an FP64 block on a tree-like graph is smoothed 8 columns at a time (all
//     sweeps of one column part, then the next), so the working set of a part
//     stays in the memory-side cache;
//   - in reduced precision, rows longer than 256 entries (hubs of power-law
//     graphs) are taken out and swept by a whole workgroup each.
#include <cstdlib>
#include <mutex>
#include <type_traits>
#include <vector>

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
constexpr int kSumMaxBlocks = 2048;

template <typename TIN>
__global__ __launch_bounds__(kSumThreads) void k_colsum_partial(int64_t n, int32_t k, const TIN *__restrict__ x,
                                                                int64_t rows_per_block, DD *partial) {
    __shared__ double shi[kSumThreads], slo[kSumThreads];
    const int rpi = kSumThreads / k;
    const int c = threadIdx.x % k, r0 = threadIdx.x / k;
    DD acc{0.0, 0.0};
    const int64_t start = (int64_t)blockIdx.x * rows_per_block;
    const int64_t end = start + rows_per_block < n ? start + rows_per_block : n;
    if (r0 < rpi) {
        int64_t row = start + r0;
        for (; row + 3 * rpi < end; row += 4 * rpi) {
            const double a0 = cvt<double>(x[row * k + c]);
            const double a1 = cvt<double>(x[(row + rpi) * k + c]);
            const double a2 = cvt<double>(x[(row + 2 * rpi) * k + c]);
            const double a3 = cvt<double>(x[(row + 3 * rpi) * k + c]);
            acc = dd_add1(acc, a0);
            acc = dd_add1(acc, a1);
            acc = dd_add1(acc, a2);
            acc = dd_add1(acc, a3);
        }
        for (; row < end; row += rpi) acc = dd_add1(acc, cvt<double>(x[row * k + c]));
    }
    shi[threadIdx.x] = acc.hi;
    slo[threadIdx.x] = acc.lo;
    __syncthreads();
    if ((int)threadIdx.x < k) {
        DD s{0.0, 0.0};
        for (int rr = 0; rr < rpi; ++rr) s = dd_add(s, DD{shi[rr * k + threadIdx.x], slo[rr * k + threadIdx.x]});
        partial[(int64_t)blockIdx.x * k + threadIdx.x] = s;
    }
}

// One workgroup per column: strided partial sums, then a fixed-shape tree.
__global__ __launch_bounds__(256) void k_colsum_final(int32_t nb, int32_t k, const DD *__restrict__ partial,
                                                      int64_t n, double *mean) {
    __shared__ double shi[256], slo[256];
    const int c = blockIdx.x, t = threadIdx.x;
    DD s{0.0, 0.0};
    for (int b = t; b < nb; b += 256) s = dd_add(s, partial[(int64_t)b * k + c]);
    shi[t] = s.hi;
    slo[t] = s.lo;
    __syncthreads();
    for (int stride = 128; stride > 0; stride >>= 1) {
        if (t < stride) {
            DD r = dd_add(DD{shi[t], slo[t]}, DD{shi[t + stride], slo[t + stride]});
            shi[t] = r.hi;
            slo[t] = r.lo;
        }
        __syncthreads();
    }
    // shi[0] is shi[0] + slo[0] rounded to nearest (quick_two_sum normalises)
    if (t == 0) mean[c] = shi[0] / (double)n;
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

// Load VPL consecutive block values as the accumulation type.  With CENTER
// the source is the raw FP64 block: subtract the column mean, round to the
// storage type, then widen -- the same values a separate centring pass
// would have stored.
template <typename TIN, typename TX, typename TA, int VPL, bool CENTER>
__device__ __forceinline__ void load_row(const TIN *p, const double *mo, TA (&out)[VPL]) {
    const Vec<TIN, VPL> v = *reinterpret_cast<const Vec<TIN, VPL> *>(p);
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
        if constexpr (CENTER)
            out[i] = cvt<TA>(cvt<TX>(cvt<double>(v.v[i]) - mo[i]));
        else
            out[i] = cvt<TA>(v.v[i]);
    }
}

template <typename TIN, typename TX, typename TO, typename TW, typename TA, int VPL, int U, bool CENTER>
__global__ __launch_bounds__(256) void k_sweep(int64_t nthreads, int32_t lpr, int32_t lpr_log2, int32_t ldx,
                                               int32_t ldy, int32_t max_len, const int32_t *__restrict__ rows,
                                               const int32_t *__restrict__ rowptr,
                                               const int32_t *__restrict__ col, const TW *__restrict__ val,
                                               const TW *__restrict__ deg, const TIN *__restrict__ x,
                                               const double *__restrict__ mean, TO *__restrict__ y, TA keep,
                                               TA omega) {
    const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t t = (int64_t)b * 256 + threadIdx.x;
    if (t >= nthreads) return;
    const int64_t ri = lpr_log2 >= 0 ? (t >> lpr_log2) : t / lpr;
    const int32_t off = (int32_t)(t - ri * lpr) * VPL;
    // rows == nullptr: every row in order; else only the listed rows
    const int64_t row = rows ? (int64_t)rows[ri] : ri;
    double mo[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) mo[i] = CENTER ? mean[off + i] : 0.0;
    const int32_t j0 = rowptr[row], j1 = rowptr[row + 1];
    if (j1 - j0 > max_len) return;      // a long row: k_sweep_long handles it
    TA self[VPL];
    load_row<TIN, TX, TA, VPL, CENTER>(x + row * ldx + off, mo, self);
    const TA d = cvt<TA>(deg[row]);
    TA acc[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) acc[i] = TA(0);
    for (int32_t j = j0; j < j1; j += U) {
        int32_t cj[U];
        TA wj[U];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const int32_t jj = (j + i < j1) ? j + i : j1 - 1;     // clamped: a valid, cached entry
            cj[i] = col[jj];
            wj[i] = cvt<TA>(val[jj]);
        }
        TA xv[U][VPL];
#pragma unroll
        for (int i = 0; i < U; ++i) load_row<TIN, TX, TA, VPL, CENTER>(x + (int64_t)cj[i] * ldx + off, mo, xv[i]);
#pragma unroll
        for (int i = 0; i < U; ++i) {
            if (j + i < j1) {
#pragma unroll
                for (int q = 0; q < VPL; ++q) acc[q] = madd(acc[q], wj[i], xv[i][q]);
            }
        }
    }
    Vec<TO, VPL> out;
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
        const TA a = keep * self[i];
        const TA q = acc[i] / d;
        const TA bo = omega * q;
        out.v[i] = cvt<TO>(a + bo);
    }
    *reinterpret_cast<Vec<TO, VPL> *>(y + row * ldy + off) = out;
}

// Rows longer than max_len (hubs of power-law graphs), reduced precision
// only: one workgroup per row.  Its 256/lpr lane groups take interleaved
// entries of the row, then their partial sums are combined in LDS by a
// fixed-shape tree, so the result is deterministic (the order differs from
// the sequential one, which FP64 keeps).
template <typename TIN, typename TX, typename TO, typename TW, typename TA, int VPL, bool CENTER>
__global__ __launch_bounds__(256) void k_sweep_long(int32_t lpr, int32_t ldx, int32_t ldy,
                                                    const int32_t *__restrict__ long_rows,
                                                    const int32_t *__restrict__ long_cnt,
                                                    const int32_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ col, const TW *__restrict__ val,
                                                    const TW *__restrict__ deg, const TIN *__restrict__ x,
                                                    const double *__restrict__ mean, TO *__restrict__ y, TA keep,
                                                    TA omega) {
    __shared__ TA part[256 * VPL];
    const int t = threadIdx.x;
    const int ngroups = 256 / lpr;
    const int g = t / lpr, l = t % lpr;
    const int off = l * VPL;
    const bool active = g < ngroups;
    double mo[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) mo[i] = (CENTER && active) ? mean[off + i] : 0.0;
    const int32_t cnt = *long_cnt;
    for (int32_t r = blockIdx.x; r < cnt; r += gridDim.x) {
        const int64_t row = long_rows[r];
        const int32_t j0 = rowptr[row], j1 = rowptr[row + 1];
        TA acc[VPL];
#pragma unroll
        for (int i = 0; i < VPL; ++i) acc[i] = TA(0);
        if (active) {
            for (int32_t j = j0 + g; j < j1; j += ngroups) {
                const int64_t c = col[j];
                const TA wv = cvt<TA>(val[j]);
                TA xv[VPL];
                load_row<TIN, TX, TA, VPL, CENTER>(x + c * ldx + off, mo, xv);
#pragma unroll
                for (int i = 0; i < VPL; ++i) acc[i] = madd(acc[i], wv, xv[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < VPL; ++i) part[t * VPL + i] = acc[i];
        __syncthreads();
        for (int st = 1; st < ngroups; st <<= 1) {
            if (active && (g % (2 * st)) == 0 && g + st < ngroups) {
#pragma unroll
                for (int i = 0; i < VPL; ++i) part[t * VPL + i] += part[(t + st * lpr) * VPL + i];
            }
            __syncthreads();
        }
        if (g == 0) {
            TA self[VPL];
            load_row<TIN, TX, TA, VPL, CENTER>(x + row * ldx + off, mo, self);
            const TA d = cvt<TA>(deg[row]);
            Vec<TO, VPL> out;
#pragma unroll
            for (int i = 0; i < VPL; ++i) {
                const TA a = keep * self[i];
                const TA q = part[l * VPL + i] / d;
                const TA bo = omega * q;
                out.v[i] = cvt<TO>(a + bo);
            }
            *reinterpret_cast<Vec<TO, VPL> *>(y + row * ldy + off) = out;
        }
        __syncthreads();
    }
}

// Multicolour Gauss-Seidel reading of the smoother: the listed rows (one
// colour class: no two adjacent) are updated in place from the current block,
// each row with the Jacobi sweep's arithmetic.  x is read and written, so it
// carries no restrict qualifier; the rows read are of other colours and are
// not written by this launch.
template <typename T, int VPL, int U>
__global__ __launch_bounds__(256) void k_sweep_color(int64_t nthreads, int32_t lpr, int32_t lpr_log2, int32_t k,
                                                     const int32_t *__restrict__ rows,
                                                     const int32_t *__restrict__ rowptr,
                                                     const int32_t *__restrict__ col, const T *__restrict__ val,
                                                     const T *__restrict__ deg, T *x, T keep, T omega) {
    const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t t = (int64_t)b * 256 + threadIdx.x;
    if (t >= nthreads) return;
    const int64_t ri = lpr_log2 >= 0 ? (t >> lpr_log2) : t / lpr;
    const int32_t off = (int32_t)(t - ri * lpr) * VPL;
    const int64_t row = rows[ri];
    const double mo[VPL] = {};
    const int32_t j0 = rowptr[row], j1 = rowptr[row + 1];
    T self[VPL];
    load_row<T, T, T, VPL, false>(x + row * k + off, mo, self);
    const T d = deg[row];
    T acc[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) acc[i] = T(0);
    for (int32_t j = j0; j < j1; j += U) {
        int32_t cj[U];
        T wj[U];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const int32_t jj = (j + i < j1) ? j + i : j1 - 1;
            cj[i] = col[jj];
            wj[i] = val[jj];
        }
        T xv[U][VPL];
#pragma unroll
        for (int i = 0; i < U; ++i) load_row<T, T, T, VPL, false>(x + (int64_t)cj[i] * k + off, mo, xv[i]);
#pragma unroll
        for (int i = 0; i < U; ++i) {
            if (j + i < j1) {
#pragma unroll
                for (int q = 0; q < VPL; ++q) acc[q] = madd(acc[q], wj[i], xv[i][q]);
            }
        }
    }
    Vec<T, VPL> out;
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
        const T a = keep * self[i];
        const T q = acc[i] / d;
        const T bo = omega * q;
        out.v[i] = a + bo;
    }
    *reinterpret_cast<Vec<T, VPL> *>(x + row * k + off) = out;
}

// Rows handled by k_sweep_long (device list and count), and the length above
// which k_sweep skips a row.  Default: none, every row in k_sweep.
// FP64 hub rows (listed only when the caller knows the graph has rows over
// 256 entries): the sum k_sweep's lane group would form -- entries in stored
// order, acc = acc + w * x, one rounding per operation, then the same
// epilogue -- so the result is bit-identical, but the row's weights and
// neighbour values are gathered by the whole workgroup into LDS, chunk by
// chunk, and lane c adds column c from there: the dependent chain is over
// LDS reads instead of over global gathers.
constexpr int kHubLds = 4096;   // doubles of staged neighbour values per chunk (32 KB)

template <typename TIN, typename TX, typename TO, bool CENTER>
__global__ __launch_bounds__(256) void k_sweep_hub64(int32_t kw, int32_t ldx, int32_t ldy,
                                                     const int32_t *__restrict__ hub_rows,
                                                     const int32_t *__restrict__ hub_cnt,
                                                     const int32_t *__restrict__ rowptr,
                                                     const int32_t *__restrict__ col,
                                                     const double *__restrict__ val, const double *__restrict__ deg,
                                                     const TIN *__restrict__ x, const double *__restrict__ mean,
                                                     TO *__restrict__ y, double keep, double omega) {
    __shared__ double sx[kHubLds];
    __shared__ double sw[256];
    __shared__ int32_t sc[256];
    constexpr int kPer = kHubLds / 256;    // values a thread stages per chunk
    const int chunk = kHubLds / kw < 256 ? kHubLds / kw : 256;
    const int t = threadIdx.x;
    const int32_t cnt = *hub_cnt;
    for (int32_t r = blockIdx.x; r < cnt; r += gridDim.x) {
        const int64_t row = hub_rows[r];
        const int32_t j0 = rowptr[row], j1 = rowptr[row + 1];
        double mo[1] = {0.0};
        if (CENTER && t < kw) mo[0] = mean[t];
        double acc = 0.0;
        for (int32_t jc = j0; jc < j1; jc += chunk) {
            const int32_t len = (j1 - jc) < chunk ? (j1 - jc) : chunk;
            // the chunk's columns and weights, then its neighbour values: every thread's loads in flight
            // before its LDS stores
            if (t < len) {
                sc[t] = col[jc + t];
                sw[t] = val[jc + t];
            }
            __syncthreads();
            double vv[kPer];
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const int32_t i = t + 256 * q;
                if (i < len * kw) {
                    const int32_t e = i / kw, c = i - e * kw;
                    double v[1];
                    const double m1[1] = {CENTER ? mean[c] : 0.0};
                    load_row<TIN, TX, double, 1, CENTER>(x + (int64_t)sc[e] * ldx + c, m1, v);
                    vv[q] = v[0];
                }
            }
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const int32_t i = t + 256 * q;
                if (i < len * kw) sx[i] = vv[q];
            }
            __syncthreads();
            if (t < kw) {
                // entry order kept: products (independent of acc) read ahead, then the dependent adds
                int32_t e = 0;
                for (; e + 8 <= len; e += 8) {
                    double pr[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) pr[q] = sw[e + q] * sx[(e + q) * kw + t];
#pragma unroll
                    for (int q = 0; q < 8; ++q) acc = acc + pr[q];
                }
                for (; e < len; ++e) acc = madd(acc, sw[e], sx[e * kw + t]);
            }
            __syncthreads();
        }
        if (t < kw) {
            double self[1];
            load_row<TIN, TX, double, 1, CENTER>(x + row * ldx + t, mo, self);
            const double d = deg[row];
            const double a = keep * self[0];
            const double q = acc / d;
            const double bo = omega * q;
            y[row * ldy + t] = cvt<TO>(a + bo);
        }
    }
}

struct LongRows {
    const int32_t *rows = nullptr;
    const int32_t *count = nullptr;
    int32_t max_len = 0x7fffffff;
    // with a side stream, the hub rows of an iterate run there beside the main
    // sweep of the same iterate (they write disjoint rows): es marks the last
    // main sweep done, ez the last hub-row sweep
    hipStream_t side = nullptr;
    hipEvent_t es = nullptr, ez = nullptr;
};

// One side stream per device (default priority), created on first use and
// kept for the process.
hipStream_t side_stream() {
    static std::mutex mu;
    static hipStream_t streams[64] = {};
    int dev = 0;
    SFG_HIP(hipGetDevice(&dev));
    SFG_REQUIRE(dev >= 0 && dev < 64, SFG_EUNSUPPORTED, "smooth: device index over 63");
    std::lock_guard<std::mutex> lock(mu);
    if (!streams[dev]) SFG_HIP(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking));
    return streams[dev];
}

int ilog2_exact(int x) {
    for (int r = 0; r < 31; ++r)
        if ((1 << r) == x) return r;
    return -1;
}

int env_int(const char *name, int dflt) {
    const char *e = getenv(name);
    return e ? atoi(e) : dflt;
}

// One sweep over the kw columns [c0, c0 + kw) of the block: x and y point at
// column c0 of row 0, ldx and ldy are their row strides (elements), mean (when
// centring) at the mean of column c0.  vpl columns per lane, u-fold neighbour
// unroll.
struct SweepShape {
    int32_t kw, ldx, ldy, vpl, u;
};

// Workgroups of the hub-row kernel (a grid-stride loop over the device-side
// list of rows over 256 entries).  Graphs averaging 8 or more entries per row
// (power-law graphs and their dense coarse levels) get 16,384, so that many
// hub rows are in flight at once: 355 against 377 ms for the 4M-node Chung-Lu
// hierarchy.  Others get 1,024, since every launch dispatches its workgroups
// even when the list is empty: 16,384 there cost 1.4 us per sweep.
inline unsigned long_row_blocks(const sfg_csr *H) { return H->nnz >= 8 * H->n ? 16384u : 1024u; }

template <typename TIN, typename TX, typename TO, typename TW, typename TA, int VPL, int U, bool CENTER>
void launch_sweep_u(const sfg_csr *H, const SweepShape &sh, const TIN *x, const double *mean, TO *y, double omega,
                    const int32_t *rows, int64_t nrows, const LongRows &lr, hipStream_t s) {
    const int lpr = sh.kw / VPL;
    const int64_t nthreads = nrows * (int64_t)lpr;
    if (nthreads == 0) return;
    // the previous iterate's hub rows must be done before the main sweep reads
    // them or overwrites the rows they read (waiting on a never-recorded event
    // is a no-op)
    if (lr.side) SFG_HIP(hipStreamWaitEvent(s, lr.ez, 0));
    hipLaunchKernelGGL((k_sweep<TIN, TX, TO, TW, TA, VPL, U, CENTER>), dim3(grid_for(nthreads, 256)), dim3(256), 0, s,
                       nthreads, lpr, ilog2_exact(lpr), sh.ldx, sh.ldy, lr.max_len, rows, H->rowptr, H->col,
                       (const TW *)H->val, (const TW *)H->deg, x, mean, y, (TA)(1.0 - omega), (TA)omega);
    SFG_LAUNCH_CHECK();
    // hub rows: on the side stream after the previous main sweep, beside this one
    hipStream_t zs = s;
    if (lr.side && lr.rows) {
        zs = lr.side;
        SFG_HIP(hipStreamWaitEvent(zs, lr.es, 0));
    }
    if constexpr (sizeof(TA) == 8) {
        if (lr.rows) {
            hipLaunchKernelGGL((k_sweep_hub64<TIN, TX, TO, CENTER>), dim3(long_row_blocks(H)), dim3(256), 0, zs, sh.kw,
                               sh.ldx, sh.ldy, lr.rows, lr.count, H->rowptr, H->col, (const double *)H->val,
                               (const double *)H->deg, x, mean, y, 1.0 - omega, omega);
            SFG_LAUNCH_CHECK();
        }
    }
    if constexpr (sizeof(TA) == 4) {
        if (lr.rows) {
            hipLaunchKernelGGL((k_sweep_long<TIN, TX, TO, TW, TA, VPL, CENTER>), dim3(long_row_blocks(H)), dim3(256),
                               0, zs, lpr, sh.ldx, sh.ldy, lr.rows, lr.count, H->rowptr, H->col, (const TW *)H->val,
                               (const TW *)H->deg, x, mean, y, (TA)(1.0 - omega), (TA)omega);
            SFG_LAUNCH_CHECK();
        }
    }
    if (lr.side && lr.rows) {
        SFG_HIP(hipEventRecord(lr.ez, zs));
        SFG_HIP(hipEventRecord(lr.es, s));
    }
}

template <typename TIN, typename TX, typename TO, typename TW, typename TA, int VPL, bool CENTER>
void launch_sweep_v(const sfg_csr *H, const SweepShape &sh, const TIN *x, const double *mean, TO *y, double omega,
                    const int32_t *rows, int64_t nrows, const LongRows &lr, hipStream_t s) {
    if (sh.u <= 2)
        launch_sweep_u<TIN, TX, TO, TW, TA, VPL, 2, CENTER>(H, sh, x, mean, y, omega, rows, nrows, lr, s);
    else if (sh.u <= 4)
        launch_sweep_u<TIN, TX, TO, TW, TA, VPL, 4, CENTER>(H, sh, x, mean, y, omega, rows, nrows, lr, s);
    else
        launch_sweep_u<TIN, TX, TO, TW, TA, VPL, 8, CENTER>(H, sh, x, mean, y, omega, rows, nrows, lr, s);
}

// Columns per lane: the widest run that divides kw and spans at most maxb
// bytes.  SFG_VPL overrides it, up to 64 bytes, for tuning.
template <typename TX>
int pick_vpl(int32_t kw, int maxb) {
    static const int forced = env_int("SFG_VPL", 0);
    if (forced > 0 && kw % forced == 0 && forced * (int)sizeof(TX) <= 64) return forced;
    int best = 1;
    for (int v = 1; v * (int)sizeof(TX) <= maxb; v <<= 1)
        if (kw % v == 0) best = v;
    return best;
}

// Launch shape of a sweep over the whole block (k columns, stride k).
// Measured best on the 1M-node power grid's spanning tree: 4 lanes per
// 16-vector row (32 bytes per lane in FP64, 16 otherwise), neighbour unroll 2
// for FP64 rows averaging <= 3 entries, else 4.  SFG_SWEEP_U overrides the
// unroll (2, 4 or 8).
template <typename TX>
SweepShape full_shape(const sfg_csr *H, int32_t k) {
    static const int forced_u = env_int("SFG_SWEEP_U", 0);
    SweepShape sh;
    sh.kw = sh.ldx = sh.ldy = k;
    sh.vpl = pick_vpl<TX>(k, sizeof(TX) == 8 ? 32 : 16);
    sh.u = forced_u ? forced_u : ((sizeof(TX) == 8 && H->nnz <= 3 * H->n) ? 2 : 4);
    return sh;
}

template <typename TIN, typename TX, typename TO, typename TW, typename TA, bool CENTER>
void launch_sweep(const sfg_csr *H, const SweepShape &sh, const TIN *x, const double *mean, TO *y, double omega,
                  hipStream_t s, const int32_t *rows = nullptr, int64_t nrows = -1, const LongRows &lr = LongRows()) {
    if (nrows < 0) nrows = H->n;
    constexpr int maxv = 64 / (int)sizeof(TX);
    switch (sh.vpl) {
        case 1: launch_sweep_v<TIN, TX, TO, TW, TA, 1, CENTER>(H, sh, x, mean, y, omega, rows, nrows, lr, s); return;
        case 2: launch_sweep_v<TIN, TX, TO, TW, TA, 2, CENTER>(H, sh, x, mean, y, omega, rows, nrows, lr, s); return;
        case 4: launch_sweep_v<TIN, TX, TO, TW, TA, 4, CENTER>(H, sh, x, mean, y, omega, rows, nrows, lr, s); return;
        case 8: launch_sweep_v<TIN, TX, TO, TW, TA, 8, CENTER>(H, sh, x, mean, y, omega, rows, nrows, lr, s); return;
        case 16:
            if constexpr (maxv >= 16) {
                launch_sweep_v<TIN, TX, TO, TW, TA, 16, CENTER>(H, sh, x, mean, y, omega, rows, nrows, lr, s);
                return;
            }
            break;
        default: break;
    }
    fail(SFG_EUNSUPPORTED, "smooth: no kernel for this lane split");
}

template <typename TIN, typename TX, typename TO, typename TW, typename TA, bool CENTER>
void launch_sweep(const sfg_csr *H, int32_t k, const TIN *x, const double *mean, TO *y, double omega, hipStream_t s,
                  const int32_t *rows = nullptr, int64_t nrows = -1, const LongRows &lr = LongRows()) {
    launch_sweep<TIN, TX, TO, TW, TA, CENTER>(H, full_shape<TX>(H, k), x, mean, y, omega, s, rows, nrows, lr);
}

// Column parts for the full smoothing.  An FP64 block of k >= 16 vectors on a
// sparse graph (<= 3 entries per row on average: spanning trees, sparsifiers)
// whose sweep working set (X_t, X_t+1 and the graph) exceeds the 256 MB
// memory-side cache, while that of an 8-column part stays within 192 MB of
// it, is swept 8 columns (64-byte rows) at a time, all sweeps of one part
// before the next: the part's two ping-pong buffers and the graph then stay
// cache-resident, and 64-byte rows take 4 lanes of 16 bytes with a 4-fold
// neighbour unroll (measured on the 1M-node power grid's tree: 59 us per
// 16-vector sweep against 74 us unsplit).  A part that does not fit gains
// nothing and repeats the neighbour gathers (measured slower on a 2M-node kNN
// tree with random node order), so it is not split.  Each column's arithmetic
// is unchanged: the result is bit-identical.  SFG_SWEEP_SPLIT (read at every
// call) = 0 turns it off, 2 forces it for any FP64 block of k >= 16, k % 8 == 0
// (tests use it to cover the part sweeps on small graphs).  SFG_SWEEP_U
// overrides the part sweeps' unroll too, for tuning.
template <typename TX>
SweepShape part_shape(const sfg_csr *H, int32_t k) {
    const int split = env_int("SFG_SWEEP_SPLIT", 1);
    constexpr double kCache = 256.0 * (1 << 20), kPartBudget = 192.0 * (1 << 20);
    const double sx = (double)sizeof(TX), sw = (double)dtype_size(H->vt);
    const double graph = 4.0 * (H->n + 1) + (double)H->nnz * (4.0 + sw) + (double)H->n * sw;
    const double full = 2.0 * H->n * k * sx + graph, part = 2.0 * H->n * 8 * sx + graph;
    const bool fits = H->nnz <= 3 * H->n && full > kCache && part <= kPartBudget;
    if (sizeof(TX) == 8 && k >= 16 && k % 8 == 0 && (split == 2 || (split == 1 && fits))) {
        SweepShape sh;
        sh.kw = 8;
        sh.ldx = sh.ldy = 8;
        sh.vpl = pick_vpl<TX>(8, 16);
        static const int forced_u = env_int("SFG_SWEEP_U", 0);
        sh.u = forced_u ? forced_u : 4;
        return sh;
    }
    return full_shape<TX>(H, k);
}

struct SmoothPlan {
    DD *partial;
    double *mean;
    void *buf0, *buf1;
    int32_t *lflag, *lpos, *lrows, *lscan;
};

constexpr int32_t kLongRow = 256;   // reduced precision: rows above this go to k_sweep_long

__global__ void k_long_flag(int64_t n, const int32_t *__restrict__ rowptr, int32_t len, int32_t *flag) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) flag[p] = (rowptr[p + 1] - rowptr[p] > len) ? 1 : 0;
}

__global__ void k_long_scatter(int64_t n, const int32_t *__restrict__ flag, const int32_t *__restrict__ pos,
                               int32_t *rows) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n && flag[p]) rows[pos[p]] = (int32_t)p;
}

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
    p.lflag = c.take<int32_t>(n + 1);
    p.lpos = c.take<int32_t>(n + 1);
    p.lrows = c.take<int32_t>(n + 1);
    p.lscan = c.take<int32_t>(scan_scratch_ints(n + 1));
    return p;
}

template <typename TIN>
void launch_column_means(const TIN *x, int64_t n, int32_t k, DD *partial, double *mean, hipStream_t s) {
    const int nb = colsum_blocks(n);
    const int64_t rpb = (n + nb - 1) / nb;
    hipLaunchKernelGGL(k_colsum_partial<TIN>, dim3(nb), dim3(kSumThreads), 0, s, n, k, x, rpb, partial);
    SFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_colsum_final, dim3(k), dim3(256), 0, s, nb, k, partial, n, mean);
    SFG_LAUNCH_CHECK();
}

template <typename TX, typename TW, typename TA>
void run_smooth(const sfg_csr *H, int32_t k, int32_t sweeps, double omega, const double *x0, bool final_f32,
                bool hub_rows, void *xout, const SmoothPlan &p, hipStream_t s) {
    const int64_t n = H->n;
    const int64_t total = n * (int64_t)k;
    // a2: column means (the block becomes orthogonal to the all-one vector)
    launch_column_means<double>(x0, n, k, p.partial, p.mean, s);
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
    // reduced precision, and FP64 when the caller knows there are hub rows: list
    // the rows over kLongRow entries once for all sweeps (device-side count)
    LongRows lr;
    if (sizeof(TA) == 4 || hub_rows) {
        hipLaunchKernelGGL(k_long_flag, dim3(grid_for(n, 256)), dim3(256), 0, s, n, H->rowptr, kLongRow, p.lflag);
        SFG_LAUNCH_CHECK();
        exclusive_scan_i32(p.lflag, p.lpos, n, p.lscan, s);
        hipLaunchKernelGGL(k_long_scatter, dim3(grid_for(n, 256)), dim3(256), 0, s, n, p.lflag, p.lpos, p.lrows);
        SFG_LAUNCH_CHECK();
        lr.rows = p.lrows;
        lr.count = p.lpos + n;
        lr.max_len = kLongRow;
    }
    // graphs whose hub rows take long (power-law graphs, their dense coarse
    // levels; FP64 hub rows when listed) sweep them on a side stream
    struct Side {
        hipEvent_t es = nullptr, ez = nullptr;
        ~Side() {
            if (es) (void)hipEventDestroy(es);
            if (ez) (void)hipEventDestroy(ez);
        }
    } side;
    if (lr.rows && sweeps > 0 && (sizeof(TA) == 8 || H->nnz >= 8 * H->n)) {
        lr.side = side_stream();
        SFG_HIP(hipEventCreateWithFlags(&side.es, hipEventDisableTiming));
        SFG_HIP(hipEventCreateWithFlags(&side.ez, hipEventDisableTiming));
        lr.es = side.es;
        lr.ez = side.ez;
        SFG_HIP(hipEventRecord(lr.es, s));   // the side stream starts after everything so far
    }
    // a3: sweeps, column part by column part; the first sweep of a part
    // centres on the fly from x0, the last writes the part's columns of xout
    const SweepShape ps = part_shape<TX>(H, k);
    for (int32_t c0 = 0; c0 < k; c0 += ps.kw) {
        SweepShape first = ps, mid = ps;
        first.ldx = k;
        for (int32_t t = 0; t < sweeps; ++t) {
            const bool last = (t == sweeps - 1);
            SweepShape sh = (t == 0) ? first : mid;
            if (last) sh.ldy = k;
            TX *dst = (t % 2 == 0) ? b0 : b1;
            if (t == 0) {
                if (last && final_f32)
                    launch_sweep<double, TX, float, TW, TA, true>(H, sh, x0 + c0, p.mean + c0,
                                                                  (float *)xout + c0, omega, s, nullptr, -1, lr);
                else
                    launch_sweep<double, TX, TX, TW, TA, true>(H, sh, x0 + c0, p.mean + c0,
                                                               last ? (TX *)xout + c0 : dst, omega, s, nullptr, -1,
                                                               lr);
                continue;
            }
            const TX *src = (t % 2 == 0) ? b1 : b0;
            if (last && final_f32)
                launch_sweep<TX, TX, float, TW, TA, false>(H, sh, src, nullptr, (float *)xout + c0, omega, s, nullptr,
                                                           -1, lr);
            else
                launch_sweep<TX, TX, TX, TW, TA, false>(H, sh, src, nullptr, last ? (TX *)xout + c0 : dst, omega, s,
                                                        nullptr, -1, lr);
        }
    }
    if (lr.side) SFG_HIP(hipStreamWaitEvent(s, lr.ez, 0));   // join: the last hub rows before anything after
}

// ------------------------------------------------------------------ several sweeps per pass through LDS
// Rows are taken in blocks of kMpkRows consecutive entries of a caller's
// order (a permutation of the nodes; a spanning tree's preorder keeps a
// block's neighbourhood small).  For block b, layer L0 is its rows and layer
// L(h+1) the neighbours of Lh not in L0..Lh.  A layout pass for H hops gives
// every block a slot per node of L0..LH, layer by layer (L0 in the order's
// sequence), and a local CSR of the rows of L0..L(H-1): each entry's
// neighbour as a slot, its weight, in the row's stored order, and the rows'
// degrees.  One workgroup then loads X_t of every slot into LDS and forms
// m <= H sweeps there: sweep j+1 for the rows of L0..L(m-1-j), whose
// neighbours all lie one layer further out, and writes X_t+m of L0 only.
// X is read about (|L0..Lm| / |L0|) times and written once per m sweeps
// instead of twice per sweep.  Every row's value is formed with the single
// sweep's arithmetic -- entries in stored order, the same epilogue, every
// intermediate iterate rounded to the storage type -- so the result is
// bit-identical to m single sweeps.
constexpr int kMpkRows = 64;      // rows of L0 per block
constexpr int kMpkRowBytes = 128; // row width the LDS holds: 16 FP64 or 32 FP32 columns
constexpr int kMpkMeta = 8;       // ints of a block's sizes: layer ends e_0..e_H, then the local entries at [7]
constexpr int kMpkMaxHops = 4;

// Capacities per block for H hops: slots of L0..LH, rows of L0..L(H-1),
// local CSR entries, node->slot map entries.  Measured on the 200^3 mesh's
// spanning tree in preorder (64-row blocks; largest block of 125,000):
// H = 2: 155 slots, 106 rows, 249 entries; H = 3: 211, 155, 357;
// H = 4: 272, 211, 479.
template <int H> struct MpkCaps;
template <> struct MpkCaps<2> {
    static constexpr int kSlots = 168, kRows = 112, kEnt = 288, kHash = 512;
    using Col = uint8_t;
};
template <> struct MpkCaps<3> {
    static constexpr int kSlots = 224, kRows = 160, kEnt = 384, kHash = 512;
    using Col = uint8_t;
};
template <> struct MpkCaps<4> {
    static constexpr int kSlots = 288, kRows = 224, kEnt = 512, kHash = 1024;
    using Col = uint16_t;
};

// Blocks over the common-case launch's slot capacity are swept by that
// launch too, gathering their first sweep's X_t from global memory, rather
// than by a second launch at the layout's full capacity -- where the
// common-case launch holds the layout's every row (its slots at least the
// layout's rows), so that only X of the outer slots is missing.
constexpr bool kMpkGatherWide = true;
template <int H, int KS>
constexpr bool mpk_gathers() { return kMpkGatherWide && KS < MpkCaps<H>::kSlots && MpkCaps<H>::kRows <= KS; }

// Per-block layout at the capacities of the hop count it was built for
// (views into the workspace, sized for the largest).
struct MpkDev {
    int32_t *meta;      // [nb kMpkMeta]
    int32_t *node;      // [nb kSlots]: node of each slot
    uint16_t *rowoff;   // [nb (kRows + 1)]: local CSR row starts
    void *lcol;         // [nb kEnt] of Col: slot of each entry's neighbour
    void *lval;         // [nb kEnt] of the graph's value type: entry weights
    void *ldeg;         // [nb kRows] of that type: degrees of the local rows
};

__device__ __forceinline__ int wave_incl_sum(int x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

constexpr int kMpkRegCols = 8;    // row entries the layout pass holds in registers; longer rows are re-read

__device__ __forceinline__ int mpk_hash(int32_t q, int bits) {
    return (int)(((uint32_t)q * 0x9E3779B1u) >> (32 - bits));
}

// Node -> slot map of one block in LDS (open addressing, linear probing).
// Inserts q: new -> takes the next slot from *next (its node into snode when
// within nslots) and returns 1; present -> 0; table full -> -1.
template <int HASH>
__device__ __forceinline__ int hs_insert(int32_t *keys, int32_t *vals, int32_t *next, int32_t *snode, int nslots,
                                         int32_t q) {
    constexpr int bits = HASH == 1024 ? 10 : 9;
    int h = mpk_hash(q, bits);
    for (int probe = 0; probe < HASH; ++probe) {
        const int32_t old = atomicCAS(&keys[h], -1, q);
        if (old == -1) {
            const int32_t slot = atomicAdd(next, 1);
            vals[h] = slot;
            if (slot < nslots) snode[slot] = q;
            return 1;
        }
        if (old == q) return 0;
        h = (h + 1) & (HASH - 1);
    }
    return -1;
}

template <int HASH>
__device__ __forceinline__ int32_t hs_find(const int32_t *keys, const int32_t *vals, int32_t q) {
    constexpr int bits = HASH == 1024 ? 10 : 9;
    int h = mpk_hash(q, bits);
    for (int probe = 0; probe < HASH; ++probe) {
        const int32_t kk = keys[h];
        if (kk == q) return vals[h];
        if (kk == -1) return -1;
        h = (h + 1) & (HASH - 1);
    }
    return -1;
}

// The first kMpkRegCols column indices of a row, loaded together (the loops
// over them are unrolled so that they stay in registers).
__device__ __forceinline__ void row_cols(const int32_t *__restrict__ col, int32_t j0, int32_t len,
                                         int32_t (&cc)[kMpkRegCols]) {
#pragma unroll
    for (int t = 0; t < kMpkRegCols; ++t) cc[t] = t < len ? col[j0 + t] : -1;
}

// Order check, no atomics and no cleared memory: every order[i] in [0, n),
// and seen[order[i]] = i stored by k_mpk_mark, then read back by
// k_mpk_verify.  A node listed twice keeps only one of its positions, so the
// other position finds a different value: any duplicate sets flag bit 0.
// Each XCD takes a contiguous range of positions, whose nodes (a part of a
// traversal) share the lines of seen in its L2.
__global__ void k_mpk_mark(int64_t n, const int32_t *__restrict__ order, int32_t *seen, int32_t *flag) {
    const int64_t i = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t v = order[i];
    if (v < 0 || v >= n)
        atomicOr(flag, 1);
    else
        seen[v] = (int32_t)i;
}

__global__ void k_mpk_verify(int64_t n, const int32_t *__restrict__ order, const int32_t *__restrict__ seen,
                             int32_t *flag) {
    const int64_t i = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t v = order[i];
    if (v >= 0 && v < n && seen[v] != (int32_t)i) atomicOr(flag, 1);
}

// Layout of one block for H hops, one 64-lane workgroup per block.  A block
// that does not fit (a layer, the rows or the local CSR over the capacities,
// a row the single sweep would not form in entry order, an order entry
// outside [0, n)) gets zero sizes and sets flag bit 2; the
// caller then lays out for fewer hops, or runs the single sweeps.  Slots of
// L1..LH are numbered in discovery order: which slot a node takes changes
// where its row sits in the LDS, not any value.
template <int H, typename TW>
__global__ __launch_bounds__(64) void k_mpk_build(int64_t n, const int32_t *__restrict__ order,
                                                  const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ col, const TW *__restrict__ val,
                                                  const TW *__restrict__ deg, MpkDev L, int32_t *flag) {
    using C = MpkCaps<H>;
    using Col = typename C::Col;
    // rows the single sweep forms in entry order: all FP64 rows (sfg_smooth keeps them in k_sweep), reduced
    // precision rows up to kLongRow entries (longer ones go to k_sweep_long's lane-group sums there)
    constexpr int kMaxRow = sizeof(TW) == 8 ? C::kEnt : (kLongRow < C::kEnt ? kLongRow : C::kEnt);
    __shared__ int32_t keys[C::kHash];
    __shared__ int32_t vals[C::kHash];
    __shared__ int32_t snode[C::kSlots];
    __shared__ int32_t next;
    __shared__ int32_t full;
    const int lane = threadIdx.x;
    // consecutive blocks (neighbouring parts of the order) on one XCD: the
    // rows they share stay in that XCD's L2
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t base = b * kMpkRows;
    const int s0 = (int)(n - base < kMpkRows ? n - base : kMpkRows);
#pragma unroll
    for (int i = 0; i < C::kHash / 64; ++i) keys[i * 64 + lane] = -1;
    if (lane == 0) {
        next = s0;
        full = 0;
    }
    const int32_t p = lane < s0 ? (order ? order[base + lane] : (int32_t)(base + lane)) : -1;
    const bool bad = lane < s0 && (p < 0 || p >= n);
    bool over = __ballot(bad) != 0ull;
    __syncthreads();
    // L0: slot = position in the order
    if (!over && lane < s0) {
        snode[lane] = p;
        int h = mpk_hash(p, C::kHash == 1024 ? 10 : 9);
        for (int probe = 0; probe < C::kHash; ++probe) {
            const int32_t old = atomicCAS(&keys[h], -1, p);
            if (old == -1) {
                vals[h] = lane;
                break;
            }
            if (old == p) break;        // a repeated order entry: refused by the order check
            h = (h + 1) & (C::kHash - 1);
        }
    }
    __syncthreads();
    // L(h+1): neighbours of the rows of Lh not yet in the map.  Row r belongs
    // to lane r % 64 as its row q = r / 64 from its discovery to the local CSR
    // below: its entry range and first columns stay in registers.  A level
    // whose rows run past Q 64 (beyond the layout's rows anyway) fails the
    // block.
    constexpr int Q = (C::kRows + 63) / 64;
    int32_t sj0[Q], slen[Q], scol[Q][kMpkRegCols];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        sj0[q] = 0;
        slen[q] = 0;
    }
    int ends[H + 1];
    ends[0] = s0;
    int lo = 0;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        if (!over) {
            if (ends[h] > Q * 64 && lane == 0) full = 1;
#pragma unroll
            for (int qq = 0; qq < Q; ++qq) {
                const int r = qq * 64 + lane;
                if (r < lo || r >= ends[h]) continue;
                const int32_t q = snode[r];
                const int32_t j0 = rowptr[q], len = rowptr[q + 1] - j0;
                if (len > kMaxRow) {
                    full = 1;
                    continue;
                }
                int32_t cc[kMpkRegCols];
                row_cols(col, j0, len, cc);
                sj0[qq] = j0;
                slen[qq] = len;
#pragma unroll
                for (int t = 0; t < kMpkRegCols; ++t) scol[qq][t] = cc[t];
#pragma unroll
                for (int t = 0; t < kMpkRegCols; ++t)
                    if (t < len && hs_insert<C::kHash>(keys, vals, &next, snode, C::kSlots, cc[t]) < 0) full = 1;
                for (int t = kMpkRegCols; t < len; ++t)
                    if (hs_insert<C::kHash>(keys, vals, &next, snode, C::kSlots, col[j0 + t]) < 0) full = 1;
            }
        }
        __syncthreads();
        ends[h + 1] = next;
        over = over || full != 0 || ends[h + 1] > C::kSlots;
        lo = ends[h];
        __syncthreads();
    }
    const int R = ends[H - 1], S = ends[H];
    over = over || R > C::kRows;
    // local CSR of rows [0, R): row q 64 + lane, q < Q, every one of them
    // discovered above unless the block failed
    int32_t rq[Q], j0q[Q], lenq[Q], startq[Q];
    int nent = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int r = q * 64 + lane;
        rq[q] = (!over && r < R) ? snode[r] : -1;
        j0q[q] = rq[q] >= 0 ? sj0[q] : 0;
        lenq[q] = rq[q] >= 0 ? slen[q] : 0;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int incl = wave_incl_sum(lenq[q]);
        startq[q] = nent + incl - lenq[q];
        nent += __shfl(incl, 63, 64);
    }
    over = over || nent > C::kEnt;
    if (over) {
        if (lane < kMpkMeta) L.meta[kMpkMeta * b + lane] = 0;
        if (lane == 0) atomicOr(flag, 2);
        return;
    }
    uint16_t *ro = L.rowoff + b * (C::kRows + 1);
    Col *lc = (Col *)L.lcol + b * C::kEnt;
    TW *lv = (TW *)L.lval + b * C::kEnt;
    TW *ld = (TW *)L.ldeg + b * C::kRows;
    int32_t cr[Q][kMpkRegCols];
    TW vr[Q][kMpkRegCols];
    TW dq[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
#pragma unroll
        for (int t = 0; t < kMpkRegCols; ++t) cr[q][t] = scol[q][t];
#pragma unroll
        for (int t = 0; t < kMpkRegCols; ++t) vr[q][t] = t < lenq[q] ? val[j0q[q] + t] : TW(0);
        dq[q] = rq[q] >= 0 ? deg[rq[q]] : TW(0);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (rq[q] < 0) continue;
        const int r = q * 64 + lane, at = startq[q], len = lenq[q], j0 = j0q[q];
        ro[r] = (uint16_t)at;
        ld[r] = dq[q];
#pragma unroll
        for (int t = 0; t < kMpkRegCols; ++t)
            if (t < len) {
                lc[at + t] = (Col)hs_find<C::kHash>(keys, vals, cr[q][t]);
                lv[at + t] = vr[q][t];
            }
        for (int t = kMpkRegCols; t < len; ++t) {
            lc[at + t] = (Col)hs_find<C::kHash>(keys, vals, col[j0 + t]);
            lv[at + t] = val[j0 + t];
        }
    }
    if (lane == 0) ro[R] = (uint16_t)nent;
    int32_t *nd = L.node + b * C::kSlots;
    for (int i = lane; i < S; i += 64) nd[i] = snode[i];
#pragma unroll
    for (int h = 0; h <= H; ++h)
        if (lane == h) L.meta[kMpkMeta * b + h] = ends[h];
    if (lane == kMpkMeta - 1) L.meta[kMpkMeta * b + lane] = nent;
}

// LDS of one pass workgroup holding up to `slots` slots: X of every slot for
// KC columns, the slot nodes, the local CSR of up to min(rows, slots) rows.
constexpr int mpk_lds_bytes(int slots, int rows, int ent, int colb, int kc, int sx, int sw) {
    const int r = rows < slots ? rows : slots;
    return slots * (kc * sx + 4) + ent * (sw + colb) + r * sw + (r + 1) * 2;
}
template <int H, int KC, int KS, typename TX, typename TW>
constexpr int mpk_pass_lds() {
    using C = MpkCaps<H>;
    return mpk_lds_bytes(KS, C::kRows, C::kEnt, (int)sizeof(typename C::Col), KC, (int)sizeof(TX), (int)sizeof(TW));
}
template <int H, int KC, int KS, typename TX, typename TW>
constexpr int mpk_pass_waves() {
    // workgroups of 4 waves a CU's 160 KB of LDS holds = waves per SIMD (registers are held to it)
    return 163840 / mpk_pass_lds<H, KC, KS, TX, TW>() > 8 ? 8 : 163840 / mpk_pass_lds<H, KC, KS, TX, TW>();
}
// Slot capacity of the common-case pass kernel: the most slots whose LDS lets
// eight workgroups share a CU (20,000 bytes each), at most the layout's.
// Blocks with more slots (a fraction of a percent on the 200^3 mesh's tree)
// are swept by the same launch from global memory where it holds all of the
// layout's rows (mpk_gathers), else by a second launch at the full capacity.
constexpr int mpk_small_slots(int slots, int rows, int ent, int colb, int kc, int sx, int sw) {
    int ks = slots;
    while (ks > 64 && mpk_lds_bytes(ks, rows, ent, colb, kc, sx, sw) > 20000) --ks;
    return ks;
}
template <int H, int KC, typename TX, typename TW>
constexpr int mpk_small_slots() {
    using C = MpkCaps<H>;
    return mpk_small_slots(C::kSlots, C::kRows, C::kEnt, (int)sizeof(typename C::Col), KC, (int)sizeof(TX),
                           (int)sizeof(TW));
}

// Blocks of a layout for H hops whose slots exceed ks, listed for the
// full-capacity launch (order irrelevant: each block writes its own rows).
template <int H>
__global__ void k_mpk_big(int64_t nb, const int32_t *__restrict__ meta, int32_t ks, int32_t *list, int32_t *cnt) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    if (meta[kMpkMeta * b + H] > ks) list[atomicAdd(cnt, 1)] = (int32_t)b;
}

// m sweeps of KC columns of one block (see above), 1 <= m <= H: workgroup w
// takes block w / (k / KC) and column group w % (k / KC), k the block's
// columns (its row stride).  VPL columns per lane; TIN the source block's
// type (the raw FP64 block when CENTER: centred on load, as the single sweep
// does).  The LDS holds X of every slot; each sweep's new rows are formed in
// registers and written over the old ones after a barrier (no row of a sweep
// reads a slot outside the next layer), so one X block's worth of LDS is
// enough.  Narrower column groups take less LDS, so more workgroups share a
// CU and hide the gathers' latency; the groups of a block are adjacent
// workgroups of one XCD, so its layout is fetched once into that XCD's L2.
// Two dependent rounds of global loads: the block's sizes and slot nodes,
// then X of the slots and the local CSR.
// KS: the slots this variant holds.  LISTED = false: every block (those with
// more than KS slots gathered, or skipped for the listed launch where the
// variant does not hold all of the layout's rows); LISTED = true: the blocks
// of list[] only.
template <int H, int KC, int KS, bool LISTED, typename TIN, typename TX, typename TO, typename TW, typename TA,
          int VPL, bool CENTER>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(mpk_pass_waves<H, KC, KS, TX, TW>()))) void
k_sweep_pass(int32_t k, int32_t m, MpkDev L, const int32_t *__restrict__ list, const TIN *__restrict__ x,
             const double *__restrict__ mean, TO *__restrict__ y, TA keep, TA omega) {
    using C = MpkCaps<H>;
    using Col = typename C::Col;
    constexpr int RK = C::kRows < KS ? C::kRows : KS;   // rows of L0..L(H-1) fit within the slots
    constexpr int LPR = KC / VPL;              // lanes per row
    constexpr int RPP = 256 / LPR;             // rows a pass
    constexpr int kSlotPasses = (KS + RPP - 1) / RPP;
    constexpr int kRowPasses = (RK + RPP - 1) / RPP;
    constexpr int kStage = kSlotPasses < 4 ? kSlotPasses : 4;
    __shared__ __align__(16) TX xs[KS * KC];
    __shared__ int32_t nodes[KS];
    __shared__ TW lval[C::kEnt];
    __shared__ TW ldeg[RK];
    __shared__ uint16_t rowoff[RK + 1];
    __shared__ Col lcol[C::kEnt];
    const int groups = k / KC;
    const uint32_t w = LISTED ? blockIdx.x : xcd_remap(blockIdx.x, gridDim.x);
    const int64_t item_b = w / groups;
    const int64_t b = LISTED ? list[item_b] : item_b;
    const int g0 = (int)(w - item_b * groups) * KC;
    const int t = threadIdx.x;
    const int32_t *mp = L.meta + kMpkMeta * b;
    int ends[H + 1];
#pragma unroll
    for (int h = 0; h <= H; ++h) ends[h] = mp[h];
    constexpr bool kGather = !LISTED && mpk_gathers<H, KS>();
    if (!LISTED && KS < C::kSlots && !kGather && ends[H] > KS) return;   // the full-capacity launch takes this block
    const int ne = mp[kMpkMeta - 1];
    int S = ends[H], R = ends[H - 1];
#pragma unroll
    for (int h = 1; h <= H; ++h)
        if (h == m) {
            S = ends[h];
            R = ends[h - 1];
        }
    // a block with more slots than this variant holds: nothing is staged, the
    // first sweep gathers X_t from global memory (the same values, converted as
    // the staging converts them), and the later sweeps read the rows it wrote to
    // the LDS.  Those are rows of the local CSR, all of which fit here (RK is the
    // layout's row capacity when kGather), as do their row starts and degrees.
    const bool gather = kGather && S > KS;
    const int s0 = ends[0];
    // round 1: slot nodes (read to this variant's capacity, used to S)
    for (int i = t; i < KS; i += 256) nodes[i] = L.node[b * C::kSlots + i];
    // round 2 issued early: the local CSR into registers
    constexpr int kEntPer = (C::kEnt + 255) / 256;
    Col ec[kEntPer];
    TW ev[kEntPer];
#pragma unroll
    for (int j = 0; j < kEntPer; ++j) {
        const int i = t + 256 * j;
        if (i < ne) {
            ec[j] = ((const Col *)L.lcol)[b * C::kEnt + i];
            ev[j] = ((const TW *)L.lval)[b * C::kEnt + i];
        }
    }
    constexpr int kRowPer = (RK + 1 + 255) / 256;
    uint16_t ro[kRowPer];
    TW dg[kRowPer];
#pragma unroll
    for (int j = 0; j < kRowPer; ++j) {
        const int i = t + 256 * j;
        if (i <= R) ro[j] = L.rowoff[b * (C::kRows + 1) + i];
        if (i < R) dg[j] = ((const TW *)L.ldeg)[b * C::kRows + i];
    }
    const int ri0 = t / LPR, c = (t % LPR) * VPL;
    const int rend = ri0 < RPP ? 0x7fffffff : 0;   // 256 % LPR lanes idle: no rows for them
    double mo[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) mo[i] = CENTER ? mean[g0 + c + i] : 0.0;
    __syncthreads();
    // X_t of slots [0, S): loads of kStage passes, then their LDS stores
#pragma unroll
    for (int p0 = 0; p0 < kSlotPasses; p0 += kStage) {
        if (p0 * RPP >= S || gather) break;
        TA v[kStage][VPL];
#pragma unroll
        for (int j = 0; j < kStage; ++j) {
            const int r = ri0 + (p0 + j) * RPP;
            if (p0 + j < kSlotPasses && r < S && r < rend)
                load_row<TIN, TX, TA, VPL, CENTER>(x + (int64_t)nodes[r] * k + g0 + c, mo, v[j]);
        }
#pragma unroll
        for (int j = 0; j < kStage; ++j) {
            const int r = ri0 + (p0 + j) * RPP;
            if (p0 + j < kSlotPasses && r < S && r < rend) {
                Vec<TX, VPL> st;
#pragma unroll
                for (int i = 0; i < VPL; ++i) st.v[i] = cvt<TX>(v[j][i]);
                *reinterpret_cast<Vec<TX, VPL> *>(xs + r * KC + c) = st;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kEntPer; ++j) {
        const int i = t + 256 * j;
        if (i < ne) {
            lcol[i] = ec[j];
            lval[i] = ev[j];
        }
    }
#pragma unroll
    for (int j = 0; j < kRowPer; ++j) {
        const int i = t + 256 * j;
        if (i <= R) rowoff[i] = ro[j];
        if (i < R) ldeg[i] = dg[j];
    }
    __syncthreads();
    // one sweep of row r from the LDS, stored as T (the storage type, or the last iterate's)
    auto row_sweep = [&](int r, auto tag) {
        using T = decltype(tag);
        TA acc[VPL];
#pragma unroll
        for (int i = 0; i < VPL; ++i) acc[i] = TA(0);
        for (int e = rowoff[r]; e < rowoff[r + 1]; ++e) {
            const TA wv = cvt<TA>(lval[e]);
            const Vec<TX, VPL> xv = *reinterpret_cast<const Vec<TX, VPL> *>(xs + (int)lcol[e] * KC + c);
#pragma unroll
            for (int i = 0; i < VPL; ++i) acc[i] = madd(acc[i], wv, cvt<TA>(xv.v[i]));
        }
        const Vec<TX, VPL> sv = *reinterpret_cast<const Vec<TX, VPL> *>(xs + r * KC + c);
        const TA d = cvt<TA>(ldeg[r]);
        Vec<T, VPL> out;
#pragma unroll
        for (int i = 0; i < VPL; ++i) {
            const TA a = keep * cvt<TA>(sv.v[i]);
            const TA q = acc[i] / d;
            const TA bo = omega * q;
            out.v[i] = cvt<T>(a + bo);
        }
        return out;
    };
    // the same sweep of row r with X_t gathered from global memory (gather mode's first sweep)
    auto row_sweep_g = [&](int r, auto tag) {
        using T = decltype(tag);
        auto xt = [&](int slot, TA (&o)[VPL]) {
            const int32_t node = slot < KS ? nodes[slot] : L.node[b * C::kSlots + slot];
            TA v[VPL];
            load_row<TIN, TX, TA, VPL, CENTER>(x + (int64_t)node * k + g0 + c, mo, v);
#pragma unroll
            for (int i = 0; i < VPL; ++i) o[i] = cvt<TA>(cvt<TX>(v[i]));
        };
        TA acc[VPL];
#pragma unroll
        for (int i = 0; i < VPL; ++i) acc[i] = TA(0);
        for (int e = rowoff[r]; e < rowoff[r + 1]; ++e) {
            const TA wv = cvt<TA>(lval[e]);
            TA xv[VPL];
            xt((int)lcol[e], xv);
#pragma unroll
            for (int i = 0; i < VPL; ++i) acc[i] = madd(acc[i], wv, xv[i]);
        }
        TA sv[VPL];
        xt(r, sv);
        const TA d = cvt<TA>(ldeg[r]);
        Vec<T, VPL> out;
#pragma unroll
        for (int i = 0; i < VPL; ++i) {
            const TA a = keep * sv[i];
            const TA q = acc[i] / d;
            const TA bo = omega * q;
            out.v[i] = cvt<T>(a + bo);
        }
        return out;
    };
    // sweeps 1..m-1: rows of L0..L(m-1-j) into registers, then over X in the LDS
    for (int j = 0; j + 1 < m; ++j) {
        int nrows = ends[0];
#pragma unroll
        for (int h = 0; h < H; ++h)
            if (h == m - 1 - j) nrows = ends[h];
        Vec<TX, VPL> xr[kRowPasses];
#pragma unroll
        for (int q = 0; q < kRowPasses; ++q) {
            const int r = ri0 + q * RPP;
            if (r < nrows && r < rend) xr[q] = (gather && j == 0) ? row_sweep_g(r, TX()) : row_sweep(r, TX());
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kRowPasses; ++q) {
            const int r = ri0 + q * RPP;
            if (r < nrows && r < rend) *reinterpret_cast<Vec<TX, VPL> *>(xs + r * KC + c) = xr[q];
        }
        __syncthreads();
    }
    // the last sweep: L0 (its neighbours all lie in L0 and L1)
    for (int r = ri0; r < s0 && r < rend; r += RPP)
        *reinterpret_cast<Vec<TO, VPL> *>(y + (int64_t)nodes[r] * k + g0 + c) =
            (gather && m == 1) ? row_sweep_g(r, TO()) : row_sweep(r, TO());
}

}  // namespace

// FP64 smoothing restricted to a dependency cone (precision form).  rows_by_dist
// lists rows in ascending hop distance from the rows whose final values are
// wanted; active[t] (host) is how many of them sweep t+1 recomputes, i.e. the
// rows within sweeps-(t+1) hops.  Every recomputed row is added exactly as in
// the full FP64 pass, so rows at distance 0 end bit-identical to it.
// Returns the buffer that holds the final iterate.
size_t cone_partial_bytes(int64_t n, int32_t k) { return (size_t)colsum_blocks(n) * k * sizeof(DD); }

// Row-normalised aggregation y = D^-1 A x of an n-by-k block (the sweep with
// omega = 1; FP32 arithmetic).  x and y are F32 or BF16; H must be F32.
// With H->deg pointing at ones it is the plain product A x.
void spmm_rownorm(const sfg_csr *H, int32_t k, sfg_dtype t, const void *x, void *y, hipStream_t s) {
    SFG_REQUIRE(H->vt == SFG_F32, SFG_EUNSUPPORTED, "aggregation needs an F32 graph");
    if (t == SFG_F32)
        launch_sweep<float, float, float, float, float, false>(H, k, (const float *)x, nullptr, (float *)y, 1.0, s);
    else if (t == SFG_BF16)
        launch_sweep<__hip_bfloat16, __hip_bfloat16, __hip_bfloat16, float, float, false>(
            H, k, (const __hip_bfloat16 *)x, nullptr, (__hip_bfloat16 *)y, 1.0, s);
    else
        fail(SFG_EUNSUPPORTED, "aggregation: F32 or BF16 activations only");
}

double *smooth_cone_f64(const sfg_csr *H, int32_t k, int32_t sweeps, double omega, const double *x0,
                        const int32_t *rows_by_dist, const int64_t *active, double *buf0, double *buf1,
                        void *partial_ws, double *mean, hipStream_t s) {
    SFG_REQUIRE(H->vt == SFG_F64, SFG_EUNSUPPORTED, "cone smoothing needs an F64 graph");
    launch_column_means<double>(x0, H->n, k, (DD *)partial_ws, mean, s);
    if (sweeps == 0) {
        const int64_t total = H->n * (int64_t)k;
        hipLaunchKernelGGL(k_center_convert<double>, dim3(grid_for(total, 256)), dim3(256), 0, s, total, k, x0,
                           mean, buf0);
        SFG_LAUNCH_CHECK();
        return buf0;
    }
    double *dst = buf0;
    for (int32_t t = 0; t < sweeps; ++t) {
        dst = (t % 2 == 0) ? buf0 : buf1;
        if (t == 0)
            launch_sweep<double, double, double, double, double, true>(H, k, x0, mean, dst, omega, s, rows_by_dist,
                                                                       active[t]);
        else
            launch_sweep<double, double, double, double, double, false>(H, k, (t % 2 == 0) ? buf1 : buf0, nullptr,
                                                                        dst, omega, s, rows_by_dist, active[t]);
    }
    return dst;
}

size_t smooth_workspace_bytes(int64_t n, int32_t k, sfg_dtype storage) {
    Carver c(nullptr);
    plan_smooth(c, n, k, storage);
    return c.used + 256;
}

namespace {
template <typename T, int VPL>
void launch_color_v(const sfg_csr *H, int32_t k, const int32_t *rows, int64_t nrows, T *x, double omega,
                    hipStream_t s) {
    const int lpr = k / VPL;
    const int64_t nthreads = nrows * (int64_t)lpr;
    if (nthreads == 0) return;
    hipLaunchKernelGGL((k_sweep_color<T, VPL, 4>), dim3(grid_for(nthreads, 256)), dim3(256), 0, s, nthreads, lpr,
                       ilog2_exact(lpr), k, rows, H->rowptr, H->col, (const T *)H->val, (const T *)H->deg, x,
                       (T)(1.0 - omega), (T)omega);
    SFG_LAUNCH_CHECK();
}

template <typename T>
void launch_color(const sfg_csr *H, int32_t k, const int32_t *rows, int64_t nrows, T *x, double omega,
                  hipStream_t s) {
    switch (pick_vpl<T>(k, sizeof(T) == 8 ? 32 : 16)) {
        case 1: launch_color_v<T, 1>(H, k, rows, nrows, x, omega, s); return;
        case 2: launch_color_v<T, 2>(H, k, rows, nrows, x, omega, s); return;
        case 4: launch_color_v<T, 4>(H, k, rows, nrows, x, omega, s); return;
        case 8: launch_color_v<T, 8>(H, k, rows, nrows, x, omega, s); return;
        default: break;
    }
    fail(SFG_EUNSUPPORTED, "smooth_gs: no kernel for this lane split");
}

}  // namespace

// Multicolour Gauss-Seidel smoothing (F64 or F32 storage): centre x0 into x,
// then `sweeps` sweeps, each the colour classes in order, in place.
// class_ptr (host) has ncolors + 1 offsets into class_rows (device).
void smooth_gs(const sfg_csr *H, int32_t k, int32_t sweeps, double omega, const double *x0, sfg_dtype storage,
               const int32_t *class_rows, const std::vector<int32_t> &class_ptr, void *x, void *ws, size_t ws_bytes,
               hipStream_t s) {
    SFG_REQUIRE(H && H->rowptr && H->deg && x0 && x && class_rows, SFG_EINVAL, "smooth_gs: null pointer");
    SFG_REQUIRE(k >= 1 && k <= 64, SFG_EINVAL, "smooth_gs: k must be in [1, 64]");
    SFG_REQUIRE(sweeps >= 0, SFG_EINVAL, "smooth_gs: sweeps must be >= 0");
    SFG_REQUIRE(omega > 0.0 && omega <= 1.0, SFG_EINVAL, "smooth_gs: omega must be in (0, 1]");
    SFG_REQUIRE(storage == SFG_F64 || storage == SFG_F32, SFG_EUNSUPPORTED, "smooth_gs: F64 or F32 storage");
    SFG_REQUIRE(H->vt == storage, SFG_EUNSUPPORTED, "smooth_gs: graph values must match the storage");
    SFG_REQUIRE(ws_bytes >= smooth_workspace_bytes(H->n, k, storage), SFG_EWORKSPACE, "smooth_gs: workspace too small");
    const int64_t n = H->n, total = n * (int64_t)k;
    Carver c(ws);
    SmoothPlan p = plan_smooth(c, n, k, storage);
    launch_column_means<double>(x0, n, k, p.partial, p.mean, s);
    const int32_t ncolors = (int32_t)class_ptr.size() - 1;
    if (storage == SFG_F64) {
        hipLaunchKernelGGL(k_center_convert<double>, dim3(grid_for(total, 256)), dim3(256), 0, s, total, k, x0,
                           p.mean, (double *)x);
        SFG_LAUNCH_CHECK();
        for (int32_t t = 0; t < sweeps; ++t)
            for (int32_t cc = 0; cc < ncolors; ++cc)
                launch_color<double>(H, k, class_rows + class_ptr[cc], class_ptr[cc + 1] - class_ptr[cc],
                                     (double *)x, omega, s);
    } else {
        hipLaunchKernelGGL(k_center_convert<float>, dim3(grid_for(total, 256)), dim3(256), 0, s, total, k, x0,
                           p.mean, (float *)x);
        SFG_LAUNCH_CHECK();
        for (int32_t t = 0; t < sweeps; ++t)
            for (int32_t cc = 0; cc < ncolors; ++cc)
                launch_color<float>(H, k, class_rows + class_ptr[cc], class_ptr[cc + 1] - class_ptr[cc],
                                    (float *)x, omega, s);
    }
}


// max_row: the longest row of H if the caller knows it, else -1.  FP64 hub
// rows (over 256 entries) go to k_sweep_hub64 only when it is known, since
// listing them costs launches on every call.
void smooth(const sfg_csr *H, int32_t k, int32_t sweeps, double omega, const double *x0, sfg_dtype storage,
            int32_t final_f32, void *x, void *ws, size_t ws_bytes, hipStream_t s, int32_t max_row) {
    SFG_REQUIRE(H && H->rowptr && H->deg && x0 && x, SFG_EINVAL, "smooth: null pointer");
    SFG_REQUIRE(H->n >= 1, SFG_EINVAL, "smooth: empty graph");
    SFG_REQUIRE(k >= 1, SFG_EINVAL, "smooth: k must be >= 1");
    SFG_REQUIRE(k <= 64, SFG_EUNSUPPORTED, "smooth: k > 64 is not supported");
    SFG_REQUIRE(sweeps >= 0, SFG_EINVAL, "smooth: sweeps must be >= 0");
    SFG_REQUIRE(omega > 0.0 && omega <= 1.0, SFG_EINVAL, "smooth: omega must be in (0, 1]");
    SFG_REQUIRE(valid_dtype(storage), SFG_EINVAL, "smooth: bad storage dtype");
    SFG_REQUIRE(H->n * (int64_t)k < (int64_t(1) << 40), SFG_EUNSUPPORTED, "smooth: block too large");
    SFG_REQUIRE(H->nnz == 0 || (H->col && H->val), SFG_EINVAL, "smooth: null pointer");
    SFG_REQUIRE(ws_bytes >= smooth_workspace_bytes(H->n, k, storage), SFG_EWORKSPACE, "smooth: workspace too small");
    const bool f32last = final_f32 && (storage == SFG_F16 || storage == SFG_BF16);
    Carver c(ws);
    SmoothPlan p = plan_smooth(c, H->n, k, storage);
    switch (storage) {
        case SFG_F64:
            SFG_REQUIRE(H->vt == SFG_F64, SFG_EUNSUPPORTED, "smooth: F64 storage needs an F64 graph");
            run_smooth<double, double, double>(H, k, sweeps, omega, x0, false, max_row > kLongRow, x, p, s);
            break;
        case SFG_F32:
            SFG_REQUIRE(H->vt == SFG_F32, SFG_EUNSUPPORTED, "smooth: F32 storage needs an F32 graph");
            run_smooth<float, float, float>(H, k, sweeps, omega, x0, false, false, x, p, s);
            break;
        case SFG_F16:
            SFG_REQUIRE(H->vt == SFG_F32, SFG_EUNSUPPORTED, "smooth: F16 storage needs an F32 graph");
            run_smooth<__half, float, float>(H, k, sweeps, omega, x0, f32last, false, x, p, s);
            break;
        case SFG_BF16:
            SFG_REQUIRE(H->vt == SFG_F32, SFG_EUNSUPPORTED, "smooth: BF16 storage needs an F32 graph");
            run_smooth<__hip_bfloat16, float, float>(H, k, sweeps, omega, x0, f32last, false, x, p, s);
            break;
    }
}

// Several sweeps per pass in a caller's row order (see k_sweep_pass).
struct MpkPlan {
    MpkDev dev;
    int32_t *seen, *flag;    // flag[1]: the number of blocks listed in big
    int32_t *big;
    int64_t nbig = 0;        // host copy of flag[1]
    int32_t small_slots = 0; // slots of the common-case launch (the layout's capacity: no second launch)
};

int64_t mpk_blocks(int64_t n) { return (n + kMpkRows - 1) / kMpkRows; }

// Sized for the largest capacities (four hops), so that any hop count fits.
MpkPlan plan_mpk(Carver &c, int64_t n, size_t sw) {
    using C = MpkCaps<kMpkMaxHops>;
    const int64_t nb = mpk_blocks(n);
    MpkPlan p;
    p.dev.meta = c.take<int32_t>(kMpkMeta * nb);
    p.dev.node = c.take<int32_t>(nb * C::kSlots);
    p.dev.rowoff = c.take<uint16_t>(nb * (C::kRows + 1));
    p.dev.lcol = c.take<char>(nb * C::kEnt * sizeof(C::Col));
    p.dev.lval = c.take<char>(nb * C::kEnt * sw);
    p.dev.ldeg = c.take<char>(nb * C::kRows * sw);
    p.seen = c.take<int32_t>(n + 1);
    p.flag = c.take<int32_t>(2);
    p.big = c.take<int32_t>(nb);
    return p;
}

size_t smooth_ordered_workspace_bytes(int64_t n, int32_t k, sfg_dtype storage) {
    Carver c(nullptr);
    plan_smooth(c, n, k, storage);
    plan_mpk(c, n, 8);
    return c.used + 512;
}

namespace {

// Columns a pass workgroup takes: the whole row (up to 128 bytes).
// SFG_PASS_COLS = 8 (FP64) or 16 (FP32) splits 128-byte rows into two
// 64-byte column groups instead, for tuning (measured on the 200^3 mesh's
// tree: no faster at 3 hops, slower at 2).
template <typename TX>
int pass_cols(int32_t k) {
    const int narrow = 64 / (int)sizeof(TX);
    const int forced = env_int("SFG_PASS_COLS", 0);
    if (forced == narrow && k % narrow == 0) return narrow;
    return k;
}

// Weights and arithmetic: FP64 for FP64 storage, FP32 otherwise (as sfg_smooth).
// The common-case launch over every block at the small capacity, then the
// blocks over it at the layout's full capacity.
// Launches of one pass: the common-case launch over every block, the
// full-capacity launch over the listed blocks.
constexpr int kPartSmall = 1, kPartListed = 2, kPartBoth = 3;

template <int H, int KC, typename TX, typename TO, bool CENTER>
void launch_pass_kc(int32_t k, int32_t m, const MpkPlan &mp, int64_t nb, const void *x, const double *mean, TO *y,
                    double omega, hipStream_t s, int parts) {
    using TIN = typename std::conditional<CENTER, double, TX>::type;
    using TA = typename std::conditional<sizeof(TX) == 8, double, float>::type;
    constexpr int KS = mpk_small_slots<H, KC, TX, TA>();
    constexpr int KF = MpkCaps<H>::kSlots;
    const int64_t items = nb * (k / KC);
    SFG_REQUIRE(items <= 0x7fffffff, SFG_EUNSUPPORTED, "smooth_ordered: too many blocks");
    SFG_REQUIRE(mp.small_slots == KS, SFG_EUNSUPPORTED, "smooth_ordered: layout listed for another capacity");
    if (parts & kPartSmall) {
        hipLaunchKernelGGL((k_sweep_pass<H, KC, KS, false, TIN, TX, TO, TA, TA, 4, CENTER>), dim3((uint32_t)items),
                           dim3(256), 0, s, k, m, mp.dev, nullptr, (const TIN *)x, mean, y, (TA)(1.0 - omega),
                           (TA)omega);
        SFG_LAUNCH_CHECK();
    }
    if constexpr (KS < KF && !mpk_gathers<H, KS>()) {
        if ((parts & kPartListed) && mp.nbig > 0) {
            hipLaunchKernelGGL((k_sweep_pass<H, KC, KF, true, TIN, TX, TO, TA, TA, 4, CENTER>),
                               dim3((uint32_t)(mp.nbig * (k / KC))), dim3(256), 0, s, k, m, mp.dev, mp.big,
                               (const TIN *)x, mean, y, (TA)(1.0 - omega), (TA)omega);
            SFG_LAUNCH_CHECK();
        }
    }
}

// Slots of the common-case launch for this storage, k and hop count (the
// same constant launch_pass_kc instantiates).
template <int H, typename TX>
int small_slots_for(int32_t k) {
    using TA = typename std::conditional<sizeof(TX) == 8, double, float>::type;
    using C = MpkCaps<H>;
    return mpk_small_slots(C::kSlots, C::kRows, C::kEnt, (int)sizeof(typename C::Col), pass_cols<TX>(k),
                           (int)sizeof(TX), (int)sizeof(TA));
}

template <int H>
int small_slots(sfg_dtype storage, int32_t k) {
    switch (storage) {
        case SFG_F64: return small_slots_for<H, double>(k);
        case SFG_F32: return small_slots_for<H, float>(k);
        default: return small_slots_for<H, __half>(k);
    }
}

template <int H, typename TX, typename TO, bool CENTER>
void launch_pass(int32_t k, int32_t m, const MpkPlan &mp, int64_t nb, const void *x, const double *mean, TO *y,
                 double omega, hipStream_t s, int parts) {
    constexpr int wide = 128 / (int)sizeof(TX);
    switch (pass_cols<TX>(k)) {
        case 4: launch_pass_kc<H, 4, TX, TO, CENTER>(k, m, mp, nb, x, mean, y, omega, s, parts); return;
        case 8: launch_pass_kc<H, 8, TX, TO, CENTER>(k, m, mp, nb, x, mean, y, omega, s, parts); return;
        case 12: launch_pass_kc<H, 12, TX, TO, CENTER>(k, m, mp, nb, x, mean, y, omega, s, parts); return;
        case 16: launch_pass_kc<H, 16, TX, TO, CENTER>(k, m, mp, nb, x, mean, y, omega, s, parts); return;
        default: break;
    }
    if constexpr (wide == 32) {
        switch (pass_cols<TX>(k)) {
            case 20: launch_pass_kc<H, 20, TX, TO, CENTER>(k, m, mp, nb, x, mean, y, omega, s, parts); return;
            case 24: launch_pass_kc<H, 24, TX, TO, CENTER>(k, m, mp, nb, x, mean, y, omega, s, parts); return;
            case 28: launch_pass_kc<H, 28, TX, TO, CENTER>(k, m, mp, nb, x, mean, y, omega, s, parts); return;
            case 32: launch_pass_kc<H, 32, TX, TO, CENTER>(k, m, mp, nb, x, mean, y, omega, s, parts); return;
            default: break;
        }
    }
    fail(SFG_EUNSUPPORTED, "smooth_ordered: no pass kernel for this width");
}

// Passes of H sweeps, the last one shorter when H does not divide the count;
// with final_f32 (16-bit storage) the very last sweep stores FP32.
// first_parts: the launches of the first pass to make here (the common-case
// one may have gone out already); first_only: stop after the first pass.
// p.mean holds the column means (enqueued earlier, on this stream or on one
// it waits for).
template <int H, typename TX>
void run_smooth_passes(const sfg_csr *H_, int32_t k, int32_t sweeps, double omega, const double *x0, void *xout,
                       bool final_f32, const SmoothPlan &p, const MpkPlan &mp, int64_t nb, hipStream_t s,
                       int first_parts, bool first_only) {
    TX *b0 = (TX *)p.buf0, *b1 = (TX *)p.buf1;
    const TX *src = nullptr;
    for (int32_t done = 0, q = 0; done < sweeps; ++q) {
        if (q == 1 && first_only) break;
        const int parts = q == 0 ? first_parts : kPartBoth;
        const int32_t m = sweeps - done < H ? sweeps - done : H;
        const bool last = done + m == sweeps;
        TX *dst = last ? (TX *)xout : (q % 2 == 0 ? b0 : b1);
        if constexpr (sizeof(TX) == 2) {
            if (last && final_f32) {
                if (q == 0)
                    launch_pass<H, TX, float, true>(k, m, mp, nb, x0, p.mean, (float *)xout, omega, s, parts);
                else
                    launch_pass<H, TX, float, false>(k, m, mp, nb, src, nullptr, (float *)xout, omega, s, parts);
                break;
            }
        }
        if (q == 0)
            launch_pass<H, TX, TX, true>(k, m, mp, nb, x0, p.mean, dst, omega, s, parts);
        else
            launch_pass<H, TX, TX, false>(k, m, mp, nb, src, nullptr, dst, omega, s, parts);
        src = dst;
        done += m;
    }
}

template <int H>
void run_passes(sfg_dtype storage, const sfg_csr *G, int32_t k, int32_t sweeps, double omega, const double *x0,
                void *x, bool final_f32, const SmoothPlan &p, const MpkPlan &mp, int64_t nb, hipStream_t s,
                int first_parts, bool first_only) {
    switch (storage) {
        case SFG_F64:
            run_smooth_passes<H, double>(G, k, sweeps, omega, x0, x, false, p, mp, nb, s, first_parts, first_only);
            return;
        case SFG_F32:
            run_smooth_passes<H, float>(G, k, sweeps, omega, x0, x, false, p, mp, nb, s, first_parts, first_only);
            return;
        case SFG_F16:
            run_smooth_passes<H, __half>(G, k, sweeps, omega, x0, x, final_f32, p, mp, nb, s, first_parts,
                                         first_only);
            return;
        case SFG_BF16:
            run_smooth_passes<H, __hip_bfloat16>(G, k, sweeps, omega, x0, x, final_f32, p, mp, nb, s, first_parts,
                                                 first_only);
            return;
        default: break;
    }
    fail(SFG_EUNSUPPORTED, "smooth_ordered: storage");
}

void run_passes_h(int hops, sfg_dtype storage, const sfg_csr *G, int32_t k, int32_t sweeps, double omega,
                  const double *x0, void *x, bool final_f32, const SmoothPlan &p, const MpkPlan &mp, int64_t nb,
                  hipStream_t s, int first_parts, bool first_only) {
    if (hops == 4) run_passes<4>(storage, G, k, sweeps, omega, x0, x, final_f32, p, mp, nb, s, first_parts, first_only);
    else if (hops == 3)
        run_passes<3>(storage, G, k, sweeps, omega, x0, x, final_f32, p, mp, nb, s, first_parts, first_only);
    else run_passes<2>(storage, G, k, sweeps, omega, x0, x, final_f32, p, mp, nb, s, first_parts, first_only);
}

template <int H>
void build_layout(const sfg_csr *G, const int32_t *order, const MpkPlan &mp, int64_t nb, hipStream_t s) {
    if (G->vt == SFG_F64)
        hipLaunchKernelGGL((k_mpk_build<H, double>), dim3((uint32_t)nb), dim3(64), 0, s, G->n, order, G->rowptr,
                           G->col, (const double *)G->val, (const double *)G->deg, mp.dev, mp.flag);
    else
        hipLaunchKernelGGL((k_mpk_build<H, float>), dim3((uint32_t)nb), dim3(64), 0, s, G->n, order, G->rowptr,
                           G->col, (const float *)G->val, (const float *)G->deg, mp.dev, mp.flag);
    SFG_LAUNCH_CHECK();
}

// The layout's two flag words, copied to pinned host memory (one buffer and
// one event per device, created on first use and kept for the process).
// begin() enqueues the copy; the host may enqueue more work before wait(),
// which blocks until the copy is done (not until the stream drains).  The
// buffer is held, under its device's lock, from begin() to wait().
class FlagRead {
  public:
    FlagRead(MpkPlan &mp, hipStream_t s) : mp_(mp), s_(s) {
        int dev = 0;
        SFG_HIP(hipGetDevice(&dev));
        SFG_REQUIRE(dev >= 0 && dev < 64, SFG_EUNSUPPORTED, "smooth_ordered: device index over 63");
        Slot &sl = slot(dev);
        lock_ = std::unique_lock<std::mutex>(sl.mu);
        if (!sl.host) {
            SFG_HIP(hipHostMalloc((void **)&sl.host, 2 * sizeof(int32_t), hipHostMallocDefault));
            SFG_HIP(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
        }
        sl_ = &sl;
        SFG_HIP(hipMemcpyAsync(sl.host, mp.flag, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        SFG_HIP(hipEventRecord(sl.ev, s));
    }
    // Left without wait() (an error in between): the copy lands before the
    // buffer goes to the next caller.
    ~FlagRead() {
        if (lock_.owns_lock()) (void)hipEventSynchronize(sl_->ev);
    }
    FlagRead(const FlagRead &) = delete;
    FlagRead &operator=(const FlagRead &) = delete;
    // The flag word; bit 0 (the order is not a permutation) raises SFG_EINVAL
    // once the stream has drained, so nothing enqueued after begin() still
    // runs when the error reaches the caller.
    int32_t wait() {
        SFG_HIP(hipEventSynchronize(sl_->ev));
        const int32_t f = sl_->host[0];
        mp_.nbig = sl_->host[1];
        lock_.unlock();
        if (f & 1) {
            SFG_HIP(hipStreamSynchronize(s_));
            fail(SFG_EINVAL, "smooth_ordered: order is not a permutation of the nodes");
        }
        return f;
    }

  private:
    struct Slot {
        std::mutex mu;
        int32_t *host = nullptr;
        hipEvent_t ev = nullptr;
    };
    static Slot &slot(int dev) {
        static Slot slots[64];
        return slots[dev];
    }
    MpkPlan &mp_;
    hipStream_t s_;
    Slot *sl_ = nullptr;
    std::unique_lock<std::mutex> lock_;
};

int32_t read_flag(MpkPlan &mp, hipStream_t s) {
    FlagRead fr(mp, s);
    return fr.wait();
}

// Lists the blocks over the common-case capacity (flag[1] counts them).
template <int H>
void list_big(MpkPlan &mp, int64_t nb, sfg_dtype storage, int32_t k, hipStream_t s) {
    mp.small_slots = small_slots<H>(storage, k);
    // no list where the common-case launch sweeps every block (mpk_gathers)
    const bool gathers = kMpkGatherWide && MpkCaps<H>::kRows <= mp.small_slots;
    if (mp.small_slots < MpkCaps<H>::kSlots && !gathers) {
        hipLaunchKernelGGL(k_mpk_big<H>, dim3(grid_for(nb, 256)), dim3(256), 0, s, nb, mp.dev.meta, mp.small_slots,
                           mp.big, mp.flag + 1);
        SFG_LAUNCH_CHECK();
    }
}

}  // namespace

// Same result as smooth(); see sfg_smooth_ordered in the header.  Returns the
// sweeps each pass over X took: 1 when the plain path ran, else 2 to 4.
// The passes are taken when sweeps x (bytes of a block row) >= kMpkMinBytes:
// the layout pass and the per-block local CSR cost about as much as a few
// sweeps of a narrow block.  Measured on the 200^3 mesh's tree (one
// smoothing call, passes of 3 against one sweep per launch): BF16 16
// vectors, 10 sweeps (320 bytes) 2.50 ms against 3.04; FP32 4 vectors, 20
// sweeps (320) 2.35 against 2.74; FP32 4 vectors, 10 sweeps (160) 1.57
// against 1.49; BF16 4 vectors, 20 sweeps (160) 2.35 against 2.28.
// Setting SFG_SWEEP_HOPS takes the passes at any width.
constexpr int64_t kMpkMinBytes = 320;
// Graphs averaging more entries per row than this (whole meshes, power-law
// graphs) have 1-hop halos beyond the layout's capacities for 64-row blocks:
// they go to the plain path without trying a layout (SFG_SWEEP_HOPS still
// forces the try).
constexpr int64_t kMpkMaxEntriesPerRow = 4;

// Hops are tried from SFG_SWEEP_HOPS (2, 3 or 4; default 2 in FP64, 3 in
// FP32) down to 2 until every block's layout fits.  Measured on the 200^3
// mesh's spanning tree in preorder, 16 vectors, per sweep: FP64 289 us with
// 2 hops, 293 with 3, 334 with 4 (the deeper passes read X fewer times but
// keep fewer workgroups a CU, and the gathers' latency then shows); FP32
// 152-163 us with 3 hops, 177 with 2, 174 with 4.
int default_hops(sfg_dtype storage) { return storage == SFG_F64 ? 2 : 3; }

// order == nullptr: the rows' own numbering (a graph already relabelled
// into a locality order).  max_row as for smooth() (the plain path's FP64 hub
// rows).
int smooth_ordered(const sfg_csr *H, const int32_t *order, int32_t k, int32_t sweeps, double omega,
                   const double *x0, sfg_dtype storage, int32_t final_f32, void *x, void *ws, size_t ws_bytes,
                   hipStream_t s, int32_t max_row) {
    SFG_REQUIRE(H, SFG_EINVAL, "smooth_ordered: null pointer");
    SFG_REQUIRE(H->n >= 1, SFG_EINVAL, "smooth_ordered: empty graph");
    SFG_REQUIRE(ws_bytes >= smooth_ordered_workspace_bytes(H->n, k < 1 ? 1 : k, storage), SFG_EWORKSPACE,
                "smooth_ordered: workspace too small");
    const int64_t n = H->n;
    Carver c(ws);
    SmoothPlan p = plan_smooth(c, n, k < 1 ? 1 : k, storage);
    MpkPlan mp = plan_mpk(c, n, 8);
    const size_t sx = dtype_size(storage);
    const int want = env_int("SFG_SWEEP_HOPS", default_hops(storage));
    const bool pays = getenv("SFG_SWEEP_HOPS") != nullptr ||
                      ((int64_t)sweeps * k * (int64_t)dtype_size(storage) >= kMpkMinBytes &&
                       H->nnz <= kMpkMaxEntriesPerRow * H->n);
    // FP64 storage on FP64 weights; FP32, FP16, BF16 storage on FP32 weights (as sfg_smooth); 16-bit rows up
    // to 16 columns
    const bool types_ok = storage == SFG_F64 ? H->vt == SFG_F64
                                             : (H->vt == SFG_F32 && (storage == SFG_F32 || k <= 16) &&
                                                (storage == SFG_F32 || storage == SFG_F16 || storage == SFG_BF16));
    const bool shape_ok = types_ok && pays && k >= 1 && k % 4 == 0 && (size_t)k * sx <= (size_t)kMpkRowBytes &&
                          sweeps >= 2 && H->nnz >= 1 && H->col && H->val && H->deg && want >= 2;
    const int64_t nb = mpk_blocks(n);
    int hops = 0;
    bool started = false;
    if (shape_ok) {
        SFG_REQUIRE(omega > 0.0 && omega <= 1.0, SFG_EINVAL, "smooth_ordered: omega must be in (0, 1]");
        SFG_REQUIRE(x0 && x, SFG_EINVAL, "smooth_ordered: null pointer");
        const bool f32last = final_f32 && (storage == SFG_F16 || storage == SFG_BF16);
        // the column means on a side stream, beside the layout pass (which
        // waits on dependent loads rather than on bandwidth); the first pass
        // waits for them
        struct Fork {
            hipEvent_t es = nullptr, ez = nullptr;
            ~Fork() {
                if (es) (void)hipEventDestroy(es);
                if (ez) (void)hipEventDestroy(ez);
            }
        } fork;
        SFG_HIP(hipEventCreateWithFlags(&fork.es, hipEventDisableTiming));
        SFG_HIP(hipEventCreateWithFlags(&fork.ez, hipEventDisableTiming));
        fill_i32(mp.flag, 2, 0, s);
        if (order) {
            // the passes take the rows in this order: it must be a permutation of the nodes
            hipLaunchKernelGGL(k_mpk_mark, dim3(grid_for(n, 256)), dim3(256), 0, s, n, order, mp.seen, mp.flag);
            SFG_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_mpk_verify, dim3(grid_for(n, 256)), dim3(256), 0, s, n, order, mp.seen, mp.flag);
            SFG_LAUNCH_CHECK();
        }
        const hipStream_t side = side_stream();
        SFG_HIP(hipEventRecord(fork.es, s));   // after everything so far on s (x0 among it)
        SFG_HIP(hipStreamWaitEvent(side, fork.es, 0));
        launch_column_means<double>(x0, n, k, p.partial, p.mean, side);
        SFG_HIP(hipEventRecord(fork.ez, side));
        const int first = want < kMpkMaxHops ? want : kMpkMaxHops;
        for (int h = first; h >= 2 && hops == 0; --h) {
            if (h == 4) {
                build_layout<4>(H, order, mp, nb, s);
                list_big<4>(mp, nb, storage, k, s);
            } else if (h == 3) {
                build_layout<3>(H, order, mp, nb, s);
                list_big<3>(mp, nb, storage, k, s);
            } else {
                build_layout<2>(H, order, mp, nb, s);
                list_big<2>(mp, nb, storage, k, s);
            }
            int32_t f;
            if (h == first) {
                // while the host waits for the flags, the GPU finishes the column means and takes the
                // common-case launch of the first pass: the start of the smoothing if the layout stands, redone
                // otherwise (blocks that do not fit have zero sizes, so the launch stays inside every buffer
                // either way)
                FlagRead fr(mp, s);
                SFG_HIP(hipStreamWaitEvent(s, fork.ez, 0));   // join: the means before the first pass
                run_passes_h(h, storage, H, k, sweeps, omega, x0, x, f32last, p, mp, nb, s, kPartSmall, true);
                f = fr.wait();
                started = !(f & 2);
            } else {
                f = read_flag(mp, s);
            }
            if (f & 2)
                fill_i32(mp.flag, 2, 0, s);     // a block did not fit: fewer hops
            else
                hops = h;
        }
        if (hops >= 2) {
            run_passes_h(hops, storage, H, k, sweeps, omega, x0, x, f32last, p, mp, nb, s,
                         started ? kPartListed : kPartBoth, false);
            return hops;
        }
    }
    // the workspace starts with the plain smoothing's layout
    smooth(H, k, sweeps, omega, x0, storage, final_f32, x, ws, smooth_workspace_bytes(n, k < 1 ? 1 : k, storage), s,
           max_row);
    return 1;
}

// Column means of a block (exact to double-double before one rounding);
// used for the affinity's centring.
void column_means(const void *x, sfg_dtype xt, int64_t n, int32_t k, double *mean, void *partial_ws,
                  hipStream_t s) {
    DD *partial = (DD *)partial_ws;
    if (xt == SFG_F64)
        launch_column_means<double>((const double *)x, n, k, partial, mean, s);
    else if (xt == SFG_F32)
        launch_column_means<float>((const float *)x, n, k, partial, mean, s);
    else
        fail(SFG_EUNSUPPORTED, "column_means: F64 or F32 block required");
}

size_t column_means_partial_bytes(int64_t n, int32_t k) { return (size_t)colsum_blocks(n) * k * sizeof(DD); }

}  // namespace sfg

extern "C" sfg_status sfg_smooth_ordered(const sfg_csr *H, const int32_t *order, int32_t k, int32_t sweeps,
                                         double omega, const double *x0, sfg_dtype storage, int32_t final_f32,
                                         void *x, int32_t *per_pass_out, void *ws, size_t ws_bytes, void *stream) {
    return sfg::guard([&] {
        SFG_REQUIRE(order, SFG_EINVAL, "smooth_ordered: null order");
        const int used = sfg::smooth_ordered(H, order, k, sweeps, omega, x0, storage, final_f32, x, ws, ws_bytes,
                                             sfg::as_stream(stream), -1);
        if (per_pass_out) *per_pass_out = used;
    });
}

extern "C" sfg_status sfg_smooth(const sfg_csr *H, int32_t k, int32_t sweeps, double omega, const double *x0,
                                 sfg_dtype storage, int32_t final_f32, void *x, void *ws, size_t ws_bytes,
                                 void *stream) {
    return sfg::guard([&] {
        sfg::smooth(H, k, sweeps, omega, x0, storage, final_f32, x, ws, ws_bytes, sfg::as_stream(stream), -1);
    });
}
