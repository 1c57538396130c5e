// Adjacency CSR and degree vector of a weighted graph (Sec. 2.1 of the
// paper: A(p,q) = w(p,q), D(p,p) = sum of the weights at p, L = D - A).
//
// Input is a canonical edge list (u < v, sorted by (u, v)), optionally
// masked.  Row p of the CSR holds first the edges (q, p) with q < p -- its
// "lower" part -- then the edges (p, q) with q > p.  Because the list is
// sorted by (u, v), ascending column order inside a row is ascending edge id
// order, and the degree is summed in that order in FP64.
//
//  1. count included edges per row (lower and upper parts) and all edges per
//     u (to find each row's slice of the edge list)
//  2. two exclusive scans: rowptr and the edge-list start of each row
//  3. drop each lower entry's edge id into its row (unordered, atomic slot)
//  4. order each row's lower part by edge id: rank = number of smaller ids
//     in the segment (a thread per short row, a wavefront per long one)
//  5. one thread per row writes col/val/eid and the degree, in column order
#include "common.hpp"

namespace sfg {

namespace {

struct CsrPlan {
    int32_t *cnt_lo, *cnt_hi, *cnt_all, *tmp, *estart, *fill, *scan, *long_cnt;
};

CsrPlan plan_csr(Carver &c, int64_t n, int64_t m) {
    (void)m;
    CsrPlan p;
    p.cnt_lo = c.take<int32_t>(n + 1);
    p.cnt_hi = c.take<int32_t>(n + 1);
    p.cnt_all = c.take<int32_t>(n + 1);
    p.tmp = c.take<int32_t>(n + 1);
    p.estart = c.take<int32_t>(n + 1);
    p.fill = c.take<int32_t>(n + 1);
    p.scan = c.take<int32_t>(scan_scratch_ints(n + 1));
    p.long_cnt = c.take<int32_t>(1);
    return p;
}

__global__ void k_count(int64_t m, const int32_t *__restrict__ u, const int32_t *__restrict__ v,
                        const uint8_t *__restrict__ mask, int32_t *cnt_lo, int32_t *cnt_hi,
                        int32_t *cnt_all) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const int32_t a = u[e], b = v[e];
    atomicAdd(&cnt_all[a], 1);
    if (mask && mask[e] == 0) return;
    atomicAdd(&cnt_hi[a], 1);
    atomicAdd(&cnt_lo[b], 1);
}

__global__ void k_row_total(int64_t n, const int32_t *cnt_lo, const int32_t *cnt_hi, int32_t *tot) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) tot[p] = cnt_lo[p] + cnt_hi[p];
}

__global__ void k_place_lower(int64_t m, const int32_t *__restrict__ v, const uint8_t *__restrict__ mask,
                              const int32_t *__restrict__ rowptr, int32_t *fill, int32_t *eid) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    if (mask && mask[e] == 0) return;
    const int32_t b = v[e];
    const int32_t slot = atomicAdd(&fill[b], 1);
    eid[rowptr[b] + slot] = (int32_t)e;
}

// Order the lower part of each row by edge id.  Reads the unordered ids from
// `eid`, writes them ordered into `col` (used as scratch here).  Ids in a
// segment are distinct, so rank = count of smaller ids.  Short segments (the
// common case) take one thread each; longer ones are queued for a wavefront.
constexpr int kShortSeg = 32;

__global__ __launch_bounds__(256) void k_rank_short(int64_t n, const int32_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ cnt_lo,
                                                    const int32_t *__restrict__ eid, int32_t *col,
                                                    int32_t *long_rows, int32_t *long_cnt) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= n) return;
    const int32_t len = cnt_lo[row];
    if (len > kShortSeg) {
        long_rows[atomicAdd(long_cnt, 1)] = (int32_t)row;
        return;
    }
    const int32_t base = rowptr[row];
    for (int32_t i = 0; i < len; ++i) {
        const int32_t mine = eid[base + i];
        int32_t rank = 0;
        for (int32_t j = 0; j < len; ++j) rank += (eid[base + j] < mine) ? 1 : 0;
        col[base + rank] = mine;
    }
}

__global__ __launch_bounds__(256) void k_rank_long(const int32_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ cnt_lo,
                                                   const int32_t *__restrict__ eid, int32_t *col,
                                                   const int32_t *__restrict__ long_rows,
                                                   const int32_t *__restrict__ long_cnt) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / kWave);
    const int32_t cnt = *long_cnt;
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; r < cnt; r += nwaves) {
        const int32_t row = long_rows[r];
        const int32_t len = cnt_lo[row];
        const int32_t base = rowptr[row];
        for (int32_t i = lane; i < len; i += kWave) {
            const int32_t mine = eid[base + i];
            int32_t rank = 0;
            for (int32_t j = 0; j < len; ++j) rank += (eid[base + j] < mine) ? 1 : 0;
            col[base + rank] = mine;
        }
    }
}

template <typename TW>
__global__ void k_fill_rows(int64_t n, const int32_t *__restrict__ u, const int32_t *__restrict__ v,
                            const TW *__restrict__ w, const uint8_t *__restrict__ mask,
                            const int32_t *__restrict__ rowptr, const int32_t *__restrict__ cnt_lo,
                            const int32_t *__restrict__ estart, int32_t *col, TW *val, int32_t *eid,
                            TW *deg) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int32_t j = rowptr[p];
    double d = 0.0;
    const int32_t nlo = cnt_lo[p];
    for (int32_t t = 0; t < nlo; ++t, ++j) {
        const int32_t e = col[j];          // ordered lower ids left by the rank kernels
        eid[j] = e;
        col[j] = u[e];
        const TW we = w[e];
        val[j] = we;
        d = d + (double)we;
    }
    const int32_t e1 = estart[p + 1];
    for (int32_t e = estart[p]; e < e1; ++e) {
        if (mask && mask[e] == 0) continue;
        eid[j] = e;
        col[j] = v[e];
        const TW we = w[e];
        val[j] = we;
        d = d + (double)we;
        ++j;
    }
    deg[p] = (TW)d;
}

}  // namespace

size_t csr_workspace_bytes(int64_t n, int64_t m) {
    Carver c(nullptr);
    plan_csr(c, n, m);
    return c.used + 256;
}

void build_csr(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
               const uint8_t *mask, int32_t *rowptr, int32_t *col, void *val, int32_t *eid, void *deg,
               void *ws, size_t ws_bytes, hipStream_t s) {
    SFG_REQUIRE(n >= 1 && m >= 0, SFG_EINVAL, "laplacian_csr: need n >= 1 and m >= 0");
    SFG_REQUIRE(2 * m < (int64_t(1) << 31), SFG_EUNSUPPORTED, "laplacian_csr: 2*m must be < 2^31");
    SFG_REQUIRE(n < (int64_t(1) << 31) - 1, SFG_EUNSUPPORTED, "laplacian_csr: n must be < 2^31-1");
    SFG_REQUIRE(wt == SFG_F64 || wt == SFG_F32, SFG_EINVAL, "laplacian_csr: weights must be F64 or F32");
    SFG_REQUIRE(ws_bytes >= csr_workspace_bytes(n, m), SFG_EWORKSPACE, "laplacian_csr: workspace too small");
    SFG_REQUIRE(rowptr && deg && (m == 0 || (u && v && w && col && val && eid)), SFG_EINVAL,
                "laplacian_csr: null pointer");
    Carver c(ws);
    CsrPlan p = plan_csr(c, n, m);
    fill_i32(p.cnt_lo, n + 1, 0, s);
    fill_i32(p.cnt_hi, n + 1, 0, s);
    fill_i32(p.cnt_all, n + 1, 0, s);
    fill_i32(p.fill, n + 1, 0, s);
    if (m > 0) {
        hipLaunchKernelGGL(k_count, dim3(grid_for(m, 256)), dim3(256), 0, s, m, u, v, mask, p.cnt_lo, p.cnt_hi,
                           p.cnt_all);
        SFG_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_row_total, dim3(grid_for(n, 256)), dim3(256), 0, s, n, p.cnt_lo, p.cnt_hi, p.tmp);
    SFG_LAUNCH_CHECK();
    exclusive_scan_i32(p.tmp, rowptr, n, p.scan, s);
    exclusive_scan_i32(p.cnt_all, p.estart, n, p.scan, s);
    if (m > 0) {
        hipLaunchKernelGGL(k_place_lower, dim3(grid_for(m, 256)), dim3(256), 0, s, m, v, mask, rowptr, p.fill,
                           eid);
        SFG_LAUNCH_CHECK();
        fill_i32(p.long_cnt, 1, 0, s);
        // p.tmp (the row totals) is free once rowptr is scanned: it holds the long-row queue
        hipLaunchKernelGGL(k_rank_short, dim3(grid_for(n, 256)), dim3(256), 0, s, n, rowptr, p.cnt_lo, eid, col,
                           p.tmp, p.long_cnt);
        SFG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_rank_long, dim3(256), dim3(256), 0, s, rowptr, p.cnt_lo, eid, col, p.tmp, p.long_cnt);
        SFG_LAUNCH_CHECK();
    }
    if (wt == SFG_F64)
        hipLaunchKernelGGL(k_fill_rows<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, n, u, v,
                           (const double *)w, mask, rowptr, p.cnt_lo, p.estart, col, (double *)val, eid,
                           (double *)deg);
    else
        hipLaunchKernelGGL(k_fill_rows<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, n, u, v,
                           (const float *)w, mask, rowptr, p.cnt_lo, p.estart, col, (float *)val, eid,
                           (float *)deg);
    SFG_LAUNCH_CHECK();
}

}  // namespace sfg

extern "C" sfg_status sfg_laplacian_csr(int64_t n, int64_t m, const int32_t *u, const int32_t *v,
                                        const void *w, sfg_dtype wt, const uint8_t *mask, int32_t *rowptr,
                                        int32_t *col, void *val, int32_t *eid, void *deg, int64_t *nnz_out,
                                        void *ws, size_t ws_bytes, void *stream) {
    return sfg::guard([&] {
        hipStream_t s = sfg::as_stream(stream);
        sfg::build_csr(n, m, u, v, w, wt, mask, rowptr, col, val, eid, deg, ws, ws_bytes, s);
        if (nnz_out) {
            int32_t nnz = 0;
            SFG_HIP(hipMemcpyAsync(&nnz, rowptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            SFG_HIP(hipStreamSynchronize(s));
            *nnz_out = nnz;
        }
    });
}
