// Adjacency CSR and degree vector of a weighted graph (Sec. 2.1 of the
// paper: A(p,q) = w(p,q), D(p,p) = sum of the weights at p, L = D - A).
//
// Input is a canonical edge list (u < v, sorted by (u, v)), optionally
// masked.  Row p of the CSR holds first the edges (q, p) with q < p -- its
// "lower" part -- then the edges (p, q) with q > p.  Because the list is
// sorted by (u, v), ascending column order inside a row is ascending edge id
// order, and the degree is summed in that order in FP64.
//
//  1. the edge-list slice of every row (its upper edges) by one coalesced
//     pass over u
//  2. sparse edge lists (at most kWalkDensity edges per node): a thread per
//     row walks its slice: it counts its included upper edges and adds one to
//     the lower count of each one's other end (integer atomics); slices over
//     kWalk edges are walked by a wavefront instead.  Denser lists: a thread
//     per edge counts, and a scan of the mask flags ranks the included edges
//     within their slices.  One scan of the row totals gives rowptr
//  3. the same walk again (denser lists: a thread per edge): each included
//     edge writes its upper entry in place, in order, and drops itself into
//     the lower part of its other row at an atomic slot (column, weight and
//     id written there)
//  4. lower parts of two or more entries are put in edge-id order: a thread
//     per row ranks up to kRegSeg entries in registers, a workgroup per longer
//     row bitonic-sorts the ids in LDS
//  5. one thread per row sums its weights in column order, in FP64; rows
//     over 256 entries (hubs) are staged through LDS by a wavefront and
//     summed by one of its lanes in the same order
#include "common.hpp"

namespace sfg {

namespace {

constexpr int kWalk = 64;           // upper slices longer than this: walked by a wavefront
constexpr int kRegSeg = 8;          // lower parts up to this length: ranked in registers by one thread
constexpr int kShortSeg = 32;       // up to this length: ranked by one thread; longer ones by a workgroup
constexpr int kLdsSeg = 8192;       // longer ones are sorted in LDS up to this length
constexpr int kDegLong = 256;       // rows longer than this: degree summed by a workgroup

struct CsrPlan {
    int32_t *estart, *up, *cnt_lo, *tot, *fill, *tmp, *walk_rows, *walk_cnt, *long_rows, *long_cnt, *deg_rows,
        *deg_cnt, *inc, *incpos, *scan;
    int32_t *zeroed;      // cnt_lo, fill, the three list counters: one contiguous range, cleared by one fill
    int64_t zeroed_len;
};

CsrPlan plan_csr(Carver &c, int64_t n, int64_t m) {
    CsrPlan p;
    p.estart = c.take<int32_t>(n + 1);
    p.up = c.take<int32_t>(n + 1);
    p.zeroed_len = 2 * (n + 1) + 3;
    p.zeroed = c.take<int32_t>(p.zeroed_len);
    p.cnt_lo = p.zeroed;
    p.fill = p.zeroed + (n + 1);
    p.walk_cnt = p.zeroed + 2 * (n + 1);
    p.long_cnt = p.walk_cnt + 1;
    p.deg_cnt = p.walk_cnt + 2;
    p.tot = c.take<int32_t>(n + 1);
    p.tmp = c.take<int32_t>(2 * m + 1);
    p.walk_rows = c.take<int32_t>(n + 1);
    p.long_rows = c.take<int32_t>(n + 1);
    p.deg_rows = c.take<int32_t>(n + 1);
    p.inc = c.take<int32_t>(m + 1);
    p.incpos = c.take<int32_t>(m + 1);
    p.scan = c.take<int32_t>(scan_scratch_ints((n > m ? n : m) + 1));
    return p;
}

// Graphs whose edge list holds at most this many edges per node (meshes,
// trees, power grids) are built by row walks; denser ones (power-law graphs,
// coarse Galerkin graphs) have many slices too long for one thread and are
// built edge-parallel.  Both give the same CSR.
constexpr int64_t kWalkDensity = 4;

// estart[p] = first edge with u >= p (p = 0..n).  The edge list is sorted by
// u, so edge e (e = 0..m, with u[-1] = -1 and u[m] = n) is that first edge for
// exactly the p in (u[e-1], u[e]]: one coalesced pass over the edges.  The
// range is clamped to [0, n], so an unsorted list cannot write out of bounds.
// A thread takes kEdgesPerThread consecutive edges (their u loads issued together).
constexpr int kEdgesPerThread = 4;

__global__ void k_estart(int64_t n, int64_t m, const int32_t *__restrict__ u, int32_t *estart) {
    const int64_t e0 = ((int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) * kEdgesPerThread;
    if (e0 > m) return;
    int64_t uu[kEdgesPerThread + 1];
#pragma unroll
    for (int t = 0; t <= kEdgesPerThread; ++t) {
        const int64_t e = e0 - 1 + t;
        uu[t] = e < 0 ? -1 : (e >= m ? n : (int64_t)u[e]);
    }
#pragma unroll
    for (int t = 0; t < kEdgesPerThread; ++t) {
        const int64_t e = e0 + t;
        if (e > m) break;
        int64_t lo = uu[t] + 1, hi = uu[t + 1];
        if (lo < 0) lo = 0;
        if (hi > n) hi = n;
        for (int64_t p = lo; p <= hi; ++p) estart[p] = (int32_t)e;
    }
}

// Row p's slice of the edge list, clamped to [0, m] (the walks never leave the
// list, whatever u held).
__device__ __forceinline__ void slice(int64_t p, int64_t m, const int32_t *__restrict__ estart, int32_t &a,
                                      int32_t &b) {
    int64_t lo = estart[p], hi = estart[p + 1];
    lo = lo < 0 ? 0 : (lo > m ? m : lo);
    hi = hi < lo ? lo : (hi > m ? m : hi);
    a = (int32_t)lo;
    b = (int32_t)hi;
}

// An edge of row p's slice that the CSR takes: in the mask, and its other end
// a node above p (anything else in a slice breaks the canonical form and is
// left out by both walks alike).
__device__ __forceinline__ bool takes(int64_t n, int64_t p, int32_t e, const int32_t *__restrict__ v,
                                      const uint8_t *__restrict__ mask, int32_t &q) {
    const bool on = mask ? mask[e] != 0 : true;
    q = v[e];
    return on && q > p && q < n;
}

constexpr int kGroup = 4;   // slice edges a thread handles with their loads and atomics issued together

// First walk: up[p] = included upper edges of row p; each adds one to the
// lower count of its other end.  Longer slices are listed for a wavefront.
// Rows go to the XCDs in contiguous ranges (xcd_remap), so the lower-part
// counters and entries of nearby rows stay in one XCD's L2.
__global__ void k_walk_count(int64_t n, int64_t m, const int32_t *__restrict__ estart, const int32_t *__restrict__ v,
                             const uint8_t *__restrict__ mask, int32_t *up, int32_t *cnt_lo, int32_t *walk_rows,
                             int32_t *walk_cnt) {
    const int64_t p = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int32_t a, b;
    slice(p, m, estart, a, b);
    if (b - a > kWalk) {
        walk_rows[atomicAdd(walk_cnt, 1)] = (int32_t)p;
        return;
    }
    int32_t c = 0;
    for (int32_t e0 = a; e0 < b; e0 += kGroup) {
        bool in[kGroup];
        int32_t q[kGroup];
#pragma unroll
        for (int t = 0; t < kGroup; ++t) in[t] = e0 + t < b && takes(n, p, e0 + t, v, mask, q[t]);
#pragma unroll
        for (int t = 0; t < kGroup; ++t)
            if (in[t]) {
                ++c;
                atomicAdd(&cnt_lo[q[t]], 1);
            }
    }
    up[p] = c;
}

// Listed slices: one wavefront per row, 64 edges at a time.
__global__ __launch_bounds__(256) void k_walk_count_long(int64_t n, int64_t m, const int32_t *__restrict__ estart,
                                                         const int32_t *__restrict__ v,
                                                         const uint8_t *__restrict__ mask, int32_t *up,
                                                         int32_t *cnt_lo, const int32_t *__restrict__ walk_rows,
                                                         const int32_t *__restrict__ walk_cnt) {
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t cnt = *walk_cnt;
    for (int32_t r = blockIdx.x * 4 + wv; r < cnt; r += gridDim.x * 4) {
        const int32_t p = walk_rows[r];
        int32_t a, b;
        slice(p, m, estart, a, b);
        int32_t c = 0;
        for (int32_t e0 = a; e0 < b; e0 += kWave) {
            const int32_t e = e0 + lane;
            int32_t q = 0;
            const bool in = e < b && takes(n, p, e, v, mask, q);
            if (in) atomicAdd(&cnt_lo[q], 1);
            c += __popcll(__ballot(in));
        }
        if (lane == 0) up[p] = c;
    }
}

__global__ void k_row_total(int64_t n, const int32_t *__restrict__ up, const int32_t *__restrict__ cnt_lo,
                            int32_t *tot) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) tot[p] = cnt_lo[p] + up[p];
}

// Edge e = (p, q) of row p's slice: the k-th included one is the upper entry
// rowptr[p] + cnt_lo[p] + k; its lower entry goes to an atomic slot of row q.
template <typename TW>
__device__ __forceinline__ void put_edge(int64_t p, int32_t q, int32_t e, int32_t k, const TW *__restrict__ w,
                                         const int32_t *__restrict__ rowptr, const int32_t *__restrict__ cnt_lo,
                                         int32_t *col, TW *val, int32_t *eid, int32_t *fill) {
    const TW we = w[e];
    const int32_t j = rowptr[p] + cnt_lo[p] + k;
    col[j] = q;
    val[j] = we;
    eid[j] = e;
    const int32_t i = rowptr[q] + atomicAdd(&fill[q], 1);
    col[i] = (int32_t)p;
    val[i] = we;
    eid[i] = e;
}

// Second walk, the same edges in the same order as the first.
template <typename TW>
__global__ void k_walk_fill(int64_t n, int64_t m, const int32_t *__restrict__ estart, const int32_t *__restrict__ v,
                            const TW *__restrict__ w, const uint8_t *__restrict__ mask,
                            const int32_t *__restrict__ rowptr, const int32_t *__restrict__ cnt_lo, int32_t *col,
                            TW *val, int32_t *eid, int32_t *fill) {
    const int64_t p = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int32_t a, b;
    slice(p, m, estart, a, b);
    if (b - a > kWalk) return;
    int32_t j = rowptr[p] + cnt_lo[p];
    for (int32_t e0 = a; e0 < b; e0 += kGroup) {
        bool in[kGroup];
        int32_t q[kGroup], at[kGroup];
        TW we[kGroup];
#pragma unroll
        for (int t = 0; t < kGroup; ++t) in[t] = e0 + t < b && takes(n, p, e0 + t, v, mask, q[t]);
#pragma unroll
        for (int t = 0; t < kGroup; ++t)
            if (in[t]) {
                we[t] = w[e0 + t];
                at[t] = rowptr[q[t]] + atomicAdd(&fill[q[t]], 1);
            }
#pragma unroll
        for (int t = 0; t < kGroup; ++t)
            if (in[t]) {
                const int32_t e = e0 + t;
                col[j] = q[t];
                val[j] = we[t];
                eid[j] = e;
                ++j;
                col[at[t]] = (int32_t)p;
                val[at[t]] = we[t];
                eid[at[t]] = e;
            }
    }
}

template <typename TW>
__global__ __launch_bounds__(256) void k_walk_fill_long(int64_t n, int64_t m, const int32_t *__restrict__ estart,
                                                        const int32_t *__restrict__ v, const TW *__restrict__ w,
                                                        const uint8_t *__restrict__ mask,
                                                        const int32_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ cnt_lo, int32_t *col, TW *val,
                                                        int32_t *eid, int32_t *fill,
                                                        const int32_t *__restrict__ walk_rows,
                                                        const int32_t *__restrict__ walk_cnt) {
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const uint64_t below = (uint64_t(1) << lane) - 1;
    const int32_t cnt = *walk_cnt;
    for (int32_t r = blockIdx.x * 4 + wv; r < cnt; r += gridDim.x * 4) {
        const int32_t p = walk_rows[r];
        int32_t a, b;
        slice(p, m, estart, a, b);
        int32_t k = 0;
        for (int32_t e0 = a; e0 < b; e0 += kWave) {
            const int32_t e = e0 + lane;
            int32_t q = 0;
            const bool in = e < b && takes(n, p, e, v, mask, q);
            const uint64_t bal = __ballot(in);
            if (in) put_edge(p, q, e, k + __popcll(bal & below), w, rowptr, cnt_lo, col, val, eid, fill);
            k += __popcll(bal);
        }
    }
}

// ---- edge-parallel build of denser graphs: mask flags and their scan give
// each included edge its rank within its row's slice; one thread per edge
// writes the upper entry in place and drops the lower entry at an atomic slot
// of its other row, as put_edge does for the walks.
__global__ void k_inc_count(int64_t m, const int32_t *__restrict__ v, const uint8_t *__restrict__ mask, int32_t *inc,
                            int32_t *cnt_lo) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const bool in = mask[e] != 0;
    inc[e] = in ? 1 : 0;
    if (in) atomicAdd(&cnt_lo[v[e]], 1);
}

__global__ void k_count_lo(int64_t m, const int32_t *__restrict__ v, int32_t *cnt_lo) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) atomicAdd(&cnt_lo[v[e]], 1);
}

__global__ void k_row_total_edges(int64_t n, const int32_t *__restrict__ estart, const int32_t *__restrict__ incpos,
                                  const int32_t *__restrict__ cnt_lo, int32_t *tot) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int32_t a = estart[p], b = estart[p + 1];
    tot[p] = cnt_lo[p] + (incpos ? incpos[b] - incpos[a] : b - a);
}

// The lower entries of this build go to their rows as edge ids only (tmp, at
// an atomic slot); k_rank_short_ids then writes them, ordered, with their
// columns and weights gathered from the edge list.
template <typename TW>
__global__ void k_fill_edges(int64_t m, const int32_t *__restrict__ u, const int32_t *__restrict__ v,
                             const TW *__restrict__ w, const uint8_t *__restrict__ mask,
                             const int32_t *__restrict__ incpos, const int32_t *__restrict__ estart,
                             const int32_t *__restrict__ rowptr, const int32_t *__restrict__ cnt_lo, int32_t *col,
                             TW *val, int32_t *eid, int32_t *fill, int32_t *tmp) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    if (mask && mask[e] == 0) return;
    const int32_t p = u[e], q = v[e];
    const int32_t k = incpos ? incpos[e] - incpos[estart[p]] : (int32_t)(e - estart[p]);
    const int32_t j = rowptr[p] + cnt_lo[p] + k;
    col[j] = q;
    val[j] = w[e];
    eid[j] = (int32_t)e;
    tmp[rowptr[q] + atomicAdd(&fill[q], 1)] = (int32_t)e;
}

// Lower parts of up to kShortSeg ids in tmp: ids in a segment are distinct,
// so the rank of an id is the number of smaller ids; the entry (column and
// weight gathered from the edge list) goes to base + rank.  Longer parts are
// listed for k_rank_long.

template <typename TW>
__global__ __launch_bounds__(256) void k_rank_short_ids(int64_t n, const int32_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ cnt_lo,
                                                        const int32_t *__restrict__ tmp,
                                                        const int32_t *__restrict__ u, const TW *__restrict__ w,
                                                        int32_t *col, TW *val, int32_t *eid, int32_t *long_rows,
                                                        int32_t *long_cnt) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= n) return;
    const int32_t len = cnt_lo[row];
    if (len > kShortSeg) {
        long_rows[atomicAdd(long_cnt, 1)] = (int32_t)row;
        return;
    }
    const int32_t base = rowptr[row];
    for (int32_t i = 0; i < len; ++i) {
        const int32_t mine = tmp[base + i];
        int32_t rank = 0;
        for (int32_t j = 0; j < len; ++j) rank += (tmp[base + j] < mine) ? 1 : 0;
        col[base + rank] = u[mine];
        val[base + rank] = w[mine];
        eid[base + rank] = mine;
    }
}

// Lower parts written in place at atomic slots (the row walks): parts of
// 2..kRegSeg entries are read into registers and each entry written back at
// its rank by edge id (ids in a row are distinct); parts up to kShortSeg are
// ranked from a copy of their ids in tmp; longer ones are listed for
// k_rank_long.  Parts of one entry are in place already.
template <typename TW>
__global__ __launch_bounds__(256) void k_rank_short(int64_t n, const int32_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ cnt_lo,
                                                    const int32_t *__restrict__ u, const TW *__restrict__ w,
                                                    int32_t *col, TW *val, int32_t *eid, int32_t *tmp,
                                                    int32_t *long_rows, int32_t *long_cnt) {
    const int64_t row = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (row >= n) return;
    const int32_t len = cnt_lo[row];
    if (len < 2) return;
    if (len > kShortSeg) {
        long_rows[atomicAdd(long_cnt, 1)] = (int32_t)row;
        return;
    }
    if (len > kRegSeg) {
        // ranked from a copy of the ids (the entries are rewritten in place), columns and weights gathered
        const int32_t b0 = rowptr[row];
        for (int32_t i = 0; i < len; ++i) tmp[b0 + i] = eid[b0 + i];
        for (int32_t i = 0; i < len; ++i) {
            const int32_t mine = tmp[b0 + i];
            int32_t rank = 0;
            for (int32_t j = 0; j < len; ++j) rank += (tmp[b0 + j] < mine) ? 1 : 0;
            col[b0 + rank] = u[mine];
            val[b0 + rank] = w[mine];
            eid[b0 + rank] = mine;
        }
        return;
    }
    // the ids first: a part already in edge-id order (half of the two-entry
    // parts) is left as it is; otherwise its columns and weights are loaded
    // too and the entries that move are written at their ranks
    const int32_t base = rowptr[row];
    int32_t id[kRegSeg], rank[kRegSeg];
#pragma unroll
    for (int i = 0; i < kRegSeg; ++i) id[i] = i < len ? eid[base + i] : INT32_MAX;
    bool moves = false;
#pragma unroll
    for (int i = 0; i < kRegSeg; ++i) {
        rank[i] = 0;
#pragma unroll
        for (int j = 0; j < kRegSeg; ++j) rank[i] += id[j] < id[i] ? 1 : 0;
        moves = moves || (i < len && rank[i] != i);
    }
    if (!moves) return;
    int32_t c[kRegSeg];
    TW x[kRegSeg];
#pragma unroll
    for (int i = 0; i < kRegSeg; ++i) {
        c[i] = i < len ? col[base + i] : 0;
        x[i] = i < len ? val[base + i] : TW(0);
    }
#pragma unroll
    for (int i = 0; i < kRegSeg; ++i)
        if (i < len && rank[i] != i) {
            col[base + rank[i]] = c[i];
            val[base + rank[i]] = x[i];
            eid[base + rank[i]] = id[i];
        }
}

template <typename TW>
__device__ __forceinline__ void put_lower(int32_t j, int32_t e, const int32_t *__restrict__ u,
                                          const TW *__restrict__ w, int32_t *col, TW *val, int32_t *eid) {
    col[j] = u[e];
    val[j] = w[e];
    eid[j] = e;
}

// Long lower parts: up to kLdsSeg ids (from tmp, or from the row's own eid
// entries) are bitonic-sorted in LDS (padded to a power of two with
// INT32_MAX); longer ones are ranked from global memory (from a copy in tmp).
template <typename TW, bool IDS_IN_TMP>
__global__ __launch_bounds__(256) void k_rank_long(const int32_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ cnt_lo, int32_t *tmp,
                                                   const int32_t *__restrict__ u,
                                                   const TW *__restrict__ w, int32_t *col, TW *val, int32_t *eid,
                                                   const int32_t *__restrict__ long_rows,
                                                   const int32_t *__restrict__ long_cnt) {
    __shared__ int32_t seg[kLdsSeg];
    const int32_t cnt = *long_cnt;
    for (int32_t r = blockIdx.x; r < cnt; r += gridDim.x) {
        const int32_t row = long_rows[r];
        const int32_t len = cnt_lo[row];
        const int32_t base = rowptr[row];
        if (len <= kLdsSeg) {
            int32_t pw = 1;
            while (pw < len) pw <<= 1;
            const int32_t *ids = IDS_IN_TMP ? tmp : eid;
            for (int32_t i = threadIdx.x; i < pw; i += blockDim.x) seg[i] = i < len ? ids[base + i] : INT32_MAX;
            __syncthreads();
            for (int32_t kk = 2; kk <= pw; kk <<= 1) {
                for (int32_t jj = kk >> 1; jj > 0; jj >>= 1) {
                    for (int32_t i = threadIdx.x; i < pw; i += blockDim.x) {
                        const int32_t ixj = i ^ jj;
                        if (ixj > i) {
                            const int32_t a = seg[i], b = seg[ixj];
                            const bool ascending = (i & kk) == 0;
                            if ((a > b) == ascending) {
                                seg[i] = b;
                                seg[ixj] = a;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            for (int32_t i = threadIdx.x; i < len; i += blockDim.x) put_lower(base + i, seg[i], u, w, col, val, eid);
        } else {
            if (!IDS_IN_TMP) {
                // ranked from a copy: the entries are rewritten in place
                for (int32_t i = threadIdx.x; i < len; i += blockDim.x) tmp[base + i] = eid[base + i];
                __syncthreads();
            }
            for (int32_t i = threadIdx.x; i < len; i += blockDim.x) {
                const int32_t mine = tmp[base + i];
                int32_t rank = 0;
                for (int32_t j = 0; j < len; ++j) rank += (tmp[base + j] < mine) ? 1 : 0;
                put_lower(base + rank, mine, u, w, col, val, eid);
            }
        }
        __syncthreads();
    }
}

// d + a[0] + a[1] + ... + a[n-1], added left to right in FP64, with 8 loads
// in flight before the 8 dependent adds (the same additions as the plain loop).
template <typename T>
__device__ __forceinline__ double seq_sum(double d, const T *__restrict__ a, int32_t n) {
    int32_t i = 0;
    for (; i + 8 <= n; i += 8) {
        double t[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) t[q] = (double)a[i + q];
#pragma unroll
        for (int q = 0; q < 8; ++q) d = d + t[q];
    }
    for (; i < n; ++i) d = d + (double)a[i];
    return d;
}

template <typename TW>
__global__ void k_degree(int64_t n, const int32_t *__restrict__ rowptr, const TW *__restrict__ val, TW *deg,
                         int32_t *long_rows, int32_t *long_cnt) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int32_t j0 = rowptr[p], j1 = rowptr[p + 1];
    if (j1 - j0 > kDegLong) {
        long_rows[atomicAdd(long_cnt, 1)] = (int32_t)p;
        return;
    }
    deg[p] = (TW)seq_sum(0.0, val + j0, j1 - j0);
}

// Hub rows: a wavefront stages the row's weights in LDS, chunk by chunk
// (coalesced), and its first lane adds them in column order -- the same sum
// as k_degree's.  One wavefront per row, four rows per workgroup.
template <typename TW>
__global__ __launch_bounds__(256) void k_degree_long(const int32_t *__restrict__ rowptr, const TW *__restrict__ val,
                                                     TW *deg, const int32_t *__restrict__ long_rows,
                                                     const int32_t *__restrict__ long_cnt) {
    constexpr int kChunk = 1024;
    __shared__ double buf[4][kChunk];
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
    double *b = buf[wv];
    const int32_t cnt = *long_cnt;
    for (int32_t r = blockIdx.x * 4 + wv; r < cnt; r += gridDim.x * 4) {
        const int32_t row = long_rows[r];
        const int32_t j0 = rowptr[row], j1 = rowptr[row + 1];
        double d = 0.0;
        for (int32_t c = j0; c < j1; c += kChunk) {
            const int32_t len = (j1 - c) < kChunk ? (j1 - c) : kChunk;
            // one wavefront runs in program order: the first lane reads what
            // all lanes wrote, and the next chunk is written after it is done
            for (int32_t i = lane; i < len; i += 64) b[i] = (double)val[c + i];
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) d = seq_sum(d, b, len);
            __builtin_amdgcn_wave_barrier();
        }
        if (lane == 0) deg[row] = (TW)d;
    }
}

template <typename TW>
void fill_entries(bool walk, int64_t n, int64_t m, const int32_t *u, const int32_t *v, const TW *w,
                  const uint8_t *mask, const CsrPlan &p, const int32_t *rowptr, int32_t *col, TW *val, int32_t *eid,
                  TW *deg, hipStream_t s) {
    const dim3 gn(grid_for(n, 256)), b(256);
    if (m > 0) {
        if (walk) {
            hipLaunchKernelGGL(k_walk_fill<TW>, gn, b, 0, s, n, m, p.estart, v, w, mask, rowptr, p.cnt_lo, col, val,
                               eid, p.fill);
            SFG_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_walk_fill_long<TW>, dim3(256), b, 0, s, n, m, p.estart, v, w, mask, rowptr,
                               p.cnt_lo, col, val, eid, p.fill, p.walk_rows, p.walk_cnt);
            SFG_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_rank_short<TW>, gn, b, 0, s, n, rowptr, p.cnt_lo, u, w, col, val, eid, p.tmp,
                               p.long_rows, p.long_cnt);
            SFG_LAUNCH_CHECK();
            hipLaunchKernelGGL((k_rank_long<TW, false>), dim3(512), b, 0, s, rowptr, p.cnt_lo, p.tmp, u, w, col, val,
                               eid, p.long_rows, p.long_cnt);
            SFG_LAUNCH_CHECK();
        } else {
            hipLaunchKernelGGL(k_fill_edges<TW>, dim3(grid_for(m, 256)), b, 0, s, m, u, v, w, mask,
                               mask ? p.incpos : nullptr, p.estart, rowptr, p.cnt_lo, col, val, eid, p.fill, p.tmp);
            SFG_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_rank_short_ids<TW>, gn, b, 0, s, n, rowptr, p.cnt_lo, p.tmp, u, w, col, val, eid,
                               p.long_rows, p.long_cnt);
            SFG_LAUNCH_CHECK();
            hipLaunchKernelGGL((k_rank_long<TW, true>), dim3(512), b, 0, s, rowptr, p.cnt_lo, p.tmp, u, w, col, val,
                               eid, p.long_rows, p.long_cnt);
            SFG_LAUNCH_CHECK();
        }
    }
    hipLaunchKernelGGL(k_degree<TW>, gn, b, 0, s, n, rowptr, val, deg, p.deg_rows, p.deg_cnt);
    SFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_degree_long<TW>, dim3(1024), b, 0, s, rowptr, val, deg, p.deg_rows, p.deg_cnt);
    SFG_LAUNCH_CHECK();
}

// ---- the CSR of a subgraph, taken from the CSR of the whole graph: row p
// keeps, in their stored (ascending column) order, the entries whose edge is
// in the mask -- exactly the rows build_csr makes from the masked edge list --
// and its degree is summed by the same kernels as build_csr's.  Entry-parallel:
// keep flags, their exclusive scan (the new position of every kept entry),
// new row starts = scan at the old row starts, a scatter of the kept entries.
__global__ void k_sub_flag(int64_t nnz, const int32_t *__restrict__ eid, const uint8_t *__restrict__ mask,
                           int32_t *keep) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < nnz) keep[j] = mask[eid[j]] != 0 ? 1 : 0;
}

__global__ void k_sub_rowptr(int64_t n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ pos,
                             int32_t *nrowptr) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p <= n) nrowptr[p] = pos[rowptr[p]];
}

template <typename TW>
__global__ void k_sub_scatter(int64_t nnz, const int32_t *__restrict__ keep, const int32_t *__restrict__ pos,
                              const int32_t *__restrict__ col, const TW *__restrict__ val,
                              const int32_t *__restrict__ eid, int32_t *__restrict__ ncol, TW *__restrict__ nval,
                              int32_t *__restrict__ neid) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nnz || keep[j] == 0) return;
    const int32_t o = pos[j];
    ncol[o] = col[j];
    nval[o] = val[j];
    neid[o] = eid[j];
}

}  // namespace

namespace {

struct SelectPlan {
    int32_t *keep, *pos, *scan, *long_rows, *long_cnt;
};

SelectPlan plan_select_csr(Carver &c, int64_t n, int64_t nnz) {
    SelectPlan p;
    p.keep = c.take<int32_t>(nnz + 1);
    p.pos = c.take<int32_t>(nnz + 1);
    p.scan = c.take<int32_t>(scan_scratch_ints(nnz + 1));
    p.long_rows = c.take<int32_t>(n + 1);
    p.long_cnt = c.take<int32_t>(1);
    return p;
}

template <typename TW>
void select_entries(const sfg_csr *G, const uint8_t *mask, const SelectPlan &p, int32_t *rowptr, int32_t *col,
                    TW *val, int32_t *eid, TW *deg, hipStream_t s) {
    const int64_t n = G->n, nnz = G->nnz;
    const dim3 b(256);
    if (nnz > 0) {
        hipLaunchKernelGGL(k_sub_flag, dim3(grid_for(nnz, 256)), b, 0, s, nnz, G->eid, mask, p.keep);
        SFG_LAUNCH_CHECK();
        exclusive_scan_i32(p.keep, p.pos, nnz, p.scan, s);
    } else {
        fill_i32(p.pos, 1, 0, s);
    }
    hipLaunchKernelGGL(k_sub_rowptr, dim3(grid_for(n + 1, 256)), b, 0, s, n, G->rowptr, p.pos, rowptr);
    SFG_LAUNCH_CHECK();
    if (nnz > 0) {
        hipLaunchKernelGGL(k_sub_scatter<TW>, dim3(grid_for(nnz, 256)), b, 0, s, nnz, p.keep, p.pos, G->col,
                           (const TW *)G->val, G->eid, col, val, eid);
        SFG_LAUNCH_CHECK();
    }
    fill_i32(p.long_cnt, 1, 0, s);
    hipLaunchKernelGGL(k_degree<TW>, dim3(grid_for(n, 256)), b, 0, s, n, rowptr, val, deg, p.long_rows, p.long_cnt);
    SFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_degree_long<TW>, dim3(1024), b, 0, s, rowptr, val, deg, p.long_rows, p.long_cnt);
    SFG_LAUNCH_CHECK();
}

}  // namespace

size_t csr_select_workspace_bytes(int64_t n, int64_t m) {
    Carver c(nullptr);
    plan_select_csr(c, n < 1 ? 1 : n, 2 * (m < 0 ? 0 : m));
    return c.used + 256;
}

void csr_select(const sfg_csr *G, const uint8_t *mask, int32_t *rowptr, int32_t *col, void *val, int32_t *eid,
                void *deg, void *ws, size_t ws_bytes, hipStream_t s) {
    SFG_REQUIRE(G && G->n >= 1 && G->nnz >= 0, SFG_EINVAL, "csr_select: need a graph with n >= 1");
    SFG_REQUIRE(G->nnz % 2 == 0 && G->nnz < (int64_t(1) << 31) - 1, SFG_EINVAL,
                "csr_select: nnz must be even (two entries per edge) and < 2^31-1");
    SFG_REQUIRE(G->vt == SFG_F64 || G->vt == SFG_F32, SFG_EINVAL, "csr_select: weights must be F64 or F32");
    SFG_REQUIRE(G->rowptr && G->deg && (G->nnz == 0 || (G->col && G->val && G->eid)), SFG_EINVAL,
                "csr_select: the graph CSR needs rowptr, col, val, eid and deg");
    SFG_REQUIRE(rowptr && deg && (G->nnz == 0 || (mask && col && val && eid)), SFG_EINVAL,
                "csr_select: null pointer");
    SFG_REQUIRE(ws_bytes >= csr_select_workspace_bytes(G->n, G->nnz / 2), SFG_EWORKSPACE,
                "csr_select: workspace too small");
    Carver c(ws);
    const SelectPlan p = plan_select_csr(c, G->n, G->nnz);
    if (G->vt == SFG_F64)
        select_entries<double>(G, mask, p, rowptr, col, (double *)val, eid, (double *)deg, s);
    else
        select_entries<float>(G, mask, p, rowptr, col, (float *)val, eid, (float *)deg, s);
}

namespace {

__global__ void k_row_max(int64_t n, const int32_t *__restrict__ rowptr, int32_t *out) {
    __shared__ int32_t part[4];
    int32_t mx = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t len = rowptr[i + 1] - rowptr[i];
        mx = len > mx ? len : mx;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const int32_t o = __shfl_down(mx, off, 64);
        mx = o > mx ? o : mx;
    }
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int w = 0; w < 4; ++w) t = part[w] > t ? part[w] : t;
        if (t) atomicMax(out, t);
    }
}

}  // namespace

// *out = the longest row of H (out is cleared first; one atomic per workgroup
// of a bounded grid).
void max_row_length(const sfg_csr *H, int32_t *out, hipStream_t s) {
    fill_i32(out, 1, 0, s);
    hipLaunchKernelGGL(k_row_max, dim3(std::min<uint32_t>(grid_for(H->n, 256), 1024u)), dim3(256), 0, s, H->n,
                       H->rowptr, out);
    SFG_LAUNCH_CHECK();
}

size_t csr_workspace_bytes(int64_t n, int64_t m) {
    Carver c(nullptr);
    plan_csr(c, n, m);
    return c.used + 256;
}

void build_csr(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
               const uint8_t *mask, int32_t *rowptr, int32_t *col, void *val, int32_t *eid, void *deg, void *ws,
               size_t ws_bytes, hipStream_t s) {
    SFG_REQUIRE(n >= 1 && m >= 0, SFG_EINVAL, "laplacian_csr: need n >= 1 and m >= 0");
    SFG_REQUIRE(2 * m < (int64_t(1) << 31), SFG_EUNSUPPORTED, "laplacian_csr: 2*m must be < 2^31");
    SFG_REQUIRE(n < (int64_t(1) << 31) - 1, SFG_EUNSUPPORTED, "laplacian_csr: n must be < 2^31-1");
    SFG_REQUIRE(wt == SFG_F64 || wt == SFG_F32, SFG_EINVAL, "laplacian_csr: weights must be F64 or F32");
    SFG_REQUIRE(ws_bytes >= csr_workspace_bytes(n, m), SFG_EWORKSPACE, "laplacian_csr: workspace too small");
    SFG_REQUIRE(rowptr && deg && (m == 0 || (u && v && w && col && val && eid)), SFG_EINVAL,
                "laplacian_csr: null pointer");
    Carver c(ws);
    CsrPlan p = plan_csr(c, n, m);
    const dim3 gn(grid_for(n, 256)), b(256);
    fill_i32(p.zeroed, p.zeroed_len, 0, s);
    hipLaunchKernelGGL(k_estart, dim3(grid_for((m + kEdgesPerThread) / kEdgesPerThread, 256)), b, 0, s, n, m, u,
                       p.estart);
    SFG_LAUNCH_CHECK();
    const bool walk = m <= kWalkDensity * n;
    if (walk) {
        hipLaunchKernelGGL(k_walk_count, gn, b, 0, s, n, m, p.estart, v, mask, p.up, p.cnt_lo, p.walk_rows,
                           p.walk_cnt);
        SFG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_walk_count_long, dim3(256), b, 0, s, n, m, p.estart, v, mask, p.up, p.cnt_lo,
                           p.walk_rows, p.walk_cnt);
        SFG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_row_total, gn, b, 0, s, n, p.up, p.cnt_lo, p.tot);
        SFG_LAUNCH_CHECK();
    } else {
        const dim3 gm(grid_for(m, 256));
        if (mask) {
            hipLaunchKernelGGL(k_inc_count, gm, b, 0, s, m, v, mask, p.inc, p.cnt_lo);
            SFG_LAUNCH_CHECK();
            exclusive_scan_i32(p.inc, p.incpos, m, p.scan, s);
        } else {
            hipLaunchKernelGGL(k_count_lo, gm, b, 0, s, m, v, p.cnt_lo);
            SFG_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(k_row_total_edges, gn, b, 0, s, n, p.estart, mask ? p.incpos : nullptr, p.cnt_lo, p.tot);
        SFG_LAUNCH_CHECK();
    }
    exclusive_scan_i32(p.tot, rowptr, n, p.scan, s);
    if (wt == SFG_F64)
        fill_entries<double>(walk, n, m, u, v, (const double *)w, mask, p, rowptr, col, (double *)val, eid,
                             (double *)deg, s);
    else
        fill_entries<float>(walk, n, m, u, v, (const float *)w, mask, p, rowptr, col, (float *)val, eid,
                            (float *)deg, s);
}

}  // namespace sfg

extern "C" sfg_status sfg_csr_select(const sfg_csr *G, const uint8_t *mask, int32_t *rowptr, int32_t *col,
                                     void *val, int32_t *eid, void *deg, int64_t *nnz_out, void *ws,
                                     size_t ws_bytes, void *stream) {
    return sfg::guard([&] {
        hipStream_t s = sfg::as_stream(stream);
        sfg::csr_select(G, mask, rowptr, col, val, eid, deg, ws, ws_bytes, s);
        if (nnz_out) {
            int32_t nnz = 0;
            SFG_HIP(hipMemcpyAsync(&nnz, rowptr + G->n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            SFG_HIP(hipStreamSynchronize(s));
            *nnz_out = nnz;
        }
    });
}

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
