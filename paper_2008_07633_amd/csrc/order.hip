// Node order for the smoothing sweeps.
//
// A Jacobi sweep (Sec. 3.1) reads, for every row, the rows of its neighbours.
// Where the input numbering scatters neighbours over the whole block (points
// of a k-NN graph in random order, say), almost every such read fetches a
// fresh cache line for one row, and a sweep moves several times the bytes it
// needs.  Numbering the nodes in the preorder of the spanning tree puts a
// node next to its first child and every subtree in a contiguous range, so
// most tree neighbours, and most near neighbours of a spatial graph, land in
// nearby rows.
//
// The relabelling changes no arithmetic: the scoring graph is copied row by
// row into the new numbering with every row's entries in their original order
// (so each row's sum is formed exactly as before), the start block is gathered
// row by row, and the edge endpoints are mapped, so sweeps and scores come out
// bit-identical to the ones in the input numbering.  A relabelled graph is
// internal: its columns are no longer ascending within a row.
#include "common.hpp"

namespace sfg {

namespace {

constexpr int kB = 256;

// Entries of H whose column is more than `window` rows from their row;
// one atomic add per workgroup onto *count (zeroed by the caller).
__global__ void k_far_count(int64_t n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                            int64_t window, unsigned long long *count) {
    __shared__ unsigned long long part[kB / 64];
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
        const int32_t a = rowptr[i], e = rowptr[i + 1];
        for (int32_t j = a; j < e; ++j) {
            const int64_t d = (int64_t)col[j] - i;
            c += (d > window || d < -window) ? 1u : 0u;
        }
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kB / 64; ++w) t += part[w];
        if (t) atomicAdd(count, t);
    }
}

__global__ void k_inverse_perm(int64_t n, const int32_t *__restrict__ order, int32_t *__restrict__ inv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) inv[order[i]] = (int32_t)i;
}

__global__ void k_row_len(int64_t n, const int32_t *__restrict__ order, const int32_t *__restrict__ rowptr,
                          int32_t *__restrict__ len) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t p = order[i];
    len[i] = rowptr[p + 1] - rowptr[p];
}

// New row i is old row order[i]: entries in their stored order, columns
// through inv, values and edge ids carried along.  A thread per entry (rows
// of power-law graphs run to thousands of entries): its new row is found by
// binary search in the new row pointers.
template <typename T>
__global__ void k_entry_copy(int64_t n, int64_t nnz, const int32_t *__restrict__ order,
                             const int32_t *__restrict__ inv, const int32_t *__restrict__ rowptr,
                             const int32_t *__restrict__ col, const T *__restrict__ val,
                             const int32_t *__restrict__ eid, const int32_t *__restrict__ nrowptr,
                             int32_t *__restrict__ ncol, T *__restrict__ nval, int32_t *__restrict__ neid) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nnz || j >= nrowptr[n]) return;
    int64_t lo = 0, hi = n - 1;     // the last row i with nrowptr[i] <= j
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (nrowptr[mid] <= j) lo = mid;
        else hi = mid - 1;
    }
    const int32_t src = rowptr[order[lo]] + (int32_t)(j - nrowptr[lo]);
    ncol[j] = inv[col[src]];
    nval[j] = val[src];
    if (neid) neid[j] = eid[src];
}

template <typename T>
__global__ void k_deg_copy(int64_t n, const int32_t *__restrict__ order, const T *__restrict__ deg,
                           T *__restrict__ ndeg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ndeg[i] = deg[order[i]];
}

__global__ void k_map_ends(int64_t m, const int32_t *__restrict__ inv, const int32_t *__restrict__ u,
                           const int32_t *__restrict__ v, int32_t *__restrict__ nu, int32_t *__restrict__ nv) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    nu[e] = inv[u[e]];
    nv[e] = inv[v[e]];
}

// dst row i = src row order[i], k doubles per row; a thread per element so
// that consecutive threads read consecutive doubles of a row.
__global__ void k_gather_block(int64_t n, int32_t k, const int32_t *__restrict__ order,
                               const double *__restrict__ src, double *__restrict__ dst) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int64_t i = t / k;
    const int32_t c = (int32_t)(t - i * k);
    dst[t] = src[(int64_t)order[i] * k + c];
}

}  // namespace

void far_entries(const sfg_csr *H, int64_t window, unsigned long long *count, hipStream_t s) {
    if (H->n <= 0) return;
    const uint32_t g = std::min<uint32_t>(grid_for(H->n, kB), 1024u);
    hipLaunchKernelGGL(k_far_count, dim3(g), dim3(kB), 0, s, H->n, H->rowptr, H->col, window, count);
    SFG_LAUNCH_CHECK();
}

void inverse_permutation(int64_t n, const int32_t *order, int32_t *inv, hipStream_t s) {
    hipLaunchKernelGGL(k_inverse_perm, dim3(grid_for(n, kB)), dim3(kB), 0, s, n, order, inv);
    SFG_LAUNCH_CHECK();
}

sfg_csr relabel_csr(const sfg_csr *H, const int32_t *order, const int32_t *inv, DevArena &A, hipStream_t s) {
    const int64_t n = H->n, nnz = H->nnz;
    const size_t vb = dtype_size(H->vt);
    int32_t *len = A.alloc<int32_t>(n + 1);
    int32_t *rowptr = A.alloc<int32_t>(n + 1);
    int32_t *col = A.alloc<int32_t>(nnz + 1);
    int32_t *eid = H->eid ? A.alloc<int32_t>(nnz + 1) : nullptr;
    void *val = A.raw((nnz + 1) * vb);
    void *deg = A.raw((n + 1) * vb);
    int32_t *scr = A.alloc<int32_t>(scan_scratch_ints(n + 1));
    const dim3 g(grid_for(n, kB)), b(kB);
    hipLaunchKernelGGL(k_row_len, g, b, 0, s, n, order, H->rowptr, len);
    SFG_LAUNCH_CHECK();
    exclusive_scan_i32(len, rowptr, n, scr, s);
    const dim3 ge(grid_for(nnz > 0 ? nnz : 1, kB));
    if (H->vt == SFG_F64) {
        if (nnz > 0)
            hipLaunchKernelGGL(k_entry_copy<double>, ge, b, 0, s, n, nnz, order, inv, H->rowptr, H->col,
                               (const double *)H->val, H->eid, rowptr, col, (double *)val, eid);
        hipLaunchKernelGGL(k_deg_copy<double>, g, b, 0, s, n, order, (const double *)H->deg, (double *)deg);
    } else {
        if (nnz > 0)
            hipLaunchKernelGGL(k_entry_copy<float>, ge, b, 0, s, n, nnz, order, inv, H->rowptr, H->col,
                               (const float *)H->val, H->eid, rowptr, col, (float *)val, eid);
        hipLaunchKernelGGL(k_deg_copy<float>, g, b, 0, s, n, order, (const float *)H->deg, (float *)deg);
    }
    SFG_LAUNCH_CHECK();
    return sfg_csr{n, nnz, rowptr, col, val, eid, deg, H->vt};
}

void map_endpoints(int64_t m, const int32_t *inv, const int32_t *u, const int32_t *v, int32_t *nu, int32_t *nv,
                   hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_map_ends, dim3(grid_for(m, kB)), dim3(kB), 0, s, m, inv, u, v, nu, nv);
    SFG_LAUNCH_CHECK();
}

void gather_block(int64_t n, int32_t k, const int32_t *order, const double *src, double *dst, hipStream_t s) {
    const int64_t t = n * (int64_t)k;
    if (t <= 0) return;
    hipLaunchKernelGGL(k_gather_block, dim3(grid_for(t, kB)), dim3(kB), 0, s, n, k, order, src, dst);
    SFG_LAUNCH_CHECK();
}

}  // namespace sfg
