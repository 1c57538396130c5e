// Maximum-weight spanning forest on the GPU (the MST the paper uses in place
// of a low-stretch tree, Sec. 3.4).  Edges are totally ordered by (weight
// descending, edge id ascending), so the forest is unique and equals the one
// Kruskal's rule picks in that order.
//
// Boruvka rounds over the edge list:
//   1. every component finds its best outgoing edge: an integer atomicMax of
//      the weight's bit pattern (positive IEEE values order like their bits),
//      then an atomicMin of the edge id among the edges that reach it;
//   2. each component hooks onto the component across its best edge; a pair
//      that chose the same edge is rooted at the smaller id (longer cycles
//      cannot occur under a total order);
//   3. pointer jumping flattens the hooks; nodes take their new roots.
// Rounds repeat until no component has an outgoing edge.  Only integer
// atomics are used, so the result does not depend on scheduling.
#include "common.hpp"

namespace sfg {

namespace {

constexpr int32_t kNone = 0x7fffffff;

__global__ void k_mst_init(int64_t n, int32_t *comp, uint64_t *best_w, int32_t *best_e) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    comp[p] = (int32_t)p;
    best_w[p] = 0;
    best_e[p] = kNone;
}

template <typename TW>
__device__ __forceinline__ uint64_t wkey(TW w) {
    const double d = (double)w;
    uint64_t k;
    __builtin_memcpy(&k, &d, sizeof(k));
    return k;
}

template <typename TW>
__global__ void k_mst_best_w(int64_t m, const int32_t *__restrict__ u, const int32_t *__restrict__ v,
                             const TW *__restrict__ w, const uint8_t *__restrict__ allowed,
                             const int32_t *__restrict__ comp, uint64_t *best_w, int32_t *live) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    if (allowed && !allowed[e]) return;
    const int32_t a = comp[u[e]], b = comp[v[e]];
    if (a == b) return;
    if (*live == 0) *live = 1;
    const uint64_t k = wkey(w[e]);
    // read first: on hub components most edges lose, and skipping their
    // atomics removes the contention (the maximum is still exact)
    if (k > best_w[a]) atomicMax((unsigned long long *)&best_w[a], (unsigned long long)k);
    if (k > best_w[b]) atomicMax((unsigned long long *)&best_w[b], (unsigned long long)k);
}

template <typename TW>
__global__ void k_mst_best_e(int64_t m, const int32_t *__restrict__ u, const int32_t *__restrict__ v,
                             const TW *__restrict__ w, const uint8_t *__restrict__ allowed,
                             const int32_t *__restrict__ comp, const uint64_t *__restrict__ best_w,
                             int32_t *best_e) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    if (allowed && !allowed[e]) return;
    const int32_t a = comp[u[e]], b = comp[v[e]];
    if (a == b) return;
    const uint64_t k = wkey(w[e]);
    if (k == best_w[a] && (int32_t)e < best_e[a]) atomicMin(&best_e[a], (int32_t)e);
    if (k == best_w[b] && (int32_t)e < best_e[b]) atomicMin(&best_e[b], (int32_t)e);
}

// Roots hook across their best edge and mark it as a tree edge.
__global__ void k_mst_hook(int64_t n, const int32_t *__restrict__ u, const int32_t *__restrict__ v,
                           const int32_t *__restrict__ comp, const int32_t *__restrict__ best_e, int32_t *parent,
                           uint8_t *in_tree) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    if (comp[c] != c) return;                  // not a root
    const int32_t e = best_e[c];
    if (e == kNone) {
        parent[c] = (int32_t)c;
        return;
    }
    const int32_t a = comp[u[e]], b = comp[v[e]];
    const int32_t d = (a == c) ? b : a;
    in_tree[e] = 1;
    // a mutual pair (both chose e) is rooted at its smaller id
    parent[c] = (best_e[d] == e && c < d) ? (int32_t)c : d;
}

__global__ void k_mst_jump(int64_t n, const int32_t *__restrict__ comp, int32_t *parent, int32_t *changed) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n || comp[c] != c) return;
    const int32_t a = parent[c];
    const int32_t b = parent[a];
    if (a != b) {
        parent[c] = b;
        *changed = 1;
    }
}

__global__ void k_mst_relabel(int64_t n, int32_t *comp, const int32_t *__restrict__ parent, uint64_t *best_w,
                              int32_t *best_e) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    comp[p] = parent[comp[p]];
    best_w[p] = 0;
    best_e[p] = kNone;
}

__global__ void k_mst_roots(int64_t n, const int32_t *__restrict__ comp, int32_t *cnt) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n && comp[p] == p) atomicAdd(cnt, 1);
}

int32_t read_flag(const int32_t *p, hipStream_t s) {
    int32_t h = 0;
    SFG_HIP(hipMemcpyAsync(&h, p, sizeof(h), hipMemcpyDeviceToHost, s));
    SFG_HIP(hipStreamSynchronize(s));
    return h;
}

}  // namespace

int64_t spanning_tree_gpu(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
                          const uint8_t *allowed, uint8_t *in_tree, DevArena &A, hipStream_t s) {
    SFG_REQUIRE(wt == SFG_F64 || wt == SFG_F32, SFG_EINVAL, "spanning_tree: weights must be F64 or F32");
    int32_t *comp = A.alloc<int32_t>(n + 1);
    int32_t *parent = A.alloc<int32_t>(n + 1);
    int32_t *best_e = A.alloc<int32_t>(n + 1);
    uint64_t *best_w = A.alloc<uint64_t>(n + 1);
    int32_t *flags = A.alloc<int32_t>(4);
    const dim3 gn(grid_for(n, 256)), gm(grid_for(m, 256)), b(256);
    hipLaunchKernelGGL(k_mst_init, gn, b, 0, s, n, comp, best_w, best_e);
    SFG_LAUNCH_CHECK();
    if (m > 0) fill_u8(in_tree, m, 0, s);
    for (int round = 0; m > 0; ++round) {
        SFG_REQUIRE(round < 64, SFG_EHIP, "spanning_tree: too many rounds");
        fill_i32(flags, 1, 0, s);
        if (wt == SFG_F64) {
            hipLaunchKernelGGL(k_mst_best_w<double>, gm, b, 0, s, m, u, v, (const double *)w, allowed, comp, best_w,
                               flags);
            SFG_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_mst_best_e<double>, gm, b, 0, s, m, u, v, (const double *)w, allowed, comp, best_w,
                               best_e);
        } else {
            hipLaunchKernelGGL(k_mst_best_w<float>, gm, b, 0, s, m, u, v, (const float *)w, allowed, comp, best_w,
                               flags);
            SFG_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_mst_best_e<float>, gm, b, 0, s, m, u, v, (const float *)w, allowed, comp, best_w,
                               best_e);
        }
        SFG_LAUNCH_CHECK();
        // no component with an outgoing edge: done.  Read every other round
        // only (each read is a host sync): a round without outgoing edges hooks
        // nothing, and its jumps and relabelling change nothing, so at most one
        // idle round runs past the end
        if (round % 2 == 1 && read_flag(flags, s) == 0) break;
        hipLaunchKernelGGL(k_mst_hook, gn, b, 0, s, n, u, v, comp, best_e, parent, in_tree);
        SFG_LAUNCH_CHECK();
        for (int it = 0;; it += 4) {   // four jumps per check of the flag (one host sync); extra jumps are no-ops
            SFG_REQUIRE(it < 64, SFG_EHIP, "spanning_tree: pointer jumping did not converge");
            fill_i32(flags + 1, 1, 0, s);
            for (int j = 0; j < 4; ++j) {
                hipLaunchKernelGGL(k_mst_jump, gn, b, 0, s, n, comp, parent, flags + 1);
                SFG_LAUNCH_CHECK();
            }
            if (read_flag(flags + 1, s) == 0) break;
        }
        hipLaunchKernelGGL(k_mst_relabel, gn, b, 0, s, n, comp, parent, best_w, best_e);
        SFG_LAUNCH_CHECK();
    }
    fill_i32(flags + 2, 1, 0, s);
    hipLaunchKernelGGL(k_mst_roots, gn, b, 0, s, n, comp, flags + 2);
    SFG_LAUNCH_CHECK();
    return read_flag(flags + 2, s);
}

}  // namespace sfg
