// Spanning-tree layout and exact tree-Laplacian solves.
//
// The condition-number estimate behind sigma-driven stopping (Eq. 2, and the
// sigma that Alg. 1 takes) needs solves with the sparsifier Laplacian L_P;
// they are done by conjugate gradients preconditioned with the spanning tree
// T inside P, and a tree Laplacian system is solved exactly in O(n) work.
//
// Layout (tree_order): root node 0; the Euler walk that crosses every tree
// edge once down and once up, taking at each node the neighbours in
// ascending id order starting after the one it came from.  On the device:
// tree CSR -> reverse arc by binary search -> successor of every arc -> list
// ranking by pointer jumping (log2(2n) rounds over packed (next, rank)
// words) -> walk position of every arc -> down arcs scanned in walk order
// give the preorder.  Per preorder position: node, parent position, subtree
// size, parent-edge weight and the walk steps that enter and leave it.
//
// Solve (tree_solve), x = L_T^+ b per column, no atomics, deterministic:
//   b is centred and gathered into preorder; the net demand below each edge
//   is a difference of two inclusive prefix sums (a subtree is a contiguous
//   preorder range); each edge's potential drop demand / w is written at its
//   down step and its negation at its up step of a walk-length array, whose
//   inclusive prefix sum at a node's down step is the node's potential
//   relative to the root (closed excursions cancel); the result is centred.
#include "common.hpp"

namespace sfg {

size_t csr_workspace_bytes(int64_t n, int64_t m);
void build_csr(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
               const uint8_t *mask, int32_t *rowptr, int32_t *col, void *val, int32_t *eid, void *deg, void *ws,
               size_t ws_bytes, hipStream_t s);

namespace {

constexpr int kB = 256;
constexpr uint32_t kNil = 0xFFFFFFFFu;

// Grid-stride over a bounded grid, one atomic per workgroup: a single
// counter takes same-address atomics one at a time, so one per wave over
// millions of edges would cost milliseconds.
constexpr uint32_t kMaskBlocks = 1024;

__global__ void k_mask_eq(int64_t m, const uint8_t *__restrict__ keep, uint8_t want, uint8_t *__restrict__ out,
                          int32_t *__restrict__ count) {
    __shared__ int32_t part[kB / kWave];
    int32_t c = 0;
    for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x; e0 < m; e0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = e0 + threadIdx.x;
        const bool in = e < m && keep[e] == want;
        if (e < m) out[e] = in ? 1 : 0;
        c += (int32_t)__popcll(__ballot(in));
    }
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int w = 0; w < kB / kWave; ++w) t += part[w];
        if (t) atomicAdd(count, t);
    }
}

__device__ __forceinline__ int32_t upper_row(const int32_t *__restrict__ rowptr, int64_t n, int32_t a) {
    // the row p with rowptr[p] <= a < rowptr[p + 1]
    int64_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (rowptr[mid] <= a) lo = mid; else hi = mid;
    }
    return (int32_t)lo;
}

// Successor of every arc a = (p -> q) in the walk: the arc after (q -> p) in
// row q, cyclically.  The arc entering the root last ends the list.  Packed
// word: low 32 bits next arc (kNil at the end), high 32 bits distance.
__global__ void k_walk_init(int64_t n, int64_t A, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                            int32_t *__restrict__ rev, int32_t *__restrict__ src, uint64_t *__restrict__ link) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= A) return;
    const int32_t p = upper_row(rowptr, n, (int32_t)a);
    const int32_t q = col[a];
    int32_t lo = rowptr[q], hi = rowptr[q + 1];
    while (lo < hi) {   // p in row q (columns ascending)
        const int32_t mid = (lo + hi) >> 1;
        if (col[mid] < p) lo = mid + 1; else hi = mid;
    }
    // p is in row q for a symmetric CSR; the clamp only keeps a malformed
    // input's indexes inside row q
    const int32_t r = lo < rowptr[q + 1] ? lo : rowptr[q];
    rev[a] = r;
    src[a] = p;
    int32_t nx = r + 1;
    if (nx == rowptr[q + 1]) nx = rowptr[q];
    const bool last = (q == 0) && (nx == rowptr[0]);
    link[a] = last ? (uint64_t)kNil : ((uint64_t)1 << 32) | (uint32_t)nx;
}

__global__ void k_walk_jump(int64_t A, const uint64_t *__restrict__ in, uint64_t *__restrict__ out) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= A) return;
    const uint64_t x = in[a];
    const uint32_t nx = (uint32_t)x;
    if (nx == kNil) {
        out[a] = x;
        return;
    }
    const uint64_t y = in[nx];
    out[a] = (((x >> 32) + (y >> 32)) << 32) | (uint32_t)y;
}

// walk position of every arc, and a down flag at each walk position
__global__ void k_walk_pos(int64_t A, const uint64_t *__restrict__ link, const int32_t *__restrict__ rev,
                           int32_t *__restrict__ pos, int32_t *__restrict__ down_at) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= A) return;
    const int32_t pa = (int32_t)(A - 1 - (int64_t)(link[a] >> 32));
    const int32_t pr = (int32_t)(A - 1 - (int64_t)(link[rev[a]] >> 32));
    pos[a] = pa;
    if (pa >= 0 && pa < A) down_at[pa] = pa < pr ? 1 : 0;
}

__global__ void k_tree_fill(int64_t A, const int32_t *__restrict__ pos, const int32_t *__restrict__ rev,
                            const int32_t *__restrict__ src, const int32_t *__restrict__ col,
                            const double *__restrict__ val, const int32_t *__restrict__ dbefore,
                            int32_t *__restrict__ pre_of, int32_t *__restrict__ order, int32_t *__restrict__ parnode,
                            int32_t *__restrict__ size, double *__restrict__ pw, int32_t *__restrict__ tdown,
                            int32_t *__restrict__ tup, int32_t *__restrict__ entered) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= A) return;
    const int32_t pa = pos[a], pr = pos[rev[a]];
    if (!(pa < pr)) return;   // up arc
    const int32_t q = col[a];
    const int32_t i = 1 + dbefore[pa];
    atomicAdd(&entered[q], 1);
    pre_of[q] = i;
    order[i] = q;
    parnode[i] = src[a];
    size[i] = (pr - pa + 1) >> 1;
    pw[i] = val[a];
    tdown[i] = pa;
    tup[i] = pr;
}

__global__ void k_tree_parent(int64_t n, const int32_t *__restrict__ entered, const int32_t *__restrict__ pre_of,
                              const int32_t *__restrict__ parnode, int32_t *__restrict__ parent,
                              int32_t *__restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // node i is entered exactly once (the root never): otherwise no spanning tree
    if (entered[i] != (i == 0 ? 0 : 1)) atomicOr(bad, 1);
    if (i > 0) {
        const int32_t pn = parnode[i];
        parent[i] = (pn >= 0 && pn < n) ? pre_of[pn] : -1;
    }
}

__global__ void k_tree_root(int64_t n, int32_t *order, int32_t *parent, int32_t *size, double *pw, int32_t *tdown,
                            int32_t *tup, int32_t *pre_of) {
    order[0] = 0;
    parent[0] = -1;
    size[0] = (int32_t)n;
    pw[0] = 0.0;
    tdown[0] = -1;
    tup[0] = -1;
    pre_of[0] = 0;
}

// ------------------------------------------------------------------ FP64 block kernels (rows x k, row-major)
//
// A workgroup is kB threads laid out as G row lanes x k column lanes (G =
// kB / k); thread (g, c) owns column c of kRpt consecutive rows.

constexpr int kRpt = 16;

__device__ __forceinline__ int lanes_g(int k) { return kB / k; }

// Column sums, stage 1: per-workgroup partial sums over a strided set of rows.
__global__ __launch_bounds__(kB) void k_colsum(int64_t rows, int32_t k, const double *__restrict__ x,
                                               double *__restrict__ partial) {
    __shared__ double sh[kB];
    const int G = lanes_g(k);
    const int g = threadIdx.x / k, c = threadIdx.x % k;
    double acc = 0.0;
    if (g < G)
        for (int64_t r = (int64_t)blockIdx.x * G + g; r < rows; r += (int64_t)gridDim.x * G) acc += x[r * k + c];
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < k) {
        double t = 0.0;
        for (int gg = 0; gg < G; ++gg) t += sh[gg * k + threadIdx.x];
        partial[(int64_t)blockIdx.x * k + threadIdx.x] = t;
    }
}

// stage 2: out[c] = scale * sum of the partials, in workgroup order
__global__ void k_colsum_finish(int32_t nb, int32_t k, const double *__restrict__ partial, double scale,
                                double *__restrict__ out) {
    const int c = threadIdx.x;
    if (c >= k) return;
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += partial[(int64_t)b * k + c];
    out[c] = t * scale;
}

// per-column dot products, stage 1 (stage 2 is k_colsum_finish)
__global__ __launch_bounds__(kB) void k_coldot(int64_t rows, int32_t k, const double *__restrict__ x,
                                               const double *__restrict__ y, double *__restrict__ partial) {
    __shared__ double sh[kB];
    const int G = lanes_g(k);
    const int g = threadIdx.x / k, c = threadIdx.x % k;
    double acc = 0.0;
    if (g < G)
        for (int64_t r = (int64_t)blockIdx.x * G + g; r < rows; r += (int64_t)gridDim.x * G)
            acc += x[r * k + c] * y[r * k + c];
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < k) {
        double t = 0.0;
        for (int gg = 0; gg < G; ++gg) t += sh[gg * k + threadIdx.x];
        partial[(int64_t)blockIdx.x * k + threadIdx.x] = t;
    }
}

// k x k Gram block X^T Y, stage 1: thread t owns entries t, t + kB, ... of
// the k*k matrix over one of L = max(1, kB / k^2) row lanes
__global__ __launch_bounds__(kB) void k_gram(int64_t rows, int32_t k, const double *__restrict__ x,
                                             const double *__restrict__ y, double *__restrict__ partial) {
    __shared__ double sh[kB * 4];
    const int P = k * k;
    const int L = P >= kB ? 1 : kB / P;
    const int lane = P >= kB ? 0 : threadIdx.x / P;
    const int e0 = P >= kB ? threadIdx.x : threadIdx.x % P;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (lane < L)
        for (int64_t r = (int64_t)blockIdx.x * L + lane; r < rows; r += (int64_t)gridDim.x * L) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = e0 + q * kB;
                if (e < P && (q == 0 || P >= kB)) acc[q] += x[r * k + e / k] * y[r * k + e % k];
            }
        }
#pragma unroll
    for (int q = 0; q < 4; ++q) sh[q * kB + threadIdx.x] = acc[q];
    __syncthreads();
    for (int e = threadIdx.x; e < P; e += kB) {
        double t = 0.0;
        if (P >= kB) {
            t = sh[(e / kB) * kB + (e % kB)];
        } else {
            for (int l = 0; l < L; ++l) t += sh[l * P + e];
        }
        partial[(int64_t)blockIdx.x * P + e] = t;
    }
}

__global__ void k_gram_finish(int32_t nb, int32_t P, const double *__restrict__ partial, double *__restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P) return;
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += partial[(int64_t)b * P + e];
    out[e] = t;
}

// per-tile column totals of a rows x k block (tile = G * kRpt rows)
__global__ __launch_bounds__(kB) void k_scan_tiles(int64_t rows, int32_t k, const double *__restrict__ x,
                                                   double *__restrict__ tile_sum) {
    __shared__ double sh[kB];
    const int G = lanes_g(k);
    const int g = threadIdx.x / k, c = threadIdx.x % k;
    const int64_t base = (int64_t)blockIdx.x * G * kRpt + (int64_t)g * kRpt;
    double acc = 0.0;
    if (g < G)
        for (int r = 0; r < kRpt; ++r)
            if (base + r < rows) acc += x[(base + r) * k + c];
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < k) {
        double t = 0.0;
        for (int gg = 0; gg < G; ++gg) t += sh[gg * k + threadIdx.x];
        tile_sum[(int64_t)blockIdx.x * k + threadIdx.x] = t;
    }
}

// Exclusive scan of the tile totals in two levels.  k_scan_mid: a workgroup
// takes a group of G * kTpl tiles (lane (g, c): kTpl consecutive tiles of
// column c), replaces each tile total by its exclusive offset inside the
// group and writes the group total.  k_scan_top (one workgroup): exclusive
// offsets of the group totals, and the column totals after them.
constexpr int kTpl = 8;

__device__ __forceinline__ int64_t tiles_per_group(int k) { return (int64_t)lanes_g(k) * kTpl; }

__global__ __launch_bounds__(kB) void k_scan_mid(int64_t tiles, int32_t k, double *__restrict__ tile_sum,
                                                 double *__restrict__ group_sum) {
    __shared__ double sh[kB];
    const int G = lanes_g(k);
    const int g = threadIdx.x / k, c = threadIdx.x % k;
    const int64_t t0 = (int64_t)blockIdx.x * G * kTpl + (int64_t)g * kTpl;
    double v[kTpl];
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < kTpl; ++q) {
        v[q] = (g < G && t0 + q < tiles) ? tile_sum[(t0 + q) * k + c] : 0.0;
        acc += v[q];
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (g >= G) return;
    double off = 0.0;
    for (int gg = 0; gg < g; ++gg) off += sh[gg * k + c];
#pragma unroll
    for (int q = 0; q < kTpl; ++q) {
        if (t0 + q < tiles) tile_sum[(t0 + q) * k + c] = off;
        off += v[q];
    }
    if (g == G - 1) group_sum[(int64_t)blockIdx.x * k + c] = off;
}

__global__ __launch_bounds__(kB) void k_scan_top(int64_t groups, int32_t k, double *__restrict__ group_sum) {
    __shared__ double sh[kB];
    const int G = lanes_g(k);
    const int g = threadIdx.x / k, c = threadIdx.x % k;
    const int64_t chunk = (groups + G - 1) / G;
    const int64_t t0 = (int64_t)g * chunk, t1 = t0 + chunk < groups ? t0 + chunk : groups;
    double acc = 0.0;
    if (g < G)
        for (int64_t t = t0; t < t1; ++t) acc += group_sum[t * k + c];
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (g >= G) return;
    double off = 0.0;
    for (int gg = 0; gg < g; ++gg) off += sh[gg * k + c];
    for (int64_t t = t0; t < t1; ++t) {
        const double x = group_sum[t * k + c];
        group_sum[t * k + c] = off;
        off += x;
    }
    if (g == 0) {   // column totals after the offsets
        double tot = 0.0;
        for (int gg = 0; gg < G; ++gg) tot += sh[gg * k + c];
        group_sum[groups * k + c] = tot;
    }
}

// inclusive prefix sums over rows: tile offset + lane offset + running sum
__global__ __launch_bounds__(kB) void k_scan_apply(int64_t rows, int32_t k, const double *__restrict__ x,
                                                   const double *__restrict__ tile_off,
                                                   const double *__restrict__ group_off, double *__restrict__ y) {
    __shared__ double sh[kB];
    const int G = lanes_g(k);
    const int g = threadIdx.x / k, c = threadIdx.x % k;
    const int64_t base = (int64_t)blockIdx.x * G * kRpt + (int64_t)g * kRpt;
    double v[kRpt];
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < kRpt; ++r) {
        v[r] = (g < G && base + r < rows) ? x[(base + r) * k + c] : 0.0;
        acc += v[r];
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (g >= G) return;
    double run = group_off[((int64_t)blockIdx.x / tiles_per_group(k)) * k + c] + tile_off[(int64_t)blockIdx.x * k + c];
    for (int gg = 0; gg < g; ++gg) run += sh[gg * k + c];
#pragma unroll
    for (int r = 0; r < kRpt; ++r) {
        run += v[r];
        if (base + r < rows) y[(base + r) * k + c] = run;
    }
}

// centred gather into preorder: bp[i] = b[order[i]] - mean
__global__ void k_gather_centre(int64_t n, int32_t k, const int32_t *__restrict__ order,
                                const double *__restrict__ b, const double *__restrict__ mean,
                                double *__restrict__ bp) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int64_t i = t / k;
    const int c = (int)(t - i * k);
    bp[t] = b[(int64_t)order[i] * k + c] - mean[c];
}

// potential drop of every parent edge, written at its down step and negated
// at its up step of the walk-length array
__global__ void k_edge_drop(int64_t n, int32_t k, const int32_t *__restrict__ size, const double *__restrict__ pw,
                            const int32_t *__restrict__ tdown, const int32_t *__restrict__ tup,
                            const double *__restrict__ S, double *__restrict__ walk) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k || t < k) return;   // the root has no parent edge
    const int64_t i = t / k;
    const int c = (int)(t - i * k);
    const double hi = S[(i + size[i] - 1) * k + c];
    const double lo = S[(i - 1) * k + c];
    const double d = (hi - lo) / pw[i];
    walk[(int64_t)tdown[i] * k + c] = d;
    walk[(int64_t)tup[i] * k + c] = -d;
}

// potentials in preorder: xp[i] = prefix of the walk array at i's down step
__global__ void k_potential(int64_t n, int32_t k, const int32_t *__restrict__ tdown, const double *__restrict__ U,
                            double *__restrict__ xp) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int64_t i = t / k;
    const int c = (int)(t - i * k);
    xp[t] = i == 0 ? 0.0 : U[(int64_t)tdown[i] * k + c];
}

// centred scatter back to node order: x[order[i]] = xp[i] - mean
__global__ void k_scatter_centre(int64_t n, int32_t k, const int32_t *__restrict__ order,
                                 const double *__restrict__ xp, const double *__restrict__ mean,
                                 double *__restrict__ x) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int64_t i = t / k;
    const int c = (int)(t - i * k);
    x[(int64_t)order[i] * k + c] = xp[t] - mean[c];
}

// Preconditioner form (blocks already in preorder): the edge drops use the
// column means from the scan totals instead of a centred copy of b.
__global__ void k_edge_drop_pre(int64_t n, int32_t k, const int32_t *__restrict__ size, const double *__restrict__ pw,
                                const int32_t *__restrict__ tdown, const int32_t *__restrict__ tup,
                                const double *__restrict__ S, const double *__restrict__ totals,
                                double *__restrict__ walk) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k || t < k) return;
    const int64_t i = t / k;
    const int c = (int)(t - i * k);
    const int32_t sz = size[i];
    const double mean = totals[c] / (double)n;
    const double f = (S[(i + sz - 1) * k + c] - S[(i - 1) * k + c]) - (double)sz * mean;
    const double d = f / pw[i];
    walk[(int64_t)tdown[i] * k + c] = d;
    walk[(int64_t)tup[i] * k + c] = -d;
}

// z[i] = prefix of the walk at i's down step (0 at the root), and per-column
// partial sums of r . z.  Row-lane layout: workgroup of G x k threads,
// thread (g, c) walks rows blockIdx * G + g + j * gridDim * G.
__global__ __launch_bounds__(kB) void k_potential_dot(int64_t n, int32_t k, const int32_t *__restrict__ tdown,
                                                      const double *__restrict__ U, const double *__restrict__ r,
                                                      double *__restrict__ z, double *__restrict__ partial) {
    __shared__ double sh[kB];
    const int G = lanes_g(k);
    const int g = threadIdx.x / k, c = threadIdx.x % k;
    double acc = 0.0;
    if (g < G)
        for (int64_t i = (int64_t)blockIdx.x * G + g; i < n; i += (int64_t)gridDim.x * G) {
            const double zi = i == 0 ? 0.0 : U[(int64_t)tdown[i] * k + c];
            z[i * k + c] = zi;
            acc += r[i * k + c] * zi;
        }
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < k) {
        double t = 0.0;
        for (int gg = 0; gg < G; ++gg) t += sh[gg * k + threadIdx.x];
        partial[(int64_t)blockIdx.x * k + threadIdx.x] = t;
    }
}

// out[c] = sum of nb partials of column c: one workgroup of 1024 threads,
// lane (g, c) adds partials g, g + G, ... into four accumulators (loads in
// flight), then a fixed pairwise tree over the lanes
constexpr int kFinish = 1024;

__global__ __launch_bounds__(kFinish) void k_partials_finish(int32_t nb, int32_t k, const double *__restrict__ partial,
                                                             double *__restrict__ out) {
    __shared__ double sh[kFinish];
    const int G = kFinish / k;
    const int g = threadIdx.x / k, c = threadIdx.x % k;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (g < G) {
        int b = g;
        for (; b + 3 * G < nb; b += 4 * G) {
            a0 += partial[(int64_t)b * k + c];
            a1 += partial[(int64_t)(b + G) * k + c];
            a2 += partial[(int64_t)(b + 2 * G) * k + c];
            a3 += partial[(int64_t)(b + 3 * G) * k + c];
        }
        for (; b < nb; b += G) a0 += partial[(int64_t)b * k + c];
    }
    sh[threadIdx.x] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    for (int st = 1; st < G; st <<= 1) {
        if (g < G && (g % (2 * st)) == 0 && g + st < G) sh[g * k + c] += sh[(g + st) * k + c];
        __syncthreads();
    }
    if ((int)threadIdx.x < k) out[threadIdx.x] = sh[threadIdx.x];
}

constexpr int kSumBlocks = 512;

int64_t scan_tiles(int64_t rows, int32_t k) {
    const int64_t tr = (int64_t)(kB / k) * kRpt;
    return (rows + tr - 1) / tr;
}

}  // namespace

// ------------------------------------------------------------------ block helpers shared by the estimate

size_t colsum_scratch_doubles(int32_t k) { return (size_t)kSumBlocks * k + 64; }

// out[c] = scale * sum_r x[r][c]; deterministic (fixed partition and order)
void block_colsum(int64_t rows, int32_t k, const double *x, double scale, double *out, double *scratch,
                  hipStream_t s) {
    int64_t nb = (rows * k + kB - 1) / kB;
    nb = nb < 1 ? 1 : (nb > kSumBlocks ? kSumBlocks : nb);
    hipLaunchKernelGGL(k_colsum, dim3((uint32_t)nb), dim3(kB), 0, s, rows, k, x, scratch);
    SFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_colsum_finish, dim3(1), dim3(64), 0, s, (int32_t)nb, k, scratch, scale, out);
    SFG_LAUNCH_CHECK();
}

// out[c] = sum_r x[r][c] * y[r][c]; deterministic
void block_dot(int64_t rows, int32_t k, const double *x, const double *y, double *out, double *scratch,
               hipStream_t s) {
    int64_t nb = (rows * k + kB - 1) / kB;
    nb = nb < 1 ? 1 : (nb > kSumBlocks ? kSumBlocks : nb);
    hipLaunchKernelGGL(k_coldot, dim3((uint32_t)nb), dim3(kB), 0, s, rows, k, x, y, scratch);
    SFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_colsum_finish, dim3(1), dim3(64), 0, s, (int32_t)nb, k, scratch, 1.0, out);
    SFG_LAUNCH_CHECK();
}

constexpr int kGramBlocks = 256;

size_t gram_scratch_doubles(int32_t k) { return (size_t)kGramBlocks * k * k + 64; }

// out (k x k, row-major) = X^T Y for rows x k blocks X, Y; k <= 32; deterministic
void block_gram(int64_t rows, int32_t k, const double *x, const double *y, double *out, double *scratch,
                hipStream_t s) {
    SFG_REQUIRE(k >= 1 && k <= 32, SFG_EINVAL, "gram: k must be in 1..32");
    const int P = k * k;
    const int L = P >= kB ? 1 : kB / P;
    int64_t nb = (rows + L - 1) / L;
    nb = nb < 1 ? 1 : (nb > kGramBlocks ? kGramBlocks : nb);
    hipLaunchKernelGGL(k_gram, dim3((uint32_t)nb), dim3(kB), 0, s, rows, k, x, y, scratch);
    SFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_gram_finish, dim3(grid_for(P, kB)), dim3(kB), 0, s, (int32_t)nb, P, scratch, out);
    SFG_LAUNCH_CHECK();
}

int64_t scan_groups(int64_t rows, int32_t k) {
    const int64_t tpg = (int64_t)(kB / k) * kTpl;
    return (scan_tiles(rows, k) + tpg - 1) / tpg;
}

// scratch: tile totals/offsets, then group totals/offsets and the column totals
size_t scan_scratch_doubles(int64_t rows, int32_t k) {
    return (size_t)(scan_tiles(rows, k) + scan_groups(rows, k) + 1) * k + 64;
}

// column totals of the last block_scan that used this scratch
const double *scan_totals(int64_t rows, int32_t k, const double *scratch) {
    return scratch + (size_t)(scan_tiles(rows, k) + scan_groups(rows, k)) * k;
}

// inclusive prefix sums down the rows of a rows x k block; y must not alias x
void block_scan(int64_t rows, int32_t k, const double *x, double *y, double *scratch, hipStream_t s) {
    if (rows <= 0) return;
    const int64_t tiles = scan_tiles(rows, k);
    hipLaunchKernelGGL(k_scan_tiles, dim3((uint32_t)tiles), dim3(kB), 0, s, rows, k, x, scratch);
    SFG_LAUNCH_CHECK();
    const int64_t groups = scan_groups(rows, k);
    double *gsum = scratch + (size_t)tiles * k;
    hipLaunchKernelGGL(k_scan_mid, dim3((uint32_t)groups), dim3(kB), 0, s, tiles, k, scratch, gsum);
    SFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kB), 0, s, groups, k, gsum);
    SFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_apply, dim3((uint32_t)tiles), dim3(kB), 0, s, rows, k, x, scratch, gsum, y);
    SFG_LAUNCH_CHECK();
}

// Grid of a row-lane kernel over `rows` rows (at most kLaneBlocks workgroups).
constexpr int kLaneBlocks = 4096;

uint32_t lane_grid(int64_t rows, int32_t k) {
    const int64_t G = kB / k;
    int64_t nb = (rows + G - 1) / G;
    return (uint32_t)(nb < 1 ? 1 : (nb > kLaneBlocks ? kLaneBlocks : nb));
}

size_t lane_partial_doubles(int32_t k) { return (size_t)kLaneBlocks * k + 64; }

void finish_partials(int32_t nb, int32_t k, const double *partial, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_partials_finish, dim3(1), dim3(kFinish), 0, s, nb, k, partial, out);
    SFG_LAUNCH_CHECK();
}

size_t tree_precond_workspace_bytes(int64_t n, int32_t k) {
    Carver c(nullptr);
    const int64_t A = 2 * (n - 1) > 0 ? 2 * (n - 1) : 1;
    c.take<double>((size_t)n * k);
    c.take<double>((size_t)A * k);
    c.take<double>((size_t)A * k);
    c.take<double>(scan_scratch_doubles(A > n ? A : n, k));
    c.take<double>(lane_partial_doubles(k));
    return c.used + 256;
}

// z = L_T^+ r up to a constant per column, for blocks in the tree's preorder
// (row i is node order[i]), and rz[c] = sum_i r[i][c] z[i][c]: the
// conjugate-gradient preconditioner (constants are in the kernel of every
// Laplacian, so they change neither the iterates' residuals nor r . z for r
// orthogonal to the all-one vector).
void tree_precond_pre(const sfg_tree *T, int32_t k, const double *r, double *z, double *rz, void *ws,
                      hipStream_t s) {
    const int64_t n = T->n;
    const int64_t A = 2 * (n - 1) > 0 ? 2 * (n - 1) : 1;
    Carver c(ws);
    double *S = c.take<double>((size_t)n * k);
    double *walk = c.take<double>((size_t)A * k);
    double *U = c.take<double>((size_t)A * k);
    double *sscr = c.take<double>(scan_scratch_doubles(A > n ? A : n, k));
    double *part = c.take<double>(lane_partial_doubles(k));
    if (n > 1) {
        block_scan(n, k, r, S, sscr, s);
        // the column totals of r stay in the scratch until the walk scan reuses it
        hipLaunchKernelGGL(k_edge_drop_pre, dim3(grid_for(n * k, kB)), dim3(kB), 0, s, n, k, T->size, T->pw,
                           T->tdown, T->tup, S, scan_totals(n, k, sscr), walk);
        SFG_LAUNCH_CHECK();
        block_scan(A, k, walk, U, sscr, s);
    }
    const uint32_t nb = lane_grid(n, k);
    hipLaunchKernelGGL(k_potential_dot, dim3(nb), dim3(kB), 0, s, n, k, T->tdown, U, r, z, part);
    SFG_LAUNCH_CHECK();
    finish_partials((int32_t)nb, k, part, rz, s);
}

// ------------------------------------------------------------------ tree layout

struct TreePlan {
    int32_t *rowptr, *col, *eid, *rev, *src, *pos, *down_at, *dbefore, *scan_scr, *pre_of, *parnode, *entered,
        *count, *bad;
    double *val, *deg;
    uint64_t *link0, *link1;
    uint8_t *mask;
    void *csr_ws;
    size_t csr_wsb;
};

static TreePlan plan_tree(Carver &c, int64_t n, int64_t m) {
    const int64_t A = 2 * (n - 1) > 0 ? 2 * (n - 1) : 0;
    TreePlan p;
    p.mask = c.take<uint8_t>(m + 1);
    p.count = c.take<int32_t>(2);
    p.bad = c.take<int32_t>(2);
    p.rowptr = c.take<int32_t>(n + 1);
    p.col = c.take<int32_t>(A + 1);
    p.eid = c.take<int32_t>(A + 1);
    p.val = c.take<double>(A + 1);
    p.deg = c.take<double>(n + 1);
    p.rev = c.take<int32_t>(A + 1);
    p.src = c.take<int32_t>(A + 1);
    p.pos = c.take<int32_t>(A + 1);
    p.down_at = c.take<int32_t>(A + 1);
    p.dbefore = c.take<int32_t>(A + 2);
    p.scan_scr = c.take<int32_t>(scan_scratch_ints(A + 1));
    p.link0 = c.take<uint64_t>(A + 1);
    p.link1 = c.take<uint64_t>(A + 1);
    p.pre_of = c.take<int32_t>(n + 1);
    p.parnode = c.take<int32_t>(n + 1);
    p.entered = c.take<int32_t>(n + 1);
    p.csr_wsb = csr_workspace_bytes(n, m);
    p.csr_ws = c.take<char>(p.csr_wsb);
    return p;
}

size_t tree_order_workspace_bytes(int64_t n, int64_t m) {
    Carver c(nullptr);
    plan_tree(c, n < 1 ? 1 : n, m < 0 ? 0 : m);
    return c.used + 256;
}

// Preorder layout of the spanning tree formed by the edges with keep[e] == 1.
// Synchronises (edge count and the spanning check).
void tree_order(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
                const uint8_t *keep, int32_t *order, int32_t *parent, int32_t *size, double *pw, int32_t *tdown,
                int32_t *tup, void *ws, size_t ws_bytes, hipStream_t s) {
    SFG_REQUIRE(n >= 1 && m >= 0, SFG_EINVAL, "tree_order: need n >= 1 and m >= 0");
    SFG_REQUIRE(2 * m < (int64_t(1) << 31), SFG_EUNSUPPORTED, "tree_order: 2*m must be < 2^31");
    SFG_REQUIRE(wt == SFG_F64, SFG_EINVAL, "tree_order: weights must be F64");
    SFG_REQUIRE(ws_bytes >= tree_order_workspace_bytes(n, m), SFG_EWORKSPACE, "tree_order: workspace too small");
    SFG_REQUIRE(order && parent && size && pw && tdown && tup && (m == 0 || (u && v && w && keep)), SFG_EINVAL,
                "tree_order: null pointer");
    Carver c(ws);
    TreePlan p = plan_tree(c, n, m);
    const int64_t A = 2 * (n - 1);
    fill_i32(p.count, 2, 0, s);
    if (m > 0) {
        hipLaunchKernelGGL(k_mask_eq, dim3(std::min(grid_for(m, kB), kMaskBlocks)), dim3(kB), 0, s, m, keep,
                           (uint8_t)1, p.mask, p.count);
        SFG_LAUNCH_CHECK();
    }
    int32_t cnt = 0;
    SFG_HIP(hipMemcpyAsync(&cnt, p.count, 4, hipMemcpyDeviceToHost, s));
    SFG_HIP(hipStreamSynchronize(s));
    SFG_REQUIRE(cnt == n - 1, SFG_EINVAL,
                "tree_order: " + std::to_string(cnt) + " edges marked 1, a spanning tree has n - 1");
    hipLaunchKernelGGL(k_tree_root, dim3(1), dim3(1), 0, s, n, order, parent, size, pw, tdown, tup, p.pre_of);
    SFG_LAUNCH_CHECK();
    if (A == 0) return;
    // tree CSR with FP64 weights, columns ascending per row
    build_csr(n, m, u, v, w, SFG_F64, p.mask, p.rowptr, p.col, p.val, p.eid, p.deg, p.csr_ws, p.csr_wsb, s);
    const dim3 ga(grid_for(A, kB)), gn(grid_for(n, kB)), b(kB);
    hipLaunchKernelGGL(k_walk_init, ga, b, 0, s, n, A, p.rowptr, p.col, p.rev, p.src, p.link0);
    SFG_LAUNCH_CHECK();
    uint64_t *a0 = p.link0, *a1 = p.link1;
    for (int64_t span = 1; span < A; span <<= 1) {
        hipLaunchKernelGGL(k_walk_jump, ga, b, 0, s, A, a0, a1);
        SFG_LAUNCH_CHECK();
        std::swap(a0, a1);
    }
    // the root's first arc must start a walk through all 2(n - 1) arcs
    uint64_t first = 0;
    SFG_HIP(hipMemcpyAsync(&first, a0, 8, hipMemcpyDeviceToHost, s));   // arc 0 = the root's first arc
    SFG_HIP(hipStreamSynchronize(s));
    if ((int64_t)(first >> 32) != A - 1)
        fail(SFG_ENOTCONN, "tree_order: the edges marked 1 do not form a spanning tree");
    hipLaunchKernelGGL(k_walk_pos, ga, b, 0, s, A, a0, p.rev, p.pos, p.down_at);
    SFG_LAUNCH_CHECK();
    exclusive_scan_i32(p.down_at, p.dbefore, A, p.scan_scr, s);
    fill_i32(p.entered, n, 0, s);
    fill_i32(p.bad, 1, 0, s);
    hipLaunchKernelGGL(k_tree_fill, ga, b, 0, s, A, p.pos, p.rev, p.src, p.col, p.val, p.dbefore, p.pre_of, order,
                       p.parnode, size, pw, tdown, tup, p.entered);
    SFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_tree_parent, gn, b, 0, s, n, p.entered, p.pre_of, p.parnode, parent, p.bad);
    SFG_LAUNCH_CHECK();
    int32_t bad = 0;
    SFG_HIP(hipMemcpyAsync(&bad, p.bad, 4, hipMemcpyDeviceToHost, s));
    SFG_HIP(hipStreamSynchronize(s));
    if (bad) fail(SFG_ENOTCONN, "tree_order: the edges marked 1 do not form a spanning tree");
}

// ------------------------------------------------------------------ tree solve

size_t tree_solve_workspace_bytes(int64_t n, int32_t k) {
    Carver c(nullptr);
    const int64_t A = 2 * (n - 1) > 0 ? 2 * (n - 1) : 1;
    c.take<double>((size_t)n * k);            // bp / xp
    c.take<double>((size_t)n * k);            // S
    c.take<double>((size_t)A * k);            // walk
    c.take<double>((size_t)A * k);            // U
    c.take<double>(128);                      // means
    c.take<double>(colsum_scratch_doubles(k));
    c.take<double>(scan_scratch_doubles(A > n ? A : n, k));
    return c.used + 256;
}

void tree_solve(const sfg_tree *T, int32_t k, const double *b, double *x, void *ws, size_t ws_bytes,
                hipStream_t s) {
    const int64_t n = T->n;
    SFG_REQUIRE(n >= 1 && k >= 1 && k <= 64, SFG_EINVAL, "tree_solve: need n >= 1 and 1 <= k <= 64");
    SFG_REQUIRE(ws_bytes >= tree_solve_workspace_bytes(n, k), SFG_EWORKSPACE, "tree_solve: workspace too small");
    SFG_REQUIRE(b && x && T->order && T->size && T->pw && T->tdown && T->tup, SFG_EINVAL, "tree_solve: null pointer");
    const int64_t A = 2 * (n - 1) > 0 ? 2 * (n - 1) : 1;
    Carver c(ws);
    double *bp = c.take<double>((size_t)n * k);
    double *S = c.take<double>((size_t)n * k);
    double *walk = c.take<double>((size_t)A * k);
    double *U = c.take<double>((size_t)A * k);
    double *mean = c.take<double>(128);
    double *csum = c.take<double>(colsum_scratch_doubles(k));
    double *sscr = c.take<double>(scan_scratch_doubles(A > n ? A : n, k));
    const dim3 gnk(grid_for(n * k, kB)), blk(kB);
    block_colsum(n, k, b, 1.0 / (double)n, mean, csum, s);
    hipLaunchKernelGGL(k_gather_centre, gnk, blk, 0, s, n, k, T->order, b, mean, bp);
    SFG_LAUNCH_CHECK();
    if (n > 1) {
        block_scan(n, k, bp, S, sscr, s);
        hipLaunchKernelGGL(k_edge_drop, gnk, blk, 0, s, n, k, T->size, T->pw, T->tdown, T->tup, S, walk);
        SFG_LAUNCH_CHECK();
        block_scan(A, k, walk, U, sscr, s);
    }
    hipLaunchKernelGGL(k_potential, gnk, blk, 0, s, n, k, T->tdown, U, bp);
    SFG_LAUNCH_CHECK();
    block_colsum(n, k, bp, 1.0 / (double)n, mean + 64, csum, s);
    hipLaunchKernelGGL(k_scatter_centre, gnk, blk, 0, s, n, k, T->order, bp, mean + 64, x);
    SFG_LAUNCH_CHECK();
}

}  // namespace sfg

extern "C" sfg_status sfg_tree_order(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w,
                                     sfg_dtype wt, const uint8_t *keep, int32_t *order, int32_t *parent,
                                     int32_t *size, double *pw, int32_t *tdown, int32_t *tup, void *ws,
                                     size_t ws_bytes, void *stream) {
    return sfg::guard([&] {
        sfg::tree_order(n, m, u, v, w, wt, keep, order, parent, size, pw, tdown, tup, ws, ws_bytes,
                        sfg::as_stream(stream));
    });
}

extern "C" sfg_status sfg_tree_solve(const sfg_tree *T, int32_t k, const double *b, double *x, void *ws,
                                     size_t ws_bytes, void *stream) {
    return sfg::guard([&] {
        SFG_REQUIRE(T, SFG_EINVAL, "tree_solve: null tree");
        sfg::tree_solve(T, k, b, x, ws, ws_bytes, sfg::as_stream(stream));
    });
}
