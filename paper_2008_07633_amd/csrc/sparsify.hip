// Sparsifier driver (the problem of Sec. 2.2, Alg. 1) and its helpers:
// input validation, candidate compaction, and workspace sizing.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <mutex>
#include <numeric>
#include <vector>

#include "common.hpp"

namespace sfg {

// from the other translation units
size_t csr_workspace_bytes(int64_t n, int64_t m);
size_t csr_select_workspace_bytes(int64_t n, int64_t m);
void build_csr(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
               const uint8_t *mask, int32_t *rowptr, int32_t *col, void *val, int32_t *eid, void *deg, void *ws,
               size_t ws_bytes, hipStream_t s);
size_t smooth_workspace_bytes(int64_t n, int32_t k, sfg_dtype storage);
size_t smooth_ordered_workspace_bytes(int64_t n, int32_t k, sfg_dtype storage);
size_t color_workspace_bytes(int64_t n);
size_t tree_order_workspace_bytes(int64_t n, int64_t m);
size_t tree_solve_workspace_bytes(int64_t n, int32_t k);
void random_block(int64_t n, int32_t k, uint64_t seed, uint32_t block, double *x, hipStream_t s);
void color_graph(const sfg_csr *H, int32_t *color, int32_t *class_rows, std::vector<int32_t> &class_ptr, void *ws,
                 size_t ws_bytes, hipStream_t s);
void smooth_gs(const sfg_csr *H, int32_t k, int32_t sweeps, double omega, const double *x0, sfg_dtype storage,
               const int32_t *class_rows, const std::vector<int32_t> &class_ptr, void *x, void *ws, size_t ws_bytes,
               hipStream_t s);
void smooth(const sfg_csr *H, int32_t k, int32_t sweeps, double omega, const double *x0, sfg_dtype storage,
            int32_t final_f32, void *x, void *ws, size_t ws_bytes, hipStream_t s, int32_t max_row);
void max_row_length(const sfg_csr *H, int32_t *out, hipStream_t s);
void edge_scores(const void *x, sfg_dtype xt, int64_t n, int32_t k, int64_t ne, const int32_t *cand,
                 const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt, void *score, sfg_dtype st,
                 hipStream_t s);
size_t select_workspace_bytes(int64_t ne);
void csr_select(const sfg_csr *G, const uint8_t *mask, int32_t *rowptr, int32_t *col, void *val, int32_t *eid,
                void *deg, void *ws, size_t ws_bytes, hipStream_t s);
void select_topk(const void *score, sfg_dtype st, int64_t ne, int64_t k, uint8_t *sel, double *tau, void *ws,
                 size_t ws_bytes, hipStream_t s);
size_t affinity_workspace_bytes(int64_t n, int32_t k);
size_t coarsen_workspace_bytes(int64_t n, int64_t m);
size_t mpnn_forward_workspace_bytes(int64_t n, sfg_dtype act);
size_t mpnn_train_workspace_bytes(int64_t n, int64_t ne);
size_t smooth_ordered_workspace_bytes(int64_t n, int32_t k, sfg_dtype storage);
int smooth_ordered(const sfg_csr *H, const int32_t *order, int32_t k, int32_t sweeps, double omega,
                   const double *x0, sfg_dtype storage, int32_t final_f32, void *x, void *ws, size_t ws_bytes,
                   hipStream_t s, int32_t max_row);
double predicted_cone_share(const sfg_csr *H, int32_t sweeps, int64_t n_cand, const int32_t *cand,
                            const int32_t *u, const int32_t *v, double band, double limit, DevArena &A,
                            hipStream_t s);
void far_entries(const sfg_csr *H, int64_t window, unsigned long long *count, hipStream_t s);
void inverse_permutation(int64_t n, const int32_t *order, int32_t *inv, hipStream_t s);
sfg_csr relabel_csr(const sfg_csr *H, const int32_t *order, const int32_t *inv, DevArena &A, hipStream_t s);
void map_endpoints(int64_t m, const int32_t *inv, const int32_t *u, const int32_t *v, int32_t *nu, int32_t *nv,
                   hipStream_t s);
void gather_block(int64_t n, int32_t k, const int32_t *order, const double *src, double *dst, hipStream_t s);
void tree_order(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
                const uint8_t *keep, int32_t *order, int32_t *parent, int32_t *size, double *pw, int32_t *tdown,
                int32_t *tup, void *ws, size_t ws_bytes, hipStream_t s);
void band_rescore(const sfg_csr *H64, int32_t k, int32_t sweeps, double omega, const double *x0, int64_t n_cand,
                  const int32_t *cand, const int32_t *u, const int32_t *v, const double *w64, const float *score_lo,
                  int64_t k_sel, double tau_lo, double band, uint8_t *sel, sfg_level_report *rep, DevArena &A,
                  hipStream_t s);
void multilevel_sparsify(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
                         const sfg_params *p, const double *x0, uint8_t *keep, sfg_report *rep, DevArena &A,
                         hipStream_t s);

// ------------------------------------------------------------------ device arena (sfg_sparsify only)

// The default pool of stream-ordered allocations returns freed memory to the
// driver at every synchronisation unless told to keep some: each call would
// then map its buffers afresh.  Keep up to 16 GiB cached per device (set once
// per device; the memory is reused by later calls, not by other allocators).
static void keep_pool_memory() {
    static bool done[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64 || done[dev]) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t keep = uint64_t(16) << 30;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    (void)hipGetLastError();
    done[dev] = true;
}

namespace {

constexpr size_t kChunkBytes = size_t(256) << 20;
constexpr size_t kCacheBytes = size_t(16) << 30;

std::mutex g_cache_mu;
std::vector<DevArena::Chunk> g_cache[kMaxDevices];
size_t g_cached[kMaxDevices];

}  // namespace

DevArena::DevArena(hipStream_t st) : s(st) {
    const char *e = getenv("SFG_FAIL_ALLOC_AFTER");
    fail_after = e ? atol(e) : -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = -1;
    (void)hipGetLastError();
    keep_pool_memory();
}

void DevArena::finish() {
    SFG_HIP(hipStreamSynchronize(s));
    synced = true;
}

DevArena::~DevArena() {
    if (synced && dev >= 0) {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        for (const Chunk &c : chunks) {
            if (g_cached[dev] + c.size <= kCacheBytes) {
                g_cache[dev].push_back(c);
                g_cached[dev] += c.size;
            } else {
                (void)hipFreeAsync(c.p, s);
            }
        }
    } else {
        for (const Chunk &c : chunks) (void)hipFreeAsync(c.p, s);
    }
    (void)hipGetLastError();
}

void *DevArena::raw(size_t bytes) {
    if (fail_after >= 0 && count >= fail_after) fail(SFG_ENOMEM, "device allocation failed (SFG_FAIL_ALLOC_AFTER)");
    ++count;
    const size_t need = ((bytes < 256 ? 256 : bytes) + 255) & ~size_t(255);
    if (!chunks.empty() && used + need <= chunks.back().size) {
        void *p = static_cast<char *>(chunks.back().p) + used;
        used += need;
        return p;
    }
    Chunk c{nullptr, 0};
    if (dev >= 0) {   // the smallest cached chunk that fits
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto &cache = g_cache[dev];
        size_t best = cache.size();
        for (size_t i = 0; i < cache.size(); ++i)
            if (cache[i].size >= need && (best == cache.size() || cache[i].size < cache[best].size)) best = i;
        if (best < cache.size()) {
            c = cache[best];
            cache.erase(cache.begin() + (long)best);
            g_cached[dev] -= c.size;
        }
    }
    if (!c.p) {
        c.size = need > kChunkBytes ? need : kChunkBytes;
        hipError_t e = hipMallocAsync(&c.p, c.size, s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail(SFG_ENOMEM, std::string("device allocation of ") + std::to_string(c.size) + " bytes failed: " +
                                 hipGetErrorString(e));
        }
    }
    chunks.push_back(c);
    used = need;
    return c.p;
}

// ------------------------------------------------------------------ validation

namespace {

template <typename TW>
__global__ void k_validate(int64_t n, int64_t m, const int32_t *__restrict__ u, const int32_t *__restrict__ v,
                           const TW *__restrict__ w, uint32_t *flag) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const int32_t a = u[e], b = v[e];
    uint32_t bad = 0;
    if (a < 0 || b >= n || a >= b) bad |= 1u;
    if (e > 0) {
        const int32_t pa = u[e - 1], pb = v[e - 1];
        if (!(pa < a || (pa == a && pb < b))) bad |= 2u;
    }
    const double we = (double)w[e];
    if (!(we > 0.0) || !(we < __builtin_inf())) bad |= 4u;
    if (bad) atomicOr(flag, bad);
}

__global__ void k_flags_eq(int64_t m, const uint8_t *__restrict__ mask, uint8_t want, int32_t *flags) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) flags[e] = (mask[e] == want) ? 1 : 0;
}

__global__ void k_scatter_ids(int64_t m, const int32_t *__restrict__ flags, const int32_t *__restrict__ pos,
                              int32_t *out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m && flags[e]) out[pos[e]] = (int32_t)e;
}

__global__ void k_f64_to_f32(int64_t m, const double *__restrict__ a, float *__restrict__ b) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) b[e] = (float)a[e];
}

__global__ void k_f32_to_f64(int64_t m, const float *__restrict__ a, double *__restrict__ b) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) b[e] = (double)a[e];
}

// keep from the base sparsifier: 0 stays 0, an earlier round's addition (2)
// stays 2, any other member is 1
__global__ void k_keep_init(int64_t m, const uint8_t *__restrict__ base, uint8_t *keep) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) keep[e] = base[e] == 2 ? 2 : (base[e] ? 1 : 0);
}

__global__ void k_keep_add(int64_t nc, const int32_t *__restrict__ cand, const uint8_t *__restrict__ sel,
                           uint8_t *keep) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nc && sel[i]) keep[cand[i]] = 2;
}

}  // namespace

void validate_edges(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
                    DevArena &A, hipStream_t s) {
    SFG_REQUIRE(n >= 1 && m >= 0, SFG_EINVAL, "edge list: need n >= 1, m >= 0");
    SFG_REQUIRE(wt == SFG_F64 || wt == SFG_F32, SFG_EINVAL, "edge list: weights must be F64 or F32");
    if (m == 0) return;
    uint32_t *flag = A.alloc<uint32_t>(1);
    fill_i32(reinterpret_cast<int32_t *>(flag), 1, 0, s);
    if (wt == SFG_F64)
        hipLaunchKernelGGL(k_validate<double>, dim3(grid_for(m, 256)), dim3(256), 0, s, n, m, u, v,
                           (const double *)w, flag);
    else
        hipLaunchKernelGGL(k_validate<float>, dim3(grid_for(m, 256)), dim3(256), 0, s, n, m, u, v, (const float *)w,
                           flag);
    SFG_LAUNCH_CHECK();
    uint32_t h = 0;
    SFG_HIP(hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, s));
    SFG_HIP(hipStreamSynchronize(s));
    if (h & 1u) fail(SFG_EINVAL, "edge list: an edge has u >= v or an id out of range");
    if (h & 2u) fail(SFG_EINVAL, "edge list: not sorted by (u, v) or has duplicates");
    if (h & 4u) fail(SFG_EINVAL, "edge list: a weight is not finite and positive");
}

// Edge ids e with mask[e] == want, ascending; returns their count (synchronises).
int64_t compact_ids(const uint8_t *mask, uint8_t want, int64_t m, int32_t *out, DevArena &A, hipStream_t s) {
    if (m == 0) return 0;
    int32_t *flags = A.alloc<int32_t>(m + 1);
    int32_t *pos = A.alloc<int32_t>(m + 1);
    int32_t *scr = A.alloc<int32_t>(scan_scratch_ints(m + 1));
    hipLaunchKernelGGL(k_flags_eq, dim3(grid_for(m, 256)), dim3(256), 0, s, m, mask, want, flags);
    SFG_LAUNCH_CHECK();
    exclusive_scan_i32(flags, pos, m, scr, s);
    hipLaunchKernelGGL(k_scatter_ids, dim3(grid_for(m, 256)), dim3(256), 0, s, m, flags, pos, out);
    SFG_LAUNCH_CHECK();
    int32_t cnt = 0;
    SFG_HIP(hipMemcpyAsync(&cnt, pos + m, sizeof(cnt), hipMemcpyDeviceToHost, s));
    SFG_HIP(hipStreamSynchronize(s));
    return cnt;
}

void convert_weights(const void *w, sfg_dtype wt, sfg_dtype want, int64_t m, void *out, hipStream_t s) {
    if (m == 0) return;
    if (wt == want) {
        SFG_HIP(hipMemcpyAsync(out, w, (size_t)m * dtype_size(wt), hipMemcpyDeviceToDevice, s));
    } else if (wt == SFG_F64 && want == SFG_F32) {
        hipLaunchKernelGGL(k_f64_to_f32, dim3(grid_for(m, 256)), dim3(256), 0, s, m, (const double *)w, (float *)out);
    } else if (wt == SFG_F32 && want == SFG_F64) {
        hipLaunchKernelGGL(k_f32_to_f64, dim3(grid_for(m, 256)), dim3(256), 0, s, m, (const float *)w, (double *)out);
    } else {
        fail(SFG_EINVAL, "weights: unsupported conversion");
    }
    SFG_LAUNCH_CHECK();
}

int64_t spanning_tree_gpu(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
                          const uint8_t *allowed, uint8_t *in_tree, DevArena &A, hipStream_t s);

// ------------------------------------------------------------------ one scoring pass

namespace {

struct Timer {
    hipEvent_t a, b;
    hipStream_t s;
    explicit Timer(hipStream_t st) : s(st) {
        SFG_HIP(hipEventCreate(&a));
        SFG_HIP(hipEventCreate(&b));
    }
    ~Timer() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
    void start() { SFG_HIP(hipEventRecord(a, s)); }
    float stop() {
        SFG_HIP(hipEventRecord(b, s));
        SFG_HIP(hipEventSynchronize(b));
        float ms = 0;
        SFG_HIP(hipEventElapsedTime(&ms, a, b));
        return ms;
    }
};

}  // namespace

// Numbering of the nodes for the sweeps of one sparsify call, decided at its
// first scored level and kept for the later batches: the input numbering, or
// the preorder of the spanning tree (the edges marked 1 in the level's base).
// The preorder is taken when the call plans at least kOrderMinLaunches
// column-part sweep launches (sweeps x ceil(k / 8) x batches), the graph has
// at least kOrderMinRows nodes and more than a quarter of the scoring graph's
// entries reach beyond kNearRows rows of their own row.  The launch bound
// comes from the 2M-point k-NN graph (20 sweeps of 32 vectors: 80 launches a
// batch): the layout costs about 1.9 ns per node once and 0.4 ns per batch
// (relabelled scoring graph, gathered start block) and saves about 10 ps per
// node and launch; one batch ran 14.6 ms in the input numbering against
// 16.6 ms in preorder, four batches 44.8 against 44.3 ms.
// SFG_NODE_ORDER=0 keeps the input numbering, =1 always takes the preorder
// (read at every call; tests use it).  Results do not depend on the choice.

namespace {

constexpr int64_t kNearRows = 4096;
constexpr int64_t kOrderMinRows = int64_t(1) << 16;
constexpr int64_t kOrderMinLaunches = 512;

int64_t planned_launches(const sfg_params *p, int64_t batches) {
    return (int64_t)p->sweeps * ((p->k + 7) / 8) * batches;
}

int node_order_mode() {
    const char *e = getenv("SFG_NODE_ORDER");
    if (e && e[0] == '0' && e[1] == 0) return 0;
    if (e && e[0] == '1' && e[1] == 0) return 1;
    return 2;
}

void make_node_order(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const double *w64,
                     const uint8_t *base, NodeOrder *no, DevArena &A, hipStream_t s) {
    no->order = A.alloc<int32_t>(n + 1);
    no->inv = A.alloc<int32_t>(n + 1);
    no->u = A.alloc<int32_t>(m + 1);
    no->v = A.alloc<int32_t>(m + 1);
    int32_t *parent = A.alloc<int32_t>(n + 1), *size = A.alloc<int32_t>(n + 1);
    int32_t *tdown = A.alloc<int32_t>(n + 1), *tup = A.alloc<int32_t>(n + 1);
    double *pw = A.alloc<double>(n + 1);
    const size_t wsb = tree_order_workspace_bytes(n, m);
    tree_order(n, m, u, v, w64, SFG_F64, base, no->order, parent, size, pw, tdown, tup, A.raw(wsb), wsb, s);
    inverse_permutation(n, no->order, no->inv, s);
    map_endpoints(m, no->inv, u, v, no->u, no->v, s);
}

}  // namespace

// Node order of one level of the hierarchy (Alg. 1): decided once per level
// and used for its sweeps on G_l (the coarsening affinities) and, when the
// level is scored, on its sparsifier.  The preorder of a spanning tree of G_l
// (`tree`: its edges marked 1; nullptr = compute the maximum one) is taken
// when the level has at least kOrderMinRows nodes, its block of k vectors
// exceeds kOrderMinBlock bytes (kOrderMinBlockNoTree when the tree would have
// to be computed first) and more than half of G_l's entries reach beyond
// kNearRows rows.  The 4M-node Chung-Lu level-0 graph (input ids in
// expected-degree order) sweeps in 1.38 ms in preorder against 3.57 ms (FP32)
// and 5.9 against 7.3 ms (FP64); its FP32 hierarchy took 293 ms against 342.
// Its 1M-node level 1 in FP64 (126 MB block, mostly served from the 256 MB
// memory-side cache) gained less than its spanning tree and relabelling cost.
// SFG_NODE_ORDER as above; results do not depend on the choice.
constexpr double kOrderMinBlock = 96.0 * (1 << 20);
constexpr double kOrderMinBlockNoTree = 256.0 * (1 << 20);

void level_node_order(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const double *w64, const sfg_csr *G,
                      const uint8_t *tree, int32_t k, sfg_dtype storage, NodeOrder *no, DevArena &A,
                      hipStream_t s) {
    no->decided = true;
    no->use = false;
    const int mode = node_order_mode();
    if (mode == 0 || n < 2) return;
    if (mode == 2) {
        const double block = (double)n * k * dtype_size(storage);
        if (n < kOrderMinRows || block <= (tree ? kOrderMinBlock : kOrderMinBlockNoTree)) return;
        unsigned long long *far = A.alloc<unsigned long long>(1);
        fill_i32((int32_t *)far, 2, 0, s);
        far_entries(G, kNearRows, far, s);
        unsigned long long far_h = 0;
        SFG_HIP(hipMemcpyAsync(&far_h, far, 8, hipMemcpyDeviceToHost, s));
        SFG_HIP(hipStreamSynchronize(s));
        if (2 * far_h <= (unsigned long long)G->nnz) return;
    }
    if (!tree) {
        uint8_t *t = A.alloc<uint8_t>(m + 1);
        spanning_tree_gpu(n, m, u, v, w64, SFG_F64, nullptr, t, A, s);
        tree = t;
    }
    no->use = true;
    make_node_order(n, m, u, v, w64, tree, no, A, s);
}

namespace {

// The scoring graph's CSR with values of type vt, in the numbering the sweeps
// use: the node order is decided at the call's first scored level (see
// NodeOrder above) and applied by copying rows in their stored entry order.
struct ScoringGraph {
    sfg_csr H{};
    int32_t max_row = -1;   // longest row when the values are FP64 (FP64 hub rows are summed through LDS)
};

ScoringGraph scoring_graph(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const double *w64,
                           const float *w32, sfg_dtype vt, const uint8_t *hmask, const uint8_t *base,
                           const sfg_params *p, NodeOrder *no, DevArena &A, hipStream_t s) {
    const void *wv = vt == SFG_F64 ? (const void *)w64 : (const void *)w32;
    int32_t *rowptr = A.alloc<int32_t>(n + 1);
    int32_t *col = A.alloc<int32_t>(2 * m + 1);
    int32_t *eid = A.alloc<int32_t>(2 * m + 1);
    void *val = A.raw((2 * m + 1) * dtype_size(vt));
    void *deg = A.raw(n * dtype_size(vt));
    const size_t wsb = csr_workspace_bytes(n, m);
    build_csr(n, m, u, v, wv, vt, hmask, rowptr, col, val, eid, deg, A.raw(wsb), wsb, s);
    ScoringGraph G;
    G.H = sfg_csr{n, 0, rowptr, col, val, eid, deg, vt};
    const int mode = node_order_mode();
    const bool decide = no && !no->decided && p->smoother == SFG_SMOOTH_JACOBI && n >= 2 && mode != 0;
    unsigned long long *far = nullptr;
    if (decide && mode == 2 && n >= kOrderMinRows && no->launches >= kOrderMinLaunches) {
        far = A.alloc<unsigned long long>(1);
        fill_i32((int32_t *)far, 2, 0, s);
        far_entries(&G.H, kNearRows, far, s);
    }
    // FP64 sums hub rows through LDS only where they are known to exist: the
    // longest row comes back with the entry count
    int32_t *mr = nullptr;
    if (vt == SFG_F64) {
        mr = A.alloc<int32_t>(1);
        max_row_length(&G.H, mr, s);
    }
    int32_t nnz = 0;
    unsigned long long far_h = 0;
    SFG_HIP(hipMemcpyAsync(&nnz, rowptr + n, 4, hipMemcpyDeviceToHost, s));
    if (far) SFG_HIP(hipMemcpyAsync(&far_h, far, 8, hipMemcpyDeviceToHost, s));
    if (mr) SFG_HIP(hipMemcpyAsync(&G.max_row, mr, 4, hipMemcpyDeviceToHost, s));
    SFG_HIP(hipStreamSynchronize(s));
    G.H.nnz = nnz;
    if (no && !no->decided) {
        no->decided = true;
        no->use = decide && (mode == 1 || (far && 4 * far_h > (unsigned long long)nnz));
        if (no->use) make_node_order(n, m, u, v, w64, base, no, A, s);
    }
    if (no && no->use) G.H = relabel_csr(&G.H, no->order, no->inv, A, s);
    return G;
}

}  // namespace

// Embed (smooth on the scoring graph), score the edges outside `base`, add
// the top k_take of them (k_take < 0: ceil(frac * n_cand)).  Writes keep
// (1 = base, 2 = added); keep may be base itself.  `no` (may be nullptr):
// the node numbering of the sweeps, decided here when not decided yet.
void score_level(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const double *w64, const float *w32,
                 const uint8_t *base, const sfg_params *p, const double *x0, uint8_t *keep, sfg_level_report *rep,
                 DevArena &A, hipStream_t s, int64_t k_take, NodeOrder *no) {
    const uint8_t *hmask = (p->embed == SFG_EMBED_GRAPH) ? nullptr : base;
    Timer tm(s);
    tm.start();
    // The precision form (reduced-precision storage with an FP64 band) needs the
    // FP64 scoring graph, for the band re-scoring or for the FP64 path the
    // prediction below may send the level to: it is built first, and the
    // reduced-precision values only when that path runs.
    const bool band_form = p->storage != SFG_F64 && p->band > 0.0;
    ScoringGraph G64, G;
    if (band_form) G64 = scoring_graph(n, m, u, v, w64, w32, SFG_F64, hmask, base, p, no, A, s);
    else G = scoring_graph(n, m, u, v, w64, w32, p->storage == SFG_F64 ? SFG_F64 : SFG_F32, hmask, base, p, no,
                           A, s);
    // su, sv, sx0: endpoints and start block in the numbering the sweeps use
    const int32_t *su = u, *sv = v;
    const double *sx0 = x0;
    if (no && no->use) {
        double *xg = A.alloc<double>((size_t)n * p->k + 1);
        gather_block(n, p->k, no->order, x0, xg, s);
        sx0 = xg;
        su = no->u;
        sv = no->v;
    }
    // Precision form: when the FP64 re-scoring cone of the expected band would
    // cover more than a quarter of the full pass's row updates, the full FP64
    // smoothing would run after the reduced-precision one anyway; take the FP64
    // path directly (the same selection as the precision form reaches whenever
    // its margin covers the error, and always the FP64 oracle's).
    // SFG_PRECISION_PREDICT=0 (read at every call) keeps the precision form
    // regardless (tests use it to exercise the band re-scoring).
    const char *pe = getenv("SFG_PRECISION_PREDICT");
    const bool predict = band_form && !(pe && atoi(pe) == 0) && p->smoother == SFG_SMOOTH_JACOBI;
    bool fallback = false;
    // candidates: edges outside the current sparsifier, ascending id
    int32_t *cand = nullptr;
    int64_t nc = -1;
    if (predict) {
        cand = A.alloc<int32_t>(m + 1);
        nc = compact_ids(base, 0, m, cand, A, s);
        const int32_t *cand0 = cand;
        const int64_t nc0 = nc;
        const int64_t ks0 = k_take >= 0 ? k_take : (int64_t)std::ceil(p->frac * (double)nc0);
        fallback = ks0 > 0 && ks0 < nc0 &&
                   4.0 * predicted_cone_share(&G64.H, p->sweeps, nc0, cand0, su, sv, p->band, 0.25, A, s) > 1.0;
    }
    sfg_params p64;
    const sfg_params *q = p;
    if (fallback) {
        p64 = *p;
        p64.storage = SFG_F64;
        p64.band = 0.0;
        p64.final_f32 = 0;
        q = &p64;
        G = G64;
    } else if (band_form) {
        G = scoring_graph(n, m, u, v, w64, w32, SFG_F32, hmask, base, p, no, A, s);
    }
    const bool f64 = q->storage == SFG_F64;
    const sfg_dtype vt = f64 ? SFG_F64 : SFG_F32;
    const void *wv = f64 ? (const void *)w64 : (const void *)w32;
    const sfg_csr &H = G.H;
    // embedding
    const bool f32last = q->final_f32 && (q->storage == SFG_F16 || q->storage == SFG_BF16);
    const sfg_dtype xt = f32last ? SFG_F32 : q->storage;
    void *x = A.raw((size_t)n * q->k * dtype_size(xt));
    // in the tree's preorder the Jacobi sweeps can take several per pass (smooth_ordered decides, same bits)
    const bool passes = no && no->use && q->smoother == SFG_SMOOTH_JACOBI;
    size_t wss = passes ? smooth_ordered_workspace_bytes(n, q->k, q->storage) : smooth_workspace_bytes(n, q->k, q->storage);
    void *wsm = A.raw(wss);
    float ms_other = tm.stop();
    tm.start();
    if (q->smoother == SFG_SMOOTH_GAUSS_SEIDEL) {
        int32_t *color = A.alloc<int32_t>(n + 1);
        int32_t *class_rows = A.alloc<int32_t>(n + 1);
        const size_t wsc = color_workspace_bytes(n);
        std::vector<int32_t> class_ptr;
        color_graph(&H, color, class_rows, class_ptr, A.raw(wsc), wsc, s);
        smooth_gs(&H, q->k, q->sweeps, q->omega, sx0, q->storage, class_rows, class_ptr, x, wsm, wss, s);
    } else if (passes) {
        const int per_pass = smooth_ordered(&H, nullptr, q->k, q->sweeps, q->omega, sx0, q->storage, q->final_f32, x,
                                            wsm, wss, s, G.max_row);
        if (rep) rep->sweeps_per_pass = per_pass;
    } else {
        smooth(&H, q->k, q->sweeps, q->omega, sx0, q->storage, q->final_f32, x, wsm, wss, s, G.max_row);
    }
    float ms_smooth = tm.stop();
    tm.start();
    if (!cand) {
        cand = A.alloc<int32_t>(m + 1);
        nc = compact_ids(base, 0, m, cand, A, s);
    }
    const sfg_dtype st = f64 ? SFG_F64 : SFG_F32;
    void *score = A.raw((nc + 1) * dtype_size(st));
    edge_scores(x, xt, n, q->k, nc, cand, su, sv, wv, vt, score, st, s);
    float ms_score = tm.stop();
    tm.start();
    const int64_t ksel = k_take >= 0 ? k_take : (int64_t)std::ceil(q->frac * (double)nc);
    SFG_REQUIRE(ksel <= nc, SFG_EINVAL, "sparsify: more edges requested than candidates");
    uint8_t *sel = A.alloc<uint8_t>(nc + 1);
    double *tau = A.alloc<double>(1);
    size_t wsel = select_workspace_bytes(nc);
    void *wse = A.raw(wsel);
    select_topk(score, st, nc, ksel, sel, tau, wse, wsel, s);
    double tau_h = 0;
    SFG_HIP(hipMemcpyAsync(&tau_h, tau, 8, hipMemcpyDeviceToHost, s));
    SFG_HIP(hipStreamSynchronize(s));
    if (tau_h != tau_h) fail(SFG_ENUMERIC, "sparsify: NaN or negative edge score");
    if (rep) {
        rep->n = n;
        rep->m = m;
        rep->n_cand = nc;
        rep->k_sel = ksel;
        rep->tau = tau_h;
        rep->band = 0;
        rep->band_above = 0;
        rep->band_rounds = 0;
        rep->cone_rows = fallback ? (int64_t)p->sweeps * n : 0;
        rep->precision_fallback = fallback ? 1 : 0;
        rep->node_order = (no && no->use) ? 1 : 0;
        rep->n_scored = nc;
        if (!passes) rep->sweeps_per_pass = 1;
    }
    if (!f64 && q->band > 0.0 && ksel > 0 && ksel < nc) {
        // precision form: FP64 re-scoring of the edges near the threshold
        band_rescore(&G64.H, q->k, q->sweeps, q->omega, sx0, nc, cand, su, sv, w64, (const float *)score, ksel,
                     tau_h, q->band, sel, rep, A, s);
    }
    hipLaunchKernelGGL(k_keep_init, dim3(grid_for(m, 256)), dim3(256), 0, s, m, base, keep);
    SFG_LAUNCH_CHECK();
    if (nc > 0) {
        hipLaunchKernelGGL(k_keep_add, dim3(grid_for(nc, 256)), dim3(256), 0, s, nc, cand, sel, keep);
        SFG_LAUNCH_CHECK();
    }
    float ms_select = tm.stop();
    if (rep) {
        rep->ms_smooth = ms_smooth;
        rep->ms_score = ms_score;
        rep->ms_select = ms_select;
        rep->ms_other = ms_other;
    }
}

void sigma_sparsify(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const double *w64, const float *w32,
                    const uint8_t *tree, const sfg_params *p, const double *x0, uint8_t *keep, sfg_report *rep,
                    DevArena &A, hipStream_t s);

bool surrogate_sparsify(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const double *w64,
                        const float *w32, const uint8_t *tree, const sfg_params *p, const double *x0, uint8_t *keep,
                        sfg_level_report *rep, DevArena &A, hipStream_t s);

void single_level_sparsify(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
                           const sfg_params *p, const double *x0, uint8_t *keep, sfg_report *rep, DevArena &A,
                           hipStream_t s) {
    double *w64 = A.alloc<double>(m + 1);
    convert_weights(w, wt, SFG_F64, m, w64, s);
    float *w32 = nullptr;
    if (p->storage != SFG_F64 || p->surrogate) {
        w32 = A.alloc<float>(m + 1);
        convert_weights(w, wt, SFG_F32, m, w32, s);
    }
    uint8_t *tree = A.alloc<uint8_t>(m + 1);
    const int64_t comps = spanning_tree_gpu(n, m, u, v, w64, SFG_F64, nullptr, tree, A, s);
    if (comps != 1) fail(SFG_ENOTCONN, "sparsify: graph has " + std::to_string(comps) + " components");
    if (p->sigma > 0.0) {
        sigma_sparsify(n, m, u, v, w64, w32, tree, p, x0, keep, rep, A, s);
        return;
    }
    if (p->surrogate) {
        if (rep) rep->levels = 1;
        if (surrogate_sparsify(n, m, u, v, w64, w32, tree, p, x0, keep, rep ? &rep->level[0] : nullptr, A, s))
            return;
        if (rep) rep->level[0].surrogate_fallback = 1;
    }
    const int32_t rounds = p->rounds > 1 ? p->rounds : 1;
    if (rep) rep->levels = rounds;
    if (rounds == 1) {
        NodeOrder no;
        no.launches = planned_launches(p, 1);
        score_level(n, m, u, v, w64, w32, tree, p, x0, keep, rep ? &rep->level[0] : nullptr, A, s, -1, &no);
        return;
    }
    // multi-round densification: the budget of the single pass in near-equal
    // quotas, each scored on the sparsifier grown so far (keep is its own base)
    const int64_t k_total = (int64_t)std::ceil(p->frac * (double)(m - (n - 1)));
    hipLaunchKernelGGL(k_keep_init, dim3(grid_for(m, 256)), dim3(256), 0, s, m, tree, keep);
    SFG_LAUNCH_CHECK();
    NodeOrder no;
    no.launches = planned_launches(p, rounds);
    for (int32_t r = 0; r < rounds; ++r) {
        const int64_t q = k_total * (r + 1) / rounds - k_total * r / rounds;
        score_level(n, m, u, v, w64, w32, keep, p, x0 + (size_t)r * n * p->k, keep,
                    rep ? &rep->level[r] : nullptr, A, s, q, &no);
    }
}

// ---------------------------------------------------------------- learned candidate pruning

namespace {

__global__ void k_first_cols(int64_t n, int32_t k, int32_t kc, const double *__restrict__ x, double *__restrict__ y) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * kc) return;
    const int64_t i = t / kc;
    y[t] = x[i * k + (t - i * kc)];
}

__global__ void k_nonfinite(int64_t len, const float *__restrict__ a, int32_t *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len && !__builtin_isfinite(a[i])) atomicOr(bad, 1);
}

__global__ void k_take_ids(int64_t nb, const int32_t *__restrict__ pos, const int32_t *__restrict__ ids,
                           int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb) out[i] = ids[pos[i]];
}

void check_status(sfg_status st) {
    if (st != SFG_OK) fail(st, sfg_last_error());
}

}  // namespace

// The plain single-level pass with the exact scoring restricted to the
// surrogate's top cand_frac of the off-tree edges (the steps are listed with
// sfg_surrogate in the header).  Returns false, having done nothing, when the
// model is not usable.
bool surrogate_sparsify(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const double *w64,
                        const float *w32, const uint8_t *tree, const sfg_params *p, const double *x0, uint8_t *keep,
                        sfg_level_report *rep, DevArena &A, hipStream_t s) {
    const sfg_surrogate &sg = *p->surrogate;
    const int64_t np = sfg_mpnn_param_count();
    int32_t *bad = A.alloc<int32_t>(1);
    fill_i32(bad, 1, 0, s);
    hipLaunchKernelGGL(k_nonfinite, dim3(grid_for(np, 256)), dim3(256), 0, s, np, sg.params, bad);
    SFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_nonfinite, dim3(1), dim3(256), 0, s, (int64_t)24, sg.norm, bad);
    SFG_LAUNCH_CHECK();
    int32_t bad_h = 0;
    SFG_HIP(hipMemcpyAsync(&bad_h, bad, 4, hipMemcpyDeviceToHost, s));
    SFG_HIP(hipStreamSynchronize(s));
    if (bad_h) return false;
    Timer tm(s);
    tm.start();
    // candidates: the off-tree edges, ascending id
    int32_t *cand = A.alloc<int32_t>(m + 1);
    const int64_t nc = compact_ids(tree, 0, m, cand, A, s);
    // G's CSR and the tree's, FP32 weights
    const size_t wsb = csr_workspace_bytes(n, m);
    void *ws = A.raw(wsb);
    int32_t *grp = A.alloc<int32_t>(n + 1), *gcol = A.alloc<int32_t>(2 * m + 1), *geid = A.alloc<int32_t>(2 * m + 1);
    float *gval = A.alloc<float>(2 * m + 1), *gdeg = A.alloc<float>(n + 1);
    build_csr(n, m, u, v, w32, SFG_F32, nullptr, grp, gcol, gval, geid, gdeg, ws, wsb, s);
    const sfg_csr G{n, 2 * m, grp, gcol, gval, geid, gdeg, SFG_F32};
    int32_t *trp = A.alloc<int32_t>(n + 1), *tcol = A.alloc<int32_t>(2 * n), *teid = A.alloc<int32_t>(2 * n);
    float *tval = A.alloc<float>(2 * n), *tdeg = A.alloc<float>(n + 1);
    const size_t wss = csr_select_workspace_bytes(n, m);
    csr_select(&G, tree, trp, tcol, tval, teid, tdeg, A.raw(wss), wss, s);
    const sfg_csr T{n, 2 * (n - 1), trp, tcol, tval, teid, tdeg, SFG_F32};
    // cheap embedding, features, prediction
    double *x0c = A.alloc<double>((size_t)n * sg.kc);
    hipLaunchKernelGGL(k_first_cols, dim3(grid_for(n * (int64_t)sg.kc, 256)), dim3(256), 0, s, n, p->k, sg.kc, x0,
                       x0c);
    SFG_LAUNCH_CHECK();
    float *xc = A.alloc<float>((size_t)n * sg.kc);
    const size_t wsc = smooth_workspace_bytes(n, sg.kc, SFG_BF16);
    smooth(&T, sg.kc, sg.tc, 0.5, x0c, SFG_BF16, 1, xc, A.raw(wsc), wsc, s, -1);
    float *nf = A.alloc<float>((size_t)n * 8);
    float *ef = A.alloc<float>((size_t)(nc + 1) * 4);
    check_status(sfg_mpnn_features(&G, &T, xc, sg.kc, nc, cand, u, v, w32, sg.norm, nf, ef, s));
    float *pred = A.alloc<float>(nc + 1);
    const size_t wsf = mpnn_forward_workspace_bytes(n, SFG_BF16);
    check_status(sfg_mpnn_forward(&G, sg.params, nf, nc, cand, u, v, ef, SFG_BF16, pred, A.raw(wsf), wsf, s));
    // the candidates scored exactly: the top cand_frac by prediction
    const int64_t kcand = std::min<int64_t>(nc, (int64_t)std::ceil(p->cand_frac * (double)nc));
    uint8_t *csel = A.alloc<uint8_t>(nc + 1);
    double *tau = A.alloc<double>(1);
    size_t wsel = select_workspace_bytes(nc);
    select_topk(pred, SFG_F32, nc, kcand, csel, tau, A.raw(wsel), wsel, s);
    int32_t *cpos = A.alloc<int32_t>(nc + 1);
    const int64_t ne = compact_ids(csel, 1, nc, cpos, A, s);
    int32_t *cand_e = A.alloc<int32_t>(ne + 1);
    if (ne > 0) {
        hipLaunchKernelGGL(k_take_ids, dim3(grid_for(ne, 256)), dim3(256), 0, s, ne, cpos, cand, cand_e);
        SFG_LAUNCH_CHECK();
    }
    float ms_other = tm.stop();
    // exact scores on the tree embedding, as the plain path computes them
    tm.start();
    const bool f64 = p->storage == SFG_F64;
    const sfg_dtype vt = f64 ? SFG_F64 : SFG_F32;
    const void *wv = f64 ? (const void *)w64 : (const void *)w32;
    sfg_csr H = T;
    if (f64) {
        int32_t *hrp = A.alloc<int32_t>(n + 1), *hcol = A.alloc<int32_t>(2 * n), *heid = A.alloc<int32_t>(2 * n);
        double *hval = A.alloc<double>(2 * n), *hdeg = A.alloc<double>(n + 1);
        build_csr(n, m, u, v, w64, SFG_F64, tree, hrp, hcol, hval, heid, hdeg, ws, wsb, s);
        H = sfg_csr{n, 2 * (n - 1), hrp, hcol, hval, heid, hdeg, SFG_F64};
    }
    void *x = A.raw((size_t)n * p->k * dtype_size(p->storage));
    const size_t wsm = smooth_workspace_bytes(n, p->k, p->storage);
    smooth(&H, p->k, p->sweeps, p->omega, x0, p->storage, 0, x, A.raw(wsm), wsm, s, -1);
    float ms_smooth = tm.stop();
    tm.start();
    void *score = A.raw((ne + 1) * dtype_size(vt));
    edge_scores(x, p->storage, n, p->k, ne, cand_e, u, v, wv, vt, score, vt, s);
    float ms_score = tm.stop();
    tm.start();
    const int64_t ktake = std::min<int64_t>(ne, (int64_t)std::ceil(p->frac * (double)nc));
    uint8_t *sel = A.alloc<uint8_t>(ne + 1);
    wsel = select_workspace_bytes(ne);
    select_topk(score, vt, ne, ktake, sel, tau, A.raw(wsel), wsel, s);
    double tau_h = 0;
    SFG_HIP(hipMemcpyAsync(&tau_h, tau, 8, hipMemcpyDeviceToHost, s));
    SFG_HIP(hipStreamSynchronize(s));
    if (tau_h != tau_h) fail(SFG_ENUMERIC, "sparsify: NaN or negative edge score");
    hipLaunchKernelGGL(k_keep_init, dim3(grid_for(m, 256)), dim3(256), 0, s, m, tree, keep);
    SFG_LAUNCH_CHECK();
    if (ne > 0) {
        hipLaunchKernelGGL(k_keep_add, dim3(grid_for(ne, 256)), dim3(256), 0, s, ne, cand_e, sel, keep);
        SFG_LAUNCH_CHECK();
    }
    float ms_select = tm.stop();
    if (rep) {
        rep->n = n;
        rep->m = m;
        rep->n_cand = nc;
        rep->k_sel = ktake;
        rep->tau = tau_h;
        rep->n_scored = ne;
        rep->ms_smooth = ms_smooth;
        rep->ms_score = ms_score;
        rep->ms_select = ms_select;
        rep->ms_other = ms_other;
    }
    return true;
}

struct KappaEstimator;
KappaEstimator *make_kappa_estimator(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const double *w64,
                                     const uint8_t *tree_marks, int32_t k, DevArena &A, hipStream_t s);
double run_kappa_estimator(KappaEstimator *e, const uint8_t *keep, const sfg_kappa_params &kp, uint64_t seed,
                           uint32_t block, sfg_kappa_report *rep);
void free_kappa_estimator(KappaEstimator *e);
sfg_kappa_params kappa_defaults(const sfg_kappa_params *in);
void check_kappa_params(const sfg_kappa_params &p, int64_t n);

// Sigma-driven stopping: from the tree, batches of ceil(frac * off-tree
// edges) top-scored edges (each scored on the sparsifier grown so far) until
// the estimate of kappa(L_G, L_P) is at most sigma^2 (Eq. 2) or the batch cap
// is reached.  Estimate j starts from random block (seed, 64 + j).
void sigma_sparsify(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const double *w64, const float *w32,
                    const uint8_t *tree, const sfg_params *p, const double *x0, uint8_t *keep, sfg_report *rep,
                    DevArena &A, hipStream_t s) {
    hipLaunchKernelGGL(k_keep_init, dim3(grid_for(m, 256)), dim3(256), 0, s, m, tree, keep);
    SFG_LAUNCH_CHECK();
    const sfg_kappa_params kp = kappa_defaults(&p->est);
    struct Holder {
        KappaEstimator *e;
        ~Holder() { free_kappa_estimator(e); }
    } h{make_kappa_estimator(n, m, u, v, w64, keep, kp.k, A, s)};
    const int32_t cap = p->rounds > 0 ? p->rounds : 16;
    const int64_t n_off = m - (n - 1);
    const int64_t q = (int64_t)std::ceil(p->frac * (double)n_off);
    const double target = p->sigma * p->sigma;
    int32_t j = 0;
    auto estimate = [&]() {
        sfg_kappa_report kr;
        std::memset(&kr, 0, sizeof(kr));
        const double kap = run_kappa_estimator(h.e, keep, kp, p->seed, 64u + (uint32_t)j, &kr);
        if (rep) {
            rep->kappa[j] = kap;
            rep->n_kappa = j + 1;
            rep->kappa_inner_iters += kr.inner_iters;
            rep->ms_kappa += kr.ms;
        }
        ++j;
        return kap;
    };
    double kap = estimate();
    NodeOrder no;   // the number of batches is not known in advance: plan for one
    no.launches = planned_launches(p, 1);
    int32_t r = 0;
    int64_t added = 0;
    while (kap > target && r < cap) {
        const int64_t take = std::min(q, n_off - added);
        if (take <= 0) break;
        score_level(n, m, u, v, w64, w32, keep, p, x0 + (size_t)r * n * p->k, keep,
                    rep ? &rep->level[r] : nullptr, A, s, take, &no);
        added += take;
        ++r;
        kap = estimate();
    }
    if (rep) rep->levels = r;
}

void check_params(const sfg_params *p) {
    SFG_REQUIRE(p, SFG_EINVAL, "sparsify: null params");
    SFG_REQUIRE(p->levels >= 1 && p->levels <= 16, SFG_EINVAL, "sparsify: levels must be in [1, 16]");
    SFG_REQUIRE(p->k >= 1, SFG_EINVAL, "sparsify: k must be >= 1");
    SFG_REQUIRE(p->k <= 64, SFG_EUNSUPPORTED, "sparsify: k > 64 is not supported");
    SFG_REQUIRE(p->sweeps >= 0, SFG_EINVAL, "sparsify: sweeps must be >= 0");
    SFG_REQUIRE(p->omega > 0.0 && p->omega <= 1.0, SFG_EINVAL, "sparsify: omega must be in (0, 1]");
    SFG_REQUIRE(p->frac >= 0.0 && p->frac <= 1.0, SFG_EINVAL, "sparsify: frac must be in [0, 1]");
    SFG_REQUIRE(p->embed == SFG_EMBED_SPARSIFIER || p->embed == SFG_EMBED_GRAPH, SFG_EINVAL, "sparsify: bad embed");
    SFG_REQUIRE(valid_dtype(p->storage), SFG_EINVAL, "sparsify: bad storage dtype");
    SFG_REQUIRE(p->band >= 0.0 && p->band < 1.0, SFG_EINVAL, "sparsify: band must be in [0, 1)");
    SFG_REQUIRE(p->rounds >= 0 && p->rounds <= 16, SFG_EINVAL, "sparsify: rounds must be in [0, 16]");
    SFG_REQUIRE(p->rounds <= 1 || p->levels == 1, SFG_EUNSUPPORTED, "sparsify: rounds > 1 needs levels = 1");
    SFG_REQUIRE(p->smoother == SFG_SMOOTH_JACOBI || p->smoother == SFG_SMOOTH_GAUSS_SEIDEL, SFG_EINVAL,
                "sparsify: bad smoother");
    SFG_REQUIRE(p->smoother == SFG_SMOOTH_JACOBI ||
                    ((p->storage == SFG_F64 || p->storage == SFG_F32) && p->band == 0.0),
                SFG_EUNSUPPORTED, "sparsify: Gauss-Seidel needs F64 or F32 storage and no band");
    SFG_REQUIRE(p->sigma >= 0.0 && p->sigma == p->sigma, SFG_EINVAL, "sparsify: sigma must be >= 0");
    SFG_REQUIRE(p->sigma == 0.0 || p->levels == 1, SFG_EUNSUPPORTED, "sparsify: sigma needs levels = 1");
    SFG_REQUIRE(p->sigma == 0.0 || p->frac > 0.0, SFG_EINVAL, "sparsify: sigma needs frac > 0 (the batch size)");
    if (p->surrogate) {
        const sfg_surrogate &sg = *p->surrogate;
        SFG_REQUIRE(p->levels == 1 && p->rounds <= 1 && p->sigma == 0.0 && p->smoother == SFG_SMOOTH_JACOBI &&
                        p->embed == SFG_EMBED_SPARSIFIER && p->band == 0.0 &&
                        (p->storage == SFG_F64 || p->storage == SFG_F32),
                    SFG_EUNSUPPORTED,
                    "sparsify: a surrogate needs one level, one round, no sigma, Jacobi, the sparsifier embedding, "
                    "no band and F64 or F32 storage");
        SFG_REQUIRE(sg.params && sg.norm, SFG_EINVAL, "sparsify: surrogate parameters or normalisation missing");
        SFG_REQUIRE(sg.kc >= 1 && sg.kc <= p->k && sg.tc >= 0, SFG_EINVAL,
                    "sparsify: surrogate needs 1 <= kc <= k and tc >= 0");
        SFG_REQUIRE(p->cand_frac > 0.0 && p->cand_frac <= 1.0, SFG_EINVAL, "sparsify: cand_frac must be in (0, 1]");
    }
}

}  // namespace sfg

extern "C" size_t sfg_workspace_bytes(int op, int64_t n, int64_t m, int32_t k, sfg_dtype t) {
    switch (op) {
        case SFG_OP_LAPLACIAN_CSR: return sfg::csr_workspace_bytes(n < 1 ? 1 : n, m);
        case SFG_OP_SMOOTH: return sfg::smooth_workspace_bytes(n < 1 ? 1 : n, k < 1 ? 1 : k, t);
        case SFG_OP_SELECT_TOPK: return sfg::select_workspace_bytes(m < 0 ? 0 : m);
        case SFG_OP_AFFINITY: return sfg::affinity_workspace_bytes(n < 1 ? 1 : n, k < 1 ? 1 : k);
        case SFG_OP_COARSEN: return sfg::coarsen_workspace_bytes(n < 1 ? 1 : n, m < 0 ? 0 : m);
        case SFG_OP_MPNN_FORWARD: return sfg::mpnn_forward_workspace_bytes(n < 1 ? 1 : n, t);
        case SFG_OP_MPNN_TRAIN: return sfg::mpnn_train_workspace_bytes(n < 1 ? 1 : n, m < 1 ? 1 : m);
        case SFG_OP_COLOR: return sfg::color_workspace_bytes(n < 1 ? 1 : n);
        case SFG_OP_TREE_ORDER: return sfg::tree_order_workspace_bytes(n < 1 ? 1 : n, m < 0 ? 0 : m);
        case SFG_OP_TREE_SOLVE: return sfg::tree_solve_workspace_bytes(n < 1 ? 1 : n, k < 1 ? 1 : k);
        case SFG_OP_CSR_SELECT: return sfg::csr_select_workspace_bytes(n, m);
        case SFG_OP_MPNN_NORM: return 512;
        case SFG_OP_SMOOTH_ORDERED: return sfg::smooth_ordered_workspace_bytes(n < 1 ? 1 : n, k < 1 ? 1 : k, t);
        default: return 0;
    }
}

extern "C" sfg_status sfg_spanning_tree(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w,
                                        sfg_dtype wt, const uint8_t *allowed, uint8_t *in_tree, int64_t *n_comp,
                                        void *stream) {
    return sfg::guard([&] {
        SFG_REQUIRE(n >= 1 && m >= 0, SFG_EINVAL, "spanning_tree: bad sizes");
        SFG_REQUIRE(wt == SFG_F64 || wt == SFG_F32, SFG_EINVAL, "spanning_tree: weights must be F64 or F32");
        SFG_REQUIRE(n_comp, SFG_EINVAL, "spanning_tree: n_comp is required");
        sfg::DevArena A(sfg::as_stream(stream));
        *n_comp = sfg::spanning_tree_gpu(n, m, u, v, w, wt, allowed, in_tree, A, sfg::as_stream(stream));
        A.finish();
    });
}

extern "C" sfg_status sfg_sparsify(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w,
                                   sfg_dtype wt, const sfg_params *p, const double *x0, uint8_t *keep,
                                   sfg_report *rep, void *stream) {
    return sfg::guard([&] {
        hipStream_t s = sfg::as_stream(stream);
        sfg::check_params(p);
        SFG_REQUIRE(keep, SFG_EINVAL, "sparsify: null pointer");
        if (p->sigma > 0.0) sfg::check_kappa_params(sfg::kappa_defaults(&p->est), n);
        sfg::DevArena A(s);
        sfg::validate_edges(n, m, u, v, w, wt, A, s);
        if (!x0) {   // draw the blocks on the device: one per level or per round
            const int32_t nb = p->levels > 1   ? p->levels
                               : p->sigma > 0.0 ? (p->rounds > 0 ? p->rounds : 16)
                                                : (p->rounds > 1 ? p->rounds : 1);
            double *gen = A.alloc<double>((size_t)nb * n * p->k);
            for (int32_t b = 0; b < nb; ++b)
                sfg::random_block(n, p->k, p->seed, (uint32_t)b, gen + (size_t)b * n * p->k, s);
            x0 = gen;
        }
        if (rep) std::memset(rep, 0, sizeof(*rep));
        if (p->levels == 1)
            sfg::single_level_sparsify(n, m, u, v, w, wt, p, x0, keep, rep, A, s);
        else
            sfg::multilevel_sparsify(n, m, u, v, w, wt, p, x0, keep, rep, A, s);
        A.finish();
    });
}
