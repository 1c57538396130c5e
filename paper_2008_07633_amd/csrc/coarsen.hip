// Spectral coarsening (Sec. 3.2-3.3 of the paper) and the multilevel
// sparsifier driver (Alg. 1).
//
// Aggregation (the paper leaves the rule open): every node points to the
// neighbour with the largest key (affinity, weight, -id).  With this total
// order a pointer cycle longer than two is impossible, so each component of
// the pointer graph is a tree hanging off one mutual pair; rooting it at the
// pair's smaller node and pointer-jumping finds the components in O(log n)
// passes.  Aggregates are numbered by their smallest member.
//
// Galerkin coarse graph (Eqs. 3-5): the fine edges between two different
// aggregates are keyed by (min aggregate, max aggregate), radix-sorted
// stably (so each key's edges stay in ascending edge id), and each run is
// reduced by one thread in that order: the FP64 sum of the weights is the
// coarse weight, the heaviest edge (first on ties) is the representative the
// backward mapping keeps.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"

namespace sfg {

size_t radix_scratch_bytes(int64_t n);
void radix_sort_pairs(uint64_t *keys, int32_t *vals, int64_t n, const int *shifts, int nshift, void *scratch,
                      hipStream_t s);
size_t csr_workspace_bytes(int64_t n, int64_t m);
void build_csr(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
               const uint8_t *mask, int32_t *rowptr, int32_t *col, void *val, int32_t *eid, void *deg, void *ws,
               size_t ws_bytes, hipStream_t s);
size_t smooth_workspace_bytes(int64_t n, int32_t k, sfg_dtype storage);
void smooth(const sfg_csr *H, int32_t k, int32_t sweeps, double omega, const double *x0, sfg_dtype storage,
            int32_t final_f32, void *x, void *ws, size_t ws_bytes, hipStream_t s, int32_t max_row);
void max_row_length(const sfg_csr *H, int32_t *out, hipStream_t s);
size_t affinity_workspace_bytes(int64_t n, int32_t k);
void affinity(const void *x, sfg_dtype xt, int64_t n, int32_t k, int64_t m, const int32_t *u, const int32_t *v,
              void *aff, sfg_dtype at, void *ws, size_t ws_bytes, hipStream_t s);
void convert_weights(const void *w, sfg_dtype wt, sfg_dtype want, int64_t m, void *out, hipStream_t s);
int64_t spanning_tree_gpu(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
                          const uint8_t *allowed, uint8_t *in_tree, DevArena &A, hipStream_t s);
void level_node_order(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const double *w64, const sfg_csr *G,
                      const uint8_t *tree, int32_t k, sfg_dtype storage, NodeOrder *no, DevArena &A, hipStream_t s);
sfg_csr relabel_csr(const sfg_csr *H, const int32_t *order, const int32_t *inv, DevArena &A, hipStream_t s);
void gather_block(int64_t n, int32_t k, const int32_t *order, const double *src, double *dst, hipStream_t s);
size_t smooth_ordered_workspace_bytes(int64_t n, int32_t k, sfg_dtype storage);
int smooth_ordered(const sfg_csr *H, const int32_t *order, int32_t k, int32_t sweeps, double omega,
                   const double *x0, sfg_dtype storage, int32_t final_f32, void *x, void *ws, size_t ws_bytes,
                   hipStream_t s, int32_t max_row);
void score_level(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const double *w64, const float *w32,
                 const uint8_t *base, const sfg_params *p, const double *x0, uint8_t *keep, sfg_level_report *rep,
                 DevArena &A, hipStream_t s, int64_t k_take, NodeOrder *no);

namespace {

// ------------------------------------------------------------------ aggregation

// key order of a neighbour entry: larger affinity, then larger weight, then smaller column
template <typename TA, typename TW>
__device__ __forceinline__ bool key_better(TA a, TW w, int32_t c, TA ba, TW bw, int32_t bc) {
    return a > ba || (a == ba && (w > bw || (w == bw && c < bc)));
}

constexpr int32_t kPtrLong = 256;   // rows above this length: one workgroup each

template <typename TA, typename TW>
__global__ void k_pointer(int64_t n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                          const TW *__restrict__ val, const int32_t *__restrict__ eid, const TA *__restrict__ aff,
                          int32_t *ptr, int32_t *long_rows, int32_t *long_cnt) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int32_t j0 = rowptr[p], j1 = rowptr[p + 1];
    if (j0 == j1) {
        ptr[p] = (int32_t)p;
        return;
    }
    if (j1 - j0 > kPtrLong) {
        long_rows[atomicAdd(long_cnt, 1)] = (int32_t)p;
        return;
    }
    int32_t best = j0;
    TA ba = aff[eid[j0]];
    TW bw = val[j0];
    for (int32_t j = j0 + 1; j < j1; ++j) {
        const TA a = aff[eid[j]];
        const TW w = val[j];
        // columns ascend, so on a full tie the earlier (smaller) neighbour stays
        if (a > ba || (a == ba && w > bw)) {
            best = j;
            ba = a;
            bw = w;
        }
    }
    ptr[p] = col[best];
}

template <typename TA, typename TW>
__global__ __launch_bounds__(256) void k_pointer_long(const int32_t *__restrict__ rowptr,
                                                      const int32_t *__restrict__ col, const TW *__restrict__ val,
                                                      const int32_t *__restrict__ eid, const TA *__restrict__ aff,
                                                      int32_t *ptr, const int32_t *__restrict__ long_rows,
                                                      const int32_t *__restrict__ long_cnt) {
    __shared__ TA sa[256];
    __shared__ TW sw[256];
    __shared__ int32_t sc[256];
    const int t = threadIdx.x;
    const int32_t cnt = *long_cnt;
    for (int32_t r = blockIdx.x; r < cnt; r += gridDim.x) {
        const int32_t p = long_rows[r];
        const int32_t j0 = rowptr[p], j1 = rowptr[p + 1];
        TA ba = TA(-1);
        TW bw = TW(0);
        int32_t bc = 0x7fffffff;
        for (int32_t j = j0 + t; j < j1; j += 256) {
            const TA a = aff[eid[j]];
            const TW w = val[j];
            const int32_t c = col[j];
            if (bc == 0x7fffffff || key_better(a, w, c, ba, bw, bc)) {
                ba = a;
                bw = w;
                bc = c;
            }
        }
        sa[t] = ba;
        sw[t] = bw;
        sc[t] = bc;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if (t < st && sc[t + st] != 0x7fffffff &&
                (sc[t] == 0x7fffffff || key_better(sa[t + st], sw[t + st], sc[t + st], sa[t], sw[t], sc[t]))) {
                sa[t] = sa[t + st];
                sw[t] = sw[t + st];
                sc[t] = sc[t + st];
            }
            __syncthreads();
        }
        if (t == 0) ptr[p] = sc[0];
        __syncthreads();
    }
}

__global__ void k_parent_init(int64_t n, const int32_t *__restrict__ ptr, int32_t *par) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int32_t q = ptr[p];
    // the smaller node of a mutual pair (or a node pointing to itself) is a root
    par[p] = (q == p || (ptr[q] == p && p < q)) ? (int32_t)p : q;
}

__global__ void k_jump(int64_t n, int32_t *par, int32_t *changed) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int32_t a = par[p];
    const int32_t b = par[a];
    if (a != b) {
        par[p] = b;
        *changed = 1;
    }
}

__global__ void k_minid(int64_t n, const int32_t *__restrict__ par, int32_t *minid) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) atomicMin(&minid[par[p]], (int32_t)p);
}

__global__ void k_minflag(int64_t n, const int32_t *__restrict__ par, const int32_t *__restrict__ minid,
                          int32_t *flag) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) flag[p] = minid[par[p]] == p ? 1 : 0;
}

__global__ void k_agg_assign(int64_t n, const int32_t *__restrict__ par, const int32_t *__restrict__ minid,
                             const int32_t *__restrict__ rank, int32_t *agg) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) agg[p] = rank[minid[par[p]]];
}

// ------------------------------------------------------------------ Galerkin

__global__ void k_inter_flag(int64_t m, const int32_t *__restrict__ u, const int32_t *__restrict__ v,
                             const int32_t *__restrict__ agg, int32_t *flag) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) flag[e] = agg[u[e]] != agg[v[e]] ? 1 : 0;
}

__global__ void k_inter_keys(int64_t m, const int32_t *__restrict__ u, const int32_t *__restrict__ v,
                             const int32_t *__restrict__ agg, const int32_t *__restrict__ flag,
                             const int32_t *__restrict__ pos, uint64_t *keys, int32_t *vals) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m || !flag[e]) return;
    const uint32_t I = (uint32_t)agg[u[e]], J = (uint32_t)agg[v[e]];
    const uint32_t lo = I < J ? I : J, hi = I < J ? J : I;
    keys[pos[e]] = ((uint64_t)lo << 32) | hi;
    vals[pos[e]] = (int32_t)e;
}

__global__ void k_seg_flag(int64_t mi, const uint64_t *__restrict__ keys, int32_t *flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < mi) flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

__global__ void k_seg_start(int64_t mi, const int32_t *__restrict__ flag, const int32_t *__restrict__ pos,
                            int32_t *start) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < mi && flag[i]) start[pos[i]] = (int32_t)i;
}

template <typename TW>
__global__ void k_seg_reduce(int64_t mc, int64_t mi, const int32_t *__restrict__ start,
                             const uint64_t *__restrict__ keys, const int32_t *__restrict__ eids,
                             const TW *__restrict__ w, int32_t *cu, int32_t *cv, TW *cw, int32_t *crep) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= mc) return;
    const int32_t i0 = start[c];
    const int32_t i1 = (c + 1 < mc) ? start[c + 1] : (int32_t)mi;
    double sum = 0.0;
    int32_t rep = eids[i0];
    double wrep = (double)w[rep];
    for (int32_t i = i0; i < i1; ++i) {
        const int32_t e = eids[i];
        const double we = (double)w[e];
        sum = sum + we;
        if (we > wrep) {
            wrep = we;
            rep = e;
        }
    }
    const uint64_t key = keys[i0];
    cu[c] = (int32_t)(key >> 32);
    cv[c] = (int32_t)(key & 0xffffffffu);
    cw[c] = (TW)sum;
    crep[c] = rep;
}

struct CoarsenPlan {
    int32_t *ptr, *par, *minid, *flag, *rank, *changed, *eflag, *epos, *eids, *sflag, *spos, *sstart, *scan,
        *long_rows, *long_cnt;
    uint64_t *keys;
    void *radix;
};

CoarsenPlan plan_coarsen(Carver &c, int64_t n, int64_t m) {
    CoarsenPlan p;
    p.ptr = c.take<int32_t>(n + 1);
    p.par = c.take<int32_t>(n + 1);
    p.minid = c.take<int32_t>(n + 1);
    p.flag = c.take<int32_t>(n + 1);
    p.rank = c.take<int32_t>(n + 1);
    p.changed = c.take<int32_t>(1);
    p.long_rows = c.take<int32_t>(n + 1);
    p.long_cnt = c.take<int32_t>(1);
    p.eflag = c.take<int32_t>(m + 1);
    p.epos = c.take<int32_t>(m + 1);
    p.eids = c.take<int32_t>(m + 1);
    p.sflag = c.take<int32_t>(m + 1);
    p.spos = c.take<int32_t>(m + 1);
    p.sstart = c.take<int32_t>(m + 1);
    p.scan = c.take<int32_t>(scan_scratch_ints((n > m ? n : m) + 1));
    p.keys = c.take<uint64_t>(m + 1);
    p.radix = c.take<char>(radix_scratch_bytes(m));
    return p;
}

int bits_for(int64_t x) {
    int b = 0;
    while (b < 63 && (int64_t(1) << b) <= x) ++b;
    return b;
}

int32_t read_i32(const int32_t *p, hipStream_t s) {
    int32_t h = 0;
    SFG_HIP(hipMemcpyAsync(&h, p, sizeof(h), hipMemcpyDeviceToHost, s));
    SFG_HIP(hipStreamSynchronize(s));
    return h;
}

}  // namespace

size_t coarsen_workspace_bytes(int64_t n, int64_t m) {
    Carver c(nullptr);
    plan_coarsen(c, n, m);
    return c.used + 256;
}

void coarsen(const sfg_csr *G, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
             const void *aff, sfg_dtype at, int32_t *agg, int64_t *n_coarse, int64_t *m_coarse, int32_t *cu,
             int32_t *cv, void *cw, int32_t *crep, void *ws, size_t ws_bytes, hipStream_t s) {
    const int64_t n = G ? G->n : 0;
    SFG_REQUIRE(G && G->rowptr && G->col && G->val && G->eid && n >= 1 && m >= 0, SFG_EINVAL,
                "coarsen: graph CSR with edge ids required");
    SFG_REQUIRE(G->nnz == 2 * m, SFG_EINVAL, "coarsen: CSR must hold every edge of the list");
    SFG_REQUIRE(n_coarse && m_coarse && agg && (m == 0 || (u && v && w && aff && cu && cv && cw && crep)),
                SFG_EINVAL, "coarsen: null pointer");
    SFG_REQUIRE(wt == SFG_F64 || wt == SFG_F32, SFG_EINVAL, "coarsen: weights must be F64 or F32");
    SFG_REQUIRE(G->vt == SFG_F64 || G->vt == SFG_F32, SFG_EINVAL, "coarsen: CSR weights must be F64 or F32");
    SFG_REQUIRE(at == SFG_F64 || at == SFG_F32, SFG_EINVAL, "coarsen: affinities must be F64 or F32");
    SFG_REQUIRE(ws_bytes >= coarsen_workspace_bytes(n, m), SFG_EWORKSPACE, "coarsen: workspace too small");
    Carver c(ws);
    CoarsenPlan p = plan_coarsen(c, n, m);
    const dim3 gn(grid_for(n, 256)), gm(grid_for(m, 256)), b(256);
    // pointers to the highest-key neighbour (long rows: one workgroup each)
    fill_i32(p.long_cnt, 1, 0, s);
    if (at == SFG_F64 && G->vt == SFG_F64) {
        hipLaunchKernelGGL((k_pointer<double, double>), gn, b, 0, s, n, G->rowptr, G->col, (const double *)G->val,
                           G->eid, (const double *)aff, p.ptr, p.long_rows, p.long_cnt);
        SFG_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_pointer_long<double, double>), dim3(512), b, 0, s, G->rowptr, G->col,
                           (const double *)G->val, G->eid, (const double *)aff, p.ptr, p.long_rows, p.long_cnt);
    } else if (at == SFG_F64) {
        hipLaunchKernelGGL((k_pointer<double, float>), gn, b, 0, s, n, G->rowptr, G->col, (const float *)G->val,
                           G->eid, (const double *)aff, p.ptr, p.long_rows, p.long_cnt);
        SFG_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_pointer_long<double, float>), dim3(512), b, 0, s, G->rowptr, G->col,
                           (const float *)G->val, G->eid, (const double *)aff, p.ptr, p.long_rows, p.long_cnt);
    } else if (G->vt == SFG_F64) {
        hipLaunchKernelGGL((k_pointer<float, double>), gn, b, 0, s, n, G->rowptr, G->col, (const double *)G->val,
                           G->eid, (const float *)aff, p.ptr, p.long_rows, p.long_cnt);
        SFG_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_pointer_long<float, double>), dim3(512), b, 0, s, G->rowptr, G->col,
                           (const double *)G->val, G->eid, (const float *)aff, p.ptr, p.long_rows, p.long_cnt);
    } else {
        hipLaunchKernelGGL((k_pointer<float, float>), gn, b, 0, s, n, G->rowptr, G->col, (const float *)G->val,
                           G->eid, (const float *)aff, p.ptr, p.long_rows, p.long_cnt);
        SFG_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_pointer_long<float, float>), dim3(512), b, 0, s, G->rowptr, G->col,
                           (const float *)G->val, G->eid, (const float *)aff, p.ptr, p.long_rows, p.long_cnt);
    }
    SFG_LAUNCH_CHECK();
    // components of the pointer graph
    hipLaunchKernelGGL(k_parent_init, gn, b, 0, s, n, p.ptr, p.par);
    SFG_LAUNCH_CHECK();
    for (int it = 0; it < 64; ++it) {
        fill_i32(p.changed, 1, 0, s);
        hipLaunchKernelGGL(k_jump, gn, b, 0, s, n, p.par, p.changed);
        SFG_LAUNCH_CHECK();
        if (read_i32(p.changed, s) == 0) break;
        SFG_REQUIRE(it < 63, SFG_EHIP, "coarsen: pointer jumping did not converge");
    }
    fill_i32(p.minid, n, 0x7fffffff, s);
    hipLaunchKernelGGL(k_minid, gn, b, 0, s, n, p.par, p.minid);
    SFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_minflag, gn, b, 0, s, n, p.par, p.minid, p.flag);
    SFG_LAUNCH_CHECK();
    exclusive_scan_i32(p.flag, p.rank, n, p.scan, s);
    hipLaunchKernelGGL(k_agg_assign, gn, b, 0, s, n, p.par, p.minid, p.rank, agg);
    SFG_LAUNCH_CHECK();
    const int64_t nc = read_i32(p.rank + n, s);
    *n_coarse = nc;
    *m_coarse = 0;
    if (m == 0) return;
    // inter-aggregate edges, keyed and sorted
    hipLaunchKernelGGL(k_inter_flag, gm, b, 0, s, m, u, v, agg, p.eflag);
    SFG_LAUNCH_CHECK();
    exclusive_scan_i32(p.eflag, p.epos, m, p.scan, s);
    hipLaunchKernelGGL(k_inter_keys, gm, b, 0, s, m, u, v, agg, p.eflag, p.epos, p.keys, p.eids);
    SFG_LAUNCH_CHECK();
    const int64_t mi = read_i32(p.epos + m, s);
    if (mi == 0) return;
    const int kb = bits_for(nc > 1 ? nc - 1 : 1);
    int shifts[16], ns = 0;
    for (int sh = 0; sh < kb; sh += 8) shifts[ns++] = sh;         // larger aggregate id
    for (int sh = 0; sh < kb; sh += 8) shifts[ns++] = 32 + sh;    // smaller aggregate id
    radix_sort_pairs(p.keys, p.eids, mi, shifts, ns, p.radix, s);
    // runs of equal keys
    const dim3 gi(grid_for(mi, 256));
    hipLaunchKernelGGL(k_seg_flag, gi, b, 0, s, mi, p.keys, p.sflag);
    SFG_LAUNCH_CHECK();
    exclusive_scan_i32(p.sflag, p.spos, mi, p.scan, s);
    hipLaunchKernelGGL(k_seg_start, gi, b, 0, s, mi, p.sflag, p.spos, p.sstart);
    SFG_LAUNCH_CHECK();
    const int64_t mc = read_i32(p.spos + mi, s);
    const dim3 gc(grid_for(mc, 256));
    if (wt == SFG_F64)
        hipLaunchKernelGGL(k_seg_reduce<double>, gc, b, 0, s, mc, mi, p.sstart, p.keys, p.eids, (const double *)w, cu,
                           cv, (double *)cw, crep);
    else
        hipLaunchKernelGGL(k_seg_reduce<float>, gc, b, 0, s, mc, mi, p.sstart, p.keys, p.eids, (const float *)w, cu,
                           cv, (float *)cw, crep);
    SFG_LAUNCH_CHECK();
    SFG_HIP(hipStreamSynchronize(s));
    *m_coarse = mc;
}

// ------------------------------------------------------------------ multilevel driver (Alg. 1)

namespace {

__global__ void k_intra_mask(int64_t m, const int32_t *__restrict__ u, const int32_t *__restrict__ v,
                             const int32_t *__restrict__ agg, uint8_t *mask) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) mask[e] = agg[u[e]] == agg[v[e]] ? 1 : 0;
}

__global__ void k_map_inter(int64_t mc, const uint8_t *__restrict__ pc, const int32_t *__restrict__ crep,
                            uint8_t *base) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < mc && pc[c]) base[crep[c]] = 1;
}

struct LevelGraph {
    int64_t n = 0, m = 0;
    int32_t *u = nullptr, *v = nullptr;
    double *w64 = nullptr;
    float *w32 = nullptr;
    int32_t *agg = nullptr;     // aggregate of each node (towards the next level)
    int32_t *crep = nullptr;    // per edge of the NEXT level: representative edge of this level
};

}  // namespace

void multilevel_sparsify(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
                         const sfg_params *p, const double *x0, uint8_t *keep, sfg_report *rep, DevArena &A,
                         hipStream_t s) {
    const bool f64 = p->storage == SFG_F64;
    const sfg_dtype vt = f64 ? SFG_F64 : SFG_F32;
    const int L = p->levels;
    std::vector<LevelGraph> lv(L);
    lv[0].n = n;
    lv[0].m = m;
    lv[0].u = const_cast<int32_t *>(u);
    lv[0].v = const_cast<int32_t *>(v);
    lv[0].w64 = A.alloc<double>(m + 1);
    convert_weights(w, wt, SFG_F64, m, lv[0].w64, s);
    if (!f64) {
        lv[0].w32 = A.alloc<float>(m + 1);
        convert_weights(w, wt, SFG_F32, m, lv[0].w32, s);
    }
    uint8_t *tree0 = A.alloc<uint8_t>(m + 1);
    {
        const int64_t comps = spanning_tree_gpu(n, m, u, v, lv[0].w64, SFG_F64, nullptr, tree0, A, s);
        if (comps != 1) fail(SFG_ENOTCONN, "sparsify: graph has " + std::to_string(comps) + " components");
    }
    // node numbering of each level's sweeps (decided when the level is coarsened, or scored if it is the last)
    std::vector<NodeOrder> ord(L);
    // ---- coarsening: G_0 .. G_{L-1}
    int built = 1;
    for (int l = 0; l + 1 < L; ++l) {
        LevelGraph &F = lv[l];
        if (F.n <= 2 || F.m == 0) break;
        const void *wf = f64 ? (const void *)F.w64 : (const void *)F.w32;
        int32_t *rowptr = A.alloc<int32_t>(F.n + 1);
        int32_t *col = A.alloc<int32_t>(2 * F.m + 1);
        int32_t *eid = A.alloc<int32_t>(2 * F.m + 1);
        void *val = A.raw((2 * F.m + 1) * dtype_size(vt));
        void *deg = A.raw(F.n * dtype_size(vt));
        const size_t wsc = csr_workspace_bytes(F.n, F.m);
        build_csr(F.n, F.m, F.u, F.v, wf, vt, nullptr, rowptr, col, val, eid, deg, A.raw(wsc), wsc, s);
        sfg_csr G{F.n, 2 * F.m, rowptr, col, val, eid, deg, vt};
        void *x = A.raw((size_t)F.n * p->k * dtype_size(vt));
        const size_t wss = smooth_workspace_bytes(F.n, p->k, vt);
        int32_t max_row = -1;
        if (f64) {
            // FP64 sums hub rows through LDS only where they are known to exist
            int32_t *mr = A.alloc<int32_t>(1);
            max_row_length(&G, mr, s);
            SFG_HIP(hipMemcpyAsync(&max_row, mr, 4, hipMemcpyDeviceToHost, s));
            SFG_HIP(hipStreamSynchronize(s));
        }
        // the sweeps on G_l, in the level's node numbering; affinities per edge id, numbering-free
        NodeOrder &no = ord[l];
        level_node_order(F.n, F.m, F.u, F.v, F.w64, &G, l == 0 ? tree0 : nullptr, p->k, vt, &no, A, s);
        const double *xl = x0 + (size_t)l * n * p->k;
        const int32_t *au = F.u, *av = F.v;
        sfg_csr Gs = G;
        if (no.use) {
            Gs = relabel_csr(&G, no.order, no.inv, A, s);
            double *xg = A.alloc<double>((size_t)F.n * p->k + 1);
            gather_block(F.n, p->k, no.order, xl, xg, s);
            xl = xg;
            au = no.u;
            av = no.v;
        }
        if (no.use) {
            // in the tree's preorder the sweeps may take several per pass (where they pay; same bits)
            const size_t wso = smooth_ordered_workspace_bytes(F.n, p->k, vt);
            smooth_ordered(&Gs, nullptr, p->k, p->sweeps, p->omega, xl, vt, 0, x, A.raw(wso), wso, s, max_row);
        } else {
            smooth(&Gs, p->k, p->sweeps, p->omega, xl, vt, 0, x, A.raw(wss), wss, s, max_row);
        }
        void *aff = A.raw((F.m + 1) * dtype_size(vt));
        const size_t wsa = affinity_workspace_bytes(F.n, p->k);
        affinity(x, vt, F.n, p->k, F.m, au, av, aff, vt, A.raw(wsa), wsa, s);
        LevelGraph &C = lv[l + 1];
        F.agg = A.alloc<int32_t>(F.n + 1);
        C.u = A.alloc<int32_t>(F.m + 1);
        C.v = A.alloc<int32_t>(F.m + 1);
        C.w64 = A.alloc<double>(F.m + 1);
        F.crep = A.alloc<int32_t>(F.m + 1);
        // the pointer step reads the CSR in the working precision; the coarse
        // weights are always FP64 sums of the FP64 fine weights
        int64_t nc = 0, mc = 0;
        const size_t wsg = coarsen_workspace_bytes(F.n, F.m);
        coarsen(&G, F.m, F.u, F.v, F.w64, SFG_F64, aff, vt, F.agg, &nc, &mc, C.u, C.v, C.w64, F.crep, A.raw(wsg),
                wsg, s);
        C.n = nc;
        C.m = mc;
        if (!f64) {
            C.w32 = A.alloc<float>(mc + 1);
            convert_weights(C.w64, SFG_F64, SFG_F32, mc, C.w32, s);
        }
        built = l + 2;
        if (nc == F.n) break;   // no progress (cannot happen for a connected graph with n >= 2)
    }
    const int lf = built - 1;
    // ---- backward: P_lf = G_lf, then map and add per level
    uint8_t *P = A.alloc<uint8_t>(lv[lf].m + 1);
    fill_u8(P, lv[lf].m, 1, s);
    if (rep) rep->levels = built;
    if (lf == 0) {
        // a single level is Alg. 1 with nothing to coarsen: the whole graph
        fill_u8(keep, m, 1, s);
        return;
    }
    for (int l = lf; l >= 1; --l) {
        LevelGraph &F = lv[l - 1], &C = lv[l];
        uint8_t *intra = A.alloc<uint8_t>(F.m + 1);
        hipLaunchKernelGGL(k_intra_mask, dim3(grid_for(F.m, 256)), dim3(256), 0, s, F.m, F.u, F.v, F.agg, intra);
        SFG_LAUNCH_CHECK();
        uint8_t *base = A.alloc<uint8_t>(F.m + 1);
        spanning_tree_gpu(F.n, F.m, F.u, F.v, F.w64, SFG_F64, intra, base, A, s);   // per-aggregate trees
        if (C.m > 0) {
            hipLaunchKernelGGL(k_map_inter, dim3(grid_for(C.m, 256)), dim3(256), 0, s, C.m, P, F.crep, base);
            SFG_LAUNCH_CHECK();
        }
        uint8_t *kp = (l == 1) ? keep : A.alloc<uint8_t>(F.m + 1);
        sfg_level_report *lr = rep ? &rep->level[l - 1] : nullptr;
        score_level(F.n, F.m, F.u, F.v, F.w64, F.w32, base, p, x0 + (size_t)(l - 1) * n * p->k, kp, lr, A, s, -1,
                    &ord[l - 1]);
        P = kp;
    }
}

}  // namespace sfg

extern "C" sfg_status sfg_coarsen(const sfg_csr *G, int64_t m, const int32_t *u, const int32_t *v, const void *w,
                                  sfg_dtype wt, const void *aff, sfg_dtype at, int32_t *agg, int64_t *n_coarse,
                                  int64_t *m_coarse, int32_t *cu, int32_t *cv, void *cw, int32_t *crep, void *ws,
                                  size_t ws_bytes, void *stream) {
    return sfg::guard([&] {
        sfg::coarsen(G, m, u, v, w, wt, aff, at, agg, n_coarse, m_coarse, cu, cv, cw, crep, ws, ws_bytes,
                     sfg::as_stream(stream));
    });
}
