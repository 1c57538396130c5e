// Precision form: candidates scored from a reduced-precision embedding are
// split around the reduced-precision threshold tau~ (the k_sel-th largest):
//   A = { s~ > (1+m) tau~ }   accepted outright,
//   B = { |s~ - tau~| <= m tau~ }   re-scored exactly in FP64,
// and the final set is A plus the best k_sel - |A| of B by FP64 score (ties:
// lower edge id).  If k_sel - |A| falls outside [0, |B|] the margin m doubles.
//
// The FP64 scores of B are recomputed only where they depend: a score after
// T sweeps depends on the T-hop neighbourhood of its endpoints, so a
// multi-source BFS (capped at T hops) orders the rows by distance and sweep
// t recomputes the rows within T - t hops, with the same per-row arithmetic
// as the full FP64 pass.  When the cone holds more than a quarter of the
// full pass's row updates (T = 20 on meshes and kNN graphs reaches most of
// the graph), the full FP64 smoothing runs instead: it sweeps rows in node
// order, several times faster per row than the distance-ordered cone, and
// gives the same bits.  predicted_cone_share makes that call before any
// smoothing, from a sample standing in for the band, so that the driver can
// skip the reduced-precision pass when the full FP64 pass is coming anyway.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"

namespace sfg {

int64_t compact_ids(const uint8_t *mask, uint8_t want, int64_t m, int32_t *out, DevArena &A, hipStream_t s);
void edge_scores(const void *x, sfg_dtype xt, int64_t n, int32_t k, int64_t ne, const int32_t *cand,
                 const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt, void *score, sfg_dtype st,
                 hipStream_t s);
size_t select_workspace_bytes(int64_t ne);
void select_topk(const void *score, sfg_dtype st, int64_t ne, int64_t k, uint8_t *sel, double *tau, void *ws,
                 size_t ws_bytes, hipStream_t s);
size_t cone_partial_bytes(int64_t n, int32_t k);
double *smooth_cone_f64(const sfg_csr *H, int32_t k, int32_t sweeps, double omega, const double *x0,
                        const int32_t *rows_by_dist, const int64_t *active, double *buf0, double *buf1,
                        void *partial_ws, double *mean, hipStream_t s);
size_t smooth_workspace_bytes(int64_t n, int32_t k, sfg_dtype storage);
void smooth(const sfg_csr *H, int32_t k, int32_t sweeps, double omega, const double *x0, sfg_dtype storage,
            int32_t final_f32, void *x, void *ws, size_t ws_bytes, hipStream_t s, int32_t max_row);

namespace {

// 0 = below the band, 1 = in the band, 2 = above it
__global__ void k_band_class(int64_t nc, const float *__restrict__ s, double lo, double hi, uint8_t *cls) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc) return;
    const double x = (double)s[i];
    cls[i] = x > hi ? 2 : (x >= lo ? 1 : 0);
}

__global__ void k_count_cls(int64_t nc, const uint8_t *__restrict__ cls, unsigned long long *cnt) {
    __shared__ unsigned int c1, c2;
    if (threadIdx.x == 0) c1 = c2 = 0;
    __syncthreads();
    unsigned int a = 0, b = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += (int64_t)gridDim.x * blockDim.x) {
        a += cls[i] == 1;
        b += cls[i] == 2;
    }
    atomicAdd(&c1, a);
    atomicAdd(&c2, b);
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&cnt[0], (unsigned long long)c1);
        atomicAdd(&cnt[1], (unsigned long long)c2);
    }
}

__global__ void k_zero_u64(unsigned long long *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

__global__ void k_gather_ids(int64_t nb, const int32_t *__restrict__ pos, const int32_t *__restrict__ cand,
                             int32_t *eids) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb) eids[i] = cand[pos[i]];
}

// Multi-source BFS capped at `cap` hops, frontier by frontier.  rows[] receives
// the reached rows grouped by distance (distance 0 first) and cnt[d] the size
// of group d; a row joins the group of the level that first claims it
// (compare-and-swap of its distance from cap + 1), so each row appears once.
// Appends are aggregated per wavefront: one atomic per wave and level step.
constexpr int kBfsBlocks = 2048;

__device__ __forceinline__ int32_t wave_max_i32(int32_t x) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) x = max(x, __shfl_xor(x, d, kWave));
    return x;
}

// Lane `mine` appends q to rows[base + slot] with slot from the group counter.
__device__ __forceinline__ void wave_append(bool mine, int32_t q, int32_t *counter, int32_t base, int32_t *rows) {
    const unsigned long long ball = __ballot(mine);
    if (!ball) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int leader = __ffsll((long long)ball) - 1;
    int32_t at = 0;
    if (lane == leader) at = atomicAdd(counter, __popcll(ball));
    at = __shfl(at, leader, kWave);
    if (mine) rows[base + at + __popcll(ball & ((1ull << lane) - 1ull))] = q;
}

__global__ __launch_bounds__(256) void k_bfs_seed(int64_t nseeds, const int32_t *__restrict__ eids,
                                                  const int32_t *__restrict__ u, const int32_t *__restrict__ v,
                                                  int32_t unreached, int32_t *dist, int32_t *cnt, int32_t *rows) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t b = wave * kWave; b < nseeds; b += nwaves * kWave) {    // uniform per wave
        const int64_t i = b + lane;
        const bool live = i < nseeds;
        const int32_t e = live ? eids[i] : 0;
#pragma unroll
        for (int end = 0; end < 2; ++end) {
            const int32_t x = live ? (end ? v[e] : u[e]) : 0;
            const bool mine = live && atomicCAS(&dist[x], unreached, 0) == unreached;
            wave_append(mine, x, &cnt[0], 0, rows);
        }
    }
}

// Expands group `level` (rows[begin, end), begin = sum of the earlier groups) into group level + 1.  With
// stop > 0 it does nothing once sum_{d <= level} cnt[d] (cap - d) exceeds stop (every workgroup reads the same
// finished counts, so all agree): the rows found so far already weigh more than the caller's limit.
__global__ __launch_bounds__(256) void k_bfs_expand(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                                    int32_t level, int32_t unreached, int32_t *dist, int32_t *cnt,
                                                    int32_t *rows, double stop) {
    int32_t begin = 0;
    double weight = 0.0;
    for (int32_t d = 0; d < level; ++d) {
        begin += cnt[d];
        weight += (double)cnt[d] * (double)(unreached - 1 - d);
    }
    if (stop > 0.0 && weight + (double)cnt[level] * (double)(unreached - 1 - level) > stop) return;
    const int32_t end = begin + cnt[level];
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t b = begin + wave * kWave; b < end; b += nwaves * kWave) {    // uniform per wave
        const int64_t i = b + lane;
        int32_t j0 = 0, len = 0;
        if (i < end) {
            const int32_t p = rows[i];
            j0 = rowptr[p];
            len = rowptr[p + 1] - j0;
        }
        const int32_t steps = wave_max_i32(len);
        for (int32_t t = 0; t < steps; ++t) {
            int32_t q = 0;
            bool mine = false;
            if (t < len) {
                q = col[j0 + t];
                mine = dist[q] == unreached && atomicCAS(&dist[q], unreached, level + 1) == unreached;
            }
            wave_append(mine, q, &cnt[level + 1], end, rows);
        }
    }
}

// Groups of rows by hop distance (0..cap) from the endpoints of the nseeds
// edges eids[]: rows (capacity n) and cnt (cap + 2 entries) on the device,
// cnt also returned on the host.  With stop > 0 the expansion ends early once
// the groups found weigh more than stop (a row at distance d weighs cap - d:
// the sweeps that recompute it); the counts are then partial.  Synchronises
// once.
std::vector<int32_t> bfs_groups(const sfg_csr *H, int64_t nseeds, const int32_t *eids, const int32_t *u,
                                const int32_t *v, int32_t cap, int32_t *dist, int32_t *cnt, int32_t *rows,
                                hipStream_t s, double stop = 0.0) {
    const int64_t n = H->n;
    fill_i32(dist, n, cap + 1, s);
    fill_i32(cnt, cap + 2, 0, s);
    const uint32_t sb = std::min<uint32_t>(grid_for(nseeds, 256), kBfsBlocks);
    hipLaunchKernelGGL(k_bfs_seed, dim3(sb), dim3(256), 0, s, nseeds, eids, u, v, cap + 1, dist, cnt, rows);
    SFG_LAUNCH_CHECK();
    const uint32_t eb = std::min<uint32_t>(grid_for(n, 256), kBfsBlocks);
    for (int32_t lvl = 0; lvl < cap; ++lvl) {
        hipLaunchKernelGGL(k_bfs_expand, dim3(eb), dim3(256), 0, s, H->rowptr, H->col, lvl, cap + 1, dist, cnt, rows,
                           stop);
        SFG_LAUNCH_CHECK();
    }
    std::vector<int32_t> hh(cap + 1);
    SFG_HIP(hipMemcpyAsync(hh.data(), cnt, sizeof(int32_t) * (cap + 1), hipMemcpyDeviceToHost, s));
    SFG_HIP(hipStreamSynchronize(s));
    return hh;
}

__global__ void k_band_final(int64_t nc, const uint8_t *__restrict__ cls, uint8_t *sel) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nc) sel[i] = cls[i] == 2 ? 1 : 0;
}

__global__ void k_band_apply(int64_t nb, const int32_t *__restrict__ pos, const uint8_t *__restrict__ selb,
                             uint8_t *sel) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb) sel[pos[i]] = selb[i];
}

}  // namespace

// Evenly strided sample of the candidates: nb edge ids (stride nc / nb)
__global__ void k_stride_sample(int64_t nb, int64_t nc, const int32_t *__restrict__ cand, int32_t *eids) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb) eids[i] = cand[(int64_t)((double)i * (double)nc / (double)nb)];
}

// Predicted share of the full pass's row updates that the FP64 re-scoring
// cone would take, before any smoothing: the band is not known yet, so its
// endpoints are stood in for by an evenly strided sample of the candidates
// of the expected band size (about band * n_cand / 2: 0.4-0.6% of the
// candidates for a 1% band on grids, meshes and kNN graphs), and the same
// capped BFS measures their T-hop neighbourhood.  The BFS stops as soon as
// the share found exceeds `limit` (the caller's decision is then made: the
// returned share is a lower bound above it); below it the share is exact.
// On the 2M-point kNN graph with 20 sweeps the full BFS cost 2.4 ms.
// Synchronises.
double predicted_cone_share(const sfg_csr *H, int32_t sweeps, int64_t n_cand, const int32_t *cand,
                            const int32_t *u, const int32_t *v, double band, double limit, DevArena &A,
                            hipStream_t s) {
    const int64_t n = H->n;
    if (n_cand <= 0 || sweeps <= 0) return 0.0;
    int64_t nb = (int64_t)std::ceil(0.5 * band * (double)n_cand);
    nb = std::max<int64_t>(1, std::min(nb, n_cand));
    int32_t *eids = A.alloc<int32_t>(nb + 1);
    hipLaunchKernelGGL(k_stride_sample, dim3(grid_for(nb, 256)), dim3(256), 0, s, nb, n_cand, cand, eids);
    SFG_LAUNCH_CHECK();
    int32_t *dist = A.alloc<int32_t>(n + 1);
    int32_t *cnt = A.alloc<int32_t>(sweeps + 2);
    int32_t *rows = A.alloc<int32_t>(n + 1);
    const std::vector<int32_t> hh =
        bfs_groups(H, nb, eids, u, v, sweeps, dist, cnt, rows, s, limit * (double)sweeps * (double)n);
    // sweep t recomputes the rows within sweeps-1-t hops
    int64_t within = 0, cone = 0;
    std::vector<int64_t> upto(sweeps + 1);
    for (int32_t d = 0; d <= sweeps; ++d) upto[d] = (within += hh[d]);
    for (int32_t t = 0; t < sweeps; ++t) cone += upto[sweeps - 1 - t];
    return (double)cone / ((double)sweeps * (double)n);
}

void band_rescore(const sfg_csr *H64, int32_t k, int32_t sweeps, double omega, const double *x0, int64_t n_cand,
                  const int32_t *cand, const int32_t *u, const int32_t *v, const double *w64, const float *score_lo,
                  int64_t k_sel, double tau_lo, double band, uint8_t *sel, sfg_level_report *rep, DevArena &A,
                  hipStream_t s) {
    const int64_t n = H64->n;
    uint8_t *cls = A.alloc<uint8_t>(n_cand + 1);
    unsigned long long *cnt = A.alloc<unsigned long long>(2);
    double m = band;
    int32_t rounds = 0;
    int64_t nB = 0, nA = 0;
    for (;;) {
        const double lo = (1.0 - m) * tau_lo, hi = (1.0 + m) * tau_lo;
        hipLaunchKernelGGL(k_band_class, dim3(grid_for(n_cand, 256)), dim3(256), 0, s, n_cand, score_lo, lo, hi, cls);
        SFG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, cnt, 2);
        SFG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_count_cls, dim3(256), dim3(256), 0, s, n_cand, cls, cnt);
        SFG_LAUNCH_CHECK();
        unsigned long long h[2];
        SFG_HIP(hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, s));
        SFG_HIP(hipStreamSynchronize(s));
        nB = (int64_t)h[0];
        nA = (int64_t)h[1];
        const int64_t need = k_sel - nA;
        if (need >= 0 && need <= nB) break;
        m *= 2.0;
        ++rounds;
        SFG_REQUIRE(rounds <= 40, SFG_ENUMERIC, "band: margin doubling did not converge");
    }
    const int64_t need = k_sel - nA;
    // B as candidate positions (ascending, so ascending edge id) and edge ids
    int32_t *posB = A.alloc<int32_t>(nB + 1);
    const int64_t nB2 = compact_ids(cls, 1, n_cand, posB, A, s);
    SFG_REQUIRE(nB2 == nB, SFG_EHIP, "band: inconsistent band size");
    int32_t *eB = A.alloc<int32_t>(nB + 1);
    if (nB > 0) {
        hipLaunchKernelGGL(k_gather_ids, dim3(grid_for(nB, 256)), dim3(256), 0, s, nB, posB, cand, eB);
        SFG_LAUNCH_CHECK();
    }
    int64_t cone_rows = 0;
    double *sB = A.alloc<double>(nB + 1);
    std::vector<int32_t> st;     // distance-group starts (host)
    if (nB > 0) {
        // dependency cone: the rows within `sweeps` hops of the band's endpoints, grouped by distance
        int32_t *dist = A.alloc<int32_t>(n + 1);
        int32_t *cnt = A.alloc<int32_t>(sweeps + 2);
        int32_t *rows = A.alloc<int32_t>(n + 1);
        const std::vector<int32_t> hh = bfs_groups(H64, nB, eB, u, v, sweeps, dist, cnt, rows, s);
        st.assign(sweeps + 2, 0);
        for (int32_t d = 0; d <= sweeps; ++d) st[d + 1] = st[d] + hh[d];
        // sweep t (0-based) recomputes the rows within sweeps-1-t hops
        std::vector<int64_t> active(sweeps > 0 ? sweeps : 1);
        for (int32_t t = 0; t < sweeps; ++t) {
            active[t] = st[sweeps - t];   // rows with dist <= sweeps-1-t
            cone_rows += active[t];
        }
        double *X = nullptr;
        if (4 * cone_rows <= (int64_t)sweeps * n) {
            // rows are already ordered by distance
            double *b0 = A.alloc<double>((size_t)n * k);
            double *b1 = A.alloc<double>((size_t)n * k);
            double *mean = A.alloc<double>(k);
            void *partial = A.raw(cone_partial_bytes(n, k));
            X = smooth_cone_f64(H64, k, sweeps, omega, x0, rows, active.data(), b0, b1, partial, mean, s);
        } else {
            cone_rows = (int64_t)sweeps * n;
            X = A.alloc<double>((size_t)n * k);
            const size_t wsb = smooth_workspace_bytes(n, k, SFG_F64);
            smooth(H64, k, sweeps, omega, x0, SFG_F64, 0, X, A.raw(wsb), wsb, s, -1);
        }
        edge_scores(X, SFG_F64, n, k, nB, eB, u, v, w64, SFG_F64, sB, SFG_F64, s);
    }
    // final: A, plus the best `need` of B by FP64 score
    hipLaunchKernelGGL(k_band_final, dim3(grid_for(n_cand, 256)), dim3(256), 0, s, n_cand, cls, sel);
    SFG_LAUNCH_CHECK();
    if (nB > 0) {
        uint8_t *selB = A.alloc<uint8_t>(nB + 1);
        double *tauB = A.alloc<double>(1);
        const size_t wsb = select_workspace_bytes(nB);
        void *ws = A.raw(wsb);
        select_topk(sB, SFG_F64, nB, need, selB, tauB, ws, wsb, s);
        hipLaunchKernelGGL(k_band_apply, dim3(grid_for(nB, 256)), dim3(256), 0, s, nB, posB, selB, sel);
        SFG_LAUNCH_CHECK();
        if (rep && need > 0) SFG_HIP(hipMemcpyAsync(&rep->tau, tauB, sizeof(double), hipMemcpyDeviceToHost, s));
    }
    if (rep) {
        rep->band = nB;
        rep->band_above = nA;
        rep->band_rounds = rounds;
        rep->cone_rows = cone_rows;
    }
    SFG_HIP(hipStreamSynchronize(s));
}

}  // namespace sfg
