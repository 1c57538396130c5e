// Edge pass: embedding-distance scores (Eq. 18 of the paper with the
// smoothed block standing in for eigenvectors; Alg. 1's edge distortion) and
// algebraic-distance node affinities (Sec. 3.2).
//
// Scores: a group of G lanes (G = 4, or 2 for 32-byte rows) takes one edge.
// Lane l loads 16-byte pieces l, l + G, l + 2G, ... of both endpoint rows of
// the node-major block, so one load instruction of a wavefront reads whole
// 64-byte (or 32-byte) row segments instead of one 16-byte piece of 64
// different rows.  The k squared differences are then added in ascending
// column order by passing the running sum from lane to lane within the group
// (a DPP rotation): lane l adds its piece when the sum reaches it.  FP64
// scores therefore equal the plain sequential definition exactly.  Row sizes
// that do not split into such groups take one lane per edge, the same
// additions.  Candidates are processed in their given (ascending edge id)
// order, so the u-endpoint rows are read nearly sequentially and the
// v-endpoint rows hit nearby cache lines on meshes.
#include "common.hpp"

namespace sfg {

void column_means(const void *x, sfg_dtype xt, int64_t n, int32_t k, double *mean, void *partial_ws, hipStream_t s);
size_t column_means_partial_bytes(int64_t n, int32_t k);

namespace {

template <typename T, int N>
struct alignas(sizeof(T) * N) Vec {
    T v[N];
};

__device__ __forceinline__ double sq_add(double acc, double d) { return acc + d * d; }
__device__ __forceinline__ float sq_add(float acc, float d) { return __builtin_fmaf(d, d, acc); }

template <typename TX, typename TW, typename TA, typename TS, int VW>
__global__ __launch_bounds__(256) void k_scores(int64_t ne, int32_t k, const int32_t *__restrict__ cand,
                                                const int32_t *__restrict__ u, const int32_t *__restrict__ v,
                                                const TW *__restrict__ w, const TX *__restrict__ x,
                                                TS *__restrict__ score) {
    const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t i = (int64_t)b * 256 + threadIdx.x;
    if (i >= ne) return;
    const int64_t e = cand ? cand[i] : i;
    const TX *xp = x + (int64_t)u[e] * k;
    const TX *xq = x + (int64_t)v[e] * k;
    TA acc = TA(0);
#pragma unroll 4
    for (int32_t c = 0; c < k; c += VW) {
        const Vec<TX, VW> a = *reinterpret_cast<const Vec<TX, VW> *>(xp + c);
        const Vec<TX, VW> bq = *reinterpret_cast<const Vec<TX, VW> *>(xq + c);
#pragma unroll
        for (int t = 0; t < VW; ++t) {
            const TA d = cvt<TA>(a.v[t]) - cvt<TA>(bq.v[t]);
            acc = sq_add(acc, d);
        }
    }
    const TA we = cvt<TA>(w[e]);
    score[i] = (TS)(we * acc);
}

// The value of lane l - 1 of the same group of G lanes (lane G - 1 for lane
// 0): quad_perm DPP, which moves data within aligned groups of four lanes.
template <int G>
__device__ __forceinline__ int rot_group(int x) {
    static_assert(G == 2 || G == 4, "groups of 2 or 4 lanes");
    constexpr int kCtrl = G == 4 ? (3 | (0 << 2) | (1 << 4) | (2 << 6)) : (1 | (0 << 2) | (3 << 4) | (2 << 6));
    return __builtin_amdgcn_update_dpp(x, x, kCtrl, 0xF, 0xF, false);
}

template <int G>
__device__ __forceinline__ float rot_group(float x) {
    return __builtin_bit_cast(float, rot_group<G>(__builtin_bit_cast(int, x)));
}

template <int G>
__device__ __forceinline__ double rot_group(double x) {
    const int lo = rot_group<G>(__double2loint(x)), hi = rot_group<G>(__double2hiint(x));
    return __hiloint2double(hi, lo);
}

// Row of K = G * VW * R elements: R rounds of G 16-byte pieces.  Every lane of
// a group runs the same steps; at step (r, j) lane j holds the sum of the
// first r*G*VW + (j+1)*VW terms, the other lanes' values are overwritten
// before they are read.  Groups never straddle the grid's end: G divides 256.
template <typename TX, typename TW, typename TA, typename TS, int G, int R>
__global__ __launch_bounds__(256) void k_scores_grp(int64_t ne, const int32_t *__restrict__ cand,
                                                    const int32_t *__restrict__ u, const int32_t *__restrict__ v,
                                                    const TW *__restrict__ w, const TX *__restrict__ x,
                                                    TS *__restrict__ score) {
    constexpr int VW = 16 / sizeof(TX);
    constexpr int K = G * VW * R;
    const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t i = ((int64_t)b * 256 + threadIdx.x) / G;
    const int l = threadIdx.x % G;
    if (i >= ne) return;
    const int64_t e = cand ? cand[i] : i;
    const TX *xp = x + (int64_t)u[e] * K + l * VW;
    const TX *xq = x + (int64_t)v[e] * K + l * VW;
    TA d[R][VW];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const Vec<TX, VW> a = *reinterpret_cast<const Vec<TX, VW> *>(xp + r * G * VW);
        const Vec<TX, VW> bq = *reinterpret_cast<const Vec<TX, VW> *>(xq + r * G * VW);
#pragma unroll
        for (int t = 0; t < VW; ++t) d[r][t] = cvt<TA>(a.v[t]) - cvt<TA>(bq.v[t]);
    }
    TA acc = TA(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int j = 0; j < G; ++j) {
            if (r + j > 0) acc = rot_group<G>(acc);
#pragma unroll
            for (int t = 0; t < VW; ++t) acc = sq_add(acc, d[r][t]);
        }
    }
    if (l == G - 1) score[i] = (TS)(cvt<TA>(w[e]) * acc);
}

template <typename TX, typename TW, typename TA, typename TS, int G, int R>
void launch_grp(int64_t ne, const int32_t *cand, const int32_t *u, const int32_t *v, const void *w, const void *x,
                void *score, hipStream_t s) {
    hipLaunchKernelGGL((k_scores_grp<TX, TW, TA, TS, G, R>), dim3(grid_for(ne * G, 256)), dim3(256), 0, s, ne, cand,
                       u, v, (const TW *)w, (const TX *)x, (TS *)score);
    SFG_LAUNCH_CHECK();
}

template <typename TX, typename TW, typename TA, typename TS>
void launch_scores(int64_t ne, int32_t k, const int32_t *cand, const int32_t *u, const int32_t *v, const void *w,
                   const void *x, void *score, hipStream_t s) {
    constexpr int VW = 16 / sizeof(TX);
    const int64_t row_bytes = (int64_t)k * (int64_t)sizeof(TX);
    switch (row_bytes) {
        case 32: return launch_grp<TX, TW, TA, TS, 2, 1>(ne, cand, u, v, w, x, score, s);
        case 64: return launch_grp<TX, TW, TA, TS, 4, 1>(ne, cand, u, v, w, x, score, s);
        case 128: return launch_grp<TX, TW, TA, TS, 4, 2>(ne, cand, u, v, w, x, score, s);
        case 256: return launch_grp<TX, TW, TA, TS, 4, 4>(ne, cand, u, v, w, x, score, s);
        default: break;
    }
    const dim3 g(grid_for(ne, 256)), blk(256);
    if (k % VW == 0)
        hipLaunchKernelGGL((k_scores<TX, TW, TA, TS, VW>), g, blk, 0, s, ne, k, cand, u, v, (const TW *)w,
                           (const TX *)x, (TS *)score);
    else
        hipLaunchKernelGGL((k_scores<TX, TW, TA, TS, 1>), g, blk, 0, s, ne, k, cand, u, v, (const TW *)w,
                           (const TX *)x, (TS *)score);
    SFG_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ affinity

template <typename TX, typename TA, typename TO>
__global__ __launch_bounds__(256) void k_affinity(int64_t m, int32_t k, const int32_t *__restrict__ u,
                                                  const int32_t *__restrict__ v, const TX *__restrict__ x,
                                                  const double *__restrict__ mean, TO *__restrict__ aff) {
    const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t e = (int64_t)b * 256 + threadIdx.x;
    if (e >= m) return;
    const TX *xp = x + (int64_t)u[e] * k;
    const TX *xq = x + (int64_t)v[e] * k;
    TA dot = TA(0), np = TA(0), nq = TA(0);
    for (int32_t c = 0; c < k; ++c) {
        const TA mc = cvt<TA>(mean[c]);
        const TA a = cvt<TA>(xp[c]) - mc;
        const TA bq = cvt<TA>(xq[c]) - mc;
        const TA t1 = a * bq, t2 = a * a, t3 = bq * bq;
        dot = dot + t1;
        np = np + t2;
        nq = nq + t3;
    }
    TA r = TA(0);
    if (np != TA(0) && nq != TA(0)) {
        const TA num = dot * dot;
        const TA den = np * nq;
        r = num / den;
    }
    aff[e] = (TO)r;
}

}  // namespace

void edge_scores(const void *x, sfg_dtype xt, int64_t n, int32_t k, int64_t ne, const int32_t *cand,
                 const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt, void *score, sfg_dtype st,
                 hipStream_t s) {
    SFG_REQUIRE(ne >= 0 && n >= 1 && k >= 1, SFG_EINVAL, "edge_scores: bad sizes");
    SFG_REQUIRE(k <= 64, SFG_EUNSUPPORTED, "edge_scores: k > 64 is not supported");
    if (ne == 0) return;
    SFG_REQUIRE(x && u && v && w && score, SFG_EINVAL, "edge_scores: null pointer");
    if (st == SFG_F64) {
        SFG_REQUIRE(xt == SFG_F64 && wt == SFG_F64, SFG_EUNSUPPORTED, "edge_scores: F64 scores need F64 x and w");
        launch_scores<double, double, double, double>(ne, k, cand, u, v, w, x, score, s);
        return;
    }
    SFG_REQUIRE(st == SFG_F32, SFG_EINVAL, "edge_scores: score dtype must be F64 or F32");
    SFG_REQUIRE(wt == SFG_F32, SFG_EUNSUPPORTED, "edge_scores: F32 scores need F32 weights");
    switch (xt) {
        case SFG_F32: launch_scores<float, float, float, float>(ne, k, cand, u, v, w, x, score, s); break;
        case SFG_F16: launch_scores<__half, float, float, float>(ne, k, cand, u, v, w, x, score, s); break;
        case SFG_BF16: launch_scores<__hip_bfloat16, float, float, float>(ne, k, cand, u, v, w, x, score, s); break;
        default: fail(SFG_EUNSUPPORTED, "edge_scores: F32 scores from an F64 block are not supported");
    }
}

size_t affinity_workspace_bytes(int64_t n, int32_t k) {
    return column_means_partial_bytes(n, k) + 64 * sizeof(double) + 512;
}

void affinity(const void *x, sfg_dtype xt, int64_t n, int32_t k, int64_t m, const int32_t *u, const int32_t *v,
              void *aff, sfg_dtype at, void *ws, size_t ws_bytes, hipStream_t s) {
    SFG_REQUIRE(n >= 1 && k >= 1 && m >= 0, SFG_EINVAL, "affinity: bad sizes");
    SFG_REQUIRE(k <= 64, SFG_EUNSUPPORTED, "affinity: k > 64 is not supported");
    SFG_REQUIRE(ws_bytes >= affinity_workspace_bytes(n, k), SFG_EWORKSPACE, "affinity: workspace too small");
    Carver c(ws);
    double *mean = c.take<double>(64);
    void *partial = c.take<char>(column_means_partial_bytes(n, k));
    column_means(x, xt, n, k, mean, partial, s);
    if (m == 0) return;
    const dim3 g(grid_for(m, 256)), blk(256);
    if (xt == SFG_F64 && at == SFG_F64)
        hipLaunchKernelGGL((k_affinity<double, double, double>), g, blk, 0, s, m, k, u, v, (const double *)x, mean,
                           (double *)aff);
    else if (xt == SFG_F32 && at == SFG_F32)
        hipLaunchKernelGGL((k_affinity<float, float, float>), g, blk, 0, s, m, k, u, v, (const float *)x, mean,
                           (float *)aff);
    else
        fail(SFG_EUNSUPPORTED, "affinity: (x, aff) dtypes must be (F64, F64) or (F32, F32)");
    SFG_LAUNCH_CHECK();
}

}  // namespace sfg

extern "C" sfg_status sfg_edge_scores(const void *x, sfg_dtype xt, int64_t n, int32_t k, int64_t ne,
                                      const int32_t *cand, const int32_t *u, const int32_t *v, const void *w,
                                      sfg_dtype wt, void *score, sfg_dtype st, void *stream) {
    return sfg::guard([&] { sfg::edge_scores(x, xt, n, k, ne, cand, u, v, w, wt, score, st, sfg::as_stream(stream)); });
}

extern "C" sfg_status sfg_affinity(const void *x, sfg_dtype xt, int64_t n, int32_t k, int64_t m, const int32_t *u,
                                   const int32_t *v, void *aff, sfg_dtype at, void *ws, size_t ws_bytes,
                                   void *stream) {
    return sfg::guard([&] { sfg::affinity(x, xt, n, k, m, u, v, aff, at, ws, ws_bytes, sfg::as_stream(stream)); });
}
