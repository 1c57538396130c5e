// Edge pass: embedding-distance scores (Eq. 18 of the paper with the
// smoothed block standing in for eigenvectors; Alg. 1's edge distortion) and
// algebraic-distance node affinities (Sec. 3.2).
//
// One thread per edge: it streams the two endpoint rows of the node-major
// block (k*elt contiguous bytes each, loaded 16 bytes at a time) and adds the
// k terms in ascending column order, so FP64 scores equal the plain
// sequential definition exactly.  Candidates are processed in their given
// (ascending edge id) order, so the u-endpoint rows are read nearly
// sequentially and the v-endpoint rows hit nearby cache lines on meshes.
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

template <typename TX, typename TW, typename TA, typename TS>
void launch_scores(int64_t ne, int32_t k, const int32_t *cand, const int32_t *u, const int32_t *v, const void *w,
                   const void *x, void *score, hipStream_t s) {
    constexpr int VW = 16 / sizeof(TX);
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
