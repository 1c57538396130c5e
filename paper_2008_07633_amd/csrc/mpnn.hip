// Learned edge-criticality surrogate: a two-layer message-passing network
// over G with an edge head, trained on the scores the plain method produces.
// (Not part of the paper; it prunes candidates before exact scoring.)
//
//   A1 = D^-1 A X            X: 8 standardised node features
//   H1 = relu([X | A1 | 1] W1)       W1: (2*8+1) x 32
//   A2 = D^-1 A H1
//   H2 = relu([H1 | A2 | 1] W2)      W2: (2*32+1) x 32
//   z_e = [|H2_p - H2_q| | H2_p * H2_q | f_e | 1]   (69)
//   yhat_e = [relu(z_e W3) | 1] . w4      W3: 69 x 32, w4: 33
// Parameters are one FP32 vector [W1 | W2 | W3 | w4] (4865 values); each
// block stacks the self weights, the neighbour weights and the bias, so a
// weight gradient is one product U^T dP of the layer's input [x | a | 1].
//
// Kernels: the aggregations reuse the smoothing sweep (omega = 1).
// Inference (BF16 activations) runs the dense layers and the edge head on the
// matrix cores: a wavefront takes 32 nodes or edges, builds their [x | a | 1]
// or z rows as BF16 MFMA operands (K padded to a multiple of 8), multiplies
// by the BF16 weights with v_mfma_f32_32x32x8_bf16 into FP32 accumulators,
// and applies the ReLU (and the head's last dot product) in FP32.  Training
// runs in FP32 on the vector units: weights in LDS, one node or edge per
// thread, 32-wide accumulators; backward sends per-edge gradients to nodes
// through an incidence CSR in ascending edge order and reduces weight
// gradients by fixed-shape block partials: no FP atomics, so training is
// deterministic.
#include <cmath>
#include <vector>

#include <type_traits>

#include "common.hpp"

namespace sfg {

void spmm_rownorm(const sfg_csr *H, int32_t k, sfg_dtype t, const void *x, void *y, hipStream_t s);
size_t csr_workspace_bytes(int64_t n, int64_t m);
void build_csr(int64_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w, sfg_dtype wt,
               const uint8_t *mask, int32_t *rowptr, int32_t *col, void *val, int32_t *eid, void *deg, void *ws,
               size_t ws_bytes, hipStream_t s);

namespace {

constexpr int kF = 8;                 // node features
constexpr int kH = 32;                // hidden width
constexpr int kE = 4;                 // edge features
constexpr int kZ = 2 * kH + kE;       // edge-head input
constexpr int kU1 = 2 * kF + 1;       // rows of W1
constexpr int kU2 = 2 * kH + 1;       // rows of W2
constexpr int kZ1 = kZ + 1;           // rows of W3
constexpr int kOffW1 = 0;
constexpr int kOffW2 = kOffW1 + kU1 * kH;
constexpr int kOffW3 = kOffW2 + kU2 * kH;
constexpr int kOffW4 = kOffW3 + kZ1 * kH;
constexpr int kParams = kOffW4 + kH + 1;
static_assert(kParams == 4865, "parameter count");
constexpr float kTiny = 1e-30f;

template <typename T>
__device__ __forceinline__ float ld(const T *p) {
    return cvt<float>(*p);
}
template <>
__device__ __forceinline__ float ld<float>(const float *p) {
    return *p;
}

// ------------------------------------------------------------------ features

// |x_p - x_q|^2 over the kc cheap vectors, added in column order (KC > 0: kc =
// KC, a multiple of 4, loaded as 16-byte vectors)
template <int KC>
__device__ __forceinline__ float dist2(const float *__restrict__ xc, int32_t kc, const float *xp, int64_t q) {
    float d2 = 0.f;
    if constexpr (KC > 0) {
#pragma unroll
        for (int c4 = 0; c4 < KC / 4; ++c4) {
            const float4 b = *reinterpret_cast<const float4 *>(xc + q * KC + 4 * c4);
            const float bq[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float d = xp[4 * c4 + c] - bq[c];
                d2 = __builtin_fmaf(d, d, d2);
            }
        }
    } else {
        const float *xq = xc + q * kc;
        for (int c = 0; c < kc; ++c) {
            const float d = xp[c] - xq[c];
            d2 = __builtin_fmaf(d, d, d2);
        }
    }
    return d2;
}

// sum_j w_j |x_p - x_col[j]|^2 over a row, in entry order, two entries in flight
template <int KC>
__device__ __forceinline__ float row_energy(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                            const float *__restrict__ val, const float *__restrict__ xc, int32_t kc,
                                            const float *xp, int64_t p) {
    float e = 0.f;
    const int32_t j0 = rp[p], j1 = rp[p + 1];
    int32_t j = j0;
    for (; j + 2 <= j1; j += 2) {
        const int64_t q0 = col[j], q1 = col[j + 1];
        const float w0 = val[j], w1 = val[j + 1];
        const float d0 = dist2<KC>(xc, kc, xp, q0), d1 = dist2<KC>(xc, kc, xp, q1);
        e = __builtin_fmaf(w0, d0, e);
        e = __builtin_fmaf(w1, d1, e);
    }
    if (j < j1) e = __builtin_fmaf(val[j], dist2<KC>(xc, kc, xp, col[j]), e);
    return e;
}

template <int KC>
__global__ void k_node_feat(int64_t n, const int32_t *__restrict__ grp, const int32_t *__restrict__ gcol,
                            const float *__restrict__ gval, const float *__restrict__ gdeg,
                            const int32_t *__restrict__ trp, const int32_t *__restrict__ tcol,
                            const float *__restrict__ tval, const float *__restrict__ tdeg,
                            const float *__restrict__ xc, int32_t kc, const float *__restrict__ norm, float *nf) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    float xp[KC > 0 ? KC : 64];
    if constexpr (KC > 0) {
#pragma unroll
        for (int c4 = 0; c4 < KC / 4; ++c4) {
            const float4 a = *reinterpret_cast<const float4 *>(xc + p * KC + 4 * c4);
            xp[4 * c4] = a.x;
            xp[4 * c4 + 1] = a.y;
            xp[4 * c4 + 2] = a.z;
            xp[4 * c4 + 3] = a.w;
        }
    } else {
        for (int c = 0; c < kc; ++c) xp[c] = xc[p * kc + c];
    }
    float amp = 0.f;
    for (int c = 0; c < (KC > 0 ? KC : kc); ++c) amp = __builtin_fmaf(xp[c], xp[c], amp);
    const float eg = row_energy<KC>(grp, gcol, gval, xc, kc, xp, p);
    const float et = row_energy<KC>(trp, tcol, tval, xc, kc, xp, p);
    float f[kF];
    f[0] = 1.f;
    f[1] = logf(gdeg[p]);
    f[2] = logf(tdeg[p]);
    f[3] = logf((float)(grp[p + 1] - grp[p]));
    f[4] = logf((float)(trp[p + 1] - trp[p]));
    f[5] = logf(amp + kTiny);
    f[6] = logf(eg / gdeg[p] + kTiny);
    f[7] = logf(et / tdeg[p] + kTiny);
    float o[kF];
#pragma unroll
    for (int i = 0; i < kF; ++i) o[i] = (norm && i > 0) ? (f[i] - norm[i]) * norm[kF + i] : f[i];
    if constexpr (KC > 0) {
        *reinterpret_cast<float4 *>(nf + p * kF) = make_float4(o[0], o[1], o[2], o[3]);
        *reinterpret_cast<float4 *>(nf + p * kF + 4) = make_float4(o[4], o[5], o[6], o[7]);
    } else {
#pragma unroll
        for (int i = 0; i < kF; ++i) nf[p * kF + i] = o[i];
    }
}

template <int KC>
__global__ void k_edge_feat(int64_t ne, const int32_t *__restrict__ cand, const int32_t *__restrict__ u,
                            const int32_t *__restrict__ v, const float *__restrict__ w, const float *__restrict__ xc,
                            int32_t kc, const float *__restrict__ tdeg, const float *__restrict__ norm, float *ef) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    const int32_t e = cand ? cand[i] : (int32_t)i;
    const int32_t p = u[e], q = v[e];
    float xp[KC > 0 ? KC : 64];
    if constexpr (KC > 0) {
#pragma unroll
        for (int c4 = 0; c4 < KC / 4; ++c4) {
            const float4 a = *reinterpret_cast<const float4 *>(xc + (int64_t)p * KC + 4 * c4);
            xp[4 * c4] = a.x;
            xp[4 * c4 + 1] = a.y;
            xp[4 * c4 + 2] = a.z;
            xp[4 * c4 + 3] = a.w;
        }
    } else {
        for (int c = 0; c < kc; ++c) xp[c] = xc[(int64_t)p * kc + c];
    }
    const float d2 = dist2<KC>(xc, kc, xp, q);
    const float lp = logf(tdeg[p]), lq = logf(tdeg[q]);
    float f[kE] = {logf(w[e]), logf(w[e] * d2 + kTiny), fminf(lp, lq), fmaxf(lp, lq)};
#pragma unroll
    for (int j = 0; j < kE; ++j) {
        float x = f[j];
        if (norm) x = (x - norm[2 * kF + j]) * norm[2 * kF + kE + j];
        ef[i * kE + j] = x;
    }
}

// ------------------------------------------------------------------ forward

template <typename TIN, typename TOUT, int FIN>
__global__ __launch_bounds__(256) void k_dense_fwd(int64_t n, const TIN *__restrict__ x, const TIN *__restrict__ a,
                                                   const float *__restrict__ W, TOUT *__restrict__ h,
                                                   float *__restrict__ pre, float *__restrict__ uin) {
    __shared__ float sw[(2 * FIN + 1) * kH];
    for (int i = threadIdx.x; i < (2 * FIN + 1) * kH; i += blockDim.x) sw[i] = W[i];
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    float acc[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) acc[j] = sw[2 * FIN * kH + j];
    for (int i = 0; i < FIN; ++i) {
        const float xi = ld(x + p * FIN + i);
        if (uin) uin[p * (2 * FIN + 1) + i] = xi;
#pragma unroll
        for (int j = 0; j < kH; ++j) acc[j] = __builtin_fmaf(xi, sw[i * kH + j], acc[j]);
    }
    for (int i = 0; i < FIN; ++i) {
        const float ai = ld(a + p * FIN + i);
        if (uin) uin[p * (2 * FIN + 1) + FIN + i] = ai;
#pragma unroll
        for (int j = 0; j < kH; ++j) acc[j] = __builtin_fmaf(ai, sw[(FIN + i) * kH + j], acc[j]);
    }
    if (uin) uin[p * (2 * FIN + 1) + 2 * FIN] = 1.f;
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        if (pre) pre[p * kH + j] = acc[j];
        h[p * kH + j] = cvt<TOUT>(fmaxf(acc[j], 0.f));
    }
}

template <typename TH>
__global__ __launch_bounds__(256) void k_head_fwd(int64_t ne, const int32_t *__restrict__ cand,
                                                  const int32_t *__restrict__ u, const int32_t *__restrict__ v,
                                                  const TH *__restrict__ h, const float *__restrict__ ef,
                                                  const float *__restrict__ W3, const float *__restrict__ w4,
                                                  float *__restrict__ pred, float *__restrict__ gsave,
                                                  float *__restrict__ zsave) {
    __shared__ float s3[kZ1 * kH];
    __shared__ float s4[kH + 1];
    for (int i = threadIdx.x; i < kZ1 * kH; i += blockDim.x) s3[i] = W3[i];
    for (int i = threadIdx.x; i < kH + 1; i += blockDim.x) s4[i] = w4[i];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    const int32_t e = cand ? cand[i] : (int32_t)i;
    const TH *hp = h + (int64_t)u[e] * kH;
    const TH *hq = h + (int64_t)v[e] * kH;
    float g[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) g[j] = s3[kZ * kH + j];
    for (int c = 0; c < kH; ++c) {
        const float a = ld(hp + c), b = ld(hq + c);
        const float z0 = fabsf(a - b), z1 = a * b;
        if (zsave) {
            zsave[i * kZ1 + c] = z0;
            zsave[i * kZ1 + kH + c] = z1;
        }
#pragma unroll
        for (int j = 0; j < kH; ++j) g[j] = __builtin_fmaf(z0, s3[c * kH + j], g[j]);
#pragma unroll
        for (int j = 0; j < kH; ++j) g[j] = __builtin_fmaf(z1, s3[(kH + c) * kH + j], g[j]);
    }
    for (int c = 0; c < kE; ++c) {
        const float z = ef[i * kE + c];
        if (zsave) zsave[i * kZ1 + 2 * kH + c] = z;
#pragma unroll
        for (int j = 0; j < kH; ++j) g[j] = __builtin_fmaf(z, s3[(2 * kH + c) * kH + j], g[j]);
    }
    if (zsave) zsave[i * kZ1 + kZ] = 1.f;
    float out = s4[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        if (gsave) gsave[i * kH + j] = g[j];
        out = __builtin_fmaf(fmaxf(g[j], 0.f), s4[j], out);
    }
    pred[i] = out;
}

// ------------------------------------------------------------------ inference on the matrix cores
//
// v_mfma_f32_32x32x8_bf16 (one 32 x 32 x 8 block per wavefront), lane l:
//   A (32 x 8):  row l % 32, columns 4 * (l / 32) + 0..3
//   B (8 x 32):  column l % 32, rows 4 * (l / 32) + 0..3
//   D (32 x 32): column l % 32, rows 8 * (r / 4) + 4 * (l / 32) + r % 4, r = 0..15

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ short bf16_bits(float x) {
    const __hip_bfloat16 b = cvt<__hip_bfloat16>(x);
    short r;
    __builtin_memcpy(&r, &b, sizeof(r));
    return r;
}

__device__ __forceinline__ float bits_float(short r) {
    __hip_bfloat16 b;
    __builtin_memcpy(&b, &r, sizeof(r));
    return cvt<float>(b);
}

// four consecutive values as BF16 operand bits
__device__ __forceinline__ bf16x4 load4(const float *p) {
    const float4 f = *reinterpret_cast<const float4 *>(p);
    return bf16x4{bf16_bits(f.x), bf16_bits(f.y), bf16_bits(f.z), bf16_bits(f.w)};
}
__device__ __forceinline__ bf16x4 load4(const __hip_bfloat16 *p) {
    return *reinterpret_cast<const bf16x4 *>(p);
}

// B operands of a (rows x 32) FP32 weight block, K padded with zeros
template <int NCH>
__device__ __forceinline__ void load_weights(const float *__restrict__ W, int rows, int half, int col,
                                             bf16x4 (&wb)[NCH]) {
#pragma unroll
    for (int t = 0; t < NCH; ++t) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 8 * t + 4 * half + i;
            wb[t][i] = bf16_bits(k < rows ? W[k * kH + col] : 0.f);
        }
    }
}

// h = relu([x | a | 1] W) for 32 nodes per wavefront; BF16 output.
template <typename TIN, int FIN>
__global__ __launch_bounds__(256) void k_dense_mfma(int64_t n, const TIN *__restrict__ x, const TIN *__restrict__ a,
                                                    const float *__restrict__ W, __hip_bfloat16 *__restrict__ h) {
    static_assert(FIN % 8 == 0, "feature width must be a multiple of 8");
    constexpr int NX = FIN / 8, NCH = 2 * NX + 1;
    const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31;
    bf16x4 wb[NCH];
    load_weights<NCH>(W, 2 * FIN + 1, half, col, wb);
    const int64_t base = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 32;
    if (base >= n) return;
    const int64_t row = base + col;
    const bool valid = row < n;
    const bf16x4 zero = {0, 0, 0, 0};
    f32x16 acc = {};
#pragma unroll
    for (int t = 0; t < NX; ++t) {
        const bf16x4 av = valid ? load4(x + row * FIN + 8 * t + 4 * half) : zero;
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, wb[t], acc, 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < NX; ++t) {
        const bf16x4 av = valid ? load4(a + row * FIN + 8 * t + 4 * half) : zero;
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, wb[NX + t], acc, 0, 0, 0);
    }
    {   // the bias column: k = 2 FIN
        const bf16x4 av = (valid && half == 0) ? bf16x4{bf16_bits(1.f), 0, 0, 0} : zero;
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, wb[2 * NX], acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t node = base + 8 * (r / 4) + 4 * half + (r % 4);
        if (node < n) h[node * kH + col] = cvt<__hip_bfloat16>(fmaxf(acc[r], 0.f));
    }
}

// yhat_e = relu(z_e W3) . w4[0:32] + w4[32] for 32 candidate edges per wavefront.
__global__ __launch_bounds__(256) void k_head_mfma(int64_t ne, const int32_t *__restrict__ cand,
                                                   const int32_t *__restrict__ u, const int32_t *__restrict__ v,
                                                   const __hip_bfloat16 *__restrict__ h,
                                                   const float *__restrict__ ef, const float *__restrict__ W3,
                                                   const float *__restrict__ w4, float *__restrict__ pred) {
    constexpr int NCH = (kZ1 + 7) / 8;      // 9: |hp - hq| (4), hp * hq (4), edge features + bias (1)
    static_assert(kH == 32 && kE == 4 && NCH == 9, "head layout");
    __shared__ float red[4][32][33];
    const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31, wv = threadIdx.x >> 6;
    bf16x4 wb[NCH];
    load_weights<NCH>(W3, kZ1, half, col, wb);
    const float w4c = w4[col];
    const int64_t base = ((int64_t)blockIdx.x * 4 + wv) * 32;
    if (base >= ne) return;
    const int64_t i = base + col;
    const bool valid = i < ne;
    const int32_t e = valid ? (cand ? cand[i] : (int32_t)i) : 0;
    const __hip_bfloat16 *hp = h + (int64_t)(valid ? u[e] : 0) * kH;
    const __hip_bfloat16 *hq = h + (int64_t)(valid ? v[e] : 0) * kH;
    const bf16x4 zero = {0, 0, 0, 0};
    f32x16 acc = {};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        bf16x4 d = zero, p = zero;
        if (valid) {
            const bf16x4 ra = load4(hp + 8 * t + 4 * half), rb = load4(hq + 8 * t + 4 * half);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float fa = bits_float(ra[q]), fb = bits_float(rb[q]);
                d[q] = bf16_bits(fabsf(fa - fb));
                p[q] = bf16_bits(fa * fb);
            }
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(d, wb[t], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(p, wb[4 + t], acc, 0, 0, 0);
    }
    {   // k = 64..67 edge features (lanes of the first half), k = 68 bias
        bf16x4 z = zero;
        if (valid) z = half == 0 ? load4(ef + i * kE) : bf16x4{bf16_bits(1.f), 0, 0, 0};
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(z, wb[8], acc, 0, 0, 0);
    }
    // the last layer: each lane scales its column, then lane m < 32 adds row m
    // in column order
#pragma unroll
    for (int r = 0; r < 16; ++r) red[wv][8 * (r / 4) + 4 * half + (r % 4)][col] = fmaxf(acc[r], 0.f) * w4c;
    __builtin_amdgcn_wave_barrier();
    if (half == 0 && valid) {
        float o = w4[kH];
        for (int j = 0; j < kH; ++j) o += red[wv][col][j];
        pred[i] = o;
    }
}

// ------------------------------------------------------------------ backward

// Per edge: output error, head hidden error, and the edge's contribution to
// the gradients of H2 at both ends.
__global__ __launch_bounds__(256) void k_head_bwd(int64_t ne, const int32_t *__restrict__ cand,
                                                  const int32_t *__restrict__ u, const int32_t *__restrict__ v,
                                                  const float *__restrict__ h, const float *__restrict__ pred,
                                                  const float *__restrict__ target, const float *__restrict__ gsave,
                                                  const float *__restrict__ W3, const float *__restrict__ w4,
                                                  float scale, float *__restrict__ dg, float *__restrict__ ah1,
                                                  float *__restrict__ dy, float *__restrict__ dhp,
                                                  float *__restrict__ dhq) {
    __shared__ float s3[kZ1 * kH];
    __shared__ float s4[kH + 1];
    for (int i = threadIdx.x; i < kZ1 * kH; i += blockDim.x) s3[i] = W3[i];
    for (int i = threadIdx.x; i < kH + 1; i += blockDim.x) s4[i] = w4[i];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    const float d = (pred[i] - target[i]) * scale;
    dy[i] = d;
    float dgl[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        const float gj = gsave[i * kH + j];
        ah1[i * (kH + 1) + j] = fmaxf(gj, 0.f);
        dgl[j] = gj > 0.f ? d * s4[j] : 0.f;
        dg[i * kH + j] = dgl[j];
    }
    ah1[i * (kH + 1) + kH] = 1.f;
    const int32_t e = cand ? cand[i] : (int32_t)i;
    const float *hp = h + (int64_t)u[e] * kH;
    const float *hq = h + (int64_t)v[e] * kH;
    for (int c = 0; c < kH; ++c) {
        float dz0 = 0.f, dz1 = 0.f;
#pragma unroll
        for (int j = 0; j < kH; ++j) {
            dz0 = __builtin_fmaf(dgl[j], s3[c * kH + j], dz0);
            dz1 = __builtin_fmaf(dgl[j], s3[(kH + c) * kH + j], dz1);
        }
        const float a = hp[c], b = hq[c];
        const float sg = a > b ? 1.f : (a < b ? -1.f : 0.f);
        dhp[i * kH + c] = dz0 * sg + dz1 * b;
        dhq[i * kH + c] = -dz0 * sg + dz1 * a;
    }
}

// dH2 at each node from its incident candidate edges, in ascending edge
// order, masked by the layer's ReLU.
__global__ void k_gather_dh(int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                            const int32_t *__restrict__ eid, const float *__restrict__ dhp,
                            const float *__restrict__ dhq, const float *__restrict__ pre, float *dpre) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    float acc[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) acc[j] = 0.f;
    for (int32_t t = rp[p]; t < rp[p + 1]; ++t) {
        const int32_t i = eid[t];
        const float *src = (col[t] > p ? dhp : dhq) + (int64_t)i * kH;
#pragma unroll
        for (int j = 0; j < kH; ++j) acc[j] += src[j];
    }
#pragma unroll
    for (int j = 0; j < kH; ++j) dpre[p * kH + j] = pre[p * kH + j] > 0.f ? acc[j] : 0.f;
}

// Input gradients of a dense layer: t1 = dP Ws^T and t2 = (dP Wn^T) / D.
template <int FIN>
__global__ __launch_bounds__(256) void k_dense_bwd(int64_t n, const float *__restrict__ dpre,
                                                   const float *__restrict__ W, const float *__restrict__ deg,
                                                   float *t1, float *t2) {
    __shared__ float sw[2 * FIN * kH];
    for (int i = threadIdx.x; i < 2 * FIN * kH; i += blockDim.x) sw[i] = W[i];
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    float dp[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) dp[j] = dpre[p * kH + j];
    const float inv = 1.f / deg[p];
    for (int i = 0; i < FIN; ++i) {
        float a = 0.f, b = 0.f;
#pragma unroll
        for (int j = 0; j < kH; ++j) {
            a = __builtin_fmaf(dp[j], sw[i * kH + j], a);
            b = __builtin_fmaf(dp[j], sw[(FIN + i) * kH + j], b);
        }
        t1[p * FIN + i] = a;
        t2[p * FIN + i] = b * inv;
    }
}

__global__ void k_add_mask(int64_t total, const float *__restrict__ a, const float *__restrict__ b,
                           const float *__restrict__ pre, float *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < total) out[i] = pre[i] > 0.f ? a[i] + b[i] : 0.f;
}

// Partial sums of A^T B over row chunks: partial[b][i*db + j] for chunk b.
constexpr int kAtbBlocks = 128;
constexpr int kAtbTile = 16;

__global__ __launch_bounds__(256) void k_atb_partial(int64_t nrows, int da, const float *__restrict__ A, int db,
                                                     const float *__restrict__ B, float *partial) {
    __shared__ float ta[kAtbTile][kZ1];
    __shared__ float tb[kAtbTile][kH + 1];
    const int64_t chunk = (nrows + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = r0 + chunk < nrows ? r0 + chunk : nrows;
    const int nent = da * db;
    float acc[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) acc[q] = 0.f;
    for (int64_t base = r0; base < r1; base += kAtbTile) {
        const int rows = (int)(r1 - base < kAtbTile ? r1 - base : kAtbTile);
        for (int x = threadIdx.x; x < kAtbTile * da; x += blockDim.x) {
            const int r = x / da, c = x % da;
            ta[r][c] = r < rows ? A[(base + r) * da + c] : 0.f;
        }
        for (int x = threadIdx.x; x < kAtbTile * db; x += blockDim.x) {
            const int r = x / db, c = x % db;
            tb[r][c] = r < rows ? B[(base + r) * db + c] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 10; ++q) {
            const int e = threadIdx.x + q * 256;
            if (e < nent) {
                const int i = e / db, j = e % db;
                float s = acc[q];
                for (int r = 0; r < kAtbTile; ++r) s = __builtin_fmaf(ta[r][i], tb[r][j], s);
                acc[q] = s;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 10; ++q) {
        const int e = threadIdx.x + q * 256;
        if (e < nent) partial[(int64_t)blockIdx.x * nent + e] = acc[q];
    }
}

__global__ void k_sum_partials(int nb, int nent, const float *__restrict__ partial, float *out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nent) return;
    float s = 0.f;
    for (int b = 0; b < nb; ++b) s += partial[(int64_t)b * nent + e];
    out[e] = s;
}

__global__ void k_sq_err_partial(int64_t ne, const float *__restrict__ pred, const float *__restrict__ target,
                                 float *partial) {
    __shared__ float red[256];
    float s = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ne; i += (int64_t)gridDim.x * blockDim.x) {
        const float d = pred[i] - target[i];
        s = __builtin_fmaf(d, d, s);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_loss_final(int nb, const float *__restrict__ partial, float inv_ne, float *loss) {
    if (threadIdx.x != 0) return;
    float s = 0.f;
    for (int b = 0; b < nb; ++b) s += partial[b];
    *loss = s * inv_ne;
}

__global__ void k_gather_uv(int64_t ne, const int32_t *__restrict__ cand, const int32_t *__restrict__ u,
                            const int32_t *__restrict__ v, int32_t *cu, int32_t *cv, float *ones) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    const int32_t e = cand ? cand[i] : (int32_t)i;
    cu[i] = u[e];
    cv[i] = v[e];
    ones[i] = 1.f;
}

__global__ void k_fill_f32(int64_t n, float val, float *p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = val;
}

__global__ void k_adam(int64_t n, float *theta, const float *__restrict__ g, float *m, float *v, float lr, float b1,
                       float b2, float c1, float c2, float eps) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    theta[i] = theta[i] - lr * mh / (sqrtf(vh) + eps);
}

// ------------------------------------------------------------------ plans

struct FwdPlan {
    void *a, *h1, *h2;
};

FwdPlan plan_fwd(Carver &c, int64_t n, sfg_dtype act) {
    FwdPlan p;
    const size_t s = dtype_size(act);
    p.a = c.take<char>((size_t)n * kH * s);
    p.h1 = c.take<char>((size_t)n * kH * s);
    p.h2 = c.take<char>((size_t)n * kH * s);
    return p;
}

struct TrainPlan {
    float *a1, *u1, *pre1, *h1, *a2, *u2, *pre2, *h2, *z, *g, *dg, *ah1, *dy, *dhp, *dhq, *dpre2, *t1, *t2, *c2,
        *dpre1, *ones_n, *ones_e, *part, *lpart, *incval, *incdeg;
    int32_t *cu, *cv, *irp, *icol, *ieid;
    void *csr_ws;
};

TrainPlan plan_train(Carver &c, int64_t n, int64_t ne) {
    TrainPlan p;
    p.a1 = c.take<float>(n * kF);
    p.u1 = c.take<float>(n * kU1);
    p.pre1 = c.take<float>(n * kH);
    p.h1 = c.take<float>(n * kH);
    p.a2 = c.take<float>(n * kH);
    p.u2 = c.take<float>(n * kU2);
    p.pre2 = c.take<float>(n * kH);
    p.h2 = c.take<float>(n * kH);
    p.z = c.take<float>((ne + 1) * kZ1);
    p.g = c.take<float>((ne + 1) * kH);
    p.dg = c.take<float>((ne + 1) * kH);
    p.ah1 = c.take<float>((ne + 1) * (kH + 1));
    p.dy = c.take<float>(ne + 1);
    p.dhp = c.take<float>((ne + 1) * kH);
    p.dhq = c.take<float>((ne + 1) * kH);
    p.dpre2 = c.take<float>(n * kH);
    p.t1 = c.take<float>(n * kH);
    p.t2 = c.take<float>(n * kH);
    p.c2 = c.take<float>(n * kH);
    p.dpre1 = c.take<float>(n * kH);
    p.ones_n = c.take<float>(n);
    p.ones_e = c.take<float>(ne + 1);
    p.part = c.take<float>((size_t)kAtbBlocks * kZ1 * kH);
    p.lpart = c.take<float>(256);
    p.incval = c.take<float>(2 * ne + 1);
    p.incdeg = c.take<float>(n);
    p.cu = c.take<int32_t>(ne + 1);
    p.cv = c.take<int32_t>(ne + 1);
    p.irp = c.take<int32_t>(n + 1);
    p.icol = c.take<int32_t>(2 * ne + 1);
    p.ieid = c.take<int32_t>(2 * ne + 1);
    p.csr_ws = c.take<char>(csr_workspace_bytes(n, ne));
    return p;
}

void atb(int64_t nrows, int da, const float *A, int db, const float *B, float *out, float *part, hipStream_t s) {
    hipLaunchKernelGGL(k_atb_partial, dim3(kAtbBlocks), dim3(256), 0, s, nrows, da, A, db, B, part);
    SFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sum_partials, dim3(grid_for(da * db, 256)), dim3(256), 0, s, kAtbBlocks, da * db, part, out);
    SFG_LAUNCH_CHECK();
}

void check_graph(const sfg_csr *G) {
    SFG_REQUIRE(G && G->rowptr && G->col && G->val && G->deg && G->n >= 1, SFG_EINVAL, "mpnn: graph CSR required");
    SFG_REQUIRE(G->vt == SFG_F32, SFG_EUNSUPPORTED, "mpnn: the graph CSR must be F32");
}

}  // namespace

size_t mpnn_forward_workspace_bytes(int64_t n, sfg_dtype act) {
    Carver c(nullptr);
    plan_fwd(c, n, act);
    return c.used + 256;
}

size_t mpnn_train_workspace_bytes(int64_t n, int64_t ne) {
    Carver c(nullptr);
    plan_train(c, n, ne);
    return c.used + 256;
}

}  // namespace sfg

extern "C" int64_t sfg_mpnn_param_count(void) { return sfg::kParams; }

extern "C" sfg_status sfg_mpnn_features(const sfg_csr *G, const sfg_csr *T, const float *xc, int32_t kc, int64_t ne,
                                        const int32_t *cand, const int32_t *u, const int32_t *v, const float *w,
                                        const float *norm, float *node_feat, float *edge_feat, void *stream) {
    return sfg::guard([&] {
        using namespace sfg;
        hipStream_t s = as_stream(stream);
        check_graph(G);
        check_graph(T);
        SFG_REQUIRE(T->n == G->n, SFG_EINVAL, "mpnn_features: G and T must have the same nodes");
        SFG_REQUIRE(xc && kc >= 1 && kc <= 64 && node_feat, SFG_EINVAL, "mpnn_features: bad block");
        SFG_REQUIRE(ne >= 0 && (ne == 0 || (u && v && w && edge_feat)), SFG_EINVAL, "mpnn_features: null pointer");
        const int64_t n = G->n;
        // 4- and 16-vector cheap embeddings with 16-byte aligned rows take vector loads
        const bool aligned = (uintptr_t)xc % 16 == 0 && (uintptr_t)node_feat % 16 == 0;
        const int kv = aligned && (kc == 4 || kc == 16) ? kc : 0;
        auto node = [&](auto kt) {
            constexpr int KC = decltype(kt)::value;
            hipLaunchKernelGGL(k_node_feat<KC>, dim3(grid_for(n, 256)), dim3(256), 0, s, n, G->rowptr, G->col,
                               (const float *)G->val, (const float *)G->deg, T->rowptr, T->col,
                               (const float *)T->val, (const float *)T->deg, xc, kc, norm, node_feat);
            SFG_LAUNCH_CHECK();
            if (ne > 0) {
                hipLaunchKernelGGL(k_edge_feat<KC>, dim3(grid_for(ne, 256)), dim3(256), 0, s, ne, cand, u, v, w, xc,
                                   kc, (const float *)T->deg, norm, edge_feat);
                SFG_LAUNCH_CHECK();
            }
        };
        if (kv == 4)
            node(std::integral_constant<int, 4>());
        else if (kv == 16)
            node(std::integral_constant<int, 16>());
        else
            node(std::integral_constant<int, 0>());
    });
}

extern "C" sfg_status sfg_mpnn_forward(const sfg_csr *G, const float *params, const float *node_feat, int64_t ne,
                                       const int32_t *cand, const int32_t *u, const int32_t *v,
                                       const float *edge_feat, sfg_dtype act, float *pred, void *ws, size_t ws_bytes,
                                       void *stream) {
    return sfg::guard([&] {
        using namespace sfg;
        hipStream_t s = as_stream(stream);
        check_graph(G);
        SFG_REQUIRE(params && node_feat, SFG_EINVAL, "mpnn_forward: null pointer");
        SFG_REQUIRE(act == SFG_F32 || act == SFG_BF16, SFG_EUNSUPPORTED, "mpnn_forward: activations F32 or BF16");
        SFG_REQUIRE(ws_bytes >= mpnn_forward_workspace_bytes(G->n, act), SFG_EWORKSPACE,
                    "mpnn_forward: workspace too small");
        const int64_t n = G->n;
        Carver c(ws);
        FwdPlan p = plan_fwd(c, n, act);
        const dim3 gn(grid_for(n, 256)), b(256);
        // layer 1 (FP32 input features; the aggregate reuses p.a)
        float *a1 = (float *)p.a;
        spmm_rownorm(G, kF, SFG_F32, node_feat, a1, s);
        if (act == SFG_F32)
            hipLaunchKernelGGL((k_dense_fwd<float, float, kF>), gn, b, 0, s, n, node_feat, a1, params + kOffW1,
                               (float *)p.h1, nullptr, nullptr);
        else
            hipLaunchKernelGGL((k_dense_mfma<float, kF>), dim3(grid_for(n, 128)), b, 0, s, n, node_feat, a1,
                               params + kOffW1, (__hip_bfloat16 *)p.h1);
        SFG_LAUNCH_CHECK();
        // layer 2
        spmm_rownorm(G, kH, act, p.h1, p.a, s);
        if (act == SFG_F32)
            hipLaunchKernelGGL((k_dense_fwd<float, float, kH>), gn, b, 0, s, n, (const float *)p.h1,
                               (const float *)p.a, params + kOffW2, (float *)p.h2, nullptr, nullptr);
        else
            hipLaunchKernelGGL((k_dense_mfma<__hip_bfloat16, kH>), dim3(grid_for(n, 128)), b, 0, s, n,
                               (const __hip_bfloat16 *)p.h1, (const __hip_bfloat16 *)p.a, params + kOffW2,
                               (__hip_bfloat16 *)p.h2);
        SFG_LAUNCH_CHECK();
        if (ne == 0) return;
        SFG_REQUIRE(u && v && edge_feat && pred, SFG_EINVAL, "mpnn_forward: null pointer");
        const dim3 ge(grid_for(ne, 256));
        if (act == SFG_F32)
            hipLaunchKernelGGL(k_head_fwd<float>, ge, b, 0, s, ne, cand, u, v, (const float *)p.h2, edge_feat,
                               params + kOffW3, params + kOffW4, pred, nullptr, nullptr);
        else
            hipLaunchKernelGGL(k_head_mfma, dim3(grid_for(ne, 128)), b, 0, s, ne, cand, u, v,
                               (const __hip_bfloat16 *)p.h2, edge_feat, params + kOffW3, params + kOffW4, pred);
        SFG_LAUNCH_CHECK();
    });
}

extern "C" sfg_status sfg_mpnn_loss_grad(const sfg_csr *G, const float *params, const float *node_feat, int64_t ne,
                                         const int32_t *cand, const int32_t *u, const int32_t *v,
                                         const float *edge_feat, const float *target, float *pred, float *loss,
                                         float *grad, void *ws, size_t ws_bytes, void *stream) {
    return sfg::guard([&] {
        using namespace sfg;
        hipStream_t s = as_stream(stream);
        check_graph(G);
        SFG_REQUIRE(ne >= 1, SFG_EINVAL, "mpnn_loss_grad: need at least one edge");
        SFG_REQUIRE(params && node_feat && u && v && edge_feat && target && pred && loss && grad, SFG_EINVAL,
                    "mpnn_loss_grad: null pointer");
        const int64_t n = G->n;
        SFG_REQUIRE(ws_bytes >= mpnn_train_workspace_bytes(n, ne), SFG_EWORKSPACE,
                    "mpnn_loss_grad: workspace too small");
        Carver c(ws);
        TrainPlan p = plan_train(c, n, ne);
        const dim3 gn(grid_for(n, 256)), ge(grid_for(ne, 256)), b(256);
        // ---- forward, keeping what the backward needs
        spmm_rownorm(G, kF, SFG_F32, node_feat, p.a1, s);
        hipLaunchKernelGGL((k_dense_fwd<float, float, kF>), gn, b, 0, s, n, node_feat, p.a1, params + kOffW1, p.h1,
                           p.pre1, p.u1);
        SFG_LAUNCH_CHECK();
        spmm_rownorm(G, kH, SFG_F32, p.h1, p.a2, s);
        hipLaunchKernelGGL((k_dense_fwd<float, float, kH>), gn, b, 0, s, n, p.h1, p.a2, params + kOffW2, p.h2, p.pre2,
                           p.u2);
        SFG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_head_fwd<float>, ge, b, 0, s, ne, cand, u, v, p.h2, edge_feat, params + kOffW3,
                           params + kOffW4, pred, p.g, p.z);
        SFG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_sq_err_partial, dim3(256), b, 0, s, ne, pred, target, p.lpart);
        SFG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, 256, p.lpart, 1.f / (float)ne, loss);
        SFG_LAUNCH_CHECK();
        // ---- backward: edge head
        hipLaunchKernelGGL(k_head_bwd, ge, b, 0, s, ne, cand, u, v, p.h2, pred, target, p.g, params + kOffW3,
                           params + kOffW4, 2.f / (float)ne, p.dg, p.ah1, p.dy, p.dhp, p.dhq);
        SFG_LAUNCH_CHECK();
        atb(ne, kZ1, p.z, kH, p.dg, grad + kOffW3, p.part, s);
        atb(ne, kH + 1, p.ah1, 1, p.dy, grad + kOffW4, p.part, s);
        // edge gradients to nodes through the incidence CSR of the candidate edges
        hipLaunchKernelGGL(k_gather_uv, ge, b, 0, s, ne, cand, u, v, p.cu, p.cv, p.ones_e);
        SFG_LAUNCH_CHECK();
        build_csr(n, ne, p.cu, p.cv, p.ones_e, SFG_F32, nullptr, p.irp, p.icol, p.incval, p.ieid, p.incdeg, p.csr_ws,
                  csr_workspace_bytes(n, ne), s);
        hipLaunchKernelGGL(k_gather_dh, gn, b, 0, s, n, p.irp, p.icol, p.ieid, p.dhp, p.dhq, p.pre2, p.dpre2);
        SFG_LAUNCH_CHECK();
        // ---- layer 2
        atb(n, kU2, p.u2, kH, p.dpre2, grad + kOffW2, p.part, s);
        hipLaunchKernelGGL((k_dense_bwd<kH>), gn, b, 0, s, n, p.dpre2, params + kOffW2, (const float *)G->deg, p.t1,
                           p.t2);
        SFG_LAUNCH_CHECK();
        // A (dP Wn^T / D): the sweep with unit degrees is the plain product
        hipLaunchKernelGGL(k_fill_f32, gn, b, 0, s, n, 1.f, p.ones_n);
        SFG_LAUNCH_CHECK();
        sfg_csr Gu = *G;
        Gu.deg = p.ones_n;
        spmm_rownorm(&Gu, kH, SFG_F32, p.t2, p.c2, s);
        hipLaunchKernelGGL(k_add_mask, dim3(grid_for(n * kH, 256)), b, 0, s, n * kH, p.t1, p.c2, p.pre1, p.dpre1);
        SFG_LAUNCH_CHECK();
        // ---- layer 1
        atb(n, kU1, p.u1, kH, p.dpre1, grad + kOffW1, p.part, s);
    });
}

extern "C" sfg_status sfg_mpnn_adam(float *params, const float *grad, float *m, float *v, int64_t n, int64_t step,
                                    double lr, double beta1, double beta2, double eps, void *stream) {
    return sfg::guard([&] {
        using namespace sfg;
        SFG_REQUIRE(params && grad && m && v && n >= 1 && step >= 1, SFG_EINVAL, "mpnn_adam: bad arguments");
        const float c1 = (float)(1.0 - std::pow(beta1, (double)step));
        const float c2 = (float)(1.0 - std::pow(beta2, (double)step));
        hipLaunchKernelGGL(k_adam, dim3(grid_for(n, 256)), dim3(256), 0, as_stream(stream), n, params, grad, m, v,
                           (float)lr, (float)beta1, (float)beta2, c1, c2, (float)eps);
        SFG_LAUNCH_CHECK();
    });
}
