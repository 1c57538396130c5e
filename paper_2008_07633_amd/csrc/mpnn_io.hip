// Learned surrogate (not in the paper): model files and the standardisation
// of its training set.
//
// Model file, version 1, little-endian:
//   bytes 0..7    magic "SFGMPNN1"
//   8..11         uint32 version (1)
//   12..15        uint32 parameter count (sfg_mpnn_param_count())
//   16..19        uint32 normalisation count (24)
//   20..23        int32 kc (cheap-embedding vectors, 1..64)
//   24..27        int32 tc (cheap-embedding sweeps, 0..1000)
//   28..31        uint32 0
//   32..39        double target mean; 40..47 double target standard deviation
//   48..          float parameters, then float normalisation
//   last 8 bytes  uint64 FNV-1a hash (64-bit, Fowler-Noll-Vo) of every byte before it
//
// Standardisation: FP64 column sums over all rows of all graphs, one
// workgroup per column with a fixed-shape reduction and the graphs added in
// order, so the result does not depend on timing; two passes (means, then
// squared deviations from them).
#include <cmath>
#include <cstdio>
#include <vector>

#include "common.hpp"

namespace sfg {

namespace {

constexpr char kMagic[8] = {'S', 'F', 'G', 'M', 'P', 'N', 'N', '1'};
constexpr uint32_t kVersion = 1;
constexpr uint32_t kNormCount = 24;
constexpr size_t kHeader = 48;
constexpr int kNodeF = 8, kEdgeF = 4;

uint64_t fnv1a64(const unsigned char *p, size_t n) {
    uint64_t h = 0xcbf29ce484222325ull;   // FNV-1a 64-bit offset basis and prime
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

template <typename T>
void put(std::vector<unsigned char> &b, size_t off, T v) {
    std::memcpy(b.data() + off, &v, sizeof(T));
}
template <typename T>
T get(const std::vector<unsigned char> &b, size_t off) {
    T v;
    std::memcpy(&v, b.data() + off, sizeof(T));
    return v;
}

// ------------------------------------------------------------------ standardisation kernels

constexpr int kMomThreads = 256;

// acc[c] += sum over rows of x[r][c] (mean == nullptr) or of (x[r][c] - mean[c])^2, in FP64.  One workgroup
// per column; thread t takes rows t, t + 256, ...; the partial sums meet in a fixed LDS tree.
__global__ __launch_bounds__(kMomThreads) void k_col_moment(const float *__restrict__ x, int64_t rows, int32_t cols,
                                                            const double *__restrict__ mean, double *acc) {
    __shared__ double part[kMomThreads];
    const int c = blockIdx.x, t = threadIdx.x;
    const double m = mean ? mean[c] : 0.0;
    double s = 0.0;
    for (int64_t r = t; r < rows; r += kMomThreads) {
        const double d = (double)x[r * cols + c] - m;
        s += mean ? d * d : d;
    }
    part[t] = s;
    __syncthreads();
    for (int st = kMomThreads / 2; st > 0; st >>= 1) {
        if (t < st) part[t] += part[t + st];
        __syncthreads();
    }
    if (t == 0) acc[c] += part[0];
}

__global__ void k_zero_f64(double *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0.0;
}

// Slots: sums and squared deviations of 8 node features, 4 edge features and the target (13 each).
constexpr int kCols = kNodeF + kEdgeF + 1;

__global__ void k_means(const double *__restrict__ sum, double n_node, double n_edge, double *mean) {
    const int j = threadIdx.x;
    if (j < kCols) mean[j] = sum[j] / (j < kNodeF ? n_node : n_edge);
}

// norm = [node means | node inverse deviations | edge means | edge inverse deviations]; node feature 0
// (the constant 1) keeps mean 0 and scale 1; deviations are floored at 1e-6.  ystat = target mean,
// deviation (1 where the targets are all equal).
__global__ void k_norm_final(const double *__restrict__ mean, const double *__restrict__ sq, double n_node,
                             double n_edge, float *norm, double *ystat) {
    const int j = threadIdx.x;
    if (j >= kCols) return;
    const bool node = j < kNodeF;
    const double sd = sqrt(sq[j] / (node ? n_node : n_edge));
    if (node) {
        norm[j] = j == 0 ? 0.f : (float)mean[j];
        norm[kNodeF + j] = j == 0 ? 1.f : (float)(1.0 / fmax(sd, 1e-6));
    } else if (j < kNodeF + kEdgeF) {
        const int e = j - kNodeF;
        norm[2 * kNodeF + e] = (float)mean[j];
        norm[2 * kNodeF + kEdgeF + e] = (float)(1.0 / fmax(sd, 1e-6));
    } else {
        ystat[0] = mean[j];
        ystat[1] = sd > 0.0 ? sd : 1.0;
    }
}

__global__ void k_standardize(int64_t n, const float *__restrict__ y, const double *__restrict__ ystat,
                              float *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)(((double)y[i] - ystat[0]) / ystat[1]);
}

}  // namespace

}  // namespace sfg

extern "C" sfg_status sfg_mpnn_save(const char *path, const float *params, const float *norm,
                                    const sfg_mpnn_meta *meta, void *stream) {
    return sfg::guard([&] {
        using namespace sfg;
        SFG_REQUIRE(path && params && norm && meta, SFG_EINVAL, "mpnn_save: null pointer");
        SFG_REQUIRE(meta->kc >= 1 && meta->kc <= 64 && meta->tc >= 0 && meta->tc <= 1000, SFG_EINVAL,
                    "mpnn_save: cheap embedding out of range (kc 1..64, tc 0..1000)");
        const uint32_t np = (uint32_t)sfg_mpnn_param_count();
        const size_t body = kHeader + 4 * (size_t)(np + kNormCount);
        std::vector<unsigned char> b(body + 8, 0);
        std::memcpy(b.data(), kMagic, 8);
        put<uint32_t>(b, 8, kVersion);
        put<uint32_t>(b, 12, np);
        put<uint32_t>(b, 16, kNormCount);
        put<int32_t>(b, 20, meta->kc);
        put<int32_t>(b, 24, meta->tc);
        put<double>(b, 32, meta->y_mean);
        put<double>(b, 40, meta->y_std);
        hipStream_t s = as_stream(stream);
        SFG_HIP(hipMemcpyAsync(b.data() + kHeader, params, 4 * (size_t)np, hipMemcpyDeviceToHost, s));
        SFG_HIP(hipMemcpyAsync(b.data() + kHeader + 4 * (size_t)np, norm, 4 * (size_t)kNormCount,
                               hipMemcpyDeviceToHost, s));
        SFG_HIP(hipStreamSynchronize(s));
        put<uint64_t>(b, body, fnv1a64(b.data(), body));
        FILE *f = std::fopen(path, "wb");
        SFG_REQUIRE(f, SFG_EINVAL, std::string("mpnn_save: cannot open ") + path);
        const size_t wrote = std::fwrite(b.data(), 1, b.size(), f);
        const int closed = std::fclose(f);
        SFG_REQUIRE(wrote == b.size() && closed == 0, SFG_EINVAL, std::string("mpnn_save: cannot write ") + path);
    });
}

extern "C" sfg_status sfg_mpnn_load(const char *path, float *params, float *norm, sfg_mpnn_meta *meta,
                                    void *stream) {
    return sfg::guard([&] {
        using namespace sfg;
        SFG_REQUIRE(path && params && norm && meta, SFG_EINVAL, "mpnn_load: null pointer");
        FILE *f = std::fopen(path, "rb");
        SFG_REQUIRE(f, SFG_EINVAL, std::string("mpnn_load: cannot open ") + path);
        std::vector<unsigned char> b;
        unsigned char chunk[4096];
        size_t got;
        while ((got = std::fread(chunk, 1, sizeof(chunk), f)) > 0) b.insert(b.end(), chunk, chunk + got);
        std::fclose(f);
        const uint32_t np = (uint32_t)sfg_mpnn_param_count();
        SFG_REQUIRE(b.size() >= kHeader + 8 && std::memcmp(b.data(), kMagic, 8) == 0, SFG_EINVAL,
                    "mpnn_load: not a surrogate model file");
        const uint32_t ver = get<uint32_t>(b, 8);
        SFG_REQUIRE(ver == kVersion, SFG_EINVAL,
                    "mpnn_load: model file version " + std::to_string(ver) + ", expected " + std::to_string(kVersion));
        SFG_REQUIRE(get<uint32_t>(b, 12) == np && get<uint32_t>(b, 16) == kNormCount, SFG_EINVAL,
                    "mpnn_load: the model has the wrong shapes");
        const size_t body = kHeader + 4 * (size_t)(np + kNormCount);
        SFG_REQUIRE(b.size() == body + 8, SFG_EINVAL, "mpnn_load: the model file has the wrong length");
        SFG_REQUIRE(get<uint64_t>(b, body) == fnv1a64(b.data(), body), SFG_EINVAL, "mpnn_load: checksum mismatch");
        sfg_mpnn_meta m;
        m.kc = get<int32_t>(b, 20);
        m.tc = get<int32_t>(b, 24);
        m.y_mean = get<double>(b, 32);
        m.y_std = get<double>(b, 40);
        SFG_REQUIRE(m.kc >= 1 && m.kc <= 64 && m.tc >= 0 && m.tc <= 1000, SFG_EINVAL,
                    "mpnn_load: bad cheap embedding (" + std::to_string(m.kc) + " vectors, " + std::to_string(m.tc) +
                        " sweeps)");
        bool finite = std::isfinite(m.y_mean) && std::isfinite(m.y_std);
        for (size_t i = 0; i < (size_t)(np + kNormCount); ++i) finite = finite && std::isfinite(get<float>(b, kHeader + 4 * i));
        SFG_REQUIRE(finite, SFG_EINVAL, "mpnn_load: the model holds non-finite values");
        hipStream_t s = as_stream(stream);
        SFG_HIP(hipMemcpyAsync(params, b.data() + kHeader, 4 * (size_t)np, hipMemcpyHostToDevice, s));
        SFG_HIP(hipMemcpyAsync(norm, b.data() + kHeader + 4 * (size_t)np, 4 * (size_t)kNormCount,
                               hipMemcpyHostToDevice, s));
        SFG_HIP(hipStreamSynchronize(s));
        *meta = m;
    });
}

extern "C" sfg_status sfg_mpnn_fit_norm(int32_t ngraphs, const float *const *node_feat, const int64_t *node_rows,
                                        const float *const *edge_feat, const float *const *target,
                                        const int64_t *edge_rows, float *norm, double *ystat, void *ws,
                                        size_t ws_bytes, void *stream) {
    return sfg::guard([&] {
        using namespace sfg;
        SFG_REQUIRE(ngraphs >= 1 && node_feat && node_rows && edge_feat && target && edge_rows && norm && ystat,
                    SFG_EINVAL, "mpnn_fit_norm: null pointer or no graphs");
        SFG_REQUIRE(ws && ws_bytes >= sfg_workspace_bytes(SFG_OP_MPNN_NORM, 0, 0, 0, SFG_F64), SFG_EWORKSPACE,
                    "mpnn_fit_norm: workspace too small");
        double nn = 0.0, ne = 0.0;
        for (int32_t i = 0; i < ngraphs; ++i) {
            SFG_REQUIRE(node_rows[i] >= 1 && edge_rows[i] >= 1 && node_feat[i] && edge_feat[i] && target[i],
                        SFG_EINVAL, "mpnn_fit_norm: every graph needs nodes, edges and its three arrays");
            nn += (double)node_rows[i];
            ne += (double)edge_rows[i];
        }
        hipStream_t s = as_stream(stream);
        double *sum = (double *)ws, *mean = sum + 16, *sq = sum + 32;
        hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(64), 0, s, sum, 48);
        SFG_LAUNCH_CHECK();
        for (int pass = 0; pass < 2; ++pass) {
            const double *m = pass ? mean : nullptr;
            double *acc = pass ? sq : sum;
            for (int32_t i = 0; i < ngraphs; ++i) {
                hipLaunchKernelGGL(k_col_moment, dim3(kNodeF), dim3(kMomThreads), 0, s, node_feat[i], node_rows[i],
                                   kNodeF, m, acc);
                hipLaunchKernelGGL(k_col_moment, dim3(kEdgeF), dim3(kMomThreads), 0, s, edge_feat[i], edge_rows[i],
                                   kEdgeF, m ? m + kNodeF : nullptr, acc + kNodeF);
                hipLaunchKernelGGL(k_col_moment, dim3(1), dim3(kMomThreads), 0, s, target[i], edge_rows[i], 1,
                                   m ? m + kNodeF + kEdgeF : nullptr, acc + kNodeF + kEdgeF);
                SFG_LAUNCH_CHECK();
            }
            if (pass == 0) {
                hipLaunchKernelGGL(k_means, dim3(1), dim3(64), 0, s, sum, nn, ne, mean);
                SFG_LAUNCH_CHECK();
            }
        }
        hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(64), 0, s, mean, sq, nn, ne, norm, ystat);
        SFG_LAUNCH_CHECK();
    });
}

extern "C" sfg_status sfg_mpnn_standardize(const float *y, int64_t n, const double *ystat, float *out, void *stream) {
    return sfg::guard([&] {
        using namespace sfg;
        SFG_REQUIRE(n >= 0 && ystat && (n == 0 || (y && out)), SFG_EINVAL, "mpnn_standardize: bad arguments");
        if (n == 0) return;
        hipLaunchKernelGGL(k_standardize, dim3(grid_for(n, 256)), dim3(256), 0, as_stream(stream), n, y, ystat, out);
        SFG_LAUNCH_CHECK();
    });
}
