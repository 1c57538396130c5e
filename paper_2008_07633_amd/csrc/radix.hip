// Stable least-significant-digit radix sort of (uint64 key, int32 value)
// pairs, 8-bit digits, only over the digit positions the caller names.
//
// Per pass: every 4096-key tile counts its digits in LDS; one exclusive scan
// over the digit-major [digit][tile] table gives each (digit, tile) its
// output base; the tile is then re-read in 16 rounds of 256 keys, and each
// key's rank among equal digits is taken from wavefront ballots (lanes with
// the same digit) plus per-wave counts in LDS, so equal keys keep their
// input order.  Integer counting only: the result is deterministic.
#include "common.hpp"

namespace sfg {

namespace {

constexpr int kRThreads = 256;
constexpr int kRRounds = 16;
constexpr int kRTile = kRThreads * kRRounds;
constexpr int kRWaves = kRThreads / kWave;

__global__ __launch_bounds__(kRThreads) void k_radix_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                          int32_t *hist, int32_t nb) {
    __shared__ int32_t h[256];
    const int t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRTile;
    for (int r = 0; r < kRRounds; ++r) {
        const int64_t i = base + (int64_t)r * kRThreads + t;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[(int64_t)t * nb + blockIdx.x] = h[t];
}

__global__ __launch_bounds__(kRThreads) void k_radix_scatter(const uint64_t *__restrict__ kin,
                                                             const int32_t *__restrict__ vin, uint64_t *kout,
                                                             int32_t *vout, int64_t n, int shift,
                                                             const int32_t *__restrict__ offs, int32_t nb) {
    __shared__ int32_t run[256];
    __shared__ int32_t wc[kRWaves][256];
    const int t = threadIdx.x, lane = t & (kWave - 1), wid = t / kWave;
    run[t] = offs[(int64_t)t * nb + blockIdx.x];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kRTile;
    for (int r = 0; r < kRRounds; ++r) {
#pragma unroll
        for (int w = 0; w < kRWaves; ++w) wc[w][t] = 0;
        __syncthreads();
        const int64_t i = base + (int64_t)r * kRThreads + t;
        const bool valid = i < n;
        uint64_t key = 0;
        int32_t val = 0;
        int d = 256;                     // out-of-range lanes form their own group
        if (valid) {
            key = kin[i];
            val = vin[i];
            d = (int)((key >> shift) & 255);
        }
        uint64_t peers = ~0ull;
#pragma unroll
        for (int bit = 0; bit < 9; ++bit) {
            const bool on = (d >> bit) & 1;
            const uint64_t bal = __ballot(on);
            peers &= on ? bal : ~bal;
        }
        const int rank = __popcll(peers & lt);
        if (valid && rank == 0) wc[wid][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int32_t pos = run[d] + rank;
            for (int w = 0; w < wid; ++w) pos += wc[w][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        int32_t add = 0;
#pragma unroll
        for (int w = 0; w < kRWaves; ++w) add += wc[w][t];
        run[t] += add;
        __syncthreads();
    }
}

}  // namespace

size_t radix_scratch_bytes(int64_t n) {
    const int64_t nb = (n + kRTile - 1) / kRTile;
    Carver c(nullptr);
    c.take<uint64_t>(n + 1);
    c.take<int32_t>(n + 1);
    c.take<int32_t>(256 * nb + 1);
    c.take<int32_t>(256 * nb + 1);
    c.take<int32_t>(scan_scratch_ints(256 * nb + 1));
    return c.used + 256;
}

// Sort in place (keys/vals hold the result).  `shifts` lists the digit
// positions (multiples of 8), least significant first.
void radix_sort_pairs(uint64_t *keys, int32_t *vals, int64_t n, const int *shifts, int nshift, void *scratch,
                      hipStream_t s) {
    if (n <= 1 || nshift == 0) return;
    const int64_t nb = (n + kRTile - 1) / kRTile;
    Carver c(scratch);
    uint64_t *ktmp = c.take<uint64_t>(n + 1);
    int32_t *vtmp = c.take<int32_t>(n + 1);
    int32_t *hist = c.take<int32_t>(256 * nb + 1);
    int32_t *offs = c.take<int32_t>(256 * nb + 1);
    int32_t *scr = c.take<int32_t>(scan_scratch_ints(256 * nb + 1));
    uint64_t *ka = keys, *kb = ktmp;
    int32_t *va = vals, *vb = vtmp;
    for (int p = 0; p < nshift; ++p) {
        hipLaunchKernelGGL(k_radix_hist, dim3((uint32_t)nb), dim3(kRThreads), 0, s, ka, n, shifts[p], hist,
                           (int32_t)nb);
        SFG_LAUNCH_CHECK();
        exclusive_scan_i32(hist, offs, 256 * nb, scr, s);
        hipLaunchKernelGGL(k_radix_scatter, dim3((uint32_t)nb), dim3(kRThreads), 0, s, ka, va, kb, vb, n, shifts[p],
                           offs, (int32_t)nb);
        SFG_LAUNCH_CHECK();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        SFG_HIP(hipMemcpyAsync(keys, ka, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        SFG_HIP(hipMemcpyAsync(vals, va, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
}

}  // namespace sfg
