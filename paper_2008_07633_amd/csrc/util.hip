// Shared device routines: exclusive scan of int32 counts, fills, last-error.
#include "common.hpp"

namespace sfg {

static thread_local std::string g_last_error;

void set_last_error(const std::string &msg) { g_last_error = msg; }
void clear_last_error() { g_last_error.clear(); }
const char *last_error_cstr() { return g_last_error.c_str(); }

// ------------------------------------------------------------------ scan
// Three passes: tile sums, one-block scan of the tile sums, tile rescans.
// A tile is 256 threads x 8 items.  Integer adds, so the result does not
// depend on the association order.  Global loads and stores are striped
// (item i of a thread at tile offset i 256 + thread), so every instruction
// covers 256 contiguous bytes; the rescan turns them into per-thread runs of 8
// consecutive items through LDS.

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int kScanSumItems = 16;   // tile sums per thread in the one-block scan

__device__ __forceinline__ int32_t wave_incl_scan(int32_t x) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int32_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

// Block-wide exclusive scan of one value per thread; returns the block total
// through `total`.  Its barriers also order every LDS access a thread made
// before the call ahead of any access made after it by another thread.
__device__ __forceinline__ int32_t block_excl_scan(int32_t x, int32_t &total) {
    __shared__ int32_t wsum[kScanThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    int32_t inc = wave_incl_scan(x);
    if (lane == kWave - 1) wsum[wid] = inc;
    __syncthreads();
    int32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        if (w < wid) off += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    total = tot;
    return off + inc - x;
}

__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const int32_t *in, int64_t n, int32_t *tsum) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
    int32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i * kScanThreads < n) s += in[base + i * kScanThreads];
    int32_t tot;
    block_excl_scan(s, tot);
    if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

// One workgroup; thread t scans tile sums t kScanSumItems .. + kScanSumItems - 1
// of each round of 256 kScanSumItems.
__global__ __launch_bounds__(kScanThreads) void k_scan_tile_sums(int32_t *tsum, int64_t nt, int32_t *grand) {
    int32_t carry = 0;
    for (int64_t base = 0; base < nt; base += kScanThreads * kScanSumItems) {
        const int64_t b0 = base + (int64_t)threadIdx.x * kScanSumItems;
        int32_t v[kScanSumItems];
        int32_t s = 0;
#pragma unroll
        for (int j = 0; j < kScanSumItems; ++j) {
            v[j] = b0 + j < nt ? tsum[b0 + j] : 0;
            s += v[j];
        }
        int32_t tot;
        int32_t run = carry + block_excl_scan(s, tot);
#pragma unroll
        for (int j = 0; j < kScanSumItems; ++j) {
            if (b0 + j < nt) tsum[b0 + j] = run;
            run += v[j];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) *grand = carry;
}

// LDS index of tile item i, one pad word per 32 against bank conflicts of the
// per-thread runs.
__device__ __forceinline__ int scan_pad(int i) { return i + (i >> 5); }

__global__ __launch_bounds__(kScanThreads) void k_tile_rescan(const int32_t *in, int32_t *out, int64_t n,
                                                              const int32_t *tsum, const int32_t *grand) {
    __shared__ int32_t sh[kScanTile + kScanTile / 32];
    const int t = threadIdx.x;
    const int64_t tile0 = (int64_t)blockIdx.x * kScanTile;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = tile0 + i * kScanThreads + t;
        sh[scan_pad(i * kScanThreads + t)] = idx < n ? in[idx] : 0;
    }
    __syncthreads();
    int32_t v[kScanItems];
    int32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = sh[scan_pad(t * kScanItems + j)];
        s += v[j];
    }
    int32_t tot;
    int32_t ex = block_excl_scan(s, tot) + tsum[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        sh[scan_pad(t * kScanItems + j)] = ex;
        ex += v[j];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = tile0 + i * kScanThreads + t;
        if (idx < n) out[idx] = sh[scan_pad(i * kScanThreads + t)];
    }
    if (blockIdx.x == 0 && t == 0) out[n] = *grand;
}

size_t scan_scratch_ints(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 2; }

void exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *scratch, hipStream_t s) {
    const int64_t nt = (n + kScanTile - 1) / kScanTile;
    int32_t *grand = scratch + nt + 1;
    if (n == 0) {
        fill_i32(out, 1, 0, s);
        return;
    }
    hipLaunchKernelGGL(k_tile_sums, dim3((uint32_t)nt), dim3(kScanThreads), 0, s, in, n, scratch);
    SFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_tile_sums, dim3(1), dim3(kScanThreads), 0, s, scratch, nt, grand);
    SFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_tile_rescan, dim3((uint32_t)nt), dim3(kScanThreads), 0, s, in, out, n, scratch, grand);
    SFG_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ fills

template <typename T>
__global__ void k_fill(T *p, int64_t n, T v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

void fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    SFG_LAUNCH_CHECK();
}

void fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<uint8_t>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    SFG_LAUNCH_CHECK();
}

}  // namespace sfg

extern "C" const char *sfg_last_error(void) { return sfg::last_error_cstr(); }
