// Top-k selection of edge scores (Alg. 1: "include top few edges with large
// distortion"): order by score descending, then position ascending, keep the
// first k.
//
// IEEE values map to unsigned keys that order like the values, so the k-th
// largest key is found by most-significant-digit radix select: per pass, a
// histogram (LDS, integer atomics) of the keys that still match the digits
// fixed so far, then one workgroup picks the digit that contains rank k.
// Passes stay on the device (no host round trips).  The third pass also
// copies the keys that match its prefix (two digits fixed: normally a tiny
// share) to a buffer, and the later passes read that buffer instead of the
// scores.  Ties at the threshold take the lowest positions: when the last
// digit's bucket is taken whole (the usual case) the keys >= the threshold
// are kept; otherwise per-tile tie counts, their scan, and a scan inside each
// tile give every tied key its rank.
#include <mutex>

#include "common.hpp"

// Scratch of sfg_select_topk_noalloc: a device array of fixed size, one copy
// per GPU, held until the process ends.  In host code this name stands for a
// host-side shadow, not a device address: host code only ever passes it to
// hipGetSymbolAddress and uses the address that returns.
static __device__ __align__(256) unsigned char scratch[sfg::kSelectNoallocBytes];

namespace sfg {

namespace {

constexpr int kBins = 2048;
constexpr int kHistThreads = 256;
// The global histogram is kept in one copy per XCD (a workgroup adds into copy
// blockIdx % kHistCopies), so the device-scope atomics of the workgroups'
// flushes spread over kHistCopies times as many addresses; the pick adds the
// copies.
constexpr int kHistCopies = kNumXcd;

constexpr int kTieTile = 4096;       // keys per workgroup in the tie count and the marking
constexpr int kCompactPass = 2;      // the pass (0-based) that copies its matching keys to the buffer

struct SelState {
    uint64_t prefix;
    uint64_t fixed;
    int64_t krem;      // rank (1-based) still sought inside the current bucket
    int64_t count_gt;  // keys known to be larger than the bucket
    uint64_t ncopy;    // keys copied to the buffer by the compacting pass
    uint32_t err;
    uint32_t all_ties; // the last pick takes every key equal to the threshold
};

template <typename TS> struct KeyOf;
template <> struct KeyOf<double> {
    using K = uint64_t;
    static constexpr int bits = 64;
};
template <> struct KeyOf<float> {
    using K = uint32_t;
    static constexpr int bits = 32;
};

// Order-preserving map of IEEE values to unsigned keys: negative values have
// all bits flipped, non-negative ones only the sign bit.
template <typename TS>
__device__ __forceinline__ typename KeyOf<TS>::K raw_bits(TS x) {
    typename KeyOf<TS>::K k;
    __builtin_memcpy(&k, &x, sizeof(k));
    return k;
}

template <typename TS>
__device__ __forceinline__ typename KeyOf<TS>::K key_of(TS x) {
    using K = typename KeyOf<TS>::K;
    const K sign = K(1) << (KeyOf<TS>::bits - 1);
    const K b = raw_bits(x);
    return (b & sign) ? ~b : (b | sign);
}

template <typename TS>
__device__ __forceinline__ TS value_of(typename KeyOf<TS>::K k) {
    using K = typename KeyOf<TS>::K;
    const K sign = K(1) << (KeyOf<TS>::bits - 1);
    const K b = (k & sign) ? (k & ~sign) : ~k;
    TS x;
    __builtin_memcpy(&x, &b, sizeof(x));
    return x;
}

template <typename TS>
__device__ __forceinline__ bool is_nan_bits(typename KeyOf<TS>::K k) {
    using K = typename KeyOf<TS>::K;
    constexpr int B = KeyOf<TS>::bits;
    constexpr int mant = (B == 64) ? 52 : 23;
    const K expmask = ((K(1) << (B - 1 - mant)) - 1) << mant;
    return ((k & expmask) == expmask) && (k & ((K(1) << mant) - 1));
}

__global__ void k_sel_init(SelState *st, int64_t k, uint32_t *hist) {
    if (threadIdx.x == 0) {
        st->prefix = 0;
        st->fixed = 0;
        st->krem = k;
        st->count_gt = 0;
        st->ncopy = 0;
        st->err = 0;
        st->all_ties = 0;
    }
    for (int b = threadIdx.x; b < kBins * kHistCopies; b += blockDim.x) hist[b] = 0;
}

// One radix pass.  FROM_BUF: read the keys the compacting pass copied (their
// count is st->ncopy) instead of the scores.  copy != nullptr: append the
// keys that match the prefix to copy[] (one atomic per wavefront).
template <typename TS, bool FROM_BUF>
__global__ __launch_bounds__(kHistThreads) void k_sel_hist(int64_t ne, const TS *__restrict__ score,
                                                           const typename KeyOf<TS>::K *__restrict__ buf,
                                                           SelState *st, int shift, int width, int check,
                                                           uint32_t *hist, typename KeyOf<TS>::K *copy) {
    using K = typename KeyOf<TS>::K;
    __shared__ uint32_t h[kBins];
    for (int b = threadIdx.x; b < kBins; b += blockDim.x) h[b] = 0;
    __syncthreads();
    const K prefix = (K)st->prefix, fixed = (K)st->fixed;
    const K dmask = (K(1) << width) - 1;
    const int64_t cnt = FROM_BUF ? (int64_t)st->ncopy : ne;
    const int lane = threadIdx.x % kWave;
    uint32_t bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x) {
        K key;
        if (FROM_BUF) {
            key = buf[i];
        } else {
            const TS sv = score[i];
            if (check) bad |= is_nan_bits<TS>(raw_bits(sv)) ? 1u : 0u;
            key = key_of(sv);
        }
        const bool match = (key & fixed) == prefix;
        if (match) atomicAdd(&h[(key >> shift) & dmask], 1u);
        if (copy) {
            const uint64_t bal = __ballot(match);
            if (bal) {
                const int leader = __ffsll((unsigned long long)bal) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd((unsigned long long *)&st->ncopy, (unsigned long long)__popcll(bal));
                base = __shfl(base, leader, kWave);
                if (match) copy[base + __popcll(bal & ((uint64_t(1) << lane) - 1))] = key;
            }
        }
    }
    if (bad) atomicOr(&st->err, 1u);   // NaN
    __syncthreads();
    uint32_t *hc = hist + (blockIdx.x % kHistCopies) * kBins;
    for (int b = threadIdx.x; b < kBins; b += blockDim.x)
        if (h[b]) atomicAdd(&hc[b], h[b]);
}

// One workgroup of 256 threads, 8 bins each; finds the digit holding rank
// krem counted from the top, updates the state and clears the histogram.
// The copies' counts are first added into LDS by coalesced loads (bin b by
// thread b % 256), and cleared the same way at the end.
__global__ __launch_bounds__(256) void k_sel_pick(SelState *st, uint32_t *hist, int shift, int width, int last) {
    __shared__ int64_t suffix[257];
    __shared__ uint32_t cnt[kBins];
    const int t = threadIdx.x;
    const int nb = 1 << width;
    const int per = (nb + 255) / 256;
    // Every thread reads the sought rank before the first barrier; the one
    // thread that updates the state below does so only after the scan's
    // barriers, so no thread can see its new value.
    const int64_t krem = st->krem;
#pragma unroll
    for (int i = 0; i < kBins / 256; ++i) {
        const int b = i * 256 + t;
        if (b < nb) {
            uint32_t c = 0;
#pragma unroll
            for (int k = 0; k < kHistCopies; ++k) c += hist[k * kBins + b];
            cnt[b] = c;
        }
    }
    __syncthreads();
    int64_t mine = 0;
    for (int i = 0; i < per; ++i) {
        const int b = t * per + i;
        if (b < nb) mine += cnt[b];
    }
    suffix[t] = mine;
    if (t == 0) suffix[256] = 0;
    __syncthreads();
    // inclusive suffix sums: suffix[t] = sum of threads >= t
    for (int d = 1; d < 256; d <<= 1) {
        int64_t add = (t + d < 256) ? suffix[t + d] : 0;
        __syncthreads();
        suffix[t] += add;
        __syncthreads();
    }
    const int64_t above = suffix[t + 1];   // suffix[256] stays 0
    if (above < krem && krem <= above + mine) {
        int64_t acc = above;
        for (int i = per - 1; i >= 0; --i) {
            const int b = t * per + i;
            if (b >= nb) continue;
            const int64_t c = cnt[b];
            if (krem <= acc + c) {
                st->count_gt += acc;
                st->krem = krem - acc;
                if (last) st->all_ties = (krem - acc == c) ? 1u : 0u;
                st->prefix |= (uint64_t)b << shift;
                st->fixed |= (uint64_t)(nb - 1) << shift;
                break;
            }
            acc += c;
        }
    }
    __syncthreads();
    if (t == 0 && suffix[0] < krem) st->err |= 2u;
#pragma unroll
    for (int i = 0; i < kBins / 256; ++i) {
        const int b = i * 256 + t;
        if (b < nb)
#pragma unroll
            for (int k = 0; k < kHistCopies; ++k) hist[k * kBins + b] = 0;
    }
}

// Keys of tile t: t*kTieTile + j*256 + thread, j = 0..15 (ascending position
// in (j, thread) order).
__device__ __forceinline__ int32_t block_sum(int32_t x) {
    __shared__ int32_t part[256 / kWave];
    for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_down(x, off, kWave);
    if (threadIdx.x % kWave == 0) part[threadIdx.x / kWave] = x;
    __syncthreads();
    int32_t t = 0;
#pragma unroll
    for (int w = 0; w < 256 / kWave; ++w) t += part[w];
    __syncthreads();
    return t;
}

// Exclusive scan over the 256 threads of the block, in thread order.
__device__ __forceinline__ int32_t block_excl(int32_t x, int32_t &total) {
    __shared__ int32_t part[256 / kWave];
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    int32_t inc = x;
    for (int d = 1; d < kWave; d <<= 1) {
        const int32_t y = __shfl_up(inc, d, kWave);
        if (lane >= d) inc += y;
    }
    if (lane == kWave - 1) part[wv] = inc;
    __syncthreads();
    int32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 256 / kWave; ++w) {
        off += w < wv ? part[w] : 0;
        tot += part[w];
    }
    __syncthreads();
    total = tot;
    return off + inc - x;
}

// Keys equal to the threshold in each tile; nothing to do when the bucket is
// taken whole.
template <typename TS>
__global__ __launch_bounds__(256) void k_sel_tiecount(int64_t ne, const TS *__restrict__ score,
                                                      const SelState *__restrict__ st, int32_t *tcnt) {
    using K = typename KeyOf<TS>::K;
    if (st->all_ties) return;
    const K thr = (K)st->prefix;
    const int64_t base = (int64_t)blockIdx.x * kTieTile + threadIdx.x;
    int32_t c = 0;
#pragma unroll 4
    for (int j = 0; j < kTieTile / 256; ++j) {
        const int64_t i = base + j * 256;
        if (i < ne && key_of(score[i]) == thr) ++c;
    }
    c = block_sum(c);
    if (threadIdx.x == 0) tcnt[blockIdx.x] = c;
}

// In-place exclusive scan of the tile counts, one workgroup.
__global__ __launch_bounds__(256) void k_sel_tiescan(int32_t *tcnt, int64_t nt, const SelState *__restrict__ st) {
    if (st->all_ties) return;
    int32_t carry = 0;
    for (int64_t b0 = 0; b0 < nt; b0 += 256) {
        const int64_t i = b0 + threadIdx.x;
        const int32_t x = i < nt ? tcnt[i] : 0;
        int32_t tot;
        const int32_t ex = block_excl(x, tot);
        if (i < nt) tcnt[i] = carry + ex;
        carry += tot;
    }
}

template <typename TS>
__global__ __launch_bounds__(256) void k_sel_mark(int64_t ne, const TS *__restrict__ score,
                                                  const SelState *__restrict__ st,
                                                  const int32_t *__restrict__ tpos, uint8_t *sel, double *tau) {
    using K = typename KeyOf<TS>::K;
    const K thr = (K)st->prefix;
    const int64_t base = (int64_t)blockIdx.x * kTieTile + threadIdx.x;
    if (base == 0) *tau = st->err ? __builtin_nan("") : (double)value_of<TS>(thr);
    if (st->all_ties) {
#pragma unroll 4
        for (int j = 0; j < kTieTile / 256; ++j) {
            const int64_t i = base + j * 256;
            if (i < ne) sel[i] = key_of(score[i]) >= thr ? 1 : 0;
        }
        return;
    }
    const int64_t krem = st->krem;
    int32_t rank = tpos[blockIdx.x];
    for (int j = 0; j < kTieTile / 256; ++j) {
        const int64_t i = base + j * 256;
        const K key = i < ne ? key_of(score[i]) : K(0);
        const int32_t tie = (i < ne && key == thr) ? 1 : 0;
        int32_t tot;
        const int32_t ex = block_excl(tie, tot);
        if (i < ne) sel[i] = (key > thr || (tie && (int64_t)(rank + ex) < krem)) ? 1 : 0;
        rank += tot;
    }
}

__global__ void k_sel_empty(double *tau) { *tau = __builtin_inf(); }

struct SelPlan {
    SelState *st;
    uint32_t *hist;
    uint64_t *buf;      // keys copied by the compacting pass (room for all ne)
    int32_t *tcnt;      // tie counts per tile, then their exclusive scan
};

SelPlan plan_select(Carver &c, int64_t ne) {
    SelPlan p;
    p.st = c.take<SelState>(1);
    p.hist = c.take<uint32_t>(kBins * kHistCopies);
    p.buf = c.take<uint64_t>(ne + 1);
    p.tcnt = c.take<int32_t>((ne + kTieTile - 1) / kTieTile + 1);
    return p;
}

template <typename TS>
void run_select(const TS *score, int64_t ne, int64_t k, uint8_t *sel, double *tau, const SelPlan &p,
                hipStream_t s) {
    constexpr int B = KeyOf<TS>::bits;
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, p.st, k, p.hist);
    SFG_LAUNCH_CHECK();
    int64_t hb = (ne + kHistThreads * 16 - 1) / (kHistThreads * 16);
    if (hb > 2048) hb = 2048;
    if (hb < 1) hb = 1;
    using K = typename KeyOf<TS>::K;
    K *buf = reinterpret_cast<K *>(p.buf);
    int hi = B, pass = 0;
    while (hi > 0) {
        const int width = hi >= 11 ? 11 : hi;
        const int shift = hi - width;
        const int last = shift == 0 ? 1 : 0;
        if (pass <= kCompactPass)
            hipLaunchKernelGGL((k_sel_hist<TS, false>), dim3((uint32_t)hb), dim3(kHistThreads), 0, s, ne, score,
                               (const K *)nullptr, p.st, shift, width, pass == 0 ? 1 : 0, p.hist,
                               (pass == kCompactPass && !last) ? buf : (K *)nullptr);
        else
            hipLaunchKernelGGL((k_sel_hist<TS, true>), dim3((uint32_t)hb), dim3(kHistThreads), 0, s, ne, score, buf,
                               p.st, shift, width, 0, p.hist, (K *)nullptr);
        SFG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(256), 0, s, p.st, p.hist, shift, width, last);
        SFG_LAUNCH_CHECK();
        hi = shift;
        ++pass;
    }
    const int64_t nt = (ne + kTieTile - 1) / kTieTile;
    hipLaunchKernelGGL(k_sel_tiecount<TS>, dim3((uint32_t)nt), dim3(256), 0, s, ne, score, p.st, p.tcnt);
    SFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sel_tiescan, dim3(1), dim3(256), 0, s, p.tcnt, nt, p.st);
    SFG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sel_mark<TS>, dim3((uint32_t)nt), dim3(256), 0, s, ne, score, p.st, p.tcnt, sel, tau);
    SFG_LAUNCH_CHECK();
}

}  // namespace

size_t select_workspace_bytes(int64_t ne) {
    Carver c(nullptr);
    plan_select(c, ne);
    return c.used + 256;
}

void select_topk(const void *score, sfg_dtype st, int64_t ne, int64_t k, uint8_t *sel, double *tau, void *ws,
                 size_t ws_bytes, hipStream_t s) {
    SFG_REQUIRE(ne >= 0 && k >= 0 && k <= ne, SFG_EINVAL, "select_topk: need 0 <= k <= ne");
    SFG_REQUIRE(ne < (int64_t(1) << 31) - 1, SFG_EUNSUPPORTED, "select_topk: ne must be < 2^31-1");
    SFG_REQUIRE(st == SFG_F64 || st == SFG_F32, SFG_EINVAL, "select_topk: scores must be F64 or F32");
    SFG_REQUIRE(tau && (ne == 0 || (score && sel)), SFG_EINVAL, "select_topk: null pointer");
    SFG_REQUIRE(ws_bytes >= select_workspace_bytes(ne), SFG_EWORKSPACE, "select_topk: workspace too small");
    if (k == 0) {
        fill_u8(sel, ne, 0, s);
        hipLaunchKernelGGL(k_sel_empty, dim3(1), dim3(1), 0, s, tau);
        SFG_LAUNCH_CHECK();
        return;
    }
    Carver c(ws);
    SelPlan p = plan_select(c, ne);
    if (st == SFG_F64)
        run_select<double>((const double *)score, ne, k, sel, tau, p, s);
    else
        run_select<float>((const float *)score, ne, k, sel, tau, p, s);
}

namespace {

std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch`, looked up once per device
// with the device current.
void *select_scratch() {
    int dev = 0;
    SFG_HIP(hipGetDevice(&dev));
    SFG_REQUIRE(dev >= 0 && dev < kMaxDevices, SFG_EUNSUPPORTED, "select_topk_noalloc: device index above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        SFG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        SFG_REQUIRE(p != nullptr, SFG_EHIP, "select_topk_noalloc: no device address for the scratch array");
        g_scratch_dev[dev] = p;
    }
    return g_scratch_dev[dev];
}

void tau_to_host(const double *tau, double *tau_host, hipStream_t s) {
    SFG_HIP(hipMemcpyAsync(tau_host, tau, sizeof(double), hipMemcpyDeviceToHost, s));
    SFG_HIP(hipStreamSynchronize(s));
    if (*tau_host != *tau_host) fail(SFG_ENUMERIC, "select_topk: NaN or negative score");
}

}  // namespace

}  // namespace sfg

extern "C" sfg_status sfg_select_topk_noalloc(const void *score, sfg_dtype st, int64_t ne, int64_t k,
                                              uint8_t *sel, double *tau, double *tau_host, void *stream) {
    return sfg::guard([&] {
        hipStream_t s = sfg::as_stream(stream);
        SFG_REQUIRE(ne >= 0 && k >= 0 && k <= ne, SFG_EINVAL, "select_topk_noalloc: need 0 <= k <= ne");
        const size_t need = sfg::select_workspace_bytes(ne);
        SFG_REQUIRE(need <= sfg::kSelectNoallocBytes, SFG_EUNSUPPORTED,
                    "select_topk_noalloc: " + std::to_string(ne) + " scores need " + std::to_string(need) +
                        " bytes of scratch, above the " + std::to_string(sfg::kSelectNoallocBytes) +
                        " the library holds per device (use sfg_select_topk with a workspace)");
        void *ws = sfg::select_scratch();
        sfg::select_topk(score, st, ne, k, sel, tau, ws, sfg::kSelectNoallocBytes, s);
        if (tau_host) sfg::tau_to_host(tau, tau_host, s);
    });
}

extern "C" sfg_status sfg_select_topk(const void *score, sfg_dtype st, int64_t ne, int64_t k, uint8_t *sel,
                                      double *tau, double *tau_host, void *ws, size_t ws_bytes, void *stream) {
    return sfg::guard([&] {
        hipStream_t s = sfg::as_stream(stream);
        sfg::select_topk(score, st, ne, k, sel, tau, ws, ws_bytes, s);
        if (tau_host) sfg::tau_to_host(tau, tau_host, s);
    });
}
