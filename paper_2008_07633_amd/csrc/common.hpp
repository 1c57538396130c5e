// Internal helpers of libsfg (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sfg.h"

namespace sfg {

// ---------------------------------------------------------------- errors

struct Error {
    sfg_status st;
    std::string msg;
};

void set_last_error(const std::string &msg);
void clear_last_error();

[[noreturn]] inline void fail(sfg_status st, const std::string &msg) { throw Error{st, msg}; }

#define SFG_HIP(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            ::sfg::fail(SFG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_) + " at " + \
                                      __FILE__ + ":" + std::to_string(__LINE__));            \
    } while (0)

#define SFG_LAUNCH_CHECK() SFG_HIP(hipGetLastError())

#define SFG_REQUIRE(cond, st, msg)               \
    do {                                         \
        if (!(cond)) ::sfg::fail((st), (msg));   \
    } while (0)

// Wrap an entry point body: maps internal errors to status codes.
template <typename F>
inline sfg_status guard(F &&f) {
    try {
        f();
        clear_last_error();
        return SFG_OK;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.st;
    } catch (const std::exception &e) {
        set_last_error(std::string("internal error: ") + e.what());
        return SFG_EHIP;
    } catch (...) {
        set_last_error("internal error");
        return SFG_EHIP;
    }
}

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ---------------------------------------------------------------- workspace carving

// Bump allocator over a caller workspace.  With base == nullptr it only
// measures, so the same plan function gives sfg_workspace_bytes().
struct Carver {
    char *base;
    size_t used = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <typename T>
    T *take(size_t count) {
        used = (used + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
        used += count * sizeof(T);
        return p;
    }
};

inline size_t dtype_size(sfg_dtype t) {
    switch (t) {
        case SFG_F64: return 8;
        case SFG_F32: return 4;
        case SFG_F16: return 2;
        case SFG_BF16: return 2;
    }
    return 0;
}

inline bool valid_dtype(int t) { return t >= SFG_F64 && t <= SFG_BF16; }

// ---------------------------------------------------------------- device helpers

constexpr int kWave = 64;
constexpr int kNumXcd = 8;
constexpr int kMaxDevices = 64;

// Size of the per-device scratch array of sfg_select_topk_noalloc.
constexpr size_t kSelectNoallocBytes = size_t(128) << 20;

// Workgroups are dealt round-robin to the 8 XCDs; remap so that each XCD
// walks one contiguous range of logical blocks (neighbouring rows share that
// XCD's L2).  Bijective for any grid size.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nb) {
    uint32_t q = nb / kNumXcd, r = nb % kNumXcd;
    uint32_t x = b % kNumXcd, i = b / kNumXcd;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

template <typename T> struct DT;
template <> struct DT<double> { static constexpr sfg_dtype id = SFG_F64; };
template <> struct DT<float> { static constexpr sfg_dtype id = SFG_F32; };
template <> struct DT<__half> { static constexpr sfg_dtype id = SFG_F16; };
template <> struct DT<__hip_bfloat16> { static constexpr sfg_dtype id = SFG_BF16; };

// value conversions (round to nearest even on narrowing)
template <typename TO, typename FROM> __device__ __forceinline__ TO cvt(FROM x);
template <> __device__ __forceinline__ double cvt<double, double>(double x) { return x; }
template <> __device__ __forceinline__ double cvt<double, float>(float x) { return (double)x; }
template <> __device__ __forceinline__ float cvt<float, float>(float x) { return x; }
template <> __device__ __forceinline__ float cvt<float, double>(double x) { return (float)x; }
template <> __device__ __forceinline__ float cvt<float, __half>(__half x) { return __half2float(x); }
template <> __device__ __forceinline__ float cvt<float, __hip_bfloat16>(__hip_bfloat16 x) {
    return __bfloat162float(x);
}
template <> __device__ __forceinline__ __half cvt<__half, float>(float x) { return __float2half(x); }
template <> __device__ __forceinline__ __hip_bfloat16 cvt<__hip_bfloat16, float>(float x) {
    return __float2bfloat16(x);
}
// FP64 to FP16 / BF16 with one rounding.  Rounding to float first and then to
// the 16-bit type rounds twice and can land one unit off (a double just above
// a 16-bit midpoint can round to that midpoint in float, then tie to even).
// Rounding to float toward zero and setting the last bit when anything was
// dropped ("round to odd") keeps the information the second rounding needs:
// with at least two extra significand bits in the intermediate format (float
// has 13 more than FP16 and 16 more than BF16, also in their subnormal ranges)
// the round to nearest even that follows gives the correctly rounded result
// (Boldo and Melquiond, "Emulation of FMA and correctly rounded sums: proved
// algorithms using rounding to odd", IEEE Trans. Computers 57(4), 2008).
__device__ __forceinline__ float round_to_odd_float(double x) {
    float f = (float)x;
    // rounded away from zero (also to infinity on overflow): one step back toward zero, which for a
    // sign-magnitude encoding is the bit pattern minus one
    if (__builtin_fabs((double)f) > __builtin_fabs(x)) f = __uint_as_float(__float_as_uint(f) - 1u);
    if ((double)f != x && f == f) f = __uint_as_float(__float_as_uint(f) | 1u);
    return f;
}
template <> __device__ __forceinline__ __half cvt<__half, double>(double x) {
    return __float2half(round_to_odd_float(x));
}
template <> __device__ __forceinline__ __hip_bfloat16 cvt<__hip_bfloat16, double>(double x) {
    return __float2bfloat16(round_to_odd_float(x));
}
template <> __device__ __forceinline__ double cvt<double, __half>(__half x) { return (double)__half2float(x); }
template <> __device__ __forceinline__ double cvt<double, __hip_bfloat16>(__hip_bfloat16 x) {
    return (double)__bfloat162float(x);
}

// ---------------------------------------------------------------- shared device routines

// Exclusive prefix sum of int32 counts; out may alias nothing.  n elements in,
// n+1 written (out[n] = total).  Scratch: scan_scratch_ints(n) ints.
size_t scan_scratch_ints(int64_t n);
void exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *scratch, hipStream_t s);

// Fill with a value (kernel, not a memset node, so it is safe under capture).
void fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
void fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s);

// Node numbering for the sweeps of a sparsify call or of one hierarchy level
// (the rules are with score_level and level_node_order).
struct NodeOrder {
    int64_t launches = 0;       // planned column-part sweep launches (set by the caller)
    bool decided = false;
    bool use = false;
    int32_t *order = nullptr;   // [n] node at new position i
    int32_t *inv = nullptr;     // [n] new position of node j
    int32_t *u = nullptr;       // [m] endpoints in the new numbering
    int32_t *v = nullptr;
};

// Device buffers owned by one allocating call (sfg_sparsify, ...), carved
// from chunks of at least 256 MB.  A call that ends with finish() (its stream
// drained) hands its chunks to a per-device cache (up to 16 GiB) that later
// calls reuse; otherwise (an error path, work possibly in flight) they are
// freed stream-ordered.  SFG_FAIL_ALLOC_AFTER=n makes the (n+1)-th buffer
// request fail, to test the error path.
struct DevArena {
    struct Chunk {
        void *p;
        size_t size;
    };
    hipStream_t s;
    std::vector<Chunk> chunks;
    size_t used = 0;   // bytes carved from the last chunk
    int dev = 0;
    bool synced = false;
    long fail_after = -1;
    long count = 0;
    explicit DevArena(hipStream_t st);
    ~DevArena();
    DevArena(const DevArena &) = delete;
    DevArena &operator=(const DevArena &) = delete;
    void *raw(size_t bytes);
    void finish();   // wait for the stream; the chunks may then be cached
    template <typename T>
    T *alloc(size_t n) {
        return static_cast<T *>(raw(n * sizeof(T)));
    }
};

inline uint32_t grid_for(int64_t items, int block) {
    int64_t g = (items + block - 1) / block;
    return (uint32_t)(g < 1 ? 1 : g);
}

}  // namespace sfg
