// Random test vectors on the device (Sec. 3.2 smooths random vectors):
// counter-based Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and
// Box-Muller normals.  Element pair j of block b of an n-by-k row-major block
// (elements 2j, 2j+1) uses counter (lo32 j, hi32 j, b, 0) and key
// (lo32 seed, hi32 seed); with output words r0..r3,
//   u1 = ((r0:r1) >> 11) 2^-53,  u2 = ((r2:r3) >> 11) 2^-53,
//   rho = sqrt(-2 log(1 - u1)),  z0 = rho cos(2 pi u2),  z1 = rho sin(2 pi u2).
// One thread per pair; the integer part is exact, the transcendental part
// uses the device math library.
#include "common.hpp"

namespace sfg {

namespace {

__device__ __forceinline__ void philox4x32_10(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3, uint32_t k0,
                                              uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9U;
            k1 += 0xBB67AE85U;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53U * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57U * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
}

__global__ void k_random_block(int64_t total, uint64_t seed, uint32_t block, double *x) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (2 * j >= total) return;
    uint32_t c0 = (uint32_t)j, c1 = (uint32_t)((uint64_t)j >> 32), c2 = block, c3 = 0;
    philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u1 = (double)(((((uint64_t)c0) << 32) | c1) >> 11) * 0x1.0p-53;
    const double u2 = (double)(((((uint64_t)c2) << 32) | c3) >> 11) * 0x1.0p-53;
    const double rho = sqrt(-2.0 * log(1.0 - u1));
    const double th = 6.283185307179586476925286766559 * u2;
    x[2 * j] = rho * cos(th);
    if (2 * j + 1 < total) x[2 * j + 1] = rho * sin(th);
}

}  // namespace

void random_block(int64_t n, int32_t k, uint64_t seed, uint32_t block, double *x, hipStream_t s) {
    SFG_REQUIRE(n >= 1 && k >= 1 && x, SFG_EINVAL, "random_block: bad arguments");
    const int64_t total = n * (int64_t)k;
    const int64_t pairs = (total + 1) / 2;
    hipLaunchKernelGGL(k_random_block, dim3(grid_for(pairs, 256)), dim3(256), 0, s, total, seed, block, x);
    SFG_LAUNCH_CHECK();
}

}  // namespace sfg

extern "C" sfg_status sfg_random_block(int64_t n, int32_t k, uint64_t seed, uint32_t block, double *x0,
                                       void *stream) {
    return sfg::guard([&] { sfg::random_block(n, k, seed, block, x0, sfg::as_stream(stream)); });
}
