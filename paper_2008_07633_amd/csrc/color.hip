// Multicolouring of a graph for the Gauss-Seidel reading of the smoother
// (Sec. 3.2 relaxes L x = 0 by Gauss-Seidel steps; colour by colour, the rows
// of one colour are independent and update in parallel).
//
// Jones-Plassmann rounds with a fixed priority (h(p), p), h a multiply-
// xorshift integer mixer: in round r every node still uncoloured whose
// priority exceeds that of all its uncoloured neighbours takes the smallest
// colour not used by a neighbour coloured in an earlier round.  A round is
// two launches (choose, then colour) and one host check; the result depends
// only on the graph.  Colour classes are then listed in ascending node order.
#include <vector>

#include "common.hpp"

namespace sfg {

void smooth_gs(const sfg_csr *H, int32_t k, int32_t sweeps, double omega, const double *x0, sfg_dtype storage,
               const int32_t *class_rows, const std::vector<int32_t> &class_ptr, void *x, void *ws, size_t ws_bytes,
               hipStream_t s);
size_t smooth_workspace_bytes(int64_t n, int32_t k, sfg_dtype storage);

namespace {

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

__device__ __forceinline__ bool prio_greater(int64_t p, int64_t q) {
    const uint32_t hp = mix32((uint32_t)p), hq = mix32((uint32_t)q);
    return hp > hq || (hp == hq && p > q);
}

__global__ void k_color_init(int64_t n, int32_t *color, int32_t *round) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    color[p] = -1;
    round[p] = -1;
}

// Round r, choose: uncoloured local maxima get round = r.  A neighbour whose
// round reads -1 or r was uncoloured when the round began.
__global__ void k_color_choose(int64_t n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                               int32_t r, int32_t *round, int32_t *more) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n || round[p] >= 0) return;
    bool is_max = true;
    for (int32_t j = rowptr[p]; j < rowptr[p + 1] && is_max; ++j) {
        const int32_t q = col[j];
        const int32_t rq = round[q];
        if ((rq < 0 || rq == r) && prio_greater(q, p)) is_max = false;
    }
    if (is_max)
        round[p] = r;
    else if (*more == 0)
        *more = 1;      // some node stays uncoloured after this round
}

// Round r, colour: the smallest colour unused by neighbours of earlier rounds.
__global__ void k_color_assign(int64_t n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                               int32_t r, const int32_t *__restrict__ round, int32_t *color, int32_t *maxc) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n || round[p] != r) return;
    const int32_t j0 = rowptr[p], j1 = rowptr[p + 1];
    uint64_t used = 0;
    for (int32_t j = j0; j < j1; ++j) {
        const int32_t q = col[j];
        const int32_t rq = round[q];
        if (rq >= 0 && rq < r) {
            const int32_t c = color[q];
            if (c < 64) used |= 1ull << c;
        }
    }
    int32_t c = used == ~0ull ? 64 : __builtin_ctzll(~used);
    if (c == 64) {      // all of 0..63 taken: search upwards
        for (;; ++c) {
            bool taken = false;
            for (int32_t j = j0; j < j1 && !taken; ++j) {
                const int32_t q = col[j];
                const int32_t rq = round[q];
                taken = rq >= 0 && rq < r && color[q] == c;
            }
            if (!taken) break;
        }
    }
    color[p] = c;
    if (c + 1 > *maxc) atomicMax(maxc, c + 1);
}

__global__ void k_color_flags(int64_t n, const int32_t *__restrict__ color, int32_t c, int32_t *flags) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) flags[p] = color[p] == c ? 1 : 0;
}

__global__ void k_color_scatter(int64_t n, const int32_t *__restrict__ flags, const int32_t *__restrict__ pos,
                                int32_t *out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n && flags[p]) out[pos[p]] = (int32_t)p;
}

struct ColorPlan {
    int32_t *round, *flags, *pos, *scan, *state;
};

ColorPlan plan_color(Carver &c, int64_t n) {
    ColorPlan p;
    p.round = c.take<int32_t>(n + 1);
    p.flags = c.take<int32_t>(n + 1);
    p.pos = c.take<int32_t>(n + 1);
    p.scan = c.take<int32_t>(scan_scratch_ints(n + 1));
    p.state = c.take<int32_t>(4);
    return p;
}

int32_t read_int(const int32_t *p, hipStream_t s) {
    int32_t h = 0;
    SFG_HIP(hipMemcpyAsync(&h, p, sizeof(h), hipMemcpyDeviceToHost, s));
    SFG_HIP(hipStreamSynchronize(s));
    return h;
}

}  // namespace

size_t color_workspace_bytes(int64_t n) {
    Carver c(nullptr);
    plan_color(c, n);
    return c.used + 256;
}

// Colours every node; fills class_rows (n: the nodes of colour 0, then 1, ...,
// each class ascending) and class_ptr (ncolors + 1 host offsets).
void color_graph(const sfg_csr *H, int32_t *color, int32_t *class_rows, std::vector<int32_t> &class_ptr, void *ws,
                 size_t ws_bytes, hipStream_t s) {
    SFG_REQUIRE(H && H->rowptr && color && class_rows, SFG_EINVAL, "color: null pointer");
    SFG_REQUIRE(H->n >= 1, SFG_EINVAL, "color: empty graph");
    SFG_REQUIRE(ws_bytes >= color_workspace_bytes(H->n), SFG_EWORKSPACE, "color: workspace too small");
    const int64_t n = H->n;
    Carver c(ws);
    ColorPlan p = plan_color(c, n);
    const dim3 gn(grid_for(n, 256)), b(256);
    hipLaunchKernelGGL(k_color_init, gn, b, 0, s, n, color, p.round);
    SFG_LAUNCH_CHECK();
    fill_i32(p.state, 2, 0, s);        // state[0] = more, state[1] = colours used
    for (int32_t r = 0;; ++r) {
        SFG_REQUIRE(r <= n, SFG_EHIP, "color: too many rounds");
        fill_i32(p.state, 1, 0, s);
        hipLaunchKernelGGL(k_color_choose, gn, b, 0, s, n, H->rowptr, H->col, r, p.round, p.state);
        SFG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_color_assign, gn, b, 0, s, n, H->rowptr, H->col, r, p.round, color, p.state + 1);
        SFG_LAUNCH_CHECK();
        if (read_int(p.state, s) == 0) break;
    }
    const int32_t ncolors = read_int(p.state + 1, s);
    class_ptr.assign(ncolors + 1, 0);
    for (int32_t cc = 0; cc < ncolors; ++cc) {
        hipLaunchKernelGGL(k_color_flags, gn, b, 0, s, n, color, cc, p.flags);
        SFG_LAUNCH_CHECK();
        exclusive_scan_i32(p.flags, p.pos, n, p.scan, s);
        hipLaunchKernelGGL(k_color_scatter, gn, b, 0, s, n, p.flags, p.pos, class_rows + class_ptr[cc]);
        SFG_LAUNCH_CHECK();
        class_ptr[cc + 1] = class_ptr[cc] + read_int(p.pos + n, s);
    }
    SFG_REQUIRE(class_ptr[ncolors] == n, SFG_EHIP, "color: classes do not cover the graph");
}

}  // namespace sfg

extern "C" sfg_status sfg_color(const sfg_csr *H, int32_t *color, int32_t *class_rows, int32_t *class_ptr,
                                int32_t *ncolors, void *ws, size_t ws_bytes, void *stream) {
    return sfg::guard([&] {
        SFG_REQUIRE(class_ptr && ncolors, SFG_EINVAL, "color: null pointer");
        hipStream_t s = sfg::as_stream(stream);
        std::vector<int32_t> cp;
        sfg::color_graph(H, color, class_rows, cp, ws, ws_bytes, s);
        SFG_HIP(hipMemcpyAsync(class_ptr, cp.data(), sizeof(int32_t) * cp.size(), hipMemcpyHostToDevice, s));
        SFG_HIP(hipStreamSynchronize(s));
        *ncolors = (int32_t)cp.size() - 1;
    });
}

extern "C" sfg_status sfg_smooth_gs(const sfg_csr *H, const int32_t *class_rows, const int32_t *class_ptr,
                                    int32_t ncolors, int32_t k, int32_t sweeps, double omega, const double *x0,
                                    sfg_dtype storage, void *x, void *ws, size_t ws_bytes, void *stream) {
    return sfg::guard([&] {
        SFG_REQUIRE(H && class_ptr && ncolors >= 1 && ncolors <= H->n, SFG_EINVAL, "smooth_gs: bad colour classes");
        hipStream_t s = sfg::as_stream(stream);
        std::vector<int32_t> cp(ncolors + 1);
        SFG_HIP(hipMemcpyAsync(cp.data(), class_ptr, sizeof(int32_t) * cp.size(), hipMemcpyDeviceToHost, s));
        SFG_HIP(hipStreamSynchronize(s));
        SFG_REQUIRE(cp[0] == 0 && cp[ncolors] == H->n, SFG_EINVAL, "smooth_gs: colour classes must cover the graph");
        for (int32_t c = 0; c < ncolors; ++c)
            SFG_REQUIRE(cp[c] <= cp[c + 1], SFG_EINVAL, "smooth_gs: colour offsets must not decrease");
        sfg::smooth_gs(H, k, sweeps, omega, x0, storage, class_rows, cp, x, ws, ws_bytes, s);
    });
}
