// Spectral coarsening (Sec. 3.2-3.3) and the multilevel driver (Alg. 1).
#include "common.hpp"

namespace sfg {

size_t coarsen_workspace_bytes(int64_t n, int64_t m) {
    (void)n;
    (void)m;
    return 256;
}

void multilevel_sparsify(int64_t, int64_t, const int32_t *, const int32_t *, const void *, sfg_dtype,
                         const sfg_params *, const double *, uint8_t *, sfg_report *, hipStream_t) {
    fail(SFG_EUNSUPPORTED, "sparsify: levels > 1 not built yet");
}

}  // namespace sfg

extern "C" sfg_status sfg_coarsen(const sfg_csr *, int64_t, const int32_t *, const int32_t *, const void *,
                                  sfg_dtype, const void *, sfg_dtype, int32_t *, int64_t *, int64_t *, int32_t *,
                                  int32_t *, void *, int32_t *, void *, size_t, void *) {
    return sfg::guard([&] { sfg::fail(SFG_EUNSUPPORTED, "coarsen: not built yet"); });
}
