// Precision form: FP64 re-scoring of the candidates near the selection
// threshold.
#include "common.hpp"

namespace sfg {

void band_rescore(const sfg_csr *, int32_t, int32_t, double, const double *, int64_t, const int32_t *,
                  const int32_t *, const int32_t *, const double *, const float *, int64_t, double, double,
                  uint8_t *, sfg_level_report *, hipStream_t) {
    fail(SFG_EUNSUPPORTED, "band re-scoring not built yet");
}

}  // namespace sfg
