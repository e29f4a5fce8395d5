#include "common.hpp"
namespace krr {
void run_fit(krr_ctx, hipStream_t, const void*, const void*, int, int64_t, int, const int32_t*, const double*, int,
             const krr_fit_params*, int, krr_model*, krr_part_info*) {
  fail(KRR_ESTATE, "fit not available in this build");
}
}
