#include "common.hpp"
namespace krr {
void run_predict(krr_ctx, hipStream_t, krr_model, const void*, int, int64_t, int, double*, int32_t*) {
  fail(KRR_ESTATE, "predict not available in this build");
}
void run_select(krr_ctx, hipStream_t, const krr_model*, int, const void*, const void*, int, int64_t, int, double*,
                int32_t*) {
  fail(KRR_ESTATE, "select not available in this build");
}
}
