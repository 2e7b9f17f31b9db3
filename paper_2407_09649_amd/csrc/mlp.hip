// mlp.hip -- learned distance correction (placeholder until its kernels land):
// every entry point reports that the correction is unavailable.
#include "gpdf_internal.hpp"

namespace gpdf {
gpdf_status mlp_apply(gpdf_ctx *c, const float *, const float *, const float *, const float *,
                      const uint8_t *, int64_t, float *) {
    return fail(c, GPDF_E_INVALID_ARG, "learned correction not available");
}
}  // namespace gpdf

using namespace gpdf;
#define GPDF_MLP_UNAVAILABLE(c) return fail(c, GPDF_E_INVALID_ARG, "learned correction not available")
extern "C" gpdf_status gpdf_mlp_init(gpdf_ctx *c, uint64_t) { GPDF_MLP_UNAVAILABLE(c); }
extern "C" gpdf_status gpdf_mlp_set_weights(gpdf_ctx *c, const float *, int64_t) { GPDF_MLP_UNAVAILABLE(c); }
extern "C" gpdf_status gpdf_mlp_get_weights(gpdf_ctx *c, float *, int64_t) { GPDF_MLP_UNAVAILABLE(c); }
extern "C" gpdf_status gpdf_mlp_set_norm(gpdf_ctx *c, const float *, const float *) { GPDF_MLP_UNAVAILABLE(c); }
extern "C" gpdf_status gpdf_mlp_features(gpdf_ctx *c, const float *, const float *, const float *,
                                         const float *, int64_t, float *) { GPDF_MLP_UNAVAILABLE(c); }
extern "C" gpdf_status gpdf_mlp_forward(gpdf_ctx *c, const float *, int64_t, float *) { GPDF_MLP_UNAVAILABLE(c); }
extern "C" gpdf_status gpdf_mlp_grad(gpdf_ctx *c, const float *, const float *, int64_t, float *, float *) {
    GPDF_MLP_UNAVAILABLE(c);
}
extern "C" gpdf_status gpdf_mlp_train(gpdf_ctx *c, const float *, const float *, int64_t, int32_t, int32_t,
                                      float, uint64_t, float *) { GPDF_MLP_UNAVAILABLE(c); }
