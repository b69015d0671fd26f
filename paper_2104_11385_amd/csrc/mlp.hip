// Learned per-box cost model (placeholder until the matrix-core kernels land).
#include "runtime.hpp"

int pic_ctx::learned_costs(double *costs, int *used) {
    (void)costs;
    *used = PIC_COST_HEURISTIC;
    return PIC_OK;
}

void pic_ctx::mlp_release() {}

extern "C" {
PIC_API int32_t pic_mlp_nparam(void) { return 16 * 64 + 64 + 64 * 64 + 64 + 64 + 1; }
PIC_API int pic_mlp_train(pic_ctx *, const float *, const float *, int64_t, int32_t, int32_t, const int32_t *,
                          const float *, uint64_t, float *) {
    return PIC_EUNSUPPORTED;
}
PIC_API int pic_mlp_predict(pic_ctx *, const float *, int64_t, float *) { return PIC_EUNSUPPORTED; }
PIC_API int pic_mlp_loss_grad(pic_ctx *, const float *, const float *, int64_t, float *, float *) {
    return PIC_EUNSUPPORTED;
}
PIC_API int pic_mlp_set_weights(pic_ctx *, const float *, int64_t) { return PIC_EUNSUPPORTED; }
PIC_API int pic_mlp_get_weights(pic_ctx *, float *, int64_t) { return PIC_EUNSUPPORTED; }
PIC_API int pic_autotune(pic_ctx *, int32_t, pic_tuning *, double *) { return PIC_EUNSUPPORTED; }
}
