// Entry points whose device implementation lands in later files; until
// then they report KPM_ERR_UNSUPPORTED.
#include "kpm_internal.h"

kpm_status kpm_learned_damping(kpm_ctx* ctx, int, const double*, double*) {
    return kpm_fail(ctx, KPM_ERR_UNSUPPORTED, "learned damping not built");
}
extern "C" int64_t kpm_mlp_param_count(void) { return 128 * 256 + 256 + 256 * 256 + 256 + 256 * 128 + 128; }
extern "C" kpm_status kpm_mlp_set_params(kpm_ctx* c, const float*) { return kpm_fail(c, KPM_ERR_UNSUPPORTED, "mlp"); }
extern "C" kpm_status kpm_mlp_get_params(kpm_ctx* c, float*) { return kpm_fail(c, KPM_ERR_UNSUPPORTED, "mlp"); }
extern "C" kpm_status kpm_mlp_forward(kpm_ctx* c, int, const float*, float*) { return kpm_fail(c, KPM_ERR_UNSUPPORTED, "mlp"); }
extern "C" kpm_status kpm_mlp_loss_grad(kpm_ctx* c, int, const float*, const float*, float, float*, float*) {
    return kpm_fail(c, KPM_ERR_UNSUPPORTED, "mlp");
}
extern "C" kpm_status kpm_mlp_train(kpm_ctx* c, int, const float*, const float*, float, int, int, float, uint64_t, float*) {
    return kpm_fail(c, KPM_ERR_UNSUPPORTED, "mlp");
}
extern "C" kpm_status kpm_mlp_init(kpm_ctx* c, uint64_t) { return kpm_fail(c, KPM_ERR_UNSUPPORTED, "mlp"); }
extern "C" kpm_status kpm_mlp_save(kpm_ctx* c, const char*) { return kpm_fail(c, KPM_ERR_UNSUPPORTED, "mlp"); }
extern "C" kpm_status kpm_mlp_load(kpm_ctx* c, const char*) { return kpm_fail(c, KPM_ERR_UNSUPPORTED, "mlp"); }
