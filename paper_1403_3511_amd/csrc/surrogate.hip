// Learned-coefficient path (placeholder until the MFMA kernels land).
#include "hs_internal.h"

extern "C" {
int32_t hs_gh_ncoef(int32_t, int32_t, int32_t *) { return hs::fail(HS_E_UNSUPPORTED, "not built"); }
int32_t hs_gh_project(int32_t, int32_t, int32_t, int32_t, const double *, int32_t, const double *, double *, void *) { return hs::fail(HS_E_UNSUPPORTED, "not built"); }
int32_t hs_mlp_create(int32_t, int32_t, int32_t, hs_mlp *m) { if (m) *m = nullptr; return hs::fail(HS_E_UNSUPPORTED, "not built"); }
int32_t hs_mlp_destroy(hs_mlp) { return HS_OK; }
int32_t hs_mlp_device_bytes(hs_mlp, int32_t, int64_t *) { return hs::fail(HS_E_UNSUPPORTED, "not built"); }
int32_t hs_mlp_upload_params(hs_mlp, void *, const float *, const float *, void *) { return hs::fail(HS_E_UNSUPPORTED, "not built"); }
int32_t hs_mlp_download_params(hs_mlp, const void *, float *, void *) { return hs::fail(HS_E_UNSUPPORTED, "not built"); }
int32_t hs_mlp_predict(hs_mlp, void *, int32_t, const double *, double *, void *) { return hs::fail(HS_E_UNSUPPORTED, "not built"); }
int32_t hs_mlp_train_step(hs_mlp, void *, int32_t, const double *, const double *, float, float *, float *, void *) { return hs::fail(HS_E_UNSUPPORTED, "not built"); }
}
