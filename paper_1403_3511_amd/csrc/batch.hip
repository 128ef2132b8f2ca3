// Batched form (placeholder until the persistent kernel lands).
#include "hs_internal.h"

extern "C" {
int32_t hs_batch_create(int32_t, const hs_index *, const void *const *, const hs_pot *, void *const *, hs_batch *out) {
  if (out) *out = nullptr;
  return hs::fail(HS_E_UNSUPPORTED, "hs_batch_create: not built");
}
int32_t hs_batch_destroy(hs_batch) { return HS_OK; }
int32_t hs_batch_offsets(hs_batch, int64_t *) { return hs::fail(HS_E_UNSUPPORTED, "not built"); }
int32_t hs_batch_device_bytes(hs_batch, int64_t *) { return hs::fail(HS_E_UNSUPPORTED, "not built"); }
int32_t hs_batch_upload(hs_batch, void *, int64_t, void *) { return hs::fail(HS_E_UNSUPPORTED, "not built"); }
int32_t hs_batch_workspace_bytes(hs_batch, int32_t, int64_t *) { return hs::fail(HS_E_UNSUPPORTED, "not built"); }
int32_t hs_batch_apply_h(hs_batch, const void *, const void *, void *, void *, void *) { return hs::fail(HS_E_UNSUPPORTED, "not built"); }
int32_t hs_batch_step(hs_batch, void *, double, double, int32_t, int32_t, void *, void *, void *) { return hs::fail(HS_E_UNSUPPORTED, "not built"); }
int32_t hs_batch_set_launch(hs_batch, int32_t, int32_t) { return hs::fail(HS_E_UNSUPPORTED, "not built"); }
int32_t hs_batch_get_launch(hs_batch, int32_t *, int32_t *) { return hs::fail(HS_E_UNSUPPORTED, "not built"); }
int32_t hs_batch_autotune_sync(hs_batch, const void *, const void *, void *, void *, void *) { return hs::fail(HS_E_UNSUPPORTED, "not built"); }
}
