// Entry points whose implementation is not in this build yet.
#include "kc_internal.h"

extern "C" kc_status kc_mlp_forward(kc_handle *h, const uint16_t *, const float *, int64_t, float *,
                                    float *, void *) {
  return kc_fail(h, KC_EUNSUPPORTED, "kc_mlp_forward not built");
}
extern "C" kc_status kc_mlp_backward(kc_handle *h, const uint16_t *, const float *, const float *,
                                     const float *, int64_t, float *, void *) {
  return kc_fail(h, KC_EUNSUPPORTED, "kc_mlp_backward not built");
}
extern "C" kc_status kc_mlp_loss(kc_handle *h, const float *, const int32_t *, const int32_t *,
                                 int32_t, int64_t, float *, float *, void *) {
  return kc_fail(h, KC_EUNSUPPORTED, "kc_mlp_loss not built");
}
extern "C" kc_status kc_mlp_adam(kc_handle *h, float *, uint16_t *, const float *, float *, float *,
                                 int32_t, float, void *) {
  return kc_fail(h, KC_EUNSUPPORTED, "kc_mlp_adam not built");
}
