// stubs.cpp -- entry points whose implementation lands later.
#include "forward.h"
#include "runtime.h"

namespace vr {
int render_with_state(vr_ctx*, vr_volume*, const vr_view*, int32_t, const vr_params*, float*, hipStream_t,
                      vr_state**) {
  return fail(VR_EUNSUPPORTED, "differentiable forward not built yet");
}
}  // namespace vr

extern "C" {
int vr_render_backward(vr_ctx*, const vr_volume*, const vr_state*, const float*, float*, float*, int, uintptr_t) {
  vr::clear_error();
  return vr::fail(VR_EUNSUPPORTED, "not built yet");
}
int vr_state_destroy(vr_state*) { return VR_OK; }
int vr_render_batch(vr_ctx*, const vr_request*, int32_t, const vr_params*, vr_batch**, uintptr_t) {
  vr::clear_error();
  return vr::fail(VR_EUNSUPPORTED, "not built yet");
}
int vr_batch_destroy(vr_batch*) { return VR_OK; }
int vr_autotune(vr_ctx*, const vr_volume*, const vr_view*, const vr_params*, vr_tune_result*, uintptr_t) {
  vr::clear_error();
  return vr::fail(VR_EUNSUPPORTED, "not built yet");
}
}
