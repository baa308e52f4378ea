// Rendering entry points (placeholder until the render kernels land).
#include <hip/hip_runtime.h>

#include "../../include/rtq.h"
#include "api_internal.h"

namespace rtq {
void release_render_scratch(rtq_scene* s) { s->scratch.release(); }
}  // namespace rtq

extern "C" {
int rtq_render(const rtq_scene*, const rtq_camera*, int32_t, int32_t, int32_t, const rtq_render_opts*, float*,
               hipStream_t) {
  return rtq::set_error(RTQ_E_INVALID_ARG, "render not available");
}
int rtq_render_backward(const rtq_scene*, const rtq_camera*, int32_t, int32_t, int32_t, const rtq_render_opts*,
                        const float*, float*, hipStream_t) {
  return rtq::set_error(RTQ_E_INVALID_ARG, "render not available");
}
}
