// Backward pass of the clipped blend and of the projection (placeholder until
// the gradient kernels land: reports RARA_ERR_UNSUPPORTED).
#include "rara_internal.h"

namespace rara {
size_t backward_workspace_bytes(int64_t n, int32_t width, int32_t height)
{
    (void)n; (void)width; (void)height;
    return 256;
}
}  // namespace rara

extern "C" rara_status rara_render_backward(const rara_gaussians* g, const rara_camera* cam, const rara_plane* plane,
                                            const rara_projected* proj, const rara_binned* bins, const float* final_T,
                                            const uint32_t* n_contrib, const float* dL_dimage, const rara_grads* grads,
                                            void* workspace, size_t ws_bytes, void* stream)
{
    (void)g; (void)cam; (void)plane; (void)proj; (void)bins; (void)final_T; (void)n_contrib; (void)dL_dimage;
    (void)grads; (void)workspace; (void)ws_bytes; (void)stream;
    return RARA_ERR_UNSUPPORTED;
}
