// Frame graphs: every kernel of one frame (preprocess, binning, sort, schedule,
// blend) captured once into a HIP graph for a fixed shape (the Gaussians, the
// image size, the buffers and the pair capacity), then replayed per request
// with only the camera- and plane-dependent kernel arguments rewritten in the
// instantiated graph.  One graph launch replaces the ~25 launches of a frame.
#include <cstdlib>
#include <cstring>
#include <vector>

#include "rara_internal.h"

using namespace rara;

struct rara_frame_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t pre_node = nullptr, blend_node = nullptr;
    hipKernelNodeParams pre{}, blend{};
    // arguments that stay fixed for the shape
    GaussPtrs g{};
    ProjPtrs proj{};
    const Splat* splat = nullptr;
    const RayRec* ray = nullptr;
    const uint32_t* vals = nullptr;
    const uint2* ranges = nullptr;
    const uint32_t* work = nullptr;
    const int32_t* overflow = nullptr;
    float* image = nullptr;
    float* final_T = nullptr;
    uint32_t* n_contrib = nullptr;
    uint32_t* n_walked = nullptr;
    int W = 0, H = 0;
};

namespace {

void destroy(rara_frame_graph* fg)
{
    if (!fg) return;
    if (fg->exec) (void)hipGraphExecDestroy(fg->exec);
    if (fg->graph) (void)hipGraphDestroy(fg->graph);
    delete fg;
}

}  // namespace

extern "C" {

rara_status rara_frame_graph_create(const rara_gaussians* g, const rara_camera* shape, const rara_projected* proj,
                                    const rara_binned* bins, int64_t pair_capacity, void* workspace, size_t ws_bytes,
                                    float* image, float* final_T, uint32_t* n_contrib, uint32_t* n_walked,
                                    rara_frame_graph** out)
{
    if (!g || !shape || !proj || !bins || !image || !final_T || !n_contrib || !out || g->n <= 0)
        return RARA_ERR_INVALID;
    *out = nullptr;
    CamParams cp;
    if (!make_cam_params(shape, &cp)) return RARA_ERR_INVALID;
    rara_plane placeholder;
    placeholder.n[0] = 0.0f;
    placeholder.n[1] = 0.0f;
    placeholder.n[2] = 1.0f;
    placeholder.d = 0.0f;
    placeholder.enabled = 1;
    const float bg0[3] = {0.0f, 0.0f, 0.0f};

    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return RARA_ERR_HIP;
    rara_frame_graph* fg = new rara_frame_graph();
    rara_status st = RARA_OK;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) st = RARA_ERR_HIP;
    if (st == RARA_OK) {
        rara_status a = rara_preprocess(g, shape, &placeholder, proj, s);
        rara_status b = a == RARA_OK ? rara_bin_sort(proj, g->n, shape, pair_capacity, workspace, ws_bytes, bins, s) : a;
        rara_status c = b == RARA_OK ? rara_render(proj, g->n, bins, shape, &placeholder, bg0, image, final_T,
                                                   n_contrib, n_walked, s)
                                     : b;
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(s, &graph);
        fg->graph = graph;
        if (c != RARA_OK) st = c;
        else if (e != hipSuccess || !graph) st = RARA_ERR_HIP;
    }
    if (st == RARA_OK) {
        size_t count = 0;
        if (hipGraphGetNodes(fg->graph, nullptr, &count) != hipSuccess) st = RARA_ERR_HIP;
        std::vector<hipGraphNode_t> nodes(count);
        if (st == RARA_OK && count && hipGraphGetNodes(fg->graph, nodes.data(), &count) != hipSuccess)
            st = RARA_ERR_HIP;
        const void* pre_fn = preprocess_kernel_handle();
        const void* blend_fn = blend_kernel_handle(n_walked != nullptr);
        for (size_t k = 0; st == RARA_OK && k < count; ++k) {
            hipGraphNodeType type;
            if (hipGraphNodeGetType(nodes[k], &type) != hipSuccess || type != hipGraphNodeTypeKernel) continue;
            hipKernelNodeParams kp{};
            if (hipGraphKernelNodeGetParams(nodes[k], &kp) != hipSuccess) continue;
            if (kp.func == pre_fn) {
                fg->pre_node = nodes[k];
                fg->pre = kp;
            } else if (kp.func == blend_fn) {
                fg->blend_node = nodes[k];
                fg->blend = kp;
            }
        }
        if (st == RARA_OK && (!fg->pre_node || !fg->blend_node)) st = RARA_ERR_HIP;
    }
    if (st == RARA_OK && hipGraphInstantiate(&fg->exec, fg->graph, nullptr, nullptr, 0) != hipSuccess)
        st = RARA_ERR_HIP;
    (void)hipStreamDestroy(s);
    if (st != RARA_OK) {
        destroy(fg);
        return st;
    }
    fg->g = GaussPtrs{g->n, g->sh_degree, g->mean, g->scale, g->quat, g->opacity, g->sh};
    fg->proj = ProjPtrs{proj->label, static_cast<Splat*>(proj->splat), static_cast<RayRec*>(proj->ray), proj->depth,
                        proj->rect, proj->tiles_touched};
    fg->splat = static_cast<const Splat*>(proj->splat);
    fg->ray = static_cast<const RayRec*>(proj->ray);
    fg->vals = bins->vals;
    fg->ranges = reinterpret_cast<const uint2*>(bins->ranges);
    fg->work = bins->work;
    fg->overflow = bins->overflow;
    fg->image = image;
    fg->final_T = final_T;
    fg->n_contrib = n_contrib;
    fg->n_walked = n_walked;
    fg->W = cp.W;
    fg->H = cp.H;
    *out = fg;
    return RARA_OK;
}

rara_status rara_frame_graph_launch(rara_frame_graph* fg, const rara_camera* cam, const rara_plane* plane,
                                    const float* bg, void* stream)
{
    if (!fg || !cam || !plane || !bg) return RARA_ERR_INVALID;
    CamParams cp;
    PlaneParams pp;
    if (!make_cam_params(cam, &cp) || !make_plane_params(plane, &pp)) return RARA_ERR_INVALID;
    if (cp.W != fg->W || cp.H != fg->H) return RARA_ERR_INVALID;
    // preprocess_kernel(GaussPtrs, CamParams, PlaneParams, ProjPtrs)
    void* pre_args[4] = {&fg->g, &cp, &pp, &fg->proj};
    hipKernelNodeParams pk = fg->pre;
    pk.kernelParams = pre_args;
    pk.extra = nullptr;
    if (hipGraphExecKernelNodeSetParams(fg->exec, fg->pre_node, &pk) != hipSuccess) return RARA_ERR_HIP;
    // blend_kernel(splats, rays, vals, ranges, work, overflow, RenderParams, image, final_T, n_contrib, n_walked)
    RenderParams rp = make_render_params(cp, pp, bg);
    void* blend_args[11] = {&fg->splat, &fg->ray, &fg->vals, &fg->ranges, &fg->work, &fg->overflow,
                            &rp, &fg->image, &fg->final_T, &fg->n_contrib, &fg->n_walked};
    hipKernelNodeParams bk = fg->blend;
    bk.kernelParams = blend_args;
    bk.extra = nullptr;
    if (hipGraphExecKernelNodeSetParams(fg->exec, fg->blend_node, &bk) != hipSuccess) return RARA_ERR_HIP;
    return hipGraphLaunch(fg->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? RARA_OK : RARA_ERR_HIP;
}

void rara_frame_graph_destroy(rara_frame_graph* fg) { destroy(fg); }

}  // extern "C"
