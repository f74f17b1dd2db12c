// Frame graphs: every kernel of one frame (preprocess, binning, sort, schedule,
// blend) captured once into a HIP graph for a fixed shape (the Gaussians, the
// image size, the buffers and the pair capacity), then replayed per request.
//
// The per-request values (camera pose, clip plane, background) live in a small
// device-resident FrameParams block.  The captured preprocess and blend
// kernels read that block through a pointer, so no kernel argument of the
// instantiated graph ever changes.  A launch writes the block into pinned
// staging memory, copies it to the device on the caller's stream and then
// enqueues the graph on the same stream: the copy and the replay are ordered
// by the stream alone.  One graph launch replaces the ~25 launches of a frame.
#include <cstdlib>
#include <cstring>

#include "rara_internal.h"

using namespace rara;

struct rara_frame_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    FrameParams* dev_params = nullptr;    // device copy read by the graph's kernels
    FrameParams* host_params = nullptr;   // pinned staging of the next copy
    hipEvent_t staged = nullptr;          // the last staging copy has been consumed
    hipEvent_t done = nullptr;            // the last replay has finished
    bool launched = false;
    int W = 0, H = 0;
};

namespace {

void destroy(rara_frame_graph* fg)
{
    if (!fg) return;
    // the buffers below are freed only once the last replay has finished
    if (fg->launched && fg->done) (void)hipEventSynchronize(fg->done);
    if (fg->exec) (void)hipGraphExecDestroy(fg->exec);
    if (fg->graph) (void)hipGraphDestroy(fg->graph);
    if (fg->staged) (void)hipEventDestroy(fg->staged);
    if (fg->done) (void)hipEventDestroy(fg->done);
    if (fg->dev_params) (void)hipFree(fg->dev_params);
    if (fg->host_params) (void)hipHostFree(fg->host_params);
    delete fg;
}

bool proj_complete(const rara_projected* p)
{
    return p->label && p->splat && p->ray && p->depth && p->tiles_touched && p->tile_rec &&
           (reinterpret_cast<uintptr_t>(p->tile_rec) & 15u) == 0;
}

}  // namespace

extern "C" {

rara_status rara_frame_graph_create(const rara_gaussians* g, const rara_camera* shape, const rara_projected* proj,
                                    const rara_binned* bins, int64_t pair_capacity, void* workspace, size_t ws_bytes,
                                    float* image, float* final_T, uint32_t* n_contrib, uint32_t* n_walked,
                                    rara_frame_graph** out)
{
    if (!out) return RARA_ERR_INVALID;
    *out = nullptr;
    if (!g || !shape || !proj || !bins || !image || !final_T || !n_contrib || g->n <= 0) return RARA_ERR_INVALID;
    if (g->sh_degree < 0 || g->sh_degree > 3) return RARA_ERR_UNSUPPORTED;
    if (!sh_layout_ok(g->sh_layout)) return RARA_ERR_INVALID;
    if (!g->mean || !g->scale || !g->quat || !g->opacity || !g->sh || !proj_complete(proj)) return RARA_ERR_INVALID;
    if (!bins->vals || !bins->ranges || !bins->overflow || !bins->work) return RARA_ERR_INVALID;
    CamParams cp;
    if (!make_cam_params(shape, &cp)) return RARA_ERR_INVALID;
    if (cp.tiles_x > 65535 || cp.tiles_y > 65535) return RARA_ERR_UNSUPPORTED;

    rara_frame_graph* fg = new rara_frame_graph();
    fg->W = cp.W;
    fg->H = cp.H;
    if (hipMalloc(reinterpret_cast<void**>(&fg->dev_params), sizeof(FrameParams)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&fg->host_params), sizeof(FrameParams), hipHostMallocDefault) !=
            hipSuccess ||
        hipEventCreateWithFlags(&fg->staged, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&fg->done, hipEventDisableTiming) != hipSuccess) {
        destroy(fg);
        return RARA_ERR_HIP;
    }

    const GaussPtrs gp{g->n, g->sh_degree, g->sh_layout, g->mean, g->scale, g->quat, g->opacity, g->sh};
    const ProjPtrs pp{proj->label, static_cast<Splat*>(proj->splat), static_cast<RayRec*>(proj->ray), nullptr,
                      proj->depth, proj->tiles_touched, reinterpret_cast<ulonglong2*>(proj->tile_rec)};
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        destroy(fg);
        return RARA_ERR_HIP;
    }
    rara_status st = RARA_OK;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) st = RARA_ERR_HIP;
    if (st == RARA_OK) {
        rara_status a = launch_preprocess_fp(gp, fg->dev_params, pp, s) == hipSuccess ? RARA_OK : RARA_ERR_HIP;
        // binning depends on the camera only through the image size
        rara_status b = a == RARA_OK ? rara_bin_sort(proj, g->n, shape, pair_capacity, workspace, ws_bytes, bins, s) : a;
        rara_status c = b;
        if (c == RARA_OK)
            c = launch_blend_fp(static_cast<const Splat*>(proj->splat), static_cast<const RayRec*>(proj->ray), *bins,
                                fg->dev_params, cp.tiles_x * cp.tiles_y, image, final_T, n_contrib, n_walked,
                                s) == hipSuccess
                    ? RARA_OK
                    : RARA_ERR_HIP;
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(s, &graph);
        fg->graph = graph;
        if (c != RARA_OK) st = c;
        else if (e != hipSuccess || !graph) st = RARA_ERR_HIP;
    }
    if (st == RARA_OK && hipGraphInstantiate(&fg->exec, fg->graph, nullptr, nullptr, 0) != hipSuccess)
        st = RARA_ERR_HIP;
    (void)hipStreamDestroy(s);
    if (st != RARA_OK) {
        destroy(fg);
        return st;
    }
    *out = fg;
    return RARA_OK;
}

rara_status rara_frame_graph_launch(rara_frame_graph* fg, const rara_camera* cam, const rara_plane* plane,
                                    const float* bg, void* stream)
{
    if (!fg || !cam || !plane || !bg) return RARA_ERR_INVALID;
    FrameParams fp;
    if (!make_cam_params(cam, &fp.cam) || !make_plane_params(plane, &fp.plane)) return RARA_ERR_INVALID;
    if (fp.cam.W != fg->W || fp.cam.H != fg->H) return RARA_ERR_INVALID;
    if (fp.plane.enabled && fp.plane.count > 1) return RARA_ERR_UNSUPPORTED;   // the graph holds the one-plane blend
    fp.render = make_render_params(fp.cam, fp.plane, bg);
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the staging block may be rewritten once the previous copy out of it ran;
    // the device block and the frame's buffers once the previous replay ended
    // (a launch on another stream must not overtake it)
    if (fg->launched && hipEventSynchronize(fg->staged) != hipSuccess) return RARA_ERR_HIP;
    if (fg->launched && hipStreamWaitEvent(s, fg->done, 0) != hipSuccess) return RARA_ERR_HIP;
    std::memcpy(fg->host_params, &fp, sizeof(FrameParams));
    if (hipMemcpyAsync(fg->dev_params, fg->host_params, sizeof(FrameParams), hipMemcpyHostToDevice, s) != hipSuccess)
        return RARA_ERR_HIP;
    if (hipEventRecord(fg->staged, s) != hipSuccess) return RARA_ERR_HIP;
    fg->launched = true;
    if (hipGraphLaunch(fg->exec, s) != hipSuccess) return RARA_ERR_HIP;
    return hipEventRecord(fg->done, s) == hipSuccess ? RARA_OK : RARA_ERR_HIP;
}

void rara_frame_graph_destroy(rara_frame_graph* fg) { destroy(fg); }

}  // extern "C"
