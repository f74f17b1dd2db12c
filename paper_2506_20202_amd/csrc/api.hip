// C ABI entry points (declared in include/rara.h): argument validation,
// per-frame constants computed once on the host in double precision, and the
// kernel launches.  Nothing here allocates or synchronises.
#include <cmath>
#include <cstring>
#include <mutex>

#include "rara_internal.h"

using namespace rara;

// Workspace of rara_bin_sort_static: one copy per GPU, held from the library's
// load until the process ends.  Host code never uses this name as an address
// (it is a host-side stand-in there): the device address of each GPU's copy
// comes from hipGetSymbolAddress, below.
static __device__ __align__(256) unsigned char scratch[RARA_STATIC_WS_BYTES];

namespace {

bool make_cam(const rara_camera* c, CamParams* p)
{
    if (!c || c->width <= 0 || c->height <= 0 || !(c->near_z > 0.0f) || !(c->fx > 0.0f) || !(c->fy > 0.0f))
        return false;
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) p->R[3 * r + k] = (double)c->world_to_cam[4 * r + k];
        p->t[r] = (double)c->world_to_cam[4 * r + 3];
    }
    for (int k = 0; k < 3; ++k) p->e[k] = -(p->R[k] * p->t[0] + p->R[3 + k] * p->t[1] + p->R[6 + k] * p->t[2]);
    p->fx = c->fx;
    p->fy = c->fy;
    p->cx = c->cx;
    p->cy = c->cy;
    p->near_z = c->near_z;
    p->W = c->width;
    p->H = c->height;
    p->limx = kGuard * (p->W / 2.0) / p->fx;
    p->limy = kGuard * (p->H / 2.0) / p->fy;
    p->tiles_x = (c->width + kTile - 1) / kTile;
    p->tiles_y = (c->height + kTile - 1) / kTile;
    return true;
}

// (n, d) / |n| of one plane; false for a zero or non-finite normal or offset
bool normalise(const float* n, float d, double* out_n, double* out_d)
{
    const double n0 = n[0], n1 = n[1], n2 = n[2];
    const double len = std::sqrt(n0 * n0 + n1 * n1 + n2 * n2);
    if (!(len > 0.0) || !std::isfinite(len) || !std::isfinite((double)d)) return false;
    out_n[0] = n0 / len;
    out_n[1] = n1 / len;
    out_n[2] = n2 / len;
    *out_d = (double)d / len;
    return true;
}

bool make_plane(const rara_plane* pl, PlaneParams* p)
{
    if (!pl) return false;
    const int mode = pl->enabled, rule = mode & 3, flags = mode & ~3;
    if (rule == 3 || (flags & ~(RARA_CLIP_TIGHT | RARA_CLIP_STRICT_MISS)) || (flags && rule != RARA_CLIP_RARA))
        return false;
    if (pl->count < 0 || pl->count > kMaxPlanes) return false;
    p->enabled = mode;
    p->count = pl->count > 1 ? pl->count : 1;
    p->n[0] = p->n[1] = p->n[2] = 0.0;
    p->d = 0.0;
    for (int k = 0; k < kMaxPlanes - 1; ++k) p->xn[k][0] = p->xn[k][1] = p->xn[k][2] = p->xd[k] = 0.0;
    if (!p->enabled) return true;
    if (!normalise(pl->n, pl->d, p->n, &p->d)) return false;
    for (int k = 1; k < p->count; ++k)
        if (!normalise(pl->extra[k - 1], pl->extra[k - 1][3], p->xn[k - 1], &p->xd[k - 1])) return false;
    return true;
}

int ceil_log2(int64_t v)
{
    int b = 0;
    while ((int64_t(1) << b) < v) ++b;
    return b;
}

bool proj_ok(const rara_projected* p)
{
    return p && p->label && p->splat && p->ray && p->depth && p->tiles_touched && p->tile_rec &&
           (reinterpret_cast<uintptr_t>(p->tile_rec) & 15u) == 0;
}

ProjPtrs proj_ptrs(const rara_projected* p)
{
    return ProjPtrs{p->label, static_cast<Splat*>(p->splat), static_cast<RayRec*>(p->ray),
                    reinterpret_cast<float2*>(p->ray_ext), p->depth,
                    p->tiles_touched, reinterpret_cast<ulonglong2*>(p->tile_rec)};
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices];   // device address of `scratch` on each device, once looked up

// Device address of the current device's copy of `scratch`, looked up on the
// first call on that device (with it current); nullptr on failure.
void* static_workspace()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

// Argument checks of rara_bin_sort (everything but the workspace); on success
// fills the camera parameters.
rara_status check_bin_args(const rara_projected* proj, int64_t n, const rara_camera* cam, int64_t pair_capacity,
                           const rara_binned* out, CamParams* cp)
{
    if (!proj || n < 0 || !out) return RARA_ERR_INVALID;
    if (pair_capacity < 1 || pair_capacity >= (int64_t(1) << 31)) return RARA_ERR_INVALID;
    if (n > 0 && !proj_ok(proj)) return RARA_ERR_INVALID;
    if (!out->keys || !out->vals || !out->ranges || !out->num_pairs || !out->overflow || !out->work)
        return RARA_ERR_INVALID;
    if (!make_cam(cam, cp)) return RARA_ERR_INVALID;
    return RARA_OK;
}

// The launches of rara_bin_sort on a checked frame and a large enough workspace.
rara_status bin_sort_launch(const rara_projected* proj, int64_t n, const CamParams& cp, int64_t pair_capacity,
                            void* workspace, const rara_binned* out, hipStream_t s)
{
    BinWorkspace ws;
    bin_workspace_layout(n, pair_capacity, &ws, static_cast<char*>(workspace));
    const int num_tiles = cp.tiles_x * cp.tiles_y;
    int tile_passes = (ceil_log2(num_tiles) + kRadixBits - 1) / kRadixBits;
    if (tile_passes < 1) tile_passes = 1;   // the last pass also writes the 64-bit keys
    hipError_t e = launch_bin(proj_ptrs(proj), n, cp, pair_capacity, ws, *out, tile_passes, s);
    if (e == hipSuccess && n == 0) e = launch_ranges_clear(*out, num_tiles, s);   // else set by launch_bin
    if (e == hipSuccess) e = launch_plan(*out, num_tiles, s);
    return e == hipSuccess ? RARA_OK : RARA_ERR_HIP;
}

}  // namespace

bool rara::make_cam_params(const rara_camera* c, CamParams* p) { return make_cam(c, p); }
bool rara::make_plane_params(const rara_plane* pl, PlaneParams* p) { return make_plane(pl, p); }

RenderParams rara::make_render_params(const CamParams& cp, const PlaneParams& pp, const float* bg)
{
    RenderParams rp;
    rp.W = cp.W;
    rp.H = cp.H;
    rp.tiles_x = cp.tiles_x;
    rp.tiles_y = cp.tiles_y;
    rp.num_tiles = cp.tiles_x * cp.tiles_y;
    rp.plane_enabled = pp.enabled;
    // per-pixel rate of the plane value along the pixel ray: (R_c n)_{x,y} / f_{x,y}
    const double rn0 = cp.R[0] * pp.n[0] + cp.R[1] * pp.n[1] + cp.R[2] * pp.n[2];
    const double rn1 = cp.R[3] * pp.n[0] + cp.R[4] * pp.n[1] + cp.R[5] * pp.n[2];
    rp.ax = (float)(rn0 / cp.fx);
    rp.ay = (float)(rn1 / cp.fy);
    rp.plane_count = pp.count;
    for (int k = 0; k < kMaxPlanes - 1; ++k) {
        const double* xn = pp.xn[k];
        const double x0 = cp.R[0] * xn[0] + cp.R[1] * xn[1] + cp.R[2] * xn[2];
        const double x1 = cp.R[3] * xn[0] + cp.R[4] * xn[1] + cp.R[5] * xn[2];
        rp.xax[k] = (float)(x0 / cp.fx);
        rp.xay[k] = (float)(x1 / cp.fy);
    }
    rp.bg[0] = bg[0];
    rp.bg[1] = bg[1];
    rp.bg[2] = bg[2];
    return rp;
}

size_t rara::bin_workspace_layout(int64_t n, int64_t cap, BinWorkspace* ws, char* base)
{
    auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
    const int64_t nn = n > 0 ? n : 1;
    int64_t scan_blocks = (nn + kScanBlock - 1) / kScanBlock;
    const int64_t depth_blocks = (nn + kDepthSortTile - 1) / kDepthSortTile;
    int64_t tile_blocks = (cap + kSortTile - 1) / kSortTile;
    if (tile_blocks < 1) tile_blocks = 1;
    const int64_t hist_cols = depth_blocks > tile_blocks ? depth_blocks : tile_blocks;
    size_t off = 0;
    BinWorkspace w;
    w.scan_blocks = scan_blocks;
    w.depth_blocks = depth_blocks;
    w.tile_blocks = tile_blocks;
    w.block_sums = reinterpret_cast<uint32_t*>(base + off);
    off += align((size_t)scan_blocks * 4);
    w.dcount = reinterpret_cast<int64_t*>(base + off);
    off += 256;
    for (int b = 0; b < 2; ++b) {
        w.dkeys[b] = reinterpret_cast<uint32_t*>(base + off);
        off += align((size_t)nn * 4);
        w.dvals[b] = reinterpret_cast<uint32_t*>(base + off);
        off += align((size_t)nn * 4);
    }
    // 16 B per Gaussian over dkeys[1], dvals[1] and 8 B more per Gaussian after them
    w.drec = reinterpret_cast<ulonglong2*>(w.dkeys[1]);
    off += align((size_t)nn * 8);
    w.tkeys = reinterpret_cast<uint32_t*>(base + off);
    off += align((size_t)cap * 4);
    w.tvals = reinterpret_cast<uint32_t*>(base + off);
    off += align((size_t)cap * 4);
    w.hist = reinterpret_cast<uint32_t*>(base + off);
    off += align((size_t)kRadix * hist_cols * 4);
    w.digit_totals = reinterpret_cast<uint32_t*>(base + off);
    off += align((size_t)kRadix * 4);
    if (ws) *ws = w;
    return off;
}

extern "C" {

const char* rara_status_string(rara_status s)
{
    switch (s) {
    case RARA_OK: return "ok";
    case RARA_ERR_INVALID: return "invalid argument";
    case RARA_ERR_CAPACITY: return "pair capacity exceeded";
    case RARA_ERR_HIP: return "HIP runtime error";
    case RARA_ERR_UNSUPPORTED: return "unsupported configuration";
    case RARA_ERR_SCRATCH: return "frame needs more than the static workspace (RARA_STATIC_WS_BYTES)";
    }
    return "unknown status";
}

const char* rara_version(void) { return "rara 0.1 gfx950"; }

size_t rara_workspace_bytes(int32_t which, int64_t n, int64_t pair_capacity, int32_t width, int32_t height)
{
    if (n < 0 || width <= 0 || height <= 0) return 0;
    if (which == RARA_WS_BIN_SORT) {
        if (pair_capacity < 1 || pair_capacity >= (int64_t(1) << 31)) return 0;
        return bin_workspace_layout(n, pair_capacity, nullptr, nullptr);
    }
    if (which == RARA_WS_BACKWARD) {
        if (pair_capacity < 1 || pair_capacity >= (int64_t(1) << 30)) return 0;
        return backward_workspace_bytes(n, pair_capacity, width, height);
    }
    return 0;
}

rara_status rara_preprocess(const rara_gaussians* g, const rara_camera* cam, const rara_plane* plane,
                            const rara_projected* out, void* stream)
{
    if (!g || g->n < 0 || !out) return RARA_ERR_INVALID;
    if (g->sh_degree < 0 || g->sh_degree > 3) return RARA_ERR_UNSUPPORTED;
    if (!sh_layout_ok(g->sh_layout)) return RARA_ERR_INVALID;
    CamParams cp;
    PlaneParams pp;
    if (!make_cam(cam, &cp) || !make_plane(plane, &pp)) return RARA_ERR_INVALID;
    if (cp.tiles_x > 65535 || cp.tiles_y > 65535) return RARA_ERR_UNSUPPORTED;
    if (g->n == 0) return RARA_OK;
    if (!g->mean || !g->scale || !g->quat || !g->opacity || !g->sh || !proj_ok(out)) return RARA_ERR_INVALID;
    if (pp.enabled && pp.count > 1 && !out->ray_ext) return RARA_ERR_INVALID;   // a region's further planes
    GaussPtrs gp{g->n, g->sh_degree, g->sh_layout, g->mean, g->scale, g->quat, g->opacity, g->sh};
    const hipError_t e = launch_preprocess(gp, cp, pp, proj_ptrs(out), static_cast<hipStream_t>(stream));
    return e == hipSuccess ? RARA_OK : RARA_ERR_HIP;
}

rara_status rara_bin_sort(const rara_projected* proj, int64_t n, const rara_camera* cam, int64_t pair_capacity,
                          void* workspace, size_t ws_bytes, const rara_binned* out, void* stream)
{
    CamParams cp;
    const rara_status st = check_bin_args(proj, n, cam, pair_capacity, out, &cp);
    if (st != RARA_OK) return st;
    if (!workspace || ws_bytes < bin_workspace_layout(n, pair_capacity, nullptr, nullptr)) return RARA_ERR_INVALID;
    return bin_sort_launch(proj, n, cp, pair_capacity, workspace, out, static_cast<hipStream_t>(stream));
}

rara_status rara_bin_sort_static(const rara_projected* proj, int64_t n, const rara_camera* cam,
                                 int64_t pair_capacity, const rara_binned* out, void* stream)
{
    CamParams cp;
    const rara_status st = check_bin_args(proj, n, cam, pair_capacity, out, &cp);
    if (st != RARA_OK) return st;
    if (bin_workspace_layout(n, pair_capacity, nullptr, nullptr) > RARA_STATIC_WS_BYTES) return RARA_ERR_SCRATCH;
    void* ws = static_workspace();
    if (!ws) return RARA_ERR_HIP;
    return bin_sort_launch(proj, n, cp, pair_capacity, ws, out, static_cast<hipStream_t>(stream));
}

rara_status rara_render(const rara_projected* proj, int64_t n, const rara_binned* bins, const rara_camera* cam,
                        const rara_plane* plane, const float* bg, float* image, float* final_T, uint32_t* n_contrib,
                        uint32_t* n_walked, uint32_t* n_eval, void* stream)
{
    if (!proj || n < 0 || !bins || !bg || !image || !final_T || !n_contrib) return RARA_ERR_INVALID;
    if (!proj->splat || !proj->ray || !bins->vals || !bins->ranges || !bins->overflow || !bins->work)
        return RARA_ERR_INVALID;
    CamParams cp;
    PlaneParams pp;
    if (!make_cam(cam, &cp) || !make_plane(plane, &pp)) return RARA_ERR_INVALID;
    if (pp.enabled && pp.count > 1 && !proj->ray_ext) return RARA_ERR_INVALID;
    const RenderParams rp = make_render_params(cp, pp, bg);
    const hipError_t e = launch_blend(static_cast<const Splat*>(proj->splat), static_cast<const RayRec*>(proj->ray),
                                      reinterpret_cast<const float2*>(proj->ray_ext), *bins, rp, image, final_T,
                                      n_contrib, n_walked, n_eval, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? RARA_OK : RARA_ERR_HIP;
}

rara_status rara_render_batch(const rara_render_item* items, int32_t count, void* stream)
{
    if (!items || count < 1 || count > RARA_MAX_BATCH) return RARA_ERR_INVALID;
    BatchArgs a;
    a.count = count;
    for (int i = 0; i < count; ++i) {
        const rara_render_item& it = items[i];
        const rara_projected* proj = it.proj;
        const rara_binned* bins = it.bins;
        if (!proj || it.n < 0 || !bins || !it.bg || !it.image || !it.final_T || !it.n_contrib) return RARA_ERR_INVALID;
        if (!proj->splat || !proj->ray || !bins->vals || !bins->ranges || !bins->overflow || !bins->work)
            return RARA_ERR_INVALID;
        CamParams cp;
        PlaneParams pp;
        if (!make_cam(it.cam, &cp) || !make_plane(it.plane, &pp)) return RARA_ERR_INVALID;
        if (pp.enabled && pp.count > 1) return RARA_ERR_UNSUPPORTED;
        BatchItem& b = a.items[i];
        b.splat = static_cast<const Splat*>(proj->splat);
        b.ray = static_cast<const RayRec*>(proj->ray);
        b.vals = bins->vals;
        b.ranges = reinterpret_cast<const uint2*>(bins->ranges);
        b.work = bins->work;
        b.overflow = bins->overflow;
        b.image = it.image;
        b.final_T = it.final_T;
        b.n_contrib = it.n_contrib;
        b.p = make_render_params(cp, pp, it.bg);
        b.first_block = 0;
    }
    const hipError_t e = launch_blend_batch(a, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? RARA_OK : RARA_ERR_HIP;
}

rara_status rara_render_backward(const rara_gaussians* g, const rara_camera* cam, const rara_plane* plane,
                                 const float* bg, const rara_projected* proj, const rara_binned* bins,
                                 int64_t pair_capacity, const float* final_T, const uint32_t* n_contrib,
                                 const float* dL_dimage, const rara_grads* grads, void* workspace, size_t ws_bytes,
                                 void* stream)
{
    if (!g || g->n < 0 || !bg || !proj || !bins || !final_T || !n_contrib || !dL_dimage || !grads || !workspace)
        return RARA_ERR_INVALID;
    if (pair_capacity < 1 || pair_capacity >= (int64_t(1) << 30)) return RARA_ERR_INVALID;
    if (g->sh_degree < 0 || g->sh_degree > 3) return RARA_ERR_UNSUPPORTED;
    if (!sh_layout_ok(g->sh_layout)) return RARA_ERR_INVALID;
    if (!proj_ok(proj) || !bins->vals || !bins->ranges || !bins->overflow || !bins->work || !bins->pair_start)
        return RARA_ERR_INVALID;
    if (!grads->plane || (g->n > 0 && (!grads->mean || !grads->scale || !grads->quat || !grads->opacity || !grads->sh)))
        return RARA_ERR_INVALID;
    if (g->n > 0 && (!g->mean || !g->scale || !g->quat || !g->opacity || !g->sh)) return RARA_ERR_INVALID;
    CamParams cp;
    PlaneParams pp;
    if (!make_cam(cam, &cp) || !make_plane(plane, &pp)) return RARA_ERR_INVALID;
    if (pp.enabled && pp.count > 1) return RARA_ERR_UNSUPPORTED;   // gradients of one plane only
    if (ws_bytes < backward_workspace_bytes(g->n, pair_capacity, cp.W, cp.H)) return RARA_ERR_INVALID;
    const RenderParams rp = make_render_params(cp, pp, bg);
    const double len = pp.enabled ? std::sqrt((double)plane->n[0] * plane->n[0] + (double)plane->n[1] * plane->n[1] +
                                              (double)plane->n[2] * plane->n[2])
                                  : 1.0;
    GaussPtrs gp{g->n, g->sh_degree, g->sh_layout, g->mean, g->scale, g->quat, g->opacity, g->sh};
    const hipError_t e = launch_backward(gp, cp, pp, len, proj_ptrs(proj), *bins, pair_capacity, rp, final_T,
                                         n_contrib, dL_dimage, *grads, workspace, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? RARA_OK : RARA_ERR_HIP;
}

}  // extern "C"
