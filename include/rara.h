/*
 * rara.h -- C ABI of the MI355X (gfx950) RaRa-clipped Gaussian-splatting
 * renderer ("RaRa Clipper: A Clipper for Gaussian Splatting Based on Ray
 * Tracer and Rasterizer", arXiv 2506.20202).
 *
 * One frame is three calls on one HIP stream:
 *   rara_preprocess  classify + project every Gaussian          (Sec. 3.2, eqs. 9-10)
 *   rara_bin_sort    tile binning and tile|depth radix sort      (Sec. 3.1, depth order)
 *   rara_render      per-tile front-to-back blend with the RaRa
 *                    decay weight for CUTOFF Gaussians           (eqs. 2, 4-8, 11, 12; Alg. 1)
 * and the differentiable path adds
 *   rara_render_backward  gradients of a pixel loss w.r.t. the Gaussians and
 *                    the plane (not in the paper, which is render-only).
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers owned by the caller; the library
 *     allocates no device memory and keeps no state between calls (frame
 *     graphs, below, are explicit host-side handles).  Struct arguments are
 *     read on the host during the call only.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *     enqueues work; results are ready when the stream reaches them.
 *   - Argument errors are reported synchronously (RARA_ERR_INVALID) before
 *     anything is enqueued.  A failed kernel launch returns RARA_ERR_HIP.
 *     Pair-capacity overflow is a device-side condition: see rara_bin_sort.
 *   - Units: scale is the linear standard deviation sigma (not log), opacity
 *     is the density delta after any activation, quat need not be unit length
 *     (it is normalised), the plane need not be normalised ((n, d)/|n| is
 *     used, |n| = 0 is rejected).  Camera: x right, y down, z forward; pixel
 *     (i, j) has its centre at image coordinate (i, j) = (fx x/z + cx,
 *     fy y/z + cy).
 *   - Tiles are 16 x 16 pixels, row-major, tiles_x = ceil(W/16).
 *   - No exception, longjmp or abort crosses this interface.
 */
#ifndef RARA_H
#define RARA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RARA_OK = 0,
    RARA_ERR_INVALID = 1,     /* bad argument (null pointer, size, plane, workspace too small) */
    RARA_ERR_CAPACITY = 2,    /* reserved for callers: device overflow flag was found set   */
    RARA_ERR_HIP = 3,         /* a HIP runtime call or kernel launch failed                 */
    RARA_ERR_UNSUPPORTED = 4, /* e.g. sh_degree > 3, image larger than 65535 tiles a side   */
    RARA_ERR_SCRATCH = 5      /* rara_bin_sort_static: the frame needs more workspace than
                                 RARA_STATIC_WS_BYTES                                       */
} rara_status;

/* Labels of Sec. 3.2 (written by rara_preprocess, one byte per Gaussian). */
enum { RARA_LABEL_INVISIBLE = 0, RARA_LABEL_VISIBLE = 1, RARA_LABEL_CUTOFF = 2 };

/* Layouts of the SH coefficients (rara_gaussians.sh_layout). */
enum {
    RARA_SH_COEFF_MAJOR = 0,    /* sh [(sh_degree+1)^2][3][n]                        */
    RARA_SH_GAUSSIAN_MAJOR = 1  /* sh [n][(sh_degree+1)^2][3]: one Gaussian's
                                   coefficients contiguous, so that a frame reads
                                   only the drawn Gaussians' cache lines (align
                                   the array to 16 bytes for vector loads)       */
};

/* Gaussians (Sec. 3.1: centre mu, covariance R S^2 R^T, opacity density
 * delta, colour c as real spherical harmonics of degree sh_degree <= 3).
 * Structure-of-arrays float32, n columns each:
 *   mean [3][n], scale [3][n], quat [4][n] (w, x, y, z), opacity [n],
 *   sh in the layout sh_layout names (coefficient-major, then RGB channel,
 *   when 0, the value of a zero-initialised struct).  Any other sh_layout is
 *   RARA_ERR_INVALID. */
typedef struct {
    int64_t n;
    int32_t sh_degree;
    int32_t sh_layout;
    const float* mean;
    const float* scale;
    const float* quat;
    const float* opacity;
    const float* sh;
} rara_gaussians;

/* Pinhole camera (Algorithm 1's pose T and resolution W x H): world point x
 * maps to R_c x + t_c with world_to_cam = [R_c | t_c] row-major 3x4.
 * Gaussians with camera depth <= near_z are not drawn. */
typedef struct {
    float world_to_cam[12];
    float fx, fy, cx, cy;
    int32_t width, height;
    float near_z;
} rara_camera;

/* Clipping plane of eq. (3): n.x + d = 0, the half-space n points into is
 * visible.  `enabled` is the clip mode:
 *   RARA_CLIP_OFF   0  no clipping (every label VISIBLE);
 *   RARA_CLIP_RARA  1  the paper's method: three-way labels of Sec. 3.2 with
 *                      r = 3 max(sigma), CUTOFF Gaussians weighted by eq. (11);
 *   RARA_CLIP_HARD  2  hard clipping, the baseline of Sec. 1 and Table 1: a
 *                      Gaussian is kept whole when its centre is on the
 *                      visible side (n.mu + d >= 0) and dropped otherwise;
 * and, only together with RARA_CLIP_RARA, the flags
 *   RARA_CLIP_TIGHT        4  r = 3 |S R^T n|, the exact half-width of the
 *                             3-sigma ellipsoid along the normal (Sec. 3.2
 *                             notes that 3 max(sigma) over-estimates it);
 *   RARA_CLIP_STRICT_MISS  8  a pixel ray that misses a CUTOFF Gaussian's
 *                             ellipsoid gets w = 1 only when its point closest
 *                             to the centre (whitened metric) is visible, else
 *                             0, instead of w = 1 (the sub-pixel case of the
 *                             paper's closing discussion).
 * Any other value is RARA_ERR_INVALID.
 *
 * Clip regions (the extension to other clipping primitives that Sec. 6
 * names; Sec. 2 cites box clipping of multi-layer fields): with count >= 2
 * the visible region is the intersection of the half-spaces of (n, d) and
 * extra[0 .. count-2], each (n.x, n.y, n.z, d); an axis-aligned box is six.
 * Every mode applies with the plane read as the region: a Gaussian is
 * INVISIBLE when it is beyond r outside any plane, VISIBLE when it is beyond
 * r inside every plane, CUTOFF otherwise; hard clipping keeps it when its
 * centre is inside every half-space; eq. (11)'s L_vis is the part of the
 * chord inside every half-space; a strict miss needs the closest approach
 * inside every half-space.  count 0 or 1 is the single plane (n, d).
 * Regions need rara_projected.ray_ext; rara_render_backward and frame graphs
 * take a single plane only (RARA_ERR_UNSUPPORTED otherwise).  A count above
 * RARA_MAX_PLANES is RARA_ERR_INVALID. */
enum {
    RARA_CLIP_OFF = 0,
    RARA_CLIP_RARA = 1,
    RARA_CLIP_HARD = 2,
    RARA_CLIP_TIGHT = 4,
    RARA_CLIP_STRICT_MISS = 8
};
#define RARA_MAX_PLANES 8
typedef struct {
    float n[3];
    float d;
    int32_t enabled;
    int32_t count;
    float extra[RARA_MAX_PLANES - 1][4];
} rara_plane;

/* Per-Gaussian results of rara_preprocess (caller-allocated, n entries each).
 *   label [n] uint8            Sec. 3.2 label of every Gaussian.
 *   splat [n] 48-byte records  written for drawn Gaussians only:
 *        double mean2d[2]      projected centre (pixels)
 *        float  conic[3]       inverse 2D covariance (a, b, c) = [[a, b], [b, c]]
 *        float  opacity        delta
 *        float  rgb[3]         colour, clamped at 0
 *        uint32 label          the label in the low byte; for a CUTOFF Gaussian,
 *                              bit 16 + k is set when plane k of the plane or
 *                              region does not hold its whole 3-sigma ellipsoid
 *                              on the visible side: n_k.mu + d_k <= 3 |S R^T n_k|
 *   ray  [n] 48-byte records   written for drawn CUTOFF Gaussians only: the
 *        whitened-space ray set-up of eq. (4) (12 floats; layout private to the
 *        library, consumed by rara_render / rara_render_backward).
 *   depth [n] float            camera depth of drawn Gaussians.
 *   tiles_touched [n] uint32   number of tiles the Gaussian is listed in (its
 *                              pair count) if drawn, else 0.
 *   tile_rec [n][2] uint64     per drawn Gaussian (zeros otherwise): word 0 its
 *                              tile rectangle tx0, ty0, tx1, ty1 (half-open; four
 *                              uint16, lowest first), word 1 the listed-tile mask: for a
 *                              rectangle of at most 64 tiles, bit k set when the
 *                              k-th tile of the rectangle (row by row) is
 *                              listed; 0 for a larger rectangle.  16-byte
 *                              aligned.  A tile is listed when the Gaussian can reach
 *                              alpha >= 1/255 in it: the minimum of its quadratic
 *                              form (float32 conic) over the box of the tile's
 *                              pixel centres is at most 1.02 * 2 ln(255 delta)
 *                              + 0.02 (none when 255 delta <= 1; all when the
 *                              float32 conic is not positive definite).  A
 *                              larger rectangle lists every tile.  Tiles left
 *                              out hold no pixel the 1/255 skip of Sec. 3.1
 *                              would not skip, so the frame is unchanged.
 *   ray_ext [n][RARA_MAX_PLANES-1][2] float   optional (NULL with a single
 *                              plane; required by a clip region): for drawn
 *                              CUTOFF Gaussians, the ray terms of the region's
 *                              further planes (private layout, like ray).
 * A Gaussian is drawn when it is not INVISIBLE, its depth exceeds near_z and
 * its footprint ceil(3 sqrt(lambda_max)) px box meets the image. */
typedef struct {
    uint8_t* label;
    void* splat;
    void* ray;
    float* depth;
    uint32_t* tiles_touched;
    float* ray_ext;
    uint64_t* tile_rec;
} rara_projected;

/* Binned, depth-sorted (tile, Gaussian) pairs (caller-allocated).
 *   keys [pair_capacity] uint64  (tile << 32) | float32 bits of depth, sorted ascending,
 *                                ties in Gaussian-index order.
 *   vals [pair_capacity] uint32  Gaussian index of each key.
 *   ranges [tiles][2] uint32     [start, end) of each tile's pairs.
 *   num_pairs [1] int64          total pairs P of the frame (written even on overflow).
 *   overflow  [1] int32          set to 1 when P > pair_capacity, else 0.
 *   work [tiles + 1] uint32      blend schedule written by rara_bin_sort: the
 *                                tiles with long lists, then the others; the last
 *                                entry is the number of long-list tiles.
 *   pair_start [n] uint32        optional (NULL: not written): for each drawn
 *                                Gaussian, the position of its first pair in emission
 *                                order (drawn Gaussians by depth, each one's listed
 *                                tiles row by row over its rectangle); not written for
 *                                Gaussians that are not drawn.  Required by
 *                                rara_render_backward, which gives every (tile,
 *                                Gaussian) pair its own gradient slot; a frame that
 *                                is only rendered can leave it NULL.
 *   keys_scratch                 0: keys holds the sorted keys above.  Nonzero: keys
 *                                only serves as scratch memory of the sort and its
 *                                contents are unspecified afterwards; rara_render and
 *                                rara_render_backward do not read it, and the last
 *                                sort pass then skips a per-pair gather of the depth.
 *                                A zero-initialised struct keeps the sorted keys. */
typedef struct {
    uint64_t* keys;
    uint32_t* vals;
    uint32_t* ranges;
    int64_t* num_pairs;
    int32_t* overflow;
    uint32_t* work;
    uint32_t* pair_start;
    int32_t keys_scratch;
} rara_binned;

/* Gradients (caller-allocated; overwritten, not accumulated):
 *   mean [3][n], scale [3][n], quat [4][n], opacity [n], and sh in the
 *   layout of the inputs' sh (sh_layout), with respect to the raw
 *   rara_gaussians inputs, and plane [4] with respect to the raw (n, d) of
 *   rara_plane. */
typedef struct {
    float* mean;
    float* scale;
    float* quat;
    float* opacity;
    float* sh;
    float* plane;
} rara_grads;

/* Workspace kinds for rara_workspace_bytes. */
enum { RARA_WS_BIN_SORT = 0, RARA_WS_BACKWARD = 1 };

/* Bytes of device workspace needed by rara_bin_sort (which = RARA_WS_BIN_SORT)
 * or rara_render_backward (RARA_WS_BACKWARD) for n Gaussians, the given pair
 * capacity and image size.  Returns 0 for invalid arguments. */
size_t rara_workspace_bytes(int32_t which, int64_t n, int64_t pair_capacity, int32_t width, int32_t height);

/* Sec. 3.2 (classification, Algorithm 1 step 1) and Sec. 3.4 eqs. (9)-(10)
 * (EWA projection) for all g->n Gaussians, plus colour, footprint and the
 * cutoff ray set-up.  Fills every array of *out (see rara_projected).
 * Errors: RARA_ERR_INVALID for n < 0, null pointers (when n > 0), a
 * non-positive image size or near_z, |plane n| = 0 with the plane enabled;
 * RARA_ERR_UNSUPPORTED for sh_degree outside 0..3 or more than 65535 tiles per
 * side. */
rara_status rara_preprocess(const rara_gaussians* g, const rara_camera* cam, const rara_plane* plane,
                            const rara_projected* out, void* stream);

/* Tile binning and depth sort (the "sorted by depth" order of Sec. 3.1, per
 * 16x16 tile): exclusive scan of tiles_touched, one (tile|depth, index) pair
 * per drawn Gaussian and listed tile (tile_rec), LSD radix sort on the
 * significant key bits, and per-tile ranges.  Needs `ws_bytes` >= rara_workspace_bytes(
 * RARA_WS_BIN_SORT, n, pair_capacity, W, H) bytes of device workspace.
 * Overflow: if the frame has more than pair_capacity pairs, *num_pairs holds
 * the required count and *overflow is 1.  The sorted pairs, ranges and
 * schedule are then not produced, and the contents of keys, vals, ranges,
 * work, pair_start and the workspace are unspecified (pairs that fit may
 * have been written).  rara_render leaves its outputs untouched and
 * rara_render_backward writes zero gradients for such a frame (both check the
 * flag on the device); the caller checks after synchronising and retries
 * with a larger capacity.
 * Errors: RARA_ERR_INVALID for null pointers, n < 0, pair_capacity outside
 * [1, 2^31), or a workspace that is too small. */
rara_status rara_bin_sort(const rara_projected* proj, int64_t n, const rara_camera* cam, int64_t pair_capacity,
                          void* workspace, size_t ws_bytes, const rara_binned* out, void* stream);

/* Front-to-back compositing (eq. 2) per pixel over its tile's sorted list,
 * with alpha = min(0.99, delta exp(-1/2 dx^T conic dx) w) (eq. 12 and
 * Algorithm 1 step 3), skip when alpha < 1/255, stop before transmittance
 * would drop below 1e-4.  w = 1 for VISIBLE Gaussians; for CUTOFF Gaussians
 * w is eq. (11): the visible fraction of the pixel ray's chord through the
 * 3-sigma ellipsoid (eqs. 4-8), and 1 when the ray meets it in fewer than two
 * points with t >= 0.
 * Outputs (device, caller-allocated): image [3][H][W] float = C + T bg,
 * final_T [H][W] float, n_contrib [H][W] uint32 (1-based index in the tile
 * list of the last composited Gaussian, used by the backward), and optional
 * n_walked [H][W] uint32 (entries examined; may be NULL), and optional
 * n_eval [2][H][W] uint32 (may be NULL), a measure of the work done rather
 * than part of the method: plane 0 counts the entries whose alpha the launch
 * evaluated for the pixel while the pixel was live (the entries a
 * conservative test lets reach the pixel's 8x8 quadrant, or in a long list
 * its 8x2 strip, with alpha >= 1/255), plane 1 how many of those needed the
 * clip weight of a CUTOFF Gaussian.  bg is a host array of 3 floats.
 * Errors: RARA_ERR_INVALID for null pointers or a camera that differs in size
 * from the one binned (not detectable: the caller must pass the same camera). */
rara_status rara_render(const rara_projected* proj, int64_t n, const rara_binned* bins, const rara_camera* cam,
                        const rara_plane* plane, const float* bg, float* image, float* final_T,
                        uint32_t* n_contrib, uint32_t* n_walked, uint32_t* n_eval, void* stream);

/* Several frames' blends in one launch, for serving many requests at once:
 * item i is the rara_render of its own frame (its own projected Gaussians,
 * binned pairs, camera, plane, background and outputs, any image size), and
 * the launch's workgroups are split among the items, so that small frames
 * share the GPU instead of running as separate small launches.  Each item's
 * outputs are bit-identical to rara_render's with the same arguments (n_walked
 * and n_eval are not produced).  An item whose overflow flag is set is left
 * untouched, as by rara_render.  The items are read on the host during the
 * call; their frames must already be binned on `stream` (or ordered before it).
 * Errors: RARA_ERR_INVALID for count outside [1, RARA_MAX_BATCH] or an item
 * rara_render would reject; RARA_ERR_UNSUPPORTED for a clip region (more than
 * one plane) in any item. */
#define RARA_MAX_BATCH 16
typedef struct {
    const rara_projected* proj;
    int64_t n;
    const rara_binned* bins;
    const rara_camera* cam;
    const rara_plane* plane;
    const float* bg;           /* host array of 3 floats */
    float* image;              /* [3][H][W] */
    float* final_T;            /* [H][W] */
    uint32_t* n_contrib;       /* [H][W] */
} rara_render_item;
rara_status rara_render_batch(const rara_render_item* items, int32_t count, void* stream);

/* Gradient of a scalar loss L given dL/dimage [3][H][W] (device), through the
 * blend (re-walking each tile list from n_contrib back to front, with the
 * transmittance rebuilt by division) and the clip weight of eq. (11), then
 * through projection and colour to the raw inputs and the plane.  g, cam,
 * plane, bg, proj, bins, final_T and n_contrib must be those of the forward
 * frame, and pair_capacity the one rara_bin_sort was given.  Needs `ws_bytes`
 * >= rara_workspace_bytes(RARA_WS_BACKWARD, n, pair_capacity, W, H) bytes of
 * device workspace: one 84-byte gradient slot per pair of capacity, written
 * once by the tile that holds the pair, then summed per Gaussian, so no
 * per-Gaussian atomics are used and repeated runs give identical gradients
 * except for the plane (a few per-tile float atomics).  Every array of *grads
 * is overwritten (Gaussians that were not drawn get zero).
 * A frame whose overflow flag is set gets zero for every gradient, the
 * plane's included (checked on the device; no pair slot is read).
 * Errors: as rara_render, plus RARA_ERR_INVALID for a short workspace, a
 * pair_capacity outside [1, 2^30), null gradient arrays or a null
 * bins->pair_start. */
rara_status rara_render_backward(const rara_gaussians* g, const rara_camera* cam, const rara_plane* plane,
                                 const float* bg, const rara_projected* proj, const rara_binned* bins,
                                 int64_t pair_capacity, const float* final_T, const uint32_t* n_contrib,
                                 const float* dL_dimage, const rara_grads* grads, void* workspace, size_t ws_bytes,
                                 void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): rara_bin_sort
 * with its workspace taken from a static device array of the library instead
 * of a caller buffer.  Same arguments (minus the workspace), same outputs and
 * overflow contract, same kernels: the results are bit-identical to
 * rara_bin_sort's.  The call allocates nothing; on its first call on a device
 * it looks up that device's copy of the array (each GPU holds its own copy of
 * RARA_STATIC_WS_BYTES = 64 MiB from the library's load until the process
 * ends).  Every call on a GPU shares that GPU's array: calls of one process
 * that overlap on one GPU (on several streams or from several threads) race
 * and must be serialised by the caller.  No part of the array needs to start
 * at zero (every byte a call reads, the call has written first), so the
 * previous call's contents do no harm.
 * Errors: those of rara_bin_sort, and RARA_ERR_SCRATCH (before anything is
 * enqueued) when rara_workspace_bytes(RARA_WS_BIN_SORT, n, pair_capacity, W, H)
 * exceeds RARA_STATIC_WS_BYTES (it does not for 1M Gaussians and 5M pairs
 * of capacity); RARA_ERR_HIP when the array's address cannot be found. */
#define RARA_STATIC_WS_BYTES ((size_t)64 << 20)
rara_status rara_bin_sort_static(const rara_projected* proj, int64_t n, const rara_camera* cam,
                                 int64_t pair_capacity, const rara_binned* out, void* stream);

/* Frame graphs (for serving many requests of one shape): the kernels of one
 * frame (rara_preprocess + rara_bin_sort + rara_render) captured once into a
 * HIP graph for fixed Gaussians, image size, buffers and pair capacity.  The
 * camera pose, plane and background of a request live in a small device
 * block owned by the handle; rara_frame_graph_launch copies them there on
 * `stream` (from pinned staging memory) and enqueues the graph after the copy
 * on the same stream: one copy and one graph launch per frame.  The results
 * are those of the three calls with the same arguments.  `shape` fixes the
 * image size (a launch with another size is rejected); its pose only serves
 * the capture.  n_walked may be NULL.  The handle owns a HIP graph, a
 * FrameParams-sized device block, pinned staging memory and two events.
 * Each replay overwrites the same outputs; a launch on another stream first
 * waits (on the device) for the previous replay of the handle to finish, and
 * on the host only until the previous launch's parameter copy has run.  rara_frame_graph_destroy waits for the last replay
 * to finish before it frees anything.  Errors: RARA_ERR_INVALID for bad or
 * mismatched arguments (n must be > 0), RARA_ERR_UNSUPPORTED for an SH degree
 * above 3 or more than 65535 tile columns or rows, RARA_ERR_HIP if an
 * allocation, the capture, the instantiation, the copy or the launch fails. */
typedef struct rara_frame_graph rara_frame_graph;
rara_status rara_frame_graph_create(const rara_gaussians* g, const rara_camera* shape, const rara_projected* proj,
                                    const rara_binned* bins, int64_t pair_capacity, void* workspace, size_t ws_bytes,
                                    float* image, float* final_T, uint32_t* n_contrib, uint32_t* n_walked,
                                    rara_frame_graph** out);
rara_status rara_frame_graph_launch(rara_frame_graph* fg, const rara_camera* cam, const rara_plane* plane,
                                    const float* bg, void* stream);
void rara_frame_graph_destroy(rara_frame_graph* fg);

/* Static description of a status code (never NULL). */
const char* rara_status_string(rara_status s);

/* Library version string, e.g. "rara 0.1 gfx950". */
const char* rara_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RARA_H */
