// Internal declarations of the gfx950 RaRa renderer: record layouts, launch
// parameter blocks and the launch helpers each .hip file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rara.h"

namespace rara {

constexpr int kTile = 16;               // 16x16-pixel screen tiles
// a tile rectangle of at most kMaskTiles tiles lists only the tiles the
// Gaussian reaches (word 1 of ProjPtrs::tile_rec); a larger one lists every tile
constexpr int kMaskTiles = 64;
constexpr float kAlphaMax = 0.99f;      // Algorithm 1 step 3 clamp
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;
constexpr double kDilation = 0.3;       // px^2 added to the projected covariance
constexpr double kGuard = 1.3;          // Jacobian guard band (fraction of the half-FOV)
constexpr float kKappa2 = 9.0f;         // traced ellipsoid |M^-1 (x - mu)|^2 = 3^2
constexpr float kLog2e = 1.4426950408889634f;

// Projected splat, 48 bytes (see rara_projected in rara.h).
struct alignas(16) Splat {
    double mx, my;
    float ca, cb, cc, op;
    float r, g, b;
    uint32_t label;
};
static_assert(sizeof(Splat) == 48, "splat record must be 48 bytes");

// Whitened-space ray set-up of a CUTOFF Gaussian, 48 bytes.  With the pixel
// offset (dx, dy) = pixel - mean2d, the pixel ray r(t) = e + t v has camera
// depth t, and in unit-sphere space (M^-1 = S^-1 R^T, eq. 4)
//   M^-1 (r(t) - mu) = z delta + s D,  t = z + s,
//   delta = gx dx + gy dy,  D = d0 + delta,
// with d0 = M^-1 (mu - e) / z and gx, gy = M^-1 R_c^T e_{x,y} / f_{x,y}.
// The plane value along the ray is  d_ep + z (ax dx + ay dy) + s g,
// g = g0 + ax dx + ay dy, g0 = n.(mu - e)/z, (ax, ay) = (R_c n)_{x,y} / f_{x,y}.
struct alignas(16) RayRec {
    float d0[3];
    float gx[3];
    float gy[3];
    float z, dep, g0;
};
static_assert(sizeof(RayRec) == 48, "ray record must be 48 bytes");

struct CamParams {
    double R[9], t[3], e[3];
    double fx, fy, cx, cy, near_z, limx, limy;
    int W, H, tiles_x, tiles_y;
};

constexpr int kMaxPlanes = RARA_MAX_PLANES;

// Clip plane, or region: plane 0 is (n, d); with count > 1 the further
// planes are xn / xd (all normalised).
struct PlaneParams {
    double n[3];
    double d;
    int enabled;   // clip mode (RARA_CLIP_*), 0 when off
    int count;     // half-spaces in the region, 1 for a single plane
    double xn[kMaxPlanes - 1][3];
    double xd[kMaxPlanes - 1];
};

struct GaussPtrs {
    int64_t n;
    int sh_degree;
    int sh_layout;   // RARA_SH_COEFF_MAJOR or RARA_SH_GAUSSIAN_MAJOR
    const float* mean;
    const float* scale;
    const float* quat;
    const float* opacity;
    const float* sh;
};

// How a kernel addresses the SH coefficients, fixed per launch on the host:
// the coefficient-major layout; Gaussian-major rows read a float at a time;
// Gaussian-major rows of a multiple of four floats in 16-byte aligned arrays,
// read and written with 16-byte accesses.  A compile-time choice, so that the
// compiler never merges the layouts' loads into one set of selected addresses.
enum { kShCoeffMajor = 0, kShRow = 1, kShRow16 = 2 };

inline int sh_mode(int sh_layout, int sh_degree, const void* a, const void* b = nullptr)
{
    if (sh_layout != RARA_SH_GAUSSIAN_MAJOR) return kShCoeffMajor;
    const int row = 3 * (sh_degree + 1) * (sh_degree + 1);
    const bool aligned = (reinterpret_cast<uintptr_t>(a) & 15u) == 0u && (reinterpret_cast<uintptr_t>(b) & 15u) == 0u;
    return row % 4 == 0 && aligned ? kShRow16 : kShRow;
}

// The 3 (D+1)^2 SH coefficients of Gaussian i as v[3k + c] (coefficient k,
// channel c).
template <int kCoef, int kMode>
__device__ inline void load_sh(const GaussPtrs& g, int64_t i, float (&v)[3 * kCoef])
{
    constexpr int kN = 3 * kCoef;
    if constexpr (kMode == kShRow16) {
        static_assert(kN % 4 == 0, "16-byte rows");
        const float4* s4 = reinterpret_cast<const float4*>(g.sh + i * kN);
#pragma unroll
        for (int j = 0; j < kN / 4; ++j) {
            const float4 q = s4[j];
            v[4 * j] = q.x;
            v[4 * j + 1] = q.y;
            v[4 * j + 2] = q.z;
            v[4 * j + 3] = q.w;
        }
    } else if constexpr (kMode == kShRow) {
        const float* src = g.sh + i * kN;
#pragma unroll
        for (int j = 0; j < kN; ++j) v[j] = src[j];
    } else {
#pragma unroll
        for (int j = 0; j < kN; ++j) v[j] = g.sh[(int64_t)j * g.n + i];
    }
}

// Orders the LDS accesses of a wave's lanes before and after it (no other wave
// takes part).
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Position (row by row in the rectangle) of the n-th listed tile of a
// rectangle with `area` tiles and listed-tile mask m.
__device__ inline uint32_t listed_tile(uint64_t m, int area, uint32_t n)
{
    if (area > kMaskTiles) return n;
    uint32_t k = 0;
#pragma unroll
    for (int half = 32; half > 0; half >>= 1) {
        const uint32_t c = (uint32_t)__popcll(m & ((1ull << half) - 1ull));
        if (n >= c) {
            n -= c;
            m >>= half;
            k += (uint32_t)half;
        }
    }
    return k;
}

// Number of listed tiles before rectangle position k (the inverse of listed_tile).
__device__ inline uint32_t listed_rank(uint64_t m, int area, uint32_t k)
{
    return area > kMaskTiles ? k : (uint32_t)__popcll(m & ((1ull << k) - 1ull));
}

// Listed tiles of a rectangle of `area` tiles with mask m.
__device__ inline uint32_t listed_count(uint64_t m, int area)
{
    return area > kMaskTiles ? (uint32_t)area : (uint32_t)__popcll(m);
}

struct ProjPtrs {
    uint8_t* label;
    Splat* splat;
    RayRec* ray;
    float2* ray_ext;   // [n][kMaxPlanes - 1] (dep, g0) of planes 1.. for a region, else unused
    float* depth;
    uint32_t* tiles_touched;
    ulonglong2* tile_rec;   // [n] (rectangle, listed-tile mask of a rectangle of at most kMaskTiles tiles)
};

struct RenderParams {
    int W, H, tiles_x, tiles_y, num_tiles;
    int plane_enabled;   // clip mode (RARA_CLIP_*)
    float ax, ay;
    float bg[3];
    int plane_count;                          // 1, or the half-spaces of a region
    float xax[kMaxPlanes - 1], xay[kMaxPlanes - 1];   // (ax, ay) of planes 1 .. count-1
};

// Everything a frame reads that depends on the camera pose, the clip plane or
// the background.  Frame graphs keep one of these in device memory and
// rewrite it with a stream-ordered copy before each replay; their kernels read
// it through a pointer, so the graph's kernel arguments never change.
struct FrameParams {
    CamParams cam;
    PlaneParams plane;
    RenderParams render;
};

// ---- blend work list --------------------------------------------------------
// Tiles whose list holds at least kHeavyList entries are blended first
// (work[] has tiles + 1 entries, see plan_kernel).
constexpr uint32_t kHeavyList = 1024;
// forward blend: one workgroup per tile, both tile groups padded to 8
// (the non-split tiles are dealt to the XCDs in chunks of kDealChunk: the
// fullest XCD holds up to 2 kDealChunk more than an even share)
constexpr uint32_t kDealChunk = 16;
inline int64_t tiles_grid(int64_t tiles) { return tiles + 16 + 16 * (int64_t)kDealChunk; }
// forward blend: the first kMaxUnitTiles long-list tiles run as four quadrant
// units each (the grid's padding, workgroups that find no work and exit, stays
// a few thousand at most); the schedule puts the up to kMaxUnitTiles longest
// lists first, found from a histogram of the long lists' lengths in buckets of
// kUnitBucket entries
constexpr uint32_t kMaxUnitTiles = 512;
constexpr uint32_t kUnitBucket = 128;
inline int64_t blend_grid(int64_t tiles)
{
    const int64_t u = tiles < (int64_t)kMaxUnitTiles ? tiles : (int64_t)kMaxUnitTiles;
    return 4 * (u + 8) + tiles_grid(tiles);
}

// ---- bin/sort workspace carve-up -------------------------------------------
constexpr int kScanBlock = 256;      // Gaussians per scan chunk
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;        // keys per thread per sort tile of the pair passes
constexpr int kSortTile = kSortThreads * kSortItems;
// the depth passes sort the drawn Gaussians (about half a million at 1080p):
// 1024-key tiles give several workgroups per CU instead of one
constexpr int kDepthSortItems = 4;
constexpr int kDepthSortTile = kSortThreads * kDepthSortItems;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

struct BinWorkspace {
    uint32_t* block_sums;    // [scan_blocks]: tile counts per kScanBlock Gaussians of the depth order
    int64_t* dcount;         // drawn-Gaussian count
    uint32_t* dkeys[2];      // depth keys, ping-pong [n]
    uint32_t* dvals[2];      // Gaussian indices, ping-pong [n]
    ulonglong2* drec;        // [n] tile records in depth order, from dkeys[1] on (dkeys[1] and dvals[1]
                             // are free once the depth sort has ended in buffer 0)
    uint32_t* tkeys;         // tile keys [cap]
    uint32_t* tvals;         // Gaussian indices [cap]
    uint32_t* hist;          // [kRadix][max(depth_blocks, tile_blocks)]
    uint32_t* digit_totals;  // [kRadix]
    int64_t scan_blocks, depth_blocks, tile_blocks;
};

size_t bin_workspace_layout(int64_t n, int64_t cap, BinWorkspace* ws, char* base);
size_t backward_workspace_bytes(int64_t n, int64_t pair_capacity, int32_t width, int32_t height);

// ---- launch helpers (each returns the hipGetLastError of its launches) ----
hipError_t launch_preprocess(const GaussPtrs& g, const CamParams& cam, const PlaneParams& pl, const ProjPtrs& out,
                             hipStream_t s);
hipError_t launch_bin(const ProjPtrs& proj, int64_t n, const CamParams& cam, int64_t cap, const BinWorkspace& ws,
                      const rara_binned& out, int tile_passes, hipStream_t s);
// First pass of the depth sort: its items are the n Gaussians in index order,
// taken when drawn (tiles_touched > 0) with the bits of their depth as keys;
// it writes the number of drawn Gaussians to count_out and sets the tile
// ranges [range_words] to (0xffffffff, 0) (no pair yet).
struct SortFirstPass {
    const float* depth;
    const uint32_t* tt;
    int64_t n;
    int64_t* count_out;
    uint32_t* ranges;
    int64_t range_words;
};
// Extra output of the last pass: for every key below num_tiles, the first
// output position (atomic min into ranges[2 key]) and one past the last
// (atomic max into ranges[2 key + 1]).
struct SortLastPass {
    uint32_t* ranges;
    uint32_t num_tiles;
};
// items: keys per thread per sort tile, kDepthSortItems or kSortItems
hipError_t sort_passes(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, int passes, int items,
                       const int64_t* count, const int32_t* overflow, int64_t blocks, uint32_t* hist,
                       uint32_t* digit_totals, uint64_t* final_keys, uint32_t* final_vals, const float* depth,
                       const SortFirstPass* first, const SortLastPass* last, hipStream_t s);
hipError_t launch_ranges_clear(const rara_binned& out, int num_tiles, hipStream_t s);
hipError_t launch_plan(const rara_binned& out, int num_tiles, hipStream_t s);
// the same kernels reading their per-frame parameters from device memory
hipError_t launch_preprocess_fp(const GaussPtrs& g, const FrameParams* fp, const ProjPtrs& out, hipStream_t s);
hipError_t launch_blend_fp(const Splat* splat, const RayRec* ray, const rara_binned& bins, const FrameParams* fp,
                           int num_tiles, float* image, float* final_T, uint32_t* n_contrib, uint32_t* n_walked,
                           hipStream_t s);
// host-side parameter blocks shared by the ABI entry points and frame graphs
inline bool sh_layout_ok(int32_t v) { return v == RARA_SH_COEFF_MAJOR || v == RARA_SH_GAUSSIAN_MAJOR; }
bool make_cam_params(const rara_camera* c, CamParams* p);
bool make_plane_params(const rara_plane* pl, PlaneParams* p);
RenderParams make_render_params(const CamParams& cp, const PlaneParams& pp, const float* bg);
hipError_t launch_backward(const GaussPtrs& g, const CamParams& cam, const PlaneParams& pl, double plane_len,
                           const ProjPtrs& proj, const rara_binned& bins, int64_t pair_capacity, const RenderParams& rp,
                           const float* final_T, const uint32_t* n_contrib, const float* dL_dimage,
                           const rara_grads& grads, void* workspace, hipStream_t s);
// one frame of a batched blend launch (rara_render_batch), passed by value
struct BatchItem {
    const Splat* splat;
    const RayRec* ray;
    const uint32_t* vals;
    const uint2* ranges;
    const uint32_t* work;
    const int32_t* overflow;
    float* image;
    float* final_T;
    uint32_t* n_contrib;
    RenderParams p;
    uint32_t first_block;   // set by launch_blend_batch
};
struct BatchArgs {
    int count;
    BatchItem items[RARA_MAX_BATCH];
};
static_assert(sizeof(BatchArgs) <= 4096, "batched blend arguments must fit the kernel argument limit");
hipError_t launch_blend_batch(BatchArgs& a, hipStream_t s);
hipError_t launch_blend(const Splat* splat, const RayRec* ray, const float2* ray_ext, const rara_binned& bins,
                        const RenderParams& p, float* image, float* final_T, uint32_t* n_contrib, uint32_t* n_walked,
                        uint32_t* n_eval, hipStream_t s);

}  // namespace rara
