// Per-tile front-to-back alpha blend with the RaRa decay weight.
//
//   alpha = min(0.99, delta exp(-1/2 dx^T conic dx) w)        (eq. 12, Alg. 1 step 3)
//   C = sum_k c_k alpha_k prod_{j<k} (1 - alpha_j)             (eq. 2)
// w = 1 for VISIBLE Gaussians; for CUTOFF ones w is the visible fraction of
// the pixel ray's chord through the 3-sigma ellipsoid (eqs. 4-8, 11).
//
// Layout: one 256-thread workgroup per 16x16 tile; wave w owns the 8x8
// quadrant w (one pixel per lane).  The tile's sorted list is walked in
// batches of 224: each of the first 224 threads gathers one 48-byte splat
// record (and, for CUTOFF Gaussians, the 48-byte ray record), converts the
// projected centre to tile-relative FP32 (exact to ~1e-6 px), folds
// -log2(e)/2 into the conic so that alpha needs one exp2, tests which
// quadrants the entry can reach, and stages it in LDS.  Each wave then
// visits, in list order, the staged entries that reach its quadrant, reading
// each as an LDS broadcast.  The CUTOFF branch is wave-uniform (labels are per
// Gaussian).
//
// The weight is evaluated in whitened space from the pixel offset, not from
// the world-space quadratic: with delta = gx dx + gy dy, D = d0 + delta,
// P = z delta, the ray is P + s D (s = camera depth minus z).  Its closest
// approach to the centre is at s_m = -P.D / D.D with squared whitened distance
// |P + s_m D|^2; the chord half-length in depth is h = sqrt((9 - that)/D.D).
// The plane value at the chord midpoint is d_ep + z (ax dx + ay dy) + s_m g,
// g = g0 + ax dx + ay dy its rate along the ray, and the visible fraction of
// the chord is clamp(1/2 + phi_m / (2 |g| h), 0, 1).  Every term stays of the
// order of the Gaussian's own size, so FP32 keeps its accuracy even for the
// 40:1 strand Gaussians (the expanded B^2 - 4AC cancels catastrophically).
#include "blend_common.h"

namespace rara {

namespace {

// One pixel's front-to-back update with one list entry of opacity
// alpha = min(0.99, a0 w), a0 = delta 2^pw (0 for pw > 0), straight-line and
// without lane masks.  The entry is taken when alpha reaches the pixel's
// threshold `thr` (1/255 while the pixel is live; a finished pixel has thr = 2,
// above any alpha, so it is left unchanged).  A taken entry that would bring T
// below 1e-4 finishes the pixel without being composited: T keeps its value,
// the final transmittance.  Otherwise a taken entry is composited (its weight
// alpha T > 0, so it is the pixel's last contributor so far); an entry not
// taken changes nothing.
__device__ inline float entry_a0(float pw, float op)
{
    return op * __builtin_amdgcn_exp2f(pw > 0.0f ? -INFINITY : pw);
}

__device__ inline void composite(float alpha, float cr, float cg, float cb, uint32_t k1, float& T, float& thr,
                                 float& C0, float& C1, float& C2, uint32_t& last, uint32_t& walked)
{
    const float tT = fmaf(-alpha, T, T);   // finite: alpha in [0, 0.99], T in [1e-4, 1]
    const bool take = alpha >= thr;
    const bool ok = take && tT >= kTMin;
    const bool fin = take && !ok;
    const float wt = ok ? alpha * T : 0.0f;
    C0 = fmaf(wt, cr, C0);
    C1 = fmaf(wt, cg, C1);
    C2 = fmaf(wt, cb, C2);
    T = ok ? tT : T;
    thr = fin ? 2.0f : thr;
    last = ok ? k1 : last;
    walked = fin ? k1 : walked;
}

constexpr int kBlendThreads = 256;   // one workgroup per tile: four waves, one per 8x8 quadrant
// entries staged per batch, one per thread of the first 224: with 64 VGPRs
// and under 20 KB of LDS a CU holds 8 workgroups (8 waves per SIMD)
constexpr int kTileBatch = 224;
constexpr int kBatchSlots = 256;     // s_c rows: four 64-entry ballots, the tail zero
// the clip-region variant stages the further planes' terms too (56 B per
// entry): 128-entry batches keep it under 20 KB of LDS
constexpr int kRegionBatch = 128;
template <bool kRegion> constexpr int batch_of() { return kRegion ? kRegionBatch : kTileBatch; }
template <bool kRegion> constexpr int slots_of() { return kRegion ? kRegionBatch : kBatchSlots; }

// One tile: thread t of wave w = t / 64 owns pixel (t % 8, (t / 8) % 8) of the
// 8x8 quadrant w.  Per batch, every thread stages one entry; after the
// barrier each wave takes, per 64 staged entries, one ballot of the entries
// that reach its quadrant and one of the CUTOFF entries, and visits the set
// bits in order.  A wave re-takes its live pixels every 16 entries and stops
// visiting once none is left; the workgroup stops when no wave has one.
// kRegion: the clip region of p.plane_count half-spaces (chord_weight_region),
// with each CUTOFF entry's further-plane terms staged in s_ext and the
// per-frame rates of those planes in s_rate.
template <bool kWalked, bool kRegion>
__device__ inline void blend_tile(const Splat* __restrict__ splats, const RayRec* __restrict__ rays,
                                  const float2* __restrict__ ray_ext, const uint32_t* __restrict__ vals,
                                  const uint2 rg, int tile, const RenderParams& p, float4* s_a, float4* s_b,
                                  float2* s_c, CutRec* s_cut, float2* s_ext, float2* s_rate,
                                  float* __restrict__ image, float* __restrict__ final_T,
                                  uint32_t* __restrict__ n_contrib, uint32_t* __restrict__ n_walked)
{
    const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ox8 = (wave & 1) * 8 + (lane & 7), oy8 = (wave >> 1) * 8 + (lane >> 3);
    const float lpx = (float)ox8, lpy = (float)oy8;
    const int px = tx * kTile + ox8, py = ty * kTile + oy8;
    const bool inside = px < p.W && py < p.H;

    float T = 1.0f, thr = inside ? kAlphaMin : 2.0f;   // pixels outside the image never take part
    float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    uint32_t last = 0u, walked = 0u;

    // Long lists set the tail of the launch: their waves get issue priority over
    // the short tiles sharing their SIMD (wave priority only; no effect on results).
    const uint32_t len = rg.y - rg.x;
    if (len >= 2048u)
        __builtin_amdgcn_s_setprio(3);
    else if (len >= 768u)
        __builtin_amdgcn_s_setprio(2);
    else if (len >= 256u)
        __builtin_amdgcn_s_setprio(1);

    const double ox = (double)(tx * kTile), oy = (double)(ty * kTile);
    const bool plane_on = p.plane_enabled != 0;
    const bool strict = (p.plane_enabled & RARA_CLIP_STRICT_MISS) != 0;
    bool live = __ballot(thr < 1.0f) != 0ull;

    constexpr int kB = batch_of<kRegion>();
    for (uint32_t base = rg.x; base < rg.y; base += kB) {
        if (!__syncthreads_or(live ? 1 : 0)) break;   // also: the previous batch has been read
        const uint32_t idx = base + (uint32_t)tid;
        float2 sc = make_float2(0.0f, 0.0f);   // label | quadrant mask << 8 = 0: reaches nothing
        if (tid < kB && idx < rg.y) {
            const uint32_t id = vals[idx];
            const Splat sp = splats[id];
            float4 sa, sb, c4;
            uint32_t qm;
            stage_entry(sp, ox, oy, 0xfu, sa, sb, c4, qm, id);
            s_a[tid] = sa;
            s_b[tid] = sb;
            sc = make_float2(c4.x, c4.y);
            if (sp.label == RARA_LABEL_CUTOFF && plane_on) {
                const float4* rr = reinterpret_cast<const float4*>(rays + id);
                const float4 r0 = rr[0], r1 = rr[1], r2 = rr[2];
                s_cut[tid].a = r0;
                s_cut[tid].b = r1;
                s_cut[tid].c = r2;
                if (kRegion)
                    for (int k = 0; k < p.plane_count - 1; ++k)
                        s_ext[tid * (kMaxPlanes - 1) + k] = ray_ext[(int64_t)id * (kMaxPlanes - 1) + k];
            }
        }
        if (tid < slots_of<kRegion>()) s_c[tid] = sc;
        __syncthreads();
        if (!live) continue;
        const uint32_t cnt = rg.y - base < (uint32_t)kB ? rg.y - base : (uint32_t)kB;
        const uint32_t kofs = base - rg.x + 1u;
        for (uint32_t sub = 0; sub < cnt && live; sub += 64) {
            const uint32_t lm = __float_as_uint(s_c[sub + lane].y);
            const uint64_t qb = __ballot((lm >> (8 + wave)) & 1u);
            const uint64_t cutb = __ballot(plane_on && (lm & 0xffu) == RARA_LABEL_CUTOFF);
            for (int chunk = 0; chunk < 64; chunk += 16) {
                uint64_t todo = qb & (0xffffull << chunk);
                if ((todo & cutb) == 0ull) {
                    // no CUTOFF entry in this chunk: w = 1 throughout
                    while (todo) {
                        const int j = (int)__builtin_ctzll(todo);
                        todo &= todo - 1ull;
                        const uint32_t e = sub + (uint32_t)j;
                        const float4 a = s_a[e], b = s_b[e];
                        const float cb_ = s_c[e].x;
                        const float dx = lpx - a.x, dy = lpy - a.y;
                        const float a0 = entry_a0(entry_power(a, b, dx, dy), b.y);
                        composite(fminf(kAlphaMax, a0), b.z, b.w, cb_, kofs + e, T, thr, C0, C1, C2, last, walked);
                    }
                } else {
                    while (todo) {
                        const int j = (int)__builtin_ctzll(todo);
                        todo &= todo - 1ull;
                        const uint32_t e = sub + (uint32_t)j;
                        const float4 a = s_a[e], b = s_b[e];
                        const float cb_ = s_c[e].x;
                        const float dx = lpx - a.x, dy = lpy - a.y;
                        const float a0 = entry_a0(entry_power(a, b, dx, dy), b.y);
                        float alpha = fminf(kAlphaMax, a0);   // w = 1
                        if ((cutb >> j) & 1ull) {
                            // alpha <= a0 (w <= 1): when no pixel can reach its threshold the
                            // entry changes nothing and its weight is not needed
                            if (__ballot(a0 >= thr) == 0ull) continue;
                            const float w = kRegion ? chord_weight_region(s_cut[e], s_ext + e * (kMaxPlanes - 1),
                                                                          p.plane_count, dx, dy, p.ax, p.ay, s_rate,
                                                                          strict)
                                                    : chord_weight_flat(s_cut[e], dx, dy, p.ax, p.ay, strict);
                            alpha = fminf(kAlphaMax, a0 * w);
                        }
                        composite(alpha, b.z, b.w, cb_, kofs + e, T, thr, C0, C1, C2, last, walked);
                    }
                }
                live = __ballot(thr < 1.0f) != 0ull;
                if (!live) break;
            }
        }
    }

    if (!inside) return;
    const int64_t HW = (int64_t)p.H * p.W;
    const int64_t pix = (int64_t)py * p.W + px;
    image[pix] = C0 + T * p.bg[0];
    image[HW + pix] = C1 + T * p.bg[1];
    image[2 * HW + pix] = C2 + T * p.bg[2];
    final_T[pix] = T;
    n_contrib[pix] = last;
    // a pixel still live at the end examined the whole list
    if (kWalked) n_walked[pix] = thr < 1.0f ? rg.y - rg.x : walked;
}

template <bool kWalked, bool kRegion>
__device__ __forceinline__ void blend_block(const Splat* __restrict__ splats, const RayRec* __restrict__ rays,
                                            const float2* __restrict__ ray_ext, const uint32_t* __restrict__ vals,
                                            const uint2* __restrict__ ranges, const uint32_t* __restrict__ work,
                                            const RenderParams& p, float* __restrict__ image,
                                            float* __restrict__ final_T, uint32_t* __restrict__ n_contrib,
                                            uint32_t* __restrict__ n_walked)
{
    uint32_t tile;
    if (!tile_of_block(blockIdx.x, work, p.num_tiles, tile)) return;
    if (tile >= (uint32_t)p.num_tiles) return;
    constexpr int kB = batch_of<kRegion>();
    __shared__ float4 s_a[kB], s_b[kB];
    __shared__ float2 s_c[slots_of<kRegion>()];
    __shared__ CutRec s_cut[kB];
    __shared__ float2 s_ext[kRegion ? kB * (kMaxPlanes - 1) : 1];
    __shared__ float2 s_rate[kMaxPlanes - 1];
    if (kRegion) {
        // the further planes' per-frame rates; the first batch's barrier orders them before any visit
        if (threadIdx.x < kMaxPlanes - 1) s_rate[threadIdx.x] = make_float2(p.xax[threadIdx.x], p.xay[threadIdx.x]);
    }
    blend_tile<kWalked, kRegion>(splats, rays, ray_ext, vals, ranges[tile], (int)tile, p, s_a, s_b, s_c, s_cut, s_ext,
                                 s_rate, image, final_T, n_contrib, n_walked);
}

template <bool kWalked>
__global__ __launch_bounds__(kBlendThreads) __attribute__((amdgpu_waves_per_eu(8)))
void blend_kernel(const Splat* __restrict__ splats, const RayRec* __restrict__ rays, const uint32_t* __restrict__ vals,
                  const uint2* __restrict__ ranges, const uint32_t* __restrict__ work,
                  const int32_t* __restrict__ overflow, RenderParams p, float* __restrict__ image,
                  float* __restrict__ final_T, uint32_t* __restrict__ n_contrib, uint32_t* __restrict__ n_walked)
{
    if (*overflow) return;
    blend_block<kWalked, false>(splats, rays, nullptr, vals, ranges, work, p, image, final_T, n_contrib, n_walked);
}

// Clip-region variant (p.plane_count > 1): the further planes' terms staged
// too, in 128-entry batches, still 8 workgroups per CU.
template <bool kWalked>
__global__ __launch_bounds__(kBlendThreads) __attribute__((amdgpu_waves_per_eu(8)))
void blend_region_kernel(const Splat* __restrict__ splats, const RayRec* __restrict__ rays,
                         const float2* __restrict__ ray_ext, const uint32_t* __restrict__ vals,
                         const uint2* __restrict__ ranges, const uint32_t* __restrict__ work,
                         const int32_t* __restrict__ overflow, RenderParams p, float* __restrict__ image,
                         float* __restrict__ final_T, uint32_t* __restrict__ n_contrib,
                         uint32_t* __restrict__ n_walked)
{
    if (*overflow) return;
    blend_block<kWalked, true>(splats, rays, ray_ext, vals, ranges, work, p, image, final_T, n_contrib, n_walked);
}

// Frame-graph variant: render parameters read from device memory.
template <bool kWalked>
__global__ __launch_bounds__(kBlendThreads) __attribute__((amdgpu_waves_per_eu(8)))
void blend_fp_kernel(const Splat* __restrict__ splats, const RayRec* __restrict__ rays,
                     const uint32_t* __restrict__ vals, const uint2* __restrict__ ranges,
                     const uint32_t* __restrict__ work, const int32_t* __restrict__ overflow,
                     const FrameParams* __restrict__ fp, float* __restrict__ image, float* __restrict__ final_T,
                     uint32_t* __restrict__ n_contrib, uint32_t* __restrict__ n_walked)
{
    if (*overflow) return;
    const RenderParams p = fp->render;
    blend_block<kWalked, false>(splats, rays, nullptr, vals, ranges, work, p, image, final_T, n_contrib, n_walked);
}

}  // namespace

hipError_t launch_blend(const Splat* splat, const RayRec* ray, const float2* ray_ext, const rara_binned& bins,
                        const RenderParams& p, float* image, float* final_T, uint32_t* n_contrib, uint32_t* n_walked,
                        hipStream_t s)
{
    const unsigned grid = (unsigned)tiles_grid(p.num_tiles);
    const uint2* ranges = reinterpret_cast<const uint2*>(bins.ranges);
    if (p.plane_enabled && p.plane_count > 1) {
        if (n_walked)
            hipLaunchKernelGGL(blend_region_kernel<true>, dim3(grid), dim3(kBlendThreads), 0, s, splat, ray, ray_ext,
                               bins.vals, ranges, bins.work, bins.overflow, p, image, final_T, n_contrib, n_walked);
        else
            hipLaunchKernelGGL(blend_region_kernel<false>, dim3(grid), dim3(kBlendThreads), 0, s, splat, ray, ray_ext,
                               bins.vals, ranges, bins.work, bins.overflow, p, image, final_T, n_contrib, n_walked);
    } else if (n_walked) {
        hipLaunchKernelGGL(blend_kernel<true>, dim3(grid), dim3(kBlendThreads), 0, s, splat, ray, bins.vals, ranges,
                           bins.work, bins.overflow, p, image, final_T, n_contrib, n_walked);
    } else {
        hipLaunchKernelGGL(blend_kernel<false>, dim3(grid), dim3(kBlendThreads), 0, s, splat, ray, bins.vals, ranges,
                           bins.work, bins.overflow, p, image, final_T, n_contrib, n_walked);
    }
    return hipGetLastError();
}

hipError_t launch_blend_fp(const Splat* splat, const RayRec* ray, const rara_binned& bins, const FrameParams* fp,
                           int num_tiles, float* image, float* final_T, uint32_t* n_contrib, uint32_t* n_walked,
                           hipStream_t s)
{
    const unsigned grid = (unsigned)tiles_grid(num_tiles);
    const uint2* ranges = reinterpret_cast<const uint2*>(bins.ranges);
    if (n_walked)
        hipLaunchKernelGGL(blend_fp_kernel<true>, dim3(grid), dim3(kBlendThreads), 0, s, splat, ray, bins.vals, ranges,
                           bins.work, bins.overflow, fp, image, final_T, n_contrib, n_walked);
    else
        hipLaunchKernelGGL(blend_fp_kernel<false>, dim3(grid), dim3(kBlendThreads), 0, s, splat, ray, bins.vals, ranges,
                           bins.work, bins.overflow, fp, image, final_T, n_contrib, n_walked);
    return hipGetLastError();
}

}  // namespace rara
