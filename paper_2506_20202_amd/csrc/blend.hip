// Per-tile front-to-back alpha blend with the RaRa decay weight.
//
//   alpha = min(0.99, delta exp(-1/2 dx^T conic dx) w)        (eq. 12, Alg. 1 step 3)
//   C = sum_k c_k alpha_k prod_{j<k} (1 - alpha_j)             (eq. 2)
// w = 1 for VISIBLE Gaussians; for CUTOFF ones w is the visible fraction of
// the pixel ray's chord through the 3-sigma ellipsoid (eqs. 4-8, 11).
//
// Layout: one 64-lane wave per 16x16 tile, each lane owning the same pixel of
// the four 8x8 quadrants.  The tile's sorted list is walked in batches of 64:
// each lane gathers one 48-byte splat record (and, for CUTOFF Gaussians, the
// 48-byte ray record) into LDS, converting the projected centre to
// tile-relative FP32 (exact to ~1e-6 px) and folding -log2(e)/2 into the conic
// so that alpha needs one exp2.  Every lane then reads each staged record as
// an LDS broadcast and evaluates its four pixels.  The CUTOFF branch is
// wave-uniform (labels are per Gaussian).
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

// One pixel's front-to-back update with one list entry, straight-line and
// without lane masks.  alpha = min(0.99, a0 w), a0 = delta 2^pw; entries with
// pw > 0 or alpha below the pixel's threshold `thr` are skipped (thr = 1/255
// while the pixel is live; a finished pixel has thr = 2, above any alpha, so
// it is left unchanged).  An entry that would take T below 1e-4 finishes the
// pixel without being composited: T keeps its value, the final transmittance.
// A live pixel always has T >= 1e-4, so a skipped entry (alpha = 0, new
// T = T) can never finish it.
__device__ inline void composite(float pw, float op, float w, float cr, float cg, float cb, uint32_t k1, float& T,
                                 float& thr, float& C0, float& C1, float& C2, uint32_t& last, uint32_t& walked)
{
    const float e = __builtin_amdgcn_exp2f(pw > 0.0f ? -INFINITY : pw);
    float alpha = fminf(kAlphaMax, (op * e) * w);
    alpha = alpha >= thr ? alpha : 0.0f;
    const float tT = fmaf(-alpha, T, T);
    const bool term = tT < kTMin;
    const float wt = term ? 0.0f : alpha * T;
    C0 = fmaf(wt, cr, C0);
    C1 = fmaf(wt, cg, C1);
    C2 = fmaf(wt, cb, C2);
    T = term ? T : tT;
    thr = term ? 2.0f : thr;
    last = wt > 0.0f ? k1 : last;
    walked = term ? k1 : walked;
}

// Pixels of one work unit: a whole 16x16 tile (kSlots = 4, each lane owns the
// same pixel of the four 8x8 quadrants) or a single quadrant of a tile with a
// long list (kSlots = 1), so that such tiles are walked by four waves at once.
//
// The list is walked in batches of 64 entries.  Each lane gathers one entry,
// stages it in LDS and tests which of the unit's quadrants the entry can
// reach; per batch, one ballot per quadrant (and one for CUTOFF entries)
// turns those tests into wave-uniform bit sets, so the entry loop itself does
// no per-entry mask reads or lane-mask branches.  Every 16 entries the
// quadrants that still hold a live pixel are re-taken and the walk ends when
// none is left.
template <int kSlots, bool kWalked>
__device__ inline void blend_unit(const Splat* __restrict__ splats, const RayRec* __restrict__ rays,
                                  const uint32_t* __restrict__ vals, const uint2 rg, int tile, int quad,
                                  const RenderParams& p, float4* s_a, float4* s_b, float4* s_c, CutRec* s_cut,
                                  float* __restrict__ image, float* __restrict__ final_T,
                                  uint32_t* __restrict__ n_contrib, uint32_t* __restrict__ n_walked)
{
    const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
    const int lane = threadIdx.x;
    const int lx = lane & 7, ly = lane >> 3;

    float lpx[kSlots], lpy[kSlots];
    float T[kSlots], thr[kSlots], C0[kSlots], C1[kSlots], C2[kSlots];
    uint32_t last[kSlots], walked[kSlots];
    int qof[kSlots];
    uint32_t want = 0u;
#pragma unroll
    for (int q = 0; q < kSlots; ++q) {
        const int qq = kSlots == 4 ? q : quad;
        qof[q] = qq;
        want |= 1u << qq;
        lpx[q] = (float)((qq & 1) * 8 + lx);
        lpy[q] = (float)((qq >> 1) * 8 + ly);
        const bool inside = (tx * kTile + (qq & 1) * 8 + lx < p.W) && (ty * kTile + (qq >> 1) * 8 + ly < p.H);
        T[q] = 1.0f;
        thr[q] = inside ? kAlphaMin : 2.0f;   // pixels outside the image never take part
        C0[q] = C1[q] = C2[q] = 0.0f;
        last[q] = walked[q] = 0u;
    }

    const double ox = (double)(tx * kTile), oy = (double)(ty * kTile);
    const bool plane_on = p.plane_enabled != 0;

    Splat nx;
    float4 nr0, nr1, nr2;
    bool have = false;
    uint32_t cur_id = 0u;
    auto fetch = [&](uint32_t base) {
        const uint32_t idx = base + lane;
        have = idx < rg.y;
        if (have) {
            const uint32_t id = vals[idx];
            cur_id = id;
            nx = splats[id];
            if (nx.label == RARA_LABEL_CUTOFF && plane_on) {
                const float4* rr = reinterpret_cast<const float4*>(rays + id);
                nr0 = rr[0];
                nr1 = rr[1];
                nr2 = rr[2];
            }
        }
    };
    // quadrants (bit qof[q]) that still hold a live pixel, wave-uniform
    auto live_quads = [&]() -> uint32_t {
        uint32_t m = 0u;
#pragma unroll
        for (int q = 0; q < kSlots; ++q) m |= __ballot(thr[q] < 1.0f) != 0ull ? (1u << qof[q]) : 0u;
        return m;
    };

    uint32_t live = live_quads();
    if (rg.x < rg.y && live) fetch(rg.x);
    for (uint32_t base = rg.x; base < rg.y && live; base += kBatch) {
        uint32_t my_mask = 0u;
        bool my_cut = false;
        __syncthreads();   // the previous batch has been read
        if (have) {
            stage_entry(nx, ox, oy, want, s_a[lane], s_b[lane], s_c[lane], my_mask, cur_id);
            my_cut = nx.label == RARA_LABEL_CUTOFF && plane_on;
            if (my_cut) {
                CutRec c;
                c.a = nr0;
                c.b = nr1;
                c.c = nr2;
                s_cut[lane] = c;
            }
        }
        __syncthreads();
        if (base + kBatch < rg.y) fetch(base + kBatch);   // overlaps with the compositing below
        uint64_t qb[kSlots];
#pragma unroll
        for (int q = 0; q < kSlots; ++q) qb[q] = __ballot((my_mask >> qof[q]) & 1u);
        const uint64_t cutb = __ballot(my_cut);
        const uint32_t kofs = base - rg.x + 1u;
        for (int chunk = 0; chunk < kBatch; chunk += 16) {
            // entries of this chunk that reach a quadrant with live pixels, in list order
            uint64_t ql[kSlots];
            uint64_t todo = 0ull;
#pragma unroll
            for (int q = 0; q < kSlots; ++q) {
                ql[q] = ((live >> qof[q]) & 1u) ? qb[q] : 0ull;
                todo |= ql[q];
            }
            todo &= 0xffffull << chunk;
            while (todo) {
                const int j = (int)__builtin_ctzll(todo);
                todo &= todo - 1ull;
                const float4 a = s_a[j], b = s_b[j];
                const float cb_ = s_c[j].x;
                const bool cut = (cutb >> j) & 1ull;
                const uint32_t k1 = kofs + (uint32_t)j;
                const float dxa = lpx[0] - a.x, dya = lpy[0] - a.y;
                const float dxb = lpx[kSlots - 1] - a.x, dyb = lpy[kSlots - 1] - a.y;
#pragma unroll
                for (int q = 0; q < kSlots; ++q) {
                    if (kSlots == 1 || ((ql[q] >> j) & 1ull)) {
                        const bool xb = kSlots == 4 ? (q & 1) : false;
                        const bool yb = kSlots == 4 ? (q >> 1) : false;
                        const float dx = xb ? dxb : dxa;
                        const float dy = yb ? dyb : dya;
                        const float pw = entry_power(a, b, dx, dy);
                        float w = 1.0f;
                        if (cut) w = chord_weight(s_cut[j], dx, dy, p.ax, p.ay);
                        composite(pw, b.y, w, b.z, b.w, cb_, k1, T[q], thr[q], C0[q], C1[q], C2[q], last[q],
                                  walked[q]);
                    }
                }
            }
            live = live_quads();
            if (!live) break;
        }
    }

    const int64_t HW = (int64_t)p.H * p.W;
#pragma unroll
    for (int q = 0; q < kSlots; ++q) {
        const int px = tx * kTile + (int)lpx[q], py = ty * kTile + (int)lpy[q];
        if (px >= p.W || py >= p.H) continue;
        const int64_t pix = (int64_t)py * p.W + px;
        image[pix] = C0[q] + T[q] * p.bg[0];
        image[HW + pix] = C1[q] + T[q] * p.bg[1];
        image[2 * HW + pix] = C2[q] + T[q] * p.bg[2];
        final_T[pix] = T[q];
        n_contrib[pix] = last[q];
        // a pixel still live at the end examined the whole list
        if (kWalked) n_walked[pix] = thr[q] < 1.0f ? rg.y - rg.x : walked[q];
    }
}

// One wave per work unit (see unit_of_block for the schedule).
template <bool kWalked>
__device__ __forceinline__ void blend_block(const Splat* __restrict__ splats, const RayRec* __restrict__ rays,
                                            const uint32_t* __restrict__ vals, const uint2* __restrict__ ranges,
                                            const uint32_t* __restrict__ work, const RenderParams& p,
                                            float* __restrict__ image, float* __restrict__ final_T,
                                            uint32_t* __restrict__ n_contrib, uint32_t* __restrict__ n_walked)
{
    uint32_t unit;
    if (!unit_of_block(blockIdx.x, work, p.num_tiles, unit)) return;
    const int tile = (int)(unit >> 3), mode = (int)(unit & 7u);
    if (tile >= p.num_tiles || mode > 4) return;
    __shared__ float4 s_a[kBatch], s_b[kBatch], s_c[kBatch];
    __shared__ CutRec s_cut[kBatch];
    const uint2 rg = ranges[tile];
    if (mode == 4)
        blend_unit<4, kWalked>(splats, rays, vals, rg, tile, 0, p, s_a, s_b, s_c, s_cut, image, final_T, n_contrib,
                               n_walked);
    else
        blend_unit<1, kWalked>(splats, rays, vals, rg, tile, mode, p, s_a, s_b, s_c, s_cut, image, final_T, n_contrib,
                               n_walked);
}

template <bool kWalked>
__global__ __launch_bounds__(64) void blend_kernel(const Splat* __restrict__ splats, const RayRec* __restrict__ rays,
                                                   const uint32_t* __restrict__ vals, const uint2* __restrict__ ranges,
                                                   const uint32_t* __restrict__ work,
                                                   const int32_t* __restrict__ overflow, RenderParams p,
                                                   float* __restrict__ image, float* __restrict__ final_T,
                                                   uint32_t* __restrict__ n_contrib, uint32_t* __restrict__ n_walked)
{
    if (*overflow) return;
    blend_block<kWalked>(splats, rays, vals, ranges, work, p, image, final_T, n_contrib, n_walked);
}

// Frame-graph variant: render parameters read from device memory.
template <bool kWalked>
__global__ __launch_bounds__(64) void blend_fp_kernel(const Splat* __restrict__ splats,
                                                      const RayRec* __restrict__ rays,
                                                      const uint32_t* __restrict__ vals,
                                                      const uint2* __restrict__ ranges,
                                                      const uint32_t* __restrict__ work,
                                                      const int32_t* __restrict__ overflow,
                                                      const FrameParams* __restrict__ fp, float* __restrict__ image,
                                                      float* __restrict__ final_T, uint32_t* __restrict__ n_contrib,
                                                      uint32_t* __restrict__ n_walked)
{
    if (*overflow) return;
    const RenderParams p = fp->render;
    blend_block<kWalked>(splats, rays, vals, ranges, work, p, image, final_T, n_contrib, n_walked);
}

}  // namespace

hipError_t launch_blend(const Splat* splat, const RayRec* ray, const rara_binned& bins, const RenderParams& p,
                        float* image, float* final_T, uint32_t* n_contrib, uint32_t* n_walked, hipStream_t s)
{
    const unsigned grid = (unsigned)work_grid(p.num_tiles);
    if (n_walked)
        hipLaunchKernelGGL(blend_kernel<true>, dim3(grid), dim3(64), 0, s, splat, ray, bins.vals,
                           reinterpret_cast<const uint2*>(bins.ranges), bins.work, bins.overflow, p, image, final_T,
                           n_contrib, n_walked);
    else
        hipLaunchKernelGGL(blend_kernel<false>, dim3(grid), dim3(64), 0, s, splat, ray, bins.vals,
                           reinterpret_cast<const uint2*>(bins.ranges), bins.work, bins.overflow, p, image, final_T,
                           n_contrib, n_walked);
    return hipGetLastError();
}

hipError_t launch_blend_fp(const Splat* splat, const RayRec* ray, const rara_binned& bins, const FrameParams* fp,
                           int num_tiles, float* image, float* final_T, uint32_t* n_contrib, uint32_t* n_walked,
                           hipStream_t s)
{
    const unsigned grid = (unsigned)work_grid(num_tiles);
    const uint2* ranges = reinterpret_cast<const uint2*>(bins.ranges);
    if (n_walked)
        hipLaunchKernelGGL(blend_fp_kernel<true>, dim3(grid), dim3(64), 0, s, splat, ray, bins.vals, ranges, bins.work,
                           bins.overflow, fp, image, final_T, n_contrib, n_walked);
    else
        hipLaunchKernelGGL(blend_fp_kernel<false>, dim3(grid), dim3(64), 0, s, splat, ray, bins.vals, ranges,
                           bins.work, bins.overflow, fp, image, final_T, n_contrib, n_walked);
    return hipGetLastError();
}

}  // namespace rara
