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
#include "rara_internal.h"

namespace rara {

namespace {

constexpr int kBatch = 64;

// Workgroups are dispatched round-robin over the 8 XCDs; hand each XCD a
// contiguous run of tiles so that neighbouring tiles (which share splats) hit
// the same L2.
__device__ inline int xcd_tile(int bid, int nblocks)
{
    const int xcd = bid & 7, local = bid >> 3;
    const int q = nblocks >> 3, r = nblocks & 7;
    return xcd * q + (xcd < r ? xcd : r) + local;
}

struct CutRec {
    float4 a;   // d0.xyz, gx.x
    float4 b;   // gx.yz, gy.xy
    float4 c;   // gy.z, z, dep, g0
};

__device__ inline float chord_weight(const CutRec& k, float dx, float dy, float ax, float ay)
{
    const float gx0 = k.a.w, gx1 = k.b.x, gx2 = k.b.y;
    const float gy0 = k.b.z, gy1 = k.b.w, gy2 = k.c.x;
    const float z = k.c.y, dep = k.c.z, g0 = k.c.w;
    const float e0 = gx0 * dx + gy0 * dy, e1 = gx1 * dx + gy1 * dy, e2 = gx2 * dx + gy2 * dy;
    const float D0 = k.a.x + e0, D1 = k.a.y + e1, D2 = k.a.z + e2;
    const float P0 = z * e0, P1 = z * e1, P2 = z * e2;
    const float DD = D0 * D0 + D1 * D1 + D2 * D2;
    const float PD = P0 * D0 + P1 * D1 + P2 * D2;
    const float iDD = __builtin_amdgcn_rcpf(DD);
    const float sm = -PD * iDD;
    const float Q0 = P0 + sm * D0, Q1 = P1 + sm * D1, Q2 = P2 + sm * D2;
    const float h2 = kKappa2 - (Q0 * Q0 + Q1 * Q1 + Q2 * Q2);
    if (!(h2 > 0.0f)) return 1.0f;                       // miss / tangent: fewer than two intersections
    const float hs = __builtin_amdgcn_sqrtf(h2 * iDD);   // chord half-length in camera depth
    if (z + sm - hs < 0.0f) return 1.0f;                 // near intersection behind the camera
    const float u = ax * dx + ay * dy;
    const float gg = g0 + u;
    const float phim = dep + z * u + sm * gg;
    if (gg == 0.0f) return phim >= 0.0f ? 1.0f : 0.0f;
    const float w = 0.5f + phim * __builtin_amdgcn_rcpf(2.0f * fabsf(gg) * hs);
    return __builtin_amdgcn_fmed3f(w, 0.0f, 1.0f);
}

__global__ __launch_bounds__(64) void blend_kernel(const Splat* __restrict__ splats, const RayRec* __restrict__ rays,
                                                   const uint32_t* __restrict__ vals, const uint2* __restrict__ ranges,
                                                   const int32_t* __restrict__ overflow, RenderParams p,
                                                   float* __restrict__ image, float* __restrict__ final_T,
                                                   uint32_t* __restrict__ n_contrib, uint32_t* __restrict__ n_walked)
{
    if (*overflow) return;
    const int tile = xcd_tile(blockIdx.x, p.num_tiles);
    const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
    const int lane = threadIdx.x;
    const int lx = lane & 7, ly = lane >> 3;

    __shared__ float4 s_a[kBatch], s_b[kBatch], s_c[kBatch];
    __shared__ CutRec s_cut[kBatch];

    float lpx[4], lpy[4];
    bool alive[4];
    float T[4], C0[4], C1[4], C2[4];
    uint32_t last[4], walked[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int ox = (q & 1) * 8 + lx, oy = (q >> 1) * 8 + ly;
        lpx[q] = (float)ox;
        lpy[q] = (float)oy;
        alive[q] = (tx * kTile + ox < p.W) && (ty * kTile + oy < p.H);
        T[q] = 1.0f;
        C0[q] = C1[q] = C2[q] = 0.0f;
        last[q] = walked[q] = 0u;
    }

    const uint2 rg = ranges[tile];
    const double ox = (double)(tx * kTile), oy = (double)(ty * kTile);
    const float kq = -0.5f * kLog2e;
    bool any_alive = __ballot(alive[0] || alive[1] || alive[2] || alive[3]) != 0ull;

    for (uint32_t base = rg.x; base < rg.y && any_alive; base += kBatch) {
        const uint32_t idx = base + lane;
        if (idx < rg.y) {
            const uint32_t id = vals[idx];
            const Splat s = splats[id];
            s_a[lane] = make_float4((float)(s.mx - ox), (float)(s.my - oy), s.ca * kq, -s.cb * kLog2e);
            s_b[lane] = make_float4(s.cc * kq, s.op, s.r, s.g);
            s_c[lane] = make_float4(s.b, __uint_as_float(s.label), 0.0f, 0.0f);
            if (s.label == RARA_LABEL_CUTOFF && p.plane_enabled) {
                const float4* rr = reinterpret_cast<const float4*>(rays + id);
                CutRec c;
                c.a = rr[0];
                c.b = rr[1];
                c.c = rr[2];
                s_cut[lane] = c;
            }
        }
        __syncthreads();
        const int cnt = (int)(rg.y - base < (uint32_t)kBatch ? rg.y - base : (uint32_t)kBatch);
        for (int j = 0; j < cnt; ++j) {
            const float4 a = s_a[j], b = s_b[j];
            const float4 c = s_c[j];
            const uint32_t k1 = base - rg.x + (uint32_t)j + 1u;
            const bool cut = (__float_as_uint(c.y) == RARA_LABEL_CUTOFF) && p.plane_enabled;
            if (cut) {
                const CutRec cr = s_cut[j];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (!alive[q]) continue;
                    walked[q] = k1;
                    const float dx = lpx[q] - a.x, dy = lpy[q] - a.y;
                    const float pw = a.z * dx * dx + b.x * dy * dy + a.w * dx * dy;
                    if (pw > 0.0f) continue;
                    float alpha = b.y * __builtin_amdgcn_exp2f(pw);
                    if (alpha < kAlphaMin) continue;   // w <= 1 cannot lift it above the threshold
                    alpha = fminf(kAlphaMax, alpha * chord_weight(cr, dx, dy, p.ax, p.ay));
                    if (alpha < kAlphaMin) continue;
                    const float tT = T[q] * (1.0f - alpha);
                    if (tT < kTMin) { alive[q] = false; continue; }
                    const float wt = alpha * T[q];
                    C0[q] += wt * b.z; C1[q] += wt * b.w; C2[q] += wt * c.x;
                    T[q] = tT;
                    last[q] = k1;
                }
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (!alive[q]) continue;
                    walked[q] = k1;
                    const float dx = lpx[q] - a.x, dy = lpy[q] - a.y;
                    const float pw = a.z * dx * dx + b.x * dy * dy + a.w * dx * dy;
                    if (pw > 0.0f) continue;
                    const float alpha = fminf(kAlphaMax, b.y * __builtin_amdgcn_exp2f(pw));
                    if (alpha < kAlphaMin) continue;
                    const float tT = T[q] * (1.0f - alpha);
                    if (tT < kTMin) { alive[q] = false; continue; }
                    const float wt = alpha * T[q];
                    C0[q] += wt * b.z; C1[q] += wt * b.w; C2[q] += wt * c.x;
                    T[q] = tT;
                    last[q] = k1;
                }
            }
            if (__ballot(alive[0] || alive[1] || alive[2] || alive[3]) == 0ull) { any_alive = false; break; }
        }
        __syncthreads();
    }

    const int64_t HW = (int64_t)p.H * p.W;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int px = tx * kTile + (q & 1) * 8 + lx, py = ty * kTile + (q >> 1) * 8 + ly;
        if (px >= p.W || py >= p.H) continue;
        const int64_t pix = (int64_t)py * p.W + px;
        image[pix] = C0[q] + T[q] * p.bg[0];
        image[HW + pix] = C1[q] + T[q] * p.bg[1];
        image[2 * HW + pix] = C2[q] + T[q] * p.bg[2];
        final_T[pix] = T[q];
        n_contrib[pix] = last[q];
        if (n_walked) n_walked[pix] = walked[q];
    }
}

}  // namespace

hipError_t launch_blend(const Splat* splat, const RayRec* ray, const rara_binned& bins, const RenderParams& p,
                        float* image, float* final_T, uint32_t* n_contrib, uint32_t* n_walked, hipStream_t s)
{
    hipLaunchKernelGGL(blend_kernel, dim3((unsigned)p.num_tiles), dim3(64), 0, s, splat, ray, bins.vals,
                       reinterpret_cast<const uint2*>(bins.ranges), bins.overflow, p, image, final_T, n_contrib,
                       n_walked);
    return hipGetLastError();
}

}  // namespace rara
