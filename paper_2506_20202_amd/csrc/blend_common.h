// Per-entry arithmetic shared by the forward blend and its backward, written
// with explicit fused multiply-adds so that both evaluate alpha and the clip
// weight with bit-identical results (the backward re-takes the forward's
// skip / composite decisions).
#pragma once

#include "rara_internal.h"

namespace rara {

constexpr int kBatch = 64;

// Whitened ray set-up of a CUTOFF Gaussian as staged in LDS.
struct CutRec {
    float4 a;   // d0.xyz, gx.x
    float4 b;   // gx.yz, gy.xy
    float4 c;   // gy.z, z, dep, g0
};

// Exponent of the 2D Gaussian, pre-scaled to base 2: a.z = -log2(e)/2 conic_a,
// a.w = -log2(e) conic_b, b.x = -log2(e)/2 conic_c.
__device__ inline float entry_power(const float4& a, const float4& b, float dx, float dy)
{
    return fmaf(dx, fmaf(a.z, dx, a.w * dy), b.x * dy * dy);
}

// Intermediates of the clip weight of eq. (11) for one pixel ray, in whitened
// space (see the derivation at the top of blend.hip).
struct Chord {
    float e[3], D[3], P[3], Q[3];
    float DD, PD, iDD, sm, h2, hs, u, gg, phim, inv;
    int kind;   // 0 miss, 1 near root behind the camera, 2 g = 0, 3 clamped, 4 interior
    float w;
};

__device__ inline void chord_eval(const CutRec& k, float dx, float dy, float ax, float ay, Chord& c)
{
    const float gx[3] = {k.a.w, k.b.x, k.b.y};
    const float gy[3] = {k.b.z, k.b.w, k.c.x};
    const float d0[3] = {k.a.x, k.a.y, k.a.z};
    const float z = k.c.y, dep = k.c.z, g0 = k.c.w;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        c.e[i] = fmaf(gx[i], dx, gy[i] * dy);
        c.D[i] = d0[i] + c.e[i];
        c.P[i] = z * c.e[i];
    }
    c.DD = fmaf(c.D[0], c.D[0], fmaf(c.D[1], c.D[1], c.D[2] * c.D[2]));
    c.PD = fmaf(c.P[0], c.D[0], fmaf(c.P[1], c.D[1], c.P[2] * c.D[2]));
    c.iDD = __builtin_amdgcn_rcpf(c.DD);
    c.sm = -c.PD * c.iDD;
#pragma unroll
    for (int i = 0; i < 3; ++i) c.Q[i] = fmaf(c.sm, c.D[i], c.P[i]);
    c.h2 = kKappa2 - fmaf(c.Q[0], c.Q[0], fmaf(c.Q[1], c.Q[1], c.Q[2] * c.Q[2]));
    c.hs = 0.0f;
    c.u = c.gg = c.phim = c.inv = 0.0f;
    if (!(c.h2 > 0.0f)) { c.kind = 0; c.w = 1.0f; return; }   // fewer than two intersections
    c.hs = __builtin_amdgcn_sqrtf(c.h2 * c.iDD);               // chord half-length in camera depth
    if ((z + c.sm) - c.hs < 0.0f) { c.kind = 1; c.w = 1.0f; return; }
    c.u = fmaf(ax, dx, ay * dy);
    c.gg = g0 + c.u;
    c.phim = fmaf(c.sm, c.gg, fmaf(z, c.u, dep));
    if (c.gg == 0.0f) { c.kind = 2; c.w = c.phim >= 0.0f ? 1.0f : 0.0f; return; }
    c.inv = __builtin_amdgcn_rcpf((2.0f * fabsf(c.gg)) * c.hs);
    const float wr = fmaf(c.phim, c.inv, 0.5f);
    c.kind = (wr > 0.0f && wr < 1.0f) ? 4 : 3;
    c.w = __builtin_amdgcn_fmed3f(wr, 0.0f, 1.0f);
}

__device__ inline float chord_weight(const CutRec& k, float dx, float dy, float ax, float ay)
{
    Chord c;
    chord_eval(k, dx, dy, ax, ay, c);
    return c.w;
}

// Staged form of one list entry.  s_a: centre (tile-relative), pre-scaled
// conic a and b; s_b: pre-scaled conic c, opacity, red, green; s_c: blue,
// label | quadrant mask << 8, Gaussian index.
__device__ inline void stage_entry(const Splat& nx, double ox, double oy, float4& sa, float4& sb, float4& sc,
                                   uint32_t& qmask, uint32_t id)
{
    const float kq = -0.5f * kLog2e;
    const float mx = (float)(nx.mx - ox), my = (float)(nx.my - oy);
    sa = make_float4(mx, my, nx.ca * kq, -nx.cb * kLog2e);
    sb = make_float4(nx.cc * kq, nx.op, nx.r, nx.g);
    // Quadrants of the tile the entry can reach with alpha >= 1/255:
    // delta exp(-m/2) >= 1/255 needs Mahalanobis^2 m <= 2 ln(255 delta),
    // whose ellipse has axis half-widths sqrt(m Vhat_00), sqrt(m Vhat_11).
    // Padded (1 % + 0.1 px) so float rounding can only widen the box; an entry
    // is never skipped for a pixel it could reach.
    qmask = 0u;
    const float s255 = 255.0f * nx.op;
    if (s255 > 1.0f) {
        const float m2 = 2.0f * __logf(s255) * 1.001f + 1e-3f;
        const float idet = 1.0f / (nx.ca * nx.cc - nx.cb * nx.cb);
        const float hx = sqrtf(m2 * nx.cc * idet) * 1.01f + 0.1f;
        const float hy = sqrtf(m2 * nx.ca * idet) * 1.01f + 0.1f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float qx = (float)((q & 1) * 8), qy = (float)((q >> 1) * 8);
            const bool hit = (mx - hx <= qx + 7.0f) && (mx + hx >= qx) && (my - hy <= qy + 7.0f) && (my + hy >= qy);
            qmask |= hit ? (1u << q) : 0u;
        }
    }
    sc = make_float4(nx.b, __uint_as_float(nx.label | (qmask << 8)), __uint_as_float(id), 0.0f);
}

// Work unit of workgroup b.  Workgroups are dispatched round-robin to the 8
// XCDs (b mod 8), each with its own L2: the four quadrant units of a split
// tile are given to one XCD (blocks b, b+8, b+16, b+24), and the whole-tile
// units are dealt out so that every XCD takes one contiguous run of tiles (a
// band of the image), keeping the tiles that share splats on one L2.
// work[4T] holds the number H of split tiles; split tile h has its quadrant
// units at work[4h..4h+3], whole tiles follow from work[4H] in tile order.
__device__ inline bool unit_of_block(uint32_t b, const uint32_t* __restrict__ work, int num_tiles, uint32_t& unit)
{
    const uint32_t H = work[4 * num_tiles];
    const uint32_t hb = 4u * ((H + 7u) & ~7u);
    if (b < hb) {
        const uint32_t x = b & 7u, r = b >> 3, h = (r >> 2) * 8u + x, q = r & 3u;
        if (h >= H) return false;
        unit = work[4 * h + q];
        return true;
    }
    const uint32_t bb = b - hb;   // hb is a multiple of 32: bb and b share an XCD
    const uint32_t nl = (uint32_t)num_tiles - H;
    const uint32_t x = bb & 7u, k = bb >> 3;
    const uint32_t q8 = nl >> 3, r8 = nl & 7u;
    const uint32_t cnt = q8 + (x < r8 ? 1u : 0u);
    if (k >= cnt) return false;
    const uint32_t start = x * q8 + (x < r8 ? x : r8);
    unit = work[4 * H + start + k];
    return true;
}

}  // namespace rara
