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

// strict: a miss (h^2 < 0) gets w = [plane value at the closest approach >= 0]
// (kind 5) instead of w = 1.
__device__ inline void chord_eval(const CutRec& k, float dx, float dy, float ax, float ay, bool strict, Chord& c)
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
    if (!(c.h2 > 0.0f)) {   // fewer than two intersections
        c.kind = 0;
        c.w = 1.0f;
        if (strict && c.h2 < 0.0f) {
            c.u = fmaf(ax, dx, ay * dy);
            c.gg = g0 + c.u;
            c.phim = fmaf(c.sm, c.gg, fmaf(z, c.u, dep));
            c.kind = 5;
            c.w = c.phim >= 0.0f ? 1.0f : 0.0f;
        }
        return;
    }
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

__device__ inline float chord_weight(const CutRec& k, float dx, float dy, float ax, float ay, bool strict)
{
    Chord c;
    chord_eval(k, dx, dy, ax, ay, strict, c);
    return c.w;
}

// chord_eval's weight without branches, for the forward: every case's value
// is formed with chord_eval's own operations on the same inputs, and the case
// is then selected, so the result is chord_eval's w bit for bit.  A wave whose
// pixels fall in different cases (rays crossing the silhouette, the near-root
// boundary) takes one straight path instead of each case in turn.
__device__ inline float chord_weight_flat(const CutRec& k, float dx, float dy, float ax, float ay, bool strict)
{
    const float gx[3] = {k.a.w, k.b.x, k.b.y};
    const float gy[3] = {k.b.z, k.b.w, k.c.x};
    const float d0[3] = {k.a.x, k.a.y, k.a.z};
    const float z = k.c.y, dep = k.c.z, g0 = k.c.w;
    float D[3], P[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float e = fmaf(gx[i], dx, gy[i] * dy);
        D[i] = d0[i] + e;
        P[i] = z * e;
    }
    const float DD = fmaf(D[0], D[0], fmaf(D[1], D[1], D[2] * D[2]));
    const float PD = fmaf(P[0], D[0], fmaf(P[1], D[1], P[2] * D[2]));
    const float iDD = __builtin_amdgcn_rcpf(DD);
    const float sm = -PD * iDD;
    float Q[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) Q[i] = fmaf(sm, D[i], P[i]);
    const float h2 = kKappa2 - fmaf(Q[0], Q[0], fmaf(Q[1], Q[1], Q[2] * Q[2]));
    const float u = fmaf(ax, dx, ay * dy);
    const float gg = g0 + u;
    const float phim = fmaf(sm, gg, fmaf(z, u, dep));
    const float step = phim >= 0.0f ? 1.0f : 0.0f;                  // cases 2 and 5
    const float hs = __builtin_amdgcn_sqrtf(h2 * iDD);              // NaN for a miss: not selected
    const float inv = __builtin_amdgcn_rcpf((2.0f * fabsf(gg)) * hs);
    float w = __builtin_amdgcn_fmed3f(fmaf(phim, inv, 0.5f), 0.0f, 1.0f);   // cases 3, 4
    w = gg == 0.0f ? step : w;                                      // case 2
    w = (z + sm) - hs < 0.0f ? 1.0f : w;                            // case 1
    const float miss = (strict && h2 < 0.0f) ? step : 1.0f;         // cases 5 and 0
    return h2 > 0.0f ? w : miss;
}

// Clip weight for a region, the intersection of `count` half-spaces: plane 0
// from the ray record, planes 1.. from ext[k - 1] = (d_ep, g0) and the
// per-frame rates[k - 1] = (ax, ay).  The chord geometry is chord_eval's.  Along the
// chord, s in [-h, h] from its midpoint (camera depth), plane k has the value
// phi_k + g_k s; the chord is visible where every one is >= 0, an interval
// [lo, hi]: planes with g_k > 0 raise lo to -phi_k / g_k, planes with g_k < 0
// lower hi to it, a plane with g_k = 0 keeps all or nothing.  The weight is
// (hi - lo) / 2h clamped to [0, 1] (for one plane this is eq. (11)'s
// 1/2 + phi / (2 |g| h)).  A miss keeps w = 1, or with the strict policy
// w = [the closest approach is inside every half-space]; a near root behind
// the camera keeps w = 1.  `mask` may leave out planes that hold the whole
// 3-sigma ellipsoid on their visible side: they bound no chord (not for the
// strict policy, whose closest approach of a miss lies outside the ellipsoid).
__device__ inline float chord_weight_region(const CutRec& k, const float2* __restrict__ ext, int count, float dx,
                                            float dy, float ax, float ay, const float2* __restrict__ rates,
                                            bool strict, uint32_t mask = 0xffu)
{
    const float gx[3] = {k.a.w, k.b.x, k.b.y};
    const float gy[3] = {k.b.z, k.b.w, k.c.x};
    const float d0[3] = {k.a.x, k.a.y, k.a.z};
    const float z = k.c.y;
    float D[3], P[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float e = fmaf(gx[i], dx, gy[i] * dy);
        D[i] = d0[i] + e;
        P[i] = z * e;
    }
    const float DD = fmaf(D[0], D[0], fmaf(D[1], D[1], D[2] * D[2]));
    const float PD = fmaf(P[0], D[0], fmaf(P[1], D[1], P[2] * D[2]));
    const float iDD = __builtin_amdgcn_rcpf(DD);
    const float sm = -PD * iDD;
    float Q[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) Q[i] = fmaf(sm, D[i], P[i]);
    const float h2 = kKappa2 - fmaf(Q[0], Q[0], fmaf(Q[1], Q[1], Q[2] * Q[2]));
    const float hs = __builtin_amdgcn_sqrtf(h2 * iDD);   // NaN for a miss: not selected
    float lo = -hs, hi = hs;
    bool empty = false, all_in = true;
    for (int p = 0; p < count; ++p) {
        if (!((mask >> p) & 1u)) continue;   // a plane the caller knows keeps the whole chord visible
        const float2 pe = p == 0 ? make_float2(k.c.z, k.c.w) : ext[p - 1];
        const float pax = p == 0 ? ax : rates[p - 1].x, pay = p == 0 ? ay : rates[p - 1].y;
        const float u = fmaf(pax, dx, pay * dy);
        const float gg = pe.y + u;
        const float phim = fmaf(sm, gg, fmaf(z, u, pe.x));
        all_in = all_in && phim >= 0.0f;
        const float c = -phim * __builtin_amdgcn_rcpf(gg);
        lo = gg > 0.0f ? fmaxf(lo, c) : lo;
        hi = gg < 0.0f ? fminf(hi, c) : hi;
        empty = empty || (gg == 0.0f && phim < 0.0f);
    }
    float w = empty ? 0.0f : __builtin_amdgcn_fmed3f((hi - lo) * __builtin_amdgcn_rcpf(2.0f * hs), 0.0f, 1.0f);
    w = (z + sm) - hs < 0.0f ? 1.0f : w;
    const float miss = (strict && h2 < 0.0f) ? (all_in ? 1.0f : 0.0f) : 1.0f;
    return h2 > 0.0f ? w : miss;
}

// Whether the alpha >= 1/255 region of an entry can reach the pixel centres
// [qx, qx + 7] x [qy, qy + 7] (tile coordinates).  alpha >= 1/255 needs the
// conic form q(d) = ca dx^2 + 2 cb dx dy + cc dy^2 at d = pixel - centre to be
// at most m2 = 2 ln(255 delta) (the clip weight only lowers alpha).  The form
// is convex, so its minimum over the box is 0 when the centre lies inside and
// otherwise the smallest of the four edge minima; along the edge dx = X it is
// cc (dy - dy*)^2 + X^2 det/cc with dy* = -cb X / cc clamped to the edge, a sum
// of two non-negative terms (no cancellation).  The caller pads m2 so that
// float rounding can only keep a quadrant, never drop one.
struct QuadForm {
    float mx, my;    // centre, tile coordinates
    float ca, cc;    // conic diagonal
    float kx, ky;    // -cb / cc, -cb / ca
    float dx_, dy_;  // det / cc, det / ca
};

// Box of pixel centres [bx, bx + w] x [by, by + h] (tile coordinates); an 8x8
// quadrant is w = h = 7.
__device__ inline bool box_reach(const QuadForm& f, float m2, float bx, float by, float w, float h)
{
    const float x0 = bx - f.mx, x1 = (bx + w) - f.mx;
    const float y0 = by - f.my, y1 = (by + h) - f.my;
    const bool inside = (x0 <= 0.0f) && (x1 >= 0.0f) && (y0 <= 0.0f) && (y1 >= 0.0f);
    auto edge_x = [&](float X) {
        const float ys = f.kx * X;
        const float t = __builtin_amdgcn_fmed3f(ys, y0, y1) - ys;
        return fmaf(f.cc * t, t, f.dx_ * (X * X));
    };
    auto edge_y = [&](float Y) {
        const float xs = f.ky * Y;
        const float t = __builtin_amdgcn_fmed3f(xs, x0, x1) - xs;
        return fmaf(f.ca * t, t, f.dy_ * (Y * Y));
    };
    const float qmin = fminf(fminf(edge_x(x0), edge_x(x1)), fminf(edge_y(y0), edge_y(y1)));
    return inside || qmin <= m2;
}

__device__ inline bool quad_reach(const QuadForm& f, float m2, float qx, float qy)
{
    return box_reach(f, m2, qx, qy, 7.0f, 7.0f);
}

// The reach test's form of a splat (centre relative to the tile) and its
// padded threshold m2; false when the opacity alone is below 1/255.
__device__ inline bool reach_form(const Splat& nx, float mx, float my, QuadForm& f, float& m2)
{
    const float s255 = 255.0f * nx.op;
    if (!(s255 > 1.0f)) return false;
    // padded by 2 % + 0.02 against the rounding of the form, det and log
    m2 = fmaf(2.0f * __logf(s255), 1.02f, 0.02f);
    const float det = fmaf(nx.ca, nx.cc, -nx.cb * nx.cb);
    const float ica = 1.0f / nx.ca, icc = 1.0f / nx.cc;
    f.mx = mx;
    f.my = my;
    f.ca = nx.ca;
    f.cc = nx.cc;
    f.kx = -nx.cb * icc;
    f.ky = -nx.cb * ica;
    f.dx_ = fmaxf(det, 0.0f) * icc;
    f.dy_ = fmaxf(det, 0.0f) * ica;
    return true;
}

// Label word of a list entry as staged for the blend: the label in the low
// byte, the plane mask (bits 16..23 of the splat's word: the planes whose
// visible side does not hold the whole 3-sigma ellipsoid) kept.  With an empty
// mask every chord lies inside every half-space, and a miss or a near root
// behind the camera keeps 1 as well, so w = 1 on every pixel ray (eq. 11): such
// a CUTOFF Gaussian is staged as VISIBLE and its weight is not evaluated.  Not
// under the strict miss policy, where a miss depends on the closest approach.
__device__ inline uint32_t staged_word(uint32_t word, bool strict)
{
    const uint32_t lab = word & 0xffu;
    const uint32_t cuts = word & 0x00ff0000u;
    const bool all_in = lab == RARA_LABEL_CUTOFF && !strict && cuts == 0u;
    return (all_in ? (uint32_t)RARA_LABEL_VISIBLE : lab) | cuts;
}

// Staged form of one list entry.  s_a: centre (tile-relative), pre-scaled
// conic a and b; s_b: pre-scaled conic c, opacity, red, green; s_c: blue,
// label | quadrant mask << 8, Gaussian index.  The quadrant mask holds bit q
// (q = 2 * row + column of the 8x8 quadrant) for every quadrant in `want`
// that the entry can reach with alpha >= 1/255; an entry is never left out of
// a quadrant it could reach.
__device__ inline void stage_entry(const Splat& nx, double ox, double oy, uint32_t want, bool strict, float4& sa,
                                   float4& sb, float4& sc, uint32_t& qmask, uint32_t id)
{
    const float kq = -0.5f * kLog2e;
    const float mx = (float)(nx.mx - ox), my = (float)(nx.my - oy);
    sa = make_float4(mx, my, nx.ca * kq, -nx.cb * kLog2e);
    sb = make_float4(nx.cc * kq, nx.op, nx.r, nx.g);
    qmask = 0u;
    QuadForm f;
    float m2;
    if (reach_form(nx, mx, my, f, m2)) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if ((want >> q) & 1u)
                qmask |= quad_reach(f, m2, (float)((q & 1) * 8), (float)((q >> 1) * 8)) ? (1u << q) : 0u;
    }
    sc = make_float4(nx.b, __uint_as_float(staged_word(nx.label, strict) | (qmask << 8)), __uint_as_float(id),
                     0.0f);
}

// The same staging for a long-list quadrant unit: bit w of the mask is set
// when the entry can reach strip w of quadrant `quad` (the pixel centres of
// quadrant rows 2w and 2w + 1, tile columns qx .. qx + 7).
__device__ inline void stage_entry_strips(const Splat& nx, double ox, double oy, int quad, bool strict, float4& sa,
                                          float4& sb, float2& sc, uint32_t& smask)
{
    const float kq = -0.5f * kLog2e;
    const float mx = (float)(nx.mx - ox), my = (float)(nx.my - oy);
    sa = make_float4(mx, my, nx.ca * kq, -nx.cb * kLog2e);
    sb = make_float4(nx.cc * kq, nx.op, nx.r, nx.g);
    smask = 0u;
    QuadForm f;
    float m2;
    if (reach_form(nx, mx, my, f, m2)) {
        const float qx = (float)((quad & 1) * 8), qy = (float)((quad >> 1) * 8);
#pragma unroll
        for (int w = 0; w < 4; ++w)
            smask |= box_reach(f, m2, qx, qy + 2.0f * (float)w, 7.0f, 1.0f) ? (1u << w) : 0u;
    }
    sc = make_float2(nx.b, __uint_as_float(staged_word(nx.label, strict) | (smask << 8)));
}

// Tile of blend workgroup b.  The work list holds the H long-list tiles
// (kHeavyList entries or more) first, then the others, each group in tile
// order, and H in its last entry.  Workgroups go to
// the 8 XCDs round robin (b mod 8), each XCD with its own L2.  The long lists
// start first, every XCD taking one contiguous run of them.  The other tiles
// are dealt to the XCDs in chunks of kDealChunk consecutive tiles (a piece of
// a tile row, whose tiles share splats in one L2), chunk c to XCD c mod 8, so
// that the dense parts of the image spread over every XCD.  tiles_grid(T)
// workgroups cover both groups.
__device__ inline bool tile_of_block_in(uint32_t b, const uint32_t* __restrict__ work, uint32_t H, uint32_t num,
                                        uint32_t& tile)
{
    const uint32_t hb = (H + 7u) & ~7u;
    if (b < hb) {
        const uint32_t x = b & 7u, k = b >> 3;
        const uint32_t q8 = H >> 3, r8 = H & 7u;
        if (k >= q8 + (x < r8 ? 1u : 0u)) return false;
        tile = work[x * q8 + (x < r8 ? x : r8) + k];
        return true;
    }
    const uint32_t bb = b - hb;   // hb is a multiple of 8: bb and b share an XCD
    const uint32_t x = bb & 7u, k = bb >> 3;
    const uint32_t i = (x + 8u * (k / kDealChunk)) * kDealChunk + k % kDealChunk;
    if (i >= num - H) return false;
    tile = work[H + i];
    return true;
}

__device__ inline bool tile_of_block(uint32_t b, const uint32_t* __restrict__ work, int num_tiles, uint32_t& tile)
{
    return tile_of_block_in(b, work, work[num_tiles], (uint32_t)num_tiles, tile);
}

// Work unit of forward blend workgroup b: the first U = min(H, kMaxUnitTiles)
// long-list tiles (the longest, which lead the schedule) are blended as four
// quadrant units each, the other H - U long-list tiles as whole tiles, and
// those whole tiles are dispatched first: they are the longest jobs of the
// launch (a unit does a quarter of a longer list's pixels four entries at a
// time).  Then the units, units 4i .. 4i + 3 of the i-th tile of an XCD on
// that XCD (b mod 8), one after the other, so that the four units of a tile
// share one L2; then the short tiles as in tile_of_block.  quad is -1 for a
// whole tile.  blend_grid(T) workgroups cover every case.
__device__ inline bool unit_of_block(uint32_t b, const uint32_t* __restrict__ work, int num_tiles, uint32_t& tile,
                                     int& quad)
{
    const uint32_t H = work[num_tiles];
    const uint32_t U = H < kMaxUnitTiles ? H : kMaxUnitTiles;
    const uint32_t ub = (U + 7u) & ~7u;
    const uint32_t hb = (H - U + 7u) & ~7u;   // the whole long-list tiles, dealt as in tile_of_block_in
    quad = -1;
    if (b < hb) return tile_of_block_in(b, work + U, H - U, H - U, tile);
    b -= hb;   // hb is a multiple of 8: b keeps its XCD
    if (b < 4u * ub) {
        const uint32_t x = b & 7u, k = b >> 3;
        const uint32_t i = k >> 2;
        const uint32_t q8 = U >> 3, r8 = U & 7u;
        if (i >= q8 + (x < r8 ? 1u : 0u)) return false;
        tile = work[x * q8 + (x < r8 ? x : r8) + i];
        quad = (int)(k & 3u);
        return true;
    }
    return tile_of_block_in(b - 4u * ub, work + H, 0u, (uint32_t)num_tiles - H, tile);
}

}  // namespace rara
