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
constexpr int kBatchSlots = 256;     // s_c rows: four 64-entry ballots, the tail zero (quadrant units)
// the clip-region variant stages the further planes' terms too (56 B per
// entry): 128-entry batches keep it under 20 KB of LDS
constexpr int kRegionBatch = 128;
template <bool kRegion> constexpr int batch_of() { return kRegion ? kRegionBatch : kTileBatch; }
template <bool kRegion> constexpr int slots_of() { return kRegion ? kRegionBatch : kBatchSlots; }
// entries per window of a whole-tile wave: four windows fill the batch arrays
template <bool kRegion> constexpr uint32_t tile_window() { return (uint32_t)batch_of<kRegion>() / 4u; }
static_assert(tile_window<false>() <= 64 && tile_window<true>() <= 64, "a window is one ballot");

// One tile: thread t of wave w = t / 64 owns pixel (t % 8, (t / 8) % 8) of the
// 8x8 quadrant w.  Each wave walks the list on its own, in windows of
// tile_window entries that its lanes stage into the wave's part of the batch
// arrays (testing their reach of its quadrant only), so no wave waits for
// another: per window, one ballot of the entries that reach the quadrant and
// one of the CUTOFF entries, and the set bits visited in order.  A wave
// re-takes its live pixels every 16 entries and stops once none is left.
// kRegion: the clip region of p.plane_count half-spaces (chord_weight_region),
// with each CUTOFF entry's further-plane terms staged in s_ext and the
// per-frame rates of those planes in s_rate.
template <bool kWalked, bool kRegion>
__device__ inline void blend_tile(const Splat* __restrict__ splats, const RayRec* __restrict__ rays,
                                  const float2* __restrict__ ray_ext, const uint32_t* __restrict__ vals,
                                  const uint2 rg, int tile, const RenderParams& p, float4* s_a, float4* s_b,
                                  float2* s_c, CutRec* s_cut, float2* s_ext, float2* s_rate,
                                  float* __restrict__ image, float* __restrict__ final_T,
                                  uint32_t* __restrict__ n_contrib, uint32_t* __restrict__ n_walked,
                                  uint32_t* __restrict__ n_eval)
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
    uint32_t ev = 0u, evc = 0u;   // evaluations while live, and clip weights among them (kWalked only)

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

    constexpr uint32_t kW = tile_window<kRegion>();
    // the region's per-frame plane rates, written by the first lanes of wave 0
    if (kRegion) __syncthreads();
    const uint32_t sub = (uint32_t)wave * kW;   // the wave's part of the batch arrays
    for (uint32_t base = rg.x; base < rg.y && live; base += kW) {
        const uint32_t idx = base + (uint32_t)lane;
        const uint32_t slot = sub + (uint32_t)lane;
        float2 sc = make_float2(0.0f, 0.0f);   // label | quadrant mask << 8 = 0: reaches nothing
        if ((uint32_t)lane < kW && idx < rg.y) {
            const uint32_t id = vals[idx];
            const Splat sp = splats[id];
            float4 sa, sb, c4;
            uint32_t qm;
            stage_entry(sp, ox, oy, 1u << wave, strict, sa, sb, c4, qm, id);
            s_a[slot] = sa;
            s_b[slot] = sb;
            sc = make_float2(c4.x, c4.y);
            if ((__float_as_uint(c4.y) & 0xffu) == RARA_LABEL_CUTOFF && plane_on) {
                const float4* rr = reinterpret_cast<const float4*>(rays + id);
                const float4 r0 = rr[0], r1 = rr[1], r2 = rr[2];
                s_cut[slot].a = r0;
                s_cut[slot].b = r1;
                s_cut[slot].c = r2;
                if (kRegion)
                    for (int k = 0; k < p.plane_count - 1; ++k)
                        s_ext[slot * (kMaxPlanes - 1) + k] = ray_ext[(int64_t)id * (kMaxPlanes - 1) + k];
            }
        }
        if ((uint32_t)lane < kW) s_c[slot] = sc;
        wave_sync();
        // entry e of the arrays (e = sub + j) is list position kofs + e, 1-based (modulo 2^32)
        const uint32_t kofs = base - rg.x + 1u - sub;
        {
            const uint32_t lm = (uint32_t)lane < kW ? __float_as_uint(s_c[sub + lane].y) : 0u;
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
                        if (kWalked) ev += thr < 1.0f ? 1u : 0u;
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
                        if (kWalked) ev += thr < 1.0f ? 1u : 0u;
                        if ((cutb >> j) & 1ull) {
                            // alpha <= a0 (w <= 1): when no pixel can reach its threshold the
                            // entry changes nothing and its weight is not needed
                            if (__ballot(a0 >= thr) == 0ull) continue;
                            float w;
                            if (kRegion) {
                                // the planes that do not hold the whole ellipsoid on their visible
                                // side (set by the preprocess); the others leave every chord whole
                                const uint32_t cuts = (__float_as_uint(s_c[e].y) >> 16) & 0xffu;
                                if (!strict && __popc(cuts) == 1) {
                                    // one plane: eq. (11) with that plane's terms
                                    const int kp = __ffs(cuts) - 1;
                                    CutRec rec = s_cut[e];
                                    float pax = p.ax, pay = p.ay;
                                    if (kp > 0) {
                                        const float2 x = s_ext[e * (kMaxPlanes - 1) + kp - 1];
                                        rec.c.z = x.x;
                                        rec.c.w = x.y;
                                        pax = s_rate[kp - 1].x;
                                        pay = s_rate[kp - 1].y;
                                    }
                                    w = chord_weight_flat(rec, dx, dy, pax, pay, false);
                                } else {
                                    w = chord_weight_region(s_cut[e], s_ext + e * (kMaxPlanes - 1), p.plane_count, dx,
                                                            dy, p.ax, p.ay, s_rate, strict, strict ? 0xffu : cuts);
                                }
                            } else {
                                w = chord_weight_flat(s_cut[e], dx, dy, p.ax, p.ay, strict);
                            }
                            alpha = fminf(kAlphaMax, a0 * w);
                            if (kWalked) evc += thr < 1.0f ? 1u : 0u;
                        }
                        composite(alpha, b.z, b.w, cb_, kofs + e, T, thr, C0, C1, C2, last, walked);
                    }
                }
                live = __ballot(thr < 1.0f) != 0ull;
                if (!live) break;
            }
        }
        wave_sync();   // the window has been read before the next one is staged
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
    if (kWalked && n_walked) n_walked[pix] = thr < 1.0f ? rg.y - rg.x : walked;
    if (kWalked && n_eval) {
        n_eval[pix] = ev;
        n_eval[HW + pix] = evc;
    }
}

// ---- long lists: quadrant units ---------------------------------------------
//
// A tile whose list holds kHeavyList entries or more runs as four
// workgroups, one per 8x8 quadrant, so that its work spreads over four CUs.
// Wave w of a unit owns strip w of the quadrant (rows 2w, 2w + 1: 16 pixels)
// with four lanes per pixel: lane 4 p + j evaluates, for pixel p, the j-th of
// the next four entries of the list that reach the strip.  The four alphas of
// a pixel are then composited in list order with a prefix product over its
// lanes: with f_j = 1 - alpha_j for a taken entry (alpha_j at or above the
// pixel's threshold) and 1 otherwise, entry j sees T_j = T prod_{i<j} f_i;
// it is composited (weight alpha_j T_j) when T_j f_j stays at or above 1e-4,
// and the first taken entry that would go below finishes the pixel with
// T = T_j (T_j f_j only decreases along the four entries, so no later entry
// is composited).  Each lane keeps its own colour sums, last contributor
// and finishing index; the four are combined when the unit ends.

// quad_perm selectors (lane i of each group of four reads lane sel[i])
constexpr int kQpPrev = 0x90;      // [0, 0, 1, 2]
constexpr int kQpPrev2 = 0x40;     // [0, 0, 0, 1]
constexpr int kQpSwap1 = 0xB1;     // [1, 0, 3, 2]
constexpr int kQpSwap2 = 0x4E;     // [2, 3, 0, 1]
constexpr int kQpLast = 0xFF;      // [3, 3, 3, 3]

template <int kSel>
__device__ inline float qperm(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), kSel, 0xf, 0xf, false));
}

template <int kSel>
__device__ inline uint32_t qperm_u(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kSel, 0xf, 0xf, false);
}

__device__ inline float quad_sum(float v)
{
    v += qperm<kQpSwap1>(v);
    return v + qperm<kQpSwap2>(v);
}

__device__ inline uint32_t quad_sum_u(uint32_t v)
{
    v += qperm_u<kQpSwap1>(v);
    return v + qperm_u<kQpSwap2>(v);
}

__device__ inline uint32_t quad_max(uint32_t v)
{
    const uint32_t a = qperm_u<kQpSwap1>(v);
    v = a > v ? a : v;
    const uint32_t b = qperm_u<kQpSwap2>(v);
    return b > v ? b : v;
}

// One step of four entries for one pixel (see above); j = lane & 3.  The
// common case, where no pixel of the wave finishes in the step, takes a short
// path: every taken entry is composited and T becomes T prod f.
__device__ inline void composite4(float alpha, float cr, float cg, float cb, uint32_t k1, int j, float& T, float& thr,
                                  float& C0, float& C1, float& C2, uint32_t& last, uint32_t& walked)
{
    const bool take = alpha >= thr;
    const float f = take ? 1.0f - alpha : 1.0f;
    // inclusive prefix product of f over the pixel's lanes (every lane takes
    // part in each DPP move; the lane's own factor is selected afterwards)
    float q = f;
    const float t1 = qperm<kQpPrev>(q);
    q = j >= 1 ? q * t1 : q;
    const float t2 = qperm<kQpPrev2>(q);
    q = j >= 2 ? q * t2 : q;
    const float qp = qperm<kQpPrev>(q);
    const float ex = j >= 1 ? qp : 1.0f;
    const float Tj = T * ex;
    const float tT = T * q;
    const float t3 = qperm<kQpLast>(tT);
    if (__ballot(take && tT < kTMin) == 0ull) {
        const float wt = take ? alpha * Tj : 0.0f;
        C0 = fmaf(wt, cr, C0);
        C1 = fmaf(wt, cg, C1);
        C2 = fmaf(wt, cb, C2);
        last = take ? k1 : last;
        T = t3;
        return;
    }
    const bool ok = take && tT >= kTMin;
    const bool fin = take && !ok;
    const float wt = ok ? alpha * Tj : 0.0f;
    C0 = fmaf(wt, cr, C0);
    C1 = fmaf(wt, cg, C1);
    C2 = fmaf(wt, cb, C2);
    last = ok ? k1 : last;
    // several lanes may be taken below 1e-4; the first of them finishes the
    // pixel, and it has the largest T_j among them (each taken entry lowers
    // T_j of the next by its factor f < 1).  v >= 0, so its bits order like
    // unsigned integers: an integer max.
    uint32_t v = fin ? __float_as_uint(Tj) : 0u;
    v = quad_max(v);
    walked = (fin && __float_as_uint(Tj) == v) ? k1 : walked;
    const bool done = v != 0u;
    T = done ? __uint_as_float(v) : t3;
    thr = done ? 2.0f : thr;
}

constexpr int kUnitBatch = 224;   // entries staged per batch, as the tile path (under 20 KB of LDS)

// kRegion: a clip region, as in blend_tile (the further planes' terms of each
// CUTOFF entry staged in s_ext, the weight from the entry's plane mask), in
// batches of kRegionBatch entries.
template <bool kWalked, bool kRegion>
__device__ inline void blend_unit(const Splat* __restrict__ splats, const RayRec* __restrict__ rays,
                                  const float2* __restrict__ ray_ext, const uint32_t* __restrict__ vals,
                                  const uint2 rg, int tile, int quad, const RenderParams& p, float4* s_a, float4* s_b,
                                  float2* s_c, CutRec* s_cut, float2* s_ext, const float2* s_rate, uint8_t* s_list,
                                  float* __restrict__ image, float* __restrict__ final_T,
                                  uint32_t* __restrict__ n_contrib, uint32_t* __restrict__ n_walked,
                                  uint32_t* __restrict__ n_eval)
{
    constexpr int kUB = kRegion ? kRegionBatch : kUnitBatch;
    const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int j = lane & 3, pp = lane >> 2;
    const int ox8 = (quad & 1) * 8 + (pp & 7), oy8 = (quad >> 1) * 8 + 2 * wave + (pp >> 3);
    const float lpx = (float)ox8, lpy = (float)oy8;
    const int px = tx * kTile + ox8, py = ty * kTile + oy8;
    const bool inside = px < p.W && py < p.H;

    float T = 1.0f, thr = inside ? kAlphaMin : 2.0f;
    float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    uint32_t last = 0u, walked = 0u, ev = 0u, evc = 0u;
    // the long lists set the tail of the launch: issue priority over the short tiles
    __builtin_amdgcn_s_setprio(3);

    const double ox = (double)(tx * kTile), oy = (double)(ty * kTile);
    const bool plane_on = p.plane_enabled != 0;
    const bool strict = (p.plane_enabled & RARA_CLIP_STRICT_MISS) != 0;
    bool live = __ballot(thr < 1.0f) != 0ull;

    for (uint32_t base = rg.x; base < rg.y; base += kUB) {
        if (!__syncthreads_or(live ? 1 : 0)) break;   // also: the previous batch has been read
        const uint32_t idx = base + (uint32_t)tid;
        float2 sc = make_float2(0.0f, 0.0f);   // reaches no strip
        if (tid < kUB && idx < rg.y) {
            const uint32_t id = vals[idx];
            const Splat sp = splats[id];
            float4 sa, sb;
            uint32_t sm;
            stage_entry_strips(sp, ox, oy, quad, strict, sa, sb, sc, sm);
            s_a[tid] = sa;
            s_b[tid] = sb;
            if ((__float_as_uint(sc.y) & 0xffu) == RARA_LABEL_CUTOFF && plane_on && sm) {
                const float4* rr = reinterpret_cast<const float4*>(rays + id);
                s_cut[tid].a = rr[0];
                s_cut[tid].b = rr[1];
                s_cut[tid].c = rr[2];
                if (kRegion)
                    for (int k = 0; k < p.plane_count - 1; ++k)
                        s_ext[tid * (kMaxPlanes - 1) + k] = ray_ext[(int64_t)id * (kMaxPlanes - 1) + k];
            }
        }
        if (tid < slots_of<kRegion>()) s_c[tid] = sc;
        __syncthreads();
        if (!live) continue;
        const uint32_t cnt = rg.y - base < (uint32_t)kUB ? rg.y - base : (uint32_t)kUB;
        const uint32_t kofs = base - rg.x + 1u;
        for (uint32_t sub = 0; sub < cnt && live; sub += 64) {
            const uint32_t lm = __float_as_uint(s_c[sub + lane].y);
            const bool mine = (lm >> (8 + wave)) & 1u;
            const uint64_t todo = __ballot(mine);
            // the window's entries that reach the strip, in list order, listed
            // in this wave's row of s_list (a wave's own LDS writes and reads
            // are ordered)
            const uint32_t pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(todo >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)todo, 0u));
            if (mine) s_list[wave * 64 + pos] = (uint8_t)lane;
            const uint32_t nsel = (uint32_t)__builtin_popcountll(todo);
            int steps = 0;
            for (uint32_t k = 0; k < nsel; k += 4) {
                // lane j of each pixel takes the (k + j)-th of them
                const bool valid = k + (uint32_t)j < nsel;
                const uint32_t e = s_list[wave * 64 + (valid ? k + (uint32_t)j : k)];
                const uint32_t E = sub + e;
                const float4 a = s_a[E], b = s_b[E];
                const float2 c2 = s_c[E];
                const float cb_ = c2.x;
                const float dx = lpx - a.x, dy = lpy - a.y;
                const float a0 = entry_a0(entry_power(a, b, dx, dy), b.y);
                float alpha = fminf(kAlphaMax, a0);   // w = 1
                const bool cut = plane_on && (__float_as_uint(c2.y) & 0xffu) == RARA_LABEL_CUTOFF;
                // alpha <= a0 (w <= 1): the weights are needed only when some live
                // pixel's CUTOFF entry can reach its threshold
                if (__ballot(valid && cut && a0 >= thr) != 0ull) {
                    float w;
                    if (kRegion) {
                        // the planes that do not hold the whole ellipsoid on their visible side
                        const uint32_t cuts = (__float_as_uint(c2.y) >> 16) & 0xffu;
                        if (!strict && __popc(cuts) == 1) {
                            // one plane: eq. (11) with that plane's terms
                            const int kp = __ffs(cuts) - 1;
                            CutRec rec = s_cut[E];
                            float pax = p.ax, pay = p.ay;
                            if (kp > 0) {
                                const float2 x = s_ext[E * (kMaxPlanes - 1) + kp - 1];
                                rec.c.z = x.x;
                                rec.c.w = x.y;
                                pax = s_rate[kp - 1].x;
                                pay = s_rate[kp - 1].y;
                            }
                            w = chord_weight_flat(rec, dx, dy, pax, pay, false);
                        } else {
                            w = chord_weight_region(s_cut[E], s_ext + E * (kMaxPlanes - 1), p.plane_count, dx, dy,
                                                    p.ax, p.ay, s_rate, strict, strict ? 0xffu : cuts);
                        }
                    } else {
                        w = chord_weight_flat(s_cut[E], dx, dy, p.ax, p.ay, strict);
                    }
                    alpha = cut ? fminf(kAlphaMax, a0 * w) : alpha;
                    if (kWalked) evc += (valid && cut && thr < 1.0f) ? 1u : 0u;
                }
                if (kWalked) ev += (valid && thr < 1.0f) ? 1u : 0u;
                composite4(valid ? alpha : 0.0f, b.z, b.w, cb_, kofs + E, j, T, thr, C0, C1, C2, last, walked);
                if (++steps == 4) {
                    steps = 0;
                    live = __ballot(thr < 1.0f) != 0ull;
                    if (!live) break;
                }
            }
            live = __ballot(thr < 1.0f) != 0ull;
        }
    }

    C0 = quad_sum(C0);
    C1 = quad_sum(C1);
    C2 = quad_sum(C2);
    last = quad_max(last);
    walked = quad_max(walked);
    if (kWalked) {
        ev = quad_sum_u(ev);
        evc = quad_sum_u(evc);
    }
    if (!inside || j != 0) return;
    const int64_t HW = (int64_t)p.H * p.W;
    const int64_t pix = (int64_t)py * p.W + px;
    image[pix] = C0 + T * p.bg[0];
    image[HW + pix] = C1 + T * p.bg[1];
    image[2 * HW + pix] = C2 + T * p.bg[2];
    final_T[pix] = T;
    n_contrib[pix] = last;
    if (kWalked && n_walked) n_walked[pix] = thr < 1.0f ? rg.y - rg.x : walked;
    if (kWalked && n_eval) {
        n_eval[pix] = ev;
        n_eval[HW + pix] = evc;
    }
}

template <bool kWalked, bool kRegion>
__device__ __forceinline__ void blend_block(const Splat* __restrict__ splats, const RayRec* __restrict__ rays,
                                            const float2* __restrict__ ray_ext, const uint32_t* __restrict__ vals,
                                            const uint2* __restrict__ ranges, const uint32_t* __restrict__ work,
                                            const RenderParams& p, float* __restrict__ image,
                                            float* __restrict__ final_T, uint32_t* __restrict__ n_contrib,
                                            uint32_t* __restrict__ n_walked, uint32_t* __restrict__ n_eval,
                                            uint32_t block)
{
    uint32_t tile;
    int quad = -1;
    // long lists as quadrant units, the others one workgroup per tile
    if (!unit_of_block(block, work, p.num_tiles, tile, quad)) return;
    if (tile >= (uint32_t)p.num_tiles) return;
    constexpr int kB = batch_of<kRegion>();
    __shared__ float4 s_a[kB], s_b[kB];
    __shared__ float2 s_c[slots_of<kRegion>()];
    __shared__ CutRec s_cut[kB];
    __shared__ float2 s_ext[kRegion ? kB * (kMaxPlanes - 1) : 1];
    __shared__ float2 s_rate[kMaxPlanes - 1];
    __shared__ uint8_t s_list[4 * 64];
    if (kRegion) {
        // the further planes' per-frame rates; a barrier orders them before any visit (the tile walk's
        // opening one, or a unit's first batch)
        if (threadIdx.x < kMaxPlanes - 1) s_rate[threadIdx.x] = make_float2(p.xax[threadIdx.x], p.xay[threadIdx.x]);
    }
    if (quad >= 0) {
        static_assert(kUnitBatch <= kTileBatch, "the units reuse the tile path's LDS");
        blend_unit<kWalked, kRegion>(splats, rays, ray_ext, vals, ranges[tile], (int)tile, quad, p, s_a, s_b, s_c,
                                     s_cut, s_ext, s_rate, s_list, image, final_T, n_contrib, n_walked, n_eval);
        return;
    }
    blend_tile<kWalked, kRegion>(splats, rays, ray_ext, vals, ranges[tile], (int)tile, p, s_a, s_b, s_c, s_cut, s_ext,
                                 s_rate, image, final_T, n_contrib, n_walked, n_eval);
}

template <bool kWalked>
__global__ __launch_bounds__(kBlendThreads) __attribute__((amdgpu_waves_per_eu(8)))
void blend_kernel(const Splat* __restrict__ splats, const RayRec* __restrict__ rays, const uint32_t* __restrict__ vals,
                  const uint2* __restrict__ ranges, const uint32_t* __restrict__ work,
                  const int32_t* __restrict__ overflow, RenderParams p, float* __restrict__ image,
                  float* __restrict__ final_T, uint32_t* __restrict__ n_contrib, uint32_t* __restrict__ n_walked,
                  uint32_t* __restrict__ n_eval)
{
    if (*overflow) return;
    blend_block<kWalked, false>(splats, rays, nullptr, vals, ranges, work, p, image, final_T, n_contrib, n_walked,
                                n_eval, blockIdx.x);
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
                         uint32_t* __restrict__ n_walked, uint32_t* __restrict__ n_eval)
{
    if (*overflow) return;
    blend_block<kWalked, true>(splats, rays, ray_ext, vals, ranges, work, p, image, final_T, n_contrib, n_walked,
                               n_eval, blockIdx.x);
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
    blend_block<kWalked, false>(splats, rays, nullptr, vals, ranges, work, p, image, final_T, n_contrib, n_walked,
                                nullptr, blockIdx.x);
}

// Several frames in one launch (rara_render_batch): item i owns the
// workgroups [first_block_i, first_block_{i+1}), each a multiple of 8 so that
// a workgroup's XCD (b mod 8) is the same in the item's own numbering.
__global__ __launch_bounds__(kBlendThreads) __attribute__((amdgpu_waves_per_eu(8)))
void blend_batch_kernel(BatchArgs a)
{
    const uint32_t b = blockIdx.x;
    int i = 0;
    while (i + 1 < a.count && b >= a.items[i + 1].first_block) ++i;
    const BatchItem& it = a.items[i];
    if (*it.overflow) return;
    blend_block<false, false>(it.splat, it.ray, nullptr, it.vals, it.ranges, it.work, it.p, it.image, it.final_T,
                              it.n_contrib, nullptr, nullptr, b - it.first_block);
}

}  // namespace

hipError_t launch_blend_batch(BatchArgs& a, hipStream_t s)
{
    uint32_t next = 0;
    for (int i = 0; i < a.count; ++i) {
        a.items[i].first_block = next;
        next += (uint32_t)((blend_grid(a.items[i].p.num_tiles) + 7) / 8 * 8);
    }
    hipLaunchKernelGGL(blend_batch_kernel, dim3(next), dim3(kBlendThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_blend(const Splat* splat, const RayRec* ray, const float2* ray_ext, const rara_binned& bins,
                        const RenderParams& p, float* image, float* final_T, uint32_t* n_contrib, uint32_t* n_walked,
                        uint32_t* n_eval, hipStream_t s)
{
    const uint2* ranges = reinterpret_cast<const uint2*>(bins.ranges);
    const bool count = n_walked || n_eval;
    if (p.plane_enabled && p.plane_count > 1) {
        const unsigned grid = (unsigned)blend_grid(p.num_tiles);
        if (count)
            hipLaunchKernelGGL(blend_region_kernel<true>, dim3(grid), dim3(kBlendThreads), 0, s, splat, ray, ray_ext,
                               bins.vals, ranges, bins.work, bins.overflow, p, image, final_T, n_contrib, n_walked,
                               n_eval);
        else
            hipLaunchKernelGGL(blend_region_kernel<false>, dim3(grid), dim3(kBlendThreads), 0, s, splat, ray, ray_ext,
                               bins.vals, ranges, bins.work, bins.overflow, p, image, final_T, n_contrib, n_walked,
                               n_eval);
        return hipGetLastError();
    }
    const unsigned grid = (unsigned)blend_grid(p.num_tiles);
    if (count)
        hipLaunchKernelGGL(blend_kernel<true>, dim3(grid), dim3(kBlendThreads), 0, s, splat, ray, bins.vals, ranges,
                           bins.work, bins.overflow, p, image, final_T, n_contrib, n_walked, n_eval);
    else
        hipLaunchKernelGGL(blend_kernel<false>, dim3(grid), dim3(kBlendThreads), 0, s, splat, ray, bins.vals, ranges,
                           bins.work, bins.overflow, p, image, final_T, n_contrib, n_walked, n_eval);
    return hipGetLastError();
}

hipError_t launch_blend_fp(const Splat* splat, const RayRec* ray, const rara_binned& bins, const FrameParams* fp,
                           int num_tiles, float* image, float* final_T, uint32_t* n_contrib, uint32_t* n_walked,
                           hipStream_t s)
{
    const unsigned grid = (unsigned)blend_grid(num_tiles);
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
