// Backward pass of the clipped frame (not in the paper, which is render-only):
// gradients of a scalar loss L, given dL/dimage, with respect to the raw
// Gaussian inputs (mean, scale, quaternion, opacity, SH) and the raw plane
// (n, d).
//
//   blend_backward  per work unit (the forward's schedule), walk the tile list
//                   back to front from each pixel's n_contrib, rebuilding the
//                   transmittance by division (alpha <= 0.99 keeps it bounded)
//                   and re-evaluating alpha and the clip weight with the
//                   forward's own arithmetic, so that the composite / skip
//                   decisions are the forward's bit for bit.  Per entry the
//                   per-pixel gradients are summed over each wave, the four
//                   waves of a tile combine them in LDS, and the 21 sums go to
//                   the pair's own slot (its position in emission order) with
//                   plain stores: no per-Gaussian atomics.
//   slot_sum        per Gaussian, the FP64 sum of its (contiguous) pair slots
//                   (a light kernel, so that many waves hide the loads);
//   project_backward per Gaussian, the FP64 chain rule from (mean2d, conic,
//                   opacity, colour, ray set-up) to (mean, scale, quaternion,
//                   opacity, SH) and the plane, through the EWA projection of
//                   eqs. (9)-(10), the SH colour and eq. (4)'s whitening.
//   plane_finalize  plane gradient from the normalised (n, d) and the
//                   per-view pixel-rate terms to the raw (n, d).
#include "blend_common.h"

namespace rara {

namespace {

// accumulator rows, each [n] floats
enum {
    A_MX = 0, A_MY, A_CA, A_CB, A_CC, A_OP, A_R, A_G, A_B,
    A_D0, A_GX = A_D0 + 3, A_GY = A_GX + 3, A_Z = A_GY + 3, A_DEP, A_G0, kAccRows
};
// plane accumulators: dn_hat[3], dd_hat, dax, day
constexpr int kPlaneAcc = 8;

// Sum over the 64 lanes, returned to every lane, with DPP row operations (no
// LDS): shifts by 1, 2, 4 and 8 within each 16-lane row leave the row sum in
// the row's last lane; broadcasting lane 15 into row 1 and row 3, then lane 31
// into rows 2 and 3, leaves the wave sum in lane 63.  Lanes a DPP move does
// not write (row edges, masked rows) take 0.
template <int kCtrl, int kRowMask>
__device__ inline float dpp_step(float v)
{
    const int moved = __builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, kRowMask, 0xf, false);
    return v + __int_as_float(moved);
}

__device__ inline float wave_sum(float v)
{
    v = dpp_step<0x111, 0xf>(v);   // row_shr:1
    v = dpp_step<0x112, 0xf>(v);   // row_shr:2
    v = dpp_step<0x114, 0xf>(v);   // row_shr:4
    v = dpp_step<0x118, 0xf>(v);   // row_shr:8
    v = dpp_step<0x142, 0xa>(v);   // row_bcast:15 into rows 1, 3
    v = dpp_step<0x143, 0xc>(v);   // row_bcast:31 into rows 2, 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Wave sums of M values at once by halving: a level at lane distance D pairs
// value i with value i + P (P = ceil(M / 2)) and swaps them with the partner
// lane l ^ D, so that lanes with bit D clear go on with the sums of the first
// half and lanes with bit D set with those of the second.  After the levels
// D = 32, 16, ..., 1 every lane holds one 64-lane sum (or padding) and
// halve_index names which.  Distances 32 and 16 use v_permlane32_swap and
// v_permlane16_swap, which exchange both halves in one instruction; 8, 2 and 1
// use DPP row_ror:8 and quad_perm; 4 uses row_half_mirror (j -> 7 - j) and then
// quad_perm [3,2,1,0] (j -> j ^ 3).  About 2.5 instructions per value instead
// of the eight of a wave_sum and its lane select.
template <int D>
__device__ inline float lane_xor(float v)
{
    const int i = __float_as_int(v);
    if constexpr (D == 8) {
        return __int_as_float(__builtin_amdgcn_update_dpp(0, i, 0x128, 0xf, 0xf, false));
    } else if constexpr (D == 4) {
        const int m = __builtin_amdgcn_update_dpp(0, i, 0x141, 0xf, 0xf, false);
        return __int_as_float(__builtin_amdgcn_update_dpp(0, m, 0x1b, 0xf, 0xf, false));
    } else if constexpr (D == 2) {
        return __int_as_float(__builtin_amdgcn_update_dpp(0, i, 0x4e, 0xf, 0xf, false));
    } else {
        static_assert(D == 1, "lane distance");
        return __int_as_float(__builtin_amdgcn_update_dpp(0, i, 0xb1, 0xf, 0xf, false));
    }
}

// a[l] + a[l ^ D] in lanes with bit D clear, b[l ^ D] + b[l] in the others
template <int D>
__device__ inline float halve_pair(float a, float b, bool hi)
{
    if constexpr (D == 32 || D == 16) {
        const auto r = D == 32 ? __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false)
                               : __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
        return __uint_as_float(r[0]) + __uint_as_float(r[1]);
    } else {
        return (hi ? b : a) + lane_xor<D>(hi ? a : b);
    }
}

template <int M, int D>
__device__ inline float halve_sum(const float (&v)[M], int lane)
{
    static_assert(M >= 1 && M <= 2 * D, "values per lane");
    constexpr int P = (M + 1) / 2;
    const bool hi = (lane & D) != 0;
    float h[P];
#pragma unroll
    for (int i = 0; i < P; ++i)
        // a value with no second-half partner is summed in both halves; the
        // upper copy is padding
        h[i] = halve_pair<D>(v[i], i + P < M ? v[i + P] : v[i], hi);
    if constexpr (D == 1)
        return h[0];
    else
        return halve_sum<P, D / 2>(h, lane);
}

// which of M values halve_sum leaves in this lane, -1 for padding
__device__ inline int halve_index(int m, int lane)
{
    int ms[7];
    ms[0] = m;
#pragma unroll
    for (int j = 0; j < 6; ++j) ms[j + 1] = (ms[j] + 1) / 2;
    int idx = 0;
#pragma unroll
    for (int j = 5; j >= 0; --j) {   // level j has lane distance 32 >> j
        idx += ((lane >> (5 - j)) & 1) ? ms[j + 1] : 0;
        if (idx >= ms[j]) return -1;
    }
    return idx;
}

__device__ inline uint32_t wave_max(uint32_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

struct BackParams {
    RenderParams rp;
    int64_t n;
};

// Backward of the interior branch of the clip weight: given dL/dw, the
// gradients of the staged ray set-up (g[0..11] = d0, gx, gy, z, dep, g0), of
// the pixel offset, and of the per-view plane rates (ax, ay).
__device__ inline void chord_backward(const CutRec& k, const Chord& c, float dx, float dy, float ax, float ay,
                                      float dw, float* g, float& ddx, float& ddy, float& dax, float& day)
{
    const float gx[3] = {k.a.w, k.b.x, k.b.y};
    const float gy[3] = {k.b.z, k.b.w, k.c.x};
    const float z = k.c.y;
    // w = 1/2 + phim inv, inv = 1 / (2 |g| hs)
    const float dphim = dw * c.inv;
    const float dden = -dw * c.phim * c.inv * c.inv;
    const float sg = c.gg > 0.0f ? 1.0f : -1.0f;
    float dgg = dden * 2.0f * c.hs * sg;
    float dhs = dden * 2.0f * fabsf(c.gg);
    // phim = dep + z u + sm g
    const float ddep = dphim;
    float dz = dphim * c.u;
    float du = dphim * z;
    float dsm = dphim * c.gg;
    dgg += dphim * c.sm;
    const float dg0 = dgg;   // g = g0 + u
    du += dgg;
    dax += du * dx;
    day += du * dy;
    ddx += du * ax;
    ddy += du * ay;
    // hs = sqrt(h2 / DD)
    const float dh2 = dhs * 0.5f * c.iDD / c.hs;
    float dDD = -dhs * 0.5f * c.hs * c.iDD;
    // h2 = 9 - Q.Q ; Q = P + sm D
    float dP[3], dD[3];
    for (int i = 0; i < 3; ++i) {
        const float dQ = -2.0f * c.Q[i] * dh2;
        dP[i] = dQ;
        dsm += dQ * c.D[i];
        dD[i] = c.sm * dQ;
    }
    // sm = -PD / DD
    const float dPD = -dsm * c.iDD;
    dDD += dsm * c.PD * c.iDD * c.iDD;
    for (int i = 0; i < 3; ++i) {
        dP[i] += dPD * c.D[i];
        dD[i] += dPD * c.P[i] + 2.0f * dDD * c.D[i];
    }
    // P = z e ; D = d0 + e ; e = gx dx + gy dy
    for (int i = 0; i < 3; ++i) {
        dz += dP[i] * c.e[i];
        const float de = z * dP[i] + dD[i];
        g[i] += dD[i];            // d0
        g[3 + i] += de * dx;      // gx
        g[6 + i] += de * dy;      // gy
        ddx += de * gx[i];
        ddy += de * gy[i];
    }
    g[9] += dz;
    g[10] += ddep;
    g[11] += dg0;
}

constexpr int kBackBatch = 128;   // entries staged per batch (threads 0..127 stage)

// Gradient slot of the pair (tile (tx, ty), Gaussian id): its position in
// emission order, the Gaussian's first pair plus the number of its listed
// tiles before this one, row by row over its rectangle.
__device__ inline uint32_t pair_slot(uint32_t first, const ulonglong2& rec, int tx, int ty)
{
    // the record's rectangle: tx0, ty0, tx1, ty1 as uint16, lowest first
    const int x0 = (int)(rec.x & 0xffffu), y0 = (int)((rec.x >> 16) & 0xffffu);
    const int x1 = (int)((rec.x >> 32) & 0xffffu), y1 = (int)(rec.x >> 48);
    const uint32_t w = (uint32_t)(x1 - x0);
    const uint32_t k = (uint32_t)(ty - y0) * w + (uint32_t)(tx - x0);
    return first + listed_rank(rec.y, (int)w * (y1 - y0), k);
}

// One tile, back to front.  Thread t of wave w = t / 64 owns pixel
// (t % 8, (t / 8) % 8) of the 8x8 quadrant w, as in the forward.  The list is
// walked from the tile's largest n_contrib down, in batches of kBackBatch
// staged entries; each wave visits, in descending order, the entries that
// reach its quadrant.  Per entry the wave sums its pixels' gradients and adds
// them to the entry's LDS accumulators (the four waves share them); after the
// batch every staged entry's 21 sums go to its pair slot with plain stores.
// Entries past the largest n_contrib get zero slots.
__device__ inline void blend_back_tile(const Splat* __restrict__ splats, const RayRec* __restrict__ rays,
                                       const uint32_t* __restrict__ vals, const uint32_t* __restrict__ pair_start,
                                       const ulonglong2* __restrict__ tile_rec,
                                       const uint2 rg, int tile,
                                       const BackParams& bp, const float* __restrict__ final_T,
                                       const uint32_t* __restrict__ n_contrib, const float* __restrict__ dL_dimage,
                                       float* __restrict__ slots, float* __restrict__ plane_acc, float4* s_a,
                                       float4* s_b, float4* s_c, CutRec* s_cut, uint32_t* s_slot,
                                       float (*s_g)[kAccRows], uint32_t* s_red)
{
    const RenderParams& p = bp.rp;
    const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int row_all = halve_index(kAccRows, lane), row_base = halve_index(A_D0, lane);
    const int ox8 = (wave & 1) * 8 + (lane & 7), oy8 = (wave >> 1) * 8 + (lane >> 3);
    const float lpx = (float)ox8, lpy = (float)oy8;
    const int px = tx * kTile + ox8, py = ty * kTile + oy8;
    const bool inside = px < p.W && py < p.H;
    const int64_t HW = (int64_t)p.H * p.W;
    const int64_t pix = (int64_t)py * p.W + px;

    float T = inside ? final_T[pix] : 0.0f;
    const float Tfin = T;
    const uint32_t nc = inside ? n_contrib[pix] : 0u;
    float dC[3], ac[3] = {0.0f, 0.0f, 0.0f}, lc[3] = {0.0f, 0.0f, 0.0f}, la = 0.0f, bgdot = 0.0f;
    for (int ch = 0; ch < 3; ++ch) {
        dC[ch] = inside ? dL_dimage[ch * HW + pix] : 0.0f;
        bgdot += p.bg[ch] * dC[ch];
    }
    // the wave's and the tile's largest n_contrib (the tile's clamped to the list length)
    const uint32_t wm = wave_max(nc);
    if (lane == 0) s_red[wave] = wm;
    __syncthreads();
    uint32_t kmax = s_red[0];
    for (int w = 1; w < 4; ++w) kmax = s_red[w] > kmax ? s_red[w] : kmax;
    if (kmax > rg.y - rg.x) kmax = rg.y - rg.x;

    const bool plane_on = p.plane_enabled != 0;
    const bool strict = (p.plane_enabled & RARA_CLIP_STRICT_MISS) != 0;
    const double ox = (double)(tx * kTile), oy = (double)(ty * kTile);
    float pax = 0.0f, pay = 0.0f;

    for (uint32_t hi = rg.x + kmax; hi > rg.x;) {
        const uint32_t lo = hi - rg.x > (uint32_t)kBackBatch ? hi - kBackBatch : rg.x;
        const uint32_t cnt = hi - lo;
        __syncthreads();   // the previous batch has been read and written out
        if (tid < kBackBatch) {
            for (int r = 0; r < kAccRows; ++r) s_g[tid][r] = 0.0f;
            float4 sc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);   // mask 0: reaches nothing
            if ((uint32_t)tid < cnt) {
                const uint32_t id = vals[lo + tid];
                const Splat sp = splats[id];
                float4 sa, sb;
                uint32_t qm;
                stage_entry(sp, ox, oy, 0xfu, strict, sa, sb, sc, qm, id);
                s_a[tid] = sa;
                s_b[tid] = sb;
                if ((__float_as_uint(sc.y) & 0xffu) == RARA_LABEL_CUTOFF && plane_on) {
                    const float4* rr = reinterpret_cast<const float4*>(rays + id);
                    const float4 r0 = rr[0], r1 = rr[1], r2 = rr[2];
                    s_cut[tid].a = r0;
                    s_cut[tid].b = r1;
                    s_cut[tid].c = r2;
                }
                s_slot[tid] = pair_slot(pair_start[id], tile_rec[id], tx, ty);
            }
            s_c[tid] = sc;
        }
        __syncthreads();
        // visit this wave's entries in descending order, 64 at a time
        for (int sub = (int)((cnt - 1) & ~63u); sub >= 0; sub -= 64) {
            const uint32_t lm = __float_as_uint(s_c[sub + lane].y);
            uint64_t todo = __ballot((lm >> (8 + wave)) & 1u);
            // entries past the wave's largest n_contrib change none of its pixels
            const uint32_t kb = lo - rg.x + (uint32_t)sub;   // entry sub + j has k1 = kb + j + 1
            if (wm <= kb)
                todo = 0ull;
            else if (wm - kb < 64u)
                todo &= (1ull << (wm - kb)) - 1ull;
            const uint64_t cutb = __ballot(plane_on && (lm & 0xffu) == RARA_LABEL_CUTOFF);
            while (todo) {
                const int j = 63 - (int)__builtin_clzll(todo);
                todo &= ~(1ull << j);
                const int e = sub + j;
                const float4 a = s_a[e], b = s_b[e], c = s_c[e];
                const uint32_t k1 = lo - rg.x + (uint32_t)e + 1u;
                const bool cut = (cutb >> j) & 1ull;
                float g_mx = 0.f, g_my = 0.f, g_ca = 0.f, g_cb = 0.f, g_cc = 0.f, g_op = 0.f;
                float g_col[3] = {0.f, 0.f, 0.f};
                float g_ray[12];
                for (int r = 0; r < 12; ++r) g_ray[r] = 0.f;
                bool contributed = false;
                if (k1 <= nc) {
                    const float dx = lpx - a.x, dy = lpy - a.y;
                    const float pw = entry_power(a, b, dx, dy);
                    const float G2 = __builtin_amdgcn_exp2f(pw);
                    const float a0 = b.y * G2;
                    Chord ch;
                    float w = 1.0f;
                    if (cut) {
                        chord_eval(s_cut[e], dx, dy, p.ax, p.ay, strict, ch);
                        w = ch.w;
                    }
                    const float aw = a0 * w;
                    const float alpha = fminf(kAlphaMax, aw);
                    if (pw <= 0.0f && alpha >= kAlphaMin) {
                        contributed = true;
                        const float inv1ma = __builtin_amdgcn_rcpf(1.0f - alpha);   // alpha <= 0.99
                        T = T * inv1ma;
                        const float col[3] = {b.z, b.w, c.x};
                        float dLda = 0.0f;
                        for (int k = 0; k < 3; ++k) {
                            ac[k] = la * lc[k] + (1.0f - la) * ac[k];
                            lc[k] = col[k];
                            dLda += (col[k] - ac[k]) * dC[k];
                            g_col[k] += alpha * T * dC[k];
                        }
                        dLda *= T;
                        la = alpha;
                        dLda += (-Tfin * inv1ma) * bgdot;
                        if (aw < kAlphaMax) {
                            const float dLda0 = dLda * w;
                            g_op += dLda0 * G2;
                            const float dpow = dLda0 * a0;   // d alpha0 / d power = alpha0
                            g_ca += dpow * (-0.5f * dx * dx);
                            g_cb += dpow * (-dx * dy);
                            g_cc += dpow * (-0.5f * dy * dy);
                            // d power / d dx = -(ca dx + cb dy) from the base-2 scaled staged conic
                            float ddx = dpow * (2.0f * a.z * dx + a.w * dy) * (1.0f / kLog2e);
                            float ddy = dpow * (a.w * dx + 2.0f * b.x * dy) * (1.0f / kLog2e);
                            if (cut && ch.kind == 4)
                                chord_backward(s_cut[e], ch, dx, dy, p.ax, p.ay, dLda * a0, g_ray, ddx, ddy, pax, pay);
                            g_mx -= ddx;
                            g_my -= ddy;
                        }
                    }
                }
                if (__ballot(contributed) != 0ull) {
                    // the wave sums, one row per lane, added with one LDS instruction
                    float sum;
                    int row;
                    if (cut) {
                        const float v[kAccRows] = {g_mx, g_my, g_ca, g_cb, g_cc, g_op, g_col[0], g_col[1], g_col[2],
                                                   g_ray[0], g_ray[1], g_ray[2], g_ray[3], g_ray[4], g_ray[5],
                                                   g_ray[6], g_ray[7], g_ray[8], g_ray[9], g_ray[10], g_ray[11]};
                        sum = halve_sum<kAccRows, 32>(v, lane);
                        row = row_all;
                    } else {
                        const float v[A_D0] = {g_mx, g_my, g_ca, g_cb, g_cc, g_op, g_col[0], g_col[1], g_col[2]};
                        sum = halve_sum<A_D0, 32>(v, lane);
                        row = row_base;
                    }
                    if (row >= 0 && sum != 0.0f) atomicAdd(&s_g[e][row], sum);
                }
            }
        }
        __syncthreads();
        if ((uint32_t)tid < cnt) {
            float* dst = slots + (int64_t)s_slot[tid] * kAccRows;
            for (int r = 0; r < kAccRows; ++r) dst[r] = s_g[tid][r];
        }
        hi = lo;
    }
    // entries after the last composited one: zero slots
    for (uint32_t k = rg.x + kmax + (uint32_t)tid; k < rg.y; k += blockDim.x) {
        const uint32_t id = vals[k];
        float* dst = slots + (int64_t)pair_slot(pair_start[id], tile_rec[id], tx, ty) * kAccRows;
        for (int r = 0; r < kAccRows; ++r) dst[r] = 0.0f;
    }
    const float sx = wave_sum(pax), sy = wave_sum(pay);
    if (lane == 0 && (sx != 0.0f || sy != 0.0f)) {
        atomicAdd(plane_acc + 4, sx);
        atomicAdd(plane_acc + 5, sy);
    }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void blend_backward_kernel(
    const Splat* __restrict__ splats, const RayRec* __restrict__ rays, const uint32_t* __restrict__ vals,
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ work, const uint32_t* __restrict__ pair_start,
    const ulonglong2* __restrict__ tile_rec, const int32_t* __restrict__ overflow,
    BackParams bp,
    const float* __restrict__ final_T, const uint32_t* __restrict__ n_contrib, const float* __restrict__ dL_dimage,
    float* __restrict__ slots, float* __restrict__ plane_acc)
{
    if (*overflow) return;
    uint32_t tile;
    if (!tile_of_block(blockIdx.x, work, bp.rp.num_tiles, tile)) return;
    if (tile >= (uint32_t)bp.rp.num_tiles) return;
    __shared__ float4 s_a[kBackBatch], s_b[kBackBatch], s_c[kBackBatch];
    __shared__ CutRec s_cut[kBackBatch];
    __shared__ uint32_t s_slot[kBackBatch];
    __shared__ float s_g[kBackBatch][kAccRows];
    __shared__ uint32_t s_red[4];
    blend_back_tile(splats, rays, vals, pair_start, tile_rec, ranges[tile], (int)tile, bp, final_T, n_contrib,
                    dL_dimage, slots, plane_acc, s_a, s_b, s_c, s_cut, s_slot, s_g, s_red);
}

__global__ __launch_bounds__(256) void fill_zero_kernel(float* __restrict__ p, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

// d Y_k / d(x, y, z) of the degree <= 3 real SH basis (same convention and
// constants as the forward), accumulated as ddir += sum_k dY_k grad Y_k.
__device__ inline void sh_backward(int deg, double x, double y, double z, const double* dY, double* dd)
{
    const double c1 = 0.4886025119029199;
    dd[0] = dd[1] = dd[2] = 0.0;
    if (deg < 1) return;
    dd[1] += -c1 * dY[1];
    dd[2] += c1 * dY[2];
    dd[0] += -c1 * dY[3];
    if (deg < 2) return;
    const double c4 = 1.0925484305920792, c6 = 0.31539156525252005, c8 = 0.5462742152960396;
    dd[0] += c4 * y * dY[4];
    dd[1] += c4 * x * dY[4];
    dd[1] += -c4 * z * dY[5];
    dd[2] += -c4 * y * dY[5];
    dd[0] += -2.0 * c6 * x * dY[6];
    dd[1] += -2.0 * c6 * y * dY[6];
    dd[2] += 4.0 * c6 * z * dY[6];
    dd[0] += -c4 * z * dY[7];
    dd[2] += -c4 * x * dY[7];
    dd[0] += 2.0 * c8 * x * dY[8];
    dd[1] += -2.0 * c8 * y * dY[8];
    if (deg < 3) return;
    const double c9 = 0.5900435899266435, c10 = 2.890611442640554, c11 = 0.4570457994644658,
                 c12 = 0.3731763325901154, c14 = 1.445305721320277;
    const double xx = x * x, yy = y * y, zz = z * z;
    dd[0] += -c9 * 6.0 * x * y * dY[9];
    dd[1] += -c9 * (3.0 * xx - 3.0 * yy) * dY[9];
    dd[0] += c10 * y * z * dY[10];
    dd[1] += c10 * x * z * dY[10];
    dd[2] += c10 * x * y * dY[10];
    dd[0] += 2.0 * c11 * x * y * dY[11];
    dd[1] += -c11 * (4.0 * zz - xx - 3.0 * yy) * dY[11];
    dd[2] += -c11 * 8.0 * y * z * dY[11];
    dd[0] += -6.0 * c12 * x * z * dY[12];
    dd[1] += -6.0 * c12 * y * z * dY[12];
    dd[2] += c12 * (6.0 * zz - 3.0 * xx - 3.0 * yy) * dY[12];
    dd[0] += -c11 * (4.0 * zz - 3.0 * xx - yy) * dY[13];
    dd[1] += 2.0 * c11 * x * y * dY[13];
    dd[2] += -8.0 * c11 * x * z * dY[13];
    dd[0] += 2.0 * c14 * x * z * dY[14];
    dd[1] += -2.0 * c14 * y * z * dY[14];
    dd[2] += c14 * (xx - yy) * dY[14];
    dd[0] += -c9 * (3.0 * xx - 3.0 * yy) * dY[15];
    dd[1] += 6.0 * c9 * x * y * dY[15];
}

__device__ inline void sh_values(int deg, double x, double y, double z, double* Y)
{
    Y[0] = 0.28209479177387814;
    if (deg < 1) return;
    Y[1] = -0.4886025119029199 * y;
    Y[2] = 0.4886025119029199 * z;
    Y[3] = -0.4886025119029199 * x;
    if (deg < 2) return;
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[4] = 1.0925484305920792 * x * y;
    Y[5] = -1.0925484305920792 * y * z;
    Y[6] = 0.31539156525252005 * (2.0 * zz - xx - yy);
    Y[7] = -1.0925484305920792 * x * z;
    Y[8] = 0.5462742152960396 * (xx - yy);
    if (deg < 3) return;
    Y[9] = -0.5900435899266435 * y * (3.0 * xx - yy);
    Y[10] = 2.890611442640554 * x * y * z;
    Y[11] = -0.4570457994644658 * y * (4.0 * zz - xx - yy);
    Y[12] = 0.3731763325901154 * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    Y[13] = -0.4570457994644658 * x * (4.0 * zz - xx - yy);
    Y[14] = 1.445305721320277 * z * (xx - yy);
    Y[15] = -0.5900435899266435 * x * (xx - 3.0 * yy);
}

struct GradPtrs {
    float *mean, *scale, *quat, *opacity, *sh;
};

// Sum of each drawn Gaussian's pair slots (contiguous in emission order) in
// FP64: rows 0..8 always, the ray set-up rows 9.. for a CUTOFF Gaussian with
// the plane on; sums[r][i].  Rows a Gaussian does not use are not written.
// A Gaussian with up to kSerialSlots slots is summed by its own thread, in
// slot order; a larger one by the whole wave (lane l takes slots l, l + 64,
// ..., then a wave sum), so that no wave waits on one long serial loop.
constexpr uint32_t kSerialSlots = 32;

__device__ inline double wave_sum_f64(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(256) void slot_sum_kernel(int64_t n, int32_t plane_enabled,
                                                       const uint8_t* __restrict__ label,
                                                       const uint32_t* __restrict__ tiles_touched,
                                                       const uint32_t* __restrict__ pair_start,
                                                       const int32_t* __restrict__ overflow,
                                                       const float* __restrict__ slots, double* __restrict__ sums)
{
    // an overflowed frame has no complete pair slots (nor pair starts): the
    // chain rule writes zero gradients without reading the sums
    if (*overflow) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const uint32_t tt = i < n ? tiles_touched[i] : 0u;
    const bool cutg = tt > 0u && plane_enabled && label[i] == RARA_LABEL_CUTOFF;
    const uint32_t first = tt > 0u ? pair_start[i] : 0u;
    if (tt > 0u && tt <= kSerialSlots) {
        double acc[kAccRows];
        for (int r = 0; r < kAccRows; ++r) acc[r] = 0.0;
        const float* src = slots + (int64_t)first * kAccRows;
        for (uint32_t j = 0; j < tt; ++j, src += kAccRows) {
#pragma unroll
            for (int r = 0; r < 9; ++r) acc[r] += (double)src[r];
            if (cutg) {
#pragma unroll
                for (int r = 9; r < kAccRows; ++r) acc[r] += (double)src[r];
            }
        }
#pragma unroll
        for (int r = 0; r < 9; ++r) sums[r * n + i] = acc[r];
        if (cutg) {
#pragma unroll
            for (int r = 9; r < kAccRows; ++r) sums[r * n + i] = acc[r];
        }
    }
    // the wave's large Gaussians, one after the other
    uint64_t big = __ballot(tt > kSerialSlots);
    while (big) {
        const int src_lane = (int)__builtin_ctzll(big);
        big &= big - 1ull;
        const uint32_t bt = __builtin_amdgcn_readlane(tt, src_lane);
        const uint32_t bfirst = __builtin_amdgcn_readlane(first, src_lane);
        const bool bcut = __builtin_amdgcn_readlane(cutg ? 1 : 0, src_lane) != 0;
        const int64_t bi = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63) + src_lane;
        double acc[kAccRows];
#pragma unroll
        for (int r = 0; r < kAccRows; ++r) acc[r] = 0.0;
        for (uint32_t j = (uint32_t)lane; j < bt; j += 64) {
            const float* src = slots + ((int64_t)bfirst + j) * kAccRows;
#pragma unroll
            for (int r = 0; r < 9; ++r) acc[r] += (double)src[r];
            if (bcut) {
#pragma unroll
                for (int r = 9; r < kAccRows; ++r) acc[r] += (double)src[r];
            }
        }
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            const double t = wave_sum_f64(acc[r]);
            if (lane == 0) sums[r * n + bi] = t;
        }
        if (bcut) {
#pragma unroll
            for (int r = 9; r < kAccRows; ++r) {
                const double t = wave_sum_f64(acc[r]);
                if (lane == 0) sums[r * n + bi] = t;
            }
        }
    }
}

template <int DEG, int kShMode>
__global__ __launch_bounds__(256) void project_backward_kernel(GaussPtrs g, CamParams cam, PlaneParams pl,
                                                               const uint8_t* __restrict__ label,
                                                               const uint32_t* __restrict__ tiles_touched,
                                                               const int32_t* __restrict__ overflow,
                                                               const double* __restrict__ sums, GradPtrs out,
                                                               float* __restrict__ plane_acc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = g.n;
    const bool overflowed = *overflow != 0;   // no sums: every gradient is zero
    constexpr int ncoef = (DEG + 1) * (DEG + 1);
    double pn[4] = {0.0, 0.0, 0.0, 0.0};   // d n_hat, d d_hat contributed by this Gaussian
    if (i < n) {
        double dmu[3] = {0.0, 0.0, 0.0}, ds[3] = {0.0, 0.0, 0.0}, dqv[4] = {0.0, 0.0, 0.0, 0.0};
        double gop = 0.0;
        const uint32_t tt = tiles_touched[i];
        const bool drawn = tt > 0 && !overflowed;
        if (drawn) {
            // the sums of this Gaussian's pair slots (slot_sum_kernel)
            const bool cutg = pl.enabled && label[i] == RARA_LABEL_CUTOFF;
            double acc[kAccRows];
#pragma unroll
            for (int r = 0; r < 9; ++r) acc[r] = sums[r * n + i];
#pragma unroll
            for (int r = 9; r < kAccRows; ++r) acc[r] = cutg ? sums[r * n + i] : 0.0;
            const double mu[3] = {g.mean[i], g.mean[n + i], g.mean[2 * n + i]};
            const double s[3] = {g.scale[i], g.scale[n + i], g.scale[2 * n + i]};
            double q4[4] = {g.quat[i], g.quat[n + i], g.quat[2 * n + i], g.quat[3 * n + i]};
            const double qlen = sqrt(q4[0] * q4[0] + q4[1] * q4[1] + q4[2] * q4[2] + q4[3] * q4[3]);
            const double iqlen = 1.0 / qlen;
            const double qw = q4[0] * iqlen, qx = q4[1] * iqlen, qy = q4[2] * iqlen, qz = q4[3] * iqlen;
            const double R[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
                                 2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
                                 2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
            const double* Rc = cam.R;
            double t[3];
            for (int a = 0; a < 3; ++a) t[a] = Rc[3 * a] * mu[0] + Rc[3 * a + 1] * mu[1] + Rc[3 * a + 2] * mu[2] + cam.t[a];
            const double z = t[2], iz = 1.0 / z;
            const double ur = t[0] * iz, vr = t[1] * iz;
            const bool ux = fabs(ur) <= cam.limx, vy = fabs(vr) <= cam.limy;
            const double u = fmin(cam.limx, fmax(-cam.limx, ur)), v = fmin(cam.limy, fmax(-cam.limy, vr));
            const double j00 = cam.fx * iz, j02 = -cam.fx * u * iz, j11 = cam.fy * iz, j12 = -cam.fy * v * iz;
            double T0[3], T1[3], TR0[3], TR1[3], K0[3], K1[3];
            for (int c = 0; c < 3; ++c) {
                T0[c] = j00 * Rc[c] + j02 * Rc[6 + c];
                T1[c] = j11 * Rc[3 + c] + j12 * Rc[6 + c];
            }
            for (int c = 0; c < 3; ++c) {
                TR0[c] = T0[0] * R[c] + T0[1] * R[3 + c] + T0[2] * R[6 + c];
                TR1[c] = T1[0] * R[c] + T1[1] * R[3 + c] + T1[2] * R[6 + c];
                K0[c] = TR0[c] * s[c];
                K1[c] = TR1[c] * s[c];
            }
            const double v00 = K0[0] * K0[0] + K0[1] * K0[1] + K0[2] * K0[2] + kDilation;
            const double v01 = K0[0] * K1[0] + K0[1] * K1[1] + K0[2] * K1[2];
            const double v11 = K1[0] * K1[0] + K1[1] * K1[1] + K1[2] * K1[2] + kDilation;
            const double det = v00 * v11 - v01 * v01;
            const double id2 = 1.0 / (det * det);
            const double gmx = acc[A_MX], gmy = acc[A_MY];
            const double gca = acc[A_CA], gcb = acc[A_CB], gcc = acc[A_CC];
            gop = acc[A_OP];
            // conic (a, b, c) = (v11, -v01, v00) / det  ->  Vhat
            const double dv00 = (-gca * v11 * v11 + gcb * v01 * v11 - gcc * v01 * v01) * id2;
            const double dv11 = (-gca * v01 * v01 + gcb * v01 * v00 - gcc * v00 * v00) * id2;
            const double dv01 = (2.0 * gca * v11 * v01 - gcb * (det + 2.0 * v01 * v01) + 2.0 * gcc * v00 * v01) * id2;
            double dR[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            double dT0[3] = {0, 0, 0}, dT1[3] = {0, 0, 0};
            for (int c = 0; c < 3; ++c) {
                const double dK0 = 2.0 * dv00 * K0[c] + dv01 * K1[c];
                const double dK1 = 2.0 * dv11 * K1[c] + dv01 * K0[c];
                ds[c] += dK0 * TR0[c] + dK1 * TR1[c];
                const double dTR0 = dK0 * s[c], dTR1 = dK1 * s[c];
                for (int m = 0; m < 3; ++m) {
                    dR[3 * m + c] += T0[m] * dTR0 + T1[m] * dTR1;
                    dT0[m] += dTR0 * R[3 * m + c];
                    dT1[m] += dTR1 * R[3 * m + c];
                }
            }
            double dj00 = 0, dj02 = 0, dj11 = 0, dj12 = 0;
            for (int m = 0; m < 3; ++m) {
                dj00 += dT0[m] * Rc[m];
                dj02 += dT0[m] * Rc[6 + m];
                dj11 += dT1[m] * Rc[3 + m];
                dj12 += dT1[m] * Rc[6 + m];
            }
            double dt[3] = {0, 0, 0};
            dt[2] += -cam.fx * iz * iz * dj00 - cam.fy * iz * iz * dj11;
            if (ux) {
                dt[0] += -cam.fx * iz * iz * dj02;
                dt[2] += 2.0 * cam.fx * t[0] * iz * iz * iz * dj02;
            } else {
                dt[2] += cam.fx * u * iz * iz * dj02;
            }
            if (vy) {
                dt[1] += -cam.fy * iz * iz * dj12;
                dt[2] += 2.0 * cam.fy * t[1] * iz * iz * iz * dj12;
            } else {
                dt[2] += cam.fy * v * iz * iz * dj12;
            }
            // projected centre
            dt[0] += gmx * cam.fx * iz;
            dt[2] -= gmx * cam.fx * t[0] * iz * iz;
            dt[1] += gmy * cam.fy * iz;
            dt[2] -= gmy * cam.fy * t[1] * iz * iz;

            // colour
            const double dvec[3] = {mu[0] - cam.e[0], mu[1] - cam.e[1], mu[2] - cam.e[2]};
            const double dlen = sqrt(dvec[0] * dvec[0] + dvec[1] * dvec[1] + dvec[2] * dvec[2]);
            const double idlen = 1.0 / dlen;
            const double dir[3] = {dvec[0] * idlen, dvec[1] * idlen, dvec[2] * idlen};
            // every coefficient is loaded before the first is used
            float shc[3 * ncoef];
            if constexpr (kShMode == kShCoeffMajor) {
#pragma unroll
                for (int k = 0; k < ncoef; ++k)
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) shc[3 * k + ch] = g.sh[((int64_t)k * 3 + ch) * n + i];
            } else {
                load_sh<ncoef, kShMode>(g, i, shc);
            }
            double Y[16], dY[16];
            sh_values(DEG, dir[0], dir[1], dir[2], Y);
            if constexpr (kShMode == kShCoeffMajor) {
#pragma unroll
                for (int k = 0; k < ncoef; ++k) dY[k] = 0.0;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    const double gcol = acc[A_R + ch];
                    double raw = 0.5;
#pragma unroll
                    for (int k = 0; k < ncoef; ++k) raw += Y[k] * (double)shc[3 * k + ch];
                    const bool pass = raw >= 0.0;   // the clamp max(0, raw colour)
#pragma unroll
                    for (int k = 0; k < ncoef; ++k) {
                        out.sh[((int64_t)k * 3 + ch) * n + i] = pass ? (float)(gcol * Y[k]) : 0.0f;
                        dY[k] += pass ? gcol * (double)shc[3 * k + ch] : 0.0;
                    }
                }
            } else {
                // the same sums in the same order, each row entry (or group of
                // four) stored as soon as it is complete
                bool pass[3];
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    double raw = 0.5;
#pragma unroll
                    for (int k = 0; k < ncoef; ++k) raw += Y[k] * (double)shc[3 * k + ch];
                    pass[ch] = raw >= 0.0;
                }
                float q4v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                float* row = out.sh + i * (3 * ncoef);
#pragma unroll
                for (int j = 0; j < 3 * ncoef; ++j) {
                    const int k = j / 3, ch = j % 3;
                    if (ch == 0) dY[k] = 0.0;
                    const double gcol = acc[A_R + ch];
                    const float gv = pass[ch] ? (float)(gcol * Y[k]) : 0.0f;
                    dY[k] += pass[ch] ? gcol * (double)shc[j] : 0.0;
                    if constexpr (kShMode == kShRow) {
                        row[j] = gv;
                    } else {
                        q4v[j & 3] = gv;
                        if ((j & 3) == 3)
                            reinterpret_cast<float4*>(row)[j >> 2] = make_float4(q4v[0], q4v[1], q4v[2], q4v[3]);
                    }
                }
            }
            double ddir[3];
            sh_backward(DEG, dir[0], dir[1], dir[2], dY, ddir);
            const double dd = ddir[0] * dir[0] + ddir[1] * dir[1] + ddir[2] * dir[2];
            for (int a = 0; a < 3; ++a) dmu[a] += (ddir[a] - dir[a] * dd) * idlen;

            // whitened ray set-up of CUTOFF Gaussians
            if (cutg) {
                double gd0[3], ggx[3], ggy[3];
                for (int a = 0; a < 3; ++a) {
                    gd0[a] = acc[A_D0 + a];
                    ggx[a] = acc[A_GX + a];
                    ggy[a] = acc[A_GY + a];
                }
                const double gz = acc[A_Z], gdep = acc[A_DEP], gg0 = acc[A_G0];
                const double v0[3] = {dvec[0] * iz, dvec[1] * iz, dvec[2] * iz};
                const double ifx = 1.0 / cam.fx, ify = 1.0 / cam.fy;
                double dv0[3] = {pl.n[0] * gg0, pl.n[1] * gg0, pl.n[2] * gg0};
                for (int a = 0; a < 3; ++a) {
                    const double ia = 1.0 / s[a];
                    double dsa = 0.0;
                    for (int b2 = 0; b2 < 3; ++b2) {
                        const double mab = R[3 * b2 + a] * ia;   // M^-1[a][b] = R[b][a] / s[a]
                        const double dM = gd0[a] * v0[b2] + ggx[a] * Rc[b2] * ifx + ggy[a] * Rc[3 + b2] * ify;
                        dv0[b2] += mab * gd0[a];
                        dR[3 * b2 + a] += dM * ia;
                        dsa -= dM * mab * ia;
                    }
                    ds[a] += dsa;
                }
                dt[2] += gz;
                for (int a = 0; a < 3; ++a) {
                    dmu[a] += pl.n[a] * gdep + dv0[a] * iz;
                    pn[a] += mu[a] * gdep + v0[a] * gg0;
                }
                pn[3] += gdep;
                dt[2] -= (dvec[0] * dv0[0] + dvec[1] * dv0[1] + dvec[2] * dv0[2]) * iz * iz;
            }
            // t = R_c mu + t_c
            for (int a = 0; a < 3; ++a) dmu[a] += Rc[a] * dt[0] + Rc[3 + a] * dt[1] + Rc[6 + a] * dt[2];
            // R(q_hat) -> q_hat -> q
            const double r_ = qw, x = qx, y = qy, zq = qz;
            double dq[4];
            dq[0] = -2 * zq * dR[1] + 2 * y * dR[2] + 2 * zq * dR[3] - 2 * x * dR[5] - 2 * y * dR[6] + 2 * x * dR[7];
            dq[1] = 2 * y * dR[1] + 2 * zq * dR[2] + 2 * y * dR[3] - 4 * x * dR[4] - 2 * r_ * dR[5] + 2 * zq * dR[6] +
                    2 * r_ * dR[7] - 4 * x * dR[8];
            dq[2] = -4 * y * dR[0] + 2 * x * dR[1] + 2 * r_ * dR[2] + 2 * x * dR[3] + 2 * zq * dR[5] - 2 * r_ * dR[6] +
                    2 * zq * dR[7] - 4 * y * dR[8];
            dq[3] = -4 * zq * dR[0] - 2 * r_ * dR[1] + 2 * x * dR[2] + 2 * r_ * dR[3] - 4 * zq * dR[4] + 2 * y * dR[5] +
                    2 * x * dR[6] + 2 * y * dR[7];
            const double qn[4] = {qw, qx, qy, qz};
            const double dot = dq[0] * qn[0] + dq[1] * qn[1] + dq[2] * qn[2] + dq[3] * qn[3];
            for (int k = 0; k < 4; ++k) dqv[k] = (dq[k] - qn[k] * dot) * iqlen;
        } else {
            // (loops, not unrolled: unrolled, their addresses are computed once
            // for both branches and held in registers across the drawn one)
            if constexpr (kShMode == kShCoeffMajor) {
#pragma unroll 1
                for (int j = 0; j < 3 * ncoef; ++j) out.sh[(int64_t)j * n + i] = 0.0f;
            } else if constexpr (kShMode == kShRow) {
#pragma unroll 1
                for (int j = 0; j < 3 * ncoef; ++j) out.sh[i * (3 * ncoef) + j] = 0.0f;
            } else {
#pragma unroll 1
                for (int j = 0; j < 3 * ncoef / 4; ++j)
                    reinterpret_cast<float4*>(out.sh + i * (3 * ncoef))[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
        }
        for (int a = 0; a < 3; ++a) {
            out.mean[a * n + i] = (float)dmu[a];
            out.scale[a * n + i] = (float)ds[a];
        }
        for (int k = 0; k < 4; ++k) out.quat[k * n + i] = (float)dqv[k];
        out.opacity[i] = (float)gop;
    }
    // plane terms: block sum, one atomic per block and component
    __shared__ float red[4][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = 0; k < 4; ++k) {
        const float s = wave_sum((float)pn[k]);
        if (lane == 0) red[k][wave] = s;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const float s = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
        if (s != 0.0f) atomicAdd(plane_acc + threadIdx.x, s);
    }
}

// raw plane gradient: n_hat = n / |n|, d_hat = d / |n|; the pixel-rate terms
// (ax, ay) = (R_c n_hat)_{x,y} / f_{x,y}.
__global__ void plane_finalize_kernel(CamParams cam, PlaneParams pl, double len, const float* __restrict__ plane_acc,
                                      const int32_t* __restrict__ overflow, float* __restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (!pl.enabled || *overflow) {
        out[0] = out[1] = out[2] = out[3] = 0.0f;
        return;
    }
    double dn[3];
    for (int a = 0; a < 3; ++a)
        dn[a] = plane_acc[a] + cam.R[a] * plane_acc[4] / cam.fx + cam.R[3 + a] * plane_acc[5] / cam.fy;
    const double dd = plane_acc[3];
    const double dot = dn[0] * pl.n[0] + dn[1] * pl.n[1] + dn[2] * pl.n[2];
    for (int a = 0; a < 3; ++a) out[a] = (float)((dn[a] - pl.n[a] * dot - pl.n[a] * pl.d * dd) / len);
    out[3] = (float)(dd / len);
}

}  // namespace

// workspace: pair slots [pair_capacity][kAccRows] float, the plane
// accumulators (256 B), per-Gaussian slot sums [kAccRows][n] double
size_t backward_workspace_bytes(int64_t n, int64_t pair_capacity, int32_t width, int32_t height)
{
    (void)width;
    (void)height;
    const size_t slot_bytes = ((size_t)kAccRows * (size_t)(pair_capacity > 0 ? pair_capacity : 1) * 4 + 255) &
                              ~size_t(255);
    return slot_bytes + 256 + (size_t)kAccRows * (size_t)(n > 0 ? n : 1) * 8;
}

hipError_t launch_backward(const GaussPtrs& g, const CamParams& cam, const PlaneParams& pl, double plane_len,
                           const ProjPtrs& proj, const rara_binned& bins, int64_t pair_capacity,
                           const RenderParams& rp, const float* final_T, const uint32_t* n_contrib,
                           const float* dL_dimage, const rara_grads& grads, void* workspace, hipStream_t s)
{
    float* slots = static_cast<float*>(workspace);
    const size_t slot_bytes = ((size_t)kAccRows * (size_t)(pair_capacity > 0 ? pair_capacity : 1) * 4 + 255) &
                              ~size_t(255);
    float* plane_acc = reinterpret_cast<float*>(static_cast<char*>(workspace) + slot_bytes);
    double* sums = reinterpret_cast<double*>(static_cast<char*>(workspace) + slot_bytes + 256);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(1), dim3(256), 0, s, plane_acc, (int64_t)kPlaneAcc);
    BackParams bp{rp, g.n};
    if (g.n > 0)
        hipLaunchKernelGGL(blend_backward_kernel, dim3((unsigned)tiles_grid(rp.num_tiles)), dim3(256), 0, s,
                           proj.splat, proj.ray, bins.vals, reinterpret_cast<const uint2*>(bins.ranges), bins.work,
                           bins.pair_start, proj.tile_rec, bins.overflow, bp, final_T, n_contrib,
                           dL_dimage, slots, plane_acc);
    if (g.n > 0) {
        const dim3 grid((unsigned)((g.n + 255) / 256));
        hipLaunchKernelGGL(slot_sum_kernel, grid, dim3(256), 0, s, g.n, pl.enabled, proj.label, proj.tiles_touched,
                           bins.pair_start, bins.overflow, slots, sums);
        GradPtrs gp{grads.mean, grads.scale, grads.quat, grads.opacity, grads.sh};
        const int mode = sh_mode(g.sh_layout, g.sh_degree, g.sh, grads.sh);
#define RARA_PB(D, M)                                                                                        \
    hipLaunchKernelGGL((project_backward_kernel<D, M>), grid, dim3(256), 0, s, g, cam, pl, proj.label,        \
                       proj.tiles_touched, bins.overflow, sums, gp, plane_acc)
        switch (g.sh_degree) {
        case 0: if (mode == kShCoeffMajor) RARA_PB(0, kShCoeffMajor); else RARA_PB(0, kShRow); break;
        case 1:
            if (mode == kShCoeffMajor) RARA_PB(1, kShCoeffMajor);
            else if (mode == kShRow) RARA_PB(1, kShRow);
            else RARA_PB(1, kShRow16);
            break;
        case 2: if (mode == kShCoeffMajor) RARA_PB(2, kShCoeffMajor); else RARA_PB(2, kShRow); break;
        default:
            if (mode == kShCoeffMajor) RARA_PB(3, kShCoeffMajor);
            else if (mode == kShRow) RARA_PB(3, kShRow);
            else RARA_PB(3, kShRow16);
            break;
        }
#undef RARA_PB
    }
    hipLaunchKernelGGL(plane_finalize_kernel, dim3(1), dim3(64), 0, s, cam, pl, plane_len, plane_acc, bins.overflow,
                       grads.plane);
    return hipGetLastError();
}

}  // namespace rara
