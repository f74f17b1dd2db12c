// Per-Gaussian stage: classification against the clipping plane (Sec. 3.2,
// Algorithm 1 step 1), EWA projection of the 3D covariance (Sec. 3.4,
// eqs. 9-10), footprint and tile rectangle, spherical-harmonic colour, and the
// whitened-space ray set-up used by the blend for CUTOFF Gaussians (eq. 4).
//
// One thread per Gaussian.  Loads are structure-of-arrays and coalesced; the
// geometry is evaluated in FP64 (full-rate vector FP64 on gfx950 costs nothing
// in an HBM-bound kernel) so that labels, footprints and depths round the same
// way as a double-precision definition would.  INVISIBLE Gaussians stop after
// reading mean and scale.
#include "rara_internal.h"

namespace rara {

namespace {

// Real spherical harmonics, degree <= 3, alternating-sign convention of the
// splatting colour model; constants are sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)-type
// normalisations evaluated to double precision.
__device__ inline void sh_eval(int deg, double x, double y, double z, double* Y)
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

// What the listed-tile test needs of a drawn Gaussian (area 0: not drawn).
struct Footprint {
    double mx, my;
    float ca, cb, cc, op;
    int tx0, ty0, w, area;
};

// kDeg: the SH degree, fixed per launch so that every coefficient load of a
// Gaussian is issued before the first one is used.  Writes every output but
// tiles_touched and tile_rec, which the listed-tile pass writes.
template <int kDeg, int kShMode>
__device__ __forceinline__ Footprint preprocess_one(const GaussPtrs& g, const CamParams& cam, const PlaneParams& pl,
                                                    const ProjPtrs& out, int64_t i)
{
    Footprint fp{};
    const int64_t n = g.n;

    // every per-Gaussian input but the SH is loaded here, once: the output
    // stores come last, so no load waits behind a store that may alias it
    const double mu[3] = {g.mean[i], g.mean[n + i], g.mean[2 * n + i]};
    const double s[3] = {g.scale[i], g.scale[n + i], g.scale[2 * n + i]};
    const float qf[4] = {g.quat[i], g.quat[n + i], g.quat[2 * n + i], g.quat[3 * n + i]};
    const float opf = g.opacity[i];

    // Sec. 3.2: d_ep = n.mu + d, r = 3 max(sigma); hard clipping keeps a
    // Gaussian by its centre's side; the tight variant takes r = 3 |S R^T n|.
    // A region (count > 1 half-spaces): INVISIBLE beyond r outside any plane,
    // VISIBLE beyond r inside every plane; hard clipping keeps a centre
    // inside every half-space.
    uint8_t label = RARA_LABEL_VISIBLE;
    double dep = 0.0;
    // for a CUTOFF Gaussian: the planes whose visible side does not hold its
    // whole 3-sigma ellipsoid (d_k <= the ellipsoid's half-width along n_k)
    uint32_t cuts = 0u;
    if (pl.enabled) {
        dep = pl.n[0] * mu[0] + pl.n[1] * mu[1] + pl.n[2] * mu[2] + pl.d;
        if ((pl.enabled & 3) == RARA_CLIP_HARD) {
            bool behind = dep < 0.0;
            for (int k = 1; k < pl.count; ++k) {
                const double* xn = pl.xn[k - 1];
                behind = behind || xn[0] * mu[0] + xn[1] * mu[1] + xn[2] * mu[2] + pl.xd[k - 1] < 0.0;
            }
            label = behind ? RARA_LABEL_INVISIBLE : RARA_LABEL_VISIBLE;
        } else {
            const bool tight = (pl.enabled & RARA_CLIP_TIGHT) != 0;
            double qw = qf[0], qx = qf[1], qy = qf[2], qz = qf[3];
            const double ql = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
            qw /= ql; qx /= ql; qy /= ql; qz /= ql;
            // 3 |S R^T n|: the half-width of the 3-sigma ellipsoid along n
            auto support = [&](const double* nn) {
                // (S R^T n)_a = sigma_a (column a of R) . n
                const double c0 = s[0] * ((1 - 2 * (qy * qy + qz * qz)) * nn[0] + 2 * (qx * qy + qw * qz) * nn[1] +
                                          2 * (qx * qz - qw * qy) * nn[2]);
                const double c1 = s[1] * (2 * (qx * qy - qw * qz) * nn[0] + (1 - 2 * (qx * qx + qz * qz)) * nn[1] +
                                          2 * (qy * qz + qw * qx) * nn[2]);
                const double c2 = s[2] * (2 * (qx * qz + qw * qy) * nn[0] + 2 * (qy * qz - qw * qx) * nn[1] +
                                          (1 - 2 * (qx * qx + qy * qy)) * nn[2]);
                return 3.0 * sqrt(c0 * c0 + c1 * c1 + c2 * c2);
            };
            const double rmax = 3.0 * fmax(fmax(s[0], s[1]), s[2]);
            const double st0 = support(pl.n);
            const double r = tight ? st0 : rmax;
            bool outside = dep < -r, inside = dep > r;
            // the planes that cut into, or hold outside, the 3-sigma ellipsoid
            // itself (the label takes the 3 max(sigma) ball unless the tight
            // flag is set)
            cuts = dep <= st0 ? 1u : 0u;
            for (int k = 1; k < pl.count; ++k) {
                const double* xn = pl.xn[k - 1];
                const double dk = xn[0] * mu[0] + xn[1] * mu[1] + xn[2] * mu[2] + pl.xd[k - 1];
                const double sk = support(xn);
                const double rk = tight ? sk : rmax;
                outside = outside || dk < -rk;
                inside = inside && dk > rk;
                cuts |= dk <= sk ? (1u << k) : 0u;
            }
            label = outside ? RARA_LABEL_INVISIBLE : (inside ? RARA_LABEL_VISIBLE : RARA_LABEL_CUTOFF);
        }
    }
    uint32_t touched = 0;

    if (label != RARA_LABEL_INVISIBLE) {
        const double tz = cam.R[6] * mu[0] + cam.R[7] * mu[1] + cam.R[8] * mu[2] + cam.t[2];
        if (tz > cam.near_z) {
            const double tx = cam.R[0] * mu[0] + cam.R[1] * mu[1] + cam.R[2] * mu[2] + cam.t[0];
            const double ty = cam.R[3] * mu[0] + cam.R[4] * mu[1] + cam.R[5] * mu[2] + cam.t[1];
            // the SH loads are issued here, so that they are in flight during
            // the projection (a Gaussian culled by its footprint wastes them)
            constexpr int ncoef = (kDeg + 1) * (kDeg + 1);
            float shv[3 * ncoef];
            load_sh<ncoef, kShMode>(g, i, shv);
            // rotation of the normalised quaternion (w, x, y, z)
            double qw = qf[0], qx = qf[1], qy = qf[2], qz = qf[3];
            const double qs = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
            qw *= qs; qx *= qs; qy *= qs; qz *= qs;
            const double R[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
                                 2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
                                 2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
            // Jacobian of the pinhole map at the guard-band-clamped point
            const double iz = 1.0 / tz;
            const double u = fmin(cam.limx, fmax(-cam.limx, tx * iz));
            const double v = fmin(cam.limy, fmax(-cam.limy, ty * iz));
            const double j00 = cam.fx * iz, j02 = -cam.fx * u * iz;
            const double j11 = cam.fy * iz, j12 = -cam.fy * v * iz;
            // T = J R_c (2x3), K = T R S (2x3), Vhat = K K^T + dilation
            double T0[3], T1[3];
            for (int c = 0; c < 3; ++c) {
                T0[c] = j00 * cam.R[c] + j02 * cam.R[6 + c];
                T1[c] = j11 * cam.R[3 + c] + j12 * cam.R[6 + c];
            }
            double K0[3], K1[3];
            for (int c = 0; c < 3; ++c) {
                K0[c] = (T0[0] * R[c] + T0[1] * R[3 + c] + T0[2] * R[6 + c]) * s[c];
                K1[c] = (T1[0] * R[c] + T1[1] * R[3 + c] + T1[2] * R[6 + c]) * s[c];
            }
            const double c00 = K0[0] * K0[0] + K0[1] * K0[1] + K0[2] * K0[2] + kDilation;
            const double c01 = K0[0] * K1[0] + K0[1] * K1[1] + K0[2] * K1[2];
            const double c11 = K1[0] * K1[0] + K1[1] * K1[1] + K1[2] * K1[2] + kDilation;
            const double det = c00 * c11 - c01 * c01;
            if (det > 0.0) {
                const double mx = cam.fx * tx * iz + cam.cx;
                const double my = cam.fy * ty * iz + cam.cy;
                const double half = 0.5 * (c00 - c11);
                const double lmax = 0.5 * (c00 + c11) + sqrt(half * half + c01 * c01);
                const double rad = ceil(3.0 * sqrt(lmax));
                const double x0 = fmax(0.0, ceil(mx - rad)), x1 = fmin((double)(cam.W - 1), floor(mx + rad));
                const double y0 = fmax(0.0, ceil(my - rad)), y1 = fmin((double)(cam.H - 1), floor(my + rad));
                if (x0 <= x1 && y0 <= y1) {
                    const int tx0 = (int)x0 >> 4, tx1 = ((int)x1 >> 4) + 1;
                    const int ty0 = (int)y0 >> 4, ty1 = ((int)y1 >> 4) + 1;
                    touched = (uint32_t)((tx1 - tx0) * (ty1 - ty0));
                    fp.tx0 = tx0;
                    fp.ty0 = ty0;
                    fp.w = tx1 - tx0;
                    fp.area = (int)touched;

                    // colour: SH in the direction from the camera centre to mu
                    double dir[3] = {mu[0] - cam.e[0], mu[1] - cam.e[1], mu[2] - cam.e[2]};
                    const double dl = 1.0 / sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
                    double Y[16];
                    sh_eval(kDeg, dir[0] * dl, dir[1] * dl, dir[2] * dl, Y);
                    double rgb[3] = {0.5, 0.5, 0.5};
#pragma unroll
                    for (int k = 0; k < ncoef; ++k)
                        for (int c = 0; c < 3; ++c) rgb[c] += Y[k] * (double)shv[3 * k + c];

                    const double idet = 1.0 / det;
                    Splat sp;
                    sp.mx = mx;
                    sp.my = my;
                    sp.ca = (float)(c11 * idet);
                    sp.cb = (float)(-c01 * idet);
                    sp.cc = (float)(c00 * idet);
                    sp.op = opf;
                    sp.r = (float)fmax(0.0, rgb[0]);
                    sp.g = (float)fmax(0.0, rgb[1]);
                    sp.b = (float)fmax(0.0, rgb[2]);
                    // bits 16.. of the record's label word: the planes that do
                    // not hold a CUTOFF Gaussian's ellipsoid inside (see staged_word)
                    sp.label = label | (label == RARA_LABEL_CUTOFF ? cuts << 16 : 0u);
                    out.splat[i] = sp;
                    fp.mx = mx;
                    fp.my = my;
                    fp.ca = sp.ca;
                    fp.cb = sp.cb;
                    fp.cc = sp.cc;
                    fp.op = opf;
                    out.depth[i] = (float)tz;

                    if (label == RARA_LABEL_CUTOFF) {
                        // M^-1 = S^-1 R^T: row a is column a of R divided by sigma_a
                        const double v0[3] = {(mu[0] - cam.e[0]) * iz, (mu[1] - cam.e[1]) * iz,
                                              (mu[2] - cam.e[2]) * iz};
                        RayRec rr;
                        for (int a = 0; a < 3; ++a) {
                            const double ia = 1.0 / s[a];
                            const double m0 = R[a] * ia, m1 = R[3 + a] * ia, m2 = R[6 + a] * ia;
                            rr.d0[a] = (float)(m0 * v0[0] + m1 * v0[1] + m2 * v0[2]);
                            rr.gx[a] = (float)((m0 * cam.R[0] + m1 * cam.R[1] + m2 * cam.R[2]) / cam.fx);
                            rr.gy[a] = (float)((m0 * cam.R[3] + m1 * cam.R[4] + m2 * cam.R[5]) / cam.fy);
                        }
                        rr.z = (float)tz;
                        rr.dep = (float)dep;
                        rr.g0 = (float)(pl.n[0] * v0[0] + pl.n[1] * v0[1] + pl.n[2] * v0[2]);
                        out.ray[i] = rr;
                        // a region's further planes: (d_ep, g0) of each
                        for (int k = 1; k < pl.count; ++k) {
                            const double* xn = pl.xn[k - 1];
                            const double dk = xn[0] * mu[0] + xn[1] * mu[1] + xn[2] * mu[2] + pl.xd[k - 1];
                            out.ray_ext[i * (kMaxPlanes - 1) + (k - 1)] =
                                make_float2((float)dk, (float)(xn[0] * v0[0] + xn[1] * v0[1] + xn[2] * v0[2]));
                        }
                    }
                }
            }
        }
    }
    out.label[i] = label;
    (void)touched;
    return fp;
}

constexpr int kPreThreads = 256;

// The 16-byte tile record of a Gaussian: its rectangle (as in rect; zero when
// not drawn) and its listed-tile mask, so that one gather fetches both.
__device__ inline ulonglong2 tile_record(const Footprint& f, uint64_t mask)
{
    const uint64_t r = f.area > 0 ? ((uint64_t)(uint16_t)f.tx0 | (uint64_t)(uint16_t)f.ty0 << 16 |
                                     (uint64_t)(uint16_t)(f.tx0 + f.w) << 32 |
                                     (uint64_t)(uint16_t)(f.ty0 + f.area / f.w) << 48)
                                  : 0ull;
    return make_ulonglong2(r, mask);
}

// Minimum of q = A x^2 + 2 B x y + C y^2 (a positive definite form, relative
// to the centre) along the edge x = X, y in [y0, y1]: q at the edge's
// stationary point -B X / C (iC = 1/C) clamped to the edge.  Every operation is
// rounded on its own (no fused multiply-add), so the result does not depend on
// where the compiler inlines it; the products are those of A X X + 2 B X y +
// C y y taken left to right (B2 = 2 B is exact), and fmin(fmax(.)) equals the
// compare form of the clamp for y0 <= y1.
__device__ inline double edge_x_min(double A, double B, double B2, double C, double iC, double X, double y0, double y1)
{
#pragma clang fp contract(off)
    const double y = fmin(fmax(-B * X * iC, y0), y1);   // stationary point of q along x = X, clamped
    return A * X * X + B2 * X * y + C * y * y;
}

// The same along the edge y = Y, x in [x0, x1], stationary at -B Y / A (iA = 1/A).
__device__ inline double edge_y_min(double A, double B, double B2, double C, double iA, double Y, double x0, double x1)
{
#pragma clang fp contract(off)
    const double x = fmin(fmax(-B * Y * iA, x0), x1);   // stationary point of q along y = Y, clamped
    return A * x * x + B2 * x * Y + C * Y * Y;
}

// FP64 minimum of q over the box [x0, x1] x [y0, y1]: zero when the box holds
// the centre.  Otherwise the minimum of the convex q lies on the boundary, and
// only the edges that face the centre can hold it: at a minimum
// inside the far edge x = X (X > 0 with the box right of the centre), dq/dy = 0
// puts the point at y = -B X / C, where dq/dx = 2 X det / C > 0 would let q fall
// into the box; a corner belongs to a facing edge too.  So the vertical edge
// nearer the centre (when the centre is outside [x0, x1]) and the horizontal
// one likewise are evaluated, and the other two cannot be lower.
__device__ inline double box_min_fp64(double A, double B, double B2, double C, double iA, double iC, double x0,
                                      double x1, double y0, double y1)
{
    const bool fx = x0 > 0.0 || x1 < 0.0, fy = y0 > 0.0 || y1 < 0.0;
    if (!fx && !fy) return 0.0;   // the box holds the centre
    const double ex = edge_x_min(A, B, B2, C, iC, x0 > 0.0 ? x0 : x1, y0, y1);
    const double ey = edge_y_min(A, B, B2, C, iA, y0 > 0.0 ? y0 : y1, x0, x1);
    return fmin(fx ? ex : INFINITY, fy ? ey : INFINITY);
}

// Whether a Gaussian reaches tile (tx, ty): the box of the tile's pixel
// centres, clipped to the W x H image and taken relative to the centre
// (mx, my), against the threshold t.
__device__ inline bool reaches_tile(double mx, double my, double A, double B, double C, double iA, double iC,
                                    double t, int tx, int ty, int W, int H)
{
    double x0, x1, y0, y1;
    {
#pragma clang fp contract(off)
        x0 = (double)(tx * kTile) - mx;
        x1 = fmin((double)(tx * kTile + kTile - 1), (double)(W - 1)) - mx;
        y0 = (double)(ty * kTile) - my;
        y1 = fmin((double)(ty * kTile + kTile - 1), (double)(H - 1)) - my;
    }
    return box_min_fp64(A, B, 2.0 * B, C, iA, iC, x0, x1, y0, y1) <= t;
}

// Row of tile li in a rectangle w tiles wide (li < 64, w <= 64): (li + 1/2) / w
// lies at least 1/128 from an integer, so the float product floors exactly.
__device__ inline int rect_row(uint32_t li, int w)
{
    return (int)(((float)li + 0.5f) * __builtin_amdgcn_rcpf((float)w));
}

constexpr uint32_t kOwnTests = 4;   // tiles each lane tests itself

// Exclusive prefix of v (below 128) over the wave, from one ballot per bit.
__device__ inline uint32_t wave_prefix7(uint32_t v, uint32_t& total)
{
    uint32_t pre = 0u, tot = 0u;
#pragma unroll
    for (int b = 0; b < 7; ++b) {
        const uint64_t m = __ballot((v >> b) & 1u);
        pre += __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u)) << b;
        tot += (uint32_t)__popcll(m) << b;
    }
    total = tot;
    return pre;
}

// Listed tiles of every lane's Gaussian (every lane of the wave calls this):
// for a drawn Gaussian whose rectangle has at most kMaskTiles tiles, bit k of
// mask is set when its k-th tile (row by row) has a pixel-centre box on which
// the float32 conic's quadratic form reaches 1.02 * 2 ln(255 delta) + 0.02 or
// less; touched is the number of listed tiles (the whole rectangle when it is
// larger).  Each lane tests the first kOwnTests tiles of its own rectangle
// (most rectangles have no more); the rest of the wave's (Gaussian, tile)
// tests are dealt over the lanes, two per lane and step, so that one large
// rectangle does not hold up the wave: the lane of test e finds its Gaussian
// by a binary search over the wave's inclusive test counts in LDS and ORs the
// tile's bit into that Gaussian's LDS mask.
__device__ inline void listed_tiles(const Footprint& f, int W, int H, uint64_t& mask, uint32_t& touched)
{
    __shared__ double s_g[kPreThreads][8];   // mx, my, A, B, C, 1/A, 1/C, threshold
    __shared__ int s_r[kPreThreads][4];      // tx0, ty0, w, inclusive end of the wave's shared tests
    __shared__ unsigned long long s_m[kPreThreads];
    const int tid = threadIdx.x, lane = tid & 63, wb = tid & ~63;
    mask = 0ull;
    touched = (uint32_t)f.area;
    bool tested = false;
    uint32_t shared = 0u;   // tests past the lane's own ones
    if (f.area > 0 && f.area <= kMaskTiles) {
        const double A = (double)f.ca, B = (double)f.cb, C = (double)f.cc;
        const double s255 = 255.0 * (double)f.op;
        touched = 0u;
        if (s255 > 1.0) {
            bool pd;
            {
#pragma clang fp contract(off)
                pd = A * C - B * B > 0.0;
            }
            if (!pd) {
                mask = f.area == 64 ? ~0ull : ((1ull << f.area) - 1ull);
                touched = (uint32_t)f.area;
            } else {
                tested = true;
                double t;
                {
#pragma clang fp contract(off)
                    t = 2.0 * log(s255) * 1.02 + 0.02;
                }
                const double iA = 1.0 / A, iC = 1.0 / C;
                const uint32_t own = (uint32_t)f.area < kOwnTests ? (uint32_t)f.area : kOwnTests;
                int col = 0, row = 0;
                for (uint32_t li = 0; li < own; ++li) {
                    if (reaches_tile(f.mx, f.my, A, B, C, iA, iC, t, f.tx0 + col, f.ty0 + row, W, H))
                        mask |= 1ull << li;
                    if (++col == f.w) {
                        col = 0;
                        ++row;
                    }
                }
                shared = (uint32_t)f.area - own;
                if (shared) {
                    s_g[tid][0] = f.mx;
                    s_g[tid][1] = f.my;
                    s_g[tid][2] = A;
                    s_g[tid][3] = B;
                    s_g[tid][4] = C;
                    s_g[tid][5] = iA;
                    s_g[tid][6] = iC;
                    s_g[tid][7] = t;
                    s_r[tid][0] = f.tx0;
                    s_r[tid][1] = f.ty0;
                    s_r[tid][2] = f.w;
                }
            }
        }
    }
    uint32_t total;
    const uint32_t incl = wave_prefix7(shared, total) + shared;   // shared <= 60
    if (total != 0u) {   // uniform over the wave
        s_r[tid][3] = (int)incl;
        s_m[tid] = 0ull;
        // every LDS entry a wave reads below belongs to the wave itself: a
        // wavefront-scope fence orders its lanes' writes before their reads
        wave_sync();
        // shared test e of the wave: its Gaussian's lane (the first lane whose
        // inclusive end exceeds e) and tile li of that Gaussian's rectangle
        auto test = [&](uint32_t e, int& o, uint32_t& li) {
            int own = 0;
#pragma unroll
            for (int step = 32; step > 0; step >>= 1)
                if ((uint32_t)s_r[wb + own + step - 1][3] <= e) own += step;
            o = wb + own;
            li = kOwnTests + e - (own ? (uint32_t)s_r[o - 1][3] : 0u);
            const int w = s_r[o][2];
            const int row = rect_row(li, w), col = (int)li - row * w;
            return reaches_tile(s_g[o][0], s_g[o][1], s_g[o][2], s_g[o][3], s_g[o][4], s_g[o][5], s_g[o][6],
                                s_g[o][7], s_r[o][0] + col, s_r[o][1] + row, W, H);
        };
        // two tests per lane and step (e and e + 64): independent chains of
        // LDS reads that overlap
        for (uint32_t e0 = 0; e0 < total; e0 += 128) {
            const uint32_t ea = e0 + (uint32_t)lane, eb = ea + 64u;
            const uint32_t ca = ea < total ? ea : total - 1u, cb = eb < total ? eb : total - 1u;
            int oa, ob;
            uint32_t la, lb;
            const bool ha = test(ca, oa, la) && ea < total;
            const bool hb = test(cb, ob, lb) && eb < total;
            if (ha) atomicOr(&s_m[oa], 1ull << la);
            if (hb) atomicOr(&s_m[ob], 1ull << lb);
        }
        wave_sync();
        if (shared) mask |= s_m[tid];
    }
    if (tested) touched = (uint32_t)__popcll(mask);
}

template <int kDeg, int kShMode>
__global__ __launch_bounds__(kPreThreads) void preprocess_kernel(GaussPtrs g, CamParams cam, PlaneParams pl,
                                                                 ProjPtrs out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    Footprint fp{};
    if (i < g.n) fp = preprocess_one<kDeg, kShMode>(g, cam, pl, out, i);
    uint64_t mask;
    uint32_t touched;
    listed_tiles(fp, cam.W, cam.H, mask, touched);
    if (i < g.n) {
        out.tiles_touched[i] = touched;
        out.tile_rec[i] = tile_record(fp, mask);
    }
}

// Frame-graph variant: camera and plane read from device memory.
template <int kDeg, int kShMode>
__global__ __launch_bounds__(kPreThreads) void preprocess_fp_kernel(GaussPtrs g, const FrameParams* __restrict__ fp,
                                                                    ProjPtrs out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // read through the pointer: a private copy of the plane arrays, indexed
    // by the plane number, would live in scratch memory
    Footprint f{};
    if (i < g.n) f = preprocess_one<kDeg, kShMode>(g, fp->cam, fp->plane, out, i);
    uint64_t mask;
    uint32_t touched;
    listed_tiles(f, fp->cam.W, fp->cam.H, mask, touched);
    if (i < g.n) {
        out.tiles_touched[i] = touched;
        out.tile_rec[i] = tile_record(f, mask);
    }
}

// Launches kernel<degree, SH mode> for the degree and SH mode of g (rows of
// degrees 0 and 2 are not a multiple of four floats: no 16-byte variant).
template <template <int, int> class L, typename... A>
void launch_by_sh(const GaussPtrs& g, A... args)
{
    const int mode = sh_mode(g.sh_layout, g.sh_degree, g.sh);
    switch (g.sh_degree) {
    case 0: mode == kShCoeffMajor ? L<0, kShCoeffMajor>::go(g, args...) : L<0, kShRow>::go(g, args...); break;
    case 1:
        mode == kShCoeffMajor ? L<1, kShCoeffMajor>::go(g, args...)
                              : (mode == kShRow ? L<1, kShRow>::go(g, args...) : L<1, kShRow16>::go(g, args...));
        break;
    case 2: mode == kShCoeffMajor ? L<2, kShCoeffMajor>::go(g, args...) : L<2, kShRow>::go(g, args...); break;
    default:
        mode == kShCoeffMajor ? L<3, kShCoeffMajor>::go(g, args...)
                              : (mode == kShRow ? L<3, kShRow>::go(g, args...) : L<3, kShRow16>::go(g, args...));
        break;
    }
}

template <int kDeg, int kShMode>
struct LaunchPre {
    static void go(const GaussPtrs& g, const CamParams& cam, const PlaneParams& pl, const ProjPtrs& out,
                   hipStream_t s)
    {
        const dim3 grid((unsigned)((g.n + kPreThreads - 1) / kPreThreads));
        hipLaunchKernelGGL((preprocess_kernel<kDeg, kShMode>), grid, dim3(kPreThreads), 0, s, g, cam, pl, out);
    }
};

template <int kDeg, int kShMode>
struct LaunchPreFp {
    static void go(const GaussPtrs& g, const FrameParams* fp, const ProjPtrs& out, hipStream_t s)
    {
        const dim3 grid((unsigned)((g.n + kPreThreads - 1) / kPreThreads));
        hipLaunchKernelGGL((preprocess_fp_kernel<kDeg, kShMode>), grid, dim3(kPreThreads), 0, s, g, fp, out);
    }
};

}  // namespace

hipError_t launch_preprocess(const GaussPtrs& g, const CamParams& cam, const PlaneParams& pl, const ProjPtrs& out,
                             hipStream_t s)
{
    if (g.n == 0) return hipSuccess;
    launch_by_sh<LaunchPre>(g, cam, pl, out, s);
    return hipGetLastError();
}

hipError_t launch_preprocess_fp(const GaussPtrs& g, const FrameParams* fp, const ProjPtrs& out, hipStream_t s)
{
    if (g.n == 0) return hipSuccess;
    launch_by_sh<LaunchPreFp>(g, fp, out, s);
    return hipGetLastError();
}

}  // namespace rara
