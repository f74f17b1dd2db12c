/*
 * FP64 CPU oracle of the RaRa-clipped Gaussian-splatting renderer
 * ("RaRa Clipper", arXiv 2506.20202).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain definition that the
 * HIP renderer is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the renderer never does.
 * It shares no code, header or constant with the HIP sources.
 *
 * Every input arrives as float32 and is promoted exactly to double; every
 * operation below is double precision, written in the order the paper states
 * it.  The functions, each citing what it follows:
 *   oracle_classify  - Sec. 3.2 three-way label from the signed distance of the
 *                      centre to the plane (eq. 3 and the three inequalities),
 *                      also step 1 of Algorithm 1.
 *   oracle_project   - Sec. 3.1 covariance V = R S^2 R^T, Sec. 3.4 eqs. (9)-(10)
 *                      EWA projection of V to the 2D covariance, plus the
 *                      splatting conventions the paper leaves to its host
 *                      renderer (footprint, tiles, spherical-harmonic colour).
 *   oracle_weight    - Sec. 3.3 eqs. (4)-(8): ray into unit-sphere space,
 *                      quadratic, roots, ray-plane parameter; Sec. 3.4 eq. (11)
 *                      visible-length decay weight (step 2 of Algorithm 1).
 *   oracle_weight_region - the same weight for a clip region that is the
 *                      intersection of several half-spaces (a box is six): the
 *                      extension to other clipping primitives of Sec. 6.
 *   oracle_lists     - depth-sorted per-tile lists (Sec. 3.1, "sorted by depth"),
 *                      over the tiles that oracle_project keeps (below).
 *   oracle_composite - Sec. 3.1 eq. (2) front-to-back compositing with the
 *                      opacity of eq. (12) and the 0.99 clamp of step 3 of
 *                      Algorithm 1.
 *
 * Readings where the paper is silent or garbled (the same list is kept in
 * the design notes):
 *   - the traced ellipsoid is the kappa-sigma one, |r~|^2 = kappa^2, kappa = 3,
 *     matching the 3-sigma extent of Sec. 3 and r_k = 3 max(sigma);
 *   - w = 1 when the ray has fewer than two intersections with t >= 0
 *     (miss, tangent, camera inside), the "otherwise" branch of eq. (11);
 *   - L_vis is the length of the part of the chord [t1, t2] on the visible
 *     side n.x + d >= 0 (the eq. (11) definition; Algorithm 1's branch order
 *     is garbled and is not followed literally);
 *   - the plane is normalised: (n, d) / |n|;
 *   - a region of several planes (Sec. 6 names other clipping primitives as
 *     the extension; Sec. 2 cites box clipping of multi-layer fields): every
 *     plane is normalised, a Gaussian is INVISIBLE when it is beyond r of any
 *     plane's visible side, VISIBLE when it is beyond r inside every plane,
 *     CUTOFF otherwise; hard clipping keeps it when its centre is inside every
 *     half-space; L_vis is the part of the chord inside every half-space;
 *   - alpha is the unnormalised delta * exp(-1/2 dx^T V^-1 dx) (the usual
 *     splatting convention), skip when alpha < 1/255, stop before a Gaussian
 *     that would take transmittance below 1e-4, dilation 0.3 px^2,
 *     footprint radius ceil(3 sqrt(lambda_max)), near plane 0.2, guard band
 *     1.3 in the Jacobian, pixel centres at integer image coordinates;
 *   - a tile of the footprint's rectangle is listed only when the Gaussian can
 *     reach alpha >= 1/255 in it (the paper lists the whole rectangle; a tile
 *     left out holds no pixel the 1/255 skip would not skip, so the image is
 *     the same): for rectangles of at most 64 tiles, the minimum of the
 *     quadratic form over the box of the tile's pixel centres must not exceed
 *     1.02 * 2 ln(255 delta) + 0.02 (a margin over the float32 evaluation of
 *     alpha), with the conic rounded to float32 as the renderer holds it;
 *     larger rectangles keep every tile.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_TILE 16
#define OR_ALPHA_MAX 0.99
#define OR_ALPHA_MIN (1.0 / 255.0)
#define OR_T_MIN 1e-4
#define OR_DILATION 0.3
#define OR_GUARD 1.3
#define OR_MAX_PLANES 8

enum { OR_INVISIBLE = 0, OR_VISIBLE = 1, OR_CUTOFF = 2 };

/* per-pixel event flags (discontinuities where FP32 and FP64 may legitimately
 * take different branches) */
enum {
    OR_EV_ALPHA_MIN = 1,  /* alpha within a relative window of 1/255 */
    OR_EV_T_MIN = 2,      /* T (1 - alpha) within a relative window of 1e-4 */
    OR_EV_SILHOUETTE = 4, /* ray grazes the traced ellipsoid (hit <-> miss) */
    OR_EV_INSIDE = 8,     /* near-root crosses t = 0 */
};

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Rotation matrix (row-major) of the normalised quaternion (w, x, y, z). */
static void quat_to_rot(double w, double x, double y, double z, double* R)
{
    double s = sqrt(w * w + x * x + y * y + z * z);
    w /= s; x /= s; y /= s; z /= s;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* Plane (n, d) normalised to unit normal; returns 0 when |n| = 0. */
static int normalise_plane(const float* p, double* n, double* d)
{
    double len = sqrt((double)p[0] * p[0] + (double)p[1] * p[1] + (double)p[2] * p[2]);
    if (!(len > 0)) return 0;
    n[0] = p[0] / len; n[1] = p[1] / len; n[2] = p[2] / len;
    *d = p[3] / len;
    return 1;
}

/* Real spherical harmonics Y_lm up to degree 3 at unit direction (x, y, z),
 * ordered l = 0..3, m = -l..l, with the alternating sign convention common in
 * Gaussian-splatting colour models.  Normalisation constants are written as
 * their closed forms. */
static void sh_basis(int deg, double x, double y, double z, double* Y)
{
    const double pi = 3.14159265358979323846;
    Y[0] = sqrt(1.0 / (4 * pi));
    if (deg < 1) return;
    double c1 = sqrt(3.0 / (4 * pi));
    Y[1] = -c1 * y; Y[2] = c1 * z; Y[3] = -c1 * x;
    if (deg < 2) return;
    double xx = x * x, yy = y * y, zz = z * z;
    Y[4] = sqrt(15.0 / (4 * pi)) * x * y;
    Y[5] = -sqrt(15.0 / (4 * pi)) * y * z;
    Y[6] = sqrt(5.0 / (16 * pi)) * (2 * zz - xx - yy);
    Y[7] = -sqrt(15.0 / (4 * pi)) * x * z;
    Y[8] = sqrt(15.0 / (16 * pi)) * (xx - yy);
    if (deg < 3) return;
    Y[9] = -sqrt(35.0 / (32 * pi)) * y * (3 * xx - yy);
    Y[10] = sqrt(105.0 / (4 * pi)) * x * y * z;
    Y[11] = -sqrt(21.0 / (32 * pi)) * y * (4 * zz - xx - yy);
    Y[12] = sqrt(7.0 / (16 * pi)) * z * (2 * zz - 3 * xx - 3 * yy);
    Y[13] = -sqrt(21.0 / (32 * pi)) * x * (4 * zz - xx - yy);
    Y[14] = sqrt(105.0 / (16 * pi)) * z * (xx - yy);
    Y[15] = -sqrt(35.0 / (32 * pi)) * x * (xx - 3 * yy);
}

void oracle_sh_basis(int deg, double x, double y, double z, double* Y) { sh_basis(deg, x, y, z, Y); }

/*
 * Sec. 3.2 / Algorithm 1 step 1.  d_ep = n.mu + d, r = 3 max(sigma):
 *   INVISIBLE if d_ep < -r, VISIBLE if d_ep > r, CUTOFF if |d_ep| <= r.
 * mode & 3 selects the rule: 0 no plane (every Gaussian VISIBLE), 1 the
 * three-way RaRa labels above, 2 hard clipping (the baseline of Sec. 1 and
 * Table 1: a Gaussian is kept whole, VISIBLE, when its centre is on the
 * visible side, d_ep >= 0, and dropped, INVISIBLE, otherwise).  mode & 4
 * (with rule 1) replaces r by the exact half-width of the 3-sigma ellipsoid
 * along the normal, r = 3 |S R^T n| (the support function of the ellipsoid;
 * the paper notes 3 max(sigma) over-estimates it).
 * mean, scale: [3][n], quat: [4][n] (w, x, y, z; only read with mode & 4).
 * planes: [count][4] rows (n, d); with count > 1 the visible region is the
 * intersection of the half-spaces: INVISIBLE when d_ep < -r for some plane,
 * VISIBLE when d_ep > r for every plane, CUTOFF otherwise (hard clipping:
 * VISIBLE when d_ep >= 0 for every plane).  d_ep, radius: [count][n].
 * Returns 0 on an invalid plane, count or mode.
 */
int oracle_classify(int64_t n, const float* mean, const float* scale, const float* quat, const float* planes,
                    int count, int mode, uint8_t* label, double* d_ep, double* radius)
{
    const int rule = mode & 3;
    const int tight = (mode & 4) != 0;
    double nn[OR_MAX_PLANES][3], d[OR_MAX_PLANES];
    if (rule == 3 || (tight && (rule != 1 || !quat))) return 0;
    if (count < 1 || count > OR_MAX_PLANES) return 0;
    for (int k = 0; k < count; k++)
        if (rule && !normalise_plane(planes + 4 * k, nn[k], &d[k])) return 0;
    for (int64_t i = 0; i < n; i++) {
        double mu[3] = {mean[i], mean[n + i], mean[2 * n + i]};
        double sig[3] = {scale[i], scale[n + i], scale[2 * n + i]};
        double R[9];
        if (tight) quat_to_rot(quat[i], quat[n + i], quat[2 * n + i], quat[3 * n + i], R);
        int any_out = 0, all_in = 1, any_behind = 0;
        for (int k = 0; k < count; k++) {
            double r = 3.0 * fmax(fmax(sig[0], sig[1]), sig[2]);
            if (tight) {
                /* (S R^T n)_a = sigma_a (column a of R) . n */
                double q2 = 0.0;
                for (int a = 0; a < 3; a++) {
                    double c = sig[a] * (R[a] * nn[k][0] + R[3 + a] * nn[k][1] + R[6 + a] * nn[k][2]);
                    q2 += c * c;
                }
                r = 3.0 * sqrt(q2);
            }
            double dist = rule ? dot3(nn[k], mu) + d[k] : INFINITY;
            if (d_ep) d_ep[(int64_t)k * n + i] = dist;
            if (radius) radius[(int64_t)k * n + i] = r;
            if (dist < -r) any_out = 1;
            if (!(dist > r)) all_in = 0;
            if (dist < 0) any_behind = 1;
        }
        if (rule == 0) label[i] = OR_VISIBLE;
        else if (rule == 2) label[i] = any_behind ? OR_INVISIBLE : OR_VISIBLE;
        else if (any_out) label[i] = OR_INVISIBLE;
        else if (all_in) label[i] = OR_VISIBLE;
        else label[i] = OR_CUTOFF;
    }
    return 1;
}

/*
 * Camera: cam[0..8] R_c row-major, cam[9..11] t_c, cam[12..15] fx fy cx cy.
 * Camera centre e = -R_c^T t_c.
 */
static void camera_centre(const double* R, const double* t, double* e)
{
    for (int k = 0; k < 3; k++) e[k] = -(R[0 * 3 + k] * t[0] + R[1 * 3 + k] * t[1] + R[2 * 3 + k] * t[2]);
}

/*
 * Minimum over the box [x0, x1] x [y0, y1] (coordinates relative to the
 * projected centre) of q(x, y) = A x^2 + 2 B x y + C y^2, for a positive
 * definite form: zero when the box holds the centre; otherwise the minimum of
 * a convex function over a box lies on its boundary, and along each edge q is
 * a parabola whose minimum is its stationary point (-B X / C on the edge
 * x = X, -B Y / A on the edge y = Y, taken with the reciprocals 1/C and 1/A)
 * clamped to the edge.
 */
double oracle_box_min(double A, double B, double C, double x0, double x1, double y0, double y1)
{
    if (x0 <= 0.0 && x1 >= 0.0 && y0 <= 0.0 && y1 >= 0.0) return 0.0;
    double iA = 1.0 / A, iC = 1.0 / C;
    double best = INFINITY;
    double xs[2] = {x0, x1}, ys[2] = {y0, y1};
    for (int k = 0; k < 2; k++) {
        double X = xs[k];
        double y = -B * X * iC;
        y = y < y0 ? y0 : (y > y1 ? y1 : y);
        double q = A * X * X + 2.0 * B * X * y + C * y * y;
        if (q < best) best = q;
        double Y = ys[k];
        double x = -B * Y * iA;
        x = x < x0 ? x0 : (x > x1 ? x1 : x);
        q = A * x * x + 2.0 * B * x * Y + C * Y * Y;
        if (q < best) best = q;
    }
    return best;
}

#define OR_CULL_MAX_TILES 64

/*
 * EWA projection and splat set-up for every Gaussian with label != INVISIBLE
 * (or every Gaussian when project_all is set, used to find boundary cases).
 *   t = R_c mu + t_c; not drawn when t_z <= near.
 *   J = [[fx/z, 0, -fx u/z], [0, fy/z, -fy u'/z]] with u = t_x/z, u' = t_y/z
 *       clamped to +-1.3 (W/2)/fx and +-1.3 (H/2)/fy.
 *   Vhat = J R_c (R S^2 R^T) R_c^T J^T + 0.3 I (the 2x2 of eq. (10)).
 *   conic = Vhat^-1; mean2d = (fx t_x/z + cx, fy t_y/z + cy); depth = t_z.
 *   radius = ceil(3 sqrt(lambda_max(Vhat))); pixel box
 *   [ceil(m - r), floor(m + r)] clipped to the image; tiles are the 16x16
 *   tiles that contain a pixel of the box (half-open tile rectangle).
 *   colour = max(0, sum_lm Y_lm(dir) sh_lm + 0.5), dir = (mu - e)/|mu - e|.
 *   minv = M^-1 = S^-1 R^T (Sec. 3.3, M = R S), row-major.
 *   listed tiles: with cull set, a rectangle of at most 64 tiles keeps the
 *   tiles whose pixel-centre box the Gaussian reaches (see the readings
 *   above), in tmask (bit k = the k-th tile of the rectangle, row by row);
 *   tiles_touched counts the listed tiles.  cull_margin is the smallest
 *   |q_min - threshold| over the tested tiles (infinity when none was tested).
 * Outputs are per Gaussian; rect = (tx0, ty0, tx1, ty1).
 */
void oracle_project(int64_t n, int sh_degree, const float* mean, const float* scale, const float* quat,
                    const float* sh, const float* cam, int W, int H, double near_z, const uint8_t* label,
                    int project_all, uint8_t* drawn, double* mean2d, double* cov2d, double* conic,
                    double* depth, float* depth32, int32_t* radius, int32_t* rect, int32_t* tiles_touched,
                    double* rgb, double* minv, double* lam_max, const float* opacity, int cull,
                    uint64_t* tmask, double* cull_margin)
{
    double Rc[9], tc[3], e[3];
    for (int k = 0; k < 9; k++) Rc[k] = cam[k];
    for (int k = 0; k < 3; k++) tc[k] = cam[9 + k];
    double fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15];
    camera_centre(Rc, tc, e);
    int tiles_x = (W + OR_TILE - 1) / OR_TILE;
    int tiles_y = (H + OR_TILE - 1) / OR_TILE;
    (void)tiles_x; (void)tiles_y;
    int ncoef = (sh_degree + 1) * (sh_degree + 1);
    double limx = OR_GUARD * (W / 2.0) / fx, limy = OR_GUARD * (H / 2.0) / fy;

    for (int64_t i = 0; i < n; i++) {
        drawn[i] = 0;
        tiles_touched[i] = 0;
        tmask[i] = 0;
        cull_margin[i] = INFINITY;
        rect[4 * i + 0] = rect[4 * i + 1] = rect[4 * i + 2] = rect[4 * i + 3] = 0;
        radius[i] = 0;
        double mu[3] = {mean[i], mean[n + i], mean[2 * n + i]};
        double s[3] = {scale[i], scale[n + i], scale[2 * n + i]};
        double R[9];
        quat_to_rot(quat[i], quat[n + i], quat[2 * n + i], quat[3 * n + i], R);
        /* M^-1 = S^-1 R^T */
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) minv[9 * i + 3 * a + b] = R[3 * b + a] / s[a];
        if (!project_all && label[i] == OR_INVISIBLE) continue;

        double t[3];
        for (int a = 0; a < 3; a++) t[a] = Rc[3 * a] * mu[0] + Rc[3 * a + 1] * mu[1] + Rc[3 * a + 2] * mu[2] + tc[a];
        depth[i] = t[2];
        depth32[i] = (float)t[2];
        if (!(t[2] > near_z)) continue;

        /* world covariance V = R S^2 R^T */
        double V[9];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++)
                V[3 * a + b] = R[3 * a] * s[0] * s[0] * R[3 * b] + R[3 * a + 1] * s[1] * s[1] * R[3 * b + 1] +
                               R[3 * a + 2] * s[2] * s[2] * R[3 * b + 2];
        /* camera covariance W V W^T with W = R_c */
        double RV[9], Vc[9];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++)
                RV[3 * a + b] = Rc[3 * a] * V[b] + Rc[3 * a + 1] * V[3 + b] + Rc[3 * a + 2] * V[6 + b];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++)
                Vc[3 * a + b] = RV[3 * a] * Rc[3 * b] + RV[3 * a + 1] * Rc[3 * b + 1] + RV[3 * a + 2] * Rc[3 * b + 2];
        double z = t[2];
        double u = fmin(limx, fmax(-limx, t[0] / z));
        double up = fmin(limy, fmax(-limy, t[1] / z));
        double J[6] = {fx / z, 0.0, -fx * u / z, 0.0, fy / z, -fy * up / z};
        double JV[6];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 3; b++)
                JV[3 * a + b] = J[3 * a] * Vc[b] + J[3 * a + 1] * Vc[3 + b] + J[3 * a + 2] * Vc[6 + b];
        double c00 = JV[0] * J[0] + JV[1] * J[1] + JV[2] * J[2] + OR_DILATION;
        double c01 = JV[0] * J[3] + JV[1] * J[4] + JV[2] * J[5];
        double c11 = JV[3] * J[3] + JV[4] * J[4] + JV[5] * J[5] + OR_DILATION;
        cov2d[3 * i] = c00; cov2d[3 * i + 1] = c01; cov2d[3 * i + 2] = c11;
        double det = c00 * c11 - c01 * c01;
        if (!(det > 0)) continue;
        conic[3 * i] = c11 / det; conic[3 * i + 1] = -c01 / det; conic[3 * i + 2] = c00 / det;
        double mx = fx * t[0] / z + cx, my = fy * t[1] / z + cy;
        mean2d[2 * i] = mx; mean2d[2 * i + 1] = my;
        double half = 0.5 * (c00 - c11);
        double lmax = 0.5 * (c00 + c11) + sqrt(half * half + c01 * c01);
        lam_max[i] = lmax;
        double r = ceil(3.0 * sqrt(lmax));
        radius[i] = (int32_t)r;
        double x0 = fmax(0.0, ceil(mx - r)), x1 = fmin((double)(W - 1), floor(mx + r));
        double y0 = fmax(0.0, ceil(my - r)), y1 = fmin((double)(H - 1), floor(my + r));
        if (x0 > x1 || y0 > y1) continue;
        int tx0 = (int)x0 / OR_TILE, tx1 = (int)x1 / OR_TILE + 1;
        int ty0 = (int)y0 / OR_TILE, ty1 = (int)y1 / OR_TILE + 1;
        rect[4 * i] = tx0; rect[4 * i + 1] = ty0; rect[4 * i + 2] = tx1; rect[4 * i + 3] = ty1;
        tiles_touched[i] = (tx1 - tx0) * (ty1 - ty0);
        drawn[i] = 1;
        if (tiles_touched[i] <= OR_CULL_MAX_TILES) {
            /* the tiles of the rectangle that the Gaussian reaches (bit k: the
             * k-th tile of the rectangle, row by row) */
            int w = tx1 - tx0, area = tiles_touched[i];
            uint64_t m = 0;
            double A = (double)(float)conic[3 * i], B = (double)(float)conic[3 * i + 1];
            double C = (double)(float)conic[3 * i + 2];
            double s255 = 255.0 * (double)opacity[i];
            if (!cull) {
                m = area == 64 ? ~(uint64_t)0 : (((uint64_t)1 << area) - 1);
            } else if (s255 > 1.0) {
                if (!(A * C - B * B > 0.0)) {
                    m = area == 64 ? ~(uint64_t)0 : (((uint64_t)1 << area) - 1);
                } else {
                    double tq = 2.0 * log(s255) * 1.02 + 0.02;
                    for (int k = 0; k < area; k++) {
                        int tx = tx0 + k % w, ty = ty0 + k / w;
                        double bx1 = fmin((double)(tx * OR_TILE + OR_TILE - 1), (double)(W - 1));
                        double by1 = fmin((double)(ty * OR_TILE + OR_TILE - 1), (double)(H - 1));
                        double q = oracle_box_min(A, B, C, tx * OR_TILE - mx, bx1 - mx, ty * OR_TILE - my, by1 - my);
                        double mg = fabs(q - tq);
                        if (mg < cull_margin[i]) cull_margin[i] = mg;
                        if (q <= tq) m |= (uint64_t)1 << k;
                    }
                }
            }
            tmask[i] = m;
            tiles_touched[i] = __builtin_popcountll(m);
        }

        /* colour from spherical harmonics in the viewing direction */
        double dir[3] = {mu[0] - e[0], mu[1] - e[1], mu[2] - e[2]};
        double len = sqrt(dot3(dir, dir));
        double Y[16];
        sh_basis(sh_degree, dir[0] / len, dir[1] / len, dir[2] / len, Y);
        for (int c = 0; c < 3; c++) {
            double acc = 0.0;
            for (int k = 0; k < ncoef; k++) acc += Y[k] * (double)sh[((int64_t)k * 3 + c) * n + i];
            rgb[3 * i + c] = fmax(0.0, acc + 0.5);
        }
    }
}

/*
 * Sec. 3.3 and 3.4 for one (ray, Gaussian):
 *   e~ = M^-1 (e - mu), v~ = M^-1 v                       (eq. 4)
 *   |r~(t)|^2 = kappa^2  ->  A t^2 + B t + C = 0            (eqs. 5, 6)
 *   A = |v~|^2, B = 2 <e~, v~>, C = |e~|^2 - kappa^2
 *   t_{1,2} = (-B -+ sqrt(B^2 - 4AC)) / 2A                  (eq. 7)
 *   t_p = -(n.e + d) / (n.v)                               (eq. 8)
 *   w = L_vis / (t2 - t1) if two intersections with t >= 0 exist, else 1 (eq. 11)
 * with L_vis the length of {t in [t1, t2] : n.(e + t v) + d >= 0}.
 * strict_miss: a ray that misses the ellipsoid (no real roots) gets
 * w = [n.(e + t* v) + d >= 0] instead of 1, t* = -B / 2A the point of the
 * ray closest to the centre in the whitened metric (the sub-pixel variant of
 * the paper's closing discussion); tangent rays and rays with a root behind
 * the camera keep w = 1.
 * info (optional, 4 doubles): disc/(4A) (the squared distance margin
 * kappa^2 - |closest whitened point|^2), t1, t2, t_p; for a strict miss,
 * info[3] is the plane value at the closest approach instead.
 */
double oracle_weight(const double* e, const double* v, const double* mu, const double* minv, const double* nrm,
                     double d, double kappa, int strict_miss, double* info)
{
    double em[3] = {e[0] - mu[0], e[1] - mu[1], e[2] - mu[2]};
    double et[3], vt[3];
    for (int a = 0; a < 3; a++) {
        et[a] = minv[3 * a] * em[0] + minv[3 * a + 1] * em[1] + minv[3 * a + 2] * em[2];
        vt[a] = minv[3 * a] * v[0] + minv[3 * a + 1] * v[1] + minv[3 * a + 2] * v[2];
    }
    double A = dot3(vt, vt);
    double B = 2.0 * dot3(et, vt);
    double C = dot3(et, et) - kappa * kappa;
    double disc = B * B - 4.0 * A * C;
    double nv = dot3(nrm, v);
    double phi_e = dot3(nrm, e) + d;
    if (info) { info[0] = disc / (4.0 * A); info[1] = info[2] = info[3] = NAN; }
    if (!(disc > 0)) {                       /* miss or tangent: keep rasterised alpha */
        if (strict_miss && disc < 0) {
            double ts = -B / (2.0 * A);
            double phis = phi_e + ts * nv;
            if (info) info[3] = phis;
            return phis >= 0 ? 1.0 : 0.0;
        }
        return 1.0;
    }
    double sq = sqrt(disc);
    double t1 = (-B - sq) / (2.0 * A);
    double t2 = (-B + sq) / (2.0 * A);
    if (info) { info[1] = t1; info[2] = t2; info[3] = nv != 0 ? -phi_e / nv : NAN; }
    if (t1 < 0) return 1.0;                  /* fewer than two intersections on the ray */
    double lvis;
    if (nv == 0) {
        lvis = phi_e >= 0 ? (t2 - t1) : 0.0;
    } else {
        double tp = -phi_e / nv;
        if (nv > 0) {                        /* visible for t >= t_p */
            double lo = fmax(t1, fmin(tp, t2));
            lvis = t2 - lo;
        } else {                             /* visible for t <= t_p */
            double hi = fmin(t2, fmax(tp, t1));
            lvis = hi - t1;
        }
    }
    return lvis / (t2 - t1);
}

/*
 * Eq. (11) for a clip region that is the intersection of `count` half-spaces
 * n_k.x + d_k >= 0 (each normalised): the extension to other clipping
 * primitives named in Sec. 6, here convex ones built from planes (a box is
 * six).  w = L_vis / (t2 - t1) as in oracle_weight, with L_vis the length of
 * the part of the chord [t1, t2] inside every half-space.  A line meets a
 * convex region in one interval: each plane with n.v > 0 bounds it from below
 * at its crossing t_p, each with n.v < 0 from above, and a plane parallel to
 * the ray keeps all of it or none.  Misses, tangent rays and rays with a root
 * behind the camera keep w = 1; strict_miss gives a miss w = [the closest
 * approach lies inside every half-space].  nrm [count][3], dd [count].
 * info as oracle_weight, except that for a strict miss info[3] is the plane
 * value of smallest magnitude at the closest approach.
 */
double oracle_weight_region(const double* e, const double* v, const double* mu, const double* minv,
                            const double* nrm, const double* dd, int count, double kappa, int strict_miss,
                            double* info)
{
    double em[3] = {e[0] - mu[0], e[1] - mu[1], e[2] - mu[2]};
    double et[3], vt[3];
    for (int a = 0; a < 3; a++) {
        et[a] = minv[3 * a] * em[0] + minv[3 * a + 1] * em[1] + minv[3 * a + 2] * em[2];
        vt[a] = minv[3 * a] * v[0] + minv[3 * a + 1] * v[1] + minv[3 * a + 2] * v[2];
    }
    double A = dot3(vt, vt);
    double B = 2.0 * dot3(et, vt);
    double C = dot3(et, et) - kappa * kappa;
    double disc = B * B - 4.0 * A * C;
    if (info) { info[0] = disc / (4.0 * A); info[1] = info[2] = info[3] = NAN; }
    if (!(disc > 0)) {
        if (strict_miss && disc < 0) {
            double ts = -B / (2.0 * A);
            double closest = INFINITY;
            int inside = 1;
            for (int k = 0; k < count; k++) {
                const double* nk = nrm + 3 * k;
                double phis = dot3(nk, e) + dd[k] + ts * dot3(nk, v);
                if (phis < 0) inside = 0;
                if (fabs(phis) < fabs(closest)) closest = phis;
            }
            if (info) info[3] = closest;
            return inside ? 1.0 : 0.0;
        }
        return 1.0;
    }
    double sq = sqrt(disc);
    double t1 = (-B - sq) / (2.0 * A);
    double t2 = (-B + sq) / (2.0 * A);
    if (info) { info[1] = t1; info[2] = t2; }
    if (t1 < 0) return 1.0;
    double lo = t1, hi = t2;
    for (int k = 0; k < count; k++) {
        const double* nk = nrm + 3 * k;
        double nv = dot3(nk, v);
        double phi_e = dot3(nk, e) + dd[k];
        if (k == 0 && info) info[3] = nv != 0 ? -phi_e / nv : NAN;
        if (nv == 0) {
            if (phi_e < 0) hi = lo;           /* parallel and outside: nothing visible */
        } else if (nv > 0) {
            lo = fmax(lo, -phi_e / nv);       /* visible for t >= t_p */
        } else {
            hi = fmin(hi, -phi_e / nv);       /* visible for t <= t_p */
        }
    }
    double lvis = hi > lo ? hi - lo : 0.0;
    return lvis / (t2 - t1);
}

/*
 * Per-tile lists: ids of drawn Gaussians that list the tile (a tile of the
 * rectangle, kept by tmask when the rectangle has at most 64 tiles), ordered
 * by (float32 depth, index).  offsets has tiles+1 entries.
 */
static int or_lists_tile(const int32_t* rect, const uint64_t* tmask, int64_t i, int tx, int ty)
{
    int w = rect[4 * i + 2] - rect[4 * i], h = rect[4 * i + 3] - rect[4 * i + 1];
    if (w * h > OR_CULL_MAX_TILES) return 1;
    int k = (ty - rect[4 * i + 1]) * w + (tx - rect[4 * i]);
    return (int)((tmask[i] >> k) & 1u);
}

typedef struct { float key; int32_t id; } or_entry;
static int cmp_entry(const void* a, const void* b)
{
    const or_entry* x = (const or_entry*)a;
    const or_entry* y = (const or_entry*)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

int64_t oracle_lists(int64_t n, const uint8_t* drawn, const int32_t* rect, const uint64_t* tmask,
                     const float* depth32, int tiles_x, int tiles_y, int64_t* offsets, int32_t* ids)
{
    int64_t T = (int64_t)tiles_x * tiles_y;
    int64_t* count = (int64_t*)calloc((size_t)T, sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) {
        if (!drawn[i]) continue;
        for (int ty = rect[4 * i + 1]; ty < rect[4 * i + 3]; ty++)
            for (int tx = rect[4 * i]; tx < rect[4 * i + 2]; tx++)
                if (or_lists_tile(rect, tmask, i, tx, ty)) count[(int64_t)ty * tiles_x + tx]++;
    }
    offsets[0] = 0;
    for (int64_t t = 0; t < T; t++) offsets[t + 1] = offsets[t] + count[t];
    int64_t P = offsets[T];
    if (ids) {
        memset(count, 0, sizeof(int64_t) * (size_t)T);
        for (int64_t i = 0; i < n; i++) {
            if (!drawn[i]) continue;
            for (int ty = rect[4 * i + 1]; ty < rect[4 * i + 3]; ty++)
                for (int tx = rect[4 * i]; tx < rect[4 * i + 2]; tx++) {
                    if (!or_lists_tile(rect, tmask, i, tx, ty)) continue;
                    int64_t t = (int64_t)ty * tiles_x + tx;
                    ids[offsets[t] + count[t]++] = (int32_t)i;
                }
        }
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t t = 0; t < T; t++) {
            int64_t m = offsets[t + 1] - offsets[t];
            if (m < 2) continue;
            or_entry* tmp = (or_entry*)malloc(sizeof(or_entry) * (size_t)m);
            for (int64_t k = 0; k < m; k++) {
                int32_t id = ids[offsets[t] + k];
                tmp[k].key = depth32[id];
                tmp[k].id = id;
            }
            qsort(tmp, (size_t)m, sizeof(or_entry), cmp_entry);
            for (int64_t k = 0; k < m; k++) ids[offsets[t] + k] = tmp[k].id;
            free(tmp);
        }
    }
    free(count);
    return P;
}

/*
 * Front-to-back compositing (eq. 2) of every pixel of the tiles
 * [tile_begin, tile_end) (row-major tile index; pass 0 and tiles_x*tiles_y
 * for the full image):
 *   for each list entry k: dx = pixel - mean2d, alpha0 = delta exp(-1/2 dx^T conic dx)
 *   (skipped if the exponent is positive); w from oracle_weight for CUTOFF
 *   Gaussians (and for VISIBLE ones too when trace_visible is set: the
 *   "without RaRa" ablation of Sec. 4.3), 1 otherwise; alpha = min(0.99,
 *   alpha0 w) (eq. 12, Algorithm 1 step 3); skip if alpha < 1/255; stop if
 *   T (1 - alpha) < 1e-4; C += alpha T c; T *= 1 - alpha.
 * The ray of pixel (i, j) starts at the camera centre with direction
 * R_c^T ((i - cx)/fx, (j - cy)/fy, 1), normalised.
 * plane_enabled is the clip mode of oracle_classify (0: no plane); with
 * mode & 8 the weight uses the strict miss policy of oracle_weight.
 * planes: [count][4]; with count > 1 the weight is oracle_weight_region.
 * Outputs: image [3][H][W] = C + T bg, final_T, n_contrib (1-based index of
 * the last composited entry), n_walked (entries examined), flags (event bits).
 * counters: [0] entries examined, [1] CUTOFF entries examined, [2] composited,
 * [3] silhouette events, [4] camera-inside events, [5] misses of CUTOFF
 * Gaussians with alpha >= 1/255, [6] alpha-threshold events, [7] T events.
 */
void oracle_composite(int64_t n, const uint8_t* label, const double* mean2d, const double* conic,
                      const float* opacity, const double* rgb, const float* mean, const double* minv,
                      const float* planes, int count, int plane_enabled, const float* cam, int W, int H,
                      const float* bg, const int64_t* offsets, const int32_t* ids, double kappa, int trace_visible,
                      int64_t tile_begin, int64_t tile_end, double tau_sil, double* image, double* final_T,
                      int32_t* n_contrib, int32_t* n_walked, uint32_t* flags, int64_t* counters)
{
    double Rc[9], tc[3], e[3], nn[OR_MAX_PLANES * 3] = {0}, dd[OR_MAX_PLANES] = {0};
    for (int k = 0; k < 9; k++) Rc[k] = cam[k];
    for (int k = 0; k < 3; k++) tc[k] = cam[9 + k];
    double fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15];
    camera_centre(Rc, tc, e);
    if (count < 1) count = 1;
    if (count > OR_MAX_PLANES) count = OR_MAX_PLANES;
    if (plane_enabled)
        for (int k = 0; k < count; k++) normalise_plane(planes + 4 * k, nn + 3 * k, &dd[k]);
    const int strict = (plane_enabled & 8) != 0;   /* strict miss policy, see oracle_weight */
    int tiles_x = (W + OR_TILE - 1) / OR_TILE;
    int64_t c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0, c5 = 0, c6 = 0, c7 = 0;

#pragma omp parallel for schedule(dynamic, 1) reduction(+ : c0, c1, c2, c3, c4, c5, c6, c7)
    for (int64_t tile = tile_begin; tile < tile_end; tile++) {
        int tx = (int)(tile % tiles_x), ty = (int)(tile / tiles_x);
        int64_t lo = offsets[tile], hi = offsets[tile + 1];
        for (int py = ty * OR_TILE; py < ty * OR_TILE + OR_TILE && py < H; py++)
            for (int px = tx * OR_TILE; px < tx * OR_TILE + OR_TILE && px < W; px++) {
                double vc[3] = {(px - cx) / fx, (py - cy) / fy, 1.0};
                double v[3];
                for (int k = 0; k < 3; k++) v[k] = Rc[k] * vc[0] + Rc[3 + k] * vc[1] + Rc[6 + k] * vc[2];
                double vl = sqrt(dot3(v, v));
                v[0] /= vl; v[1] /= vl; v[2] /= vl;
                double T = 1.0, C[3] = {0, 0, 0};
                int32_t last = 0, walked = 0;
                uint32_t fl = 0;
                for (int64_t k = lo; k < hi; k++) {
                    int32_t g = ids[k];
                    walked = (int32_t)(k - lo + 1);
                    int traced = label[g] == OR_CUTOFF || (trace_visible && label[g] == OR_VISIBLE);
                    c0++;
                    if (label[g] == OR_CUTOFF) c1++;
                    double dx = px - mean2d[2 * g], dy = py - mean2d[2 * g + 1];
                    double power = -0.5 * (conic[3 * g] * dx * dx + conic[3 * g + 2] * dy * dy) -
                                   conic[3 * g + 1] * dx * dy;
                    if (power > 0) continue;
                    double a0 = (double)opacity[g] * exp(power);
                    double w = 1.0;
                    if (traced && plane_enabled) {
                        double mu[3] = {mean[g], mean[n + g], mean[2 * n + g]};
                        double info[4];
                        w = count == 1 ? oracle_weight(e, v, mu, minv + 9 * (int64_t)g, nn, dd[0], kappa, strict, info)
                                       : oracle_weight_region(e, v, mu, minv + 9 * (int64_t)g, nn, dd, count, kappa,
                                                              strict, info);
                        if (a0 >= OR_ALPHA_MIN * (1 - 1e-3)) {
                            if (fabs(info[0]) <= tau_sil * kappa * kappa) { fl |= OR_EV_SILHOUETTE; c3++; }
                            /* strict miss: the weight steps where the closest approach crosses the plane */
                            if (strict && info[0] < 0 && fabs(info[3]) <= 1e-5) { fl |= OR_EV_SILHOUETTE; c3++; }
                            if (info[1] == info[1] && info[1] < 0 && info[2] > 0) {
                                c4++;
                                if (fabs(info[1]) <= 1e-3 * (info[2] - info[1])) fl |= OR_EV_INSIDE;
                            }
                            if (!(info[0] > 0) && a0 >= OR_ALPHA_MIN) c5++;
                        }
                    }
                    double alpha = fmin(OR_ALPHA_MAX, a0 * w);
                    if (fabs(alpha - OR_ALPHA_MIN) <= 1e-3 * OR_ALPHA_MIN) { fl |= OR_EV_ALPHA_MIN; c6++; }
                    if (alpha < OR_ALPHA_MIN) continue;
                    double testT = T * (1.0 - alpha);
                    if (fabs(testT - OR_T_MIN) <= 1e-3 * OR_T_MIN) { fl |= OR_EV_T_MIN; c7++; }
                    if (testT < OR_T_MIN) break;
                    for (int c = 0; c < 3; c++) C[c] += alpha * T * rgb[3 * g + c];
                    T = testT;
                    last = (int32_t)(k - lo + 1);
                    c2++;
                }
                int64_t pix = (int64_t)py * W + px;
                for (int c = 0; c < 3; c++) image[(int64_t)c * W * H + pix] = C[c] + T * bg[c];
                final_T[pix] = T;
                n_contrib[pix] = last;
                n_walked[pix] = walked;
                flags[pix] = fl;
            }
    }
    counters[0] = c0; counters[1] = c1; counters[2] = c2; counters[3] = c3;
    counters[4] = c4; counters[5] = c5; counters[6] = c6; counters[7] = c7;
}

/* M^-1 = S^-1 R^T of one Gaussian (Sec. 3.3, M = R S maps the unit sphere to
 * the ellipsoid), row-major. */
void oracle_minv(const double* quat, const double* scale, double* minv)
{
    double R[9];
    quat_to_rot(quat[0], quat[1], quat[2], quat[3], R);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) minv[3 * a + b] = R[3 * b + a] / scale[a];
}

void oracle_rotation(const double* quat, double* R) { quat_to_rot(quat[0], quat[1], quat[2], quat[3], R); }
