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

// kDeg: the SH degree, fixed per launch so that every coefficient load of a
// Gaussian is issued before the first one is used.
template <int kDeg, int kShMode>
__device__ __forceinline__ void preprocess_one(const GaussPtrs& g, const CamParams& cam, const PlaneParams& pl,
                                               const ProjPtrs& out, int64_t i)
{
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
                    out.depth[i] = (float)tz;
                    ushort4 rc = make_ushort4((unsigned short)tx0, (unsigned short)ty0, (unsigned short)tx1,
                                              (unsigned short)ty1);
                    *reinterpret_cast<ushort4*>(out.rect + 4 * i) = rc;

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
    out.tiles_touched[i] = touched;
}

template <int kDeg, int kShMode>
__global__ __launch_bounds__(256) void preprocess_kernel(GaussPtrs g, CamParams cam, PlaneParams pl, ProjPtrs out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < g.n) preprocess_one<kDeg, kShMode>(g, cam, pl, out, i);
}

// Frame-graph variant: camera and plane read from device memory.
template <int kDeg, int kShMode>
__global__ __launch_bounds__(256) void preprocess_fp_kernel(GaussPtrs g, const FrameParams* __restrict__ fp,
                                                            ProjPtrs out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    // read through the pointer: a private copy of the plane arrays, indexed
    // by the plane number, would live in scratch memory
    preprocess_one<kDeg, kShMode>(g, fp->cam, fp->plane, out, i);
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
        hipLaunchKernelGGL((preprocess_kernel<kDeg, kShMode>), dim3((unsigned)((g.n + 255) / 256)), dim3(256), 0, s,
                           g, cam, pl, out);
    }
};

template <int kDeg, int kShMode>
struct LaunchPreFp {
    static void go(const GaussPtrs& g, const FrameParams* fp, const ProjPtrs& out, hipStream_t s)
    {
        hipLaunchKernelGGL((preprocess_fp_kernel<kDeg, kShMode>), dim3((unsigned)((g.n + 255) / 256)), dim3(256), 0,
                           s, g, fp, out);
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
