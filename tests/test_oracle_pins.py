"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formula: each compares it with a
closed form, an invariant, an independent library routine or a brute-force
measurement (tests/independent.py), chosen so that a dropped term, a wrong
sign, a transposed matrix or a swapped index in the oracle fails at least one.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from paper_2506_20202_amd import scenes
from tests import independent

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_unit(rng):
    v = rng.standard_normal(3)
    return v / np.linalg.norm(v)


def _perp(rng, n):
    u = rng.standard_normal(3)
    u -= np.dot(u, n) * n
    return u / np.linalg.norm(u)


# ----------------------------------------------------------- primitives ----

def test_rotation_matches_scipy():
    """Quaternion (w,x,y,z) -> R agrees with scipy's independent routine,
    including for non-unit quaternions (the oracle normalises)."""
    rng = np.random.default_rng(0)
    for _ in range(200):
        q = rng.standard_normal(4) * rng.uniform(0.1, 5.0)
        R = oracle.rotation(q)
        Rs = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        np.testing.assert_allclose(R, Rs, atol=1e-13)


def test_minv_inverts_unit_sphere_map():
    """Sec. 3.3: M = R S maps the unit sphere to the ellipsoid; M^-1 M = I."""
    rng = np.random.default_rng(1)
    for _ in range(100):
        q = rng.standard_normal(4)
        s = np.exp(rng.normal(-3, 1, 3))
        M = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix() @ np.diag(s)
        np.testing.assert_allclose(oracle.minv(q, s) @ M, np.eye(3), atol=1e-10)


def test_sh_basis_orthonormal_and_matches_scipy_up_to_sign():
    """Real SH up to degree 3: orthonormal on the sphere (Gauss-Legendre x
    uniform quadrature, exact for these polynomials) and equal in magnitude to
    scipy's real harmonics.  The per-function sign is the colour-model
    convention: parity unpinned."""
    from scipy.special import sph_harm_y
    xg, wg = np.polynomial.legendre.leggauss(16)
    phis = np.linspace(0, 2 * np.pi, 33)[:-1]
    G = np.zeros((16, 16))
    for ct, wt in zip(xg, wg):
        st = math.sqrt(1 - ct * ct)
        for ph in phis:
            Y = oracle.sh_basis(3, (st * math.cos(ph), st * math.sin(ph), ct))
            G += np.outer(Y, Y) * wt * (2 * np.pi / len(phis))
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)
    rng = np.random.default_rng(2)
    for _ in range(20):
        d = _rand_unit(rng)
        theta, phi = math.acos(d[2]), math.atan2(d[1], d[0])
        Y = oracle.sh_basis(3, d)
        k = 0
        for l in range(4):
            for m in range(-l, l + 1):
                c = sph_harm_y(l, abs(m), theta, phi)
                if m > 0:
                    ref = math.sqrt(2) * c.real
                elif m < 0:
                    ref = math.sqrt(2) * c.imag
                else:
                    ref = c.real
                assert abs(abs(Y[k]) - abs(ref)) < 1e-12, (l, m)
                k += 1


# ----------------------------------------------------- classification ----

def test_labels_follow_the_three_inequalities():
    """Sec. 3.2: INVISIBLE iff d_ep < -r, VISIBLE iff d_ep > r, CUTOFF iff
    |d_ep| <= r (closed).  Built exactly at and around the boundaries."""
    sigma = np.float32(0.125)           # exact in binary, r = 0.375
    n = np.array([0.0, 0.0, 1.0], np.float32)
    zs = np.array([0.375, 0.3750001, -0.375, -0.3750001, 0.0, 2.0, -2.0], np.float32)
    mean = np.stack([np.zeros(7), np.zeros(7), zs]).astype(np.float32)
    sc = scenes.Scene(np.ascontiguousarray(mean), np.full((3, 7), sigma, np.float32),
                      np.tile(np.array([[1], [0], [0], [0]], np.float32), (1, 7)), np.full(7, 0.5, np.float32),
                      np.zeros((1, 3, 7), np.float32), 0)
    lab, dep, rad = oracle.classify(sc, scenes.Plane(n, 0.0))
    assert list(lab) == [oracle.CUTOFF, oracle.VISIBLE, oracle.CUTOFF, oracle.INVISIBLE, oracle.CUTOFF,
                         oracle.VISIBLE, oracle.INVISIBLE]
    lab2, _, _ = oracle.classify(sc, scenes.Plane(n, 0.0, enabled=False))
    assert (lab2 == oracle.VISIBLE).all()


def test_label_is_plane_scale_invariant_and_swaps_under_flip():
    """A2/I5: (n, d) and (k n, k d) give the same labels for k > 0; (-n, -d)
    swaps VISIBLE and INVISIBLE and keeps CUTOFF."""
    sc = scenes.tiny_scene(3)
    pl = scenes.tiny_plane(3)
    lab, _, _ = oracle.classify(sc, pl)
    lab2, _, _ = oracle.classify(sc, scenes.Plane(pl.n * np.float32(4.0), pl.d * 4.0))
    assert (lab == lab2).all()
    lab3, _, _ = oracle.classify(sc, scenes.Plane(-pl.n, -pl.d))
    swap = np.array([oracle.VISIBLE, oracle.INVISIBLE, oracle.CUTOFF])[lab]
    assert (lab3 == swap).all()


def test_cutoff_is_superset_of_true_straddlers():
    """Sec. 3.2 note: ignoring anisotropy only adds false cutoffs.  Every
    Gaussian whose 3-sigma ellipsoid crosses the plane (exact support
    3 |S R^T n|) is CUTOFF; VISIBLE/INVISIBLE ellipsoids lie wholly on one side."""
    sc = scenes.tiny_scene(4)
    pl = scenes.tiny_plane(4)
    lab, dep, rad = oracle.classify(sc, pl)
    n = pl.n.astype(np.float64) / np.linalg.norm(pl.n)
    for i in range(sc.n):
        q = sc.quat[:, i]
        R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        support = 3.0 * np.linalg.norm(np.diag(sc.scale[:, i].astype(np.float64)) @ R.T @ n)
        if abs(dep[i]) <= support:
            assert lab[i] == oracle.CUTOFF
        if lab[i] == oracle.VISIBLE:
            assert dep[i] - support > 0
        if lab[i] == oracle.INVISIBLE:
            assert dep[i] + support < 0


def test_hard_clip_limit():
    """I12: shrinking every sigma to zero leaves no CUTOFF and labels equal the
    side of the centre (hard clipping)."""
    sc = scenes.tiny_scene(5)
    sc.scale = np.ascontiguousarray(sc.scale * np.float32(1e-9))
    pl = scenes.tiny_plane(5)
    lab, dep, _ = oracle.classify(sc, pl)
    assert (lab != oracle.CUTOFF).all()
    assert ((lab == oracle.VISIBLE) == (dep > 0)).all()


# ---------------------------------------------------------- the weight ----

@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_isotropic_closed_form(sign):
    """I3: isotropic sigma, ray along +-n at lateral offset b: the chord has
    half-length sqrt(9 sigma^2 - b^2) and its midpoint sits at plane value
    d_ep, so w = clamp(1/2 + d_ep / (2 sqrt(9 sigma^2 - b^2)), 0, 1)."""
    rng = np.random.default_rng(6)
    for _ in range(300):
        sigma = float(np.exp(rng.normal(-2, 0.7)))
        mu = rng.uniform(-1, 1, 3)
        n = _rand_unit(rng)
        u = _perp(rng, n)
        b = rng.uniform(0, 0.95) * 3 * sigma
        dep = rng.uniform(-4, 4) * sigma
        d = dep - float(np.dot(n, mu))
        v = sign * n
        e = mu + b * u - v * (10 * sigma + 1.0)
        q = rng.standard_normal(4)
        w, _ = oracle.weight(e, v, mu, q, [sigma] * 3, n, d)
        half = math.sqrt(9 * sigma * sigma - b * b)
        expect = min(1.0, max(0.0, 0.5 + dep / (2 * half)))
        assert abs(w - expect) < 1e-9, (w, expect)


def test_weight_matches_brute_force_marching():
    """I8 on single rays: eq. (11) evaluated by the quadratic equals the
    visible fraction measured by marching and bisection of the inside test."""
    rng = np.random.default_rng(7)
    checked = 0
    for _ in range(400):
        s = np.exp(rng.normal(-2, 0.6, 3))
        q = rng.standard_normal(4)
        mu = rng.uniform(-1, 1, 3)
        n = _rand_unit(rng)
        d = -float(np.dot(n, mu)) + rng.uniform(-3, 3) * s.max()
        e = mu + _rand_unit(rng) * rng.uniform(1.0, 4.0)
        target = mu + rng.normal(0, 1.5, 3) * s
        v = target - e
        w, info = oracle.weight(e, v, mu, q, s, n, d)
        Vinv = np.linalg.inv(independent.cov3(q, s))
        w_bf, hit = independent.chord_weight(e, v, mu, Vinv, n, d)
        if abs(info[0]) < 1e-6:
            continue  # grazing ray
        assert hit == (info[0] > 0)
        assert abs(w - w_bf) < 1e-7, (w, w_bf, info)
        checked += 1
    assert checked > 300


def test_visible_and_invisible_gaussians_get_weight_one_and_zero():
    """I2 (the ablation of Sec. 4.3): tracing a VISIBLE Gaussian gives w = 1
    on every hitting ray and an INVISIBLE one gives 0, so restricting the
    trace to CUTOFF Gaussians changes nothing."""
    rng = np.random.default_rng(8)
    for _ in range(300):
        s = np.exp(rng.normal(-2, 0.6, 3))
        q = rng.standard_normal(4)
        mu = rng.uniform(-1, 1, 3)
        n = _rand_unit(rng)
        r = 3 * s.max()
        side = rng.choice([-1.0, 1.0])
        dep = side * (r * rng.uniform(1.0001, 3.0))
        d = dep - float(np.dot(n, mu))
        e = mu + _rand_unit(rng) * 3.0
        v = mu + rng.normal(0, 0.5, 3) * s - e
        w, info = oracle.weight(e, v, mu, q, s, n, d)
        if info[0] > 0:
            assert w == (1.0 if side > 0 else 0.0)


def test_weight_complement_and_invariances():
    """I5: w(n, d) + w(-n, -d) = 1 on hitting rays.  I6: w is unchanged when
    the direction is scaled, the origin slides along the ray (staying in
    front), and scene, ray and plane undergo one rigid motion."""
    rng = np.random.default_rng(9)
    for _ in range(200):
        s = np.exp(rng.normal(-2, 0.6, 3))
        q = rng.standard_normal(4)
        mu = rng.uniform(-1, 1, 3)
        n = _rand_unit(rng)
        d = -float(np.dot(n, mu)) + rng.uniform(-2, 2) * s.max()
        e = mu + _rand_unit(rng) * 3.0
        v = mu + rng.normal(0, 0.7, 3) * s - e
        w, info = oracle.weight(e, v, mu, q, s, n, d)
        if not info[0] > 1e-6:
            continue
        wf, _ = oracle.weight(e, v, mu, q, s, -n, -d)
        assert abs(w + wf - 1.0) < 1e-9
        w2, _ = oracle.weight(e + 0.3 * v / np.linalg.norm(v), 7.5 * v, mu, q, s, n, d)
        assert abs(w - w2) < 1e-9
        Q = Rotation.random(random_state=int(rng.integers(1 << 30)))
        tr = rng.uniform(-2, 2, 3)
        qq = (Q * Rotation.from_quat([q[1], q[2], q[3], q[0]])).as_quat()
        q2 = np.array([qq[3], qq[0], qq[1], qq[2]])
        n2 = Q.apply(n)
        w3, _ = oracle.weight(Q.apply(e) + tr, Q.apply(v), Q.apply(mu) + tr, q2, s, n2, d - float(np.dot(n2, tr)))
        assert abs(w - w3) < 1e-8


def test_weight_monotone_and_continuous_in_offset():
    """I7: for a fixed ray and normal, w is non-decreasing in d and moves by
    at most |dd| / (2 |n.v| h) per step (continuity claimed in Sec. 3.4)."""
    rng = np.random.default_rng(10)
    for _ in range(40):
        s = np.exp(rng.normal(-2, 0.5, 3))
        q = rng.standard_normal(4)
        mu = rng.uniform(-1, 1, 3)
        n = _rand_unit(rng)
        e = mu + _rand_unit(rng) * 3.0
        v = mu + rng.normal(0, 0.5, 3) * s - e
        base = -float(np.dot(n, mu))
        ds = np.linspace(-4 * s.max(), 4 * s.max(), 801)
        ws = np.array([oracle.weight(e, v, mu, q, s, n, base + dd)[0] for dd in ds])
        assert np.all(np.diff(ws) >= -1e-12)
        _, info = oracle.weight(e, v, mu, q, s, n, base)
        if info[0] > 1e-3:
            vv = v / np.linalg.norm(v)
            lip = 1.0 / (abs(np.dot(n, vv)) * (info[2] - info[1]))
            assert np.max(np.abs(np.diff(ws))) <= lip * (ds[1] - ds[0]) * (1 + 1e-6) + 1e-12


def test_miss_keeps_original_alpha():
    """Eq. (11) 'otherwise' branch: a ray that misses the 3-sigma ellipsoid
    (or starts inside it) keeps w = 1 even when the centre is invisible."""
    mu = np.zeros(3)
    n = np.array([0.0, 0.0, 1.0])
    s = [0.1, 0.1, 0.1]
    q = [1, 0, 0, 0]
    w, info = oracle.weight([0.31, 0, -5], [0, 0, 1], mu, q, s, n, 0.05)   # lateral 0.31 > 0.3
    assert info[0] < 0 and w == 1.0
    w, info = oracle.weight([0.0, 0, 0.0], [0, 0, 1], mu, q, s, n, 0.05)  # origin at the centre
    assert w == 1.0 and info[1] < 0 < info[2]


# ------------------------------------------------------------ projection ----

def test_ewa_isotropic_on_axis():
    """I11: an isotropic Gaussian on the optical axis at depth z projects to
    the principal point with Vhat = ((f sigma / z)^2 + 0.3) I."""
    cam = scenes.tiny_camera(129, 129)
    for sigma, zoff in [(0.05, 0.0), (0.2, 1.0), (0.01, -1.5)]:
        sc = scenes.Scene(np.array([[0.0], [0.0], [zoff]], np.float32), np.full((3, 1), sigma, np.float32),
                          np.array([[0.3], [0.1], [-0.7], [0.2]], np.float32), np.array([0.5], np.float32),
                          np.zeros((1, 3, 1), np.float32), 0)
        pr = oracle.project(sc, cam, np.array([1], np.uint8))
        z = 3.0 + zoff
        f = cam.fx
        s32 = float(np.float32(sigma))
        np.testing.assert_allclose(pr["mean2d"][0], [cam.cx, cam.cy], atol=1e-9)
        np.testing.assert_allclose(pr["cov2d"][0], [(f * s32 / z) ** 2 + 0.3, 0.0, (f * s32 / z) ** 2 + 0.3],
                                   rtol=1e-6, atol=1e-9)


def test_ewa_matches_finite_difference_jacobian():
    """Eqs. (9)-(10): the 2x2 covariance equals J W V W^T J^T with J taken by
    central differences of the pinhole map (guard-band clamp included), and
    the footprint radius is 3 sqrt of numpy's largest eigenvalue."""
    sc = scenes.tiny_scene(11)
    cam = scenes.tiny_camera()
    lab = np.ones(sc.n, np.uint8)
    pr = oracle.project(sc, cam, lab)
    for i in range(0, sc.n, 7):
        ind = independent.project_one(sc.mean[:, i], sc.quat[:, i], sc.scale[:, i], cam)
        if ind is None:
            continue
        m2, V2, z = ind
        np.testing.assert_allclose(pr["mean2d"][i], m2, rtol=1e-12, atol=1e-9)
        np.testing.assert_allclose(pr["cov2d"][i], [V2[0, 0], V2[0, 1], V2[1, 1]], rtol=1e-6, atol=1e-8)
        if pr["drawn"][i]:
            np.testing.assert_allclose(pr["conic"][i], np.linalg.inv(V2)[[0, 0, 1], [0, 1, 1]], rtol=1e-5)
            assert pr["radius"][i] == math.ceil(3 * math.sqrt(np.linalg.eigvalsh(V2).max()))


def test_footprint_covers_three_sigma_ellipse():
    """Every pixel centre inside the 3-sigma ellipse of a drawn Gaussian lies
    in a tile of its tile rectangle (so the lists never drop such pixels)."""
    sc = scenes.tiny_scene(12)
    cam = scenes.tiny_camera()
    pr = oracle.project(sc, cam, np.ones(sc.n, np.uint8))
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    for i in np.nonzero(pr["drawn"])[0][:300]:
        dx = xs - pr["mean2d"][i, 0]
        dy = ys - pr["mean2d"][i, 1]
        c00, c01, c11 = pr["cov2d"][i]
        Q = np.linalg.inv(np.array([[c00, c01], [c01, c11]]))
        m = Q[0, 0] * dx * dx + 2 * Q[0, 1] * dx * dy + Q[1, 1] * dy * dy
        inside = m <= 9.0
        tx0, ty0, tx1, ty1 = pr["rect"][i]
        tx, ty = xs // 16, ys // 16
        ok = (tx >= tx0) & (tx < tx1) & (ty >= ty0) & (ty < ty1)
        assert not np.any(inside & ~ok)


def test_spherical_harmonic_colour_degree0():
    """With SH degree 0 the colour is Y00 sh + 0.5 = the RGB the generator
    encoded (clamped at 0)."""
    sc = scenes.tiny_scene(13)
    rgb_in = np.random.default_rng(13)
    pr = oracle.project(sc, scenes.tiny_camera(), np.ones(sc.n, np.uint8))
    y00 = 1 / (2 * math.sqrt(math.pi))
    exp = np.maximum(0, sc.sh[0].T.astype(np.float64) * y00 + 0.5)
    d = pr["drawn"].astype(bool)
    np.testing.assert_allclose(pr["rgb"][d], exp[d], atol=1e-12)


# ---------------------------------------------------------- compositing ----

def _one_axis_scene(zs, ops, rgbs):
    n = len(zs)
    y00 = 1 / (2 * math.sqrt(math.pi))
    return scenes.Scene(np.array([[0.0] * n, [0.0] * n, zs], np.float32), np.full((3, n), 0.05, np.float32),
                        np.tile(np.array([[1], [0], [0], [0]], np.float32), (1, n)), np.array(ops, np.float32),
                        np.ascontiguousarray(((np.array(rgbs, np.float64).T - 0.5) / y00)[None].astype(np.float32)), 0)


def test_compositing_closed_forms():
    """I10 / eq. (2): at the pixel under an on-axis Gaussian, one Gaussian
    gives C = min(0.99, delta) c; two give c1 a1 + c2 a2 (1 - a1) in depth
    order; swapping the depth order changes the result accordingly."""
    cam = scenes.tiny_camera(129, 129)       # principal point exactly at pixel (64, 64)
    off = scenes.Plane(np.array([0, 0, 1], np.float32), 0.0, enabled=False)
    o1 = oracle.render(_one_axis_scene([0.0], [0.7], [[0.2, 0.5, 0.9]]), cam, off)
    c1 = np.float32(0.7)
    np.testing.assert_allclose(o1["image"][:, 64, 64], np.array([0.2, 0.5, 0.9]) * float(c1), atol=2e-7)
    o2 = oracle.render(_one_axis_scene([0.0, 0.5], [0.6, 0.8], [[1, 0, 0], [0, 1, 0]]), cam, off)
    a1, a2 = float(np.float32(0.6)), float(np.float32(0.8))
    exp = np.array([1, 0, 0]) * a1 + np.array([0, 1, 0]) * a2 * (1 - a1)
    np.testing.assert_allclose(o2["image"][:, 64, 64], exp, atol=2e-7)
    o3 = oracle.render(_one_axis_scene([0.5, 0.0], [0.6, 0.8], [[1, 0, 0], [0, 1, 0]]), cam, off)
    exp3 = np.array([0, 1, 0]) * a2 + np.array([1, 0, 0]) * a1 * (1 - a2)
    np.testing.assert_allclose(o3["image"][:, 64, 64], exp3, atol=2e-7)
    o4 = oracle.render(_one_axis_scene([0.0], [0.9999], [[1, 1, 1]]), cam, off)
    np.testing.assert_allclose(o4["image"][:, 64, 64], [0.99] * 3, atol=1e-12)   # the 0.99 clamp


def test_half_plane_through_centre_halves_alpha_on_axis():
    """A plane through the centre of an isotropic on-axis Gaussian, with its
    normal along the view ray, cuts every hitting chord in half: alpha at the
    centre pixel is min(0.99, delta * 1/2)."""
    cam = scenes.tiny_camera(129, 129)
    sc = _one_axis_scene([0.0], [0.8], [[1, 1, 1]])
    pl = scenes.Plane(np.array([0, 0, 1], np.float32), 0.0)
    o = oracle.render(sc, cam, pl)
    assert o["label"][0] == oracle.CUTOFF
    np.testing.assert_allclose(o["image"][:, 64, 64], [float(np.float32(0.8)) * 0.5] * 3, atol=1e-12)


def test_plane_beyond_scene_reproduces_unclipped_render():
    """I1 and Table 2 (w RaRa: L1 0, SSIM 1 for a plane at infinity): with the
    plane in front of every Gaussian the clipped image equals the plain one
    exactly; with it behind everything the image is the background."""
    with open(os.path.join(GOLDEN, "table2_plane_at_infinity.json")) as f:
        gold = json.load(f)
    sc = scenes.tiny_scene(0)
    cam = scenes.tiny_camera()
    n = scenes.tiny_plane(0).n
    sweep = scenes.plane_sweep(sc, n, count=3)
    plain = oracle.render(sc, cam, scenes.Plane(n, 0.0, enabled=False))
    front = oracle.render(sc, cam, sweep[0])
    assert (front["label"] == oracle.VISIBLE).all()
    l1 = float(np.abs(front["image"] - plain["image"]).mean())
    assert l1 == gold["w_rara"]["L1"]
    assert _ssim(front["image"], plain["image"]) == gold["w_rara"]["SSIM"]
    behind = oracle.render(sc, cam, sweep[-1], bg=(0.1, 0.2, 0.3))
    assert (behind["label"] == oracle.INVISIBLE).all()
    np.testing.assert_array_equal(behind["image"], np.broadcast_to(np.array([0.1, 0.2, 0.3])[:, None, None],
                                                                   behind["image"].shape).astype(np.float32).astype(np.float64))


def _ssim(a, b, C1=0.01 ** 2, C2=0.03 ** 2):
    """Global-statistics SSIM (enough to state 'identical gives 1')."""
    ma, mb = a.mean(), b.mean()
    va, vb = a.var(), b.var()
    cov = ((a - ma) * (b - mb)).mean()
    return float(((2 * ma * mb + C1) * (2 * cov + C2)) / ((ma * ma + mb * mb + C1) * (va + vb + C2)))


def test_without_rara_deviates_only_by_misses():
    """Sec. 4.3 ablation under our reading: tracing VISIBLE Gaussians too
    changes nothing with the plane at infinity (every hit has w = 1 and misses
    keep w = 1), so the paper's nonzero 'wo RaRa' error is not reproduced."""
    sc = scenes.tiny_scene(1)
    cam = scenes.tiny_camera()
    n = scenes.tiny_plane(1).n
    front = scenes.plane_sweep(sc, n, count=2)[0]
    a = oracle.render(sc, cam, front)
    b = oracle.render(sc, cam, front, trace_visible=True)
    np.testing.assert_array_equal(a["image"], b["image"])


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_full_render_matches_independent_brute_force(seed):
    """I8 end to end: a few large Gaussians at 32x32 rendered by the oracle
    and by the independent marcher agree to 1e-6 except on pixels the oracle
    flags as discontinuity events."""
    sc = scenes.small_scene(seed)
    cam = scenes.small_camera()
    rng = np.random.default_rng(60 + seed)
    n = _rand_unit(rng)
    pl = scenes.Plane(n.astype(np.float32), float(np.float32(rng.uniform(-0.1, 0.1))))
    o = oracle.render(sc, cam, pl)
    assert (o["label"] == oracle.CUTOFF).sum() >= 3
    ref = independent.render(sc, cam, pl)
    ok = o["flags"] == 0
    err = np.abs(o["image"] - ref).max(axis=0)
    assert err[ok].max() < 1e-6, err[ok].max()
    assert ok.mean() > 0.9


def test_rigid_motion_leaves_the_image_unchanged():
    """I6 on whole frames: moving scene, camera and plane by one rigid motion
    changes the image only by rounding (float32 inputs re-rounded)."""
    sc = scenes.tiny_scene(2)
    cam = scenes.tiny_camera()
    pl = scenes.tiny_plane(2)
    base = oracle.render(sc, cam, pl)
    Q = Rotation.from_euler("xyz", [0.3, -0.5, 1.1])
    tr = np.array([0.4, -0.2, 0.7])
    Qm = Q.as_matrix()
    mean = (Qm @ sc.mean.astype(np.float64)) + tr[:, None]
    qs = Q * Rotation.from_quat(np.stack([sc.quat[1], sc.quat[2], sc.quat[3], sc.quat[0]], 1).astype(np.float64))
    qq = qs.as_quat()
    quat = np.stack([qq[:, 3], qq[:, 0], qq[:, 1], qq[:, 2]])
    sc2 = scenes.Scene(mean.astype(np.float32), sc.scale.copy(), quat.astype(np.float32), sc.opacity.copy(),
                       sc.sh.copy(), 0)
    wc = cam.world_to_cam.astype(np.float64)
    Rc2 = wc[:, :3] @ Qm.T
    tc2 = wc[:, 3] - Rc2 @ tr
    cam2 = scenes.Camera(np.concatenate([Rc2, tc2[:, None]], 1).astype(np.float32), cam.fx, cam.fy, cam.cx, cam.cy,
                         cam.width, cam.height)
    n2 = Qm @ pl.n.astype(np.float64)
    pl2 = scenes.Plane(n2.astype(np.float32), float(pl.d - n2 @ tr))
    moved = oracle.render(sc2, cam2, pl2)
    same = (base["label"] == moved["label"]).mean()
    assert same > 0.995
    ok = (base["flags"] == 0) & (moved["flags"] == 0)
    err = np.abs(base["image"] - moved["image"]).max(axis=0)
    # float32 re-rounding of inputs moves alpha by ~1e-6; label flips (<0.5%) are local
    assert np.median(err[ok]) < 1e-4
    assert (err[ok] < 1e-3).mean() > 0.97


# ------------------------------------------------------- clip-mode variants ----

def _mode_plane(pl, mode):
    return scenes.Plane(pl.n, pl.d, enabled=mode)


@pytest.mark.parametrize("seed", [0, 3])
def test_hard_clip_equals_plain_render_of_the_kept_gaussians(seed):
    """Hard clipping (Sec. 1, Table 1 'Hard'): the render equals the unclipped
    render of the Gaussians whose centre is on the visible side, bit for bit,
    and away from the plane (|d_ep| > r) its labels are the RaRa labels."""
    sc = scenes.tiny_scene(seed)
    cam = scenes.tiny_camera()
    pl = scenes.tiny_plane(seed)
    hard = oracle.render(sc, cam, _mode_plane(pl, oracle.CLIP_HARD), bg=(0.1, 0.2, 0.3), events=False)
    n = pl.n.astype(np.float64) / np.linalg.norm(pl.n)
    d = float(pl.d) / float(np.linalg.norm(pl.n.astype(np.float64)))
    side = n @ sc.mean.astype(np.float64) + d
    keep = np.nonzero(side >= 0)[0]
    assert 0 < keep.size < sc.n
    plain = oracle.render(sc.subset(keep), cam, scenes.Plane(pl.n, pl.d, enabled=False), bg=(0.1, 0.2, 0.3),
                          events=False)
    np.testing.assert_array_equal(hard["image"], plain["image"])
    assert (hard["label"] != oracle.CUTOFF).all()
    rara, _, rad = oracle.classify(sc, pl)
    far = np.abs(side) > rad
    np.testing.assert_array_equal(hard["label"][far], rara[far])


def test_tight_radius_closed_forms_and_support():
    """f3: r = 3 |S R^T n| is the half-width of the 3-sigma ellipsoid along n:
    3 sigma for isotropic Gaussians, 3 sigma_a when n is the a-th principal
    axis, never above 3 max(sigma), and equal to the largest n.(x - mu) over
    points sampled on the ellipsoid surface (brute force, scipy rotations)."""
    rng = np.random.default_rng(11)
    for _ in range(60):
        q = rng.standard_normal(4)
        s = np.exp(rng.normal(-2, 0.8, 3))
        nrm = _rand_unit(rng)
        one = scenes.Scene(mean=np.zeros((3, 1), np.float32), scale=s.reshape(3, 1).astype(np.float32),
                           quat=q.reshape(4, 1).astype(np.float32), opacity=np.ones(1, np.float32),
                           sh=np.zeros((1, 3, 1), np.float32), sh_degree=0)
        pl = scenes.Plane(nrm.astype(np.float32), 0.0, enabled=oracle.CLIP_RARA | oracle.CLIP_TIGHT)
        _, _, r = oracle.classify(one, pl)
        qf = one.quat[:, 0].astype(np.float64)
        sf = one.scale[:, 0].astype(np.float64)
        nf = pl.n.astype(np.float64) / np.linalg.norm(pl.n.astype(np.float64))
        R = Rotation.from_quat([qf[1], qf[2], qf[3], qf[0]]).as_matrix()
        u = rng.standard_normal((3, 20000))
        u /= np.linalg.norm(u, axis=0)
        pts = R @ (3.0 * sf[:, None] * u)
        brute = float((nf @ pts).max())
        assert brute <= r[0] * (1 + 1e-12)
        assert r[0] - brute <= 2e-3 * r[0]
        assert r[0] <= 3.0 * sf.max() * (1 + 1e-12)
    # isotropic and principal-axis closed forms
    iso = scenes.Scene(mean=np.zeros((3, 1), np.float32), scale=np.full((3, 1), 0.05, np.float32),
                       quat=np.array([[0.3], [0.5], [-0.2], [0.7]], np.float32), opacity=np.ones(1, np.float32),
                       sh=np.zeros((1, 3, 1), np.float32), sh_degree=0)
    _, _, r = oracle.classify(iso, scenes.Plane(np.array([0.2, -0.9, 0.4], np.float32), 0.0,
                                                enabled=oracle.CLIP_RARA | oracle.CLIP_TIGHT))
    assert abs(r[0] - 3 * np.float64(np.float32(0.05))) < 1e-12
    ax = scenes.Scene(mean=np.zeros((3, 1), np.float32), scale=np.array([[0.01], [0.2], [0.03]], np.float32),
                      quat=np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), opacity=np.ones(1, np.float32),
                      sh=np.zeros((1, 3, 1), np.float32), sh_degree=0)
    for a in range(3):
        e = np.zeros(3, np.float32)
        e[a] = -1.0
        _, _, r = oracle.classify(ax, scenes.Plane(e, 0.0, enabled=oracle.CLIP_RARA | oracle.CLIP_TIGHT))
        assert abs(r[0] - 3 * np.float64(ax.scale[a, 0])) < 1e-15


@pytest.mark.parametrize("seed", [1, 4])
def test_tight_mode_equals_rara_without_the_miss_ring(seed):
    """f3: the tight labels only turn CUTOFF Gaussians whose 3-sigma ellipsoid
    lies wholly on one side into VISIBLE (their eq. (11) weight was exactly 1)
    or INVISIBLE (weight 0 on hits, 1 on misses: the miss ring).  So the tight
    render equals the RaRa render of the scene without the latter, exactly."""
    sc = scenes.tiny_scene(seed)
    cam = scenes.tiny_camera()
    pl = scenes.tiny_plane(seed)
    tight = oracle.render(sc, cam, _mode_plane(pl, oracle.CLIP_RARA | oracle.CLIP_TIGHT), events=False)
    rara_lab = oracle.classify(sc, pl)[0]
    gone = (rara_lab == oracle.CUTOFF) & (tight["label"] == oracle.INVISIBLE)
    came = (rara_lab == oracle.CUTOFF) & (tight["label"] == oracle.VISIBLE)
    assert gone.any() and came.any()
    assert ((rara_lab != oracle.CUTOFF) <= (tight["label"] == rara_lab)).all()
    ref = oracle.render(sc.subset(np.nonzero(~gone)[0]), cam, pl, events=False)
    np.testing.assert_array_equal(tight["image"], ref["image"])


def test_strict_miss_weight_uses_the_closest_approach_side():
    """f2: a ray that misses an isotropic Gaussian gets w = 1 exactly when the
    point of the ray closest to the centre (Euclidean, for isotropic sigma) is
    on the visible side, else 0; rays that hit keep the eq. (11) weight."""
    rng = np.random.default_rng(12)
    for _ in range(300):
        sigma = float(np.exp(rng.normal(-2, 0.5)))
        mu = rng.uniform(-1, 1, 3)
        v = _rand_unit(rng)
        u = _perp(rng, v)
        b = rng.uniform(1.05, 3.0) * 3 * sigma           # lateral offset: a miss
        e = mu + b * u - v * rng.uniform(1.0, 3.0)
        closest = e + float(np.dot(mu - e, v)) * v
        n = _rand_unit(rng)
        d = -float(np.dot(n, closest)) + rng.choice([-1, 1]) * rng.uniform(0.01, 0.5) * sigma
        q = rng.standard_normal(4)
        w_strict, info = oracle.weight(e, v, mu, q, [sigma] * 3, n, d, strict_miss=True)
        w_plain, _ = oracle.weight(e, v, mu, q, [sigma] * 3, n, d)
        assert info[0] < 0 and w_plain == 1.0
        assert w_strict == (1.0 if np.dot(n, closest) + d >= 0 else 0.0)
        # a hit through the same plane: strict and eq. (11) agree
        eh = mu + 0.5 * sigma * u - v * 2.0
        wh, ih = oracle.weight(eh, v, mu, q, [sigma] * 3, n, d, strict_miss=True)
        wp, _ = oracle.weight(eh, v, mu, q, [sigma] * 3, n, d)
        assert ih[0] > 0 and wh == wp


def test_strict_miss_weight_follows_the_whitened_closest_point_anisotropic():
    """f2 for anisotropic Gaussians: a missing ray gets w = 1 exactly when the
    point of the ray closest to the centre in the Gaussian's own metric (the
    whitened space of Sec. 3.3) is on the visible side.  That point is found
    independently: a golden-section search of the Mahalanobis distance along
    the ray, with the covariance from scipy's rotation (no closed form, no
    oracle routine).  Half of the planes pass between this point and the
    Euclidean closest point, so taking the Euclidean point (or a transposed
    whitening) would flip the weight there."""
    rng = np.random.default_rng(13)
    checked = discriminating = 0
    for it in range(400):
        s = np.exp(rng.normal(-2.0, 0.8, 3))              # axis ratios up to ~20:1
        q = rng.standard_normal(4)
        mu = rng.uniform(-1, 1, 3)
        Vinv = np.linalg.inv(independent.cov3(q, s))
        e = mu + _rand_unit(rng) * rng.uniform(1.0, 4.0)
        v = mu + _rand_unit(rng) * rng.uniform(1.1, 4.0) * 3.0 * s.max() - e   # passes beside the ellipsoid
        v = v / np.linalg.norm(v)
        xw, fmin = independent.closest_approach(e, v, mu, Vinv)
        if fmin <= 9.0 * (1.0 + 1e-6):
            continue                                       # a hit or a graze: not the strict-miss case
        xe = e + float(np.dot(mu - e, v)) * v              # Euclidean closest point
        if it % 2 == 0 and np.linalg.norm(xw - xe) > 1e-3 * s.max():
            n = (xw - xe) / np.linalg.norm(xw - xe)        # plane between the two points
            d = -float(np.dot(n, 0.5 * (xw + xe)))
        else:
            n = _rand_unit(rng)
            d = -float(np.dot(n, xw)) + rng.uniform(-0.5, 0.5) * s.min()
        side = float(np.dot(n, xw)) + d
        if abs(side) <= 1e-7 * max(1.0, float(np.linalg.norm(xw))):
            continue
        w, info = oracle.weight(e, v, mu, q, s, n, d, strict_miss=True)
        assert info[0] < 0
        assert w == (1.0 if side >= 0 else 0.0), (w, side, it)
        checked += 1
        discriminating += (side >= 0) != (float(np.dot(n, xe)) + d >= 0)
    assert checked > 250 and discriminating > 80, (checked, discriminating)


def test_clip_mode_validation():
    sc = scenes.tiny_scene(0)
    pl = scenes.tiny_plane(0)
    for bad in (3, oracle.CLIP_HARD | oracle.CLIP_TIGHT, oracle.CLIP_TIGHT):
        with pytest.raises(ValueError):
            oracle.classify(sc, _mode_plane(pl, bad))


# ---- clip regions: intersections of several half-spaces (Sec. 6 extension) ----

def _rand_case(rng):
    s = np.exp(rng.normal(-2, 0.6, 3))
    q = rng.standard_normal(4)
    mu = rng.uniform(-1, 1, 3)
    e = mu + _rand_unit(rng) * rng.uniform(1.0, 4.0)
    v = mu + rng.normal(0, 1.5, 3) * s - e
    return s, q, mu, e, v


def _plane_near(rng, mu, s, lo=-3.0, hi=3.0):
    n = _rand_unit(rng)
    return np.array([*n, -float(np.dot(n, mu)) + rng.uniform(lo, hi) * s.max()])


def test_region_of_one_plane_is_the_plane_weight():
    """A region of one half-space gives eq. (11)'s weight of that plane, the
    single-plane oracle pinned above, to rounding."""
    rng = np.random.default_rng(71)
    for _ in range(300):
        s, q, mu, e, v = _rand_case(rng)
        pl = _plane_near(rng, mu, s)
        w1, i1 = oracle.weight(e, v, mu, q, s, pl[:3], pl[3])
        w2, i2 = oracle.weight_region(e, v, mu, q, s, pl[None, :])
        assert abs(w1 - w2) <= 1e-12, (w1, w2)


def test_region_weight_matches_brute_force_marching():
    """Regions of 2-6 random planes through the Gaussian: the oracle's weight
    equals the part of the chord inside every half-space measured by marching
    and bisection."""
    rng = np.random.default_rng(72)
    checked = zero = part = 0
    for _ in range(250):
        s, q, mu, e, v = _rand_case(rng)
        # mostly keeping the centre inside, so that regions with a partly visible chord are common
        planes = np.stack([_plane_near(rng, mu, s, -1.5, 3.0) for _ in range(int(rng.integers(2, 7)))])
        w, info = oracle.weight_region(e, v, mu, q, s, planes)
        if abs(info[0]) < 1e-6:
            continue
        Vinv = np.linalg.inv(independent.cov3(q, s))
        w_bf, hit, spacing = independent.chord_weight_region(e, v, mu, Vinv, planes)
        assert hit == (info[0] > 0)
        if w_bf == 0.0 and w <= 2 * spacing:
            pass   # a visible piece narrower than the marching step
        else:
            assert abs(w - w_bf) < 1e-7, (w, w_bf, info)
        checked += 1
        zero += w == 0.0
        part += 0.0 < w < 1.0
    assert checked > 200 and zero > 10 and part > 30


def test_region_redundant_and_disjoint_planes():
    """A plane repeated, or joined by planes far outside the Gaussian, gives
    that plane's weight; two half-spaces with a gap between them leave no
    visible chord (w = 0 for every hit)."""
    rng = np.random.default_rng(73)
    for _ in range(100):
        s, q, mu, e, v = _rand_case(rng)
        pl = _plane_near(rng, mu, s)
        w1, info = oracle.weight(e, v, mu, q, s, pl[:3], pl[3])
        if not info[0] > 0:
            continue
        far = []
        for _ in range(3):
            n = _rand_unit(rng)
            far.append([*n, -float(np.dot(n, mu)) + 50.0])
        for planes in (np.stack([pl, pl]), np.stack([pl] + far)):
            w2, _ = oracle.weight_region(e, v, mu, q, s, planes)
            assert abs(w1 - w2) <= 1e-12
        n = _rand_unit(rng)
        gap = np.stack([[*n, -float(np.dot(n, mu)) - 10.0], [*(-n), float(np.dot(n, mu)) - 10.0]])
        w3, info3 = oracle.weight_region(e, v, mu, q, s, gap)
        if info3[0] > 0 and info3[1] >= 0:
            assert w3 == 0.0


def test_region_strict_miss_uses_every_plane():
    """Strict miss policy in a region: a missing ray gets w = 1 exactly when
    its closest approach to the centre (whitened metric) is inside every
    half-space."""
    rng = np.random.default_rng(74)
    seen = {0.0: 0, 1.0: 0}
    for _ in range(400):
        s, q, mu, e, _ = _rand_case(rng)
        v = mu + _rand_unit(rng) * 5.0 * s.max() - e     # aims beside the ellipsoid
        planes = np.stack([_plane_near(rng, mu, s) for _ in range(3)])
        w, info = oracle.weight_region(e, v, mu, q, s, planes, strict_miss=True)
        if not info[0] < -1e-9:
            continue
        Minv = oracle.minv(q, s)
        vv = v / np.linalg.norm(v)
        et, vt = Minv @ (e - mu), Minv @ vv
        ts = -np.dot(et, vt) / np.dot(vt, vt)
        x = e + ts * vv
        pa = planes / np.linalg.norm(planes[:, :3], axis=1)[:, None]
        vals = pa[:, :3] @ x + pa[:, 3]
        if np.abs(vals).min() < 1e-9:
            continue
        assert w == (1.0 if (vals >= 0).all() else 0.0)
        seen[w] += 1
    assert seen[0.0] > 20 and seen[1.0] > 5


def test_region_labels_follow_the_inequalities():
    """Labels for a box of six half-spaces, from per-plane distances computed
    here: INVISIBLE beyond r outside any face, VISIBLE beyond r inside every
    face, CUTOFF otherwise; hard clipping keeps exactly the centres inside."""
    sc = scenes.tiny_scene(5)
    box = scenes.box_region((-0.75, -0.8, -0.7), (0.8, 0.7, 0.75))
    label, dep, rad = oracle.classify(sc, box)
    pa = box.planes_array().astype(np.float64)
    nn = pa[:, :3] / np.linalg.norm(pa[:, :3], axis=1)[:, None]
    dist = nn @ sc.mean.astype(np.float64) + (pa[:, 3] / np.linalg.norm(pa[:, :3], axis=1))[:, None]
    r = 3.0 * sc.scale.astype(np.float64).max(0)
    want = np.where((dist < -r).any(0), 0, np.where((dist > r).all(0), 1, 2))
    np.testing.assert_array_equal(label, want)
    np.testing.assert_allclose(dep, dist, atol=1e-12)
    assert (label == 0).sum() > 50 and (label == 1).sum() > 50 and (label == 2).sum() > 50
    hard, _, _ = oracle.classify(sc, scenes.Plane(box.n, box.d, 2, box.extra))
    np.testing.assert_array_equal(hard, (dist >= 0).all(0).astype(np.uint8))


def test_box_around_the_scene_is_the_plain_render():
    """A box that holds every Gaussian's 3-sigma ball leaves the frame
    unclipped: the image equals the render without a plane exactly."""
    sc = scenes.tiny_scene(6)
    cam = scenes.tiny_camera()
    m = sc.mean.astype(np.float64)
    pad = 3.0 * float(sc.scale.max()) + 0.05
    box = scenes.box_region(m.min(1) - pad, m.max(1) + pad)
    a = oracle.render(sc, cam, box, events=False)
    b = oracle.render(sc, cam, scenes.Plane(box.n, box.d, False), events=False)
    assert (a["label"] == 1).all()
    np.testing.assert_array_equal(a["image"], b["image"])


def test_plane_plus_far_planes_renders_as_the_plane():
    """A region of one plane and five planes far outside the scene renders
    the single-plane frame exactly (labels, image, n_contrib)."""
    sc = scenes.tiny_scene(7)
    cam = scenes.tiny_camera()
    pl = scenes.tiny_plane(7)
    rng = np.random.default_rng(75)
    far = [(scenes._f32(n), 40.0) for n in (_rand_unit(rng) for _ in range(5))]
    reg = scenes.Plane(pl.n, pl.d, True, tuple(far))
    a = oracle.render(sc, cam, reg, events=False)
    b = oracle.render(sc, cam, pl, events=False)
    np.testing.assert_array_equal(a["label"], b["label"])
    np.testing.assert_array_equal(a["image"], b["image"])
    np.testing.assert_array_equal(a["n_contrib"], b["n_contrib"])
    assert (a["label"] == 2).sum() > 20


def test_box_render_matches_independent_marcher():
    """End to end on a box: the oracle frame of a few large Gaussians equals a
    brute-force render whose weights come from the region marcher, except
    on pixels the oracle flags as discontinuity events."""
    sc = scenes.small_scene(3)
    cam = scenes.small_camera()
    box = scenes.box_region((-0.25, -0.2, -0.3), (0.2, 0.3, 0.25))
    o = oracle.render(sc, cam, box)
    img = independent.render_region(sc, cam, box)
    ok = o["flags"] == 0
    assert ok.mean() > 0.9 and (o["label"] == 2).sum() >= 3
    err = np.abs(o["image"] - img).max(0)[ok]
    assert err.max() < 1e-5, err.max()


# ------------------------------------------------------------ listed tiles ----

def test_box_min_separable_closed_form():
    """Listed-tile reading: with B = 0 the form is separable and convex in
    each coordinate, so its minimum over a box is at the centre clamped into
    the box, A clamp(0)^2 + C clamp(0)^2; a box holding the centre gives 0."""
    rng = np.random.default_rng(5)
    for _ in range(500):
        A, C = rng.uniform(0.01, 3.0, 2)
        x0, y0 = rng.uniform(-40.0, 40.0, 2)
        x1, y1 = x0 + rng.uniform(0.0, 15.0), y0 + rng.uniform(0.0, 15.0)
        want = A * float(np.clip(0.0, x0, x1)) ** 2 + C * float(np.clip(0.0, y0, y1)) ** 2
        got = oracle.box_min(A, 0.0, C, x0, x1, y0, y1)
        assert got == pytest.approx(want, rel=1e-12, abs=1e-300)
    assert oracle.box_min(1.0, 0.4, 2.0, -3.0, 12.0, -0.5, 14.5) == 0.0


def test_box_min_rotated_forms_against_dense_sampling():
    """Rotated forms with eigenvalue ratios up to 1000: the minimum is no
    larger than q at any point of a 301x301 grid over the box, and the grid's
    best point lies within its spacing times the gradient bound of it."""
    rng = np.random.default_rng(6)
    for _ in range(300):
        th = rng.uniform(0.0, math.pi)
        l1 = rng.uniform(1e-3, 3.0)
        l2 = l1 * rng.uniform(1.0, 1000.0) ** (1 if rng.uniform() < 0.5 else -1)
        c, s = math.cos(th), math.sin(th)
        A = l1 * c * c + l2 * s * s
        B = (l1 - l2) * c * s
        C = l1 * s * s + l2 * c * c
        x0, y0 = rng.uniform(-30.0, 30.0, 2)
        x1, y1 = x0 + 15.0, y0 + 15.0
        gx = np.linspace(x0, x1, 301)
        gy = np.linspace(y0, y1, 301)
        X, Y = np.meshgrid(gx, gy)
        q = A * X * X + 2.0 * B * X * Y + C * Y * Y
        smin = float(q.min())
        got = oracle.box_min(A, B, C, x0, x1, y0, y1)
        assert got <= smin * (1.0 + 1e-12) + 1e-12
        corner = max(abs(x0), abs(x1)) + max(abs(y0), abs(y1))
        slack = 2.0 * max(l1, l2) * corner * (15.0 / 300.0) * math.sqrt(2.0)
        assert smin - got <= slack


def _listed_tile_scene():
    """4,000 general-scene Gaussians and 16 large ones near the origin: a
    few footprint rectangles of 33-64 tiles and of more than 64."""
    sc = scenes.concat(scenes.general_scene(seed=3, n=4000, sh_degree=0),
                       scenes.small_scene(7, n=16, spread=0.35, logscale_mean=0.0))
    cam = scenes.general_views(count=4, width=200, height=120, radius=9.0)[1]
    return sc, cam


def test_listed_tiles_leave_out_only_tiles_no_pixel_reaches():
    """Every (Gaussian, tile) pair that the listed-tile reading leaves out of
    a rectangle has alpha = delta exp(-q/2) < 1/255 at every pixel centre of
    the tile (FP64 conic, the one the compositor uses), so no pixel would
    have taken it; pairs are left out on this scene, and a rectangle of more
    than 64 tiles keeps all of them."""
    sc, cam = _listed_tile_scene()
    lab = np.ones(sc.n, np.uint8)
    pc = oracle.project(sc, cam, lab)
    pf = oracle.project(sc, cam, lab, cull=False)
    np.testing.assert_array_equal(pc["rect"], pf["rect"])
    area = (pf["rect"][:, 2] - pf["rect"][:, 0]) * (pf["rect"][:, 3] - pf["rect"][:, 1])
    assert pc["tiles_touched"].sum() < 0.9 * pf["tiles_touched"].sum()
    big = (pf["drawn"] == 1) & (area > 64)
    np.testing.assert_array_equal(pc["tiles_touched"][big], area[big])
    dropped = 0
    for i in np.flatnonzero((pf["drawn"] == 1) & (area <= 64)):
        tx0, ty0, tx1, ty1 = pf["rect"][i]
        w = tx1 - tx0
        gone = int(pf["tmask"][i]) & ~int(pc["tmask"][i])
        assert int(pc["tmask"][i]) & ~int(pf["tmask"][i]) == 0
        assert pc["tiles_touched"][i] == bin(int(pc["tmask"][i])).count("1")
        A, B, C = pc["conic"][i]
        mx, my = pc["mean2d"][i]
        for k in range(int(area[i])):
            if not (gone >> k) & 1:
                continue
            dropped += 1
            tx, ty = tx0 + k % w, ty0 + k // w
            xs = np.arange(tx * 16, min(tx * 16 + 16, cam.width)) - mx
            ys = np.arange(ty * 16, min(ty * 16 + 16, cam.height)) - my
            X, Y = np.meshgrid(xs, ys)
            q = A * X * X + 2.0 * B * X * Y + C * Y * Y
            alpha = float(sc.opacity[i]) * np.exp(-0.5 * q)
            assert alpha.max() < 1.0 / 255.0, (i, k)
    assert dropped > 100


def test_listed_tiles_render_the_same_frame():
    """The oracle frame over the listed tiles and over whole rectangles (the
    paper's binning): the same image, transmittance and last contributor
    (as a Gaussian id), bit for bit, with a plane that clips."""
    sc, cam = _listed_tile_scene()
    rng = np.random.default_rng(7)
    n = _rand_unit(rng)
    pl = scenes.Plane(n.astype(np.float32), float(np.float32(0.2)))
    a = oracle.render(sc, cam, pl, events=False)
    b = oracle.render(sc, cam, pl, events=False, cull=False)
    assert (a["label"] == oracle.CUTOFF).sum() > 50
    assert a["ids"].size < 0.9 * b["ids"].size
    np.testing.assert_array_equal(a["image"], b["image"])
    np.testing.assert_array_equal(a["final_T"], b["final_T"])

    def last_ids(o):
        tx = (cam.width + 15) // 16
        ys, xs = np.mgrid[0:cam.height, 0:cam.width]
        tile = (ys // 16) * tx + xs // 16
        nc = o["n_contrib"]
        pos = o["offsets"][tile] + np.maximum(nc, 1) - 1
        return np.where(nc > 0, o["ids"][np.minimum(pos, o["ids"].size - 1)], -1)

    np.testing.assert_array_equal(last_ids(a), last_ids(b))


def test_listed_tile_masks_match_an_independent_edge_search():
    """Every mask bit of a frame (rectangles of at most 64 tiles) against the
    rule re-derived without the stationary-point formula: the minimum over
    the tile's pixel-centre box (clipped to the image) is 0 when the box holds
    the centre, else the least of 10,001 samples along each of its four
    edges (a convex form's minimum over a box lies on its boundary).  Bits
    within 1e-6 of the threshold are not judged."""
    sc, cam = _listed_tile_scene()
    p = oracle.project(sc, cam, np.ones(sc.n, np.uint8))
    r = p["rect"][p["drawn"] == 1]
    areas = (r[:, 2] - r[:, 0]) * (r[:, 3] - r[:, 1])
    assert ((areas > 32) & (areas <= 64)).sum() >= 5 and (areas > 64).sum() >= 1
    u = np.linspace(0.0, 1.0, 10001)
    judged = kept = 0
    for i in np.flatnonzero(p["drawn"] == 1):
        tx0, ty0, tx1, ty1 = p["rect"][i]
        w, area = tx1 - tx0, (tx1 - tx0) * (ty1 - ty0)
        if area > 64:
            continue
        A, B, C = (float(np.float32(v)) for v in p["conic"][i])
        s255 = 255.0 * float(sc.opacity[i])
        t = 2.0 * math.log(s255) * 1.02 + 0.02 if s255 > 1.0 else -1.0
        mx, my = p["mean2d"][i]
        for k in range(area):
            tx, ty = tx0 + k % w, ty0 + k // w
            x0, x1 = tx * 16 - mx, min(tx * 16 + 15, cam.width - 1) - mx
            y0, y1 = ty * 16 - my, min(ty * 16 + 15, cam.height - 1) - my
            if x0 <= 0 <= x1 and y0 <= 0 <= y1:
                qmin = 0.0
            else:
                xs = np.concatenate([x0 + (x1 - x0) * u, x0 + (x1 - x0) * u, np.full_like(u, x0), np.full_like(u, x1)])
                ys = np.concatenate([np.full_like(u, y0), np.full_like(u, y1), y0 + (y1 - y0) * u, y0 + (y1 - y0) * u])
                qmin = float((A * xs * xs + 2.0 * B * xs * ys + C * ys * ys).min())
            if s255 > 1.0 and abs(qmin - t) <= 1e-6 * max(1.0, t):
                continue
            bit = (int(p["tmask"][i]) >> k) & 1
            assert bit == (s255 > 1.0 and qmin <= t), (i, k, qmin, t)
            judged += 1
            kept += bit
    assert judged > 5000 and 0.3 * judged < kept < 0.9 * judged
