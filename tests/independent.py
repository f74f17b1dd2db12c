"""An independent brute-force renderer used to pin the oracle.

It shares nothing with ``oracle/`` beyond the conventions both are written
to (thresholds, dilation, tile footprint, pixel centres).  Where the oracle
uses closed forms, this file uses different routes to the same quantity:

* rotations come from ``scipy.spatial.transform.Rotation``;
* the projection Jacobian is a central finite difference of the pinhole map;
* the 2D footprint radius comes from ``numpy.linalg.eigvalsh``;
* the decay weight of eq. (11) is measured by marching the ray through the
  ellipsoid with the inside test ``(x-mu)^T V^-1 (x-mu) <= 9`` and refining
  the entry, exit and plane crossing by bisection -- no quadratic formula.

It is slow (Python loops per pixel) and meant for scenes of a few Gaussians
at 32x32 pixels.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial.transform import Rotation

KAPPA2 = 9.0
Y00 = 1.0 / (2.0 * math.sqrt(math.pi))


def rot(q_wxyz) -> np.ndarray:
    w, x, y, z = (float(c) for c in q_wxyz)
    return Rotation.from_quat([x, y, z, w]).as_matrix()


def cov3(q_wxyz, s) -> np.ndarray:
    R = rot(q_wxyz)
    return R @ np.diag(np.asarray(s, np.float64) ** 2) @ R.T


def pinhole_map(p, fx, fy, cx, cy):
    return np.array([fx * p[0] / p[2] + cx, fy * p[1] / p[2] + cy])


def project_one(mu, q, s, cam):
    """Returns (mean2d, cov2d incl. dilation, depth) or None if behind near."""
    wc = np.asarray(cam.world_to_cam, np.float64).reshape(3, 4)
    Rc, tc = wc[:, :3], wc[:, 3]
    t = Rc @ np.asarray(mu, np.float64) + tc
    if t[2] <= cam.near:
        return None
    fx, fy, cx, cy = (float(v) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    limx, limy = 1.3 * (cam.width / 2.0) / fx, 1.3 * (cam.height / 2.0) / fy
    tcl = np.array([np.clip(t[0] / t[2], -limx, limx) * t[2], np.clip(t[1] / t[2], -limy, limy) * t[2], t[2]])
    J = np.zeros((2, 3))
    for k in range(3):
        h = 1e-6 * max(1.0, abs(tcl[k]))
        dp = np.zeros(3)
        dp[k] = h
        J[:, k] = (pinhole_map(tcl + dp, fx, fy, cx, cy) - pinhole_map(tcl - dp, fx, fy, cx, cy)) / (2 * h)
    V2 = J @ Rc @ cov3(q, s) @ Rc.T @ J.T + 0.3 * np.eye(2)
    return pinhole_map(t, fx, fy, cx, cy), V2, t[2]


def chord_weight(e, v, mu, Vinv, n, d, samples: int = 4000):
    """Eq. (11) by marching: returns (w, hit).  v need not be normalised."""
    e = np.asarray(e, np.float64)
    v = np.asarray(v, np.float64)
    mu = np.asarray(mu, np.float64)
    vv = v / np.linalg.norm(v)
    # bounding sphere of the 3-sigma ellipsoid: radius 3 sqrt(max eig V)
    rb = 3.0 / math.sqrt(np.linalg.eigvalsh(Vinv).min())
    tc = float(np.dot(mu - e, vv))
    lo, hi = max(0.0, tc - rb * 1.01), tc + rb * 1.01
    if hi <= 0:
        return 1.0, False

    def inside(t):
        x = e[None, :] + np.atleast_1d(t)[:, None] * vv[None, :] - mu[None, :]
        return np.einsum("ni,ij,nj->n", x, Vinv, x) <= KAPPA2

    ts = np.linspace(lo, hi, samples)
    ins = inside(ts)
    if not ins.any():
        return 1.0, False
    if ins[0] and lo == 0.0:
        return 1.0, True  # camera inside: one intersection on the ray
    i0, i1 = int(np.argmax(ins)), samples - 1 - int(np.argmax(ins[::-1]))

    def bisect(a, b, fa_inside):
        for _ in range(80):
            m = 0.5 * (a + b)
            if inside(m)[0] == fa_inside:
                a = m
            else:
                b = m
        return 0.5 * (a + b)

    t1 = bisect(ts[i0 - 1], ts[i0], False) if i0 > 0 else ts[0]
    t2 = bisect(ts[i1], ts[i1 + 1], True) if i1 < samples - 1 else ts[-1]
    nn = np.asarray(n, np.float64)
    L = np.linalg.norm(nn)
    nn, dd = nn / L, float(d) / L

    def vis(t):
        return float(np.dot(nn, e + t * vv)) + dd >= 0

    a_vis, b_vis = vis(t1), vis(t2)
    if a_vis and b_vis:
        return 1.0, True
    if not a_vis and not b_vis:
        return 0.0, True
    a, b = t1, t2
    for _ in range(100):
        m = 0.5 * (a + b)
        if vis(m) == a_vis:
            a = m
        else:
            b = m
    tp = 0.5 * (a + b)
    lvis = (tp - t1) if a_vis else (t2 - tp)
    return lvis / (t2 - t1), True


def render(scene, cam, plane, bg=(0.0, 0.0, 0.0), trace_visible=False):
    """Brute-force RaRa render of an SH-degree-0 scene.  Returns image [3][H][W]."""
    assert scene.sh_degree == 0
    W, H = cam.width, cam.height
    wc = np.asarray(cam.world_to_cam, np.float64).reshape(3, 4)
    e = -wc[:, :3].T @ wc[:, 3]
    n = scene.n
    mean = scene.mean.astype(np.float64)
    # one plane, or several whose half-spaces intersect (a region)
    rows = [np.array([*np.asarray(plane.n, np.float64), float(plane.d)])]
    rows += [np.array([*np.asarray(n_, np.float64), float(d_)]) for n_, d_ in getattr(plane, "extra", ())]
    planes = np.stack(rows)
    Lk = np.linalg.norm(planes[:, :3], axis=1)
    recs = []
    for i in range(n):
        mu = mean[:, i]
        s = scene.scale[:, i].astype(np.float64)
        q = scene.quat[:, i].astype(np.float64)
        if plane.enabled:
            dep = planes[:, :3] @ mu / Lk + planes[:, 3] / Lk
            r = 3.0 * s.max()
            lab = 0 if (dep < -r).any() else (1 if (dep > r).all() else 2)
        else:
            lab = 1
        if lab == 0:
            continue
        pr = project_one(mu, q, s, cam)
        if pr is None:
            continue
        m2, V2, z = pr
        rad = math.ceil(3.0 * math.sqrt(np.linalg.eigvalsh(V2).max()))
        x0, x1 = max(0, math.ceil(m2[0] - rad)), min(W - 1, math.floor(m2[0] + rad))
        y0, y1 = max(0, math.ceil(m2[1] - rad)), min(H - 1, math.floor(m2[1] + rad))
        if x0 > x1 or y0 > y1:
            continue
        col = np.maximum(0.0, scene.sh[0, :, i].astype(np.float64) * Y00 + 0.5)
        recs.append(dict(i=i, lab=lab, m2=m2, Q=np.linalg.inv(V2), z32=np.float32(z), op=float(scene.opacity[i]),
                         col=col, rect=(x0 // 16, y0 // 16, x1 // 16 + 1, y1 // 16 + 1), mu=mu,
                         Vinv=np.linalg.inv(cov3(q, s))))
    recs.sort(key=lambda r: (float(r["z32"]), r["i"]))
    img = np.zeros((3, H, W))
    fx, fy, cx, cy = (float(v) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    for py in range(H):
        for px in range(W):
            tx, ty = px // 16, py // 16
            T, C = 1.0, np.zeros(3)
            v = wc[:, :3].T @ np.array([(px - cx) / fx, (py - cy) / fy, 1.0])
            for r in recs:
                x0, y0, x1, y1 = r["rect"]
                if not (x0 <= tx < x1 and y0 <= ty < y1):
                    continue
                dx = np.array([px, py], np.float64) - r["m2"]
                p = -0.5 * float(dx @ r["Q"] @ dx)
                if p > 0:
                    continue
                a0 = r["op"] * math.exp(p)
                w = 1.0
                if plane.enabled and (r["lab"] == 2 or (trace_visible and r["lab"] == 1)):
                    if len(planes) == 1:
                        w, _ = chord_weight(e, v, r["mu"], r["Vinv"], plane.n, plane.d)
                    else:
                        w, _, _ = chord_weight_region(e, v, r["mu"], r["Vinv"], planes, samples=4000)
                a = min(0.99, a0 * w)
                if a < 1.0 / 255.0:
                    continue
                tT = T * (1 - a)
                if tT < 1e-4:
                    break
                C += a * T * r["col"]
                T = tT
            img[:, py, px] = C + T * np.asarray(bg)
    return img


def chord_weight_region(e, v, mu, Vinv, planes, samples: int = 20000):
    """Visible fraction of the 3-sigma chord inside every half-space of
    ``planes`` ([count][4] rows (n, d)) by marching and bisection: returns
    (w, hit, spacing) with spacing the marching step over the chord length
    (an interval narrower than that may be missed)."""
    e = np.asarray(e, np.float64)
    v = np.asarray(v, np.float64)
    mu = np.asarray(mu, np.float64)
    vv = v / np.linalg.norm(v)
    rb = 3.0 / math.sqrt(np.linalg.eigvalsh(Vinv).min())
    tc = float(np.dot(mu - e, vv))
    lo, hi = max(0.0, tc - rb * 1.01), tc + rb * 1.01
    if hi <= 0:
        return 1.0, False, 0.0

    def inside(t):
        x = e[None, :] + np.atleast_1d(t)[:, None] * vv[None, :] - mu[None, :]
        return np.einsum("ni,ij,nj->n", x, Vinv, x) <= KAPPA2

    ts = np.linspace(lo, hi, samples)
    ins = inside(ts)
    if not ins.any():
        return 1.0, False, 0.0
    if ins[0] and lo == 0.0:
        return 1.0, True, 0.0
    i0, i1 = int(np.argmax(ins)), samples - 1 - int(np.argmax(ins[::-1]))

    def bisect(a, b, pred, a_val):
        for _ in range(90):
            m = 0.5 * (a + b)
            if pred(m) == a_val:
                a = m
            else:
                b = m
        return 0.5 * (a + b)

    ins1 = lambda t: bool(inside(t)[0])
    t1 = bisect(ts[i0 - 1], ts[i0], ins1, False) if i0 > 0 else ts[0]
    t2 = bisect(ts[i1], ts[i1 + 1], ins1, True) if i1 < samples - 1 else ts[-1]
    pa = np.asarray(planes, np.float64).reshape(-1, 4)
    L = np.linalg.norm(pa[:, :3], axis=1)
    nn, dd = pa[:, :3] / L[:, None], pa[:, 3] / L

    def vis(t):
        t = np.atleast_1d(t)
        x = e[None, :] + t[:, None] * vv[None, :]
        return np.all(x @ nn.T + dd[None, :] >= 0, axis=1)

    tt = np.linspace(t1, t2, samples)
    vs = vis(tt)
    spacing = 1.0 / (samples - 1)
    if not vs.any():
        return 0.0, True, spacing
    j0, j1 = int(np.argmax(vs)), samples - 1 - int(np.argmax(vs[::-1]))
    vis1 = lambda t: bool(vis(t)[0])
    a = bisect(tt[j0 - 1], tt[j0], vis1, False) if j0 > 0 else t1
    b = bisect(tt[j1], tt[j1 + 1], vis1, True) if j1 < samples - 1 else t2
    return (b - a) / (t2 - t1), True, spacing


render_region = render   # render takes a plane or a region (a Plane with extra planes)


def closest_approach(e, v, mu, Vinv, iters: int = 200):
    """Point of the line e + t v closest to mu in the metric of Vinv (the
    whitened distance of Sec. 3.3), found by golden-section search on the
    convex function f(t) = (e + t v - mu)^T Vinv (e + t v - mu) after
    bracketing its minimum; no closed form.  Returns (point, f at it)."""
    e, v, mu = (np.asarray(a, np.float64) for a in (e, v, mu))

    def f(t):
        r = e + t * v - mu
        return float(r @ Vinv @ r)

    step = max(1.0, float(np.linalg.norm(mu - e))) / max(float(np.linalg.norm(v)), 1e-300)
    lo, hi = -step, step
    while f(lo) < f(lo + 0.5 * step) or f(hi) < f(hi - 0.5 * step):
        lo, hi, step = lo - 2 * step, hi + 2 * step, 2 * step
    g = (math.sqrt(5.0) - 1.0) / 2.0
    a, b = lo, hi
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = f(c), f(d)
    for _ in range(iters):
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = f(d)
        if b - a <= 1e-13 * max(1.0, abs(a)):
            break
    t = 0.5 * (a + b)
    return e + t * v, f(t)
