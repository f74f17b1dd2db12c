"""Gradient oracle: the oracle's forward re-expressed with torch float64 CPU
ops so that autograd differentiates it.

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle/``).  The
discrete decisions of the forward -- labels (Sec. 3.2), which Gaussians are
drawn, their tile rectangles and depth order -- are taken from the C oracle,
so this module only re-writes the continuous part of the frame:

  * EWA projection V_hat = J W V W^T J^T + 0.3 I, mean2d (eqs. 9-10);
  * spherical-harmonic colour, clamped at 0;
  * the eq. (11) weight of CUTOFF Gaussians by the literal world-space ray /
    ellipsoid quadratic and ray / plane parameter (eqs. 4-8);
  * alpha = min(0.99, delta exp(power) w) (eq. 12) and front-to-back
    compositing (eq. 2) with the 1/255 skip and the 1e-4 stop, the skip and
    stop decisions taken on detached values.

It is dense over (pixel, list entry) and meant for scenes of a few hundred
Gaussians at 64x64 pixels.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import CUTOFF, INVISIBLE, VISIBLE, TILE
from . import classify as _classify
from . import project as _project
from . import tile_lists as _tile_lists

DT = torch.float64
KAPPA = 3.0


def _rot(q):
    """Rotation matrices [n,3,3] of quaternions [4,n] (w,x,y,z), normalised."""
    q = q / torch.linalg.norm(q, dim=0, keepdim=True)
    w, x, y, z = q[0], q[1], q[2], q[3]
    R = torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)
    return R


def _sh(deg, d):
    """Real SH basis [n, (deg+1)^2] at unit directions d [n,3] (same
    convention as the C oracle: closed-form normalisations, alternating signs)."""
    pi = math.pi
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    Y = [torch.full_like(x, math.sqrt(1 / (4 * pi)))]
    if deg >= 1:
        c1 = math.sqrt(3 / (4 * pi))
        Y += [-c1 * y, c1 * z, -c1 * x]
    if deg >= 2:
        xx, yy, zz = x * x, y * y, z * z
        Y += [math.sqrt(15 / (4 * pi)) * x * y, -math.sqrt(15 / (4 * pi)) * y * z,
              math.sqrt(5 / (16 * pi)) * (2 * zz - xx - yy), -math.sqrt(15 / (4 * pi)) * x * z,
              math.sqrt(15 / (16 * pi)) * (xx - yy)]
    if deg >= 3:
        Y += [-math.sqrt(35 / (32 * pi)) * y * (3 * xx - yy), math.sqrt(105 / (4 * pi)) * x * y * z,
              -math.sqrt(21 / (32 * pi)) * y * (4 * zz - xx - yy), math.sqrt(7 / (16 * pi)) * z * (2 * zz - 3 * xx - 3 * yy),
              -math.sqrt(21 / (32 * pi)) * x * (4 * zz - xx - yy), math.sqrt(105 / (16 * pi)) * z * (xx - yy),
              -math.sqrt(35 / (32 * pi)) * x * (xx - 3 * yy)]
    return torch.stack(Y, -1)


def params_from_scene(scene, plane, requires_grad=True):
    """Leaf float64 tensors (mean, scale, quat, opacity, sh, plane[4])."""
    t = lambda a: torch.tensor(np.asarray(a, np.float64), dtype=DT, requires_grad=requires_grad)
    pl = np.array([plane.n[0], plane.n[1], plane.n[2], plane.d], np.float64)
    return dict(mean=t(scene.mean), scale=t(scene.scale), quat=t(scene.quat), opacity=t(scene.opacity),
                sh=t(scene.sh), plane=t(pl))


def structure(scene, cam, plane):
    """Discrete structure of the frame from the C oracle: labels, drawn set,
    per-pixel padded lists of Gaussian ids in depth order."""
    label, _, _ = _classify(scene, plane)
    proj = _project(scene, cam, label)
    offsets, ids = _tile_lists(proj, cam)
    W, H = cam.width, cam.height
    tx = (W + TILE - 1) // TILE
    ys, xs = np.mgrid[0:H, 0:W]
    tile = (ys // TILE) * tx + xs // TILE
    lens = (offsets[1:] - offsets[:-1])[tile.reshape(-1)]
    Lmax = max(int(lens.max()) if lens.size else 0, 1)
    idx = np.zeros((H * W, Lmax), np.int64)
    valid = np.zeros((H * W, Lmax), bool)
    starts = offsets[:-1][tile.reshape(-1)]
    for k in range(Lmax):
        ok = k < lens
        valid[:, k] = ok
        idx[ok, k] = ids[starts[ok] + k]
    return dict(label=label, drawn=proj["drawn"].astype(bool), idx=idx, valid=valid,
                px=xs.reshape(-1).astype(np.float64), py=ys.reshape(-1).astype(np.float64))


def render(p, scene, cam, plane_enabled, st, bg=(0.0, 0.0, 0.0), sh_degree=None, aux=False):
    """Differentiable frame: returns the image [3,H,W] (float64 tensor), and
    with ``aux`` also the discrete decisions taken (composited entries, rays
    meeting the ellipsoid twice) so that finite differences can avoid them."""
    deg = scene.sh_degree if sh_degree is None else sh_degree
    W, H = cam.width, cam.height
    wc = torch.tensor(np.asarray(cam.world_to_cam, np.float32).astype(np.float64).reshape(3, 4), dtype=DT)
    Rc, tc = wc[:, :3], wc[:, 3]
    e = -Rc.T @ tc
    fx, fy, cx, cy = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    mu = p["mean"].T                                  # [n,3]
    s = p["scale"].T                                  # [n,3]
    R = _rot(p["quat"])                               # [n,3,3]
    t = mu @ Rc.T + tc                                # camera coordinates
    z = t[:, 2]
    limx, limy = 1.3 * (W / 2.0) / fx, 1.3 * (H / 2.0) / fy
    u = torch.clamp(t[:, 0] / z, -limx, limx)
    v = torch.clamp(t[:, 1] / z, -limy, limy)
    zero = torch.zeros_like(z)
    J = torch.stack([torch.stack([fx / z, zero, -fx * u / z], -1), torch.stack([zero, fy / z, -fy * v / z], -1)], -2)
    V = R @ torch.diag_embed(s * s) @ R.transpose(1, 2)
    Vc = Rc @ V @ Rc.T
    V2 = J @ Vc @ J.transpose(1, 2) + 0.3 * torch.eye(2, dtype=DT)
    det = V2[:, 0, 0] * V2[:, 1, 1] - V2[:, 0, 1] * V2[:, 1, 0]
    ca, cb, cc = V2[:, 1, 1] / det, -V2[:, 0, 1] / det, V2[:, 0, 0] / det
    mx = fx * t[:, 0] / z + cx
    my = fy * t[:, 1] / z + cy
    d = mu - e
    d = d / torch.linalg.norm(d, dim=1, keepdim=True)
    Y = _sh(deg, d)                                   # [n,K]
    sh = p["sh"]                                      # [K,3,n]
    col = torch.einsum("nk,kcn->nc", Y, sh) + 0.5
    col = torch.clamp(col, min=0.0)

    idx = torch.as_tensor(st["idx"])
    valid = torch.as_tensor(st["valid"])
    px = torch.as_tensor(st["px"], dtype=DT)[:, None]
    py = torch.as_tensor(st["py"], dtype=DT)[:, None]
    dx = px - mx[idx]
    dy = py - my[idx]
    power = -0.5 * (ca[idx] * dx * dx + cc[idx] * dy * dy) - cb[idx] * dx * dy
    a0 = p["opacity"][idx] * torch.exp(power)
    w = torch.ones_like(a0)
    two_mask = torch.zeros_like(a0, dtype=torch.bool)
    lab = torch.as_tensor(st["label"].astype(np.int64))
    cut = (lab[idx] == CUTOFF) & valid
    if plane_enabled and bool(cut.any()):
        nraw = p["plane"][:3]
        L = torch.linalg.norm(nraw)
        nn, dd = nraw / L, p["plane"][3] / L
        rays = torch.stack([(px[:, 0] - cx) / fx, (py[:, 0] - cy) / fy, torch.ones_like(px[:, 0])], -1) @ Rc
        rays = rays / torch.linalg.norm(rays, dim=1, keepdim=True)          # [P,3]
        pi_, ki = torch.nonzero(cut, as_tuple=True)
        g = idx[pi_, ki]
        Minv = torch.diag_embed(1.0 / s) @ R.transpose(1, 2)                # [n,3,3]
        vv = rays[pi_]
        et = torch.einsum("nab,nb->na", Minv[g], (e[None, :] - mu[g]))
        vt = torch.einsum("nab,nb->na", Minv[g], vv)
        A = (vt * vt).sum(1)
        B = 2 * (et * vt).sum(1)
        C = (et * et).sum(1) - KAPPA * KAPPA
        disc = B * B - 4 * A * C
        hit = disc > 0
        sq = torch.sqrt(torch.where(hit, disc, torch.ones_like(disc)))
        t1 = (-B - sq) / (2 * A)
        t2 = (-B + sq) / (2 * A)
        two = hit & (t1 >= 0)
        nv = vv @ nn
        phe = nn @ e + dd
        nvs = torch.where(nv == 0, torch.ones_like(nv), nv)
        tp = -phe / nvs
        lpos = t2 - torch.maximum(t1, torch.minimum(tp, t2))
        lneg = torch.minimum(t2, torch.maximum(tp, t1)) - t1
        lzero = torch.where(phe >= 0, t2 - t1, torch.zeros_like(t1))
        lvis = torch.where(nv > 0, lpos, torch.where(nv < 0, lneg, lzero))
        wk = torch.where(two, lvis / torch.where(two, t2 - t1, torch.ones_like(t1)), torch.ones_like(t1))
        w = w.index_put((pi_, ki), wk)
        two_mask = two_mask.index_put((pi_, ki), two)
    alpha = torch.clamp(a0 * w, max=0.99)
    with torch.no_grad():
        ok = valid & (power <= 0) & (alpha >= 1.0 / 255.0)
        al = torch.where(ok, alpha, torch.zeros_like(alpha))
        Tex = torch.cumprod(torch.cat([torch.ones_like(al[:, :1]), 1 - al[:, :-1]], 1), 1)
        term = ok & (Tex * (1 - al) < 1e-4)
        dead = torch.cumsum(term.to(torch.int64), 1) > 0        # the stopping entry and every later one
        keep = ok & ~dead
    af = torch.where(keep, alpha, torch.zeros_like(alpha))
    T = torch.cumprod(torch.cat([torch.ones_like(af[:, :1]), 1 - af], 1), 1)
    Texc, Tfin = T[:, :-1], T[:, -1]
    colk = col[idx]                                                 # [P,L,3]
    Cimg = ((af * Texc)[:, :, None] * colk).sum(1) + Tfin[:, None] * torch.tensor(bg, dtype=DT)[None, :]
    img = Cimg.T.reshape(3, H, W)
    if aux:
        clamp = (a0 * w >= 0.99) & keep
        colclip = (torch.einsum("nk,kcn->nc", Y, sh) + 0.5 <= 0)
        return img, dict(keep=keep, two=two_mask, clamp=clamp.detach(), colclip=colclip.detach())
    return img
