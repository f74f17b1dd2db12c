"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bar: labels, drawn sets, tile rectangles, float32 depth keys and per-tile
lists identical; projected floats to float32 rounding; image max |error| over
clamp(RGB, 0, 1) <= 1e-3 on every pixel the oracle does not flag as a
discontinuity event (alpha at the 1/255 skip, transmittance at the 1e-4 stop,
a ray grazing the traced ellipsoid, a Gaussian within 1e-6 of a label or
footprint boundary).
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from paper_2506_20202_amd import scenes
from tests import gpu_helpers as H
from tests import independent

pytestmark = pytest.mark.gpu

TOL = 1e-3


def _tile_pixel_mask(cam, t0, t1):
    tx = (cam.width + 15) // 16
    m = np.zeros((cam.height, cam.width), bool)
    for t in range(t0, t1):
        y, x = divmod(t, tx)
        m[y * 16:(y + 1) * 16, x * 16:(x + 1) * 16] = True
    return m


def _full_check(sc, cam, pl, bg=(0.0, 0.0, 0.0)):
    o = oracle.render(sc, cam, pl, bg=bg)
    g = H.gpu_frame(sc, cam, pl, bg=bg)
    bad, rects = H.check_projection(g, o)
    assert g["P"] == len(o["ids"]) or len(bad)
    skip = H.tiles_of(rects, cam.tiles[0])
    H.check_lists(g, o, skip=skip)
    excl = oracle.tile_mask(cam, rects)
    err, flagged, _ = H.image_error(g["image"], o, exclude=excl)
    print(f"n={sc.n} {cam.width}x{cam.height} P={g['P']} max_err={err:.2e} flagged={flagged:.4f} "
          f"boundary={len(o['boundary_ids'])} mismatched={len(bad)} cutoff={(o['label'] == 2).sum()} "
          f"counters={o['counters'].tolist()}", flush=True)
    assert err <= TOL
    assert flagged < 0.05
    ok = (o["flags"] == 0) & ~excl
    np.testing.assert_array_equal(g["n_contrib"][ok], o["n_contrib"][ok])
    np.testing.assert_array_equal(g["n_walked"][ok], o["n_walked"][ok])
    np.testing.assert_allclose(g["final_T"][ok], o["final_T"][ok], rtol=1e-3, atol=1e-6)
    # work counts: evaluations for live pixels (a long-list step of four entries
    # may evaluate up to three past the pixel's last), clip weights among them
    ev = g["n_eval"].astype(np.int64)
    assert (ev[0] <= g["n_walked"].astype(np.int64) + 3).all() and (ev[1] <= ev[0]).all()
    return g, o


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_tiny_scene_parity(seed):
    sc, pl = scenes.tiny_scene(seed), scenes.tiny_plane(seed)
    g, o = _full_check(sc, scenes.tiny_camera(), pl)
    _check_plane_mask(g, o, sc, pl)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_small_large_gaussians_parity(seed):
    """A few large Gaussians covering many tiles, most of them CUTOFF."""
    sc = scenes.small_scene(seed, n=24)
    cam = scenes.small_camera(96)
    rng = np.random.default_rng(70 + seed)
    n = rng.standard_normal(3)
    pl = scenes.Plane((n / np.linalg.norm(n)).astype(np.float32), float(rng.uniform(-0.1, 0.1)))
    g, o = _full_check(sc, cam, pl)
    _check_plane_mask(g, o, sc, pl)


def test_ragged_image_and_background():
    """Image size not a multiple of the tile; nonzero background."""
    sc = scenes.tiny_scene(7)
    cam = scenes.tiny_camera(100, 75)
    _full_check(sc, cam, scenes.tiny_plane(7), bg=(0.2, 0.4, 0.6))


def test_plain_render_parity():
    sc = scenes.tiny_scene(8)
    _full_check(sc, scenes.tiny_camera(), scenes.Plane(np.array([0, 0, 1], np.float32), 0.0, enabled=False))


def test_plane_beyond_scene_is_bitwise_plain():
    """Table 2 / I1 on the GPU: the clipped image with the plane in front of
    every Gaussian equals the unclipped GPU image bit for bit."""
    sc = scenes.tiny_scene(0)
    cam = scenes.tiny_camera()
    n = scenes.tiny_plane(0).n
    front = scenes.plane_sweep(sc, n, count=2)[0]
    a = H.gpu_frame(sc, cam, front)
    b = H.gpu_frame(sc, cam, scenes.Plane(n, 0.0, enabled=False))
    assert (a["label"] == 1).all()
    np.testing.assert_array_equal(a["image"], b["image"])
    np.testing.assert_array_equal(a["final_T"], b["final_T"])


def test_plane_behind_scene_gives_background():
    sc = scenes.tiny_scene(0)
    cam = scenes.tiny_camera()
    back = scenes.plane_sweep(sc, scenes.tiny_plane(0).n, count=2)[-1]
    g = H.gpu_frame(sc, cam, back, bg=(0.25, 0.5, 0.75))
    assert (g["label"] == 0).all() and g["P"] == 0
    assert not g["ranges"].any()
    H.check_schedule(g["work"], np.zeros(len(g["ranges"]), np.int64))
    np.testing.assert_array_equal(g["image"], np.broadcast_to(np.array([0.25, 0.5, 0.75], np.float32)[:, None, None],
                                                              g["image"].shape).astype(np.float64))


def test_forward_is_deterministic():
    sc = scenes.tiny_scene(9)
    cam = scenes.tiny_camera()
    pl = scenes.tiny_plane(9)
    a = H.gpu_frame(sc, cam, pl)
    b = H.gpu_frame(sc, cam, pl)
    for k in ("image", "final_T", "n_contrib", "keys", "vals"):
        np.testing.assert_array_equal(a[k], b[k])


def test_empty_scene():
    sc = scenes.tiny_scene(0).subset(np.arange(0))
    g = H.gpu_frame(sc, scenes.tiny_camera(), scenes.tiny_plane(0), bg=(0.1, 0.1, 0.1))
    assert g["P"] == 0
    assert not g["ranges"].any()
    H.check_schedule(g["work"], np.zeros(len(g["ranges"]), np.int64))
    np.testing.assert_allclose(g["image"], 0.1, atol=1e-7)


def test_single_gaussian_closed_form():
    """One on-axis Gaussian cut through its centre by a plane along the view
    ray: alpha at the centre pixel is delta / 2."""
    y00 = 1 / (2 * np.sqrt(np.pi))
    sc = scenes.Scene(np.zeros((3, 1), np.float32), np.full((3, 1), 0.05, np.float32),
                      np.array([[1], [0], [0], [0]], np.float32), np.array([0.8], np.float32),
                      np.full((1, 3, 1), 0.5 / y00, np.float32), 0)
    cam = scenes.tiny_camera(129, 129)
    g = H.gpu_frame(sc, cam, scenes.Plane(np.array([0, 0, 1], np.float32), 0.0))
    assert g["label"][0] == 2
    np.testing.assert_allclose(g["image"][:, 64, 64], 0.4 * 1.0, atol=2e-6)


def test_capacity_overflow_reported_and_frame_untouched():
    import torch
    from paper_2506_20202_amd import renderer as R
    sc = scenes.tiny_scene(0)
    cam = scenes.tiny_camera()
    pl = scenes.tiny_plane(0)
    o = oracle.render(sc, cam, pl, events=False)
    P = len(o["ids"])
    ds = R.DeviceScene.from_scene(sc, torch.device("cuda:0"))
    fr = R.Frame(sc.n, cam.width, cam.height, P // 2, torch.device("cuda:0"))
    fr.out.image.fill_(-7.0)
    R.enqueue_frame(ds, fr, cam, pl)
    torch.cuda.synchronize()
    assert int(fr.bins.overflow.item()) == 1
    assert int(fr.bins.num_pairs.item()) == P
    assert (fr.out.image == -7.0).all()
    assert not fr.bins.ranges.any()   # no tile gets a list from an overflowing frame
    H.check_schedule(fr.bins.work.cpu().numpy().view(np.uint32), np.zeros(fr.bins.ranges.numel() // 2, np.int64))
    out = R.render_checked(ds, fr, cam, pl)
    assert int(fr.bins.overflow.item()) == 0 and fr.capacity >= P
    H.check_lists(H.collect(fr, out, sc.n), o)


@pytest.mark.parametrize("view,offset", [(0, 8), (5, 6), (11, 10)])
def test_general_scene_1080p_full_frame(view, offset):
    """The 1M-Gaussian general scene at 1920x1080 with planes that clip
    (offsets 6-10 of the 16-offset sweep): every label, rectangle and tile list
    checked, and the whole image (every tile the oracle composites)."""
    sc = scenes.general_scene(1)
    cam = scenes.general_views()[view]
    pl = scenes.plane_sweep(sc, scenes.general_plane_normal(1))[offset]
    g = H.gpu_frame(sc, cam, pl, capacity=12_000_000)
    o = oracle.render(sc, cam, pl, events=True)
    bad, rects = H.check_projection(g, o)
    skip = H.tiles_of(rects, cam.tiles[0])
    H.check_lists(g, o, skip=skip)
    excl = oracle.tile_mask(cam, rects)
    err, fl, _ = H.image_error(g["image"], o, exclude=excl)
    print(f"general v{view} o{offset}: P={g['P']} boundary={len(o['boundary_ids'])} mismatched={len(bad)} "
          f"cutoff={(o['label'] == 2).sum()} invisible={(o['label'] == 0).sum()} max_err={err:.2e} "
          f"flagged={fl:.4f}", flush=True)
    assert (o["label"] == 2).sum() > 0 and (o["label"] == 0).sum() > 0   # the plane clips
    assert err <= TOL
    assert fl < 0.05
    ok = (o["flags"] == 0) & ~excl
    np.testing.assert_array_equal(g["n_contrib"][ok], o["n_contrib"][ok])


def test_strand_scene_full_frame():
    """3.2M strand Gaussians (40:1:1) at 1024x1024 with an oblique plane:
    labels and lists exact, the whole image within the bar."""
    sc = scenes.strand_scene(2)
    cam = scenes.strand_views()[0]
    pl = scenes.strand_planes(0)[1]
    g = H.gpu_frame(sc, cam, pl, capacity=40_000_000)
    tx = cam.tiles[0]
    o = oracle.render(sc, cam, pl, events=True)
    bad, rects = H.check_projection(g, o)
    skip = H.tiles_of(rects, tx)
    H.check_lists(g, o, skip=skip)
    err, fl, _ = H.image_error(g["image"], o, exclude=oracle.tile_mask(cam, rects))
    print(f"strands: P={g['P']} cutoff={(o['label'] == 2).sum()} boundary={len(o['boundary_ids'])} "
          f"mismatched={len(bad)} max_err={err:.2e} flagged={fl:.4f}", flush=True)
    assert err <= TOL


@pytest.mark.parametrize("view,box_index", [(1, 2), (4, 5)])
def test_box_workload_full_frame(view, box_index):
    """The box workload at its full size: the 1.5M-Gaussian multi-layer scene
    (SH2) at 1024x1024, a camera on the radius-5 sphere and an axis-aligned
    box (six half-spaces) around a point near the centre, drawn as the
    benchmark draws them: labels, rectangles, listed-tile masks and every tile
    list exact, the whole image within the bar (the region kernel, its
    quadrant units and the per-wave tile walk at full size)."""
    rng = np.random.default_rng(9)
    sc = scenes.multilayer_scene(32, per_shell=300_000, sh_degree=2)
    cams = [scenes.random_camera_on_sphere(rng, 5.0, 1024, 1024) for _ in range(8)]
    c = rng.uniform(-0.2, 0.2, 3)
    h = np.linspace(2.3, 0.5, 8)[box_index]
    box = scenes.box_region(c - h * np.array([1.0, 0.8, 0.9]), c + h * np.array([0.9, 1.0, 0.8]))
    cam = cams[view]
    g = H.gpu_frame(sc, cam, box, capacity=8_000_000)
    o = oracle.render(sc, cam, box, events=True)
    bad, rects = H.check_projection(g, o)
    skip = H.tiles_of(rects, cam.tiles[0])
    H.check_lists(g, o, skip=skip)
    excl = oracle.tile_mask(cam, rects)
    err, fl, _ = H.image_error(g["image"], o, exclude=excl)
    lens = g["ranges"][:, 1] - g["ranges"][:, 0]
    print(f"box v{view} b{box_index}: P={g['P']} cutoff={(o['label'] == 2).sum()} "
          f"invisible={(o['label'] == 0).sum()} long={(lens >= H.HEAVY_LIST).sum()} boundary={len(o['boundary_ids'])} "
          f"mismatched={len(bad)} max_err={err:.2e} flagged={fl:.4f}", flush=True)
    assert (o["label"] == 2).sum() > 1000 and (o["label"] == 0).sum() > 1000   # the box clips
    assert err <= TOL
    assert fl < 0.05
    ok = (o["flags"] == 0) & ~excl
    np.testing.assert_array_equal(g["n_contrib"][ok], o["n_contrib"][ok])


CLIP_MODES = [("hard", oracle.CLIP_HARD), ("tight", oracle.CLIP_RARA | oracle.CLIP_TIGHT),
              ("strict_miss", oracle.CLIP_RARA | oracle.CLIP_STRICT_MISS),
              ("tight_strict", oracle.CLIP_RARA | oracle.CLIP_TIGHT | oracle.CLIP_STRICT_MISS)]


@pytest.mark.parametrize("name,mode", CLIP_MODES)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_clip_mode_parity(name, mode, seed):
    """Hard clipping, tight classification and the strict miss policy: labels
    and lists exact, images within the bar."""
    pl = scenes.tiny_plane(seed)
    _full_check(scenes.tiny_scene(seed), scenes.tiny_camera(), scenes.Plane(pl.n, pl.d, enabled=mode))


@pytest.mark.parametrize("name,mode", CLIP_MODES)
def test_clip_mode_parity_large_gaussians(name, mode):
    sc = scenes.small_scene(1, n=24)
    rng = np.random.default_rng(71)
    n = rng.standard_normal(3)
    pl = scenes.Plane((n / np.linalg.norm(n)).astype(np.float32), float(rng.uniform(-0.1, 0.1)), enabled=mode)
    _full_check(sc, scenes.small_camera(96), pl)


@pytest.mark.parametrize("mode", [oracle.CLIP_RARA, oracle.CLIP_RARA | oracle.CLIP_TIGHT,
                                  oracle.CLIP_RARA | oracle.CLIP_STRICT_MISS])
@pytest.mark.parametrize("normal", [(0.3, -0.5, 0.8), (1.0, 0.2, 0.1)])
def test_camera_inside_cutoff_gaussian(mode, normal):
    """Eq. (11)'s "otherwise" case with the near root behind the camera: a
    CUTOFF Gaussian (sigma 0.3) centred 0.5 in front of the camera, cut by a
    plane through its centre, holds the camera inside its 3-sigma ellipsoid,
    so every pixel ray meets it once at t >= 0 and keeps w = 1.  Labels,
    lists and image as the oracle, whose camera-inside counter covers every
    pixel."""
    cam = scenes.grad_camera(128)
    ins = scenes.inside_gaussian(cam)
    sc = scenes.concat(scenes.grad_scene(20, n=150), ins)
    base = scenes.plane_through(ins.mean[:, 0], normal)
    pl = scenes.Plane(base.n, base.d, mode)
    g, o = _full_check(sc, cam, pl)
    assert o["label"][-1] == oracle.CUTOFF and g["label"][-1] == oracle.CUTOFF
    assert g["tiles_touched"][-1] == 64
    assert o["counters"][4] >= cam.width * cam.height * 0.99


def test_bin_sort_without_pair_start_matches():
    """pair_start is optional in rara_binned: a frame binned without it renders
    and sorts exactly as one with it."""
    import torch
    from paper_2506_20202_amd import renderer as R
    sc = scenes.tiny_scene(4)
    cam, pl = scenes.tiny_camera(), scenes.tiny_plane(4)
    dev = torch.device("cuda:0")
    ds = R.DeviceScene.from_scene(sc, dev)
    outs = []
    for ps in (True, False):
        fr = R.Frame(sc.n, cam.width, cam.height, 1 << 18, dev, walked=True, pair_start=ps)
        R.render_checked(ds, fr, cam, pl)
        P = int(fr.bins.num_pairs.item())
        outs.append((fr.out.image.clone(), fr.bins.keys[:P].clone(), fr.bins.vals[:P].clone(),
                     fr.out.n_contrib.clone(), fr.out.n_walked.clone()))
    for a, b in zip(*outs):
        assert torch.equal(a, b)


# ---- clip regions (several half-spaces; a box is six) ----

def _tiny_box(seed):
    rng = np.random.default_rng(300 + seed)
    lo = rng.uniform(-0.8, -0.2, 3)
    hi = rng.uniform(0.2, 0.8, 3)
    return scenes.box_region(lo, hi)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_box_region_parity(seed):
    """A box of six half-spaces: labels and lists exact, images within the bar
    (the region blend kernel against the region oracle)."""
    box = _tiny_box(seed)
    g, o = _full_check(scenes.tiny_scene(seed), scenes.tiny_camera(), box)
    assert (o["label"] == 2).sum() > 20 and (o["label"] == 0).sum() > 20
    _check_plane_mask(g, o, scenes.tiny_scene(seed), box)


def _check_plane_mask(g, o, sc, pl):
    """The preprocess marks, for each drawn CUTOFF Gaussian, the planes whose
    visible side does not hold its whole 3-sigma ellipsoid: d_k <= 3 sqrt(n_k^T
    Sigma n_k), the ellipsoid's half-width along n_k.  The oracle's per-plane
    distances and a covariance built here decide the same, off a 1e-6 boundary.
    A CUTOFF Gaussian with no plane marked is blended as VISIBLE (every chord
    lies inside every half-space)."""
    cut = np.flatnonzero((o["label"] == 2) & (g["tiles_touched"] > 0))
    dep = np.atleast_2d(o["d_ep"])
    normals = [np.asarray(pl.n, np.float64)] + [np.asarray(n, np.float64) for n, _ in pl.extra]
    want = np.zeros(len(cut), np.int64)
    near = np.zeros(len(cut), bool)
    for j, i in enumerate(cut):
        cov = independent.cov3(sc.quat[:, i], sc.scale[:, i])
        for k, nk in enumerate(normals):
            nk = nk / np.linalg.norm(nk)
            sup = 3.0 * math.sqrt(nk @ cov @ nk)
            want[j] |= int(dep[k, i] <= sup) << k
            near[j] |= abs(dep[k, i] - sup) <= 1e-6
    got = g["splat_cuts"][cut].astype(np.int64)
    ok = ~near
    assert ok.sum() > 10
    np.testing.assert_array_equal(got[ok], want[ok])
    planes = np.bincount([bin(v).count("1") for v in got[ok]])
    print(f"marked planes per CUTOFF Gaussian: {planes}", flush=True)


@pytest.mark.parametrize("name,mode", CLIP_MODES)
def test_box_region_clip_modes(name, mode):
    box = _tiny_box(7)
    _full_check(scenes.tiny_scene(7), scenes.tiny_camera(), scenes.Plane(box.n, box.d, mode, box.extra))


@pytest.mark.parametrize("count", [2, 3, 8])
def test_random_region_parity(count):
    """Regions of random planes through the scene, up to the maximum count."""
    rng = np.random.default_rng(400 + count)
    sc = scenes.tiny_scene(10 + count)
    planes = []
    for _ in range(count):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        planes.append((n, float(rng.uniform(0.2, 0.7))))   # the origin is inside every half-space
    pl = scenes.region(planes)
    g, o = _full_check(sc, scenes.tiny_camera(), pl)
    _check_plane_mask(g, o, sc, pl)


def test_box_region_large_gaussians():
    """Large Gaussians cut by box faces and edges (most of them CUTOFF)."""
    sc = scenes.small_scene(2, n=24)
    box = scenes.box_region((-0.15, -0.2, -0.1), (0.2, 0.1, 0.15))
    g, o = _full_check(sc, scenes.small_camera(96), box)
    assert (o["label"] == 2).sum() >= 8
    _check_plane_mask(g, o, sc, box)


# One 16x16 tile holding the whole list: lists of about 1000, 3000 and 9600
# entries (the depth passes of the sort then run over several 2048-key sort
# tiles whose digit runs all land in one tile's range).  Copies of one
# Gaussian's shape at one point near the origin make runs of 6 and 40 equal
# depths, which must keep index order.  Opacities are scaled to 2 % and kept at
# 0.01 or more, so every Gaussian can reach alpha 1/255 and is listed.
def _one_tile_scene(n, runs, seed=5):
    sc = scenes.small_scene(seed, n=n, spread=0.3, logscale_mean=-2.5)
    mean, scale, quat = sc.mean.copy(), sc.scale.copy(), sc.quat.copy()
    for k, (start, length) in enumerate(runs):
        mean[:, start: start + length] = np.array([[0.01 - 0.03 * k], [0.02], [0.03 + 0.02 * k]], np.float32)
        for a in (scale, quat):
            a[:, start + 1: start + length] = a[:, start:start + 1]
    op = np.maximum(sc.opacity * 0.02, 0.01).astype(np.float32)
    return dataclasses.replace(sc, mean=mean, scale=scale, quat=quat, opacity=op)


@pytest.mark.parametrize("n", [1000, 3000, 10000])
@pytest.mark.parametrize("runs", [((100, 6),), ((100, 6), (300, 40))], ids=["run6", "run6_run40"])
def test_one_tile_long_lists_and_equal_depths(n, runs):
    sc = _one_tile_scene(n, runs)
    cam, pl = scenes.small_camera(16), scenes.tiny_plane(0)
    lab, _, _ = oracle.classify(sc, pl)
    proj = oracle.project(sc, cam, lab)
    offs, ids = oracle.tile_lists(proj, cam)
    g = H.gpu_frame(sc, cam, pl, capacity=2 * n)
    d = proj["depth32"][ids]
    runs_found = np.diff(np.flatnonzero(np.diff(np.concatenate([[np.nan], d, [np.nan]])) != 0))
    print(f"n={n} list={len(ids)} longest equal-depth run={runs_found.max()}", flush=True)
    assert runs_found.max() == max(length for _, length in runs)
    assert g["P"] == len(ids)
    H.check_lists(g, {"offsets": offs, "ids": ids})
    # the sorted keys carry each entry's float32 depth bits
    np.testing.assert_array_equal((g["keys"] & np.uint64(0xFFFFFFFF)).astype(np.uint32),
                                  d.astype(np.float32).view(np.uint32))


# Long lists: thousands of overlapping Gaussians over a few tiles, most of them
# CUTOFF, so tiles hold 2000-7600 entries (the blend dispatches tiles of 1024
# entries or more first, each XCD taking a run of them).  With that many
# entries per pixel, many pixels carry an oracle event (an alpha
# within 0.1 % of 1/255 or a grazing ray); the rest are checked to the usual bar.
DENSE_NORMAL = (np.array([0.3, 0.2, -0.93]) / np.linalg.norm([0.3, 0.2, -0.93])).astype(np.float32)


def _dense_scene(seed, n, opacity_scale, logscale_mean):
    sc = scenes.small_scene(seed, n=n, spread=0.35, logscale_mean=logscale_mean)
    return dataclasses.replace(sc, opacity=(sc.opacity * opacity_scale).astype(np.float32))


def _dense_check(sc, cam, pl, tiles=None, min_long=1):
    g = H.gpu_frame(sc, cam, pl, capacity=max(1 << 20, 400 * sc.n))
    o = oracle.render(sc, cam, pl, tiles=tiles)
    bad, rects = H.check_projection(g, o)
    skip = H.tiles_of(rects, cam.tiles[0])
    t0, t1 = tiles if tiles is not None else (0, cam.tiles[0] * cam.tiles[1])
    H.check_lists(g, o, tiles=range(t0, t1), skip=skip)
    lens = g["ranges"][:, 1] - g["ranges"][:, 0]
    region = _tile_pixel_mask(cam, t0, t1)
    excl = oracle.tile_mask(cam, rects)
    err, flagged, _ = H.image_error(g["image"], o, exclude=excl, region=region)
    ok = (o["flags"] == 0) & ~excl & region
    print(f"n={sc.n} {cam.width}x{cam.height} P={g['P']} long={(lens >= H.HEAVY_LIST).sum()} max_len={lens.max()} "
          f"max_err={err:.2e} flagged={flagged:.4f} checked={ok.sum()} mismatched={len(bad)}", flush=True)
    assert (lens >= H.HEAVY_LIST).sum() >= min_long
    assert ok.sum() >= 0.25 * region.sum()
    assert err <= TOL
    np.testing.assert_array_equal(g["n_contrib"][ok], o["n_contrib"][ok])
    np.testing.assert_array_equal(g["n_walked"][ok], o["n_walked"][ok])
    np.testing.assert_allclose(g["final_T"][ok], o["final_T"][ok], rtol=1e-3, atol=1e-6)
    return g, o


@pytest.mark.parametrize("seed,opacity_scale,size", [(0, 1.0, 72), (1, 0.03, 72), (2, 0.05, 100)])
def test_long_list_parity(seed, opacity_scale, size):
    """Opaque (pixels terminate early) and faint (every list walked to its
    end); at 72 px the right quadrants of the last tile column lie outside
    the image.  Six or more lists of 1024 entries or more each (the faint
    Gaussians list fewer tiles than their rectangles)."""
    n, ls = (4000, -2.3) if size < 100 else (6000, -2.5)
    _dense_check(_dense_scene(seed, n, opacity_scale, ls), scenes.small_camera(size),
                 scenes.Plane(DENSE_NORMAL, 0.02), min_long=6)


@pytest.mark.parametrize("name,mode", CLIP_MODES)
def test_long_list_clip_modes(name, mode):
    _dense_check(_dense_scene(1, 5000, 0.03, -2.3), scenes.small_camera(72),
                 scenes.Plane(DENSE_NORMAL, 0.02, enabled=mode), min_long=4)


@pytest.mark.parametrize("name,mode", [("rara", oracle.CLIP_RARA)] + CLIP_MODES)
def test_long_list_box_region(name, mode):
    """Long lists cut by a box (six half-spaces): the quadrant units with the
    region weight, the one-plane weight for entries that only one face cuts,
    and the strict miss policy over the whole region.  Hard clipping keeps
    only the centres inside the box: one long list."""
    box = scenes.box_region((-0.25, -0.2, -0.3), (0.2, 0.25, 0.15), enabled=mode)
    sc = _dense_scene(1, 5000, 0.03, -2.3)
    g, o = _dense_check(sc, scenes.small_camera(72), box, min_long=1 if mode == oracle.CLIP_HARD else 4)
    if mode != oracle.CLIP_HARD:   # hard clipping has no CUTOFF label
        assert (o["label"] == 2).sum() >= 100
        _check_plane_mask(g, o, sc, box)


@pytest.mark.parametrize("seed,size", [(1, 72), (2, 100)])
def test_long_list_plain(seed, size):
    """Long lists without a plane: lists of 4096 entries or more still run
    as quadrant units (four lanes per pixel), shorter ones as whole tiles."""
    n, ls = (4000, -2.3) if size < 100 else (6000, -2.5)
    g, _ = _dense_check(_dense_scene(seed, n, 0.03, ls), scenes.small_camera(size),
                        scenes.Plane(DENSE_NORMAL, 0.02, enabled=False), min_long=4)
    lens = g["ranges"][:, 1] - g["ranges"][:, 0]
    print(f"lists of 4096 or more: {(lens >= 4096).sum()}, of 1024-4095: {((lens >= 1024) & (lens < 4096)).sum()}",
          flush=True)


def test_many_long_list_tiles():
    """576 tiles of 2500-7600 entries each, every tile in the long-list group;
    a band near the top and the bottom row are checked."""
    sc = _dense_scene(3, 12000, 0.04, -2.6)
    cam = scenes.pinhole((0.3, -0.4, -3.0), (0.0, 0.0, 0.0), 384, 384, 12.0)
    pl = scenes.Plane(DENSE_NORMAL, 0.05)
    tx = cam.tiles[0]
    for band in [(5 * tx, 6 * tx), (23 * tx, 24 * tx)]:
        g, _ = _dense_check(sc, cam, pl, tiles=band, min_long=576)


def test_long_list_forward_is_deterministic():
    sc = _dense_scene(2, 6000, 0.05, -2.5)
    cam = scenes.small_camera(100)
    pl = scenes.Plane(DENSE_NORMAL, 0.02)
    a = H.gpu_frame(sc, cam, pl, capacity=1 << 22)
    b = H.gpu_frame(sc, cam, pl, capacity=1 << 22)
    for k in ("image", "final_T", "n_contrib", "n_walked"):
        np.testing.assert_array_equal(a[k], b[k])


def test_scratch_keys_frame_matches_sorted_keys_frame():
    """keys_scratch = 1 (the sorted 64-bit keys not written): the same lists,
    ranges, schedule and image as a frame that writes them."""
    import torch
    from paper_2506_20202_amd import renderer as R
    sc = _dense_scene(2, 6000, 0.05, -2.5)
    cam = scenes.small_camera(100)
    pl = scenes.Plane(DENSE_NORMAL, 0.02)
    dev = torch.device("cuda:0")
    ds = R.DeviceScene.from_scene(sc, dev)
    outs = []
    for sorted_keys in (True, False):
        fr = R.Frame(sc.n, cam.width, cam.height, 1 << 22, dev, sorted_keys=sorted_keys)
        fr.bins.keys.fill_(-1)
        out = R.render_checked(ds, fr, cam, pl)
        outs.append((fr, H.collect(fr, out, sc.n)))
    (fa, a), (fb, b) = outs
    H.check_ranges(a)
    P = a["P"]
    assert P == b["P"] and P > 0
    for k in ("vals", "ranges", "image", "final_T", "n_contrib", "n_walked"):
        np.testing.assert_array_equal(a[k], b[k])
    np.testing.assert_array_equal(fa.bins.work.cpu().numpy(), fb.bins.work.cpu().numpy())


@pytest.mark.parametrize("mode", [0, oracle.CLIP_RARA, oracle.CLIP_RARA | oracle.CLIP_TIGHT])
def test_degenerate_gaussians(mode):
    """Gaussians behind the camera, at the camera centre, on both sides of the
    near plane, with a zero quaternion, a zero scale or a 1e-6 scale, one
    centred on the clip plane: labels, culling, lists and image as the oracle
    decides, with the rest of the scene unchanged."""
    sc = scenes.tiny_scene(3, n=200)
    cam = scenes.tiny_camera()
    pl0 = scenes.tiny_plane(3)
    mean, quat, scale = sc.mean.copy(), sc.quat.copy(), sc.scale.copy()
    eye = np.array([0.0, 0.0, -3.0], np.float32)
    mean[:, 0] = [0.0, 0.0, -4.0]          # behind the camera
    mean[:, 1] = eye                       # at the camera centre
    mean[:, 2] = [0.0, 0.0, -2.81]         # just inside the near plane (z = 0.19)
    mean[:, 3] = [0.05, 0.0, -2.79]        # just beyond it (z = 0.21)
    quat[:, 4] = 0.0                       # zero quaternion
    scale[:, 5] = 0.0                      # zero scale
    scale[:, 6] = 1e-6
    n = np.asarray(pl0.n, np.float64)
    mean[:, 7] = (-pl0.d * n).astype(np.float32)   # centred on the plane
    sc2 = scenes.Scene(mean, scale, quat, sc.opacity, sc.sh, sc.sh_degree)
    g, o = _full_check(sc2, cam, scenes.Plane(pl0.n, pl0.d, enabled=mode))
    np.testing.assert_array_equal(g["label"][:8], o["label"][:8])
    np.testing.assert_array_equal(g["tiles_touched"][:8], o["proj"]["tiles_touched"][:8])
    assert np.isfinite(g["image"]).all()


def test_pipelined_general_1080p_equals_alone():
    """The configuration the bench times -- the 1M-Gaussian general scene at
    1920x1080 through the three-stream frame pipeline, render-only frames
    (scratch keys, no pair starts) -- renders each frame bit-identically to a
    single frame with sorted keys.  The first pick is the frame that
    test_general_scene_1080p_sampled checks against the oracle."""
    import torch
    from paper_2506_20202_amd import renderer as R
    dev = torch.device("cuda:0")
    sc = scenes.general_scene(1)
    cams = scenes.general_views()
    planes = scenes.plane_sweep(sc, scenes.general_plane_normal(1))
    picks = [(cams[0], planes[8]), (cams[3], planes[2]), (cams[7], planes[12]), (cams[11], planes[5]),
             (cams[0], planes[8]), (cams[15], planes[0]), (cams[5], scenes.Plane(planes[8].n, planes[8].d, 0))]
    ds = R.DeviceScene.from_scene(sc, dev)
    W, H = cams[0].width, cams[0].height
    fr = R.Frame(sc.n, W, H, 12_000_000, dev)
    refs, maxp = [], 0
    for cam, pl in picks:
        out = R.render_checked(ds, fr, cam, pl)
        torch.cuda.synchronize()
        refs.append(out.image.clone())
        maxp = max(maxp, int(fr.bins.num_pairs.item()))
    del fr
    pipe = R.FramePipeline(ds, W, H, int(maxp * 1.05) + 4096, streams=3, walked=False)
    got = []
    for cam, pl in picks:
        pipe.submit(cam, pl, consume=lambda f: got.append(f.out.image.clone()))
    pipe.join()
    torch.cuda.synchronize()
    assert not pipe.overflowed()
    pipe.close()
    for k, (a, b) in enumerate(zip(got, refs)):
        assert torch.equal(a, b), f"frame {k} differs"


def test_schedule_over_many_tiles():
    """A frame of 147 x 147 = 21609 tiles: the plan kernel takes three blocks of
    8192 tiles, and long lists fall in more than one of them.  Ranges and the
    schedule are checked against the sorted keys (no oracle render)."""
    sc = scenes.small_scene(5, n=40_000, spread=0.8, logscale_mean=-3.0)
    cam = scenes.tiny_camera(2352, 2352)
    off = scenes.Plane(scenes.tiny_plane(5).n, 0.0, False)
    g = H.gpu_frame(sc, cam, off, capacity=1 << 24)
    assert g["overflow"] == 0
    H.check_ranges(g)   # also the schedule
    lens = g["ranges"][:, 1] - g["ranges"][:, 0]
    long_tiles = np.nonzero(lens >= H.HEAVY_LIST)[0]
    print(f"P={g['P']} tiles={len(lens)} long={len(long_tiles)}", flush=True)
    assert len(lens) == 147 * 147
    assert len(np.unique(long_tiles // 8192)) >= 2


def _scene_with_sh_layout(sc, dev, layout, aligned=True):
    """sc on the device with its SH in `layout`; aligned=False puts a
    Gaussian-major array 4 bytes past a 16-byte boundary (the kernels then
    read it a float at a time)."""
    import torch
    from paper_2506_20202_amd import binding as B
    from paper_2506_20202_amd import renderer as R
    ds = R.DeviceScene.from_scene(sc, dev, sh_layout=layout)
    if layout == B.SH_GAUSSIAN_MAJOR and not aligned:
        buf = torch.zeros(ds.sh.numel() + 1, dtype=torch.float32, device=dev)
        buf[1:] = ds.sh.reshape(-1)
        ds.sh = buf[1:].view(ds.sh.shape)
        assert ds.sh.data_ptr() % 16 != 0
    return ds


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_sh_layouts_give_identical_frames(deg):
    """The coefficient-major and the Gaussian-major SH layouts (16-byte aligned
    or not) give bit-identical projected splats and frames; the frame also
    matches the oracle."""
    import torch
    from paper_2506_20202_amd import binding as B
    dev = torch.device("cuda:0")
    sc, cam, pl = scenes.grad_scene(7, n=400, sh_degree=deg), scenes.grad_camera(96), scenes.grad_plane(7)
    print(f"deg={deg} n={sc.n}", flush=True)
    ref = H.gpu_frame(sc, cam, pl, dscene=_scene_with_sh_layout(sc, dev, B.SH_COEFF_MAJOR))
    for aligned in (True, False):
        g = H.gpu_frame(sc, cam, pl, dscene=_scene_with_sh_layout(sc, dev, B.SH_GAUSSIAN_MAJOR, aligned))
        for k in ("label", "tiles_touched", "vals", "ranges", "image", "final_T", "n_contrib"):
            np.testing.assert_array_equal(g[k], ref[k], err_msg=f"{k} aligned={aligned}")
        # the per-Gaussian records are written for drawn Gaussians only
        drawn = ref["tiles_touched"] > 0
        assert drawn.any()
        for k in ["rect", "depth"] + [k for k in ref if k.startswith("splat_")]:
            np.testing.assert_array_equal(g[k][drawn], ref[k][drawn], err_msg=f"{k} aligned={aligned}")
    o = oracle.render(sc, cam, pl)
    H.check_projection(ref, o)
    err, flagged, _ = H.image_error(ref["image"], o)
    assert err <= TOL and flagged < 0.05
