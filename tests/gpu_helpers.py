"""Helpers shared by the GPU tests: run one frame through the C ABI and bring
every output back to the host, and compare with the oracle."""
from __future__ import annotations

import numpy as np
import torch

from paper_2506_20202_amd import renderer as R

TILE = 16


def gpu_frame(scene, cam, plane, bg=(0.0, 0.0, 0.0), capacity=None, dscene=None):
    dev = torch.device("cuda:0")
    ds = dscene if dscene is not None else R.DeviceScene.from_scene(scene, dev)
    cap = capacity if capacity is not None else max(1 << 16, 64 * max(scene.n, 1))
    fr = R.Frame(scene.n, cam.width, cam.height, cap, dev)
    out = R.render_checked(ds, fr, cam, plane, bg)
    return collect(fr, out, scene.n)


def collect(fr, out, n):
    P = int(fr.bins.num_pairs.item())
    res = dict(
        P=P,
        overflow=int(fr.bins.overflow.item()),
        label=fr.proj.label[:n].cpu().numpy(),
        tiles_touched=fr.proj.tiles_touched[:n].cpu().numpy().view(np.uint32),
        rect=fr.proj.rect[: 4 * n].cpu().numpy().view(np.uint16).reshape(-1, 4).astype(np.int32),
        depth=fr.proj.depth[:n].cpu().numpy(),
        keys=fr.bins.keys[:P].cpu().numpy().view(np.uint64),
        vals=fr.bins.vals[:P].cpu().numpy().view(np.uint32),
        ranges=fr.bins.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2),
        image=out.image.cpu().numpy().astype(np.float64),
        final_T=out.final_T.cpu().numpy(),
        n_contrib=out.n_contrib.cpu().numpy(),
        n_walked=out.n_walked.cpu().numpy() if out.n_walked is not None else None,
    )
    res.update({"splat_" + k: v for k, v in R.splat_fields(fr.proj).items()})
    return res


def tile_list(res, tile):
    s, e = res["ranges"][tile]
    return res["vals"][s:e]


def check_projection(g, o, n_boundary_ok=0):
    """Labels, drawn set, rectangles, depths, projected floats."""
    lab_mis = np.nonzero(g["label"] != o["label"])[0]
    assert len(lab_mis) <= n_boundary_ok, f"label mismatches {len(lab_mis)} at {lab_mis[:10]}"
    drawn = o["proj"]["drawn"].astype(bool)
    gd = g["tiles_touched"] > 0
    both = drawn & gd
    assert (gd != drawn).sum() <= n_boundary_ok, f"drawn mismatches {(gd != drawn).sum()}"
    np.testing.assert_array_equal(g["tiles_touched"][both], o["proj"]["tiles_touched"][both])
    np.testing.assert_array_equal(g["rect"][both], o["proj"]["rect"][both])
    np.testing.assert_array_equal(g["depth"][both], o["proj"]["depth32"][both])
    np.testing.assert_allclose(g["splat_mean2d"][both], o["proj"]["mean2d"][both], rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(g["splat_conic"][both], o["proj"]["conic"][both], rtol=2e-6, atol=1e-9)
    np.testing.assert_allclose(g["splat_rgb"][both], o["proj"]["rgb"][both], rtol=2e-6, atol=1e-6)
    return both


def check_lists(g, o, tiles=None):
    """Per-tile lists identical to the oracle's (ids and order)."""
    offs, ids = o["offsets"], o["ids"]
    T = len(offs) - 1
    tiles = range(T) if tiles is None else tiles
    bad = []
    for t in tiles:
        ref = ids[offs[t]:offs[t + 1]]
        got = tile_list(g, t)
        if len(ref) != len(got) or not np.array_equal(ref, got):
            bad.append(t)
    assert not bad, f"{len(bad)} tile lists differ, first {bad[:5]}"


def image_error(g_img, o):
    """Max abs error over clamp(RGB, 0, 1) on pixels without oracle events,
    and the fraction of pixels flagged."""
    a = np.clip(g_img, 0, 1)
    b = np.clip(o["image"], 0, 1)
    err = np.abs(a - b).max(axis=0)
    ok = o["flags"] == 0
    return float(err[ok].max() if ok.any() else 0.0), float(1 - ok.mean()), err
