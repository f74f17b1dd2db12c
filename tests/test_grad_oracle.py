"""The gradient oracle (torch float64 autograd of the oracle's forward):
its forward equals the C oracle and its gradient equals central finite
differences of that forward, parameter by parameter."""
import numpy as np
import pytest
import torch

import oracle
from oracle import torch_ref as TR
from paper_2506_20202_amd import scenes


def _setup(seed=4):
    sc = scenes.grad_scene(seed)
    cam = scenes.grad_camera()
    pl = scenes.grad_plane(seed)
    return sc, cam, pl


@pytest.mark.parametrize("which", ["tiny", "grad"])
def test_torch_forward_equals_c_oracle(which):
    if which == "tiny":
        sc, cam, pl = scenes.tiny_scene(1), scenes.tiny_camera(), scenes.tiny_plane(1)
    else:
        sc, cam, pl = _setup()
    o = oracle.render(sc, cam, pl)
    st = TR.structure(sc, cam, pl)
    img = TR.render(TR.params_from_scene(sc, pl, requires_grad=False), sc, cam, pl.enabled, st)
    ok = o["flags"] == 0
    err = np.abs(img.numpy() - o["image"]).max(axis=0)
    assert err[ok].max() < 1e-10


def test_gradient_matches_central_differences():
    sc, cam, pl = _setup()
    st = TR.structure(sc, cam, pl)
    assert (st["label"] == oracle.CUTOFF).sum() >= 20
    rng = np.random.default_rng(0)
    wimg = torch.tensor(rng.normal(size=(3, cam.height, cam.width)))
    p = TR.params_from_scene(sc, pl)
    img, aux0 = TR.render(p, sc, cam, pl.enabled, st, aux=True)
    (img * wimg).sum().backward()
    # parameters of Gaussians that are drawn; a few per group
    drawn = np.nonzero(st["drawn"])[0]
    cut = np.nonzero(st["drawn"] & (st["label"] == oracle.CUTOFF))[0]
    picks = []
    for name, rows in [("mean", 3), ("scale", 3), ("quat", 4), ("opacity", 0), ("sh", 0)]:
        for _ in range(8):
            g = int(rng.choice(cut if rng.random() < 0.5 else drawn))
            if name == "opacity":
                picks.append((name, (g,)))
            elif name == "sh":
                picks.append((name, (int(rng.integers(16)), int(rng.integers(3)), g)))
            else:
                picks.append((name, (int(rng.integers(rows)), g)))
    for k in range(4):
        picks.append(("plane", (k,)))
    checked = 0
    for name, ix in picks:
        base = {k: v.detach().clone() for k, v in p.items()}
        th = float(base[name][ix])
        h = 1e-6 * max(1.0, abs(th))
        vals = []
        auxs = []
        for sgn in (1, -1):
            q = {k: v.clone() for k, v in base.items()}
            q[name][ix] = th + sgn * h
            im, ax = TR.render(q, sc, cam, pl.enabled, st, aux=True)
            vals.append(float((im * wimg).sum()))
            auxs.append(ax)
        if any(not torch.equal(auxs[0][k], auxs[1][k]) for k in ("keep", "two", "clamp", "colclip")):
            continue   # the perturbation crosses a discontinuity of the forward
        fd = (vals[0] - vals[1]) / (2 * h)
        ad = float(p[name].grad[ix])
        assert abs(fd - ad) <= 1e-5 * max(1.0, abs(ad)), (name, ix, fd, ad)
        checked += 1
    assert checked >= 30
