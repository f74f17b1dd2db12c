"""GPU gradients (rara_render_backward through the autograd Function) against
the float64 autograd gradient of the oracle forward.

Bar per parameter group (mean, scale, quat, opacity, SH, plane): relative L2
error <= 5e-3 and cosine similarity >= 0.9999.  The loss is a fixed random
linear functional of the image, zeroed on pixels the oracle flags as
discontinuity events (where the float32 forward may take the other branch).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import torch_ref as TR
from paper_2506_20202_amd import scenes

pytestmark = pytest.mark.gpu


def _grads_gpu(sc, cam, pl, wimg, bg=(0.0, 0.0, 0.0)):
    from paper_2506_20202_amd import autograd as AG
    dev = torch.device("cuda:0")
    t = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device=dev, requires_grad=True)
    mean, scale, quat, op, sh = t(sc.mean), t(sc.scale), t(sc.quat), t(sc.opacity), t(sc.sh)
    plane4 = torch.tensor([pl.n[0], pl.n[1], pl.n[2], pl.d], dtype=torch.float32, requires_grad=True)
    img = AG.render(mean, scale, quat, op, sh, plane4, cam, pl.enabled, bg)
    loss = (img * torch.tensor(wimg, dtype=torch.float32, device=dev)).sum()
    loss.backward()
    return dict(mean=mean.grad.cpu().numpy(), scale=scale.grad.cpu().numpy(), quat=quat.grad.cpu().numpy(),
                opacity=op.grad.cpu().numpy(), sh=sh.grad.cpu().numpy(), plane=plane4.grad.numpy()), img


def _grads_ref(sc, cam, pl, wimg, bg=(0.0, 0.0, 0.0)):
    st = TR.structure(sc, cam, pl)
    p = TR.params_from_scene(sc, pl)
    img = TR.render(p, sc, cam, pl.enabled, st, bg=bg)
    (img * torch.tensor(wimg)).sum().backward()
    return {k: (v.grad.numpy() if v.grad is not None else np.zeros(v.shape)) for k, v in p.items()}, img


def _compare(g, r, groups):
    for k in groups:
        a, b = g[k].astype(np.float64).reshape(-1), r[k].reshape(-1)
        nb = np.linalg.norm(b)
        if nb == 0.0:   # an exactly zero reference gradient (e.g. no partial clip weight anywhere)
            print(f"  {k:8s} |ref|=0 |gpu|={np.linalg.norm(a):.3e}", flush=True)
            assert np.all(a == 0.0), k
            continue
        rel = np.linalg.norm(a - b) / max(nb, 1e-30)
        cos = float(a @ b / max(np.linalg.norm(a) * nb, 1e-30))
        print(f"  {k:8s} |ref|={nb:.3e} rel_l2={rel:.2e} cos={cos:.7f}", flush=True)
        assert rel <= 5e-3, (k, rel)
        assert cos >= 0.9999, (k, cos)


@pytest.mark.parametrize("seed", [4, 5, 6])
def test_clipped_gradients_match_oracle(seed):
    sc, cam, pl = scenes.grad_scene(seed), scenes.grad_camera(), scenes.grad_plane(seed)
    o = oracle.render(sc, cam, pl)
    rng = np.random.default_rng(seed)
    wimg = rng.normal(size=(3, cam.height, cam.width)) * (o["flags"] == 0)[None]
    g, img = _grads_gpu(sc, cam, pl, wimg)
    r, rimg = _grads_ref(sc, cam, pl, wimg)
    ok = o["flags"] == 0
    assert np.abs(img.detach().cpu().numpy() - rimg.detach().numpy()).max(0)[ok].max() < 1e-3
    print(f"seed {seed}: cutoff={(o['label'] == 2).sum()}", flush=True)
    _compare(g, r, ["mean", "scale", "quat", "opacity", "sh", "plane"])


def test_plain_gradients_match_oracle():
    sc, cam = scenes.grad_scene(7), scenes.grad_camera()
    pl = scenes.Plane(np.array([0, 0, 1], np.float32), 0.0, enabled=False)
    o = oracle.render(sc, cam, pl)
    rng = np.random.default_rng(7)
    wimg = rng.normal(size=(3, cam.height, cam.width)) * (o["flags"] == 0)[None]
    g, _ = _grads_gpu(sc, cam, pl, wimg, bg=(0.1, 0.2, 0.3))
    r, _ = _grads_ref(sc, cam, pl, wimg, bg=(0.1, 0.2, 0.3))
    _compare(g, r, ["mean", "scale", "quat", "opacity", "sh"])
    assert np.all(g["plane"] == 0)


def _check_case(sc, cam, pl, seed, min_unflagged=0.5, bg=(0.0, 0.0, 0.0)):
    o = oracle.render(sc, cam, pl, bg=bg)
    ok = o["flags"] == 0
    assert ok.mean() >= min_unflagged, ok.mean()
    rng = np.random.default_rng(seed)
    wimg = rng.normal(size=(3, cam.height, cam.width)) * ok[None]
    g, img = _grads_gpu(sc, cam, pl, wimg, bg)
    r, rimg = _grads_ref(sc, cam, pl, wimg, bg)
    assert np.abs(img.detach().cpu().numpy() - rimg.detach().numpy()).max(0)[ok].max() < 1e-3
    groups = ["mean", "scale", "quat", "opacity", "sh"] + (["plane"] if pl.enabled else [])
    _compare(g, r, groups)
    return o, g


@pytest.mark.parametrize("seed", [0, 1])
def test_wide_gaussian_gradients_match_oracle(seed):
    """Gaussians spanning more than 32 tiles, whose pair slots the backward
    sums with a whole wave instead of one thread, at 128x128 (64 tiles), most
    of them CUTOFF, among 150 general-scene Gaussians."""
    cam = scenes.grad_camera(128)
    sc = scenes.concat(scenes.grad_scene(10 + seed, n=150), scenes.wide_gaussians(seed))
    pl = scenes.grad_plane(10 + seed)
    o, _ = _check_case(sc, cam, pl, 100 + seed)
    tt = o["proj"]["tiles_touched"]
    print(f"wide seed {seed}: Gaussians over 32 tiles: {(tt > 32).sum()}, largest {tt.max()}", flush=True)
    assert (tt > 32).sum() >= 5
    assert (o["label"][tt > 32] == oracle.CUTOFF).sum() >= 5


@pytest.mark.parametrize("clipped", [False, True])
def test_long_faint_list_gradients_match_oracle(clipped):
    """Tile lists of 1500 faint entries (alpha about 0.005), every one of them
    composited: the backward rebuilds the transmittance by division over the
    whole list.  Clipped: a plane that leaves partial weights on the CUTOFF
    entries (the final transmittance rises from 1.7e-4 to 4.5e-4)."""
    cam = scenes.faint_camera()
    sc = scenes.faint_list_scene(0)
    nrm = np.array([0.2, 0.3, 1.0])
    pl = scenes.Plane((nrm / np.linalg.norm(nrm)).astype(np.float32), 1.8, enabled=clipped)
    o, _ = _check_case(sc, cam, pl, 7 + int(clipped))
    ok = o["flags"] == 0
    lens = np.diff(o["offsets"])
    print(f"faint list clipped={clipped}: list lengths {lens.min()}-{lens.max()}, n_contrib on checked pixels "
          f"{o['n_contrib'][ok].min()}-{o['n_contrib'][ok].max()}, T min {o['final_T'].min():.2e}", flush=True)
    assert lens.min() >= 1500
    assert o["n_contrib"][ok].min() >= 1500


@pytest.mark.parametrize("normal", [(0.3, -0.5, 0.8), (1.0, 0.2, 0.1)])
def test_camera_inside_gradients_match_oracle(normal):
    """A CUTOFF Gaussian holding the camera inside its 3-sigma ellipsoid (the
    near root behind the camera, w = 1 on every pixel ray: eq. (11)'s
    "otherwise" case) in front of 150 general-scene Gaussians."""
    cam = scenes.grad_camera(64)
    ins = scenes.inside_gaussian(cam)
    sc = scenes.concat(scenes.grad_scene(21, n=150), ins)
    pl = scenes.plane_through(ins.mean[:, 0], normal)
    o, g = _check_case(sc, cam, pl, 31)
    assert o["label"][-1] == oracle.CUTOFF
    assert o["counters"][4] >= cam.width * cam.height * 0.99
    if (o["label"] == oracle.CUTOFF).sum() == 1:
        # the camera-inside Gaussian is the only CUTOFF one: w = 1 on every ray,
        # so nothing depends on the plane
        assert np.all(g["plane"] == 0.0)


def test_backward_of_an_overflowed_frame_is_zero():
    """rara_render_backward on a frame whose pair capacity overflowed writes
    zero to every gradient (the pair slots and pair starts of such a frame
    are incomplete and are not read)."""
    from paper_2506_20202_amd import binding as B
    from paper_2506_20202_amd import renderer as R
    dev = torch.device("cuda:0")
    sc, cam, pl = scenes.grad_scene(4), scenes.grad_camera(), scenes.grad_plane(4)
    o = oracle.render(sc, cam, pl, events=False)
    P = len(o["ids"])
    ds = R.DeviceScene.from_scene(sc, dev)
    fr = R.Frame(sc.n, cam.width, cam.height, P // 2, dev, walked=False)
    fr.out.final_T.fill_(0.5)
    fr.out.n_contrib.fill_(3)
    R.enqueue_frame(ds, fr, cam, pl)
    torch.cuda.synchronize()
    assert int(fr.bins.overflow.item()) == 1
    g = {k: torch.full_like(getattr(ds, k), float("nan")) for k in ("mean", "scale", "quat", "opacity", "sh")}
    dplane = torch.full((4,), float("nan"), dtype=torch.float32, device=dev)
    gs = B.Grads()
    gs.mean, gs.scale, gs.quat = g["mean"].data_ptr(), g["scale"].data_ptr(), g["quat"].data_ptr()
    gs.opacity, gs.sh, gs.plane = g["opacity"].data_ptr(), g["sh"].data_ptr(), dplane.data_ptr()
    ws_bytes = B.workspace_bytes(B.RARA_WS_BACKWARD, sc.n, fr.capacity, cam.width, cam.height)
    ws = torch.full((ws_bytes,), 0xAB, dtype=torch.uint8, device=dev)
    dimg = torch.ones((3, cam.height, cam.width), dtype=torch.float32, device=dev)
    stream = int(torch.cuda.current_stream(dev).cuda_stream)
    B.render_backward(ds.struct(), B.make_camera(cam), B.make_plane(pl), (0.0, 0.0, 0.0), fr.proj.struct(),
                      fr.bins.struct(), fr.capacity, fr.out.final_T.data_ptr(), fr.out.n_contrib.data_ptr(),
                      dimg.data_ptr(), gs, ws.data_ptr(), ws_bytes, stream)
    torch.cuda.synchronize()
    for k, v in g.items():
        assert bool((v == 0).all()), k
    assert bool((dplane == 0).all())


def test_pair_starts_stay_within_the_pairs():
    """For a frame that fits, every drawn Gaussian's pair slots
    [pair_start, pair_start + tiles_touched) lie inside [0, num_pairs): the
    bound the backward's slot reads rely on."""
    from paper_2506_20202_amd import renderer as R
    dev = torch.device("cuda:0")
    for sc, cam, pl in ((scenes.grad_scene(4), scenes.grad_camera(), scenes.grad_plane(4)),
                        (scenes.tiny_scene(1), scenes.tiny_camera(), scenes.tiny_plane(1))):
        ds = R.DeviceScene.from_scene(sc, dev)
        fr = R.Frame(sc.n, cam.width, cam.height, 1 << 16, dev, walked=False)
        R.render_checked(ds, fr, cam, pl)
        P = int(fr.bins.num_pairs.item())
        tt = fr.proj.tiles_touched[: sc.n].cpu().numpy().view(np.uint32).astype(np.int64)
        ps = fr.bins.pair_start[: sc.n].cpu().numpy().view(np.uint32).astype(np.int64)
        drawn = tt > 0
        assert drawn.any()
        assert (ps[drawn] + tt[drawn] <= P).all()
        # the slots of the drawn Gaussians tile [0, P) exactly
        cover = np.zeros(P, np.int64)
        for a, b in zip(ps[drawn], tt[drawn]):
            cover[a:a + b] += 1
        assert (cover == 1).all()


def test_differentiable_batch_full_size():
    """The 500k-Gaussian, 8 views x 800x800 differentiable workload: L2 loss
    against a perturbed-scene target; gradients finite, zero for Gaussians no
    view draws, and a gradient step along -grad lowers the loss."""
    from paper_2506_20202_amd import autograd as AG
    dev = torch.device("cuda:0")
    sc = scenes.general_scene(4, n=500_000)
    cams, planes = scenes.diff_views(scene=sc)
    tgt = scenes.perturbed(sc)
    t = lambda a, g=True: torch.tensor(np.asarray(a), dtype=torch.float32, device=dev, requires_grad=g)
    with torch.no_grad():
        targets = []
        for cam, pl in zip(cams, planes):
            p4 = torch.tensor([pl.n[0], pl.n[1], pl.n[2], pl.d])
            targets.append(AG.render(t(tgt.mean, False), t(tgt.scale, False), t(tgt.quat, False),
                                     t(tgt.opacity, False), t(tgt.sh, False), p4, cam, True))
    params = [t(sc.mean), t(sc.scale), t(sc.quat), t(sc.opacity), t(sc.sh)]

    def loss_fn(ps):
        tot = 0.0
        for cam, pl, tg in zip(cams, planes, targets):
            p4 = torch.tensor([pl.n[0], pl.n[1], pl.n[2], pl.d], requires_grad=True)
            img = AG.render(*ps, p4, cam, True)
            tot = tot + ((img - tg) ** 2).mean()
        return tot / len(cams)

    L0 = loss_fn(params)
    L0.backward()
    for p in params:
        assert torch.isfinite(p.grad).all()
    gn = sum(float((p.grad ** 2).sum()) for p in params)
    assert gn > 0
    with torch.no_grad():
        step = 1e-3 / np.sqrt(gn)
        moved = [(p - step * p.grad).detach() for p in params]
        L1 = loss_fn(moved)
    print(f"diff batch: L0={float(L0):.6e} L1={float(L1):.6e} |g|={np.sqrt(gn):.3e}", flush=True)
    assert float(L1) < float(L0)


def _frame_gradients(ds, sc, cam, pl, dimg):
    """Forward, then rara_render_backward of the image gradient dimg, through
    the C ABI; the gradients in the layout of ds."""
    from paper_2506_20202_amd import binding as B
    from paper_2506_20202_amd import renderer as R
    dev = ds.mean.device
    fr = R.Frame(sc.n, cam.width, cam.height, 1 << 16, dev, walked=False)
    R.render_checked(ds, fr, cam, pl)
    g = {k: torch.full_like(getattr(ds, k), float("nan")) for k in ("mean", "scale", "quat", "opacity", "sh")}
    dplane = torch.full((4,), float("nan"), dtype=torch.float32, device=dev)
    gs = B.Grads()
    gs.mean, gs.scale, gs.quat = g["mean"].data_ptr(), g["scale"].data_ptr(), g["quat"].data_ptr()
    gs.opacity, gs.sh, gs.plane = g["opacity"].data_ptr(), g["sh"].data_ptr(), dplane.data_ptr()
    ws_bytes = B.workspace_bytes(B.RARA_WS_BACKWARD, sc.n, fr.capacity, cam.width, cam.height)
    ws = torch.zeros((ws_bytes,), dtype=torch.uint8, device=dev)
    stream = int(torch.cuda.current_stream(dev).cuda_stream)
    B.render_backward(ds.struct(), B.make_camera(cam), B.make_plane(pl), (0.0, 0.0, 0.0), fr.proj.struct(),
                      fr.bins.struct(), fr.capacity, fr.out.final_T.data_ptr(), fr.out.n_contrib.data_ptr(),
                      dimg.data_ptr(), gs, ws.data_ptr(), ws_bytes, stream)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in g.items()}
    out["plane"] = dplane.cpu().numpy()
    return out


@pytest.mark.parametrize("deg", [1, 3])
def test_sh_layouts_give_identical_gradients(deg):
    """rara_render_backward gives the same gradients for the coefficient-major
    and the Gaussian-major SH layouts (16-byte aligned or not); the SH
    gradient comes back in the layout of the input.  Equal to float rounding,
    not bit for bit: the four quadrant waves of a tile add a pair's sums with
    LDS float atomics, in an order that varies from run to run."""
    from paper_2506_20202_amd import binding as B
    from paper_2506_20202_amd import renderer as R
    dev = torch.device("cuda:0")
    sc, cam, pl = scenes.grad_scene(5, sh_degree=deg), scenes.grad_camera(), scenes.grad_plane(5)
    print(f"deg={deg} n={sc.n}", flush=True)
    dimg = torch.from_numpy(np.random.default_rng(3).normal(0.0, 1.0, (3, cam.height, cam.width))).to(
        device=dev, dtype=torch.float32).contiguous()
    ref = _frame_gradients(R.DeviceScene.from_scene(sc, dev), sc, cam, pl, dimg)
    assert np.isfinite(ref["sh"]).all() and np.abs(ref["sh"]).max() > 0
    for aligned in (True, False):
        ds = R.DeviceScene.from_scene(sc, dev, sh_layout=B.SH_GAUSSIAN_MAJOR)
        if not aligned:
            buf = torch.zeros(ds.sh.numel() + 1, dtype=torch.float32, device=dev)
            buf[1:] = ds.sh.reshape(-1)
            ds.sh = buf[1:].view(ds.sh.shape)
        got = _frame_gradients(ds, sc, cam, pl, dimg)
        want = dict(ref, sh=np.transpose(ref["sh"], (2, 0, 1)))
        for k in ("mean", "scale", "quat", "opacity", "plane", "sh"):
            assert got[k].shape == want[k].shape, k
            bound = 1e-5 * float(np.abs(want[k]).max())
            diff = float(np.abs(got[k].astype(np.float64) - want[k]).max())
            assert diff <= bound, (k, aligned, diff, bound)


def test_deferred_overflow_check_gives_the_same_gradients():
    """render(check=False) only enqueues the frame: images and gradients equal
    those of the checked render (to the backward's float-atomic rounding), and
    overflowed() reads the flags of several frames at once, true for a frame
    whose pair capacity is too small."""
    from paper_2506_20202_amd import autograd as AG
    from paper_2506_20202_amd import renderer as R
    dev = torch.device("cuda:0")
    sc, cam, pl = scenes.grad_scene(6), scenes.grad_camera(), scenes.grad_plane(6)
    p4 = torch.tensor([float(pl.n[0]), float(pl.n[1]), float(pl.n[2]), float(pl.d)])

    def run(check):
        ps = [torch.tensor(np.asarray(a), dtype=torch.float32, device=dev, requires_grad=True)
              for a in (sc.mean, sc.scale, sc.quat, sc.opacity, sc.sh)]
        fr = R.Frame(sc.n, cam.width, cam.height, 1 << 16, dev, walked=False, sorted_keys=False)
        img = AG.render(*ps, p4, cam, True, frame=fr, check=check)
        (img ** 2).mean().backward()
        assert not AG.overflowed([fr])
        return img.detach().cpu().numpy(), [p.grad.cpu().numpy() for p in ps]

    img0, g0 = run(True)
    img1, g1 = run(False)
    np.testing.assert_array_equal(img1, img0)
    for a, b in zip(g1, g0):
        assert np.abs(a.astype(np.float64) - b).max() <= 1e-5 * np.abs(b).max()
    o = oracle.render(sc, cam, pl, events=False)
    small = R.Frame(sc.n, cam.width, cam.height, max(1, len(o["ids"]) // 2), dev, walked=False, sorted_keys=False)
    ok = R.Frame(sc.n, cam.width, cam.height, 1 << 16, dev, walked=False, sorted_keys=False)
    ds = R.DeviceScene.from_scene(sc, dev)
    R.enqueue_frame(ds, ok, cam, pl)
    R.enqueue_frame(ds, small, cam, pl)
    assert AG.overflowed([ok, small]) and not AG.overflowed([ok])
