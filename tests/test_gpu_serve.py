"""GPU serving: captured frame graphs replay the eager frame exactly, and every
request served in a mix equals the same request rendered alone, bit for bit."""
import numpy as np
import pytest
import torch

from paper_2506_20202_amd import renderer as R
from paper_2506_20202_amd import scenes
from paper_2506_20202_amd.serve import Engine

pytestmark = pytest.mark.gpu


def _alone(ds, cam, pl, bg=(0.0, 0.0, 0.0)):
    fr = R.Frame(ds.n, cam.width, cam.height, 1 << 20, torch.device("cuda:0"), walked=False)
    out = R.render_checked(ds, fr, cam, pl, bg)
    return out.image.clone()


def test_frame_graph_replays_match_eager():
    dev = torch.device("cuda:0")
    sc = scenes.multilayer_scene(5, per_shell=4000, sh_degree=2)
    ds = R.DeviceScene.from_scene(sc, dev)
    rng = np.random.default_rng(5)
    W, H = 192, 160
    fr = R.Frame(sc.n, W, H, 1 << 20, dev, walked=False)
    g = R.FrameGraph(ds, fr, scenes.pinhole((0.0, 0.0, -5.0), (0, 0, 0), W, H, 50.0))
    try:
        for k in range(5):
            cam = scenes.random_camera_on_sphere(rng, 5.0, W, H)
            pl = scenes.random_plane_through(rng, sc)
            if k == 3:
                pl = scenes.Plane(pl.n, pl.d, enabled=False)
            ref = _alone(ds, cam, pl, (0.1, 0.2, 0.3))
            torch.cuda.synchronize()
            g.launch(cam, pl, (0.1, 0.2, 0.3))
            torch.cuda.synchronize()
            assert int(fr.bins.overflow.item()) == 0
            assert torch.equal(fr.out.image, ref), f"replay {k} differs"
            # unrelated eager work between replays
            _ = (torch.randn(1 << 16, device=dev) * 2).sum().item()
    finally:
        g.close()


def _mixed_requests(rng, names_scenes, n_req):
    sizes = [(128, 128), (256, 192), (320, 320)]
    reqs = []
    for _ in range(n_req):
        name, sc = names_scenes[int(rng.integers(len(names_scenes)))]
        W, H = sizes[int(rng.integers(len(sizes)))]
        cam = scenes.random_camera_on_sphere(rng, 5.0, W, H)
        pl = scenes.random_plane_through(rng, sc)
        reqs.append((name, cam, pl))
    return reqs


@pytest.mark.parametrize("use_graphs", [True, False])
def test_served_results_equal_alone(use_graphs):
    rng = np.random.default_rng(11)
    ns = [("A", scenes.multilayer_scene(3, per_shell=3000, sh_degree=0)),
          ("B", scenes.multilayer_scene(4, per_shell=4000, sh_degree=2)),
          ("C", scenes.multilayer_scene(6, per_shell=5000, sh_degree=3))]
    eng = Engine(hbm_budget=2 << 30, max_slots=6, use_graphs=use_graphs)
    for name, sc in ns:
        eng.add_scene(name, sc)
    reqs = _mixed_requests(rng, ns, 24)
    futs = [eng.submit(*r) for r in reqs]          # all queued at once: the slots overlap on the device
    eng.run_until_idle(timeout=300)
    st = eng.stats()
    print(f"graphs={use_graphs} stats={st}", flush=True)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["max_inflight"] >= 2
    bad = []
    for k, ((name, cam, pl), f) in enumerate(zip(reqs, futs)):
        img, ref = f.result(timeout=0), _alone(eng.ex.scenes[name], cam, pl)
        if not torch.equal(img, ref):
            d = (img - ref).abs()
            bad.append((k, name, cam.width, cam.height, float(d.max()), int((d > 0).sum())))
    eng.close()
    assert not bad, f"served != alone for (request, scene, W, H, max diff, differing values): {bad}"


def test_overflow_is_retried_with_larger_capacity():
    rng = np.random.default_rng(12)
    sc = scenes.multilayer_scene(7, per_shell=3000, sh_degree=1)
    eng = Engine(hbm_budget=2 << 30, max_slots=2, capacity_of=lambda shape: 256)
    eng.add_scene("A", sc)
    reqs = _mixed_requests(rng, [("A", sc)], 4)
    futs = [eng.submit(*r) for r in reqs]
    eng.run_until_idle(timeout=300)
    st = eng.stats()
    print(f"stats={st} hints={eng.sched.capacity_hint}", flush=True)
    assert st["retries"] >= 1 and st["completed"] == 4
    bad = []
    for k, ((name, cam, pl), f) in enumerate(zip(reqs, futs)):
        img, ref = f.result(timeout=0), _alone(eng.ex.scenes[name], cam, pl)
        if not torch.equal(img, ref):
            d = (img - ref).abs()
            bad.append((k, cam.width, cam.height, float(d.max()), int((d > 0).sum())))
    eng.close()
    assert not bad, f"served != alone for (request, W, H, max diff, differing values): {bad}"


@pytest.mark.parametrize("streams", [1, 2, 3])
def test_pipelined_frames_equal_alone(streams):
    """FramePipeline (consecutive frames in flight on their own streams, each
    buffer set reused every `streams` frames): every frame's image, copied out
    through the consume hook, equals the frame rendered alone."""
    dev = torch.device("cuda:0")
    sc = scenes.multilayer_scene(3, per_shell=20000, sh_degree=1)
    ds = R.DeviceScene.from_scene(sc, dev)
    rng = np.random.default_rng(17 + streams)
    W, H = 256, 192
    frames = []
    for k in range(11):
        cam = scenes.random_camera_on_sphere(rng, 5.0, W, H)
        pl = scenes.random_plane_through(rng, sc)
        if k == 4:
            pl = scenes.Plane(pl.n, pl.d, enabled=False)
        frames.append((cam, pl))
    refs = [_alone(ds, cam, pl) for cam, pl in frames]
    torch.cuda.synchronize()
    pipe = R.FramePipeline(ds, W, H, 1 << 20, streams=streams, walked=False)
    got = []
    for cam, pl in frames:
        pipe.submit(cam, pl, consume=lambda f: got.append(f.out.image.clone()))
    pipe.join()
    torch.cuda.synchronize()
    assert not pipe.overflowed()
    pipe.close()
    for k, (a, b) in enumerate(zip(got, refs)):
        assert torch.equal(a, b), f"frame {k} differs"
