"""GPU serving: captured frame graphs replay the eager frame exactly, a
batched blend launch equals each frame's own rara_render, every request served
in a mix equals the same request rendered alone, bit for bit, and served
images agree with the FP64 oracle."""
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


@pytest.mark.parametrize("use_graphs,batch", [(True, False), (False, False), (False, True)])
def test_served_results_equal_alone(use_graphs, batch):
    rng = np.random.default_rng(11)
    ns = [("A", scenes.multilayer_scene(3, per_shell=3000, sh_degree=0)),
          ("B", scenes.multilayer_scene(4, per_shell=4000, sh_degree=2)),
          ("C", scenes.multilayer_scene(6, per_shell=5000, sh_degree=3))]
    eng = Engine(hbm_budget=2 << 30, max_slots=6, use_graphs=use_graphs, batch=batch)
    for name, sc in ns:
        eng.add_scene(name, sc)
    reqs = _mixed_requests(rng, ns, 24)
    futs = [eng.submit(*r) for r in reqs]          # all queued at once: the slots overlap on the device
    eng.run_until_idle(timeout=300)
    st = eng.stats()
    print(f"graphs={use_graphs} batch={batch} stats={st}", flush=True)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["max_inflight"] >= 2
    if batch:
        assert st["max_batch"] >= 2   # requests admitted together share a blend launch
    bad = []
    for k, ((name, cam, pl), f) in enumerate(zip(reqs, futs)):
        img, ref = f.result(timeout=0), _alone(eng.ex.scenes[name], cam, pl)
        if not torch.equal(img, ref):
            d = (img - ref).abs()
            bad.append((k, name, cam.width, cam.height, float(d.max()), int((d > 0).sum())))
    eng.close()
    assert not bad, f"served != alone for (request, scene, W, H, max diff, differing values): {bad}"


def test_render_batch_equals_render():
    """One rara_render_batch launch over frames of different scenes, sizes
    (ragged ones included), clip modes and backgrounds, one of them
    overflowing its pair capacity: every image, final transmittance and
    n_contrib equals rara_render's for the same frame bit for bit, and the
    overflowing frame's outputs are left untouched."""
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(21)
    scs = [scenes.multilayer_scene(8, per_shell=3000, sh_degree=1), scenes.tiny_scene(3),
           scenes.multilayer_scene(9, per_shell=6000, sh_degree=3)]
    dss = [R.DeviceScene.from_scene(sc, dev) for sc in scs]
    sizes = [(128, 128), (200, 120), (96, 160), (256, 256), (64, 48)]
    jobs, refs = [], []
    for k in range(7):
        i = k % len(scs)
        W, H = sizes[k % len(sizes)]
        cam = scenes.random_camera_on_sphere(rng, 5.0 if i != 1 else 3.0, W, H)
        pl = scenes.random_plane_through(rng, scs[i])
        if k == 2:
            pl = scenes.Plane(pl.n, pl.d, enabled=False)
        if k == 4:
            pl = scenes.Plane(pl.n, pl.d, enabled=2)   # hard clipping
        bg = (0.1 * k, 0.2, 0.3)
        cap = 64 if k == 5 else 1 << 20
        fr = R.Frame(dss[i].n, W, H, cap, dev, walked=False)
        ref = R.Frame(dss[i].n, W, H, cap, dev, walked=False)
        for f in (fr, ref):
            f.out.image.fill_(-3.0)
            f.out.final_T.fill_(-3.0)
        R.enqueue_frame(dss[i], fr, cam, pl, bg, stages=("pre", "bin"))
        R.enqueue_frame(dss[i], ref, cam, pl, bg)
        jobs.append((dss[i], fr, cam, pl, bg))
        refs.append(ref)
    R.enqueue_render_batch(jobs)
    torch.cuda.synchronize()
    for k, ((_, fr, cam, _, _), ref) in enumerate(zip(jobs, refs)):
        assert int(fr.bins.overflow.item()) == (1 if k == 5 else 0)
        if k == 5:
            assert bool((fr.out.image == -3.0).all()) and bool((fr.out.final_T == -3.0).all())
            continue
        assert torch.equal(fr.out.image, ref.out.image), f"frame {k} image"
        assert torch.equal(fr.out.final_T, ref.out.final_T), f"frame {k} final_T"
        assert torch.equal(fr.out.n_contrib, ref.out.n_contrib), f"frame {k} n_contrib"


def test_served_results_match_oracle():
    """Requests served in a mix (batched blends) against the FP64 oracle:
    image within 1e-3 on the pixels the oracle does not flag."""
    import oracle
    rng = np.random.default_rng(23)
    ns = [("A", scenes.multilayer_scene(13, per_shell=1500, sh_degree=0)),
          ("B", scenes.multilayer_scene(14, per_shell=2500, sh_degree=3))]
    eng = Engine(hbm_budget=2 << 30, max_slots=6)
    for name, sc in ns:
        eng.add_scene(name, sc)
    reqs = []
    for k in range(6):
        name, sc = ns[k % 2]
        W, H = [(128, 128), (160, 120), (96, 96)][k % 3]
        reqs.append((name, sc, scenes.random_camera_on_sphere(rng, 5.0, W, H), scenes.random_plane_through(rng, sc)))
    futs = [eng.submit(name, cam, pl) for name, _, cam, pl in reqs]
    eng.run_until_idle(timeout=300)
    st = eng.stats()
    assert st["completed"] == len(reqs) and st["max_batch"] >= 2
    for k, ((name, sc, cam, pl), f) in enumerate(zip(reqs, futs)):
        img = f.result(timeout=0).cpu().numpy().astype(np.float64)
        o = oracle.render(sc, cam, pl)
        ok = o["flags"] == 0
        err = np.abs(np.clip(img, 0, 1) - np.clip(o["image"], 0, 1)).max(axis=0)
        print(f"request {k}: {name} {cam.width}x{cam.height} cutoff={(o['label'] == 2).sum()} "
              f"max_err={err[ok].max():.2e} flagged={1 - ok.mean():.4f}", flush=True)
        assert (o["label"] == 2).sum() > 0
        assert ok.mean() > 0.9 and err[ok].max() <= 1e-3
    eng.close()


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
