"""GPU test of rara_bin_sort_static, the bin/sort entry point for callers that
cannot allocate (its workspace is a static device array of the library):
through the C ABI, its outputs equal rara_bin_sort's bit for bit (pair count,
overflow flag, sorted keys and values, tile ranges, blend schedule, pair
starts) and so does the image rendered from them, on two calls in a row, the
second with a smaller input (fewer Gaussians, a smaller image, a smaller
capacity) over the first call's workspace contents."""
import numpy as np
import pytest
import torch

from paper_2506_20202_amd import binding as B
from paper_2506_20202_amd import renderer as R
from paper_2506_20202_amd import scenes

pytestmark = pytest.mark.gpu


def _binned_outputs(fr, n):
    P = int(fr.bins.num_pairs.item())
    drawn = fr.proj.tiles_touched[:n].cpu().numpy().view(np.uint32) > 0
    return dict(P=P, overflow=int(fr.bins.overflow.item()),
                keys=fr.bins.keys[:P].cpu().numpy().view(np.uint64),
                vals=fr.bins.vals[:P].cpu().numpy().view(np.uint32),
                ranges=fr.bins.ranges.cpu().numpy().view(np.uint32),
                work=fr.bins.work.cpu().numpy().view(np.uint32),
                pair_start=fr.bins.pair_start[:n].cpu().numpy().view(np.uint32)[drawn],
                image=fr.out.image.cpu().numpy(), n_contrib=fr.out.n_contrib.cpu().numpy())


def _both(sc, cam, pl, cap):
    dev = torch.device("cuda:0")
    ds = R.DeviceScene.from_scene(sc, dev)
    stream = int(torch.cuda.current_stream(dev).cuda_stream)
    c, p = B.make_camera(cam), B.make_plane(pl)
    res = []
    for static in (False, True):
        fr = R.Frame(sc.n, cam.width, cam.height, cap, dev, walked=False)
        fr.bins.keys.fill_(-1)
        fr.bins.vals.fill_(-1)
        R.enqueue_frame(ds, fr, cam, pl, stages=("pre",))
        pj, bn = fr.proj.struct(), fr.bins.struct()
        if static:
            B.bin_sort_static(pj, sc.n, c, cap, bn, stream)
        else:
            B.bin_sort(pj, sc.n, c, cap, fr.bins.workspace.data_ptr(), fr.bins.ws_bytes, bn, stream)
        R.enqueue_frame(ds, fr, cam, pl, stages=("render",))
        torch.cuda.synchronize()
        res.append(_binned_outputs(fr, sc.n))
    return res


def test_static_bin_sort_matches_bin_sort_on_two_calls():
    cases = [(scenes.tiny_scene(3, n=4000), scenes.tiny_camera(256, 192), scenes.tiny_plane(3), 1 << 17),
             (scenes.tiny_scene(5, n=700), scenes.tiny_camera(100, 75), scenes.tiny_plane(5), 1 << 13)]
    for k, (sc, cam, pl, cap) in enumerate(cases):
        print(f"call {k + 1}: n={sc.n} {cam.width}x{cam.height} capacity={cap}", flush=True)
        assert B.workspace_bytes(B.RARA_WS_BIN_SORT, sc.n, cap, cam.width, cam.height) <= B.STATIC_WS_BYTES
        ref, got = _both(sc, cam, pl, cap)
        assert ref["overflow"] == 0 and ref["P"] > 1000
        for key in ref:
            np.testing.assert_array_equal(got[key], ref[key], err_msg=key)


def test_static_bin_sort_reports_overflow_like_bin_sort():
    sc, cam, pl = scenes.tiny_scene(2), scenes.tiny_camera(), scenes.tiny_plane(2)
    ref, got = _both(sc, cam, pl, 1000)
    assert ref["overflow"] == 1 and got["overflow"] == 1 and got["P"] == ref["P"] > 1000
