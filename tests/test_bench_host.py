"""Host-side pieces of bench.py that need no GPU: the oracle timing leg (it
calls the oracle's C entry points directly) and the workload generators."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2506_20202_amd import scenes  # noqa: E402


def test_oracle_timing_leg_runs_for_planes_and_regions():
    sc, cam = scenes.tiny_scene(0), scenes.tiny_camera()
    for pl in (scenes.tiny_plane(0), scenes.box_region((-0.5, -0.5, -0.5), (0.5, 0.5, 0.5))):
        r = bench.oracle_frame(sc, cam, pl, 1.0)
        assert r["value"] > 0 and r["kind"] == "oracle" and r["cores"] >= 1


def test_gpu_count_above_one_is_refused(capsys, monkeypatch):
    import pytest
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err


def test_clip_order_strides_views_and_offsets():
    """The timed frames: any prefix strides views and offsets, and one full
    pass visits every clipping (view, offset) pair exactly once."""
    clip = [list(range(3, 13))] * 16
    order = bench.clip_order(clip)
    assert len(order) == 160 and len(set(order)) == 160
    assert all(o in range(3, 13) for _, o in order)
    head = order[:20]
    assert [v for v, _ in head] == list(range(16)) + [0, 1, 2, 3]
    assert len({o for _, o in head}) == 10          # every clipping offset within the first 20 frames
    # unequal offset lists per view: every pair still appears
    clip2 = [[0, 1], [2], [1, 2, 3]]
    order2 = bench.clip_order(clip2)
    assert {(v, o) for v in range(3) for o in clip2[v]} == set(order2)
    import pytest
    with pytest.raises(ValueError):
        bench.clip_order([[1], []])


def test_stage_byte_models():
    """Per-stage algorithmic bytes: the preprocess of a scene where nothing is
    live moves 45 B per Gaussian; one drawn SH3 Gaussian adds 16 + 4 + 192 +
    52 B; the sort's tile passes follow the tile count (2 passes for the
    8160 tiles of 1080p, 1 for 64)."""
    assert bench.preprocess_bytes(1000, 3, 0, 0, 0) == 45000
    assert bench.preprocess_bytes(1, 3, 1, 1, 0) - 45 == 16 + 4 + 192 + 52
    assert bench.preprocess_bytes(1, 3, 1, 1, 1) - bench.preprocess_bytes(1, 3, 1, 1, 0) == 48
    one = bench.bin_sort_bytes(0, 0, 1, 64) - bench.bin_sort_bytes(0, 0, 0, 64)
    two = bench.bin_sort_bytes(0, 0, 1, 8160) - bench.bin_sort_bytes(0, 0, 0, 8160)
    assert one == 8 + 12 and two == 8 + 16 + 12


def test_backward_byte_model():
    """Backward bytes: 172 B per pair (entry + slot written and read), 216 B
    per drawn Gaussian (+48 for a CUTOFF one's ray record), 20 B per pixel,
    and parameters read plus gradients written (236 B each way at SH degree
    3)."""
    base = bench.backward_bytes(0, 3, 0, 0, 0, 0)
    assert base == 0
    assert bench.backward_bytes(0, 3, 0, 0, 1, 0) == 172
    assert bench.backward_bytes(0, 3, 1, 1, 0, 0) == 216 + 48
    assert bench.backward_bytes(0, 3, 0, 0, 0, 10) == 200
    assert bench.backward_bytes(1, 3, 0, 0, 0, 0) == 2 * 236
    assert bench.backward_bytes(1, 0, 0, 0, 0, 0) == 2 * 56
