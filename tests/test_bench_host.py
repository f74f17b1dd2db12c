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
