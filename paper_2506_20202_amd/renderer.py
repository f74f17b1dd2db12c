"""Device-side buffers and a frame renderer over the C ABI.

PyTorch provides device memory and the current HIP stream; every value of
the frame is computed by the library's kernels.  A frame is three enqueued
calls (preprocess, bin_sort, render) with no host synchronisation; the pair
capacity is a caller decision and ``render_checked`` grows it when the device
reports overflow.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import torch

from . import binding as B


def _ptr(t: Optional[torch.Tensor]) -> int:
    return 0 if t is None else int(t.data_ptr())


@dataclasses.dataclass
class DeviceScene:
    """A scene resident in HBM, structure-of-arrays float32 (rara_gaussians)."""

    mean: torch.Tensor
    scale: torch.Tensor
    quat: torch.Tensor
    opacity: torch.Tensor
    sh: torch.Tensor
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    @staticmethod
    def from_scene(scene, device="cuda") -> "DeviceScene":
        t = lambda a: torch.from_numpy(a).to(device=device, dtype=torch.float32).contiguous()
        return DeviceScene(t(scene.mean), t(scene.scale), t(scene.quat), t(scene.opacity), t(scene.sh),
                           int(scene.sh_degree))

    def struct(self) -> B.Gaussians:
        g = B.Gaussians()
        g.n = self.n
        g.sh_degree = self.sh_degree
        g.mean, g.scale, g.quat = _ptr(self.mean), _ptr(self.scale), _ptr(self.quat)
        g.opacity, g.sh = _ptr(self.opacity), _ptr(self.sh)
        return g

    def nbytes(self) -> int:
        return sum(t.numel() * 4 for t in (self.mean, self.scale, self.quat, self.opacity, self.sh))


class ProjectedBuffers:
    """rara_projected for up to ``n`` Gaussians."""

    def __init__(self, n: int, device="cuda"):
        m = max(int(n), 1)
        self.n = int(n)
        self.label = torch.empty(m, dtype=torch.uint8, device=device)
        self.splat = torch.empty(m * B.SPLAT_BYTES // 4, dtype=torch.float32, device=device)
        self.ray = torch.empty(m * B.RAY_BYTES // 4, dtype=torch.float32, device=device)
        self.depth = torch.empty(m, dtype=torch.float32, device=device)
        self.rect = torch.empty(m * 4, dtype=torch.int16, device=device)
        self.tiles_touched = torch.empty(m, dtype=torch.int32, device=device)

    def struct(self) -> B.Projected:
        p = B.Projected()
        p.label, p.splat, p.ray = _ptr(self.label), _ptr(self.splat), _ptr(self.ray)
        p.depth, p.rect, p.tiles_touched = _ptr(self.depth), _ptr(self.rect), _ptr(self.tiles_touched)
        return p

    def nbytes(self) -> int:
        return self.n * (1 + B.SPLAT_BYTES + B.RAY_BYTES + 4 + 8 + 4)


class BinBuffers:
    """rara_binned plus the bin/sort workspace for a pair capacity."""

    def __init__(self, n: int, width: int, height: int, capacity: int, device="cuda"):
        self.capacity = int(capacity)
        tiles = ((width + 15) // 16) * ((height + 15) // 16)
        self.keys = torch.empty(self.capacity, dtype=torch.int64, device=device)
        self.vals = torch.empty(self.capacity, dtype=torch.int32, device=device)
        self.ranges = torch.empty(tiles * 2, dtype=torch.int32, device=device)
        self.num_pairs = torch.zeros(1, dtype=torch.int64, device=device)
        self.overflow = torch.zeros(1, dtype=torch.int32, device=device)
        self.work = torch.empty(4 * tiles + 1, dtype=torch.int32, device=device)
        self.pair_start = torch.empty(max(int(n), 1), dtype=torch.int32, device=device)
        self.ws_bytes = B.workspace_bytes(B.RARA_WS_BIN_SORT, n, self.capacity, width, height)
        if self.ws_bytes == 0:
            raise ValueError("invalid bin/sort workspace request")
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)

    def struct(self) -> B.Binned:
        b = B.Binned()
        b.keys, b.vals, b.ranges = _ptr(self.keys), _ptr(self.vals), _ptr(self.ranges)
        b.num_pairs, b.overflow = _ptr(self.num_pairs), _ptr(self.overflow)
        b.work = _ptr(self.work)
        b.pair_start = _ptr(self.pair_start)
        return b

    def nbytes(self) -> int:
        return self.capacity * 12 + self.ranges.numel() * 4 + self.pair_start.numel() * 4 + self.ws_bytes


class ImageBuffers:
    def __init__(self, width: int, height: int, device="cuda", walked: bool = True):
        self.image = torch.empty((3, height, width), dtype=torch.float32, device=device)
        self.final_T = torch.empty((height, width), dtype=torch.float32, device=device)
        self.n_contrib = torch.empty((height, width), dtype=torch.int32, device=device)
        self.n_walked = torch.empty((height, width), dtype=torch.int32, device=device) if walked else None


class Frame:
    """All device buffers of one frame shape (n Gaussians, W x H, capacity)."""

    def __init__(self, n: int, width: int, height: int, capacity: int, device="cuda", walked: bool = True):
        self.n, self.width, self.height = int(n), int(width), int(height)
        self.device = device
        self.proj = ProjectedBuffers(n, device)
        self.bins = BinBuffers(n, width, height, capacity, device)
        self.out = ImageBuffers(width, height, device, walked)

    @property
    def capacity(self) -> int:
        return self.bins.capacity

    def grow(self, capacity: int):
        self.bins = BinBuffers(self.n, self.width, self.height, capacity, self.device)


def enqueue_frame(scene: DeviceScene, frame: Frame, cam, plane, bg=(0.0, 0.0, 0.0), stream=None,
                  stages=("pre", "bin", "render")):
    """Enqueue preprocess -> bin_sort -> render on ``stream`` (default: torch's
    current stream).  No synchronisation."""
    if stream is None:
        stream = torch.cuda.current_stream(scene.mean.device)
    sp = int(stream.cuda_stream)
    c = B.make_camera(cam)
    p = B.make_plane(plane)
    pj = frame.proj.struct()
    bn = frame.bins.struct()
    if "pre" in stages:
        B.preprocess(scene.struct(), c, p, pj, sp)
    if "bin" in stages:
        B.bin_sort(pj, scene.n, c, frame.capacity, _ptr(frame.bins.workspace), frame.bins.ws_bytes, bn, sp)
    if "render" in stages:
        o = frame.out
        B.render(pj, scene.n, bn, c, p, bg, _ptr(o.image), _ptr(o.final_T), _ptr(o.n_contrib), _ptr(o.n_walked), sp)


def render_checked(scene: DeviceScene, frame: Frame, cam, plane, bg=(0.0, 0.0, 0.0), slack: float = 1.25):
    """Render one frame, growing the pair capacity (and re-rendering) when the
    device reports overflow.  Synchronises once."""
    enqueue_frame(scene, frame, cam, plane, bg)
    torch.cuda.synchronize()
    if int(frame.bins.overflow.item()):
        need = int(frame.bins.num_pairs.item())
        frame.grow(max(int(need * slack) + 1024, frame.capacity * 2))
        enqueue_frame(scene, frame, cam, plane, bg)
        torch.cuda.synchronize()
        assert not int(frame.bins.overflow.item())
    return frame.out


class FramePipeline:
    """Renders a sequence of frames of one shape with ``depth`` frames in
    flight over two streams: preprocess and binning of frame i+1 run on one
    stream while the blend of frame i runs on the other, so the latency-bound
    sort kernels fill the CUs the blend leaves idle.  Frame i uses buffer set
    i mod depth, whose preprocess waits for the blend that last read the set.
    Both streams keep the default priority."""

    def __init__(self, scene: DeviceScene, width: int, height: int, capacity: int, depth: int = 2,
                 walked: bool = True):
        dev = scene.mean.device
        self.scene = scene
        self.frames = [Frame(scene.n, width, height, capacity, dev, walked) for _ in range(depth)]
        self.bin_stream = torch.cuda.Stream(dev)
        self.blend_stream = torch.cuda.Stream(dev)
        self.binned = [torch.cuda.Event() for _ in range(depth)]
        self.blended = [torch.cuda.Event() for _ in range(depth)]
        self.count = 0
        self.start()

    def start(self, stream=None):
        """Order the pipeline after the work already on ``stream``."""
        if stream is None:
            stream = torch.cuda.current_stream(self.scene.mean.device)
        self.bin_stream.wait_stream(stream)
        self.blend_stream.wait_stream(stream)

    def submit(self, cam, plane, bg=(0.0, 0.0, 0.0), consume=None) -> Frame:
        """Enqueue one frame and return its Frame.  Its outputs are valid once
        the blend stream has passed the frame (``join``) and until the same
        set is reused ``depth`` submissions later.  ``consume(frame)``, if
        given, is called with the blend stream as torch's current stream,
        after the render: work it enqueues (a copy of the image, a loss) runs
        before the set can be reused, without waiting for later frames."""
        k = self.count % len(self.frames)
        fr = self.frames[k]
        if self.count >= len(self.frames):
            self.bin_stream.wait_event(self.blended[k])
        enqueue_frame(self.scene, fr, cam, plane, bg, stream=self.bin_stream, stages=("pre", "bin"))
        self.binned[k].record(self.bin_stream)
        self.blend_stream.wait_event(self.binned[k])
        enqueue_frame(self.scene, fr, cam, plane, bg, stream=self.blend_stream, stages=("render",))
        if consume is not None:
            with torch.cuda.stream(self.blend_stream):
                consume(fr)
        self.blended[k].record(self.blend_stream)
        self.count += 1
        return fr

    def join(self, stream=None):
        """Order ``stream`` after every submitted frame."""
        if stream is None:
            stream = torch.cuda.current_stream(self.scene.mean.device)
        stream.wait_stream(self.bin_stream)
        stream.wait_stream(self.blend_stream)

    def grow(self, capacity: int):
        torch.cuda.synchronize(self.scene.mean.device)
        for fr in self.frames:
            fr.grow(capacity)

    @property
    def capacity(self) -> int:
        return self.frames[0].capacity

    def overflowed(self) -> bool:
        return any(int(fr.bins.overflow.item()) for fr in self.frames)


def splat_fields(proj: ProjectedBuffers) -> dict:
    """Decode the 48-byte splat records (host copy) for inspection and tests."""
    import numpy as np
    raw = proj.splat.detach().cpu().numpy().view(np.uint8).reshape(-1, B.SPLAT_BYTES)[: proj.n]
    mean2d = raw[:, 0:16].copy().view(np.float64).reshape(-1, 2)
    f = raw[:, 16:48].copy().view(np.float32).reshape(-1, 8)
    lab = raw[:, 44:48].copy().view(np.uint32).reshape(-1)
    return dict(mean2d=mean2d, conic=f[:, 0:3].copy(), opacity=f[:, 3].copy(), rgb=f[:, 4:7].copy(), label=lab)


class FrameGraph:
    """A captured frame (rara_frame_graph) bound to one DeviceScene and one
    Frame; ``launch`` replays it for a new camera pose and plane."""

    def __init__(self, scene: DeviceScene, frame: Frame, shape_cam):
        self.scene, self.frame = scene, frame
        o = frame.out
        self.handle = B.frame_graph_create(scene.struct(), B.make_camera(shape_cam), frame.proj.struct(),
                                           frame.bins.struct(), frame.capacity, _ptr(frame.bins.workspace),
                                           frame.bins.ws_bytes, _ptr(o.image), _ptr(o.final_T), _ptr(o.n_contrib),
                                           _ptr(o.n_walked))

    def launch(self, cam, plane, bg=(0.0, 0.0, 0.0), stream=None):
        if stream is None:
            stream = torch.cuda.current_stream(self.scene.mean.device)
        B.frame_graph_launch(self.handle, B.make_camera(cam), B.make_plane(plane), bg, int(stream.cuda_stream))

    def close(self):
        if self.handle:
            B.frame_graph_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
