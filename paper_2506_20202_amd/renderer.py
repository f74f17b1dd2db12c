"""Device-side buffers and a frame renderer over the C ABI.

PyTorch provides device memory and the current HIP stream; every value of
the frame is computed by the library's kernels.  A frame is three enqueued
calls (preprocess, bin_sort, render) with no host synchronisation; the pair
capacity is a caller decision and ``render_checked`` grows it when the device
reports overflow.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional

import torch

from . import binding as B


def _ptr(t: Optional[torch.Tensor]) -> int:
    return 0 if t is None else int(t.data_ptr())


@dataclasses.dataclass
class DeviceScene:
    """A scene resident in HBM, structure-of-arrays float32 (rara_gaussians).
    ``sh`` is [(D+1)^2][3][n] (``SH_COEFF_MAJOR``) or [n][(D+1)^2][3]
    (``SH_GAUSSIAN_MAJOR``: a frame then reads only the drawn Gaussians'
    coefficients); gradients of ``sh`` come back in the same layout."""

    mean: torch.Tensor
    scale: torch.Tensor
    quat: torch.Tensor
    opacity: torch.Tensor
    sh: torch.Tensor
    sh_degree: int
    sh_layout: int = B.SH_COEFF_MAJOR

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    @staticmethod
    def from_scene(scene, device="cuda", sh_layout: int = B.SH_COEFF_MAJOR) -> "DeviceScene":
        """Uploads a host scene (SH coefficient-major), converting the SH to
        ``sh_layout`` once on the way."""
        t = lambda a: torch.from_numpy(a).to(device=device, dtype=torch.float32).contiguous()
        sh = t(scene.sh)
        if sh_layout == B.SH_GAUSSIAN_MAJOR:
            sh = sh.permute(2, 0, 1).contiguous()
        elif sh_layout != B.SH_COEFF_MAJOR:
            raise ValueError(f"unknown SH layout {sh_layout}")
        return DeviceScene(t(scene.mean), t(scene.scale), t(scene.quat), t(scene.opacity), sh,
                           int(scene.sh_degree), int(sh_layout))

    def struct(self) -> B.Gaussians:
        g = B.Gaussians()
        g.n = self.n
        g.sh_degree = self.sh_degree
        g.sh_layout = self.sh_layout
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
        self.tiles_touched = torch.empty(m, dtype=torch.int32, device=device)
        self.tile_rec = torch.empty(2 * m, dtype=torch.int64, device=device)   # 16 B per Gaussian
        self.ray_ext = None   # a clip region's further-plane terms, allocated on first use
        self.device = device

    def ensure_ray_ext(self):
        if self.ray_ext is None:
            m = max(self.n, 1)
            self.ray_ext = torch.empty(m * B.RAY_EXT_FLOATS, dtype=torch.float32, device=self.device)

    def struct(self) -> B.Projected:
        p = B.Projected()
        p.label, p.splat, p.ray = _ptr(self.label), _ptr(self.splat), _ptr(self.ray)
        p.depth, p.tiles_touched = _ptr(self.depth), _ptr(self.tiles_touched)
        p.ray_ext = _ptr(self.ray_ext)
        p.tile_rec = _ptr(self.tile_rec)
        return p

    def nbytes(self) -> int:
        ext = self.ray_ext.numel() * 4 if self.ray_ext is not None else 0
        return self.n * (1 + B.SPLAT_BYTES + B.RAY_BYTES + 4 + 4 + 16) + ext


class BinBuffers:
    """rara_binned plus the bin/sort workspace for a pair capacity.
    ``pair_start`` (needed only by the backward) is allocated on request;
    ``sorted_keys=False`` leaves ``keys`` as sort scratch (the frame's tile
    lists, ranges and image are the same; only the 64-bit keys are not
    written)."""

    def __init__(self, n: int, width: int, height: int, capacity: int, device="cuda", pair_start: bool = True,
                 sorted_keys: bool = True):
        self.capacity = int(capacity)
        self.sorted_keys = bool(sorted_keys)
        tiles = ((width + 15) // 16) * ((height + 15) // 16)
        self.keys = torch.empty(self.capacity, dtype=torch.int64, device=device)
        self.vals = torch.empty(self.capacity, dtype=torch.int32, device=device)
        self.ranges = torch.empty(tiles * 2, dtype=torch.int32, device=device)
        self.num_pairs = torch.zeros(1, dtype=torch.int64, device=device)
        self.overflow = torch.zeros(1, dtype=torch.int32, device=device)
        self.work = torch.empty(tiles + 1, dtype=torch.int32, device=device)
        self.pair_start = torch.empty(max(int(n), 1), dtype=torch.int32, device=device) if pair_start else None
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
        b.keys_scratch = 0 if self.sorted_keys else 1
        return b

    def nbytes(self) -> int:
        ps = self.pair_start.numel() * 4 if self.pair_start is not None else 0
        return self.capacity * 12 + self.ranges.numel() * 4 + ps + self.ws_bytes


class ImageBuffers:
    """image, final_T, n_contrib; with ``walked`` also n_walked and n_eval
    (work counts: [2][H][W], evaluations and clip weights per pixel)."""

    def __init__(self, width: int, height: int, device="cuda", walked: bool = True):
        self.image = torch.empty((3, height, width), dtype=torch.float32, device=device)
        self.final_T = torch.empty((height, width), dtype=torch.float32, device=device)
        self.n_contrib = torch.empty((height, width), dtype=torch.int32, device=device)
        self.n_walked = torch.empty((height, width), dtype=torch.int32, device=device) if walked else None
        self.n_eval = torch.empty((2, height, width), dtype=torch.int32, device=device) if walked else None


class Frame:
    """All device buffers of one frame shape (n Gaussians, W x H, capacity).
    ``pair_start`` keeps the per-Gaussian pair offsets the backward needs and
    ``sorted_keys`` the 64-bit sorted keys; a frame that is only rendered can
    go without both."""

    def __init__(self, n: int, width: int, height: int, capacity: int, device="cuda", walked: bool = True,
                 pair_start: bool = True, sorted_keys: bool = True):
        self.n, self.width, self.height = int(n), int(width), int(height)
        self.device = device
        self.proj = ProjectedBuffers(n, device)
        self.bins = BinBuffers(n, width, height, capacity, device, pair_start, sorted_keys)
        self.out = ImageBuffers(width, height, device, walked)

    @property
    def capacity(self) -> int:
        return self.bins.capacity

    def grow(self, capacity: int):
        self.bins = BinBuffers(self.n, self.width, self.height, capacity, self.device,
                               self.bins.pair_start is not None, self.bins.sorted_keys)


def enqueue_frame(scene: DeviceScene, frame: Frame, cam, plane, bg=(0.0, 0.0, 0.0), stream=None,
                  stages=("pre", "bin", "render")):
    """Enqueue preprocess -> bin_sort -> render on ``stream`` (default: torch's
    current stream).  No synchronisation."""
    if stream is None:
        stream = torch.cuda.current_stream(scene.mean.device)
    sp = int(stream.cuda_stream)
    c = B.make_camera(cam)
    p = B.make_plane(plane)
    if p.count > 1:
        frame.proj.ensure_ray_ext()   # a clip region: further-plane terms per CUTOFF Gaussian
    pj = frame.proj.struct()
    bn = frame.bins.struct()
    if "pre" in stages:
        B.preprocess(scene.struct(), c, p, pj, sp)
    if "bin" in stages:
        B.bin_sort(pj, scene.n, c, frame.capacity, _ptr(frame.bins.workspace), frame.bins.ws_bytes, bn, sp)
    if "render" in stages:
        o = frame.out
        B.render(pj, scene.n, bn, c, p, bg, _ptr(o.image), _ptr(o.final_T), _ptr(o.n_contrib), _ptr(o.n_walked), sp,
                 _ptr(o.n_eval))


def enqueue_render_batch(jobs, stream=None):
    """One rara_render_batch launch over frames already binned on ``stream``
    (or ordered before it): ``jobs`` is a list of (scene, frame, cam, plane,
    bg).  No synchronisation."""
    if stream is None:
        stream = torch.cuda.current_stream(jobs[0][0].mean.device)
    items = []
    for scene, frame, cam, plane, bg in jobs:
        o = frame.out
        items.append((frame.proj.struct(), scene.n, frame.bins.struct(), B.make_camera(cam), B.make_plane(plane), bg,
                      _ptr(o.image), _ptr(o.final_T), _ptr(o.n_contrib)))
    B.render_batch(items, int(stream.cuda_stream))


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


_hip_runtime = None


def new_stream(device) -> "torch.cuda.ExternalStream":
    """A HIP stream with a hardware queue of its own on ``device`` (default
    priority); release it with ``destroy_stream``.  It is created with a CU
    mask that enables every CU, which gives the stream a dedicated queue: plain
    streams share the process's four queues in an order set by the streams
    created and destroyed before them, and a frame pipeline on three of them
    ran at 2500-3600 frames/s depending on that history (3570-3600 on
    dedicated queues)."""
    global _hip_runtime
    if _hip_runtime is None:
        _hip_runtime = ctypes.CDLL("libamdhip64.so")
        _hip_runtime.hipExtStreamCreateWithCUMask.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32,
                                                              ctypes.POINTER(ctypes.c_uint32)]
        _hip_runtime.hipStreamDestroy.argtypes = [ctypes.c_void_p]
    ncu = torch.cuda.get_device_properties(device).multi_processor_count
    words = (ncu + 31) // 32
    mask = (ctypes.c_uint32 * words)(*([0xFFFFFFFF] * words))
    h = ctypes.c_void_p()
    with torch.cuda.device(device):
        status = _hip_runtime.hipExtStreamCreateWithCUMask(ctypes.byref(h), words, mask)
    if status != 0:
        raise RuntimeError(f"hipExtStreamCreateWithCUMask failed ({status})")
    return torch.cuda.ExternalStream(h.value, device=device)


def destroy_stream(stream) -> None:
    stream.synchronize()
    _hip_runtime.hipStreamDestroy(ctypes.c_void_p(stream.cuda_stream))


class FramePipeline:
    """Renders a sequence of frames of one shape with ``streams`` frames in
    flight: frame i runs all of its stages on stream i mod streams, in buffer
    set i mod streams, so frames on different streams overlap (one frame's
    latency-bound sort kernels and the tail of another's blend fill the CUs a
    single frame leaves idle) while each stream keeps its frames in order and
    reuses its set only after its previous frame.  Each stream has a hardware
    queue of its own (``new_stream``) and the default priority.  On the 1080p
    clipping frames: 3 streams about 4560 frames/s, 2 streams 3905, 4 streams
    3629, one frame at a time about 2650."""

    def __init__(self, scene: DeviceScene, width: int, height: int, capacity: int, streams: int = 3,
                 walked: bool = True):
        dev = scene.mean.device
        if streams < 1:
            raise ValueError("streams must be at least 1")
        self.scene = scene
        self.frames = [Frame(scene.n, width, height, capacity, dev, walked, pair_start=False, sorted_keys=False)
                       for _ in range(streams)]
        self.streams = [new_stream(dev) for _ in range(streams)]
        self.count = 0
        self.start()

    def start(self, stream=None):
        """Order the pipeline after the work already on ``stream``."""
        if stream is None:
            stream = torch.cuda.current_stream(self.scene.mean.device)
        for st in self.streams:
            st.wait_stream(stream)

    def submit(self, cam, plane, bg=(0.0, 0.0, 0.0), consume=None) -> Frame:
        """Enqueue one frame and return its Frame.  Its outputs are valid once
        its stream has passed the frame (``join``) and until the same set is
        reused ``streams`` submissions later.  ``consume(frame)``, if given, is
        called with the frame's stream as torch's current stream, after the
        render: work it enqueues (a copy of the image, a loss) runs before the
        set is reused."""
        k = self.count % len(self.streams)
        fr, st = self.frames[k], self.streams[k]
        enqueue_frame(self.scene, fr, cam, plane, bg, stream=st)
        if consume is not None:
            with torch.cuda.stream(st):
                consume(fr)
        self.count += 1
        return fr

    def join(self, stream=None):
        """Order ``stream`` after every submitted frame."""
        if stream is None:
            stream = torch.cuda.current_stream(self.scene.mean.device)
        for st in self.streams:
            stream.wait_stream(st)

    def grow(self, capacity: int):
        torch.cuda.synchronize(self.scene.mean.device)
        for fr in self.frames:
            fr.grow(capacity)

    @property
    def capacity(self) -> int:
        return self.frames[0].capacity

    def overflowed(self) -> bool:
        return any(int(fr.bins.overflow.item()) for fr in self.frames)

    def close(self):
        """Wait for every submitted frame and release the streams."""
        streams, self.streams = self.streams, []
        for st in streams:
            destroy_stream(st)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def splat_fields(proj: ProjectedBuffers) -> dict:
    """Decode the 48-byte splat records (host copy) for inspection and tests."""
    import numpy as np
    raw = proj.splat.detach().cpu().numpy().view(np.uint8).reshape(-1, B.SPLAT_BYTES)[: proj.n]
    mean2d = raw[:, 0:16].copy().view(np.float64).reshape(-1, 2)
    f = raw[:, 16:48].copy().view(np.float32).reshape(-1, 8)
    word = raw[:, 44:48].copy().view(np.uint32).reshape(-1)
    return dict(mean2d=mean2d, conic=f[:, 0:3].copy(), opacity=f[:, 3].copy(), rgb=f[:, 4:7].copy(),
                label=word & 0xFF, cuts=word >> 16)


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
