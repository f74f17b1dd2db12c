"""ctypes binding of librara.so (include/rara.h).  Argument marshalling only:
every step of the renderer runs in the library's HIP kernels.  Raises
RuntimeError when the library has not been built -- there is no fallback."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librara.so")

RARA_OK, RARA_ERR_INVALID, RARA_ERR_CAPACITY, RARA_ERR_HIP, RARA_ERR_UNSUPPORTED, RARA_ERR_SCRATCH = 0, 1, 2, 3, 4, 5
STATIC_WS_BYTES = 64 << 20   # RARA_STATIC_WS_BYTES: workspace of rara_bin_sort_static
RARA_WS_BIN_SORT, RARA_WS_BACKWARD = 0, 1
LABEL_INVISIBLE, LABEL_VISIBLE, LABEL_CUTOFF = 0, 1, 2
# clip modes (rara_plane.enabled): a rule, plus flags that go with RARA_CLIP_RARA
RARA_CLIP_OFF, RARA_CLIP_RARA, RARA_CLIP_HARD, RARA_CLIP_TIGHT, RARA_CLIP_STRICT_MISS = 0, 1, 2, 4, 8
SPLAT_BYTES = 48
RAY_BYTES = 48

_P = ctypes.c_void_p


# rara_gaussians.sh_layout
SH_COEFF_MAJOR = 0      # sh [(D+1)^2][3][n]
SH_GAUSSIAN_MAJOR = 1   # sh [n][(D+1)^2][3]


class Gaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("sh_layout", ctypes.c_int32), ("mean", _P),
                ("scale", _P), ("quat", _P), ("opacity", _P), ("sh", _P)]


class Camera(ctypes.Structure):
    _fields_ = [("world_to_cam", ctypes.c_float * 12), ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("near_z", ctypes.c_float)]


MAX_PLANES = 8
RAY_EXT_FLOATS = 2 * (MAX_PLANES - 1)   # per Gaussian, rara_projected.ray_ext


class Plane(ctypes.Structure):
    _fields_ = [("n", ctypes.c_float * 3), ("d", ctypes.c_float), ("enabled", ctypes.c_int32),
                ("count", ctypes.c_int32), ("extra", (ctypes.c_float * 4) * (MAX_PLANES - 1))]


class Projected(ctypes.Structure):
    _fields_ = [("label", _P), ("splat", _P), ("ray", _P), ("depth", _P), ("tiles_touched", _P), ("ray_ext", _P),
                ("tile_rec", _P)]


class Binned(ctypes.Structure):
    _fields_ = [("keys", _P), ("vals", _P), ("ranges", _P), ("num_pairs", _P), ("overflow", _P), ("work", _P),
                ("pair_start", _P), ("keys_scratch", ctypes.c_int32)]


MAX_BATCH = 16   # RARA_MAX_BATCH


class RenderItem(ctypes.Structure):
    _fields_ = [("proj", ctypes.POINTER(Projected)), ("n", ctypes.c_int64), ("bins", ctypes.POINTER(Binned)),
                ("cam", ctypes.POINTER(Camera)), ("plane", ctypes.POINTER(Plane)),
                ("bg", ctypes.POINTER(ctypes.c_float)), ("image", _P), ("final_T", _P), ("n_contrib", _P)]


class Grads(ctypes.Structure):
    _fields_ = [("mean", _P), ("scale", _P), ("quat", _P), ("opacity", _P), ("sh", _P), ("plane", _P)]


EXPORTS = ["rara_preprocess", "rara_bin_sort", "rara_render", "rara_render_backward", "rara_workspace_bytes",
           "rara_status_string", "rara_version", "rara_frame_graph_create", "rara_frame_graph_launch",
           "rara_frame_graph_destroy", "rara_bin_sort_static", "rara_render_batch"]

_lib = None


class RaraError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn} failed: {status_string(status)} ({status})")
        self.status = status


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"librara.so is not built ({LIB_PATH}); run __graft_entry__.build() "
                               "or python -m paper_2506_20202_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        PG, PC, PP = ctypes.POINTER(Gaussians), ctypes.POINTER(Camera), ctypes.POINTER(Plane)
        PJ, PB, PR = ctypes.POINTER(Projected), ctypes.POINTER(Binned), ctypes.POINTER(Grads)
        L.rara_preprocess.argtypes = [PG, PC, PP, PJ, _P]
        L.rara_bin_sort.argtypes = [PJ, ctypes.c_int64, PC, ctypes.c_int64, _P, ctypes.c_size_t, PB, _P]
        L.rara_bin_sort_static.argtypes = [PJ, ctypes.c_int64, PC, ctypes.c_int64, PB, _P]
        L.rara_render_batch.argtypes = [ctypes.POINTER(RenderItem), ctypes.c_int32, _P]
        L.rara_render.argtypes = [PJ, ctypes.c_int64, PB, PC, PP, ctypes.POINTER(ctypes.c_float), _P, _P, _P, _P, _P,
                                  _P]
        L.rara_render_backward.argtypes = [PG, PC, PP, ctypes.POINTER(ctypes.c_float), PJ, PB, ctypes.c_int64, _P, _P,
                                           _P, PR, _P, ctypes.c_size_t, _P]
        L.rara_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                           ctypes.c_int32]
        L.rara_workspace_bytes.restype = ctypes.c_size_t
        L.rara_status_string.argtypes = [ctypes.c_int]
        L.rara_status_string.restype = ctypes.c_char_p
        L.rara_version.restype = ctypes.c_char_p
        L.rara_frame_graph_create.argtypes = [PG, PC, PJ, PB, ctypes.c_int64, _P, ctypes.c_size_t, _P, _P, _P, _P,
                                              ctypes.POINTER(_P)]
        L.rara_frame_graph_launch.argtypes = [_P, PC, PP, ctypes.POINTER(ctypes.c_float), _P]
        L.rara_frame_graph_destroy.argtypes = [_P]
        L.rara_frame_graph_destroy.restype = None
        for f in ("rara_preprocess", "rara_bin_sort", "rara_render", "rara_render_backward", "rara_frame_graph_create",
                  "rara_frame_graph_launch", "rara_bin_sort_static", "rara_render_batch"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().rara_status_string(int(status)).decode()


def version() -> str:
    return lib().rara_version().decode()


def _check(fn: str, status: int):
    if status != RARA_OK:
        raise RaraError(fn, status)


def make_camera(cam) -> Camera:
    c = Camera()
    wc = [float(v) for v in list(cam.world_to_cam.reshape(-1))]
    c.world_to_cam = (ctypes.c_float * 12)(*wc)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    c.near_z = float(cam.near)
    return c


def make_plane(plane) -> Plane:
    """rara_plane of a plane, or of a region (a plane with ``extra`` planes)."""
    p = Plane()
    p.n = (ctypes.c_float * 3)(*[float(v) for v in plane.n])
    p.d = float(plane.d)
    p.enabled = int(plane.enabled)   # clip mode: False/True -> off/RaRa, ints pass through
    extra = list(getattr(plane, "extra", ()))
    if len(extra) > MAX_PLANES - 1:
        raise ValueError(f"a clip region has at most {MAX_PLANES} planes")
    p.count = 1 + len(extra)
    for k, (n, d) in enumerate(extra):
        p.extra[k] = (ctypes.c_float * 4)(float(n[0]), float(n[1]), float(n[2]), float(d))
    return p


def workspace_bytes(which: int, n: int, pair_capacity: int, width: int, height: int) -> int:
    return int(lib().rara_workspace_bytes(which, n, pair_capacity, width, height))


def preprocess(g: Gaussians, cam: Camera, plane: Plane, out: Projected, stream: int):
    _check("rara_preprocess", lib().rara_preprocess(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(plane),
                                                    ctypes.byref(out), _P(stream)))


def bin_sort(proj: Projected, n: int, cam: Camera, pair_capacity: int, workspace: int, ws_bytes: int,
             out: Binned, stream: int):
    _check("rara_bin_sort", lib().rara_bin_sort(ctypes.byref(proj), n, ctypes.byref(cam), pair_capacity,
                                                _P(workspace), ws_bytes, ctypes.byref(out), _P(stream)))


def bin_sort_static(proj: Projected, n: int, cam: Camera, pair_capacity: int, out: Binned, stream: int):
    """rara_bin_sort with the library's static workspace (no caller buffer)."""
    _check("rara_bin_sort_static", lib().rara_bin_sort_static(ctypes.byref(proj), n, ctypes.byref(cam),
                                                              pair_capacity, ctypes.byref(out), _P(stream)))


def render(proj: Projected, n: int, bins: Binned, cam: Camera, plane: Plane, bg, image: int, final_T: int,
           n_contrib: int, n_walked: int, stream: int, n_eval: int = 0):
    bgc = (ctypes.c_float * 3)(*[float(v) for v in bg])
    _check("rara_render", lib().rara_render(ctypes.byref(proj), n, ctypes.byref(bins), ctypes.byref(cam),
                                            ctypes.byref(plane), bgc, _P(image), _P(final_T), _P(n_contrib),
                                            _P(n_walked or None), _P(n_eval or None), _P(stream)))


def render_batch(items, stream: int):
    """rara_render_batch over a list of (proj, n, bins, cam, plane, bg, image,
    final_T, n_contrib) with ctypes structs and device pointers; the structs
    are kept alive for the call."""
    if not 1 <= len(items) <= MAX_BATCH:
        raise ValueError(f"a batch holds 1 to {MAX_BATCH} frames")
    arr = (RenderItem * len(items))()
    keep = []
    for k, (proj, n, bins, cam, plane, bg, image, final_T, n_contrib) in enumerate(items):
        bgc = (ctypes.c_float * 3)(*[float(v) for v in bg])
        keep += [proj, bins, cam, plane, bgc]
        arr[k].proj, arr[k].n, arr[k].bins = ctypes.pointer(proj), int(n), ctypes.pointer(bins)
        arr[k].cam, arr[k].plane, arr[k].bg = ctypes.pointer(cam), ctypes.pointer(plane), bgc
        arr[k].image, arr[k].final_T, arr[k].n_contrib = image, final_T, n_contrib
    _check("rara_render_batch", lib().rara_render_batch(arr, len(items), _P(stream)))


def render_backward(g: Gaussians, cam: Camera, plane: Plane, bg, proj: Projected, bins: Binned, pair_capacity: int,
                    final_T: int, n_contrib: int, dL_dimage: int, grads: Grads, workspace: int, ws_bytes: int,
                    stream: int):
    bgc = (ctypes.c_float * 3)(*[float(v) for v in bg])
    _check("rara_render_backward",
           lib().rara_render_backward(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(plane), bgc, ctypes.byref(proj),
                                      ctypes.byref(bins), ctypes.c_int64(pair_capacity), _P(final_T), _P(n_contrib),
                                      _P(dL_dimage), ctypes.byref(grads), _P(workspace), ws_bytes, _P(stream)))


def frame_graph_create(g: Gaussians, shape: Camera, proj: Projected, bins: Binned, pair_capacity: int, workspace: int,
                       ws_bytes: int, image: int, final_T: int, n_contrib: int, n_walked: int) -> int:
    h = _P()
    _check("rara_frame_graph_create",
           lib().rara_frame_graph_create(ctypes.byref(g), ctypes.byref(shape), ctypes.byref(proj), ctypes.byref(bins),
                                         pair_capacity, _P(workspace), ws_bytes, _P(image), _P(final_T),
                                         _P(n_contrib), _P(n_walked or None), ctypes.byref(h)))
    return h.value


def frame_graph_launch(handle: int, cam: Camera, plane: Plane, bg, stream: int):
    bgc = (ctypes.c_float * 3)(*[float(v) for v in bg])
    _check("rara_frame_graph_launch", lib().rara_frame_graph_launch(_P(handle), ctypes.byref(cam), ctypes.byref(plane),
                                                                    bgc, _P(stream)))


def frame_graph_destroy(handle: int):
    if handle:
        lib().rara_frame_graph_destroy(_P(handle))


# ---- attainable-peak probes (include/rara_peak.h, libpeak.so) ---------------

PEAK_LIB_PATH = os.path.join(HERE, "libpeak.so")
PEAK_EXPORTS = ["rara_peak_copy", "rara_peak_fma", "rara_peak_fma_flops"]
_peak = None


def peak_lib():
    global _peak
    if _peak is None:
        if not os.path.exists(PEAK_LIB_PATH):
            raise RuntimeError(f"libpeak.so is not built ({PEAK_LIB_PATH}); run __graft_entry__.build()")
        L = ctypes.CDLL(PEAK_LIB_PATH)
        L.rara_peak_copy.argtypes = [_P, _P, ctypes.c_size_t, ctypes.c_int, _P]
        L.rara_peak_copy.restype = ctypes.c_int
        L.rara_peak_fma.argtypes = [_P, ctypes.c_int, ctypes.c_int, _P]
        L.rara_peak_fma.restype = ctypes.c_int
        L.rara_peak_fma_flops.argtypes = [ctypes.c_int, ctypes.c_int]
        L.rara_peak_fma_flops.restype = ctypes.c_double
        _peak = L
    return _peak


def peak_copy(dst: int, src: int, nbytes: int, blocks: int, stream: int):
    st = peak_lib().rara_peak_copy(_P(dst), _P(src), nbytes, blocks, _P(stream))
    if st != 0:
        raise RuntimeError(f"rara_peak_copy failed ({st})")


def peak_fma(out: int, blocks: int, iters: int, stream: int) -> float:
    """Enqueue the FMA loop; returns its flop count."""
    L = peak_lib()
    st = L.rara_peak_fma(_P(out), blocks, iters, _P(stream))
    if st != 0:
        raise RuntimeError(f"rara_peak_fma failed ({st})")
    return float(L.rara_peak_fma_flops(blocks, iters))
