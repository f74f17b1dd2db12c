"""Differentiable clipped render: a torch.autograd.Function over the C ABI.

Forward = rara_preprocess + rara_bin_sort + rara_render; backward =
rara_render_backward, which recomputes each tile's list from the saved
per-pixel n_contrib and final transmittance (no per-pixel lists are stored).
Tensors must be contiguous float32 on the GPU; the plane is a 4-vector
(n, d) whose values are read on the host.
"""
from __future__ import annotations

import torch

from . import binding as B
from . import renderer as R


class RaraRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mean, scale, quat, opacity, sh, plane4, cam, plane_enabled, bg, frame, check):
        sh_degree = int(round(sh.shape[0] ** 0.5)) - 1
        ds = R.DeviceScene(mean.detach(), scale.detach(), quat.detach(), opacity.detach(), sh.detach(), sh_degree)
        pv = [float(v) for v in plane4.detach().cpu().tolist()]
        import numpy as np
        from .scenes import Plane
        plane = Plane(np.array(pv[:3], np.float32), pv[3], int(plane_enabled))   # clip mode
        if check:
            out = R.render_checked(ds, frame, cam, plane, bg)
        else:
            R.enqueue_frame(ds, frame, cam, plane, bg)
            out = frame.out
        ctx.save_for_backward(mean, scale, quat, opacity, sh, plane4)
        ctx.frame, ctx.cam, ctx.plane, ctx.bg, ctx.ds = frame, cam, plane, bg, ds
        return out.image.clone()

    @staticmethod
    def backward(ctx, dimage):
        mean, scale, quat, opacity, sh, plane4 = ctx.saved_tensors
        fr, ds = ctx.frame, ctx.ds
        dev = mean.device
        g = {k: torch.empty_like(v) for k, v in
             dict(mean=mean, scale=scale, quat=quat, opacity=opacity, sh=sh).items()}
        dplane = torch.empty(4, dtype=torch.float32, device=dev)
        gs = B.Grads()
        gs.mean, gs.scale, gs.quat = g["mean"].data_ptr(), g["scale"].data_ptr(), g["quat"].data_ptr()
        gs.opacity, gs.sh, gs.plane = g["opacity"].data_ptr(), g["sh"].data_ptr(), dplane.data_ptr()
        ws_bytes = B.workspace_bytes(B.RARA_WS_BACKWARD, ds.n, fr.capacity, fr.width, fr.height)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
        dimg = dimage.contiguous().to(torch.float32)
        stream = int(torch.cuda.current_stream(dev).cuda_stream)
        B.render_backward(ds.struct(), B.make_camera(ctx.cam), B.make_plane(ctx.plane), ctx.bg, fr.proj.struct(),
                          fr.bins.struct(), fr.capacity, fr.out.final_T.data_ptr(), fr.out.n_contrib.data_ptr(),
                          dimg.data_ptr(),
                          gs, ws.data_ptr(), ws_bytes, stream)
        return (g["mean"], g["scale"], g["quat"], g["opacity"], g["sh"], dplane.to(plane4.device, plane4.dtype),
                None, None, None, None, None)


def render(mean, scale, quat, opacity, sh, plane4, cam, plane_enabled=True, bg=(0.0, 0.0, 0.0), frame=None,
           capacity=None, check=True):
    """Differentiable RaRa-clipped image [3][H][W] of one camera.

    check=True synchronises once to read the frame's overflow flag and grows
    the pair capacity and re-renders when it is set.  check=False only
    enqueues the frame: the caller reads ``frame.bins.overflow`` later (for
    example once for all the views of a batch, see ``overflowed``) and
    discards the result when it is set."""
    if frame is None:
        n = int(mean.shape[1])
        frame = R.Frame(n, cam.width, cam.height, capacity or max(1 << 16, 16 * n), mean.device, walked=False,
                        sorted_keys=False)
    return RaraRender.apply(mean, scale, quat, opacity, sh, plane4, cam, plane_enabled, tuple(bg), frame, bool(check))


def overflowed(frames) -> bool:
    """Whether any of the frames' pair capacity overflowed (one
    synchronisation for all of them)."""
    flags = torch.stack([f.bins.overflow.reshape(()) for f in frames])
    return bool(flags.any().item())
