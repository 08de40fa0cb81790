"""PyTorch autograd wrappers over the C ABI (the paper exposes its renderer as
a PyTorch custom operation with a backward pass, Sec. 4.4 last paragraph).

* :class:`SphereCamera` -- camera frame (12 floats: eye, fwd, right, up) from
  a pose on the enclosing sphere (yaw, pitch, dist, fovy in radians; Sec. 5.1);
  backward runs ``ddvr_camera_grad_to_sphere``.
* :class:`DDVRFunction` -- forward = ``ddvr_render_forward`` on the stored copy
  of a float32 master grid (f32 / f16 / bf16 storage, cast by
  ``ddvr_cast_volume``); backward = ``ddvr_render_adjoint`` in AUTO mode, i.e.
  the inversion trick with the segment-checkpoint fallback for nearly opaque
  rays.  Gradients are returned in float32 for the master grid.
* :class:`BatchFunction` -- V views of one grid rendered by one batched
  forward launch (``ddvr_batch_run``, forward pass) and differentiated by one
  batched adjoint launch (AUTO mode), with gradients to the grid, the TF, every
  view's camera frame and the shared step.  The batch is planned once in the
  forward and kept for the backward.
* :class:`ViewpointFunction` -- the same render with the camera given as its
  sphere pose; the gradients of the pose and the step come from forward-mode
  derivatives (``ddvr_render_tangent``, "forward-delayed" of Sec. 5.1: the
  backward re-traces the rays with the forward variables and contracts them
  with the upstream gradient in the kernel), those of the grid and the TF from
  the adjoint.

All arithmetic runs in the HIP library; these classes only allocate outputs
and pass pointers.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import ddvr as _d


def _camera_struct(frame: torch.Tensor, width: int, height: int) -> _d.Camera:
    f = [float(x) for x in frame.detach().to("cpu", torch.float64).tolist()]
    cam = _d.Camera()
    for a in range(3):
        cam.eye[a], cam.fwd[a], cam.right[a], cam.up[a] = f[a], f[3 + a], f[6 + a], f[9 + a]
    cam.width, cam.height = int(width), int(height)
    return cam


class SphereCamera(torch.autograd.Function):
    """(yaw, pitch, dist, fovy) scalar tensors -> frame [12] (float32, CPU)."""

    @staticmethod
    def forward(ctx, yaw, pitch, dist, fovy, width: int, height: int):
        vals = [float(t) for t in (yaw, pitch, dist, fovy)]
        cam = _d.camera_from_sphere(*vals, width, height)
        ctx.vals = vals
        ctx.wh = (int(width), int(height))
        return torch.tensor(cam.frame(), dtype=torch.float32)

    @staticmethod
    def backward(ctx, g_frame):
        gs = _d.camera_grad_to_sphere(*ctx.vals, *ctx.wh, g_frame.to("cpu").tolist())
        out = [torch.tensor(v, dtype=torch.float32) for v in gs]
        return out[0], out[1], out[2], out[3], None, None


class DDVRFunction(torch.autograd.Function):
    """image = render(volume, tf, frame, step).

    volume  float32 [nz][ny][nx] device tensor (the master copy), or
            [nz][ny][nx][4] (r, g, b, tau) for the colour-volume model
    tf      float32 [R][4] device tensor, or None (absorption-only, colour)
    frame   float32 [12] tensor (any device) -- camera frame
    step    scalar tensor, world units
    Returns [H][W][4] (emission-absorption, colour) or [H][W] (absorption-only).
    """

    @staticmethod
    def forward(ctx, volume, tf, frame, step, model: int, width: int, height: int,
                storage: torch.dtype = torch.float32, flags: int = 0):
        if not volume.is_cuda:
            raise ValueError("volume must be a device tensor")
        volume = volume.contiguous()
        if volume.dtype != torch.float32:
            raise ValueError("the master grid is float32; choose the stored form with `storage`")
        if storage == torch.float32:
            stored = volume
        else:
            stored = torch.empty_like(volume, dtype=storage)
            _d.cast_volume(volume, stored)
        if model == _d.EMISSION_ABSORPTION:
            if tf is None:
                raise ValueError("emission-absorption needs a transfer function")
            tf = tf.contiguous()
        cam = _camera_struct(frame, width, height)
        C = 1 if model == _d.ABSORPTION else 4
        image = torch.empty((height, width, C) if C == 4 else (height, width),
                            device=volume.device, dtype=torch.float32)
        trans = torch.empty((height, width), device=volume.device, dtype=torch.float32)
        s = float(step)
        _d.render_forward(stored, tf, cam, s, model, image, trans, flags=flags & _d.LAUNCH_PLAIN)
        ctx.save_for_backward(stored, tf if tf is not None else torch.empty(0), image, trans)
        ctx.has_tf = tf is not None
        ctx.cam = cam
        ctx.step = s
        ctx.model = model
        ctx.flags = flags
        ctx.frame_device = frame.device
        ctx.step_device = step.device if isinstance(step, torch.Tensor) else torch.device("cpu")
        return image

    @staticmethod
    def backward(ctx, g_image):
        stored, tf, image, trans = ctx.saved_tensors
        tf = tf if ctx.has_tf else None
        need_v, need_tf, need_cam, need_step = ctx.needs_input_grad[:4]
        dev = stored.device
        dV = torch.zeros(stored.shape, device=dev, dtype=torch.float32) if need_v else None
        dTF = torch.zeros_like(tf) if (need_tf and tf is not None) else None
        dcam = torch.zeros(12, device=dev, dtype=torch.float32) if need_cam else None
        dstep = torch.zeros(1, device=dev, dtype=torch.float32) if need_step else None
        if dV is None and dTF is None and dcam is None and dstep is None:
            return (None,) * 9
        n = _d.adjoint_workspace_size(stored, ctx.cam, ctx.step, ctx.model, ctx.flags)
        ws = torch.empty((n + 3) // 4, device=dev, dtype=torch.int32) if n else None
        _d.render_adjoint(stored, tf, ctx.cam, ctx.step, ctx.model, image, trans,
                          g_image.contiguous().to(torch.float32),
                          _d.grads_desc(dV, dTF, dcam, dstep), flags=ctx.flags, workspace=ws)
        g_frame = dcam.to(ctx.frame_device) if dcam is not None else None
        g_step = dstep.reshape(()).to(ctx.step_device) if dstep is not None else None
        return dV, dTF, g_frame, g_step, None, None, None, None, None


def _stored(volume, storage):
    if not volume.is_cuda:
        raise ValueError("volume must be a device tensor")
    volume = volume.contiguous()
    if volume.dtype != torch.float32:
        raise ValueError("the master grid is float32; choose the stored form with `storage`")
    if storage == torch.float32:
        return volume
    out = torch.empty_like(volume, dtype=storage)
    _d.cast_volume(volume, out)
    return out


class ViewpointFunction(torch.autograd.Function):
    """image = render(volume, tf, camera on the sphere (yaw, pitch, dist, fovy;
    radians), step); pose and step gradients by forward mode."""

    @staticmethod
    def forward(ctx, volume, tf, yaw, pitch, dist, fovy, step, model: int, width: int,
                height: int, storage: torch.dtype = torch.float32):
        stored = _stored(volume, storage)
        if model == _d.EMISSION_ABSORPTION:
            if tf is None:
                raise ValueError("emission-absorption needs a transfer function")
            tf = tf.contiguous()
        pose = [float(t) for t in (yaw, pitch, dist, fovy)]
        cam = _d.camera_from_sphere(*pose, width, height)
        C = 1 if model == _d.ABSORPTION else 4
        image = torch.empty((height, width, C) if C == 4 else (height, width),
                            device=volume.device, dtype=torch.float32)
        trans = torch.empty((height, width), device=volume.device, dtype=torch.float32)
        s = float(step)
        _d.render_forward(stored, tf, cam, s, model, image, trans)
        ctx.save_for_backward(stored, tf if tf is not None else torch.empty(0), image, trans)
        ctx.has_tf = tf is not None
        ctx.cam, ctx.pose, ctx.step, ctx.model, ctx.wh = cam, pose, s, model, (width, height)
        return image

    @staticmethod
    def backward(ctx, g_image):
        stored, tf, image, trans = ctx.saved_tensors
        tf = tf if ctx.has_tf else None
        need = ctx.needs_input_grad
        dev = stored.device
        g = g_image.contiguous().to(torch.float32)
        # forward mode for the pose (yaw, pitch, dist, fovy) and the step
        J = _d.camera_sphere_tangents(*ctx.pose, *ctx.wh)
        dirs, slots = [], []
        for k in range(4):
            if need[2 + k]:
                dirs.append(J[k] + [0.0])
                slots.append(2 + k)
        if need[6]:
            dirs.append([0.0] * 12 + [1.0])
            slots.append(6)
        grads = [None] * 11
        if dirs:
            d_dir = torch.zeros(len(dirs), device=dev, dtype=torch.float32)
            for c in range(0, len(dirs), _d.MAX_DIRECTIONS):
                _d.render_tangent(stored, tf, ctx.cam, ctx.step, ctx.model,
                                  dirs[c:c + _d.MAX_DIRECTIONS], d_image=g,
                                  d_dir=d_dir[c:c + _d.MAX_DIRECTIONS])
            vals = d_dir.to("cpu")
            for j, slot in enumerate(slots):
                grads[slot] = vals[j].clone()
        # the adjoint for the grid and the TF
        if need[0] or (need[1] and tf is not None):
            dV = torch.zeros(stored.shape, device=dev, dtype=torch.float32) if need[0] else None
            dTF = torch.zeros_like(tf) if (need[1] and tf is not None) else None
            n = _d.adjoint_workspace_size(stored, ctx.cam, ctx.step, ctx.model, 0)
            ws = torch.empty((n + 3) // 4, device=dev, dtype=torch.int32) if n else None
            _d.render_adjoint(stored, tf, ctx.cam, ctx.step, ctx.model, image, trans, g,
                              _d.grads_desc(dV, dTF), workspace=ws)
            grads[0], grads[1] = dV, dTF
        return tuple(grads)


class BatchFunction(torch.autograd.Function):
    """images = render(volume, tf, frames[v], step) for v < V.

    volume  float32 master grid, as for DDVRFunction (colour: [nz][ny][nx][4])
    tf      float32 [R][4] device tensor, or None (absorption-only, colour)
    frames  float32 [V][12] tensor (any device) -- one camera frame per view
    step    scalar tensor, world units, shared by the views
    Returns [V][H][W][4] (emission-absorption, colour) or [V][H][W].
    """

    @staticmethod
    def forward(ctx, volume, tf, frames, step, model: int, width: int, height: int,
                storage: torch.dtype = torch.float32):
        stored = _stored(volume, storage)
        if model == _d.EMISSION_ABSORPTION:
            if tf is None:
                raise ValueError("emission-absorption needs a transfer function")
            tf = tf.contiguous()
        else:
            tf = None
        if frames.dim() != 2 or frames.shape[1] != 12 or frames.shape[0] < 1:
            raise ValueError("frames must be [V][12]")
        nview = frames.shape[0]
        dev = volume.device
        need = ctx.needs_input_grad
        C = 1 if model == _d.ABSORPTION else 4
        shape = (nview, height, width, C) if C == 4 else (nview, height, width)
        images = torch.empty(shape, device=dev, dtype=torch.float32)
        trans = torch.empty((nview, height, width), device=dev, dtype=torch.float32)
        g_buf = torch.zeros_like(images)          # upstream gradient, filled by backward
        dV = torch.zeros(stored.shape, device=dev, dtype=torch.float32) if need[0] else None
        dTF = torch.zeros_like(tf) if (need[1] and tf is not None) else None
        dcam = torch.zeros((nview, 12), device=dev, dtype=torch.float32) if need[2] else None
        dstep = torch.zeros(1, device=dev, dtype=torch.float32) if need[3] else None
        s = float(step)
        host = frames.detach().to("cpu", torch.float32)
        views = [_d.make_view(0, _camera_struct(host[i], width, height), s, images[i], trans[i],
                              d_image=g_buf[i], d_camera=None if dcam is None else dcam[i],
                              d_step=dstep, tf_index=0 if tf is not None else -1)
                 for i in range(nview)]
        batch = _d.Batch([stored], None if tf is None else [tf], views, model,
                         d_volumes=None if dV is None else [dV],
                         d_tfs=None if dTF is None else [dTF])
        batch.run(_d.PASS_FORWARD)
        # the batch keeps raw pointers to the grid, the TF and the images: the
        # version check of saved tensors catches in-place changes to any of
        # them before the adjoint reads them
        ctx.save_for_backward(stored, tf if tf is not None else torch.empty(0), images, trans)
        ctx.batch = batch
        ctx.bufs = (g_buf, dV, dTF, dcam, dstep)
        ctx.frames_device = frames.device
        ctx.step_device = step.device if isinstance(step, torch.Tensor) else torch.device("cpu")
        return images

    @staticmethod
    def backward(ctx, g_images):
        stored = ctx.saved_tensors[0]
        g_buf, dV, dTF, dcam, dstep = ctx.bufs
        if dV is None and dTF is None and dcam is None and dstep is None:
            return (None,) * 8
        g_buf.copy_(g_images)
        for t in (dV, dTF, dcam, dstep):
            if t is not None:
                t.zero_()
        n = ctx.batch.workspace_size()
        ws = torch.empty((n + 3) // 4, device=stored.device, dtype=torch.int32) if n else None
        ctx.batch.run(_d.PASS_ADJOINT, workspace=ws)
        g_frames = dcam.to(ctx.frames_device) if dcam is not None else None
        g_step = dstep.reshape(()).to(ctx.step_device) if dstep is not None else None
        return dV, dTF, g_frames, g_step, None, None, None, None


def render_batch(volume: torch.Tensor, tf: Optional[torch.Tensor], frames: torch.Tensor, step,
                 model: int, width: int, height: int,
                 storage: torch.dtype = torch.float32) -> torch.Tensor:
    """Differentiable render of V views of one grid in one batched launch per
    pass (see BatchFunction)."""
    if not isinstance(step, torch.Tensor):
        step = torch.tensor(float(step))
    return BatchFunction.apply(volume, tf, frames, step, model, width, height, storage)


def render_viewpoint(volume: torch.Tensor, tf: Optional[torch.Tensor], yaw, pitch, dist, fovy,
                     step, model: int, width: int, height: int,
                     storage: torch.dtype = torch.float32) -> torch.Tensor:
    """Differentiable render from a sphere pose; pose/step gradients by forward
    mode (see ViewpointFunction)."""
    t = [x if isinstance(x, torch.Tensor) else torch.tensor(float(x))
         for x in (yaw, pitch, dist, fovy, step)]
    return ViewpointFunction.apply(volume, tf, t[0], t[1], t[2], t[3], t[4], model, width,
                                   height, storage)


def camera_frame(yaw, pitch, dist, fovy, width: int, height: int) -> torch.Tensor:
    """Differentiable camera frame from a sphere pose (radians)."""
    t = [x if isinstance(x, torch.Tensor) else torch.tensor(float(x)) for x in (yaw, pitch, dist, fovy)]
    return SphereCamera.apply(t[0], t[1], t[2], t[3], width, height)


def render(volume: torch.Tensor, tf: Optional[torch.Tensor], frame: torch.Tensor, step,
           model: int, width: int, height: int, storage: torch.dtype = torch.float32,
           flags: int = 0) -> torch.Tensor:
    """Differentiable render of one view (see DDVRFunction)."""
    if not isinstance(step, torch.Tensor):
        step = torch.tensor(float(step))
    return DDVRFunction.apply(volume, tf, frame, step, model, width, height, storage, flags)
