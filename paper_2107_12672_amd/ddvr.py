"""Thin ctypes binding of ``libddvr.so`` (declared in include/ddvr.h).

Names follow the C ABI without the ``ddvr_`` prefix.  The functions only
marshal arguments: torch tensors supply device pointers and torch's current
HIP stream supplies the stream; every step of the rendering runs in the HIP
kernels of the library.  Loading fails loudly when the library has not been
built -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddvr.so")

OK = 0
ERR_NULL, ERR_SHAPE, ERR_DTYPE, ERR_VALUE, ERR_HIP, ERR_UNSUPPORTED, ERR_WORKSPACE = \
    -1, -2, -3, -4, -5, -6, -7
F32, F16, BF16 = 0, 1, 2
ABSORPTION, EMISSION_ABSORPTION, COLOR = 0, 1, 2
ADJ_AUTO, ADJ_INVERT_T, ADJ_INVERT_ALPHA, ADJ_CHECKPOINT, ADJ_RESIDUAL = 0, 1, 2, 3, 4
LAUNCH_PLAIN = 0x10
LOSS_L1 = 0x20
PASS_FORWARD, PASS_ADJOINT, PASS_FUSED = 0, 1, 2
PLAN_LOSS_GIVEN, PLAN_LOSS_FUSED, PLAN_LOSS_NEG_ENTROPY = 0, 1, 2

EXPORTED = [
    "ddvr_abi_version", "ddvr_last_error", "ddvr_camera_from_sphere",
    "ddvr_camera_grad_to_sphere", "ddvr_render_forward", "ddvr_adjoint_workspace_size",
    "ddvr_render_adjoint", "ddvr_render_fused_l2", "ddvr_batch_create", "ddvr_batch_destroy",
    "ddvr_batch_workspace_size", "ddvr_batch_run", "ddvr_batch_run_graph",
    "ddvr_batch_sample_count", "ddvr_cast_volume", "ddvr_set_tuning", "ddvr_get_tuning",
    "ddvr_render_tangent", "ddvr_camera_sphere_tangents", "ddvr_density_from_color",
    "ddvr_color_tau_max", "ddvr_tf_prior", "ddvr_volume_prior", "ddvr_opacity_entropy",
    "ddvr_adam_step", "ddvr_resample_volume", "ddvr_resample_channels",
    "ddvr_batch_graph_builds", "ddvr_plan_create", "ddvr_plan_execute", "ddvr_plan_loss_terms",
    "ddvr_plan_destroy", "ddvr_valu_probe", "ddvr_render_adjoint_noalloc",
]
MAX_DIRECTIONS = 4


class DDVRError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"ddvr status {status}: {message}")
        self.status = status


class Volume(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("nz", ctypes.c_int32)]


class TF(ctypes.Structure):
    _fields_ = [("rgba_tau", ctypes.c_void_p), ("R", ctypes.c_int32)]


class Camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_float * 3), ("fwd", ctypes.c_float * 3),
                ("right", ctypes.c_float * 3), ("up", ctypes.c_float * 3),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]

    def frame(self) -> List[float]:
        return list(self.eye) + list(self.fwd) + list(self.right) + list(self.up)


class Tuning(ctypes.Structure):
    _fields_ = [("waves", ctypes.c_int32), ("lds_cap", ctypes.c_int32),
                ("slab_k", ctypes.c_int32), ("slab_kmax", ctypes.c_int32),
                ("cell_acc", ctypes.c_int32), ("lane_map", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("slab_axis", ctypes.c_int32)]


class Grads(ctypes.Structure):
    _fields_ = [("d_volume", ctypes.c_void_p), ("d_tf", ctypes.c_void_p),
                ("d_camera", ctypes.c_void_p), ("d_step", ctypes.c_void_p)]


class View(ctypes.Structure):
    _fields_ = [("volume", ctypes.c_int32), ("tf", ctypes.c_int32), ("cam", Camera),
                ("step_world", ctypes.c_float), ("image", ctypes.c_void_p),
                ("transmittance", ctypes.c_void_p), ("d_image", ctypes.c_void_p),
                ("target", ctypes.c_void_p), ("d_camera", ctypes.c_void_p),
                ("d_step", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded library (raw ctypes handle)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2107_12672_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, F, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float, ctypes.c_size_t
    sig = {
        "ddvr_abi_version": ([], ctypes.c_int),
        "ddvr_last_error": ([], ctypes.c_char_p),
        "ddvr_camera_from_sphere": ([F, F, F, F, I32, I32, P], ctypes.c_int),
        "ddvr_camera_grad_to_sphere": ([F, F, F, F, I32, I32, P, P], ctypes.c_int),
        "ddvr_render_forward": ([P, P, P, F, I32, P, P, I32, P], ctypes.c_int),
        "ddvr_adjoint_workspace_size": ([P, P, F, I32, I32, P], ctypes.c_int),
        "ddvr_render_adjoint": ([P, P, P, F, I32, P, P, P, P, I32, P, SZ, P, P], ctypes.c_int),
        "ddvr_render_fused_l2": ([P, P, P, F, I32, P, F, P, P, P, I32, P, SZ, P, P, P],
                                 ctypes.c_int),
        "ddvr_batch_create": ([P, I32, P, I32, P, I32, I32, I32, P, P, P, P], ctypes.c_int),
        "ddvr_batch_destroy": ([P], None),
        "ddvr_batch_workspace_size": ([P, P], ctypes.c_int),
        "ddvr_batch_run": ([P, I32, F, P, P, SZ, P], ctypes.c_int),
        "ddvr_batch_run_graph": ([P, I32, F, P, P, SZ, P], ctypes.c_int),
        "ddvr_batch_sample_count": ([P, P], ctypes.c_int),
        "ddvr_cast_volume": ([P, P, I32, ctypes.c_int64, P], ctypes.c_int),
        "ddvr_set_tuning": ([P], ctypes.c_int),
        "ddvr_get_tuning": ([P], ctypes.c_int),
        "ddvr_render_tangent": ([P, P, P, F, I32, P, I32, P, P, P, P, I32, P], ctypes.c_int),
        "ddvr_camera_sphere_tangents": ([F, F, F, F, I32, I32, P], ctypes.c_int),
        "ddvr_density_from_color": ([P, P, P, F, F, ctypes.c_uint64, I32, I32, P, P, P, P],
                                    ctypes.c_int),
        "ddvr_color_tau_max": ([P, P, P], ctypes.c_int),
        "ddvr_tf_prior": ([P, I32, F, P, P, P], ctypes.c_int),
        "ddvr_volume_prior": ([P, I32, I32, I32, F, P, P, P], ctypes.c_int),
        "ddvr_opacity_entropy": ([P, ctypes.c_int64, I32, P, P, P, F, P], ctypes.c_int),
        "ddvr_adam_step": ([P, P, P, P, ctypes.c_int64, I32, F, F, F, F, F, F, P, I32, I32, P],
                           ctypes.c_int),
        "ddvr_resample_volume": ([P, I32, I32, I32, P, I32, I32, I32, P], ctypes.c_int),
        "ddvr_resample_channels": ([P, I32, I32, I32, I32, P, I32, I32, I32, P], ctypes.c_int),
        "ddvr_batch_graph_builds": ([P, P], ctypes.c_int),
        "ddvr_plan_create": ([P, I32, F, P, P, SZ, P, P], ctypes.c_int),
        "ddvr_plan_execute": ([P, P], ctypes.c_int),
        "ddvr_plan_loss_terms": ([P, P, I32, P], ctypes.c_int),
        "ddvr_plan_destroy": ([P], None),
        "ddvr_valu_probe": ([I32, I32, I32, P, P, P], ctypes.c_int),
        "ddvr_render_adjoint_noalloc": ([P, P, P, F, I32, P, P, P, P, I32, P, P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def last_error() -> str:
    return lib().ddvr_last_error().decode()


def _check(status: int):
    if status != OK:
        raise DDVRError(status, last_error())


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def dtype_code(t) -> int:
    import torch
    return {torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}[t.dtype]


def volume_desc(vol) -> Volume:
    """Descriptor of a contiguous [nz][ny][nx] device tensor, or of a colour
    volume [nz][ny][nx][4] (r, g, b, tau per vertex)."""
    assert vol.is_contiguous() and (vol.dim() == 3 or (vol.dim() == 4 and vol.shape[3] == 4))
    nz, ny, nx = vol.shape[:3]
    return Volume(vol.data_ptr(), dtype_code(vol), nx, ny, nz)


def tf_desc(tf) -> TF:
    if tf is None:
        return TF(None, 0)
    assert tf.is_contiguous() and tf.dim() == 2 and tf.shape[1] == 4
    return TF(tf.data_ptr(), tf.shape[0])


def grads_desc(d_volume=None, d_tf=None, d_camera=None, d_step=None) -> Grads:
    return Grads(_ptr(d_volume), _ptr(d_tf), _ptr(d_camera), _ptr(d_step))


class Direction(ctypes.Structure):
    _fields_ = [("d_frame", ctypes.c_float * 12), ("d_step", ctypes.c_float)]


def render_tangent(volume, tf, cam: Camera, step: float, model: int, dirs, image=None,
                   image_dot=None, d_image=None, d_dir=None, flags: int = 0, stream=None):
    """Forward-mode derivatives along up to 4 directions; dirs is a sequence of
    13 numbers each (d frame[12], d step) -- see include/ddvr.h."""
    dirs = [list(map(float, x)) for x in dirs]
    arr = (Direction * max(len(dirs), 1))()
    for k, x in enumerate(dirs):
        if len(x) != 13:
            raise ValueError("a direction has 13 components (frame[12], step)")
        arr[k].d_frame[:] = x[:12]
        arr[k].d_step = x[12]
    v, t = volume_desc(volume), tf_desc(tf)
    _check(lib().ddvr_render_tangent(ctypes.byref(v), ctypes.byref(t), ctypes.byref(cam), step,
                                     model, arr, len(dirs), _ptr(image), _ptr(image_dot),
                                     _ptr(d_image), _ptr(d_dir), flags, _stream(stream)))


def camera_sphere_tangents(yaw, pitch, dist, fovy, width, height):
    """[4][12]: d frame / d (yaw, pitch, dist, fovy), angles in radians."""
    out = (ctypes.c_float * 48)()
    _check(lib().ddvr_camera_sphere_tangents(yaw, pitch, dist, fovy, width, height, out))
    return [list(out[12 * k:12 * k + 12]) for k in range(4)]


def abi_version() -> int:
    return lib().ddvr_abi_version()


def camera_from_sphere(yaw: float, pitch: float, dist: float, fovy: float, width: int,
                       height: int) -> Camera:
    """Angles in radians (see include/ddvr.h)."""
    cam = Camera()
    _check(lib().ddvr_camera_from_sphere(yaw, pitch, dist, fovy, width, height,
                                         ctypes.byref(cam)))
    return cam


def camera_grad_to_sphere(yaw, pitch, dist, fovy, width, height, d_frame: Sequence[float]):
    df = (ctypes.c_float * 12)(*[float(x) for x in d_frame])
    out = (ctypes.c_float * 4)()
    _check(lib().ddvr_camera_grad_to_sphere(yaw, pitch, dist, fovy, width, height, df, out))
    return list(out)


TUNING_DEFAULT = {"waves": 4, "lds_cap": 7168, "slab_k": 64, "slab_kmax": 256, "cell_acc": 1,
                  "lane_map": 2, "schedule": 0, "slab_axis": 1}


def set_tuning(**kw):
    """Set the process-wide launch shape; unspecified fields keep their value."""
    cur = get_tuning()
    cur.update(kw)
    t = Tuning(*[int(cur[f]) for f, _ in Tuning._fields_])
    _check(lib().ddvr_set_tuning(ctypes.byref(t)))


def get_tuning() -> dict:
    t = Tuning()
    _check(lib().ddvr_get_tuning(ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in Tuning._fields_}


def cast_volume(src, dst, stream=None):
    """dst (f32/f16/bf16 device tensor) <- src (float32 device tensor), RNE."""
    assert src.numel() == dst.numel() and src.is_contiguous() and dst.is_contiguous()
    _check(lib().ddvr_cast_volume(_ptr(src), _ptr(dst), dtype_code(dst), src.numel(),
                                  _stream(stream)))


def render_forward(volume, tf, cam: Camera, step: float, model: int, image, transmittance=None,
                   flags: int = 0, stream=None):
    v, t = volume_desc(volume), tf_desc(tf)
    _check(lib().ddvr_render_forward(ctypes.byref(v), ctypes.byref(t), ctypes.byref(cam), step,
                                     model, _ptr(image), _ptr(transmittance), flags,
                                     _stream(stream)))


def adjoint_workspace_size(volume, cam: Camera, step: float, model: int, flags: int = 0) -> int:
    v = volume_desc(volume)
    n = ctypes.c_size_t(0)
    _check(lib().ddvr_adjoint_workspace_size(ctypes.byref(v), ctypes.byref(cam), step, model,
                                             flags, ctypes.byref(n)))
    return n.value


def render_adjoint(volume, tf, cam: Camera, step: float, model: int, image, transmittance,
                   d_image, grads: Grads, flags: int = 0, workspace=None,
                   count_fallback: bool = False, stream=None) -> int:
    v, t = volume_desc(volume), tf_desc(tf)
    nfb = ctypes.c_int32(0)
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(lib().ddvr_render_adjoint(
        ctypes.byref(v), ctypes.byref(t), ctypes.byref(cam), step, model, _ptr(image),
        _ptr(transmittance), _ptr(d_image), ctypes.byref(grads), flags, _ptr(workspace),
        ws_bytes, ctypes.byref(nfb) if count_fallback else None, _stream(stream)))
    return nfb.value


def render_adjoint_noalloc(volume, tf, cam: Camera, step: float, model: int, image,
                           transmittance, d_image, grads: Grads, flags: int = 0,
                           count_fallback: bool = False, stream=None) -> int:
    """render_adjoint with the fallback's scratch in the library's static
    device array (no workspace, no allocation)."""
    v, t = volume_desc(volume), tf_desc(tf)
    nfb = ctypes.c_int32(0)
    _check(lib().ddvr_render_adjoint_noalloc(
        ctypes.byref(v), ctypes.byref(t), ctypes.byref(cam), step, model, _ptr(image),
        _ptr(transmittance), _ptr(d_image), ctypes.byref(grads), flags,
        ctypes.byref(nfb) if count_fallback else None, _stream(stream)))
    return nfb.value


def render_fused_l2(volume, tf, cam: Camera, step: float, model: int, target, loss_scale: float,
                    image, transmittance, grads: Grads, flags: int = 0, workspace=None,
                    loss_out=None, count_fallback: bool = False, stream=None) -> int:
    v, t = volume_desc(volume), tf_desc(tf)
    nfb = ctypes.c_int32(0)
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(lib().ddvr_render_fused_l2(
        ctypes.byref(v), ctypes.byref(t), ctypes.byref(cam), step, model, _ptr(target),
        loss_scale, _ptr(image), _ptr(transmittance), ctypes.byref(grads), flags,
        _ptr(workspace), ws_bytes, ctypes.byref(nfb) if count_fallback else None,
        _ptr(loss_out), _stream(stream)))
    return nfb.value


class Batch:
    """Many views (of one or several grids) rendered in one launch per pass."""

    def __init__(self, volumes, tfs, views: Sequence[View], model: int, flags: int = 0,
                 d_volumes=None, d_tfs=None, stream=None):
        self._keep = (volumes, tfs, views, d_volumes, d_tfs)
        nv = len(volumes)
        vd = (Volume * nv)(*[volume_desc(v) for v in volumes])
        ntf = 0 if not tfs else len(tfs)
        td = (TF * max(ntf, 1))(*[tf_desc(t) for t in (tfs or [])])
        vw = (View * len(views))(*views)
        dvs = None
        if d_volumes is not None:
            dvs = (ctypes.c_void_p * nv)(*[_ptr(d) for d in d_volumes])
        dts = None
        if d_tfs is not None:
            dts = (ctypes.c_void_p * max(ntf, 1))(*[_ptr(d) for d in d_tfs])
        h = ctypes.c_void_p()
        _check(lib().ddvr_batch_create(vd, nv, td if ntf else None, ntf, vw, len(views), model,
                                       flags, dvs, dts, _stream(stream), ctypes.byref(h)))
        self.handle = h

    def workspace_size(self) -> int:
        n = ctypes.c_size_t(0)
        _check(lib().ddvr_batch_workspace_size(self.handle, ctypes.byref(n)))
        return n.value

    def sample_count(self) -> int:
        n = ctypes.c_int64(0)
        _check(lib().ddvr_batch_sample_count(self.handle, ctypes.byref(n)))
        return n.value

    def run(self, pass_: int, loss_scale: float = 0.0, loss_out=None, workspace=None,
            graph: bool = False, stream=None):
        ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
        fn = lib().ddvr_batch_run_graph if graph else lib().ddvr_batch_run
        _check(fn(self.handle, pass_, loss_scale, _ptr(loss_out), _ptr(workspace), ws_bytes,
                  _stream(stream)))

    def graph_builds(self) -> int:
        """Graphs recorded by run(graph=True) so far."""
        n = ctypes.c_int64(0)
        _check(lib().ddvr_batch_graph_builds(self.handle, ctypes.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "handle", None):
            lib().ddvr_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """The whole step of a batch (forward, loss gradient, adjoint, fallback)
    recorded once into one HIP graph; run() replays it."""

    def __init__(self, batch: Batch, loss: int, loss_scale: float = 1.0, loss_out=None,
                 workspace=None, stream=None):
        self._keep = (batch, loss_out, workspace)
        self.n_views = len(batch._keep[2])
        ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
        h = ctypes.c_void_p()
        _check(lib().ddvr_plan_create(batch.handle, loss, loss_scale, _ptr(loss_out),
                                      _ptr(workspace), ws_bytes, _stream(stream),
                                      ctypes.byref(h)))
        self.handle = h

    def run(self, stream=None):
        _check(lib().ddvr_plan_execute(self.handle, _stream(stream)))

    def loss_terms(self, stream=None) -> List[float]:
        """Entropy plans: OE of every view at the last replay (synchronises)."""
        out = (ctypes.c_double * self.n_views)()
        _check(lib().ddvr_plan_loss_terms(self.handle, out, self.n_views, _stream(stream)))
        return list(out)

    def close(self):
        if getattr(self, "handle", None):
            lib().ddvr_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def valu_probe(mode: int, blocks: int, iters: int, out, stream=None) -> int:
    """One launch of the VALU issue-rate probe (mode 0 float32 FMA, 1 int add);
    returns the lane-operations it executes."""
    n = ctypes.c_int64(0)
    _check(lib().ddvr_valu_probe(mode, blocks, iters, _ptr(out), ctypes.byref(n),
                                 _stream(stream)))
    return n.value


def make_view(volume_index: int, cam: Camera, step: float, image, transmittance=None,
              d_image=None, target=None, d_camera=None, d_step=None, tf_index: int = -1) -> View:
    return View(volume_index, tf_index, cam, step, _ptr(image), _ptr(transmittance),
                _ptr(d_image), _ptr(target), _ptr(d_camera), _ptr(d_step))


def color_tau_max(color, out, stream=None):
    """out (device float32 tensor of one element) = max of the colour volume's
    extinction channel."""
    v = volume_desc(color)
    _check(lib().ddvr_color_tau_max(ctypes.byref(v), _ptr(out), _stream(stream)))


def density_from_color(color, tf, d_out, d_prev=None, alpha=None, beta: float = 1.0,
                       seed: int = 0, sweep: int = 0, ncand: int = 256, cost_out=None,
                       n_changed=None, stream=None):
    """One density-from-colour sweep (Sec. 5.4) into d_out.  alpha=None takes
    the paper's 1/max(tau_T), reduced on the device and read back."""
    v, t = volume_desc(color), tf_desc(tf)
    if alpha is None:
        import torch
        mx = torch.empty(1, dtype=torch.float32, device=d_out.device)
        color_tau_max(color, mx, stream)
        alpha = 1.0 / float(mx.item())
    _check(lib().ddvr_density_from_color(
        ctypes.byref(v), ctypes.byref(t), _ptr(d_prev), float(alpha), float(beta),
        ctypes.c_uint64(seed), int(sweep), int(ncand), _ptr(d_out), _ptr(cost_out),
        _ptr(n_changed), _stream(stream)))
    return alpha


# ---------------------------------------------------------------------------
# the reconstruction loop (Sec. 5.1-5.3)
# ---------------------------------------------------------------------------
def tf_prior(tf, lam: float, d_tf=None, loss_out=None, stream=None):
    """loss_out += lam L_prior(tf), d_tf += its gradient (device tensors)."""
    assert tf.is_contiguous() and tf.dim() == 2 and tf.shape[1] == 4
    _check(lib().ddvr_tf_prior(_ptr(tf), tf.shape[0], float(lam), _ptr(d_tf), _ptr(loss_out),
                               _stream(stream)))


def volume_prior(volume, lam: float, d_volume=None, loss_out=None, stream=None):
    """The smoothing prior on a [nz][ny][nx] float32 grid in 3D."""
    assert volume.is_contiguous() and volume.dim() == 3
    nz, ny, nx = volume.shape
    _check(lib().ddvr_volume_prior(_ptr(volume), nx, ny, nz, float(lam), _ptr(d_volume),
                                   _ptr(loss_out), _stream(stream)))


def opacity_entropy(image, work, value_out=None, d_image=None, scale: float = 1.0, stream=None):
    """OE of an [H][W][4] (alpha = channel 3) or [H][W] image; work: 2 float64."""
    ch = 4 if (image.dim() == 3 and image.shape[-1] == 4) else 1
    _check(lib().ddvr_opacity_entropy(_ptr(image), image.numel() // ch, ch, _ptr(work),
                                      _ptr(value_out), _ptr(d_image), float(scale),
                                      _stream(stream)))


def adam_step(param, grad, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8, lo: float = float("-inf"), hi: float = float("inf"),
              store=None, zero_grad: bool = False, stream=None):
    """One fused Adam step on float32 tensors (optionally writing the storage
    copy `store` and zeroing `grad`)."""
    st = dtype_code(store) if store is not None else F32
    _check(lib().ddvr_adam_step(_ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(), int(t),
                                float(lr), float(beta1), float(beta2), float(eps), float(lo),
                                float(hi), _ptr(store), st, 1 if zero_grad else 0,
                                _stream(stream)))


def resample_volume(src, dst, stream=None):
    """Trilinear resampling of src [sz][sy][sx] onto dst [dz][dy][dx] (float32),
    or of [..][C] grids of C interleaved channels, each on its own."""
    if src.dim() == 4:
        if dst.dim() != 4 or dst.shape[3] != src.shape[3]:
            raise ValueError("src and dst need the same channel count")
        sz, sy, sx, C = src.shape
        dz, dy, dx, _ = dst.shape
        _check(lib().ddvr_resample_channels(_ptr(src), C, sx, sy, sz, _ptr(dst), dx, dy, dz,
                                            _stream(stream)))
        return
    sz, sy, sx = src.shape
    dz, dy, dx = dst.shape
    _check(lib().ddvr_resample_volume(_ptr(src), sx, sy, sz, _ptr(dst), dx, dy, dz,
                                      _stream(stream)))
