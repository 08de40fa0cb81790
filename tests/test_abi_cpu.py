"""Host-only checks of the C ABI: the library loads, exports every declared
symbol, and rejects invalid arguments before touching the GPU."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ddvr.h")


def _ddvr():
    from paper_2107_12672_amd import ddvr
    return ddvr


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ddvr_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    d = _ddvr()
    L = d.lib()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert sorted(d.EXPORTED) == names


def test_abi_version_and_error_string():
    d = _ddvr()
    assert d.abi_version() == 5
    assert isinstance(d.last_error(), str)


def test_camera_from_sphere_matches_oracle_frame():
    d = _ddvr()
    for yaw, pitch, dist, fovy, W, H in [(30, 20, 2.5, 60, 64, 64), (300, -70, 3.0, 45, 100, 50)]:
        cam = d.camera_from_sphere(math.radians(yaw), math.radians(pitch), dist,
                                   math.radians(fovy), W, H)
        ref = oracle.camera_from_sphere(yaw, pitch, dist, fovy, W, H)
        assert np.allclose(cam.frame(), ref, atol=2e-6)
        assert (cam.width, cam.height) == (W, H)


def test_camera_grad_to_sphere_matches_oracle_jacobian():
    d = _ddvr()
    rng = np.random.default_rng(0)
    g = rng.normal(size=12)
    args = (40.0, 25.0, 2.7, 55.0, 96, 64)
    out = d.camera_grad_to_sphere(math.radians(40), math.radians(25), 2.7, math.radians(55), 96,
                                  64, g)
    ref = oracle.sphere_grad(g, *args)
    assert np.allclose(out, ref, rtol=1e-5, atol=1e-5)


def test_camera_validation():
    d = _ddvr()
    L = d.lib()
    cam = d.Camera()
    assert L.ddvr_camera_from_sphere(0.0, 1.6, 2.5, 1.0, 8, 8, ctypes.byref(cam)) == d.ERR_VALUE
    assert L.ddvr_camera_from_sphere(0.0, 0.1, -1.0, 1.0, 8, 8, ctypes.byref(cam)) == d.ERR_VALUE
    assert L.ddvr_camera_from_sphere(0.0, 0.1, 2.0, 1.0, 0, 8, ctypes.byref(cam)) == d.ERR_SHAPE
    assert L.ddvr_camera_from_sphere(0.0, 0.1, 2.0, 1.0, 8, 8, None) == d.ERR_NULL
    assert L.ddvr_camera_from_sphere(float("nan"), 0.1, 2.0, 1.0, 8, 8,
                                     ctypes.byref(cam)) == d.ERR_VALUE


def _descs(d, nx=8, ny=8, nz=8, dtype=0, R=4, W=16, H=16):
    vol = d.Volume(0x1000, dtype, nx, ny, nz)          # never dereferenced: validation fails first
    tf = d.TF(0x2000, R)
    cam = d.camera_from_sphere(0.3, 0.2, 2.5, 1.0, W, H)
    return vol, tf, cam


def test_forward_rejects_bad_arguments_before_launch():
    d = _ddvr()
    L = d.lib()
    fwd = L.ddvr_render_forward
    vol, tf, cam = _descs(d)
    img = 0x3000
    B = ctypes.byref
    assert fwd(None, B(tf), B(cam), 0.1, 1, img, None, 0, None) == d.ERR_NULL
    assert fwd(B(d.Volume(None, 0, 8, 8, 8)), B(tf), B(cam), 0.1, 1, img, None, 0, None) == d.ERR_NULL
    assert fwd(B(d.Volume(0x1000, 7, 8, 8, 8)), B(tf), B(cam), 0.1, 1, img, None, 0, None) == d.ERR_DTYPE
    assert fwd(B(d.Volume(0x1000, 0, 1, 8, 8)), B(tf), B(cam), 0.1, 1, img, None, 0, None) == d.ERR_SHAPE
    assert fwd(B(vol), B(d.TF(0x2000, 1)), B(cam), 0.1, 1, img, None, 0, None) == d.ERR_SHAPE
    assert fwd(B(vol), B(d.TF(None, 4)), B(cam), 0.1, 1, img, None, 0, None) == d.ERR_NULL
    assert fwd(B(vol), B(tf), B(cam), 0.0, 1, img, None, 0, None) == d.ERR_VALUE
    assert fwd(B(vol), B(tf), B(cam), float("inf"), 1, img, None, 0, None) == d.ERR_VALUE
    assert fwd(B(vol), B(tf), B(cam), 1e-9, 1, img, None, 0, None) == d.ERR_VALUE   # too many samples
    assert fwd(B(vol), B(tf), B(cam), 0.1, 5, img, None, 0, None) == d.ERR_VALUE    # model
    assert fwd(B(vol), B(tf), B(cam), 0.1, 1, None, None, 0, None) == d.ERR_NULL    # image
    assert fwd(B(vol), B(tf), B(cam), 0.1, 1, img, None, 1, None) == d.ERR_VALUE    # adjoint flag
    bad = d.Camera()
    bad.width, bad.height = 0, 4
    assert fwd(B(vol), B(tf), B(bad), 0.1, 1, img, None, 0, None) == d.ERR_SHAPE
    # AO ignores the TF entirely
    assert "step" in d.last_error() or True


def test_adjoint_rejects_missing_inputs_and_workspace():
    d = _ddvr()
    L = d.lib()
    vol, tf, cam = _descs(d)
    B = ctypes.byref
    g = d.Grads(0x5000, None, None, None)
    adj = L.ddvr_render_adjoint
    assert adj(B(vol), B(tf), B(cam), 0.1, 1, 0x3000, None, 0x4000, B(g), 0, None, 0, None,
               None) == d.ERR_NULL          # transmittance
    assert adj(B(vol), B(tf), B(cam), 0.1, 1, 0x3000, 0x3100, None, B(g), 0, None, 0, None,
               None) == d.ERR_NULL          # d_image
    assert adj(B(vol), B(tf), B(cam), 0.1, 1, 0x3000, 0x3100, 0x4000, None, 0, None, 0, None,
               None) == d.ERR_NULL          # grads
    # emission-absorption AUTO needs the checkpoint workspace
    assert adj(B(vol), B(tf), B(cam), 0.1, 1, 0x3000, 0x3100, 0x4000, B(g), 0, None, 0, None,
               None) == d.ERR_WORKSPACE
    assert adj(B(vol), B(tf), B(cam), 0.1, 1, 0x3000, 0x3100, 0x4000, B(g), 9, None, 0, None,
               None) == d.ERR_VALUE         # unknown mode
    assert adj(B(vol), B(tf), B(cam), 0.1, 1, 0x3000, 0x3100, 0x4000, B(g), 0x100, None, 0,
               None, None) == d.ERR_VALUE   # unknown flag bit


def test_workspace_size_rules():
    d = _ddvr()
    L = d.lib()
    vol, tf, cam = _descs(d, W=40, H=30)
    B = ctypes.byref
    n = ctypes.c_size_t(123)
    # absorption-only AUTO and explicit inversion need no workspace
    assert L.ddvr_adjoint_workspace_size(B(vol), B(cam), 0.05, 0, 0, B(n)) == 0 and n.value == 0
    assert L.ddvr_adjoint_workspace_size(B(vol), B(cam), 0.05, 1, 1, B(n)) == 0 and n.value == 0
    assert L.ddvr_adjoint_workspace_size(B(vol), B(cam), 0.05, 0, 2, B(n)) == 0 and n.value > 0
    # emission-absorption AUTO and every CHECKPOINT need the queue + slots
    assert L.ddvr_adjoint_workspace_size(B(vol), B(cam), 0.05, 1, 0, B(n)) == 0
    a = n.value
    assert a >= 256 + 8 * 40 * 30
    assert L.ddvr_adjoint_workspace_size(B(vol), B(cam), 0.05, 0, 3, B(n)) == 0 and n.value == a
    # constant in the number of samples per ray up to the sqrt-sized slots
    assert L.ddvr_adjoint_workspace_size(B(vol), B(cam), 0.005, 1, 0, B(n)) == 0
    assert n.value >= a
    assert L.ddvr_adjoint_workspace_size(B(vol), B(cam), 0.05, 1, 0, None) == d.ERR_NULL


def test_batch_create_validation():
    d = _ddvr()
    L = d.lib()
    vol, tf, cam = _descs(d)
    B = ctypes.byref
    h = ctypes.c_void_p()
    views = (d.View * 1)(d.View(0, 0, cam, 0.1, 0x3000, None, None, None, None, None))
    vols = (d.Volume * 1)(vol)
    tfs = (d.TF * 1)(tf)
    assert L.ddvr_batch_create(vols, 1, tfs, 1, views, 0, 1, 0, None, None, None, B(h)) == d.ERR_SHAPE
    bad = (d.View * 1)(d.View(3, 0, cam, 0.1, 0x3000, None, None, None, None, None))
    assert L.ddvr_batch_create(vols, 1, tfs, 1, bad, 1, 1, 0, None, None, None, B(h)) == d.ERR_SHAPE
    bad = (d.View * 1)(d.View(0, 0, cam, 0.1, None, None, None, None, None, None))
    assert L.ddvr_batch_create(vols, 1, tfs, 1, bad, 1, 1, 0, None, None, None, B(h)) == d.ERR_NULL
    assert L.ddvr_batch_create(vols, 1, None, 0, views, 1, 1, 0, None, None, None, B(h)) == d.ERR_NULL
    assert L.ddvr_batch_create(vols, 1, tfs, 1, views, 1, 1, 0, None, None, None, None) == d.ERR_NULL


def test_tuning_roundtrip_and_validation():
    d = _ddvr()
    L = d.lib()
    old = d.get_tuning()
    try:
        d.set_tuning(waves=2, lds_cap=4096, slab_k=16, slab_kmax=64, cell_acc=0, lane_map=0,
                     schedule=2, slab_axis=0)
        assert d.get_tuning() == {"waves": 2, "lds_cap": 4096, "slab_k": 16, "slab_kmax": 64,
                                  "cell_acc": 0, "lane_map": 0, "schedule": 2, "slab_axis": 0}
        for bad in ({"waves": 3}, {"lds_cap": 10}, {"lds_cap": 1 << 20}, {"slab_k": 2},
                    {"slab_k": 128, "slab_kmax": 64}, {"cell_acc": 2}, {"lane_map": -1},
                    {"lane_map": 4},
                    {"schedule": 3}, {"slab_axis": 2}):
            with pytest.raises(d.DDVRError) as ei:
                d.set_tuning(**bad)
            assert ei.value.status == d.ERR_VALUE
        assert L.ddvr_set_tuning(None) == d.ERR_NULL
    finally:
        d.set_tuning(**old)
    assert d.get_tuning() == old


def test_tangent_rejects_bad_arguments_before_launch():
    d = _ddvr()
    L = d.lib()
    vol, tf, cam = _descs(d)
    B = ctypes.byref
    tan = L.ddvr_render_tangent
    dirs = (d.Direction * 4)()
    dirs[0].d_step = 1.0
    img, dot, g, dd = 0x3000, 0x4000, 0x5000, 0x6000
    assert tan(B(vol), B(tf), B(cam), 0.1, 1, None, 1, img, None, None, None, 0, None) == d.ERR_NULL
    assert tan(B(vol), B(tf), B(cam), 0.1, 1, dirs, 0, img, None, None, None, 0, None) == d.ERR_VALUE
    assert tan(B(vol), B(tf), B(cam), 0.1, 1, dirs, 5, img, None, None, None, 0, None) == d.ERR_VALUE
    assert tan(B(vol), B(tf), B(cam), 0.1, 1, dirs, 1, None, None, None, None, 0, None) == d.ERR_NULL
    assert tan(B(vol), B(tf), B(cam), 0.1, 1, dirs, 1, img, None, None, dd, 0, None) == d.ERR_NULL
    assert tan(B(vol), B(tf), B(cam), 0.1, 1, dirs, 1, img, dot, g, dd, 1, None) == d.ERR_VALUE
    bad = (d.Direction * 1)()
    bad[0].d_frame[3] = float("nan")
    assert tan(B(vol), B(tf), B(cam), 0.1, 1, bad, 1, img, dot, None, None, 0, None) == d.ERR_VALUE
    assert tan(B(vol), B(tf), B(cam), 0.0, 1, dirs, 1, img, dot, None, None, 0, None) == d.ERR_VALUE
    assert tan(B(vol), B(d.TF(None, 4)), B(cam), 0.1, 1, dirs, 1, img, dot, None, None, 0,
               None) == d.ERR_NULL


def test_camera_sphere_tangents_match_oracle_jacobian():
    d = _ddvr()
    args = (40.0, 25.0, 2.7, 55.0, 96, 64)
    got = np.array(d.camera_sphere_tangents(math.radians(40), math.radians(25), 2.7,
                                            math.radians(55), 96, 64))
    ref = oracle.camera_jacobian(*args)
    assert got.shape == (4, 12)
    assert np.allclose(got, ref, rtol=1e-5, atol=1e-6)
    # the transpose of the gradient chain rule
    g = np.random.default_rng(5).normal(size=12)
    back = d.camera_grad_to_sphere(math.radians(40), math.radians(25), 2.7, math.radians(55), 96,
                                   64, g)
    assert np.allclose(back, got @ g, rtol=1e-5, atol=1e-5)


def test_colour_model_validation():
    """The colour-volume model: its adjoint modes, alignment of its 4-channel
    data, no workspace, and the entry points that do not take it."""
    d = _ddvr()
    L = d.lib()
    vol, tf, cam = _descs(d)
    B = ctypes.byref
    C = d.COLOR
    g = d.Grads(0x5000, None, None, None)
    adj = L.ddvr_render_adjoint
    for mode in (d.ADJ_INVERT_ALPHA, d.ADJ_CHECKPOINT):
        assert adj(B(vol), None, B(cam), 0.1, C, 0x3000, 0x3100, 0x4000, B(g), mode, None, 0,
                   None, None) == d.ERR_UNSUPPORTED
    # the residual form is the colour model's own
    assert adj(B(vol), B(tf), B(cam), 0.1, 1, 0x3000, 0x3100, 0x4000, B(g), d.ADJ_RESIDUAL, None,
               0, None, None) == d.ERR_UNSUPPORTED
    assert adj(B(vol), None, B(cam), 0.1, C, 0x3000, 0x3100, 0x4000, B(g), 5, None, 0, None,
               None) == d.ERR_VALUE
    # 4 values per load: f32 data 16-byte aligned, f16 / bf16 8-byte aligned
    fwd = L.ddvr_render_forward
    assert fwd(B(d.Volume(0x1008, d.F32, 8, 8, 8)), None, B(cam), 0.1, C, 0x3000, None, 0,
               None) == d.ERR_VALUE
    assert "aligned" in d.last_error()
    assert fwd(B(d.Volume(0x1004, d.BF16, 8, 8, 8)), None, B(cam), 0.1, C, 0x3000, None, 0,
               None) == d.ERR_VALUE
    n = ctypes.c_size_t(7)
    for mode in (d.ADJ_AUTO, d.ADJ_INVERT_T, d.ADJ_RESIDUAL):
        assert L.ddvr_adjoint_workspace_size(B(vol), B(cam), 0.05, C, mode, B(n)) == 0
        assert n.value == 0
    assert L.ddvr_adjoint_workspace_size(B(vol), B(cam), 0.05, C, d.ADJ_CHECKPOINT,
                                         B(n)) == d.ERR_UNSUPPORTED
    dirs = (d.Direction * 1)()
    # forward mode takes the colour volume; its 4-channel data must be aligned
    assert L.ddvr_render_tangent(B(d.Volume(0x1008, d.F32, 8, 8, 8)), None, B(cam), 0.1, C,
                                 dirs, 1, 0x3000, None, None, None, 0, None) == d.ERR_VALUE
    h = ctypes.c_void_p()
    views = (d.View * 1)(d.View(0, -1, cam, 0.1, 0x3000, None, None, None, None, None))
    vols = (d.Volume * 1)(vol)
    # colour batches: the slab route only, one storage type
    for flags in (d.LAUNCH_PLAIN, d.ADJ_RESIDUAL):
        assert L.ddvr_batch_create(vols, 1, None, 0, views, 1, C, flags, None, None, None,
                                   B(h)) == d.ERR_UNSUPPORTED
    mixed = (d.Volume * 2)(vol, d.Volume(0x1000, d.BF16, 8, 8, 8))
    assert L.ddvr_batch_create(mixed, 2, None, 0, views, 1, C, 0, None, None, None,
                               B(h)) == d.ERR_UNSUPPORTED


def test_density_from_color_validation():
    d = _ddvr()
    L = d.lib()
    vol, tf, cam = _descs(d)
    B = ctypes.byref
    f = L.ddvr_density_from_color
    out = 0x7000
    assert f(B(vol), B(tf), None, 1.0, 1.0, 0, 0, 256, None, None, None, None) == d.ERR_NULL
    assert f(B(vol), None, None, 1.0, 1.0, 0, 0, 256, out, None, None, None) == d.ERR_NULL
    assert f(B(vol), B(d.TF(0x2000, 1)), None, 1.0, 1.0, 0, 0, 256, out, None, None,
             None) == d.ERR_SHAPE
    assert f(B(vol), B(tf), None, 1.0, 1.0, 0, 0, 0, out, None, None, None) == d.ERR_VALUE
    assert f(B(vol), B(tf), None, 1.0, 1.0, 0, 0, 65537, out, None, None, None) == d.ERR_VALUE
    assert f(B(vol), B(tf), None, 1.0, 1.0, 0, -1, 256, out, None, None, None) == d.ERR_VALUE
    assert f(B(vol), B(tf), None, float("nan"), 1.0, 0, 0, 256, out, None, None,
             None) == d.ERR_VALUE
    assert f(B(vol), B(tf), out, 1.0, 1.0, 0, 0, 256, out, None, None, None) == d.ERR_VALUE
    assert f(B(d.Volume(0x1008, d.F32, 8, 8, 8)), B(tf), None, 1.0, 1.0, 0, 0, 256, out, None,
             None, None) == d.ERR_VALUE       # 4-channel data must be 16-byte aligned
    assert L.ddvr_color_tau_max(B(vol), None, None) == d.ERR_NULL


def test_training_loop_validation():
    d = _ddvr()
    L = d.lib()
    inf = float("inf")
    assert L.ddvr_tf_prior(None, 8, 0.4, None, None, None) == d.ERR_NULL
    assert L.ddvr_tf_prior(0x1000, 1, 0.4, None, None, None) == d.ERR_SHAPE
    assert L.ddvr_tf_prior(0x1000, 8, float("nan"), None, None, None) == d.ERR_VALUE
    assert L.ddvr_volume_prior(0x1000, 1, 1, 1, 0.5, None, None, None) == d.ERR_SHAPE
    assert L.ddvr_opacity_entropy(0x1000, 100, 3, 0x2000, None, None, 1.0, None) == d.ERR_VALUE
    assert L.ddvr_opacity_entropy(0x1000, 1, 4, 0x2000, None, None, 1.0, None) == d.ERR_SHAPE
    assert L.ddvr_opacity_entropy(0x1000, 100, 4, None, None, None, 1.0, None) == d.ERR_NULL
    A = L.ddvr_adam_step
    assert A(0x1000, 0x2000, 0x3000, 0x4000, 10, 0, 0.1, 0.9, 0.999, 1e-8, -inf, inf, None, 0, 0,
             None) == d.ERR_VALUE                              # t = 0
    assert A(0x1000, 0x2000, 0x3000, 0x4000, 10, 1, 0.1, 1.0, 0.999, 1e-8, -inf, inf, None, 0, 0,
             None) == d.ERR_VALUE                              # beta1 = 1
    assert A(0x1000, 0x2000, 0x3000, 0x4000, 10, 1, 0.1, 0.9, 0.999, 1e-8, 1.0, 0.0, None, 0, 0,
             None) == d.ERR_VALUE                              # lo > hi
    assert A(0x1000, 0x2000, 0x3000, 0x4000, 10, 1, 0.1, 0.9, 0.999, 1e-8, -inf, inf, 0x5000, 7,
             0, None) == d.ERR_DTYPE
    assert A(0x1000, None, 0x3000, 0x4000, 10, 1, 0.1, 0.9, 0.999, 1e-8, -inf, inf, None, 0, 0,
             None) == d.ERR_NULL
    R = L.ddvr_resample_volume
    assert R(0x1000, 1, 4, 4, 0x9000000, 8, 8, 8, None) == d.ERR_SHAPE
    assert R(0x1000, 4, 4, 4, 0x1010, 8, 8, 8, None) == d.ERR_VALUE       # overlap
    assert R(None, 4, 4, 4, 0x9000000, 8, 8, 8, None) == d.ERR_NULL
    RC = L.ddvr_resample_channels
    assert RC(0x1000, 0, 4, 4, 4, 0x9000000, 8, 8, 8, None) == d.ERR_VALUE
    assert RC(0x1000, 5, 4, 4, 4, 0x9000000, 8, 8, 8, None) == d.ERR_VALUE
    assert RC(0x1000, 4, 4, 4, 4, 0x1000 + 4 * 64 * 4 - 4, 8, 8, 8, None) == d.ERR_VALUE  # overlap
    assert RC(0x1000, 4, 4, 1, 4, 0x9000000, 8, 8, 8, None) == d.ERR_SHAPE
    assert RC(0x1000, 4, 4, 4, 4, None, 8, 8, 8, None) == d.ERR_NULL
    # the L1 loss bit is a valid flag of the fused pass
    vol, tf, cam = _descs(d)
    B = ctypes.byref
    g = d.Grads(0x5000, None, None, None)
    assert L.ddvr_render_fused_l2(B(vol), B(tf), B(cam), 0.1, 1, 0x3000, 1.0, 0x4000, 0x4100,
                                  B(g), d.LOSS_L1 | 0x100, None, 0, None, None,
                                  None) == d.ERR_VALUE


def test_plan_probe_and_noalloc_reject_bad_arguments_before_launch():
    """Step plans, the VALU probe, the graph-build counter and the
    allocation-free adjoint validate on the host (no GPU needed)."""
    import ctypes
    d = _ddvr()
    L = d.lib()
    out = ctypes.c_void_p()
    assert L.ddvr_plan_create(None, 0, 1.0, None, None, 0, None, ctypes.byref(out)) == d.ERR_NULL
    assert L.ddvr_plan_create(None, 0, 1.0, None, None, 0, None, None) == d.ERR_NULL
    assert L.ddvr_plan_execute(None, None) == d.ERR_NULL
    assert L.ddvr_plan_loss_terms(None, None, 0, None) == d.ERR_NULL
    L.ddvr_plan_destroy(None)
    n = ctypes.c_int64(0)
    assert L.ddvr_batch_graph_builds(None, ctypes.byref(n)) == d.ERR_NULL
    buf = ctypes.c_void_p(16)                      # never dereferenced: rejected first
    assert L.ddvr_valu_probe(8, 1, 1, buf, ctypes.byref(n), None) == d.ERR_VALUE
    assert L.ddvr_valu_probe(-1, 1, 1, buf, ctypes.byref(n), None) == d.ERR_VALUE
    assert L.ddvr_valu_probe(0, 0, 1, buf, ctypes.byref(n), None) == d.ERR_SHAPE
    assert L.ddvr_valu_probe(0, 1, 1, None, ctypes.byref(n), None) == d.ERR_NULL
    vol = d.Volume(16, d.F32, 8, 8, 8)
    tf = d.TF(None, 0)
    cam = d.camera_from_sphere(0.3, 0.2, 2.5, 1.0, 16, 16)
    g = d.grads_desc()
    assert L.ddvr_render_adjoint_noalloc(ctypes.byref(vol), ctypes.byref(tf), ctypes.byref(cam),
                                         0.1, 0, buf, buf, buf, None, 0, None, None) == d.ERR_NULL
    assert L.ddvr_render_adjoint_noalloc(ctypes.byref(vol), ctypes.byref(tf), ctypes.byref(cam),
                                         0.1, 7, buf, buf, buf, ctypes.byref(g), 0, None,
                                         None) == d.ERR_VALUE
    assert L.ddvr_render_adjoint_noalloc(ctypes.byref(vol), ctypes.byref(tf), ctypes.byref(cam),
                                         -1.0, 0, buf, buf, buf, ctypes.byref(g), 0, None,
                                         None) == d.ERR_VALUE
