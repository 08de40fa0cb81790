"""The allocation-free adjoint (ddvr_render_adjoint_noalloc): the checkpoint
fallback's scratch lives in the library's static device array instead of a
caller's workspace.  Its results must equal ddvr_render_adjoint's (with a
workspace) on problems whose rays take the fallback, on two calls in a row
(the second smaller: the array keeps the first call's contents), and a view
too large for the array is refused before any launch."""
import numpy as np
import pytest

from harness import (Problem, assert_dv_close, assert_grad_close, device_volume, gpu_camera,
                     oracle_forward, tie_mask)
from test_gpu_parity import ea_problem

pytestmark = pytest.mark.gpu


def _run(p, flags, noalloc):
    import torch
    from paper_2107_12672_amd import ddvr as d
    vol = device_volume(p)
    tf = torch.from_numpy(p.tf).cuda() if p.tf is not None else None
    cam = gpu_camera(p)
    img = torch.zeros(p.H * p.W * p.C, device="cuda")
    tr = torch.zeros(p.H * p.W, device="cuda")
    d.render_forward(vol, tf, cam, p.step, p.model, img, tr)
    rng = np.random.default_rng(13)
    g = torch.from_numpy((rng.normal(size=p.H * p.W * p.C) / (p.H * p.W)).astype(np.float32)).cuda()
    dV = torch.zeros(p.volume.shape, device="cuda")
    dTF = torch.zeros_like(tf) if tf is not None else None
    dcam = torch.zeros(12, device="cuda")
    dstep = torch.zeros(1, device="cuda")
    grads = d.grads_desc(dV, dTF, dcam, dstep)
    if noalloc:
        nfb = d.render_adjoint_noalloc(vol, tf, cam, p.step, p.model, img, tr, g, grads,
                                       flags=flags, count_fallback=True)
    else:
        n = d.adjoint_workspace_size(vol, cam, p.step, p.model, flags)
        ws = torch.zeros(n // 4 + 1, dtype=torch.int32, device="cuda")
        nfb = d.render_adjoint(vol, tf, cam, p.step, p.model, img, tr, g, grads, flags=flags,
                               workspace=ws, count_fallback=True)
    torch.cuda.synchronize()
    return (nfb, dV.double().cpu().numpy(),
            dTF.double().cpu().numpy() if dTF is not None else None,
            dcam.double().cpu().numpy(), float(dstep.item()))


def _same(a, b, what):
    """The same kernels on the same inputs: equal up to the order of float
    atomics (density 1e-5 norm-wise; TF, camera and step entries 1e-4 of
    max(|x|, 1e-2 of the array's scale), inside the 1e-3 parity bound)."""
    assert a[0] == b[0] and a[0] > 0, (what, a[0], b[0])      # the fallback ran
    assert_dv_close(a[1], b[1], f"{what} dV", 1e-5)
    if a[2] is not None:
        assert_grad_close(a[2], b[2], f"{what} dTF", 1e-4)
    assert_grad_close(a[3], b[3], f"{what} dcam", 1e-4)
    assert_grad_close([a[4]], [b[4]], f"{what} dstep", 1e-4)


def test_noalloc_adjoint_equals_the_workspace_adjoint_twice():
    print("[case] no-alloc adjoint: EA opaque 48x40, then 32x24", flush=True)
    big = ea_problem(W=48, H=40, tau_max=2000.0, seed=11)
    small = ea_problem(n=(20, 24, 22), W=32, H=24, tau_max=2000.0, seed=12)
    for p in (big, small):
        ref = _run(p, 0, noalloc=False)
        got = _run(p, 0, noalloc=True)
        _same(got, ref, f"EA {p.W}x{p.H}")
    # absorption-only alpha-form: rays with T_N < 2^-10 take the fallback
    ao = Problem(0, big.volume * 40.0, "f32", None, big.yaw, big.pitch, big.dist, big.fovy,
                 40, 36, big.step)
    _same(_run(ao, 2, noalloc=True), _run(ao, 2, noalloc=False), "AO alpha-form")


def test_noalloc_adjoint_refuses_views_beyond_the_static_scratch():
    import torch
    from paper_2107_12672_amd import ddvr as d
    print("[case] no-alloc adjoint: oversize view refused", flush=True)
    p = ea_problem(W=3000, H=3000)
    vol = device_volume(p)
    tf = torch.from_numpy(p.tf).cuda()
    tiny = torch.zeros(16, device="cuda")
    with pytest.raises(d.DDVRError) as e:
        d.render_adjoint_noalloc(vol, tf, gpu_camera(p), p.step, 1, tiny, tiny, tiny,
                                 d.grads_desc(tiny), flags=0)
    assert e.value.status == d.ERR_WORKSPACE and "static scratch" in str(e.value)
