"""The torch.autograd wrapper on the GPU against the FP64 oracle, and a
directional finite difference of the oracle's own forward (independent of
any adjoint) at a full configuration."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from harness import (Problem, assert_dv_close, assert_grad_close, assert_images_close,
                     dequantized, gpu_camera, kink_mask, oracle_adjoint, oracle_camera,
                     oracle_forward, tie_mask)

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _ea(storage="f32", W=64, H=48):
    rng = np.random.default_rng(21)
    vol = synth.blob_volume((36, 40, 32), 5, rng, sigma_world=(0.12, 0.3), amplitude=0.6,
                            noise=0.02)
    tf = synth.random_tf(12, rng, 10.0)
    return Problem(1, vol, storage, tf, 117.0, 28.0, 2.4, 55.0, W, H, 0.5 * 2 / 39)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_autograd_matches_oracle_all_parameters(storage):
    import torch
    from paper_2107_12672_amd import autograd as ag, ddvr as d
    p = _ea(storage)
    _say(f"autograd EA storage={storage}")
    ora = oracle_forward(p)
    mask = tie_mask(ora["ratio"]) | kink_mask(p)
    rng = np.random.default_rng(22)
    g = rng.normal(size=ora["image"].shape) / ora["image"].size
    g[mask] = 0.0
    dev = torch.device("cuda")
    V = torch.from_numpy(p.volume).to(dev).requires_grad_(True)
    T = torch.from_numpy(p.tf).to(dev).requires_grad_(True)
    yaw, pitch, dist = (torch.tensor(math.radians(p.yaw), requires_grad=True),
                        torch.tensor(math.radians(p.pitch), requires_grad=True),
                        torch.tensor(p.dist, requires_grad=True))
    step = torch.tensor(p.step, requires_grad=True)
    frame = ag.camera_frame(yaw, pitch, dist, math.radians(p.fovy), p.W, p.H)
    sdt = {"f32": torch.float32, "bf16": torch.bfloat16}[storage]
    img = ag.render(V, T, frame, step, d.EMISSION_ABSORPTION, p.W, p.H, storage=sdt)
    gt = torch.from_numpy(g.reshape(p.H, p.W, 4).astype(np.float32)).to(dev)
    (img * gt).sum().backward()
    ref = oracle_adjoint(p, g)
    assert_dv_close(V.grad.double().cpu().numpy(), ref["dV"], "autograd dV")
    assert_grad_close(T.grad.double().cpu().numpy(), ref["dTF"], "autograd dTF")
    sph = oracle.sphere_grad(ref["dcam"], p.yaw, p.pitch, p.dist, p.fovy, p.W, p.H)
    got = np.array([yaw.grad.item(), pitch.grad.item(), dist.grad.item()])
    assert_grad_close(got, sph[:3], "autograd yaw/pitch/dist")
    assert_grad_close([step.grad.item()], [ref["dstep"]], "autograd step")


def test_directional_derivative_against_oracle_finite_difference_c2():
    """(L(th + e v) - L(th - e v)) / 2e of the FP64 oracle forward on a pixel
    subset vs <grad L, v> from the GPU adjoint (autograd path), full C2 size."""
    import torch
    from paper_2107_12672_amd import autograd as ag, ddvr as d
    w = synth.make_c2()
    v = w.views[0]
    p = Problem(1, w.volume, "f32", w.tf, v.yaw, v.pitch, v.dist, v.fovy, v.width, v.height,
                w.step_world)
    _say("C2 directional FD")
    rng = np.random.default_rng(23)
    pix = np.sort(rng.choice(p.W * p.H, size=1500, replace=False)).astype(np.int32)
    ora = oracle_forward(p, pix=pix)
    hit = ora["nsamp"] > 0
    keep = hit & ~tie_mask(ora["ratio"]) & ~kink_mask(p, pix=pix)
    pix = pix[keep]
    wts = rng.normal(size=(pix.size, 4))
    dev = torch.device("cuda")
    V = torch.from_numpy(p.volume).to(dev).requires_grad_(True)
    T = torch.from_numpy(p.tf).to(dev).requires_grad_(True)
    yaw = torch.tensor(math.radians(p.yaw), requires_grad=True)
    step = torch.tensor(p.step, requires_grad=True)
    frame = ag.camera_frame(yaw, math.radians(p.pitch), p.dist, math.radians(p.fovy), p.W, p.H)
    img = ag.render(V, T, frame, step, d.EMISSION_ABSORPTION, p.W, p.H)
    gfull = torch.zeros(p.H * p.W, 4, device=dev)
    gfull[torch.from_numpy(pix.astype(np.int64)).to(dev)] = torch.from_numpy(
        wts.astype(np.float32)).to(dev)
    (img.reshape(-1, 4) * gfull).sum().backward()
    # random direction in (V, TF, yaw, step)
    dV = rng.normal(size=p.volume.shape) * 0.01
    dT = rng.normal(size=p.tf.shape) * np.array([0.05, 0.05, 0.05, 0.5])
    dyaw, dstep = 0.01, 0.01 * p.step
    lin = float((V.grad.double().cpu().numpy() * dV).sum() + (T.grad.double().cpu().numpy() * dT).sum()
                + yaw.grad.item() * dyaw + step.grad.item() * dstep)

    def loss(eps):
        vol = p.volume.astype(np.float64) + eps * dV
        tf = p.tf.astype(np.float64) + eps * dT
        cam = oracle.camera_from_sphere(p.yaw + math.degrees(eps * dyaw), p.pitch, p.dist,
                                        p.fovy, p.W, p.H)
        out = oracle.render(vol, tf, cam, p.W, p.H, p.step + eps * dstep, 1, pix=pix)
        return float((out["image"] * wts).sum())

    eps = 1e-4
    fd = (loss(eps) - loss(-eps)) / (2 * eps)
    # a central difference of the oracle, not the oracle's gradient: its own
    # truncation (eps^2 times the third derivative, which the TF's kinks make
    # large along a random direction) sets the bound here, twice the parity
    # bound of the gradient checks above
    print(f"[result] directional FD {fd:.6g}, linearisation {lin:.6g}, "
          f"relative {abs(fd - lin) / max(abs(fd), 1e-300):.3g}", flush=True)
    assert abs(fd - lin) <= 2e-3 * abs(fd) + 1e-6, (fd, lin)


def test_viewpoint_autograd_forward_mode_matches_oracle():
    """render_viewpoint: pose (yaw, pitch, dist, fovy) and step gradients by
    forward mode, grid and TF gradients by the adjoint, all against the
    oracle's adjoint chained to the sphere pose."""
    import torch
    from paper_2107_12672_amd import autograd as ag, ddvr as d
    p = _ea("f32")
    _say("viewpoint autograd (forward mode)")
    ora = oracle_forward(p)
    mask = tie_mask(ora["ratio"]) | kink_mask(p)
    rng = np.random.default_rng(24)
    g = rng.normal(size=ora["image"].shape) / ora["image"].size
    g[mask] = 0.0
    dev = torch.device("cuda")
    V = torch.from_numpy(p.volume).to(dev).requires_grad_(True)
    T = torch.from_numpy(p.tf).to(dev).requires_grad_(True)
    pose = [torch.tensor(x, requires_grad=True) for x in
            (math.radians(p.yaw), math.radians(p.pitch), p.dist, math.radians(p.fovy))]
    step = torch.tensor(p.step, requires_grad=True)
    img = ag.render_viewpoint(V, T, *pose, step, d.EMISSION_ABSORPTION, p.W, p.H)
    gt = torch.from_numpy(g.reshape(p.H, p.W, 4).astype(np.float32)).to(dev)
    (img * gt).sum().backward()
    ref = oracle_adjoint(p, g)
    sph = oracle.sphere_grad(ref["dcam"], p.yaw, p.pitch, p.dist, p.fovy, p.W, p.H)
    got = np.array([t.grad.item() for t in pose])
    assert_grad_close(got, sph, "forward-mode yaw/pitch/dist/fovy")
    assert_grad_close([step.grad.item()], [ref["dstep"]], "forward-mode step")
    assert_dv_close(V.grad.double().cpu().numpy(), ref["dV"], "viewpoint dV")
    assert_grad_close(T.grad.double().cpu().numpy(), ref["dTF"], "viewpoint dTF")


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_autograd_colour_volume(storage):
    """The wrapper on the pre-shaded colour volume: gradients of the 4-channel
    master grid, the pose and the step against the oracle."""
    import torch
    from paper_2107_12672_amd import autograd as ag, ddvr as d
    from test_gpu_color import color_problem
    p = color_problem(storage=storage, W=48, H=40)
    _say(f"autograd colour storage={storage}")
    ora = oracle_forward(p)
    mask = tie_mask(ora["ratio"]) | kink_mask(p)
    rng = np.random.default_rng(23)
    g = rng.normal(size=ora["image"].shape) / ora["image"].size
    g[mask] = 0.0
    dev = torch.device("cuda")
    V = torch.from_numpy(p.volume).to(dev).requires_grad_(True)
    yaw, pitch = (torch.tensor(math.radians(p.yaw), requires_grad=True),
                  torch.tensor(math.radians(p.pitch), requires_grad=True))
    step = torch.tensor(p.step, requires_grad=True)
    frame = ag.camera_frame(yaw, pitch, torch.tensor(p.dist), math.radians(p.fovy), p.W, p.H)
    sdt = {"f32": torch.float32, "bf16": torch.bfloat16}[storage]
    img = ag.render(V, None, frame, step, d.COLOR, p.W, p.H, storage=sdt)
    assert img.shape == (p.H, p.W, 4)
    gt = torch.from_numpy(g.reshape(p.H, p.W, 4).astype(np.float32)).to(dev)
    (img * gt).sum().backward()
    ref = oracle_adjoint(p, g)
    assert V.grad.shape == V.shape
    assert_dv_close(V.grad.double().cpu().numpy(), ref["dV"], "autograd colour dV")
    sph = oracle.sphere_grad(ref["dcam"], p.yaw, p.pitch, p.dist, p.fovy, p.W, p.H)
    got = np.array([yaw.grad.item(), pitch.grad.item()])
    assert_grad_close(got, sph[:2], "autograd colour yaw/pitch")
    assert_grad_close([step.grad.item()], [ref["dstep"]], "autograd colour step")


def test_viewpoint_autograd_colour_volume():
    """The forward-mode viewpoint wrapper on the colour volume: pose and step
    gradients from the tangent pass, volume gradient from the adjoint."""
    import torch
    from paper_2107_12672_amd import autograd as ag, ddvr as d
    from test_gpu_color import color_problem
    p = color_problem(W=48, H=40)
    _say("viewpoint autograd colour")
    ora = oracle_forward(p)
    mask = tie_mask(ora["ratio"]) | kink_mask(p)
    rng = np.random.default_rng(25)
    g = rng.normal(size=ora["image"].shape) / ora["image"].size
    g[mask] = 0.0
    dev = torch.device("cuda")
    V = torch.from_numpy(p.volume).to(dev).requires_grad_(True)
    yaw, pitch, dist = (torch.tensor(math.radians(p.yaw), requires_grad=True),
                        torch.tensor(math.radians(p.pitch), requires_grad=True),
                        torch.tensor(p.dist, requires_grad=True))
    step = torch.tensor(p.step, requires_grad=True)
    img = ag.render_viewpoint(V, None, yaw, pitch, dist, math.radians(p.fovy), step, d.COLOR,
                              p.W, p.H)
    gt = torch.from_numpy(g.reshape(p.H, p.W, 4).astype(np.float32)).to(dev)
    (img * gt).sum().backward()
    ref = oracle_adjoint(p, g)
    assert_dv_close(V.grad.double().cpu().numpy(), ref["dV"], "viewpoint colour dV")
    sph = oracle.sphere_grad(ref["dcam"], p.yaw, p.pitch, p.dist, p.fovy, p.W, p.H)
    got = np.array([yaw.grad.item(), pitch.grad.item(), dist.grad.item()])
    assert_grad_close(got, sph[:3], "viewpoint colour yaw/pitch/dist")
    assert_grad_close([step.grad.item()], [ref["dstep"]], "viewpoint colour step")


@pytest.mark.parametrize("case", ["ea-f32", "ea-bf16", "ao-bf16", "colour-bf16"])
def test_batch_autograd_matches_oracle(case):
    """The batched wrapper: 3 views of one grid in one forward and one adjoint
    launch.  Images per view, the grid (and TF) gradient summed over the views,
    every view's camera-frame gradient and the shared step gradient, against
    the oracle view by view."""
    import dataclasses
    import torch
    from paper_2107_12672_amd import autograd as ag, ddvr as d
    from test_gpu_color import color_problem
    model_name, storage = case.split("-")
    if model_name == "colour":
        base = color_problem(storage=storage, W=48, H=40)
    else:
        base = _ea(storage)
        if model_name == "ao":
            base = dataclasses.replace(base, model=0, tf=None)
    poses = [(base.yaw, base.pitch), (base.yaw + 71.0, base.pitch - 20.0),
             (base.yaw - 133.0, base.pitch + 9.0)]
    probs = [dataclasses.replace(base, yaw=y, pitch=pt) for y, pt in poses]
    _say(f"batched autograd {case}, {len(probs)} views {base.W}x{base.H}")
    rng = np.random.default_rng(25)
    gs, oras = [], []
    for p in probs:
        ora = oracle_forward(p)
        g = rng.normal(size=ora["image"].shape) / ora["image"].size
        g[tie_mask(ora["ratio"]) | kink_mask(p)] = 0.0
        gs.append(g)
        oras.append(ora)
    dev = torch.device("cuda")
    V = torch.from_numpy(base.volume).to(dev).requires_grad_(True)
    T = None
    if base.model == 1:
        T = torch.from_numpy(base.tf).to(dev).requires_grad_(True)
    step = torch.tensor(base.step, requires_grad=True)
    frames = torch.tensor([gpu_camera(p).frame() for p in probs], dtype=torch.float32,
                          requires_grad=True)
    sdt = {"f32": torch.float32, "bf16": torch.bfloat16}[storage]
    model = {"ea": d.EMISSION_ABSORPTION, "ao": d.ABSORPTION, "colour": d.COLOR}[model_name]
    imgs = ag.render_batch(V, T, frames, step, model, base.W, base.H, storage=sdt)
    C = base.C
    shape = (base.H, base.W, C) if C == 4 else (base.H, base.W)
    assert imgs.shape == (len(probs),) + shape
    for i, ora in enumerate(oras):
        got = imgs[i].detach().double().cpu().numpy().reshape(ora["image"].shape)
        assert_images_close(got, ora, f"batched {case} view {i} image")
    gt = torch.from_numpy(np.stack([g.reshape(shape) for g in gs]).astype(np.float32)).to(dev)
    (imgs * gt).sum().backward()
    refs = [oracle_adjoint(p, g) for p, g in zip(probs, gs)]
    dV = sum(r["dV"] for r in refs)
    assert_dv_close(V.grad.double().cpu().numpy(), dV, f"batched {case} dV")
    if T is not None:
        assert_grad_close(T.grad.double().cpu().numpy(), sum(r["dTF"] for r in refs),
                          f"batched {case} dTF")
    for i, r in enumerate(refs):
        assert_grad_close(frames.grad[i].double().numpy(), r["dcam"], f"batched {case} view {i} dcam")
    assert_grad_close([step.grad.item()], [sum(r["dstep"] for r in refs)], f"batched {case} step")
    # a second backward through a new forward reuses nothing stale
    V.grad = None
    imgs2 = ag.render_batch(V, T, frames.detach(), float(base.step), model, base.W, base.H,
                            storage=sdt)
    (imgs2 * gt).sum().backward()
    assert_dv_close(V.grad.double().cpu().numpy(), dV, f"batched {case} dV again")
    if storage == "f32":
        # the float32 grid is rendered in place: changing it before the
        # backward must be refused, not differentiated at the new values
        imgs3 = ag.render_batch(V, T, frames.detach(), float(base.step), model, base.W, base.H)
        with torch.no_grad():
            V.mul_(1.0)
        with pytest.raises(RuntimeError):
            imgs3.sum().backward()


@pytest.mark.parametrize("batched", [False, True])
def test_autograd_through_the_checkpoint_fallback_on_opaque_rays(batched):
    """tau up to 2000 per world unit: over a fifth of the rays reach
    T_N < 2^-100, where the float32 inversion fails (Sec. 4.4: alpha = 1 is not
    reached in practice, but nearly opaque rays are); the wrappers' adjoint
    (AUTO) hands them to the segment-checkpoint fallback, and the gradients
    must still match the oracle's stored tape."""
    import dataclasses
    import torch
    from paper_2107_12672_amd import autograd as ag, ddvr as d
    from test_gpu_parity import ea_problem
    base = ea_problem(W=48, H=40, tau_max=2000.0, seed=11)
    probs = [base] if not batched else [base, dataclasses.replace(base, yaw=base.yaw + 97.0)]
    _say(f"autograd opaque rays, batched={batched}")
    rng = np.random.default_rng(27)
    gs = []
    for p in probs:
        ora = oracle_forward(p)
        hit = ora["nsamp"] > 0
        assert (ora["trans"][hit] < 2.0 ** -100).mean() > 0.2
        g = rng.normal(size=ora["image"].shape) / ora["image"].size
        g[tie_mask(ora["ratio"]) | kink_mask(p)] = 0.0
        gs.append(g)
    dev = torch.device("cuda")
    V = torch.from_numpy(base.volume).to(dev).requires_grad_(True)
    T = torch.from_numpy(base.tf).to(dev).requires_grad_(True)
    step = torch.tensor(base.step, requires_grad=True)
    frames = torch.tensor([gpu_camera(p).frame() for p in probs], dtype=torch.float32,
                          requires_grad=True)
    if batched:
        imgs = ag.render_batch(V, T, frames, step, d.EMISSION_ABSORPTION, base.W, base.H)
    else:
        imgs = ag.render(V, T, frames[0], step, d.EMISSION_ABSORPTION, base.W, base.H)[None]
    gt = torch.from_numpy(np.stack([g.reshape(base.H, base.W, 4) for g in gs])
                          .astype(np.float32)).to(dev)
    (imgs * gt).sum().backward()
    refs = [oracle_adjoint(p, g) for p, g in zip(probs, gs)]
    assert_dv_close(V.grad.double().cpu().numpy(), sum(r["dV"] for r in refs), "opaque dV")
    assert_grad_close(T.grad.double().cpu().numpy(), sum(r["dTF"] for r in refs), "opaque dTF")
    assert_grad_close([step.grad.item()], [sum(r["dstep"] for r in refs)], "opaque step")
    for i, r in enumerate(refs):
        assert_grad_close(frames.grad[i].double().numpy(), r["dcam"], f"opaque view {i} dcam",
                          floor_frac=5e-2)
