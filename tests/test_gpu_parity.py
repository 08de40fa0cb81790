"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Tolerances and tie handling are defined in harness.py."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from harness import (Problem, assert_dv_close, assert_dv_elementwise, assert_grad_close,
                     assert_images_close, gpu_adjoint, gpu_forward, kink_mask, oracle_adjoint,
                     oracle_camera, oracle_forward, quantisation_image_bound, tie_mask)

pytestmark = pytest.mark.gpu

PLAIN = 0x10


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def c1_problem():
    w = synth.make_c1()
    v = w.views[0]
    return Problem(0, w.volume, "f32", None, v.yaw, v.pitch, v.dist, v.fovy, v.width, v.height,
                   w.step_world), w


def ea_problem(n=(40, 48, 44), W=80, H=72, R=16, storage="f32", seed=7, tau_max=12.0,
               step_vox=0.5, yaw=63.0, pitch=-21.0):
    rng = np.random.default_rng(seed)
    vol = synth.blob_volume(n, 6, rng, sigma_world=(0.1, 0.3), amplitude=0.6, noise=0.02)
    tf = synth.random_tf(R, rng, tau_max)
    h = 2.0 / (max(n) - 1)
    return Problem(1, vol, storage, tf, yaw, pitch, 2.5, 60.0, W, H, step_vox * h)


def l2_seed(p, target_img, ties=None):
    """d_image of loss = mean((img - target)^2), zero on tie rays."""
    def f(img):
        g = 2.0 * (img - target_img) / img.size
        if ties is not None:
            g[ties] = 0.0
        return g
    return f


@pytest.mark.parametrize("flags", [0, PLAIN])
def test_c1_forward_matches_oracle(flags):
    p, _ = c1_problem()
    _say(f"C1 forward flags={flags}")
    img, tr = gpu_forward(p, flags)
    ora = oracle_forward(p)
    worst, ties = assert_images_close(img, ora, "C1 image")
    keep = ~tie_mask(ora["ratio"])
    assert np.abs(tr[keep] - ora["trans"][keep]).max() <= 1e-4
    assert (ora["nsamp"] > 0).sum() > 1000


def test_forward_is_bitwise_identical_with_and_without_lds_staging():
    """Emission-absorption: the staged and the plain launch run the same
    per-sample arithmetic, bit for bit.  Absorption-only: the staged launch
    sums each cell's run of samples in closed form, the plain one sample by
    sample -- the same sum up to float32 rounding."""
    p = ea_problem()
    _say("EA forward staged vs plain")
    a, ta = gpu_forward(p, 0)
    b, tb = gpu_forward(p, PLAIN)
    assert np.array_equal(a, b) and np.array_equal(ta, tb)
    p, _ = c1_problem()
    a, ta = gpu_forward(p, 0)
    b, tb = gpu_forward(p, PLAIN)
    assert np.abs(a - b).max() <= 1e-6 and np.abs(ta - tb).max() <= 1e-6


@pytest.mark.parametrize("flags", [0, PLAIN, 1, 2, 3])
def test_c1_adjoint_matches_oracle(flags):
    p, w = c1_problem()
    _say(f"C1 adjoint flags={flags}")
    ora = oracle_forward(p)
    ties = tie_mask(ora["ratio"]) | kink_mask(p)
    # L2 loss against the render of a second blob volume (C1 recipe)
    pt = Problem(0, w.target_volume, "f32", None, p.yaw, p.pitch, p.dist, p.fovy, p.W, p.H, p.step)
    tgt = oracle_forward(pt)["image"]
    g = 2.0 * (ora["image"] - tgt) / ora["image"].size
    g[ties] = 0.0
    got = gpu_adjoint(p, g, flags=flags)
    ref = oracle_adjoint(p, g)
    assert_dv_close(got["dV"], ref["dV"], "C1 dV")
    r = assert_dv_elementwise(got["dV"], ref["dV"], "C1 dV")
    print(f"[result] C1 flags={flags}: dV element-wise worst {r:.3g} of the bound", flush=True)
    assert_grad_close(got["dcam"], ref["dcam"], "C1 dcam")
    assert_grad_close([got["dstep"]], [ref["dstep"]], "C1 dstep")


def _c1_l2_seed():
    p, w = c1_problem()
    ora = oracle_forward(p)
    ties = tie_mask(ora["ratio"]) | kink_mask(p)
    pt = Problem(0, w.target_volume, "f32", None, p.yaw, p.pitch, p.dist, p.fovy, p.W, p.H, p.step)
    g = 2.0 * (ora["image"] - oracle_forward(pt)["image"]) / ora["image"].size
    g[ties] = 0.0
    return p, g


@pytest.mark.parametrize("flags", [0, 1])
@pytest.mark.parametrize("scale", [1.0, 1e25, 1e-30])
def test_absorption_closed_form_density_gradient_is_accurate_at_any_scale(scale, flags):
    """The absorption-only adjoint (closed form, AUTO; and the T-form
    inversion, whose d_hat is the same up to float32 drift) adds its per-cell
    sums to the LDS brick in 32-bit fixed point with a power-of-two scale
    chosen per tile from a bound on every entry; the result must stay far
    inside the float32 tolerance, for upstream gradients of ordinary, huge and
    tiny size (the last takes the float route: its scale would leave the
    exponent range)."""
    p, g = _c1_l2_seed()
    _say(f"C1 AO dV accuracy, flags={flags}, seed scale {scale:g}")
    ref = oracle_adjoint(p, g)["dV"] * scale
    got = gpu_adjoint(p, g * scale, flags=flags, want=("V",))["dV"]
    assert np.isfinite(got).all()
    assert_dv_close(got, ref, "AO dV", 2e-5)
    assert_dv_elementwise(got, ref, "AO dV")


@pytest.mark.parametrize("flags,scale", [(0, 1.0), (0, 1e20), (1, 1.0), (2, 1.0)])
def test_emission_absorption_density_gradient_fixed_point_accuracy(flags, scale):
    """Emission-absorption density gradients add to the LDS brick in 64-bit
    fixed point with a scale from a bound on every sample's d_hat (blend
    adjoint invariant and TF slopes); the bound is loose (a sum of per-ray
    worst cases over the tile), which the 22 extra bits absorb: with
    random-sign upstream gradients (heavy cancellation) the result must stay
    inside half the float32 tolerance (5e-4 norm-wise) on the T-form (AUTO,
    INVERT_T) and alpha-form routes."""
    p = ea_problem()
    _say(f"EA fixed-point dV flags={flags} scale={scale:g}")
    ora = oracle_forward(p)
    ties = tie_mask(ora["ratio"])
    rng = np.random.default_rng(17)
    g = rng.normal(size=ora["image"].shape) / ora["image"].size
    g[ties] = 0.0
    ref = oracle_adjoint(p, g)["dV"] * scale
    got = gpu_adjoint(p, g * scale, flags=flags, want=("V",))["dV"]
    assert np.isfinite(got).all()
    e = assert_dv_close(got, ref, "EA dV", 5e-4)
    print(f"[result] EA fixed-point dV error {e:.3g}", flush=True)


def test_non_finite_upstream_gradient_propagates():
    """A NaN in d_image reaches the density gradient (the tile holding it takes
    the float route); every other voxel matches the oracle without that ray."""
    p, g = _c1_l2_seed()
    _say("C1 NaN upstream gradient")
    pix = int(np.argmax(np.abs(g[:, 0])))
    g_nan = g.copy()
    g_nan[pix, 0] = np.nan
    got = gpu_adjoint(p, g_nan, want=("V",))["dV"]
    bad = np.isnan(got)
    assert bad.any() and bad.mean() < 0.05
    g0 = g.copy()
    g0[pix, 0] = 0.0
    ref = oracle_adjoint(p, g0)["dV"]
    assert_dv_close(got[~bad], ref[~bad], "dV away from the NaN ray", 2e-5)


@pytest.mark.parametrize("flags", [0, PLAIN])
def test_ea_forward_ragged_tiles(flags):
    p = ea_problem()
    _say(f"EA forward ragged flags={flags}")
    img, tr = gpu_forward(p, flags)
    ora = oracle_forward(p)
    assert_images_close(img, ora, "EA image")
    assert (ora["nsamp"] > 0).sum() > 2000


@pytest.mark.parametrize("flags", [0, PLAIN, 1, 2, 3])
def test_ea_adjoint_all_gradients(flags):
    p = ea_problem()
    _say(f"EA adjoint flags={flags}")
    ora = oracle_forward(p)
    ties = tie_mask(ora["ratio"]) | kink_mask(p)
    rng = np.random.default_rng(3)
    g = rng.normal(size=ora["image"].shape) / ora["image"].size
    g[ties] = 0.0
    got = gpu_adjoint(p, g, flags=flags)
    ref = oracle_adjoint(p, g)
    assert_dv_close(got["dV"], ref["dV"], "EA dV")
    assert_grad_close(got["dTF"], ref["dTF"], "EA dTF")
    assert_grad_close(got["dcam"], ref["dcam"], "EA dcam")
    assert_grad_close([got["dstep"]], [ref["dstep"]], "EA dstep")


@pytest.mark.parametrize("flags", [0, PLAIN, 1, 2, 3])
def test_ea_density_gradient_element_wise_under_an_l2_loss(flags):
    """The density gradient of an L2 image loss (against the render of another
    grid) voxel by voxel: |g - o| <= 1e-3 max(|o|, 1e-2 max|o|) on every
    route (64-bit fixed-point brick, float atomics, checkpoint)."""
    p = ea_problem()
    _say(f"EA element-wise dV, L2 loss, flags={flags}")
    ora = oracle_forward(p)
    ties = tie_mask(ora["ratio"]) | kink_mask(p)
    q = ea_problem(seed=8)
    pt = Problem(1, q.volume, "f32", p.tf, p.yaw, p.pitch, p.dist, p.fovy, p.W, p.H, p.step)
    g = 2.0 * (ora["image"] - oracle_forward(pt)["image"]) / ora["image"].size
    g[ties] = 0.0
    got = gpu_adjoint(p, g, flags=flags, want=("V",))
    ref = oracle_adjoint(p, g)
    e = assert_dv_close(got["dV"], ref["dV"], "EA dV")
    r = assert_dv_elementwise(got["dV"], ref["dV"], "EA dV")
    print(f"[result] EA L2 flags={flags}: dV norm {e:.3g}, element-wise worst {r:.3g} of the "
          f"bound", flush=True)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_low_precision_storage_against_dequantized_oracle(storage):
    p = ea_problem(storage=storage, W=64, H=64)
    _say(f"EA {storage} storage")
    img, _ = gpu_forward(p)
    ora = oracle_forward(p)
    assert_images_close(img, ora, f"{storage} image")
    ties = tie_mask(ora["ratio"])
    rng = np.random.default_rng(4)
    g = rng.normal(size=ora["image"].shape) / ora["image"].size
    g[ties] = 0.0
    got = gpu_adjoint(p, g)
    ref = oracle_adjoint(p, g)
    assert_dv_close(got["dV"], ref["dV"], f"{storage} dV")
    assert_grad_close(got["dTF"], ref["dTF"], f"{storage} dTF")
    # against the float32 master: within the a-priori bound of the storage
    # rounding (per pixel) plus the float32 image tolerance
    p32 = Problem(p.model, p.volume, "f32", p.tf, p.yaw, p.pitch, p.dist, p.fovy, p.W, p.H, p.step)
    om = oracle_forward(p32)["image"]
    pix = np.arange(p.W * p.H, dtype=np.int32)
    qb = quantisation_image_bound(p.volume, p.tf, oracle_camera(p), p.W, p.H, p.step, storage,
                                  pix, oracle.EA)
    keep = ~ties
    qerr = np.abs(img - om)
    assert np.all(qerr[keep] <= qb[keep] + 1e-4), float((qerr - qb)[keep].max())
    print(f"[result] {storage} storage: image effect {float(qerr[keep].max()):.3g}, at most "
          f"{float((qerr[keep] / (qb[keep] + 1e-4)).max()):.3g} of the bound", flush=True)


def test_c2_full_config():
    w = synth.make_c2()
    v = w.views[0]
    p = Problem(1, w.volume, "f32", w.tf, v.yaw, v.pitch, v.dist, v.fovy, v.width, v.height,
                w.step_world)
    _say("C2 full")
    img, tr = gpu_forward(p)
    ora = oracle_forward(p)
    assert_images_close(img, ora, "C2 image")
    hit = ora["nsamp"] > 0
    med = float(np.median(ora["trans"][hit]))
    assert 0.05 < med < 0.7, med
    ties = tie_mask(ora["ratio"]) | kink_mask(p)
    tv = w.meta["target_view"]
    pt = Problem(1, w.volume, "f32", w.meta["target_tf"], tv.yaw, tv.pitch, tv.dist, tv.fovy,
                 tv.width, tv.height, w.meta["target_step_vox"] * 2.0 / 127)
    tgt = oracle_forward(pt)["image"]
    g = 2.0 * (ora["image"] - tgt) / ora["image"].size
    g[ties] = 0.0
    got = gpu_adjoint(p, g)
    ref = oracle_adjoint(p, g)
    assert_dv_close(got["dV"], ref["dV"], "C2 dV")
    r = assert_dv_elementwise(got["dV"], ref["dV"], "C2 dV")
    print(f"[result] C2 dV element-wise worst {r:.3g} of the bound", flush=True)
    assert_grad_close(got["dTF"], ref["dTF"], "C2 dTF")
    assert_grad_close(got["dcam"], ref["dcam"], "C2 dcam")
    assert_grad_close([got["dstep"]], [ref["dstep"]], "C2 dstep")


def test_nearly_opaque_rays_take_the_checkpoint_fallback():
    # tau up to 2000 per world unit: most rays reach T_N < 2^-100 where the
    # float32 inversion fails (Sec. 4.4 "alpha < 1"); AUTO routes them to the
    # segment-checkpoint kernel and the gradients still match the stored tape.
    p = ea_problem(W=48, H=40, tau_max=2000.0, seed=11)
    _say("EA opaque fallback")
    ora = oracle_forward(p)
    ties = tie_mask(ora["ratio"]) | kink_mask(p)
    hit = ora["nsamp"] > 0
    assert (ora["trans"][hit] < 2.0 ** -100).mean() > 0.2
    rng = np.random.default_rng(5)
    g = rng.normal(size=ora["image"].shape) / ora["image"].size
    g[ties] = 0.0
    got = gpu_adjoint(p, g, flags=0, count_fallback=True)
    assert got["n_fallback"] > 0
    ref = oracle_adjoint(p, g)
    assert_dv_close(got["dV"], ref["dV"], "opaque dV")
    assert_grad_close(got["dTF"], ref["dTF"], "opaque dTF")
    assert_grad_close(got["dcam"], ref["dcam"], "opaque dcam", floor_frac=5e-2)


@pytest.mark.parametrize("W,H,n", [(16, 12, (96, 96, 96)), (64, 48, (40, 48, 44))])
def test_checkpoint_for_every_ray_in_lds_bricks_and_global_windows(W, H, n):
    # CHECKPOINT sends every hit ray through the segment-checkpoint kernel.  At
    # 16x12 pixels over a 96^3 grid an 8x8 block of rays spans about 70
    # voxels, so no window of samples fits the wave's LDS brick and the density
    # gradient takes the per-cell global atomics; at 64x48 over a 48-voxel
    # grid the windows fit and it goes through the LDS bricks.  Either way the
    # gradients match the oracle's stored tape (Sec. 4.4, alpha < 1: the
    # transmittance is recomputed forward, never inverted).
    from paper_2107_12672_amd import ddvr as d
    p = ea_problem(n=n, W=W, H=H, seed=13)
    _say(f"checkpoint every ray {W}x{H} over {n}")
    ora = oracle_forward(p)
    ties = tie_mask(ora["ratio"]) | kink_mask(p)
    hit = ora["nsamp"] > 0
    assert hit.sum() > 0.3 * hit.size
    rng = np.random.default_rng(6)
    g = rng.normal(size=ora["image"].shape) / ora["image"].size
    g[ties] = 0.0
    got = gpu_adjoint(p, g, flags=d.ADJ_CHECKPOINT, count_fallback=True)
    # every hit ray with a nonzero upstream gradient is queued (a ray grazing
    # the box within float32 error may count on one side only)
    seeded = hit & np.any(g.reshape(hit.shape + (-1,)) != 0.0, axis=-1)
    assert abs(got["n_fallback"] - seeded.sum()) <= 2, (got["n_fallback"], seeded.sum())
    ref = oracle_adjoint(p, g)
    assert_dv_close(got["dV"], ref["dV"], "checkpoint dV")
    assert_grad_close(got["dTF"], ref["dTF"], "checkpoint dTF")
    assert_grad_close(got["dcam"], ref["dcam"], "checkpoint dcam", floor_frac=5e-2)
    assert_grad_close([got["dstep"]], [ref["dstep"]], "checkpoint dstep")


def test_checkpoint_batch_of_two_grids_and_three_tfs():
    # CHECKPOINT on an uneven batch (two grids, f16 and f32, three views with
    # their own TFs and ragged image sizes): the checkpoint kernel's waves take
    # queued rays of different views, so where a wave's rays write different
    # gradient grids the density gradient goes out by per-cell global atomics,
    # and with three TF gradients there is no shared LDS table.  Every
    # gradient matches the sum of the oracle's per-view stored-tape adjoints.
    import torch
    from paper_2107_12672_amd import ddvr as d
    from harness import device_volume, gpu_camera
    probs = [ea_problem(W=40, H=24, seed=71, storage="f16"),
             ea_problem(W=72, H=56, seed=72, yaw=200.0),
             ea_problem(W=33, H=47, seed=71, yaw=-40.0, pitch=30.0, storage="f16")]
    probs[2].volume = probs[0].volume
    vidx = [0, 1, 0]
    _say("checkpoint batch, two grids, three TFs")
    rng = np.random.default_rng(17)
    seeds, refs = [], []
    for p in probs:
        ora = oracle_forward(p)
        g = rng.normal(size=ora["image"].shape) / ora["image"].size
        g[tie_mask(ora["ratio"]) | kink_mask(p)] = 0.0
        seeds.append(g)
        refs.append(oracle_adjoint(p, g))
    vols = [device_volume(probs[0]), device_volume(probs[1])]
    tfs = [torch.from_numpy(p.tf).cuda() for p in probs]
    n = len(probs)
    imgs = [torch.zeros(p.H * p.W * 4, device="cuda") for p in probs]
    trs = [torch.zeros(p.H * p.W, device="cuda") for p in probs]
    gs = [torch.from_numpy(np.ascontiguousarray(g, dtype=np.float32).ravel()).cuda() for g in seeds]
    dcam = torch.zeros((n, 12), device="cuda")
    dstep = torch.zeros(n, device="cuda")
    dvs = [torch.zeros(v.shape, device="cuda") for v in vols]
    dtfs = [torch.zeros_like(t) for t in tfs]
    views = [d.make_view(vidx[k], gpu_camera(p), p.step, imgs[k], transmittance=trs[k],
                         d_image=gs[k], d_camera=dcam[k], d_step=dstep[k:k + 1], tf_index=k)
             for k, p in enumerate(probs)]
    b = d.Batch(vols, tfs, views, d.EMISSION_ABSORPTION, flags=d.ADJ_CHECKPOINT, d_volumes=dvs,
                d_tfs=dtfs)
    ws = torch.zeros(b.workspace_size() // 4 + 1, dtype=torch.int32, device="cuda")
    b.run(d.PASS_FORWARD)
    b.run(d.PASS_ADJOINT, workspace=ws)
    torch.cuda.synchronize()
    b.close()
    assert_dv_close(dvs[0].cpu().numpy(), refs[0]["dV"] + refs[2]["dV"], "batch grid 0 dV")
    assert_dv_close(dvs[1].cpu().numpy(), refs[1]["dV"], "batch grid 1 dV")
    for k in range(n):
        assert_grad_close(dtfs[k].cpu().numpy(), refs[k]["dTF"], f"batch view {k} dTF")
        assert_grad_close(dcam[k].cpu().numpy(), refs[k]["dcam"], f"batch view {k} dcam",
                          floor_frac=5e-2)
        assert_grad_close([dstep[k].item()], [refs[k]["dstep"]], f"batch view {k} dstep")


def test_rays_that_miss_give_exact_zeros():
    p = ea_problem(W=32, H=24)
    p.yaw, p.pitch, p.fovy = 10.0, 10.0, 120.0
    _say("miss rays")
    img, tr = gpu_forward(p)
    ora = oracle_forward(p)
    miss = ora["nsamp"] == 0
    assert miss.sum() > 10 and (~miss).sum() > 10
    # a ray grazing the box within float32 error may still take one sample
    exact = np.all(img[miss] == 0.0, axis=1) & (tr[miss] == 1.0)
    assert exact.mean() >= 0.99, exact.mean()
    # camera looking away from the grid: everything misses, no gradient
    import torch
    from paper_2107_12672_amd import ddvr as d
    from harness import device_volume
    cam = d.Camera()
    for a, (e, f, r, u) in enumerate(zip((3.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 0.0, -0.5),
                                         (0.0, 0.5, 0.0))):
        cam.eye[a], cam.fwd[a], cam.right[a], cam.up[a] = e, f, r, u
    cam.width, cam.height = 24, 20
    vol = device_volume(p)
    tf = torch.from_numpy(p.tf).cuda()
    img = torch.full((20 * 24 * 4,), 7.0, device="cuda")
    tr = torch.full((20 * 24,), 7.0, device="cuda")
    d.render_forward(vol, tf, cam, p.step, 1, img, tr)
    dV = torch.zeros(p.volume.shape, device="cuda")
    dTF = torch.zeros_like(tf)
    dcam = torch.zeros(12, device="cuda")
    dstep = torch.zeros(1, device="cuda")
    n = d.adjoint_workspace_size(vol, cam, p.step, 1, 0)
    ws = torch.zeros(n // 4 + 1, dtype=torch.int32, device="cuda")
    gimg = torch.randn(20 * 24 * 4, device="cuda")
    d.render_adjoint(vol, tf, cam, p.step, 1, img, tr, gimg, d.grads_desc(dV, dTF, dcam, dstep),
                     workspace=ws)
    torch.cuda.synchronize()
    assert torch.all(img == 0) and torch.all(tr == 1)
    assert torch.all(dV == 0) and torch.all(dTF == 0) and torch.all(dcam == 0) and dstep.item() == 0


def test_tiny_grid_and_two_knot_tf():
    rng = np.random.default_rng(9)
    vol = rng.uniform(0, 1, (2, 2, 2)).astype(np.float32)
    tf = synth.random_tf(2, rng, 5.0)
    p = Problem(1, vol, "f32", tf, 20.0, 30.0, 2.5, 60.0, 17, 19, 0.05)
    _say("2^3 grid, R=2")
    img, _ = gpu_forward(p)
    ora = oracle_forward(p)
    assert_images_close(img, ora, "tiny image")
    g = rng.normal(size=ora["image"].shape) / ora["image"].size
    g[tie_mask(ora["ratio"])] = 0
    got = gpu_adjoint(p, g)
    ref = oracle_adjoint(p, g)
    assert_dv_close(got["dV"], ref["dV"], "tiny dV")
    assert_grad_close(got["dTF"], ref["dTF"], "tiny dTF")


@pytest.mark.parametrize("lane_map", [0, 1, 2, 3])
def test_fused_l2_equals_forward_then_adjoint(lane_map):
    """The fused pass (forward, in-kernel L2 seed, adjoint) gives the forward's
    images bitwise and the separate adjoint's gradients, for every pair of
    lane maps (2 and 3 hand each ray over to another lane between the passes;
    the ragged image leaves lanes without a pixel)."""
    from paper_2107_12672_amd import ddvr as d
    old = d.get_tuning()
    try:
        d.set_tuning(lane_map=lane_map)
        _fused_vs_separate(d)
    finally:
        d.set_tuning(**old)


def _fused_vs_separate(d):
    import torch
    from harness import device_volume, gpu_camera
    for p in (ea_problem(W=56, H=44), c1_problem()[0]):
        _say(f"fused model={p.model} lane_map={d.get_tuning()['lane_map']}")
        vol = device_volume(p)
        tf = torch.from_numpy(p.tf).cuda() if p.tf is not None else None
        cam = gpu_camera(p)
        rng = np.random.default_rng(6)
        tgt = torch.from_numpy(rng.uniform(0, 1, (p.H * p.W * p.C,)).astype(np.float32)).cuda()
        scale = 1.0 / (p.H * p.W * p.C)
        img = torch.zeros(p.H * p.W * p.C, device="cuda")
        tr = torch.zeros(p.H * p.W, device="cuda")
        dV = torch.zeros(p.volume.shape, device="cuda")
        dTF = torch.zeros_like(tf) if tf is not None else None
        dcam = torch.zeros(12, device="cuda")
        dstep = torch.zeros(1, device="cuda")
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        n = d.adjoint_workspace_size(vol, cam, p.step, p.model, 0)
        ws = torch.zeros(max(n, 4) // 4, dtype=torch.int32, device="cuda")
        d.render_fused_l2(vol, tf, cam, p.step, p.model, tgt, scale, img, tr,
                          d.grads_desc(dV, dTF, dcam, dstep), workspace=ws, loss_out=loss)
        img2 = torch.zeros_like(img)
        tr2 = torch.zeros_like(tr)
        d.render_forward(vol, tf, cam, p.step, p.model, img2, tr2)
        torch.cuda.synchronize()
        assert torch.equal(img, img2) and torch.equal(tr, tr2)
        ref_loss = float(((img2.double() - tgt.double()) ** 2).sum() * scale)
        assert abs(loss.item() - ref_loss) <= 1e-5 * ref_loss + 1e-12
        g = 2.0 * scale * (img2 - tgt)
        dV2 = torch.zeros_like(dV)
        dTF2 = torch.zeros_like(dTF) if dTF is not None else None
        dcam2 = torch.zeros_like(dcam)
        dstep2 = torch.zeros_like(dstep)
        d.render_adjoint(vol, tf, cam, p.step, p.model, img2, tr2, g,
                         d.grads_desc(dV2, dTF2, dcam2, dstep2), workspace=ws)
        torch.cuda.synchronize()
        assert_dv_close(dV.cpu().double().numpy(), dV2.cpu().double().numpy(), "fused dV", 1e-5)
        if dTF is not None:
            assert_grad_close(dTF.cpu().numpy(), dTF2.cpu().numpy(), "fused dTF", 1e-5)
        assert_grad_close(dcam.cpu().numpy(), dcam2.cpu().numpy(), "fused dcam", 1e-4)


@pytest.mark.parametrize("tuning", [
    {"waves": 1, "lds_cap": 1024, "slab_k": 8, "cell_acc": 0, "lane_map": 0},
    {"waves": 2, "lds_cap": 2048, "slab_k": 64, "cell_acc": 1, "lane_map": 1},
    {"waves": 4, "lds_cap": 512, "slab_k": 16, "cell_acc": 1, "lane_map": 0},
    {"waves": 4, "lds_cap": 8192, "slab_k": 128, "cell_acc": 0, "lane_map": 1},
    {"waves": 4, "lds_cap": 7168, "slab_k": 64, "cell_acc": 1, "lane_map": 2},
    {"waves": 2, "lds_cap": 3072, "slab_k": 32, "cell_acc": 1, "lane_map": 3},
    {"waves": 4, "lds_cap": 7168, "slab_k": 64, "cell_acc": 1, "lane_map": 2, "slab_axis": 0},
    {"waves": 1, "lds_cap": 1024, "slab_k": 8, "cell_acc": 1, "lane_map": 0, "slab_axis": 0},
])
def test_results_do_not_depend_on_the_launch_shape(tuning):
    """Forward bitwise identical across tile shapes, brick sizes, slab
    lengths and slab shapes (axis slabs or distance shells: the per-sample
    emission-absorption arithmetic does not depend on the tiling, which also
    catches LDS staging / barrier races); gradients equal up to summation
    order and matching the oracle."""
    from paper_2107_12672_amd import ddvr as d
    p = ea_problem(W=56, H=40)
    _say(f"tuning {tuning}")
    base_img, base_tr = gpu_forward(p)
    old = d.get_tuning()
    try:
        d.set_tuning(**tuning)
        img, tr = gpu_forward(p)
        assert np.array_equal(img, base_img) and np.array_equal(tr, base_tr)
        ora = oracle_forward(p)
        ties = tie_mask(ora["ratio"]) | kink_mask(p)
        rng = np.random.default_rng(8)
        g = rng.normal(size=ora["image"].shape) / ora["image"].size
        g[ties] = 0.0
        got = gpu_adjoint(p, g)
        ref = oracle_adjoint(p, g)
        assert_dv_close(got["dV"], ref["dV"], "dV")
        assert_grad_close(got["dTF"], ref["dTF"], "dTF")
        assert_grad_close(got["dcam"], ref["dcam"], "dcam")
        c, w = c1_problem()
        co = oracle_forward(c)
        cg = rng.normal(size=co["image"].shape) / co["image"].size
        cg[tie_mask(co["ratio"]) | kink_mask(c)] = 0.0
        assert_dv_close(gpu_adjoint(c, cg)["dV"], oracle_adjoint(c, cg)["dV"], "AO dV")
    finally:
        d.set_tuning(**old)


def test_batch_schedules_agree_and_match_single_views():
    """An uneven batch (two grids, three image sizes) run one-workgroup-per-tile
    and as a persistent longest-first queue (also replayed from a graph) gives
    bitwise the same images as single-view launches, and the same gradients
    up to summation order."""
    import torch
    from paper_2107_12672_amd import ddvr as d
    from harness import device_volume, gpu_camera
    probs = [ea_problem(W=40, H=24, seed=61), ea_problem(W=72, H=56, seed=62, yaw=200.0),
             ea_problem(W=33, H=47, seed=61, yaw=-40.0, pitch=30.0)]
    probs[2].volume = probs[0].volume           # views 0 and 2 share grid 0
    _say("batch schedules")
    vols = [device_volume(probs[0]), device_volume(probs[1])]
    vidx = [0, 1, 0]
    tfs = [torch.from_numpy(p.tf).cuda() for p in probs]
    rng = np.random.default_rng(63)
    gs = [torch.from_numpy(rng.normal(size=(p.H * p.W * 4,)).astype(np.float32)).cuda()
          for p in probs]
    # single-view references
    ref_img, ref_dv = [], [torch.zeros(v.shape, device="cuda") for v in vols]
    for k, p in enumerate(probs):
        img = torch.zeros(p.H * p.W * 4, device="cuda")
        tr = torch.zeros(p.H * p.W, device="cuda")
        cam = gpu_camera(p)
        d.render_forward(vols[vidx[k]], tfs[k], cam, p.step, 1, img, tr)
        ws = torch.zeros(d.adjoint_workspace_size(vols[vidx[k]], cam, p.step, 1) // 4 + 1,
                         dtype=torch.int32, device="cuda")
        d.render_adjoint(vols[vidx[k]], tfs[k], cam, p.step, 1, img, tr, gs[k],
                         d.grads_desc(ref_dv[vidx[k]]), workspace=ws)
        ref_img.append(img)
    torch.cuda.synchronize()
    old = d.get_tuning()
    try:
        for sched, graph in ((1, False), (2, False), (2, True)):
            d.set_tuning(schedule=sched)
            imgs = [torch.full((p.H * p.W * 4,), float("nan"), device="cuda") for p in probs]
            trs = [torch.zeros(p.H * p.W, device="cuda") for p in probs]
            dvs = [torch.zeros(v.shape, device="cuda") for v in vols]
            views = [d.make_view(vidx[k], gpu_camera(p), p.step, imgs[k], transmittance=trs[k],
                                 d_image=gs[k], tf_index=k) for k, p in enumerate(probs)]
            b = d.Batch(vols, tfs, views, d.EMISSION_ABSORPTION, d_volumes=dvs)
            ws = torch.zeros(b.workspace_size() // 4 + 1, dtype=torch.int32, device="cuda")
            for rep in range(2 if graph else 1):
                for dv in dvs:
                    dv.zero_()
                b.run(d.PASS_FORWARD, graph=graph)
                b.run(d.PASS_ADJOINT, workspace=ws)
                torch.cuda.synchronize()
                for k in range(3):
                    assert torch.equal(imgs[k], ref_img[k]), (sched, graph, k)
                for j in range(2):
                    e = float((dvs[j] - ref_dv[j]).norm() / ref_dv[j].norm())
                    assert e < 1e-5, (sched, graph, j, e)
            b.close()
    finally:
        d.set_tuning(**old)


@pytest.mark.parametrize("slab_axis", [1, 0])
@pytest.mark.parametrize("case", ["eye_inside_ea", "wide_fov_ao"])
def test_eye_inside_the_grid_and_a_wide_field_of_view(case, slab_axis):
    """Rays that start inside the grid (t0 = 0, no entry plane) and a 150-degree
    field of view, whose edge tiles hold strongly diverging rays (where a
    tile's rays may not all advance along its axis and the tile walks
    distance shells): images, density, TF, camera and step gradients against
    the oracle with axis slabs and with shells."""
    from paper_2107_12672_amd import ddvr as d
    rng = np.random.default_rng(91)
    if case == "eye_inside_ea":
        n = (36, 40, 34)
        vol = synth.blob_volume(n, 6, rng, sigma_world=(0.1, 0.3), amplitude=0.6, noise=0.02)
        tf = synth.random_tf(12, rng, 2.0)
        p = Problem(1, vol, "f32", tf, 40.0, 25.0, 0.45, 90.0, 64, 48, 0.5 * 2.0 / 39)
    else:
        n = (40, 40, 40)
        vol = synth.blob_volume(n, 5, rng, sigma_world=(0.1, 0.3), amplitude=0.5, noise=0.02)
        p = Problem(0, vol, "f32", None, -70.0, 35.0, 1.6, 150.0, 96, 64, 0.5 * 2.0 / 39)
    _say(f"{case}, slab_axis={slab_axis}")
    old = d.get_tuning()
    try:
        d.set_tuning(slab_axis=slab_axis)
        img, tr = gpu_forward(p)
        ora = oracle_forward(p)
        assert_images_close(img, ora, f"{case} image")
        ties = tie_mask(ora["ratio"]) | kink_mask(p)
        g = rng.normal(size=ora["image"].shape) / ora["image"].size
        g[ties] = 0.0
        got = gpu_adjoint(p, g)
        ref = oracle_adjoint(p, g)
        e = assert_dv_close(got["dV"], ref["dV"], f"{case} dV")
        if p.model == 1:
            assert_grad_close(got["dTF"], ref["dTF"], f"{case} dTF")
        assert_grad_close(got["dcam"], ref["dcam"], f"{case} dcam")
        assert_grad_close([got["dstep"]], [ref["dstep"]], f"{case} dstep")
        print(f"[result] {case} slab_axis={slab_axis}: dV norm {e:.3g}", flush=True)
    finally:
        d.set_tuning(**old)
