"""Shared helpers of the GPU parity tests: run a problem on the HIP path and on
the FP64 oracle from the same seeded inputs, and compare.

Tolerances (stated once, used by every parity test):
  * images: absolute 1e-4 per element (float32 path vs float64 oracle);
  * density gradient: norm-wise relative 1e-3, ||g - o|| <= 1e-3 ||o||;
  * TF / camera / step gradients: element-wise |g - o| <= 1e-3 * max(|o|, floor)
    with floor = 1e-2 * max|o| of that array (gradients are sums of many
    float32 terms; entries far below the array's scale are compared at the
    scale's precision).
Rays whose chord length is within 1e-3 samples of an integer number of steps
(L/dt near an integer) may take a different sample count in float32 than in
float64; they are excluded from image comparisons and carry zero upstream
gradient in adjoint comparisons, and their count is reported.
Rays with a sample within float32 position error of a point where Alg. 1 is
not differentiable (interior cell face: the trilinear gradient jumps; TF knot
or clamp end: the TF slope jumps) have two valid one-sided gradients; float32
and float64 may pick different sides, so such rays also carry zero upstream
gradient where camera / step gradients are compared (kink_mask).
At full size, emission-absorption camera gradients of long rays through steep
TFs are ill-conditioned away from kinks too: a 1e-7 relative perturbation of
the camera frame (float32 rounding of the input alone) moves some rays' float64
camera gradient by more than 1e-3 of its size.  Such rays are screened by
re-running the oracle at perturbed frames (sensitive_mask) and carry zero
upstream gradient where camera / step gradients are compared.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np

import oracle

IMG_ATOL = 1e-4
GRAD_RTOL = 1e-3
TIE_TOL = 1e-3

# Storage rounding (round to nearest even): |V_q - V| <= U_Q |V| + ETA_Q, with
# U_Q the unit roundoff of the format and ETA_Q half the spacing of its
# subnormals (the relative bound fails below the normal range).
U_Q = {"f32": 2.0 ** -24, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}
ETA_Q = {"f32": 2.0 ** -150, "f16": 2.0 ** -25, "bf16": 2.0 ** -134}


def torch_mod():
    import torch
    return torch


def ddvr_mod():
    from paper_2107_12672_amd import ddvr
    return ddvr


@dataclass
class Problem:
    model: int                 # 0 AO, 1 EA, 2 colour volume
    volume: np.ndarray         # float32 [nz][ny][nx] (colour: [nz][ny][nx][4]), master
    storage: str               # f32 / f16 / bf16
    tf: Optional[np.ndarray]   # float32 [R][4]
    yaw: float
    pitch: float
    dist: float
    fovy: float
    W: int
    H: int
    step: float                # world units

    def __post_init__(self):
        # both sides take the step the kernels see: float32
        self.step = float(np.float32(self.step))

    @property
    def C(self):
        return 1 if self.model == 0 else 4


def storage_dtype(storage):
    torch = torch_mod()
    return {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[storage]


def device_volume(p: Problem):
    torch = torch_mod()
    v = torch.from_numpy(np.ascontiguousarray(p.volume)).to("cuda")
    return v.to(storage_dtype(p.storage)).contiguous()


def dequantized(p: Problem) -> np.ndarray:
    """The grid values the GPU actually reads (round-to-nearest-even cast)."""
    torch = torch_mod()
    v = torch.from_numpy(np.ascontiguousarray(p.volume)).to(storage_dtype(p.storage))
    return v.to(torch.float64).numpy()


def frame32(yaw, pitch, dist, fovy, W, H) -> np.ndarray:
    """The camera frame both sides take: the oracle's frame of the pose,
    rounded to float32 (the kernels' precision), so that the GPU and the
    oracle render exactly the same input."""
    return oracle.camera_from_sphere(yaw, pitch, dist, fovy, W, H).astype(np.float32)


def camera_of_frame(f32, W, H):
    """ddvr.Camera holding a float32 frame [eye, fwd, right, up]."""
    d = ddvr_mod()
    cam = d.Camera()
    for a in range(3):
        cam.eye[a], cam.fwd[a] = float(f32[a]), float(f32[3 + a])
        cam.right[a], cam.up[a] = float(f32[6 + a]), float(f32[9 + a])
    cam.width, cam.height = W, H
    return cam


def gpu_camera(p: Problem):
    return camera_of_frame(frame32(p.yaw, p.pitch, p.dist, p.fovy, p.W, p.H), p.W, p.H)


def oracle_camera(p: Problem):
    return frame32(p.yaw, p.pitch, p.dist, p.fovy, p.W, p.H).astype(np.float64)


def gpu_forward(p: Problem, flags=0, vol=None):
    torch = torch_mod()
    d = ddvr_mod()
    vol = device_volume(p) if vol is None else vol
    tf = torch.from_numpy(p.tf).cuda() if p.tf is not None else None
    img = torch.full((p.H * p.W * p.C,), float("nan"), device="cuda")
    tr = torch.full((p.H * p.W,), float("nan"), device="cuda")
    d.render_forward(vol, tf, gpu_camera(p), p.step, p.model, img, tr, flags=flags)
    torch.cuda.synchronize()
    return img.view(p.H * p.W, p.C).cpu().numpy(), tr.cpu().numpy()


def gpu_adjoint(p: Problem, d_image: np.ndarray, flags=0, want=("V", "TF", "cam", "step"),
                count_fallback=False):
    torch = torch_mod()
    d = ddvr_mod()
    vol = device_volume(p)
    tf = torch.from_numpy(p.tf).cuda() if p.tf is not None else None
    img = torch.zeros(p.H * p.W * p.C, device="cuda")
    tr = torch.zeros(p.H * p.W, device="cuda")
    cam = gpu_camera(p)
    fwd_flags = flags & d.LAUNCH_PLAIN
    d.render_forward(vol, tf, cam, p.step, p.model, img, tr, flags=fwd_flags)
    g = torch.from_numpy(np.ascontiguousarray(d_image, dtype=np.float32)).cuda()
    dV = torch.zeros(p.volume.shape, device="cuda") if "V" in want else None
    dTF = torch.zeros_like(tf) if (tf is not None and "TF" in want) else None
    dcam = torch.zeros(12, device="cuda") if "cam" in want else None
    dstep = torch.zeros(1, device="cuda") if "step" in want else None
    grads = d.grads_desc(dV, dTF, dcam, dstep)
    ws_n = d.adjoint_workspace_size(vol, cam, p.step, p.model, flags)
    ws = torch.zeros(max(ws_n // 4, 1), dtype=torch.int32, device="cuda") if ws_n else None
    nfb = d.render_adjoint(vol, tf, cam, p.step, p.model, img, tr, g, grads, flags=flags,
                           workspace=ws, count_fallback=count_fallback)
    torch.cuda.synchronize()
    out = {
        "dV": dV.cpu().double().numpy() if dV is not None else None,
        "dTF": dTF.cpu().double().numpy() if dTF is not None else None,
        "dcam": dcam.cpu().double().numpy() if dcam is not None else None,
        "dstep": float(dstep.item()) if dstep is not None else None,
        "n_fallback": nfb,
    }
    return out


def oracle_forward(p: Problem, pix=None):
    V = dequantized(p)
    return oracle.render(V, p.tf, oracle_camera(p), p.W, p.H, p.step, p.model, pix=pix)


def oracle_adjoint(p: Problem, d_image, pix=None, variant=oracle.TAPE):
    V = dequantized(p)
    return oracle.adjoint(V, p.tf, oracle_camera(p), p.W, p.H, p.step, p.model, d_image,
                          variant=variant, pix=pix)


def kink_mask(p: Problem, pix=None) -> np.ndarray:
    """True for rays with a sample so close to a non-differentiable point
    (interior cell face, TF knot or clamp end) that float32 and float64 may
    evaluate different one-sided derivatives there.  Position error of the
    float32 march is ~ulp(q) ~ 1e-7 * max(n) voxels; density error ~1e-7."""
    V = dequantized(p)
    face, knot, entry = oracle.kinks(V, p.tf, oracle_camera(p), p.W, p.H, p.step, p.model,
                                     pix=pix, with_entry=True)
    nmax = max(p.volume.shape[:3])
    # the entry point x_o = e + t0*omega inherits direction errors amplified by
    # t0/|omega_a| (entry plane a): grazing entries move all samples further
    face_tol = 1e-6 * nmax + 1e-4 + 4e-7 * 0.5 * (nmax - 1) * entry
    knot_tol = 1e-5 * (p.tf.shape[0] if p.tf is not None else 1)
    return (face < face_tol) | (knot < knot_tol)


def sensitive_mask(p: Problem, pix, g, rel=1e-7, thresh=1e-3, trials=3, seed=0):
    """True for rays whose oracle camera / step gradient moves by more than
    `thresh` (relative to its own size) when the camera frame is perturbed by
    `rel` relative, the size of float32 rounding.  Such rays are
    ill-conditioned: no float32 evaluation can match the float64 gradient
    better than that spread."""
    V = dequantized(p)
    cam = oracle_camera(p)
    rng = np.random.default_rng(seed)
    out = np.zeros(len(pix), dtype=bool)
    for q in range(len(pix)):
        gq = g[q:q + 1]
        if not np.any(gq):
            continue
        base = oracle.adjoint(V, p.tf, cam, p.W, p.H, p.step, p.model, gq, pix=pix[q:q + 1],
                              want_dV=False)
        b = np.r_[base["dcam"], base["dstep"]]
        worst = 0.0
        for _ in range(trials):
            pc = cam * (1.0 + rel * rng.normal(size=12))
            a = oracle.adjoint(V, p.tf, pc, p.W, p.H, p.step, p.model, gq, pix=pix[q:q + 1],
                               want_dV=False)
            worst = max(worst, float(np.abs(np.r_[a["dcam"], a["dstep"]] - b).max()))
        out[q] = worst > thresh * max(float(np.abs(b).max()), 1e-30)
    return out


def camera_bounds(per_ray):
    """Element-wise bounds of a sum over rays of camera-frame (12) and step (1)
    gradients, per_ray [n][13]: 1e-3 max(|o_k|, 1e-2 max_j |o_j|) for the frame
    entries (the floor: a hundredth of the gradient's scale), and for the step
    1e-3 max(|o_step|, 1e-2 sum_r |b_r,step|) -- a scalar's scale is the size of
    the terms it sums, which cancel in the sum."""
    o = per_ray.sum(axis=0)
    bound = np.empty(13)
    bound[:12] = 1e-3 * np.maximum(np.abs(o[:12]), 1e-2 * np.abs(o[:12]).max())
    bound[12] = 1e-3 * max(abs(o[12]), 1e-2 * float(np.abs(per_ray[:, 12]).sum()))
    return bound


def screen_camera_rays(p: Problem, pix, g, rel=1e-7, trials=3, seed=0):
    """Rays to leave out of an element-wise camera / step comparison.

    Each ray's float64 camera-frame and step gradients are recomputed at
    frames and steps perturbed by `rel` relative (the size of float32 rounding
    of the inputs); a ray is screened when its own movement on the entries
    would push the kept rays' summed movements past 0.3 of an entry's bound
    for the sum over the kept rays (camera_bounds): the most sensitive ray is
    dropped until they fit (at least a fifth of the seeded rays are kept).
    Returns (mask of screened rays, per-ray gradients [n][13])."""
    V = dequantized(p)
    cam = oracle_camera(p)
    rng = np.random.default_rng(seed)
    n = len(pix)
    base = np.zeros((n, 13))
    sens = np.zeros((n, 13))
    seeded = np.array([bool(np.any(g[q])) for q in range(n)])
    pert = [(cam * (1.0 + rel * rng.normal(size=12)), p.step * (1.0 + rel * rng.normal()))
            for _ in range(trials)]
    for q in np.nonzero(seeded)[0]:
        gq = g[q:q + 1]
        a = oracle.adjoint(V, p.tf, cam, p.W, p.H, p.step, p.model, gq, pix=pix[q:q + 1],
                           want_dV=False)
        base[q] = np.r_[a["dcam"], a["dstep"]]
        for pc, ps in pert:
            b = oracle.adjoint(V, p.tf, pc, p.W, p.H, ps, p.model, gq, pix=pix[q:q + 1],
                               want_dV=False)
            sens[q] = np.maximum(sens[q], np.abs(np.r_[b["dcam"], b["dstep"]] - base[q]))
    # drop the most sensitive ray until the kept rays' sensitivities, added up,
    # stay inside 0.3 of every entry's bound (keeping at least a fifth)
    screened = ~seeded
    while True:
        kept = ~screened
        bound = np.maximum(camera_bounds(base[kept]), 1e-300)
        share = sens / bound[None, :]
        if share[kept].sum(axis=0).max() <= 0.3 or kept.sum() <= max(1, seeded.sum() // 5):
            break
        worst = np.where(kept, share.max(axis=1), -1.0)
        screened[int(np.argmax(worst))] = True
    screened &= seeded
    return screened, base


def oracle_spread(p: Problem, pix, g, rel=1e-7, trials=3, seed=1, per_ray=None):
    """Relative spread of the oracle's camera (norm-wise) and step gradients
    when the camera frame and the step are perturbed by `rel` relative (float32
    rounding of the inputs).  Returns (cam_spread, step_spread, elem): elem is
    the largest movement of any of the 13 entries (frame, step) as a fraction
    of its element-wise bound (camera_bounds of the per-ray gradients
    `per_ray`, [n][13], if given)."""
    V = dequantized(p)
    cam = oracle_camera(p)
    rng = np.random.default_rng(seed)
    base = oracle.adjoint(V, p.tf, cam, p.W, p.H, p.step, p.model, g, pix=pix, want_dV=False)
    o = np.r_[base["dcam"], base["dstep"]]
    bound = camera_bounds(o[None, :]) if per_ray is None else camera_bounds(per_ray)
    cs = ss = el = 0.0
    for _ in range(trials):
        a = oracle.adjoint(V, p.tf, cam * (1.0 + rel * rng.normal(size=12)), p.W, p.H,
                           p.step * (1.0 + rel * rng.normal()), p.model, g, pix=pix,
                           want_dV=False)
        cs = max(cs, rel_norm_err(a["dcam"], base["dcam"]))
        ss = max(ss, abs(a["dstep"] - base["dstep"]) / max(abs(base["dstep"]), 1e-300))
        el = max(el, float((np.abs(np.r_[a["dcam"], a["dstep"]] - o) /
                            np.maximum(bound, 1e-300)).max()))
    return cs, ss, el


def tie_mask(ratio: np.ndarray) -> np.ndarray:
    """True for rays whose sample count is ambiguous between precisions."""
    return np.abs(ratio - np.round(ratio)) < TIE_TOL


def assert_images_close(gpu_img, ora, what=""):
    ties = tie_mask(ora["ratio"])
    keep = ~ties
    err = np.abs(gpu_img[keep] - ora["image"][keep])
    worst = float(err.max()) if err.size else 0.0
    assert worst <= IMG_ATOL, f"{what}: max |image error| {worst:.3g} > {IMG_ATOL} " \
                              f"({int(ties.sum())} tie rays excluded)"
    return worst, int(ties.sum())


def rel_norm_err(g, o):
    no = float(np.linalg.norm(o))
    return float(np.linalg.norm(g - o)) / max(no, 1e-300)


def assert_grad_close(g, o, what, rtol=GRAD_RTOL, floor_frac=1e-2):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    scale = float(np.abs(o).max())
    floor = floor_frac * scale
    rel = np.abs(g - o) / np.maximum(np.maximum(np.abs(o), floor), 1e-300)
    print(f"[grad] {what}: worst relative error {float(rel.max()):.3g} (rtol {rtol:g}, "
          f"floor {floor_frac:g} of the scale)", flush=True)
    bad = rel > rtol
    assert not bad.any(), f"{what}: {int(bad.sum())} entries off; worst {float(np.abs(g - o).max()):.3g} " \
                          f"at scale {scale:.3g}"
    return float(rel.max())


def assert_dv_close(g, o, what, rtol=GRAD_RTOL):
    e = rel_norm_err(g, o)
    assert e <= rtol, f"{what}: norm-wise relative dV error {e:.3g} > {rtol}"
    return e


def assert_dv_elementwise(g, o, what, rtol=GRAD_RTOL, floor_frac=1e-2):
    """Density gradient voxel by voxel: |g - o| <= rtol * max(|o|, floor_frac *
    max|o|).  Returns the worst ratio of error to bound."""
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    scale = float(np.abs(o).max())
    bound = rtol * np.maximum(np.abs(o), floor_frac * scale)
    ratio = np.abs(g - o) / np.maximum(bound, 1e-300)
    worst = float(ratio.max())
    bad = int((ratio > 1.0).sum())
    assert bad == 0, f"{what}: {bad} of {ratio.size} voxels off element-wise; worst " \
                     f"{worst:.3g} x the bound (scale {scale:.3g})"
    return worst


def quantisation_image_bound(V, tf, cam, W, H, step, storage, pix, model):
    """A-priori bound, per sampled pixel, on |image(V_q) - image(V)| for a
    non-negative float32 master grid V stored as V_q (RNE cast to `storage`).

    Every vertex moves by at most u|V| + eta, so every sample's density by at
    most u d_i + eta, and the ray's density integral D = dt sum d_i (the
    absorption-only optical depth, -log T_N of the AO render of V) by at most
    u D + eta L, L = N dt the ray's length.
      * absorption-only: |alpha_q - alpha| = |T_N - T_N'| <= T_N (e^E - 1),
        E = u D + eta L;
      * emission-absorption: the optical depth moves by at most E = L_tau (u D
        + eta L), L_tau = (R-1) max |tau_(j+1) - tau_j| the TF's slope bound, so
        |alpha_q - alpha| <= T_N (e^E - 1) with the EA transmittance T_N; the
        blend weights w_i = T_i alpha_i move by at most 2E in total (their
        derivatives: -dt w_i per earlier tau_j, dt T_i e_i for their own), the
        colours by at most L_rgb (u + eta) (density clamped to [0, 1]), so
        |C_q - C|_c <= 2 E max|rgb| + L_rgb (u + eta).
    Returns [npix][C] bounds (C = 1 AO, 4 EA: r, g, b, alpha)."""
    u, eta = U_Q[storage], ETA_Q[storage]
    assert np.all(np.asarray(V) >= 0.0), "the bound assumes a non-negative grid"
    ao = oracle.render(V, None, cam, W, H, step, oracle.AO, pix=pix)
    Tn = ao["trans"]
    with np.errstate(divide="ignore"):
        D = np.where(Tn > 0.0, -np.log(np.maximum(Tn, 1e-300)), np.inf)
    L = ao["nsamp"] * step
    if model == oracle.AO:
        E = u * D + eta * L
        return (Tn * np.expm1(E))[:, None]
    tf = np.asarray(tf, np.float64)
    R = tf.shape[0]
    L_tau = (R - 1) * float(np.abs(np.diff(tf[:, 3])).max())
    L_rgb = (R - 1) * float(np.abs(np.diff(tf[:, :3], axis=0)).max())
    m = float(np.abs(tf[:, :3]).max())
    ea = oracle.render(V, tf, cam, W, H, step, oracle.EA, pix=pix)
    E = L_tau * (u * D + eta * L)
    b_alpha = ea["trans"] * np.expm1(E)
    b_rgb = 2.0 * E * m + L_rgb * (u + eta)
    return np.stack([b_rgb, b_rgb, b_rgb, b_alpha], axis=1)
