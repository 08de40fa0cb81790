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


def gpu_camera(p: Problem):
    d = ddvr_mod()
    return d.camera_from_sphere(math.radians(p.yaw), math.radians(p.pitch), p.dist,
                                math.radians(p.fovy), p.W, p.H)


def oracle_camera(p: Problem):
    return oracle.camera_from_sphere(p.yaw, p.pitch, p.dist, p.fovy, p.W, p.H)


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


def oracle_spread(p: Problem, pix, g, rel=1e-7, trials=3, seed=1):
    """Relative spread of the oracle's camera (norm-wise) and step gradients
    when the camera frame and the step are perturbed by `rel` relative (float32
    rounding of the inputs).  Returns (cam_spread, step_spread)."""
    V = dequantized(p)
    cam = oracle_camera(p)
    rng = np.random.default_rng(seed)
    base = oracle.adjoint(V, p.tf, cam, p.W, p.H, p.step, p.model, g, pix=pix, want_dV=False)
    cs = ss = 0.0
    for _ in range(trials):
        a = oracle.adjoint(V, p.tf, cam * (1.0 + rel * rng.normal(size=12)), p.W, p.H,
                           p.step * (1.0 + rel * rng.normal()), p.model, g, pix=pix,
                           want_dV=False)
        cs = max(cs, rel_norm_err(a["dcam"], base["dcam"]))
        ss = max(ss, abs(a["dstep"] - base["dstep"]) / max(abs(base["dstep"]), 1e-300))
    return cs, ss


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
    bound = rtol * np.maximum(np.abs(o), floor)
    bad = np.abs(g - o) > bound
    assert not bad.any(), f"{what}: {int(bad.sum())} entries off; worst {float(np.abs(g - o).max()):.3g} " \
                          f"at scale {scale:.3g}"


def assert_dv_close(g, o, what, rtol=GRAD_RTOL):
    e = rel_norm_err(g, o)
    assert e <= rtol, f"{what}: norm-wise relative dV error {e:.3g} > {rtol}"
    return e
