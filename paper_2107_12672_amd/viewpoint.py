"""Best-viewpoint selection (Sec. 5.1) through the library's entry points.

The camera sits on a sphere around the volume, looking at its centre, and is
parameterised by longitude (yaw) and latitude (pitch).  The objective is the
opacity entropy OE(C) = H(C[:, :, 3]) of the emission-absorption image, H the
normalised entropy, which the runs maximise.  Per iteration:
  1. render the view (``ddvr_render_forward``);
  2. OE and its image gradient (``ddvr_opacity_entropy``);
  3. d OE / d (yaw, pitch) by forward mode, forward-delayed: one tangent pass
     along the two pose directions contracted with the image gradient in the
     kernel (``ddvr_camera_sphere_tangents``, ``ddvr_render_tangent``).
The runs start from the paper's eight poses (longitudes 45, 135, 225, 315
degrees, latitudes +-45 degrees) and take 20 iterations each.

Reading (the paper gives neither the step rule nor its length): a step moves
the pose by `step` radians along the normalised gradient; a step that does
not raise OE is not taken and halves the step length, so every run's OE is
non-decreasing.  The latitude is kept `pole_margin` radians away from the
poles, where the camera's up vector is undefined.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

from . import ddvr as d

PAPER_STARTS = [(math.radians(lon), math.radians(lat))
                for lat in (45.0, -45.0) for lon in (45.0, 135.0, 225.0, 315.0)]


@dataclass
class ViewpointSchedule:
    iterations: int = 20
    step: float = 0.2            # radians, first step length
    dist: float = 2.5
    fovy: float = math.radians(60.0)
    width: int = 128
    height: int = 128
    pole_margin: float = 0.05


@dataclass
class Run:
    poses: List[Tuple[float, float]] = field(default_factory=list)   # accepted (yaw, pitch)
    oe: List[float] = field(default_factory=list)                    # OE after each iteration


class _Objective:
    def __init__(self, volume, tf, step_world, sched, stream):
        import torch
        dev = volume.device
        self.volume, self.tf, self.step_world, self.s, self.stream = (volume, tf, step_world,
                                                                      sched, stream)
        self.img = torch.empty((sched.height, sched.width, 4), device=dev)
        self.trans = torch.empty((sched.height, sched.width), device=dev)
        self.g = torch.zeros_like(self.img)
        self.work = torch.zeros(2, dtype=torch.float64, device=dev)
        self.val = torch.zeros(1, dtype=torch.float64, device=dev)
        self.d_dir = torch.zeros(2, device=dev)

    def camera(self, yaw, pitch):
        s = self.s
        return d.camera_from_sphere(yaw, pitch, s.dist, s.fovy, s.width, s.height)

    def value(self, yaw, pitch, with_grad=False) -> float:
        cam = self.camera(yaw, pitch)
        d.render_forward(self.volume, self.tf, cam, self.step_world, d.EMISSION_ABSORPTION,
                         self.img, self.trans, stream=self.stream)
        self.g.zero_()
        d.opacity_entropy(self.img, self.work, self.val, self.g if with_grad else None,
                          stream=self.stream)
        return float(self.val.item())

    def gradient(self, yaw, pitch) -> Tuple[float, float]:
        """d OE / d (yaw, pitch) at the pose of the last `value(..., True)`."""
        s = self.s
        J = d.camera_sphere_tangents(yaw, pitch, s.dist, s.fovy, s.width, s.height)
        self.d_dir.zero_()
        d.render_tangent(self.volume, self.tf, self.camera(yaw, pitch), self.step_world,
                         d.EMISSION_ABSORPTION, [J[0] + [0.0], J[1] + [0.0]], d_image=self.g,
                         d_dir=self.d_dir, stream=self.stream)
        gy, gp = self.d_dir.tolist()
        return gy, gp


def optimize_viewpoint(volume, tf, step_world: float, sched: ViewpointSchedule = None,
                       starts: Sequence[Tuple[float, float]] = PAPER_STARTS,
                       stream=None) -> List[Run]:
    """volume: stored grid (device); tf: [R][4] float32 (device).  Returns one
    Run per start; run.oe[0] is the OE at the start."""
    sched = sched or ViewpointSchedule()
    obj = _Objective(volume, tf, step_world, sched, stream)
    lat_max = 0.5 * math.pi - sched.pole_margin
    runs = []
    for yaw, pitch in starts:
        run = Run()
        cur = obj.value(yaw, pitch, with_grad=True)
        run.poses.append((yaw, pitch))
        run.oe.append(cur)
        length = sched.step
        for _ in range(sched.iterations):
            gy, gp = obj.gradient(yaw, pitch)
            norm = math.hypot(gy, gp)
            if not norm > 0.0:
                break
            ny = yaw + length * gy / norm
            npitch = min(max(pitch + length * gp / norm, -lat_max), lat_max)
            new = obj.value(ny, npitch, with_grad=True)
            if new > cur:
                yaw, pitch, cur = ny, npitch, new
            else:
                length *= 0.5
                obj.value(yaw, pitch, with_grad=True)   # the image gradient at the kept pose
            run.poses.append((yaw, pitch))
            run.oe.append(cur)
        runs.append(run)
    return runs
