"""Seeded synthetic inputs for differentiable direct volume rendering.

This module only *draws* inputs: density grids, transfer-function tables,
camera poses on a sphere (yaw / pitch / distance), loss targets.  It holds
none of the rendering arithmetic (no camera frames, no ray marching, no
blending), so both the FP64 oracle and the HIP path can consume its arrays
without sharing any part of the method.

The paper's datasets (tooth / head / thorax CT, skull, jetstream, C60
potential, smoke plume; Sec. 5) are not available.  The generators below
stand in for their shapes and value structure:

* smooth Gaussian blobs       -> potential-field data (C60),
* piecewise-constant ellipsoids -> CT tissue (skull / thorax, Sec. 5.3),
* thresholded multi-scale noise -> sparse smoke / plume structures.

Layout conventions shared by every consumer:
  volume  float32 [nz][ny][nx]  (x fastest), values are vertex densities
  tf      float32 [R][4]        (r, g, b, tau) at knots k/(R-1)
  angles  degrees (yaw, pitch), distance in world units (grid spans [-1,1]
          along its longest axis)
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

SEED_BASE = 210712672


def seed_for(config: int, k: int = 0) -> int:
    """Seed of draw ``k`` of configuration ``config`` (1..5)."""
    return SEED_BASE + 100 * int(config) + int(k)


def rng_for(config: int, k: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.PCG64(seed_for(config, k)))


# --------------------------------------------------------------------------
# density grids
# --------------------------------------------------------------------------
def _axis_coords(shape_zyx: Tuple[int, int, int]):
    nz, ny, nx = shape_zyx
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    return z, y, x


def blob_volume(shape_zyx, n_blobs: int, rng: np.random.Generator, *,
                sigma_vox: Tuple[float, float] = None,
                sigma_world: Tuple[float, float] = None,
                amplitude: float = 0.5,
                centre_frac: Tuple[float, float] = (0.25, 0.75),
                noise: float = 0.0) -> np.ndarray:
    """Sum of isotropic Gaussian blobs (+ optional i.i.d. U[0, noise]).

    Widths are drawn either in voxels (``sigma_vox``) or in world units
    (``sigma_world``; the longest axis spans 2 world units).
    """
    nz, ny, nx = shape_zyx
    nmax = max(shape_zyx)
    vox_per_world = (nmax - 1) / 2.0
    z, y, x = _axis_coords(shape_zyx)
    vol = np.zeros(shape_zyx, dtype=np.float64)
    for _ in range(n_blobs):
        if sigma_vox is not None:
            s = rng.uniform(*sigma_vox)
        else:
            s = rng.uniform(*sigma_world) * vox_per_world
        c = [rng.uniform(*centre_frac) * (n - 1) for n in (nx, ny, nz)]
        r2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2
        vol += amplitude * np.exp(-0.5 * r2 / (s * s))
    if noise > 0:
        vol += rng.uniform(0.0, noise, size=shape_zyx)
    return vol.astype(np.float32)


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, a, b, c = q
    return np.array([
        [1 - 2 * (b * b + c * c), 2 * (a * b - c * w), 2 * (a * c + b * w)],
        [2 * (a * b + c * w), 1 - 2 * (a * a + c * c), 2 * (b * c - a * w)],
        [2 * (a * c - b * w), 2 * (b * c + a * w), 1 - 2 * (a * a + b * b)],
    ])


def ellipsoid_volume(shape_zyx, n_ell: int, rng: np.random.Generator, *,
                     centre: Tuple[float, float] = (-0.6, 0.6),
                     semi_axes: Tuple[float, float] = (0.1, 0.45),
                     density: Tuple[float, float] = (0.2, 1.0)) -> np.ndarray:
    """Piecewise-constant randomly rotated ellipsoids combined with max."""
    nz, ny, nx = shape_zyx
    nmax = max(shape_zyx)
    h = 2.0 / (nmax - 1)
    zs = (np.arange(nz) - (nz - 1) / 2.0) * h
    ys = (np.arange(ny) - (ny - 1) / 2.0) * h
    xs = (np.arange(nx) - (nx - 1) / 2.0) * h
    vol = np.zeros(shape_zyx, dtype=np.float32)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    P = np.stack([X, Y, Z], axis=-1).astype(np.float32)
    for _ in range(n_ell):
        c = rng.uniform(*centre, size=3)
        a = rng.uniform(*semi_axes, size=3)
        Rm = _random_rotation(rng)
        dens = rng.uniform(*density)
        local = (P - c.astype(np.float32)) @ Rm.astype(np.float32)
        inside = ((local / a.astype(np.float32)) ** 2).sum(-1) <= 1.0
        vol = np.where(inside, np.maximum(vol, np.float32(dens)), vol)
    return vol.astype(np.float32)


def _value_noise(shape_zyx, lattice: int, rng: np.random.Generator) -> np.ndarray:
    """Trilinearly upsampled i.i.d. lattice noise (one octave), separable."""
    nz, ny, nx = shape_zyx
    lat = rng.uniform(0.0, 1.0, size=(lattice + 1,) * 3)

    def upsample(a, n, axis):
        t = np.arange(n) * (lattice / max(n - 1, 1))
        i = np.minimum(np.floor(t).astype(np.int64), lattice - 1)
        f = (t - i).reshape([-1 if k == axis else 1 for k in range(3)])
        return np.take(a, i, axis=axis) * (1.0 - f) + np.take(a, i + 1, axis=axis) * f

    out = upsample(lat, nx, 2)
    out = upsample(out, ny, 1)
    return upsample(out, nz, 0)


def sparse_noise_volume(shape_zyx, rng: np.random.Generator, *,
                        octaves: int = 5, base_lattice: int = 8,
                        nonzero_frac: float = 0.10) -> np.ndarray:
    """Octave value noise, normalised to [0,1], thresholded to a sparse set."""
    acc = np.zeros(shape_zyx, dtype=np.float64)
    for o in range(octaves):
        acc += (2.0 ** -o) * _value_noise(shape_zyx, base_lattice * 2 ** o, rng)
    acc -= acc.min()
    acc /= max(acc.max(), 1e-30)
    theta = float(np.quantile(acc, 1.0 - nonzero_frac))
    d = np.clip((acc - theta) / max(1.0 - theta, 1e-30), 0.0, 1.0)
    return d.astype(np.float32)


# --------------------------------------------------------------------------
# transfer functions
# --------------------------------------------------------------------------
def random_tf(R: int, rng: np.random.Generator, tau_max: float) -> np.ndarray:
    """[R][4] table: rgb ~ U[0,1]^3, tau_0 = 0, tau_k ~ U[0, tau_max]."""
    tf = np.empty((R, 4), dtype=np.float64)
    tf[:, :3] = rng.uniform(0.0, 1.0, size=(R, 3))
    tf[:, 3] = rng.uniform(0.0, tau_max, size=R)
    tf[0, 3] = 0.0
    return tf.astype(np.float32)


# --------------------------------------------------------------------------
# camera poses
# --------------------------------------------------------------------------
def fibonacci_sphere(n: int) -> List[Tuple[float, float]]:
    """(yaw, pitch) in degrees of ``n`` near-uniform directions.

    z_i = 1 - (2i+1)/n, azimuth i*pi*(3 - sqrt 5); the direction is
    returned as yaw/pitch of the sphere parameterisation
    e = (cos p cos y, sin p, cos p sin y), with the Fibonacci z playing the
    role of the vertical (y) component.
    """
    out = []
    ga = np.pi * (3.0 - np.sqrt(5.0))
    for i in range(n):
        up = 1.0 - (2.0 * i + 1.0) / n
        az = i * ga
        pitch = np.degrees(np.arcsin(np.clip(up, -1.0, 1.0)))
        yaw = np.degrees(az) % 360.0
        out.append((float(yaw), float(pitch)))
    return out


@dataclass
class View:
    yaw: float      # degrees
    pitch: float    # degrees
    dist: float     # world units
    width: int
    height: int
    fovy: float = 60.0   # degrees


@dataclass
class Workload:
    """One seeded problem instance (inputs only)."""
    name: str
    model: str                      # "ao", "ea" or "color"
    volume: np.ndarray              # float32 [nz][ny][nx] (colour: [nz][ny][nx][4])
    storage: str                    # "f32" | "f16" | "bf16"
    tf: Optional[np.ndarray]        # float32 [R][4] or None for AO
    views: List[View]
    step_vox: float                 # step in voxels
    target_volume: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.volume.shape

    @property
    def step_world(self) -> float:
        n = max(self.volume.shape[:3])
        return float(self.step_vox * 2.0 / (n - 1))


# --------------------------------------------------------------------------
# the five configurations (C1..C5) and a small scaled-down variant of each
# --------------------------------------------------------------------------
# Calibrated extinction scales for the EA configs: chosen so that the median
# transmittance of rays that hit the grid is in [0.1, 0.5] (C2) and that at
# least 1% of rays are nearly opaque (C5).  Frozen constants.
C2_TAU_MAX = 12.0
C4_TAU_MAX = 12.0
C5_TAU_MAX = 60.0


def make_c1(n: int = 32, image: int = 64) -> Workload:
    rng = rng_for(1, 0)
    vol = blob_volume((n, n, n), 4, rng, sigma_vox=(3.0, 8.0), amplitude=0.5)
    tgt = blob_volume((n, n, n), 4, rng_for(1, 1), sigma_vox=(3.0, 8.0), amplitude=0.5)
    return Workload("C1: AO 32^3 f32 blobs, 64x64, step 0.5 vox", "ao", vol, "f32",
                    None, [View(30.0, 20.0, 2.5, image, image)], 0.5,
                    target_volume=tgt)


def make_c2(n: int = 128, image: int = 256, R: int = 16) -> Workload:
    rng = rng_for(2, 0)
    vol = blob_volume((n, n, n), 8, rng, sigma_world=(0.1, 0.25), amplitude=0.5,
                      noise=0.02)
    tf = random_tf(R, rng, C2_TAU_MAX)
    yaw = float(rng.uniform(0.0, 360.0))
    pitch = float(rng.uniform(-60.0, 60.0))
    rng1 = rng_for(2, 1)
    tf_t = np.clip(tf + rng1.normal(0.0, 0.05, size=tf.shape).astype(np.float32)
                   * np.array([1, 1, 1, C2_TAU_MAX], np.float32), 0.0, None)
    tf_t[0, 3] = 0.0
    return Workload("C2: EA 128^3 f32 blobs+noise, R=16, 256x256, step 0.5 vox", "ea",
                    vol, "f32", tf, [View(yaw, pitch, 2.5, image, image)], 0.5,
                    meta={"target_tf": tf_t.astype(np.float32),
                          "target_view": View(yaw + 3.0, pitch - 2.0, 2.45, image, image),
                          "target_step_vox": 0.55})


def make_c3(n: int = 256, n_views: int = 64, image: int = 512,
            step_vox: float = 0.2) -> Workload:
    rng = rng_for(3, 0)
    gt = ellipsoid_volume((n, n, n), 12, rng)
    views = [View(y, p, 2.5, image, image) for (y, p) in fibonacci_sphere(n_views)]
    recon = np.zeros((n, n, n), dtype=np.float32)
    return Workload(f"C3: AO tomography {n}^3 bf16, {n_views} views {image}^2, "
                    f"step {step_vox} vox", "ao", recon, "bf16", None, views, step_vox,
                    target_volume=gt)


def make_c4(n_vol: int = 16, edge: Tuple[int, int] = (64, 384),
            image: Tuple[int, int] = (128, 1024)) -> List[Workload]:
    rng = rng_for(4, 0)
    out = []
    for v in range(n_vol):
        shape = tuple(int(rng.integers(edge[0], edge[1] + 1)) for _ in range(3))
        storage = "f16" if rng.uniform() < 0.5 else "f32"
        vol = blob_volume(shape, 8, rng, sigma_world=(0.1, 0.25), amplitude=0.5,
                          noise=0.02)
        R = int(rng.integers(8, 65))
        tf = random_tf(R, rng, C4_TAU_MAX)
        side = int(rng.integers(image[0], image[1] + 1))
        yaw = float(rng.uniform(0.0, 360.0))
        pitch = float(rng.uniform(-60.0, 60.0))
        step = float(rng.uniform(0.25, 1.0))
        out.append(Workload(f"C4[{v}]", "ea", vol, storage, tf,
                            [View(yaw, pitch, 2.5, side, side)], step))
    return out


def make_c5(n: int = 512, n_views: int = 32, image: int = 1024, R: int = 32,
            step_vox: float = 0.25) -> Workload:
    rng = rng_for(5, 0)
    vol = sparse_noise_volume((n, n, n), rng)
    tf = random_tf(R, rng, C5_TAU_MAX)
    views = [View(y, p, 2.5, image, image) for (y, p) in fibonacci_sphere(n_views)]
    return Workload(f"C5: EA {n}^3 f16 sparse noise, R={R}, {n_views} views {image}^2, "
                    f"step {step_vox} vox", "ea", vol, "f16", tf, views, step_vox)


def color_volume(shape_zyx, rng: np.random.Generator, tau_max: float, n_blobs: int = 6,
                 noise: float = 0.02) -> np.ndarray:
    """[nz][ny][nx][4] pre-shaded colour volume (r, g, b, tau) per vertex:
    three independent blob fields clipped to [0, 1] for the emission and a
    fourth, scaled to [0, tau_max], for the extinction (the four-channel
    volume Sec. 5.4 reconstructs in place of a density + TF)."""
    out = np.empty(tuple(shape_zyx) + (4,), dtype=np.float32)
    for ch in range(4):
        f = blob_volume(shape_zyx, n_blobs, rng, sigma_world=(0.1, 0.3), amplitude=0.6,
                        noise=noise)
        out[..., ch] = np.clip(f, 0.0, 1.0) * (tau_max if ch == 3 else 1.0)
    return out


# Extinction scale of the colour-volume workload: median transmittance of the
# rays that hit the grid in [0.1, 0.5] at 256^3 (frozen constant).
COLOR_TAU_MAX = 48.0


def make_color(n: int = 256, n_views: int = 64, image: int = 512,
               step_vox: float = 0.2, storage: str = "bf16") -> Workload:
    """Colour-volume reconstruction (Sec. 5.4 first stage): the C3 setting
    (grid, views, step) with a four-channel volume; the volume is a
    mid-optimisation state, the targets are drawn per view by the caller."""
    rng = rng_for(6, 0)
    vol = color_volume((n, n, n), rng, COLOR_TAU_MAX)
    views = [View(y, p, 2.5, image, image) for (y, p) in fibonacci_sphere(n_views)]
    return Workload(f"colour volume {n}^3x4 {storage}, {n_views} views {image}^2, "
                    f"step {step_vox} vox", "color", vol, storage, None, views, step_vox)


def image_target(rng: np.random.Generator, n_pix: int, channels: int) -> np.ndarray:
    """Seeded loss target / upstream gradient, U[0,1)."""
    return rng.uniform(0.0, 1.0, size=(n_pix, channels)).astype(np.float32)


def random_params(rng: np.random.Generator, shape, scale: float = 1.0) -> np.ndarray:
    return (scale * rng.uniform(0.0, 1.0, size=shape)).astype(np.float32)
