"""FP64 CPU oracle for differentiable direct volume rendering (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and
by the CPU-baseline leg of the benchmark -- never by the product package.
It shares no code with the HIP library; the two meet only through the seeded
arrays drawn by ``synth``.

Every function takes plain numpy arrays (converted to float64) and returns
float64 results.  Camera poses are frames of 12 numbers
``[eye, fwd, right*s_x, up*s_y]`` (Sec. 4.1 f_camera; the pose on the sphere
of Sec. 5.1 is converted by :func:`camera_from_sphere`).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ddvr_oracle.cpp")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "libddvr_oracle.so")

TAPE, INV_T, INV_ALPHA, CHECKPOINT, RESIDUAL = 0, 1, 2, 3, 4
AO, EA, COLOR = 0, 1, 2     # COLOR: pre-shaded colour volume [nz][ny][nx][4] = (r, g, b, tau)

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (OpenMP, -O2, strict IEEE: no fast-math)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared",
               "-ffp-contract=off", "-o", tmp, _SRC]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    d = ctypes.c_double
    i = ctypes.c_int
    p = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.oracle_set_threads.argtypes = [i]
    lib.oracle_set_threads.restype = ctypes.c_int
    lib.oracle_camera_from_sphere.argtypes = [d, d, d, d, i, i, p]
    lib.oracle_camera_jacobian.argtypes = [d, d, d, d, i, i, p]
    lib.oracle_render.argtypes = [p, i, i, i, p, i, p, i, i, d, i, p, i64, p, p, p, p]
    lib.oracle_adjoint.argtypes = [p, i, i, i, p, i, p, i, i, d, i, p, i64, p, i, i,
                                   p, p, p, p]
    lib.oracle_render_dual.argtypes = [p, p, i, i, i, p, p, i, p, p, i, i, d, d, i, p,
                                       i64, p, p, p, p]
    lib.oracle_trilinear.argtypes = [p, i, i, i, p, p]
    lib.oracle_tf_lookup.argtypes = [p, i, d, p]
    lib.oracle_ray.argtypes = [p, i, i, i, i, i, i, i, d, p]
    lib.oracle_trace_ray.argtypes = [p, i, i, i, p, i, p, i, i, i, i, d, i, i, p, p, p, p]
    lib.oracle_kinks.argtypes = [p, i, i, i, p, i, p, i, i, d, i, p, i64, p, p, p]
    u64 = ctypes.c_uint64
    lib.oracle_splitmix64.argtypes = [u64, u64, p]
    lib.oracle_density_from_color.argtypes = [p, i, i, i, p, i, p, d, d, u64, i, i, p, i64,
                                              p, p, p, p, p]
    for f in (lib.oracle_camera_from_sphere, lib.oracle_camera_jacobian, lib.oracle_render,
              lib.oracle_adjoint, lib.oracle_render_dual, lib.oracle_trilinear,
              lib.oracle_tf_lookup, lib.oracle_ray, lib.oracle_num_threads,
              lib.oracle_trace_ray, lib.oracle_kinks):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a):
    if a is None:
        return None
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with status {rc}")


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_threads(n: int) -> int:
    """Threads the oracle's parallel loops use from now on; returns the count."""
    return _load().oracle_set_threads(int(n))


def camera_from_sphere(yaw_deg, pitch_deg, dist, fovy_deg, W, H) -> np.ndarray:
    out = np.zeros(12, np.float64)
    _check(_load().oracle_camera_from_sphere(np.radians(yaw_deg), np.radians(pitch_deg),
                                             float(dist), np.radians(fovy_deg), int(W),
                                             int(H), _ptr(out)), "camera_from_sphere")
    return out


def camera_jacobian(yaw_deg, pitch_deg, dist, fovy_deg, W, H) -> np.ndarray:
    """[4][12]: d frame / d (yaw, pitch, dist, fovy), angles in RADIANS."""
    out = np.zeros(48, np.float64)
    _check(_load().oracle_camera_jacobian(np.radians(yaw_deg), np.radians(pitch_deg),
                                          float(dist), np.radians(fovy_deg), int(W), int(H),
                                          _ptr(out)), "camera_jacobian")
    return out.reshape(4, 12)


def _pix(pix):
    if pix is None:
        return None, 0
    p = np.ascontiguousarray(np.asarray(pix, dtype=np.int32))
    return p, int(p.size)


def render(volume, tf, cam, W, H, step, model, pix=None):
    """Returns dict(image [npix,C], trans [npix], nsamp [npix], ratio [npix])."""
    V = _f64(volume)
    nz, ny, nx = V.shape[:3]
    T = _f64(tf) if model == EA else None
    R = 0 if T is None else T.shape[0]
    cam = _f64(cam)
    p, npix = _pix(pix)
    n = npix if p is not None else W * H
    C = 1 if model == AO else 4
    image = np.zeros((n, C), np.float64)
    trans = np.zeros(n, np.float64)
    nsamp = np.zeros(n, np.int32)
    ratio = np.zeros(n, np.float64)
    _check(_load().oracle_render(_ptr(V), nx, ny, nz, _ptr(T), R, _ptr(cam), int(W), int(H),
                                 float(step), int(model), _ptr(p), npix, _ptr(image),
                                 _ptr(trans), _ptr(nsamp), _ptr(ratio)), "render")
    return {"image": image, "trans": trans, "nsamp": nsamp, "ratio": ratio}


def adjoint(volume, tf, cam, W, H, step, model, d_image, variant=TAPE, pix=None, ck_K=0,
            want_dV=True):
    """Gradients of <d_image, image> -> dict(dV, dTF, dcam, dstep)."""
    V = _f64(volume)
    nz, ny, nx = V.shape[:3]
    T = _f64(tf) if model == EA else None
    R = 0 if T is None else T.shape[0]
    cam = _f64(cam)
    p, npix = _pix(pix)
    g = _f64(d_image)
    dV = np.zeros_like(V) if want_dV else None
    dTF = np.zeros((max(R, 1), 4), np.float64) if T is not None else None
    dcam = np.zeros(12, np.float64)
    dstep = np.zeros(1, np.float64)
    _check(_load().oracle_adjoint(_ptr(V), nx, ny, nz, _ptr(T), R, _ptr(cam), int(W), int(H),
                                  float(step), int(model), _ptr(p), npix, _ptr(g),
                                  int(variant), int(ck_K), _ptr(dV), _ptr(dTF), _ptr(dcam),
                                  _ptr(dstep)), "adjoint")
    return {"dV": dV, "dTF": dTF, "dcam": dcam, "dstep": float(dstep[0])}


def render_dual(volume, tf, cam, W, H, step, model, V_dir=None, tf_dir=None, cam_dir=None,
                step_dir=0.0, pix=None):
    """Forward mode along one direction -> dict(image, image_dot, trans, trans_dot)."""
    V = _f64(volume)
    nz, ny, nx = V.shape[:3]
    T = _f64(tf) if model == EA else None
    R = 0 if T is None else T.shape[0]
    cam = _f64(cam)
    p, npix = _pix(pix)
    n = npix if p is not None else W * H
    C = 1 if model == AO else 4
    image = np.zeros((n, C)); image_dot = np.zeros((n, C))
    trans = np.zeros(n); trans_dot = np.zeros(n)
    _check(_load().oracle_render_dual(
        _ptr(V), _ptr(_f64(V_dir)), nx, ny, nz, _ptr(T), _ptr(_f64(tf_dir)), R, _ptr(cam),
        _ptr(_f64(cam_dir)), int(W), int(H), float(step), float(step_dir), int(model), _ptr(p),
        npix, _ptr(image), _ptr(image_dot), _ptr(trans), _ptr(trans_dot)), "render_dual")
    return {"image": image, "image_dot": image_dot, "trans": trans, "trans_dot": trans_dot}


def trilinear(volume, x) -> float:
    V = _f64(volume)
    nz, ny, nx = V.shape[:3]
    xx = _f64(x)
    out = np.zeros(1)
    _check(_load().oracle_trilinear(_ptr(V), nx, ny, nz, _ptr(xx), _ptr(out)), "trilinear")
    return float(out[0])


def tf_lookup(tf, d) -> np.ndarray:
    T = _f64(tf)
    out = np.zeros(4)
    _check(_load().oracle_tf_lookup(_ptr(T), T.shape[0], float(d), _ptr(out)), "tf_lookup")
    return out


def ray(cam, shape_zyx, W, H, px, py, step):
    """(N, x_o, omega, t0, L/dt) of one pixel's ray."""
    out = np.zeros(8)
    nz, ny, nx = shape_zyx
    N = _load().oracle_ray(_ptr(_f64(cam)), nx, ny, nz, int(W), int(H), int(px), int(py),
                           float(step), _ptr(out))
    if N < 0:
        raise ValueError("oracle ray failed")
    return N, out[0:3].copy(), out[3:6].copy(), float(out[6]), float(out[7])


def sphere_grad(dcam, yaw_deg, pitch_deg, dist, fovy_deg, W, H) -> np.ndarray:
    """Chain a frame gradient to (yaw, pitch, dist, fovy) [angles in radians]."""
    J = camera_jacobian(yaw_deg, pitch_deg, dist, fovy_deg, W, H)
    return J @ np.asarray(dcam, np.float64)


def trace_ray(volume, tf, cam, W, H, px, py, step, model, cap=100000):
    """Per-sample (d, tau, T_before, x) of one pixel's ray."""
    V = _f64(volume)
    nz, ny, nx = V.shape[:3]
    T = _f64(tf) if model == EA else None
    R = 0 if T is None else T.shape[0]
    d = np.zeros(cap); tau = np.zeros(cap); Tb = np.zeros(cap); x = np.zeros(3 * cap)
    N = _load().oracle_trace_ray(_ptr(V), nx, ny, nz, _ptr(T), R, _ptr(_f64(cam)), int(W),
                                 int(H), int(px), int(py), float(step), int(model), int(cap),
                                 _ptr(d), _ptr(tau), _ptr(Tb), _ptr(x))
    if N < 0:
        raise ValueError("oracle trace_ray failed")
    m = min(N, cap)
    return {"N": N, "d": d[:m], "tau": tau[:m], "T": Tb[:m], "x": x[:3 * m].reshape(m, 3)}


def kinks(volume, tf, cam, W, H, step, model, pix=None, with_entry=False):
    """Per ray: (min distance of a sample to an interior cell face [voxels],
    min distance of d*(R-1) to a TF knot [EA]) and, with_entry, t0/|omega_a|
    of the entry plane a."""
    V = _f64(volume)
    nz, ny, nx = V.shape[:3]
    T = _f64(tf) if model == EA else None
    R = 0 if T is None else T.shape[0]
    p, npix = _pix(pix)
    n = npix if p is not None else W * H
    face = np.zeros(n)
    knot = np.zeros(n)
    entry = np.zeros(n)
    _check(_load().oracle_kinks(_ptr(V), nx, ny, nz, _ptr(T), R, _ptr(_f64(cam)), int(W), int(H),
                                float(step), int(model), _ptr(p), npix, _ptr(face), _ptr(knot),
                                _ptr(entry)), "kinks")
    return (face, knot, entry) if with_entry else (face, knot)


# ---------------------------------------------------------------------------
# density from colour (Sec. 5.4)
# ---------------------------------------------------------------------------
def splitmix64(seed: int, n: int) -> int:
    """Output n of the SplitMix64 stream of `seed` (the candidates' generator)."""
    out = ctypes.c_uint64(0)
    _check(_load().oracle_splitmix64(ctypes.c_uint64(seed), ctypes.c_uint64(n),
                                     ctypes.byref(out)), "splitmix64")
    return int(out.value)


def density_from_color(CV, tf, d_prev=None, alpha=1.0, beta=1.0, seed=0, iteration=0,
                       ncand=256, all_costs=False, voxels=None):
    """One estimation sweep: per voxel the least-cost candidate density.
    CV [nz][ny][nx][4], tf [R][4], d_prev [nz][ny][nx] or None; voxels: flat
    indices to evaluate (outputs then follow that list), or None for all.
    Returns dict(d, cost, index[, costs, cands: [voxel][ncand]])."""
    V = _f64(CV)
    nz, ny, nx = V.shape[:3]
    T = _f64(tf)
    P = None if d_prev is None else _f64(d_prev)
    sel = None if voxels is None else np.ascontiguousarray(np.asarray(voxels, dtype=np.int64))
    shape = (nz, ny, nx) if sel is None else (len(sel),)
    nq = int(np.prod(shape))
    d = np.zeros(shape)
    c = np.zeros(shape)
    idx = np.zeros(shape, dtype=np.int32)
    allc = np.zeros((nq, ncand)) if all_costs else None
    alld = np.zeros((nq, ncand)) if all_costs else None
    _check(_load().oracle_density_from_color(
        _ptr(V), nx, ny, nz, _ptr(T), T.shape[0], _ptr(P), float(alpha), float(beta),
        ctypes.c_uint64(seed), int(iteration), int(ncand),
        None if sel is None else sel.ctypes.data_as(ctypes.c_void_p), 0 if sel is None else len(sel),
        _ptr(d), _ptr(c), idx.ctypes.data_as(ctypes.c_void_p), _ptr(allc), _ptr(alld)),
        "density_from_color")
    out = {"d": d, "cost": c, "index": idx}
    if all_costs:
        out["costs"] = allc
        out["cands"] = alld
    return out
