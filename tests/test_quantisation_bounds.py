"""The a-priori bounds on the effect of storing the density grid in bf16 /
f16 (round to nearest even), checked on the CPU with the FP64 oracle: the
image of the rounded grid stays within the bound of the image of the float32
master, pixel by pixel, for absorption-only and emission-absorption rendering,
and the absorption-only density gradient within its bound.  The cases are
chosen so that each part of the bound is needed: dropping the TF's extinction
slope, the transmittance factor or the colour-slope term makes a case fail;
each test also checks that the rounding effect reaches a fair share of the
bound, so that a bound loose by orders of magnitude fails too."""
import numpy as np
import pytest
import torch

import oracle
import synth
from harness import ETA_Q, U_Q, quantisation_image_bound


def _rounded(V, storage):
    dt = {"f16": torch.float16, "bf16": torch.bfloat16}[storage]
    return torch.from_numpy(V).to(dt).to(torch.float64).numpy()


def _problem(seed, n=(18, 20, 16), W=24, H=20, R=8, tau_max=40.0):
    rng = np.random.default_rng(seed)
    V = synth.blob_volume(n, 5, rng, sigma_world=(0.15, 0.4), amplitude=0.9, noise=0.02)
    tf = synth.random_tf(R, rng, tau_max)
    cam = oracle.camera_from_sphere(37.0, 21.0, 2.5, 60.0, W, H)
    step = 0.5 * 2.0 / (max(n) - 1)
    return V.astype(np.float32), tf, cam, W, H, step


@pytest.mark.parametrize("storage", ["bf16", "f16"])
@pytest.mark.parametrize("model", [oracle.AO, oracle.EA])
def test_rounded_grid_images_stay_within_the_bound(storage, model):
    worst = 0.0
    for seed in (1, 2, 3):
        V, tf, cam, W, H, step = _problem(seed)
        pix = np.arange(W * H, dtype=np.int32)
        t = tf if model == oracle.EA else None
        a = oracle.render(V, t, cam, W, H, step, model, pix=pix)["image"]
        b = oracle.render(_rounded(V, storage), t, cam, W, H, step, model, pix=pix)["image"]
        bound = quantisation_image_bound(V, t, cam, W, H, step, storage, pix, model)
        assert np.all(np.abs(b - a) <= bound * (1 + 1e-9) + 1e-15), (seed, storage, model)
        hit = bound > 0
        worst = max(worst, float((np.abs(b - a)[hit] / bound[hit]).max()))
    # the bound is not vacuous: the rounding effect reaches a fair share of it
    assert worst > 0.02, worst


def test_absorption_only_bound_is_sharp_for_a_uniform_slab():
    """Uniform density v stored with relative error u: alpha moves by
    T (e^{u D} - 1) to first order exactly -- the bound with equality."""
    n = 9
    v = np.float32(0.7)
    V = np.full((n, n, n), v, np.float32)
    W = H = 3
    cam = oracle.camera_from_sphere(0.0, 0.0, 2.5, 10.0, W, H)
    step = 0.25 * 2.0 / (n - 1)
    pix = np.array([4], np.int32)            # the centre pixel: the axis ray
    for storage in ("bf16", "f16"):
        Vq = _rounded(V, storage)
        delta = (float(Vq.flat[0]) - float(v)) / float(v)
        assert abs(delta) <= U_Q[storage]
        a = oracle.render(V, None, cam, W, H, step, oracle.AO, pix=pix)["image"][0, 0]
        b = oracle.render(Vq, None, cam, W, H, step, oracle.AO, pix=pix)["image"][0, 0]
        bound = quantisation_image_bound(V, None, cam, W, H, step, storage, pix, oracle.AO)[0, 0]
        assert abs(b - a) <= bound
        # the actual effect is the bound with this grid's own rounding error
        T = 1.0 - a
        D = -np.log(T)
        assert abs((b - a) + T * np.expm1(-delta * D)) <= 1e-12


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_absorption_only_gradient_bound(storage):
    """Absorption-only: the adjoint is the projector of dt g T_N
    (the inversion in closed form), so rounding the grid scales each ray's
    contribution by T_N'/T_N = e^{-(D'-D)}: |dV_q - dV| <= P^T(dt |g| T_N rho)
    with rho = e^{E} - 1 per ray."""
    V, tf, cam, W, H, step = _problem(4)
    pix = np.arange(W * H, dtype=np.int32)
    rng = np.random.default_rng(7)
    g = rng.normal(size=(W * H, 1))
    a = oracle.adjoint(V, None, cam, W, H, step, oracle.AO, g, pix=pix)["dV"]
    b = oracle.adjoint(_rounded(V, storage), None, cam, W, H, step, oracle.AO, g, pix=pix)["dV"]
    ao = oracle.render(V, None, cam, W, H, step, oracle.AO, pix=pix)
    D = -np.log(ao["trans"])
    rho = np.expm1(U_Q[storage] * D + ETA_Q[storage] * ao["nsamp"] * step)
    absb = oracle.adjoint(V, None, cam, W, H, step, oracle.AO, np.abs(g) * rho[:, None],
                          pix=pix)["dV"]
    assert np.all(np.abs(b - a) <= absb * (1 + 1e-9) + 1e-18)
    assert float((np.abs(b - a) / np.maximum(absb, 1e-300)).max()) > 0.02


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_colour_slope_term_of_the_bound(storage):
    """Constant extinction, steep colour ramp: the optical depth does not move
    (E = 0), so only the TF's colour slope L_rgb (u + eta) bounds the change."""
    V, tf, cam, W, H, step = _problem(5)
    R = tf.shape[0]
    tf = tf.copy()
    tf[:, 3] = 30.0
    tf[:, 0] = np.linspace(0.0, 1.0, R)
    tf[:, 1] = np.linspace(1.0, 0.0, R)
    pix = np.arange(W * H, dtype=np.int32)
    a = oracle.render(V, tf, cam, W, H, step, oracle.EA, pix=pix)["image"]
    b = oracle.render(_rounded(V, storage), tf, cam, W, H, step, oracle.EA, pix=pix)["image"]
    bound = quantisation_image_bound(V, tf, cam, W, H, step, storage, pix, oracle.EA)
    assert np.all(bound[:, 3] == 0.0)
    assert np.all(np.abs(b - a) <= bound * (1 + 1e-9) + 1e-15)
    assert float((np.abs(b - a)[:, :3] / bound[:, :3]).max()) > 0.03
