"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formulas: each checks a closed form,
an invariant, a symmetry, an independent differentiation route (dual numbers,
finite differences) or a reduction to a textbook operation (the linear
trilinear projector of absorption-only tomography, Sec. 5.3).
"""
import math

import numpy as np
import pytest

import oracle
import synth

AO, EA = oracle.AO, oracle.EA


def _cube(n, value):
    return np.full((n, n, n), value, dtype=np.float64)


# ---------------------------------------------------------------------------
# geometry (f_camera, Alg. 1; sphere pose, Sec. 5.1)
# ---------------------------------------------------------------------------
def test_camera_frame_is_orthonormal_pinhole():
    for yaw, pitch, dist, fovy, W, H in [(30, 20, 2.5, 60, 64, 64), (200, -55, 3.1, 45, 80, 48)]:
        f = oracle.camera_from_sphere(yaw, pitch, dist, fovy, W, H)
        e, F, R, U = f[0:3], f[3:6], f[6:9], f[9:12]
        assert np.linalg.norm(e) == pytest.approx(dist, rel=1e-14)
        assert np.allclose(F, -e / dist, atol=1e-14)           # faces the centre
        sy = math.tan(math.radians(fovy) / 2)
        sx = sy * W / H
        assert np.linalg.norm(R) == pytest.approx(sx, rel=1e-13)
        assert np.linalg.norm(U) == pytest.approx(sy, rel=1e-13)
        assert abs(R @ F) < 1e-14 and abs(U @ F) < 1e-14 and abs(R @ U) < 1e-14
        assert R[1] == 0.0                                      # horizon stays level
        assert U[1] > 0                                         # up is +y
        # right-handed: right x up points back toward the eye
        assert np.cross(R / sx, U / sy) @ F == pytest.approx(-1.0, abs=1e-13)


def test_camera_jacobian_matches_finite_differences():
    args = (40.0, 25.0, 2.7, 55.0, 96, 64)
    J = oracle.camera_jacobian(*args)
    for p in range(4):
        a = list(args)
        h_deg = 1e-5
        hp = [math.radians(h_deg), math.radians(h_deg), 1e-6, math.radians(h_deg)][p]
        step = [h_deg, h_deg, 1e-6, h_deg][p]
        a[p] += step
        fp = oracle.camera_from_sphere(*a)
        a[p] -= 2 * step
        fm = oracle.camera_from_sphere(*a)
        fd = (fp - fm) / (2 * hp)
        assert np.allclose(J[p], fd, rtol=1e-7, atol=1e-8), p


def test_axis_ray_length_and_sample_count():
    # eye on +x looking at the origin; centre pixel of an odd image is the axis ray
    n = 17
    cam = oracle.camera_from_sphere(0.0, 0.0, 2.5, 60.0, 5, 5)
    for step in (0.1, 0.3, 0.07):
        N, xo, om, t0, ratio = oracle.ray(cam, (n, n, n), 5, 5, 2, 2, step)
        assert np.allclose(om, [-1, 0, 0], atol=1e-15)
        assert t0 == pytest.approx(1.5, abs=1e-14)             # enters at x = +1
        assert np.allclose(xo, [1, 0, 0], atol=1e-14)
        assert ratio == pytest.approx(2.0 / step, rel=1e-14)   # L = 2 exactly
        assert N == math.ceil(2.0 / step - 1e-12)


def _slab_length(e, om, lo, hi):
    tn, tf = -np.inf, np.inf
    for a in range(3):
        if om[a] == 0:
            if not (lo[a] <= e[a] <= hi[a]):
                return 0.0, 0.0
            continue
        t1, t2 = (lo[a] - e[a]) / om[a], (hi[a] - e[a]) / om[a]
        tn, tf = max(tn, min(t1, t2)), min(tf, max(t1, t2))
    t0 = max(tn, 0.0)
    return (t0, tf - t0) if tf > t0 else (0.0, 0.0)


def test_sample_counts_match_independent_box_clip():
    shape = (20, 33, 27)  # nz, ny, nx -> longest axis y spans [-1, 1]
    h = 2.0 / 32
    half = np.array([(27 - 1) * h / 2, (33 - 1) * h / 2, (20 - 1) * h / 2])
    W, H = 23, 19
    cam = oracle.camera_from_sphere(70, -30, 2.2, 60, W, H)
    step = 0.037
    rng = np.random.default_rng(3)
    for _ in range(40):
        px, py = int(rng.integers(W)), int(rng.integers(H))
        u = 2 * (px + 0.5) / W - 1
        v = 1 - 2 * (py + 0.5) / H
        w = cam[3:6] + u * cam[6:9] + v * cam[9:12]
        om = w / np.linalg.norm(w)
        t0, L = _slab_length(cam[0:3], om, -half, half)
        N, xo, om2, t0o, ratio = oracle.ray(cam, shape, W, H, px, py, step)
        if L == 0:
            assert N == 0
            continue
        assert np.allclose(om, om2, atol=1e-15)
        assert t0o == pytest.approx(t0, abs=1e-13)
        assert ratio == pytest.approx(L / step, rel=1e-12)
        if abs(L / step - round(L / step)) > 1e-9:
            assert N == math.ceil(L / step)


def test_missing_rays_are_exact_zeros_and_carry_no_gradient():
    n, W, H = 8, 24, 24
    rng = np.random.default_rng(4)
    V = rng.uniform(0, 1, (n, n, n))
    tf = synth.random_tf(6, rng, 5.0)
    cam = oracle.camera_from_sphere(10, 10, 2.5, 90, W, H)   # wide fov: corners miss
    out = oracle.render(V, tf, cam, W, H, 0.05, EA)
    miss = out["nsamp"] == 0
    assert miss.sum() > 20 and (~miss).sum() > 20
    assert np.all(out["image"][miss] == 0.0) and np.all(out["trans"][miss] == 1.0)
    g = np.zeros((W * H, 4))
    g[miss] = rng.normal(size=(miss.sum(), 4))
    adj = oracle.adjoint(V, tf, cam, W, H, 0.05, EA, g)
    assert np.all(adj["dV"] == 0) and np.all(adj["dTF"] == 0)
    assert np.all(adj["dcam"] == 0) and adj["dstep"] == 0


def test_rotating_the_volume_rotates_the_image():
    n, W = 12, 16
    rng = np.random.default_rng(5)
    V = rng.uniform(0, 1, (n, n, n))
    cam = oracle.camera_from_sphere(0.0, 0.0, 2.5, 50, W, W)   # looks along -x
    base = oracle.render(V, None, cam, W, W, 0.043, AO)["image"].reshape(W, W)
    # rotate by 90 degrees about the x (view) axis: (z, y) plane of the array
    Vr = np.rot90(V, k=1, axes=(0, 1)).copy()
    rot = oracle.render(Vr, None, cam, W, W, 0.043, AO)["image"].reshape(W, W)
    errs = [np.abs(rot - np.rot90(base, k)).max() for k in (1, 3)]
    assert min(errs) < 1e-12 and max(errs) > 1e-3


# ---------------------------------------------------------------------------
# trilinear interpolation (f_interpolate, Sec. 3.1)
# ---------------------------------------------------------------------------
def test_trilinear_reproduces_affine_fields_and_vertices():
    nz, ny, nx = 5, 9, 7
    h = 2.0 / 8
    zs = (np.arange(nz) - (nz - 1) / 2) * h
    ys = (np.arange(ny) - (ny - 1) / 2) * h
    xs = (np.arange(nx) - (nx - 1) / 2) * h
    a, gx, gy, gz = 0.3, 1.7, -0.4, 2.9
    V = a + gx * xs[None, None, :] + gy * ys[None, :, None] + gz * zs[:, None, None]
    rng = np.random.default_rng(6)
    lo = np.array([xs[0], ys[0], zs[0]])
    hi = np.array([xs[-1], ys[-1], zs[-1]])
    for _ in range(50):
        x = rng.uniform(lo, hi)
        assert oracle.trilinear(V, x) == pytest.approx(a + gx * x[0] + gy * x[1] + gz * x[2],
                                                       abs=1e-13)
    # exact vertex values of a random field, including the upper faces
    R = rng.uniform(0, 1, (nz, ny, nx))
    for (k, j, i) in [(0, 0, 0), (4, 8, 6), (2, 3, 1), (4, 0, 6)]:
        x = np.array([xs[i], ys[j], zs[k]])
        assert oracle.trilinear(R, x) == pytest.approx(R[k, j, i], abs=1e-14)
    # partition of unity
    assert oracle.trilinear(np.full((nz, ny, nx), 0.77), rng.uniform(lo, hi)) == \
        pytest.approx(0.77, abs=1e-15)


# ---------------------------------------------------------------------------
# transfer function (f_TF: R regularly spaced knots, linear in between)
# ---------------------------------------------------------------------------
def test_tf_knots_constant_and_ramp():
    rng = np.random.default_rng(7)
    R = 9
    T = rng.uniform(0, 1, (R, 4))
    for k in range(R):
        assert np.allclose(oracle.tf_lookup(T, k / (R - 1)), T[k], atol=1e-14)
    # midpoint between knots is their average
    assert np.allclose(oracle.tf_lookup(T, 2.5 / (R - 1)), 0.5 * (T[2] + T[3]), atol=1e-14)
    # clamping to [0, 1]
    assert np.allclose(oracle.tf_lookup(T, -0.3), T[0]) and np.allclose(oracle.tf_lookup(T, 1.7), T[-1])
    const = np.tile([0.2, 0.4, 0.6, 3.0], (R, 1))
    for d in rng.uniform(-0.5, 1.5, 20):
        assert np.allclose(oracle.tf_lookup(const, d), const[0], atol=1e-15)
    ramp = np.tile((np.arange(R) / (R - 1))[:, None], (1, 4))
    for d in rng.uniform(-0.5, 1.5, 20):
        assert oracle.tf_lookup(ramp, d)[3] == pytest.approx(min(max(d, 0.0), 1.0), abs=1e-14)


# ---------------------------------------------------------------------------
# Beer-Lambert closed forms on homogeneous slabs (Sec. 3.1, eq. integral2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("step", [0.05, 0.11, 0.3])
def test_absorption_only_constant_density_closed_form(step):
    n, W = 9, 7
    d0 = 0.83
    cam = oracle.camera_from_sphere(23, 17, 2.6, 40, W, W)
    out = oracle.render(_cube(n, d0), None, cam, W, W, step, AO)
    hit = out["nsamp"] > 0
    assert hit.sum() > 10
    N = out["nsamp"][hit]
    expect = 1 - np.exp(-N * step * d0)
    assert np.allclose(out["image"][hit, 0], expect, rtol=0, atol=1e-14)
    # continuum limit of eq. (integral2): |alpha - (1 - e^{-L d})| <= dt*d*e^{-L d}
    L = out["ratio"][hit] * step
    assert np.all(np.abs(out["image"][hit, 0] - (1 - np.exp(-L * d0))) <=
                  step * d0 * np.exp(-L * d0) + 1e-15)


def test_emission_absorption_constant_tf_closed_form():
    n, W, step = 7, 9, 0.07
    rgb, tau = np.array([0.3, 0.5, 0.9]), 2.2
    tf = np.tile(np.r_[rgb, tau], (5, 1))
    rng = np.random.default_rng(8)
    V = rng.uniform(-0.2, 1.2, (n, n, n))     # any density: the TF is constant
    cam = oracle.camera_from_sphere(120, -35, 2.4, 50, W, W)
    out = oracle.render(V, tf, cam, W, W, step, EA)
    hit = out["nsamp"] > 0
    a = 1 - np.exp(-out["nsamp"][hit] * step * tau)
    assert np.allclose(out["image"][hit, 3], a, atol=1e-14)
    assert np.allclose(out["image"][hit, :3], a[:, None] * rgb[None, :], atol=1e-14)


def test_linear_ramp_density_arithmetic_series():
    n, W = 33, 5
    h = 2.0 / (n - 1)
    xs = (np.arange(n) - (n - 1) / 2) * h
    a, b = 0.6, 0.25
    V = np.broadcast_to(a + b * xs[None, None, :], (n, n, n)).copy()
    cam = oracle.camera_from_sphere(0.0, 0.0, 2.5, 30, W, W)     # axis ray along -x
    for step in (0.013, 0.1, 0.17):
        out = oracle.render(V, None, cam, W, W, step, AO, pix=[2 * W + 2])
        N = int(out["nsamp"][0])
        # x_i = 1 - i*dt, d_i = a + b*x_i
        depth = step * (N * (a + b) - b * step * N * (N - 1) / 2)
        assert out["image"][0, 0] == pytest.approx(1 - math.exp(-depth), abs=1e-14)


def test_invariants_alpha_transmittance_colour_bounds():
    rng = np.random.default_rng(9)
    n, W = 10, 12
    V = rng.uniform(0, 1, (n, n, n))
    tf = synth.random_tf(7, rng, 15.0)
    cam = oracle.camera_from_sphere(250, 40, 2.5, 60, W, W)
    out = oracle.render(V, tf, cam, W, W, 0.04, EA)
    a = out["image"][:, 3]
    assert np.all(a >= 0) and np.all(a < 1)
    assert np.allclose(out["trans"], 1 - a, atol=1e-15)
    assert np.all(out["image"][:, :3] <= a[:, None] * tf[:, :3].max() + 1e-15)
    for px, py in [(3, 4), (6, 6), (9, 2)]:
        tr = oracle.trace_ray(V, tf, cam, W, W, px, py, 0.04, EA)
        assert tr["N"] > 0
        T = tr["T"]
        assert T[0] == 1.0 and np.all(np.diff(T) <= 0) and np.all(T > 0)
        # every sample lies inside the grid box
        assert np.all(np.abs(tr["x"]) <= 1 + 1e-12)


# ---------------------------------------------------------------------------
# adjoint (Alg. 2) against independent routes
# ---------------------------------------------------------------------------
def _problem(model, seed=11, n=(6, 7, 5), W=9, H=8, R=5):
    rng = np.random.default_rng(seed)
    V = rng.uniform(0, 1, n)
    tf = synth.random_tf(R, rng, 8.0).astype(np.float64) if model == EA else None
    cam = oracle.camera_from_sphere(37, 25, 2.3, 50, W, H)
    C = 4 if model == EA else 1
    g = rng.normal(size=(W * H, C))
    return rng, V, tf, cam, W, H, 0.13, g


@pytest.mark.parametrize("model", [AO, EA])
def test_adjoint_variants_agree_with_stored_tape(model):
    rng, V, tf, cam, W, H, step, g = _problem(model)
    ref = oracle.adjoint(V, tf, cam, W, H, step, model, g, variant=oracle.TAPE)
    for var in (oracle.INV_T, oracle.INV_ALPHA, oracle.CHECKPOINT, oracle.RESIDUAL):
        got = oracle.adjoint(V, tf, cam, W, H, step, model, g, variant=var)
        for k in ("dV", "dTF", "dcam"):
            if ref[k] is None:
                continue
            scale = np.abs(ref[k]).max()
            assert np.abs(got[k] - ref[k]).max() <= 1e-12 * scale, (var, k)
        assert got["dstep"] == pytest.approx(ref["dstep"], rel=1e-12)


@pytest.mark.parametrize("model", [AO, EA])
def test_adjoint_equals_forward_mode_dual_numbers(model):
    # Sec. 5.1: adjoint and forward differentiation give the same gradients
    rng, V, tf, cam, W, H, step, g = _problem(model, seed=12)
    adj = oracle.adjoint(V, tf, cam, W, H, step, model, g)
    # random joint direction
    Vd = rng.normal(size=V.shape)
    tfd = rng.normal(size=tf.shape) if model == EA else None
    cd = rng.normal(size=12)
    sd = float(rng.normal())
    dual = oracle.render_dual(V, tf, cam, W, H, step, model, Vd, tfd, cd, sd)
    lhs = float((g * dual["image_dot"]).sum())
    rhs = float((adj["dV"] * Vd).sum() + (adj["dcam"] * cd).sum() + adj["dstep"] * sd)
    if model == EA:
        rhs += float((adj["dTF"] * tfd).sum())
    assert lhs == pytest.approx(rhs, rel=1e-11)
    # each camera component and the step individually
    for k in range(12):
        e = np.zeros(12); e[k] = 1
        dk = oracle.render_dual(V, tf, cam, W, H, step, model, cam_dir=e)
        assert float((g * dk["image_dot"]).sum()) == pytest.approx(adj["dcam"][k], rel=1e-10, abs=1e-12)
    ds = oracle.render_dual(V, tf, cam, W, H, step, model, step_dir=1.0)
    assert float((g * ds["image_dot"]).sum()) == pytest.approx(adj["dstep"], rel=1e-11)
    if model == EA:
        for j in range(tf.shape[0]):
            for c in range(4):
                e = np.zeros_like(tf); e[j, c] = 1
                dk = oracle.render_dual(V, tf, cam, W, H, step, model, tf_dir=e)
                assert float((g * dk["image_dot"]).sum()) == pytest.approx(
                    adj["dTF"][j, c], rel=1e-10, abs=1e-12)


def test_adjoint_equals_dual_numbers_per_voxel_on_tiny_grid():
    rng = np.random.default_rng(13)
    V = rng.uniform(0, 1, (4, 4, 4))
    tf = synth.random_tf(4, rng, 6.0).astype(np.float64)
    W = H = 6
    cam = oracle.camera_from_sphere(-50, 33, 2.2, 60, W, H)
    g = rng.normal(size=(W * H, 4))
    adj = oracle.adjoint(V, tf, cam, W, H, 0.09, EA, g)
    for idx in np.ndindex(V.shape):
        e = np.zeros_like(V); e[idx] = 1
        dk = oracle.render_dual(V, tf, cam, W, H, 0.09, EA, V_dir=e)
        assert float((g * dk["image_dot"]).sum()) == pytest.approx(adj["dV"][idx], rel=1e-10, abs=1e-13)


@pytest.mark.parametrize("model", [AO, EA])
def test_adjoint_matches_central_finite_differences(model):
    rng, V, tf, cam, W, H, step, g = _problem(model, seed=14)
    adj = oracle.adjoint(V, tf, cam, W, H, step, model, g)

    def loss(Vx, tfx, camx, sx):
        return float((g * oracle.render(Vx, tfx, camx, W, H, sx, model)["image"]).sum())

    for _ in range(3):
        Vd = rng.normal(size=V.shape)
        tfd = rng.normal(size=tf.shape) if model == EA else np.zeros(1)
        cd = rng.normal(size=12)
        sd = float(rng.normal())
        eps = 1e-6
        tp = tf + eps * tfd if model == EA else None
        tm = tf - eps * tfd if model == EA else None
        fd = (loss(V + eps * Vd, tp, cam + eps * cd, step + eps * sd) -
              loss(V - eps * Vd, tm, cam - eps * cd, step - eps * sd)) / (2 * eps)
        an = float((adj["dV"] * Vd).sum() + (adj["dcam"] * cd).sum() + adj["dstep"] * sd)
        if model == EA:
            an += float((adj["dTF"] * tfd).sum())
        assert fd == pytest.approx(an, rel=1e-6)


def test_slab_closed_form_gradients():
    # constant density: grad d = 0, so the step derivative is the Beer-Lambert
    # term alone: d alpha / d dt = N d e^{-N dt d}; voxel gradients sum to
    # N dt e^{-N dt d} (trilinear weights sum to one).
    n, W, d0, step = 9, 5, 0.7, 0.09
    V = _cube(n, d0)
    cam = oracle.camera_from_sphere(31, 12, 2.5, 30, W, W)
    pix = [2 * W + 2]
    out = oracle.render(V, None, cam, W, W, step, AO, pix=pix)
    N = int(out["nsamp"][0])
    adj = oracle.adjoint(V, None, cam, W, W, step, AO, np.ones((1, 1)), pix=pix)
    ex = math.exp(-N * step * d0)
    assert adj["dstep"] == pytest.approx(N * d0 * ex, rel=1e-12)
    assert adj["dV"].sum() == pytest.approx(N * step * ex, rel=1e-12)
    assert np.all(adj["dV"] >= 0)
    # EA with a density sitting inside one TF segment: only that segment's two
    # knots receive gradient, split (1-phi, phi)
    R = 6
    dseg = 0.5 / (R - 1) + 2.0 / (R - 1)          # phi = 0.5 in segment 2
    rng = np.random.default_rng(15)
    tf = synth.random_tf(R, rng, 4.0).astype(np.float64)
    out = oracle.render(_cube(n, dseg), tf, cam, W, W, step, EA, pix=pix)
    gch = np.array([[0.3, -0.2, 0.5, 0.7]])
    adj = oracle.adjoint(_cube(n, dseg), tf, cam, W, W, step, EA, gch, pix=pix)
    nz = np.nonzero(np.abs(adj["dTF"]).sum(1))[0]
    assert list(nz) == [2, 3]
    assert np.allclose(adj["dTF"][2], adj["dTF"][3], rtol=1e-12)


def test_absorption_only_is_a_linear_projector_dot_product():
    # Sec. 5.3: absorption-only rendering is linear tomography.  Optical depth
    # -log(1 - alpha) = dt * P_w V is linear in V, and the adjoint at V = 0
    # (T_N = 1) must be the transpose: <P_w V', W> = <V', P_w^T W>.
    rng = np.random.default_rng(16)
    n = (7, 6, 8)
    W_, H_ = 11, 10
    cam = oracle.camera_from_sphere(144, -21, 2.4, 55, W_, H_)
    step = 0.061
    Vp = rng.uniform(0, 1, n)
    Wt = rng.normal(size=(W_ * H_, 1))
    depth = -np.log1p(-oracle.render(Vp, None, cam, W_, H_, step, AO)["image"])
    adj0 = oracle.adjoint(np.zeros(n), None, cam, W_, H_, step, AO, Wt)
    assert float((depth * Wt).sum()) == pytest.approx(float((Vp * adj0["dV"]).sum()), rel=1e-12)
    # at any V the gradient is the backprojection of (g * T_N) (footnote form)
    V = rng.uniform(0, 1, n)
    out = oracle.render(V, None, cam, W_, H_, step, AO)
    adjV = oracle.adjoint(V, None, cam, W_, H_, step, AO, Wt)
    adjB = oracle.adjoint(np.zeros(n), None, cam, W_, H_, step, AO, Wt * out["trans"][:, None])
    assert np.allclose(adjV["dV"], adjB["dV"], rtol=1e-12, atol=1e-14)


def test_alpha_form_inversion_degrades_when_nearly_opaque():
    # Sec. 4.4: inversion needs alpha < 1.  With a huge optical depth the
    # paper's alpha-form loses T^(i) to cancellation while the stored tape and
    # segment checkpointing stay exact.
    n, W, step = 9, 5, 0.05
    V = _cube(n, 60.0)                           # optical depth ~ 120 through the grid
    cam = oracle.camera_from_sphere(0, 0, 2.5, 20, W, W)
    pix = [2 * W + 2]
    g = np.ones((1, 1))
    ref = oracle.adjoint(V, None, cam, W, W, step, AO, g, variant=oracle.TAPE, pix=pix)
    ck = oracle.adjoint(V, None, cam, W, W, step, AO, g, variant=oracle.CHECKPOINT, pix=pix)
    al = oracle.adjoint(V, None, cam, W, W, step, AO, g, variant=oracle.INV_ALPHA, pix=pix)
    assert np.array_equal(ck["dV"], ref["dV"])
    scale = np.abs(ref["dV"]).max()
    assert scale > 0
    assert np.abs(al["dV"] - ref["dV"]).max() > 0.5 * scale
    # the T-form inversion stays accurate while T_N is representable
    it = oracle.adjoint(V, None, cam, W, W, step, AO, g, variant=oracle.INV_T, pix=pix)
    assert np.abs(it["dV"] - ref["dV"]).max() <= 1e-10 * scale


# ---------------------------------------------------------------------------
# pre-shaded colour volume (Sec. 5.4): (r, g, b, tau) per voxel, interpolated
# per channel, same Beer-Lambert segment and blend
# ---------------------------------------------------------------------------
COLOR = oracle.COLOR


def _shaded(V, tf2):
    """Colour volume of a density grid under an affine (two-knot) TF: shading
    commutes with trilinear interpolation when every density is in [0, 1]."""
    a, b = tf2[0], tf2[1]
    return a[None, None, None, :] + V[..., None] * (b - a)[None, None, None, :]


def _color_problem(seed=31, n=(7, 6, 8), W=10, H=9):
    rng = np.random.default_rng(seed)
    V = rng.uniform(0.0, 1.0, n[::-1])
    tf2 = np.array([[0.9, 0.2, 0.1, 0.5], [0.1, 0.7, 0.8, 6.0]])
    cam = oracle.camera_from_sphere(35, 22, 2.3, 60, W, H)
    step = 0.4 * 2 / (max(n) - 1)
    return rng, V, tf2, cam, W, H, step


def test_colour_volume_of_an_affine_tf_renders_like_the_tf():
    rng, V, tf2, cam, W, H, step = _color_problem()
    CV = _shaded(V, tf2)
    a = oracle.render(V, tf2, cam, W, H, step, EA)
    b = oracle.render(CV, None, cam, W, H, step, COLOR)
    assert (a["nsamp"] > 0).sum() > 20
    assert np.abs(a["image"] - b["image"]).max() < 1e-13
    assert np.array_equal(a["nsamp"], b["nsamp"])
    # the chain rule through the shading: dL/dV = sum_c dL/dCV_c * (b - a)_c,
    # camera and step gradients identical
    g = rng.normal(size=a["image"].shape)
    ga = oracle.adjoint(V, tf2, cam, W, H, step, EA, g)
    gb = oracle.adjoint(CV, None, cam, W, H, step, COLOR, g)
    assert gb["dV"].shape == CV.shape
    chained = (gb["dV"] * (tf2[1] - tf2[0])[None, None, None, :]).sum(-1)
    assert np.abs(chained - ga["dV"]).max() <= 1e-12 * np.abs(ga["dV"]).max()
    assert np.allclose(gb["dcam"], ga["dcam"], rtol=1e-11, atol=1e-14)
    assert gb["dstep"] == pytest.approx(ga["dstep"], rel=1e-11)


def test_colour_volume_homogeneous_slab_closed_form():
    n, W = 9, 5
    rgbt = np.array([0.3, 0.6, 0.9, 2.5])
    CV = np.broadcast_to(rgbt, (n, n, n, 4)).copy()
    cam = oracle.camera_from_sphere(0, 0, 2.5, 40, W, W)
    step = 0.07
    out = oracle.render(CV, None, cam, W, W, step, COLOR)
    hit = out["nsamp"] > 0
    N = out["nsamp"][hit]
    a = 1.0 - np.exp(-N * step * rgbt[3])
    assert np.allclose(out["image"][hit, 3], a, rtol=1e-13)
    for c in range(3):
        assert np.allclose(out["image"][hit, c], rgbt[c] * a, rtol=1e-13)


def test_colour_volume_adjoint_variants_dual_numbers_and_finite_differences():
    rng, V, tf2, cam, W, H, step = _color_problem(seed=32)
    CV = rng.uniform(0.0, 1.0, V.shape + (4,)) * np.array([1.0, 1.0, 1.0, 8.0])
    g = rng.normal(size=(W * H, 4))
    ref = oracle.adjoint(CV, None, cam, W, H, step, COLOR, g, variant=oracle.TAPE)
    for var in (oracle.INV_T, oracle.INV_ALPHA, oracle.CHECKPOINT, oracle.RESIDUAL):
        got = oracle.adjoint(CV, None, cam, W, H, step, COLOR, g, variant=var)
        assert np.abs(got["dV"] - ref["dV"]).max() <= 1e-11 * np.abs(ref["dV"]).max(), var
        assert np.allclose(got["dcam"], ref["dcam"], rtol=1e-11, atol=1e-14), var
    # dual numbers along a joint direction
    Vd = rng.normal(size=CV.shape)
    cd = rng.normal(size=12)
    sd = float(rng.normal())
    dual = oracle.render_dual(CV, None, cam, W, H, step, COLOR, Vd, None, cd, sd)
    lhs = float((g * dual["image_dot"]).sum())
    rhs = float((ref["dV"] * Vd).sum() + (ref["dcam"] * cd).sum() + ref["dstep"] * sd)
    assert lhs == pytest.approx(rhs, rel=1e-11)
    # central finite differences

    def loss(C, camx, sx):
        return float((g * oracle.render(C, None, camx, W, H, sx, COLOR)["image"]).sum())

    eps = 1e-6
    fd = (loss(CV + eps * Vd, cam + eps * cd, step + eps * sd) -
          loss(CV - eps * Vd, cam - eps * cd, step - eps * sd)) / (2 * eps)
    assert fd == pytest.approx(rhs, rel=1e-6)


# ---------------------------------------------------------------------------
# density from colour (Sec. 5.4): least-cost random candidates per voxel
# ---------------------------------------------------------------------------
def test_candidate_generator_known_outputs_and_uniformity():
    # first outputs of the SplitMix64 stream of seed 0 (the published generator)
    assert [oracle.splitmix64(0, n) for n in range(3)] == [
        0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, 0x06c45d188009454f]
    u = np.array([(oracle.splitmix64(977, n) >> 40) / 2.0 ** 24 for n in range(40000)])
    assert abs(u.mean() - 0.5) < 0.01 and abs(u.var() - 1.0 / 12.0) < 0.003
    # Kolmogorov-Smirnov distance to U[0, 1)
    s = np.sort(u)
    ks = max(np.max(np.arange(1, len(s) + 1) / len(s) - s), np.max(s - np.arange(len(s)) / len(s)))
    assert ks < 1.63 / np.sqrt(len(s))          # 1% level


def _candidates(seed, iteration, nvox, v, ncand):
    return np.array([(oracle.splitmix64(seed, (iteration * nvox + v) * ncand + k) >> 40)
                     / 2.0 ** 24 for k in range(ncand)])


def test_density_from_colour_colour_term_picks_the_nearest_candidate():
    """TF rgb = (d, 1 - d, 0.5), alpha = beta = 0: the cost is 2 (d - a)^2 for
    a target colour (a, 1 - a, 0.5), so the nearest candidate to a wins."""
    rng = np.random.default_rng(40)
    shape = (3, 4, 5)
    a = rng.uniform(0, 1, shape)
    CV = np.stack([a, 1 - a, np.full(shape, 0.5), rng.uniform(0, 3, shape)], axis=-1)
    tf = np.array([[0.0, 1.0, 0.5, 0.0], [1.0, 0.0, 0.5, 2.0]])
    out = oracle.density_from_color(CV, tf, alpha=0.0, beta=0.0, seed=5, iteration=2, ncand=64)
    nvox = a.size
    for v in range(nvox):
        c = _candidates(5, 2, nvox, v, 64)
        k = int(np.argmin(np.abs(c - a.flat[v])))
        assert out["index"].flat[v] == k and out["d"].flat[v] == c[k]
        assert out["cost"].flat[v] == pytest.approx(2 * (c[k] - a.flat[v]) ** 2, abs=1e-15)


def test_density_from_colour_extinction_term_picks_the_nearest_candidate():
    """Constant TF colour and tau(d) = 1 + 9 d: alpha log(1 + |tau_T - tau(d)|)
    grows with |d - (tau_T - 1)/9|, so the nearest candidate to that wins."""
    rng = np.random.default_rng(41)
    shape = (2, 3, 4)
    ds = rng.uniform(0, 1, shape)
    CV = np.stack([np.full(shape, 0.2), np.full(shape, 0.4), np.full(shape, 0.6), 1 + 9 * ds],
                  axis=-1)
    tf = np.array([[0.2, 0.4, 0.6, 1.0], [0.2, 0.4, 0.6, 10.0]])
    out = oracle.density_from_color(CV, tf, alpha=0.5, beta=0.0, seed=9, iteration=0, ncand=48)
    for v in range(ds.size):
        c = _candidates(9, 0, ds.size, v, 48)
        k = int(np.argmin(np.abs(c - ds.flat[v])))
        assert out["index"].flat[v] == k
        assert out["cost"].flat[v] == pytest.approx(
            0.5 * np.log1p(9 * abs(c[k] - ds.flat[v])), rel=1e-12, abs=1e-15)


def test_density_from_colour_neighbour_term_picks_the_candidate_nearest_the_mean():
    """Constant TF: beta sum_i (d - d_i)^2 = beta (n (d - m)^2 + const) over the
    n neighbours present (6 inside, 3 at a corner), m their mean."""
    rng = np.random.default_rng(42)
    shape = (4, 3, 5)
    prev = rng.uniform(0, 1, shape)
    CV = np.tile(np.array([0.3, 0.3, 0.3, 1.0]), shape + (1,))
    tf = np.array([[0.3, 0.3, 0.3, 1.0], [0.3, 0.3, 0.3, 1.0]])
    out = oracle.density_from_color(CV, tf, prev, alpha=1.0, beta=2.0, seed=3, iteration=1,
                                    ncand=32)
    nz, ny, nx = shape
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                nb = [prev[zz, yy, xx] for zz, yy, xx in
                      ((z, y, x - 1), (z, y, x + 1), (z, y - 1, x), (z, y + 1, x),
                       (z - 1, y, x), (z + 1, y, x))
                      if 0 <= zz < nz and 0 <= yy < ny and 0 <= xx < nx]
                v = (z * ny + y) * nx + x
                c = _candidates(3, 1, prev.size, v, 32)
                k = int(np.argmin(np.abs(c - np.mean(nb))))
                assert out["index"][z, y, x] == k, (z, y, x, len(nb))
                assert out["cost"][z, y, x] == pytest.approx(
                    2.0 * sum((c[k] - q) ** 2 for q in nb), rel=1e-12)


def test_density_from_colour_voxel_selection_and_candidate_listing():
    rng = np.random.default_rng(43)
    shape = (3, 5, 4)
    CV = rng.uniform(0, 1, shape + (4,)) * np.array([1, 1, 1, 6.0])
    tf = rng.uniform(0, 1, (7, 4)) * np.array([1, 1, 1, 6.0])
    prev = rng.uniform(0, 1, shape)
    full = oracle.density_from_color(CV, tf, prev, alpha=0.3, beta=0.7, seed=11, iteration=4,
                                     ncand=20)
    sel = np.array([0, 7, 33, 59, 21])
    part = oracle.density_from_color(CV, tf, prev, alpha=0.3, beta=0.7, seed=11, iteration=4,
                                     ncand=20, voxels=sel, all_costs=True)
    assert np.array_equal(part["d"], full["d"].ravel()[sel])
    assert np.array_equal(part["index"], full["index"].ravel()[sel])
    for q, v in enumerate(sel):
        assert np.array_equal(part["cands"][q], _candidates(11, 4, prev.size, v, 20))
        assert part["costs"][q].min() == part["cost"][q]
        assert part["costs"][q][part["index"][q]] == part["cost"][q]


# ---------------------------------------------------------------------------
# losses, priors and optimiser of the reconstruction loop (Sec. 5.1-5.3)
# ---------------------------------------------------------------------------
from oracle import losses as OL


def _fd(f, x, h=1e-6):
    g = np.zeros_like(x)
    it = np.nditer(x, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        xp = x.copy(); xp[i] += h
        xm = x.copy(); xm[i] -= h
        g[i] = (f(xp) - f(xm)) / (2 * h)
    return g


def test_l1_loss_and_seed_by_hand():
    loss, g = OL.l1_loss_and_seed([0.5, 0.2, 0.7], [0.25, 0.2, 1.0], 0.5)
    assert loss == pytest.approx(0.5 * (0.25 + 0.0 + 0.3))
    assert list(g) == [0.5, 0.0, -0.5]


def test_tf_prior_closed_forms_and_finite_differences():
    R = 9
    lam = 0.4
    T = np.tile(np.array([0.1, 0.5, 0.9, 3.0]), (R, 1))
    loss, g = OL.tf_prior(T, lam)
    assert loss == 0.0 and not g.any()
    b = np.array([0.1, -0.05, 0.02, 0.5])
    T = np.array([0.0, 0.3, 0.6, 1.0]) + np.arange(R)[:, None] * b
    loss, g = OL.tf_prior(T, lam)
    assert loss == pytest.approx(lam * (b ** 2).sum() / 4.0, rel=1e-12)
    assert np.abs(g[1:-1]).max() < 1e-15                     # second differences vanish
    assert np.allclose(g[0], -2 * lam * b / (4 * (R - 1))) and np.allclose(g[-1], -g[0])
    T = np.random.default_rng(60).normal(size=(R, 4))
    assert np.allclose(OL.tf_prior(T, lam)[1], _fd(lambda t: OL.tf_prior(t, lam)[0], T),
                       atol=1e-8)


def test_volume_prior_closed_forms_and_finite_differences():
    lam = 0.5
    nz, ny, nx = 4, 5, 6
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    V = 0.3 + 0.2 * x
    loss, g = OL.volume_prior(V, lam)
    pairs = (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
    assert loss == pytest.approx(lam * (nx - 1) * ny * nz * 0.04 / pairs, rel=1e-12)
    assert np.abs(g[:, :, 1:-1]).max() < 1e-15              # affine: zero inside
    V = np.random.default_rng(61).normal(size=(3, 4, 5))
    assert np.allclose(OL.volume_prior(V, lam)[1], _fd(lambda v: OL.volume_prior(v, lam)[0], V),
                       atol=1e-8)


def test_opacity_entropy_closed_forms_invariance_and_finite_differences():
    N = 37
    H, g = OL.opacity_entropy(np.full(N, 0.3))
    assert H == pytest.approx(1.0, rel=1e-14)                 # uniform: -log2(1/N)/log2 N
    assert np.abs(g).max() < 1e-15                             # the uniform point is stationary
    one = np.zeros(N); one[5] = 0.7
    assert OL.opacity_entropy(one)[0] == 0.0                   # one-hot: 1 log 1 = 0
    two = np.zeros(N); two[[3, 9]] = 0.2
    assert OL.opacity_entropy(two)[0] == pytest.approx(1.0 / np.log2(N), rel=1e-14)  # 1 bit
    x = np.random.default_rng(62).uniform(0.05, 1.0, (5, 7))
    H, g = OL.opacity_entropy(x)
    assert 0.0 < H < 1.0                                       # between one-hot and uniform
    assert OL.opacity_entropy(3.0 * x)[0] == pytest.approx(H, rel=1e-13)   # scale-free
    assert abs((x * g).sum()) < 1e-12                          # Euler: degree-0 homogeneous
    assert np.allclose(g, _fd(lambda a: OL.opacity_entropy(a)[0], x), atol=1e-8)


def test_adam_first_step_and_clamp():
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    x0 = np.array([0.2, 0.4, 0.6, 0.8])
    x, m, v = OL.adam_step(x0[:3], g[:3], np.zeros(3), np.zeros(3), 1, lr=0.1, eps=0.0)
    # t = 1: bias-corrected moments are g and g^2, the step is lr sign(g)
    assert np.allclose(x, x0[:3] - 0.1 * np.sign(g[:3]), rtol=1e-14)
    x, m, v = OL.adam_step(x0, g, np.zeros(4), np.zeros(4), 1, lr=0.1)
    assert x[3] == x0[3]                      # no gradient, no move
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    x, _, _ = OL.adam_step(x0, g, np.zeros(4), np.zeros(4), 1, lr=0.5, eps=1e-8, lo=0.0, hi=1.0)
    assert x.min() >= 0.0 and x.max() <= 1.0 and x[0] == 0.0
    assert x[1] == pytest.approx(0.9, rel=1e-8)


def test_resample_reproduces_affine_fields_and_matches_trilinear():
    nz, ny, nx = 5, 4, 6
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    V = 0.1 + 0.2 * x - 0.3 * y + 0.05 * z
    out = OL.resample(V, (9, 7, 11))
    Z, Y, X = np.meshgrid(np.arange(9) * 4 / 8, np.arange(7) * 3 / 6, np.arange(11) * 5 / 10,
                          indexing="ij")
    assert np.allclose(out, 0.1 + 0.2 * X - 0.3 * Y + 0.05 * Z, atol=1e-14)
    assert np.allclose(OL.resample(V, V.shape), V, rtol=1e-15, atol=1e-15)
    # random field: against the renderer oracle's trilinear at the same points
    W = np.random.default_rng(63).normal(size=(5, 4, 6))
    out = OL.resample(W, (8, 9, 7))
    h = 2.0 / (6 - 1)
    bmin = -0.5 * (np.array([6, 4, 5]) - 1) * h
    for (k, j, i) in [(0, 0, 0), (7, 8, 6), (3, 4, 2), (5, 1, 6), (2, 7, 3)]:
        q = np.array([i * 5 / 6, j * 3 / 8, k * 4 / 7])       # input grid units (x, y, z)
        assert out[k, j, i] == pytest.approx(oracle.trilinear(W, bmin + q * h), abs=1e-12)


def test_kink_distances_match_a_recomputation_on_an_affine_grid():
    """oracle.kinks (the parity harness's mask of non-differentiable points)
    against numpy: sample positions from trace_ray (pinned above), the density
    of an affine grid in closed form, the distance of each sample to the
    nearest interior cell face (faces 1..n-2 of each axis) and of d (R-1) to
    the nearest TF knot 0..R-1; rays that miss report 1e30."""
    n, R = 9, 6
    h, bmin = 2.0 / (n - 1), -1.0
    c0, c = 0.5, np.array([0.2, 0.1, -0.15])            # d = c0 + c . x, inside [0, 1]
    ax = bmin + h * np.arange(n)
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    V = c0 + c[0] * X + c[1] * Y + c[2] * Z
    tf = synth.random_tf(R, np.random.default_rng(2), 5.0)
    W, H, step = 16, 12, 0.37 * h
    cam = oracle.camera_from_sphere(20.0, 15.0, 2.5, 50.0, W, H)
    face, knot = oracle.kinks(V, tf, cam, W, H, step, oracle.EA)
    hits = 0
    for p in range(W * H):
        tr = oracle.trace_ray(V, tf, cam, W, H, p % W, p // W, step, oracle.EA)
        if tr["N"] <= 0:
            assert face[p] == 1e30 and knot[p] == 1e30
            continue
        hits += 1
        x = tr["x"]
        q = (x - bmin) / h
        k = np.round(q)
        inner = (k >= 1) & (k <= n - 2)
        fmin = np.where(inner, np.abs(q - k), 1e30).min()
        u = (c0 + x @ c) * (R - 1)
        kmin = np.abs(u - np.round(u)).min()
        assert abs(face[p] - fmin) <= 1e-9, (p, face[p], fmin)
        assert abs(knot[p] - kmin) <= 1e-9, (p, knot[p], kmin)
    assert hits > W * H // 4
