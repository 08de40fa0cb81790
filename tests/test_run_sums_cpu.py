"""The identity behind the absorption-only cell runs of the kernels: over the
m equally spaced samples of a ray inside one cell, a trilinear interpolant
(and each corner's trilinear weight) sums to m (g(mu) + s2/2 g''), mu the
midpoint, s2 = (m^2 - 1)/12, g'' the second derivative per sample -- checked
here in float64 against the per-sample sums, with the mixed-derivative and
sign bookkeeping the kernels use (run_density_sum, run_weight_sums)."""
import numpy as np


def _weights(f):
    X, Y, Z = (1 - f[0], f[0]), (1 - f[1], f[1]), (1 - f[2], f[2])
    return np.array([X[k & 1] * Y[(k >> 1) & 1] * Z[k >> 2] for k in range(8)])


def _run_density_sum(v, f, m, dq):
    x0, x1, x2, x3 = v[1] - v[0], v[3] - v[2], v[5] - v[4], v[7] - v[6]
    c00, c10, c01, c11 = f[0] * x0 + v[0], f[0] * x1 + v[2], f[0] * x2 + v[4], f[0] * x3 + v[6]
    c0, c1 = f[1] * (c10 - c00) + c00, f[1] * (c11 - c01) + c01
    d = f[2] * (c1 - c0) + c0
    d_xy = f[2] * ((x3 - x2) - (x1 - x0)) + (x1 - x0)
    d_xz = f[1] * ((x3 - x1) - (x2 - x0)) + (x2 - x0)
    d_yz = (c11 - c01) - (c10 - c00)
    curv = dq[0] * dq[1] * d_xy + dq[0] * dq[2] * d_xz + dq[1] * dq[2] * d_yz
    return m * (d + (m * m - 1) / 12.0 * curv)


def _run_weight_sums(f, m, dq):
    s2 = (m * m - 1) / 12.0
    e = {"xy": s2 * dq[0] * dq[1], "xz": s2 * dq[0] * dq[2], "yz": s2 * dq[1] * dq[2]}
    X, Y, Z = (1 - f[0], f[0]), (1 - f[1], f[1]), (1 - f[2], f[2])
    out = []
    for k in range(8):
        cx, cy, cz = k & 1, (k >> 1) & 1, k >> 2
        sg = lambda a, b: 1.0 if a == b else -1.0
        t = (X[cx] * Y[cy] * Z[cz] + sg(cx, cy) * e["xy"] * Z[cz] + sg(cx, cz) * e["xz"] * Y[cy]
             + sg(cy, cz) * e["yz"] * X[cx])
        out.append(m * t)
    return np.array(out)


def test_run_sums_equal_per_sample_sums():
    rng = np.random.default_rng(3)
    for _ in range(3000):
        v = rng.uniform(-1, 1, 8)
        dq = rng.uniform(-0.5, 0.5, 3)
        m = int(rng.integers(1, 40))
        f0 = rng.uniform(0, 1, 3)
        W = np.array([_weights(f0 + j * dq) for j in range(m)])
        mid = f0 + 0.5 * (m - 1) * dq
        assert abs(_run_density_sum(v, mid, m, dq) - (W @ v).sum()) <= 1e-12 * max(1.0, m)
        assert np.abs(_run_weight_sums(mid, m, dq) - W.sum(axis=0)).max() <= 1e-12 * max(1.0, m)


def test_a_dropped_curvature_term_is_caught():
    """Without the second-derivative term the sums are off for m >= 2 on
    oblique rays: the identity test above is not vacuous."""
    rng = np.random.default_rng(4)
    v = rng.uniform(-1, 1, 8)
    dq = np.array([0.3, -0.4, 0.25])
    f0 = np.array([0.1, 0.9, 0.2])
    m = 3
    W = np.array([_weights(f0 + j * dq) for j in range(m)])
    mid = f0 + 0.5 * (m - 1) * dq
    assert abs(m * (_weights(mid) @ v) - (W @ v).sum()) > 1e-3
