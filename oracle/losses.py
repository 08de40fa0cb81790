"""FP64 reference of the losses, priors and optimiser of the reconstruction
loop (plain numpy).

TEST INFRASTRUCTURE ONLY: used by the test-suite (and nothing on the product
path).  It shares no code with the HIP library.

What it computes (Weiss & Westermann, arXiv 2107.12672):
  * the L1 image loss of eq. (tf-loss), L1 = 1/(N W H) sum |x - y|, and its
    upstream gradient (sign(x - y) / (N W H), 0 where x = y);
  * the TF smoothing prior of eq. (tf-loss),
    L_prior(T) = 1/(4 (R-1)) sum_c sum_r (T_{c,r+1} - T_{c,r})^2;
  * the same prior on the densities in 3D (Sec. 5.3: "computed on the
    reconstructed volume densities in 3D"), read as the mean over all pairs of
    grid neighbours along x, y and z of the squared difference;
  * the opacity entropy of Sec. 5.1, OE(C) = H(C[:, :, 3]) with H the
    normalised entropy H(x) = -1/log2(N) sum_i p_i log2 p_i,
    p_i = x_i / sum_j x_j (0 log 0 = 0), in [0, 1] -- the paper prints H
    without the minus sign but reports positive entropies, which viewpoint
    selection maximises, so the sign is read as lost -- and its gradient;
    pixels with zero alpha, where the derivative is unbounded, get none;
  * one Adam step (Kingma and Ba 2014, Algorithm 1), with an optional clamp of
    the parameters after the step;
  * trilinear resampling of a vertex grid onto a finer one spanning the same
    box (the multi-resolution schedule of Sec. 5.3).
"""
from __future__ import annotations

import numpy as np


def l1_loss_and_seed(image, target, scale):
    """loss = scale * sum |image - target|, seed = scale * sign(image - target)."""
    x = np.asarray(image, np.float64)
    y = np.asarray(target, np.float64)
    return scale * np.abs(x - y).sum(), scale * np.sign(x - y)


def tf_prior(T, lam):
    """lam * L_prior(T) and its gradient, T [R][4]."""
    T = np.asarray(T, np.float64)
    R = T.shape[0]
    diff = T[1:] - T[:-1]                       # [R-1][4]
    w = lam / (4.0 * (R - 1))
    g = np.zeros_like(T)
    g[1:] += 2.0 * w * diff
    g[:-1] -= 2.0 * w * diff
    return w * (diff ** 2).sum(), g


def volume_prior(V, lam):
    """lam * mean over neighbour pairs of (V_p - V_q)^2 and its gradient,
    V [nz][ny][nx]."""
    V = np.asarray(V, np.float64)
    pairs = 0
    total = 0.0
    g = np.zeros_like(V)
    for ax in range(3):
        n = V.shape[ax]
        if n < 2:
            continue
        hi = np.take(V, np.arange(1, n), axis=ax)
        lo = np.take(V, np.arange(0, n - 1), axis=ax)
        d = hi - lo
        pairs += d.size
        total += (d ** 2).sum()
        gh = np.zeros_like(V)
        idx_hi = [slice(None)] * 3
        idx_lo = [slice(None)] * 3
        idx_hi[ax] = slice(1, n)
        idx_lo[ax] = slice(0, n - 1)
        gh[tuple(idx_hi)] += 2.0 * d
        gh[tuple(idx_lo)] -= 2.0 * d
        g += gh
    w = lam / max(pairs, 1)
    return w * total, w * g


def opacity_entropy(alpha):
    """OE = H(alpha) over the linearised alpha channel (normalised entropy,
    in [0, 1]), and dOE/dalpha."""
    x = np.asarray(alpha, np.float64).ravel()
    N = x.size
    S = x.sum()
    p = x / S
    pos = p > 0
    lp = np.zeros_like(p)
    lp[pos] = np.log2(p[pos])
    H = -(p * lp).sum() / np.log2(N)
    # dH/dx_j = (sum_i p_i log2 p_i - log2 p_j) / (S log2 N), derived from
    # d p_i / d x_j = (delta_ij - p_i) / S; unbounded at p_j = 0 (none given)
    g = np.zeros_like(p)
    g[pos] = ((p * lp).sum() - lp[pos]) / (S * np.log2(N))
    return H, g.reshape(np.shape(alpha))


def adam_step(x, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, lo=None, hi=None):
    """One Adam update at step t >= 1; returns (x, m, v)."""
    x = np.asarray(x, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    x = x - lr * mh / (np.sqrt(vh) + eps)
    if lo is not None or hi is not None:
        x = np.clip(x, -np.inf if lo is None else lo, np.inf if hi is None else hi)
    return x, m, v


def resample(V, shape):
    """Trilinear resampling of the vertex grid V [nz][ny][nx] onto `shape`
    vertices spanning the same box: output vertex i of an axis with n_out
    vertices sits at i (n_in - 1)/(n_out - 1) in input grid units."""
    V = np.asarray(V, np.float64)
    out = V
    for ax in range(3):
        n_in = out.shape[ax]
        n_out = shape[ax]
        q = np.arange(n_out) * ((n_in - 1) / (n_out - 1)) if n_out > 1 else np.zeros(1)
        k = np.clip(np.floor(q).astype(np.int64), 0, max(n_in - 2, 0))
        f = q - k
        a = np.take(out, k, axis=ax)
        b = np.take(out, np.minimum(k + 1, n_in - 1), axis=ax)
        sh = [1, 1, 1]
        sh[ax] = n_out
        out = a + f.reshape(sh) * (b - a)
    return out
