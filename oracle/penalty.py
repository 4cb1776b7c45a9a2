"""Roughness penalties and their separable surrogates (FP64).

Quadratic penalty: Methods, eq:quadraticSmoothess (single material) and
quadReg_summation (cross material).  R(x) = 1/2 x^T (beta (x) Gamma) x with
Gamma the 4-neighbour graph Laplacian: Gamma_jj = |N_j|, Gamma_jj' = -1 for
j' in N_j; neighbours outside the image are dropped, so |N_j| is 2, 3 or 4.
The double sum over j and j' in N_j of quadReg_summation counts each pair
twice; the Hessian beta^1/2 Gamma beta^1/2 that follows it is used as the
definition here (so R = 1/2 x^T (beta (x) Gamma) x exactly).

Huber penalty (single material, not in the paper):
R = beta sum_{unordered pairs} psi_delta(x_j - x_j'),
psi(t) = t^2/2 for |t| <= delta, delta |t| - delta^2/2 otherwise; it
reduces to the quadratic one as delta -> infinity.

Separable surrogate curvatures (used by SPS, Methods, "The Separable
Parabolic Surrogates Algorithm"): for the quadratic form the row sums of
|beta (x) Gamma|, i.e. sum_k' |beta_kk'| 2|N_j|; for Huber the De Pierro
split of Huber's quadratic majoriser, 2 beta sum_{j' in N_j} omega(x_j-x_j')
with omega(t) = psi'(t)/t.
"""

from __future__ import annotations

import numpy as np


def _diffs(img):
    """Horizontal and vertical neighbour differences of an [ny, nx] image."""
    return img[:, 1:] - img[:, :-1], img[1:, :] - img[:-1, :]


def laplacian(img):
    """Gamma img for one [ny, nx] image (4-neighbour, free boundary)."""
    out = np.zeros_like(img)
    h, v = _diffs(img)
    out[:, 1:] += h
    out[:, :-1] -= h
    out[1:, :] += v
    out[:-1, :] -= v
    return out


def neighbour_count(ny, nx):
    """|N_j| for every pixel."""
    n = np.full((ny, nx), 4.0)
    n[0, :] -= 1
    n[-1, :] -= 1
    n[:, 0] -= 1
    n[:, -1] -= 1
    return n


def huber_psi(t, delta):
    a = np.abs(t)
    return np.where(a <= delta, 0.5 * t * t, delta * a - 0.5 * delta * delta)


def huber_dpsi(t, delta):
    return np.clip(t, -delta, delta)


def huber_omega(t, delta):
    """psi'(t) / t, equal to 1 on |t| <= delta."""
    a = np.abs(t)
    return np.where(a <= delta, 1.0, delta / np.maximum(a, delta))


def value(prob, x):
    P = prob.penalty
    beta = P["beta"]
    if P["kind"] == "huber":
        h, v = _diffs(x[0])
        d = P["delta"]
        return float(beta[0, 0] * (huber_psi(h, d).sum() + huber_psi(v, d).sum()))
    Gx = np.stack([laplacian(xk) for xk in x])
    return 0.5 * float(np.einsum("kl,kyx,lyx->", beta, x, Gx))


def gradient(prob, x):
    """dR/dx: (beta (x) Gamma) x, or beta sum_{j'} psi'(x_j - x_j')."""
    P = prob.penalty
    beta = P["beta"]
    if P["kind"] == "huber":
        h, v = _diffs(x[0])
        dh, dv = huber_dpsi(h, P["delta"]), huber_dpsi(v, P["delta"])
        g = np.zeros_like(x[0])
        g[:, 1:] += dh
        g[:, :-1] -= dh
        g[1:, :] += dv
        g[:-1, :] -= dv
        return beta[0, 0] * g[None]
    Gx = np.stack([laplacian(xk) for xk in x])
    return np.einsum("kl,lyx->kyx", beta, Gx)


def sps_curvature(prob, x):
    """Separable surrogate curvature d_R [N_k, ny, nx] at x."""
    P = prob.penalty
    beta = P["beta"]
    ny, nx = x.shape[1:]
    if P["kind"] == "huber":
        h, v = _diffs(x[0])
        wh, wv = huber_omega(h, P["delta"]), huber_omega(v, P["delta"])
        s = np.zeros((ny, nx))
        s[:, 1:] += wh
        s[:, :-1] += wh
        s[1:, :] += wv
        s[:-1, :] += wv
        return (2.0 * beta[0, 0] * s)[None]
    rows = np.abs(beta).sum(axis=1)
    return rows[:, None, None] * (2.0 * neighbour_count(ny, nx))[None]


def curvature_quadform(prob, x, p):
    """p^T R'' p for the step size: R'' = beta (x) Gamma, or for Huber the
    majoriser curvature beta sum_pairs omega(x_j - x_j') (p_j - p_j')^2."""
    P = prob.penalty
    beta = P["beta"]
    if P["kind"] == "huber":
        h, v = _diffs(x[0])
        ph, pv = _diffs(p[0])
        return float(beta[0, 0] * (np.sum(huber_omega(h, P["delta"]) * ph * ph)
                                   + np.sum(huber_omega(v, P["delta"]) * pv * pv)))
    Gp = np.stack([laplacian(pk) for pk in p])
    return float(np.einsum("kl,kyx,lyx->", beta, p, Gp))


def hessian_apply(prob, p):
    """(beta (x) Gamma) p: the quadratic Hessian, also used for Huber when
    building preconditioners."""
    Gp = np.stack([laplacian(pk) for pk in p])
    return np.einsum("kl,lyx->kyx", prob.penalty["beta"], Gp)
