"""Polyenergetic forward model, WLS objective and its gradient (FP64).

Follows Methods, "Generalized Models for Data Acquisition and Estimation"
(eq:meanModel and eq:mapEstimator) and the one-step MBMD instantiation.
"""

from __future__ import annotations

import numpy as np

from . import projector
from . import penalty as pen


def line_integrals(prob, x):
    """l_k = A x_k for every material k  ->  [N_k, V, B]."""
    return projector.project(prob.geom, x)


def energy_line_integrals(prob, l):
    """l_iE = sum_k Q_Ek l_ik  ->  [N_E, V, B]  (the AA x of eq:meanModel)."""
    return np.einsum("ek,kvb->evb", prob.Q, l)


def transmission(prob, l):
    """t_iE = exp(-l_iE)."""
    return np.exp(-energy_line_integrals(prob, l))


def blur_matrix(prob, c):
    """B_c [B, B] of channel c: entry (b, b + d) = taps[c, d + h] for |d| <= h."""
    taps = prob.blur[c]
    h = (taps.size - 1) // 2
    nb = prob.geom["n_bins"]
    return sum(taps[d + h] * np.eye(nb, k=d) for d in range(-h, h + 1))


def blur(prob, z, transpose=False):
    """B z (or B^T z) for z [N_c, V, B], per channel along each view's bins;
    z itself when the problem has no blur."""
    if prob.blur is None:
        return z
    out = np.empty_like(z)
    for c in range(prob.n_chan):
        Bm = blur_matrix(prob, c)
        out[c] = z[c] @ (Bm if transpose else Bm.T)
    return out


def mean_counts(prob, t):
    """ybar_ic = (B_c sum_E S_cE t_E)_i  (BB exp(-AA x))."""
    return blur(prob, np.einsum("ce,evb->cvb", prob.S, t))


def forward(prob, x):
    """ybar(x) for an image stack x [N_k, ny, nx]."""
    return mean_counts(prob, transmission(prob, line_integrals(prob, x)))


def data_objective(prob, x):
    """L = 1/2 (y - ybar)^T Sigma^-1 (y - ybar) with Sigma^-1 = diag(w)."""
    r = prob.y - forward(prob, x)
    return 0.5 * float(np.sum(prob.w * r * r))


def objective(prob, x):
    """Phi = L + R (eq:mapEstimator)."""
    return data_objective(prob, x) + pen.value(prob, x)


def hdot(prob, t):
    """dL/dl_iE = -t_iE sum_c S_cE [B_c^T W_c (ybar_c - y_c)]_i."""
    ybar = mean_counts(prob, t)
    r = blur(prob, prob.w * (ybar - prob.y), transpose=True)
    return -t * np.einsum("ce,cvb->evb", prob.S, r)


def data_gradient(prob, x):
    """dL/dx_k = A^T (sum_E Q_Ek dL/dl_iE)  (chain rule through AA = Q (x) A)."""
    t = transmission(prob, line_integrals(prob, x))
    u = np.einsum("ek,evb->kvb", prob.Q, hdot(prob, t))
    return projector.backproject(prob.geom, u)


def gradient(prob, x):
    return data_gradient(prob, x) + pen.gradient(prob, x)


def forward_vjp(prob, x, gbar):
    """Vector-Jacobian product of ybar(x): returns d<gbar, ybar(x)>/dx.

    = A^T [ sum_E Q_Ek (-t_iE) sum_c S_cE (B_c^T gbar_c)_i ], the backward of
    the polyenergetic forward model.
    """
    t = transmission(prob, line_integrals(prob, x))
    gb = blur(prob, gbar, transpose=True)
    s = np.einsum("ek,evb->kvb", prob.Q, -t * np.einsum("ce,cvb->evb", prob.S, gb))
    return projector.backproject(prob.geom, s)
