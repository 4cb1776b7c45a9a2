"""Plain and preconditioned separable-paraboloidal-surrogate iterations (FP64).

Plain SPS follows Methods, "The Separable Parabolic Surrogates Algorithm",
with these readings of its garbled or silent points:
  * rho (the linear coefficient of the decoupled surrogate) is written there
    with x^(n) where the transmission t^(n) = exp(-AA x^(n)) is meant:
        rho = BB^T Sigma^-1 BB t - D{eta} t - BB^T Sigma^-1 y
            = S^T B^T W (ybar - y) - eta * t ;
  * the surrogate gradient reads AA^T(-D{eta} t^2 - D{rho} t) (the printed
    D{gamma} is a typo for D{eta}); it equals the true gradient at x^(n);
  * the maximum curvature f_c is that of h(l) = eta/2 e^-2l + rho e^-l over
    l >= 0, reached at l = 0:  c = max(2 eta + rho, 0);
  * the surrogate Hessian is D{AA^T D{gamma} c} with gamma = AA 1;
  * x^(0) = 0 and no non-negativity clamp unless asked for.

The preconditioned iteration follows Methods, "Preconditioned
Optimization": the SPS step is taken in x' with x = M x'.  The paper leaves
the x'-space curvature undefined for a mixed-sign AA M; the reading used
here is a unit curvature in x' (the preconditioner is built so that
M^T H M ~ I), i.e. the direction p = -M M^T grad Phi, followed by the exact
minimiser of the 1D majoriser of Phi(x + alpha p) that uses the same
per-ray maximum curvatures c:
    alpha = -g^T p / (sum_iE c_iE q_iE^2 + p^T R'' p),  q = AA p.
For the identity geometry without a penalty the problem separates by ray
and alpha is taken per ray.
"""

from __future__ import annotations

import numpy as np

from . import model, projector
from . import penalty as pen

TINY = 1e-30


def gamma(prob):
    """gamma = AA 1 per (energy, ray): (A 1)_i sum_k Q_Ek."""
    ones = np.ones((1, prob.geom["ny"], prob.geom["nx"]))
    gA = projector.project(prob.geom, ones)[0]
    return gA[None] * prob.Q.sum(axis=1)[:, None, None]


def eta(prob):
    """eta = BB^T Sigma^-1 BB 1 per (energy, ray), BB = B S:
    sum_c S_cE (sum_E' S_cE') [B_c^T W_c B_c 1]_i."""
    row = prob.S.sum(axis=1)                                  # sum_E' S_cE'
    wb = model.blur(prob, prob.w * model.blur(prob, np.ones_like(prob.w)), transpose=True)
    return np.einsum("ce,cvb->evb", prob.S, wb * row[:, None, None])


def ray_terms(prob, l):
    """(t, ybar, rho, hdot, c) at line integrals l [N_k, V, B]."""
    t = model.transmission(prob, l)
    ybar = model.mean_counts(prob, t)
    et = eta(prob)
    rho = np.einsum("ce,cvb->evb", prob.S,
                    model.blur(prob, prob.w * (ybar - prob.y), transpose=True)) - et * t
    hdot = -et * t * t - rho * t
    c = np.maximum(2.0 * et + rho, 0.0)
    return t, ybar, rho, hdot, c


def surrogate_terms(prob, x):
    """SPS gradient and curvature images of the data term at x."""
    l = model.line_integrals(prob, x)
    _, _, _, hdot, c = ray_terms(prob, l)
    u = np.einsum("ek,evb->kvb", prob.Q, hdot)
    v = np.einsum("ek,evb->kvb", prob.Q, gamma(prob) * c)
    return projector.backproject(prob.geom, u), projector.backproject(prob.geom, v)


def sps_plain(prob, n_iter, x0=None, clamp=False, trace=True):
    """n_iter plain SPS updates x <- x - (g + dR)/(d + d_R).  Returns (x, Phi trace)."""
    x = np.zeros(prob.image_shape) if x0 is None else np.array(x0, dtype=np.float64)
    gam = gamma(prob)
    phis = [model.objective(prob, x)] if trace else []
    for _ in range(n_iter):
        l = model.line_integrals(prob, x)
        _, _, _, hdot, c = ray_terms(prob, l)
        u = np.einsum("ek,evb->kvb", prob.Q, hdot)
        v = np.einsum("ek,evb->kvb", prob.Q, gam * c)
        g = projector.backproject(prob.geom, u) + pen.gradient(prob, x)
        d = projector.backproject(prob.geom, v) + pen.sps_curvature(prob, x)
        x = x - g / np.maximum(d, TINY)
        if clamp:
            x = np.maximum(x, 0.0)
        if trace:
            phis.append(model.objective(prob, x))
    return x, np.array(phis)


def _separable_by_ray(prob):
    return prob.geom["kind"] == "identity" and not np.any(prob.penalty["beta"])


def precond_step(prob, x, tables):
    """One preconditioned SPS update; returns (x_new, alpha)."""
    from . import precond
    l = model.line_integrals(prob, x)
    _, _, _, hdot, c = ray_terms(prob, l)
    u = np.einsum("ek,evb->kvb", prob.Q, hdot)
    g = projector.backproject(prob.geom, u) + pen.gradient(prob, x)
    p = -precond.apply_M(tables, precond.apply_Mt(tables, g))
    q = model.line_integrals(prob, p)
    qE = model.energy_line_integrals(prob, q)
    if _separable_by_ray(prob):
        num = -np.sum(g * p, axis=0)                        # per ray (pixel of the sinogram)
        den = np.sum(c * qE * qE, axis=0)
        alpha = np.where(den > 0.0, num / np.where(den > 0.0, den, 1.0), 0.0)
        return x + alpha[None] * p, alpha
    num = -float(np.sum(g * p))
    den = float(np.sum(c * qE * qE)) + pen.curvature_quadform(prob, x, p)
    alpha = num / den if den > 0.0 else 0.0
    return x + alpha * p, alpha


def sps_precond(prob, tables, n_iter, x0=None, trace=True):
    """n_iter preconditioned SPS updates.  Returns (x, Phi trace, alphas)."""
    x = np.zeros(prob.image_shape) if x0 is None else np.array(x0, dtype=np.float64)
    phis = [model.objective(prob, x)] if trace else []
    alphas = []
    for _ in range(n_iter):
        x, a = precond_step(prob, x, tables)
        alphas.append(a)
        if trace:
            phis.append(model.objective(prob, x))
    return x, np.array(phis), alphas
