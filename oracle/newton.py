"""Exact minimiser of the objective by Newton's method with the dense Hessian (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The estimator of Methods, "Generalized Models for Data Acquisition and
Estimation" (eq:mapEstimator) is x_hat = argmin Phi(x), Phi = L + R.  The SPS
iterations and every preconditioned form of "Preconditioned Optimization"
converge to the same x_hat (any invertible M leaves the minimiser unchanged),
so x_hat is the reference that iterates of any method are compared with at
convergence, and that time-to-RMSE is measured against.

Hessian of the data term.  Per ray i with material line integrals l_i
(l_ik = (A x_k)_i), energy line integrals l_iE = sum_k Q_Ek l_ik, t_iE =
exp(-l_iE), mean ybar_ic = sum_E S_cE t_iE and residual r_ic = ybar_ic - y_ic
(no projection-domain blur):
    dybar_ic / dl_ik            = J_ic,k = -sum_E S_cE Q_Ek t_iE,
    d2ybar_ic / dl_ik dl_ik'    = sum_E S_cE Q_Ek Q_Ek' t_iE,
    d2L_i / dl_ik dl_ik'        = h_i[k,k'] = sum_c w_ic (J_ic,k J_ic,k' + r_ic d2ybar_ic/dl_ik dl_ik'),
and the Hessian of L in x is block (k, k') = A^T D{h[k,k']} A.  The quadratic
penalty R = 1/2 x^T (beta (x) Gamma) x adds beta (x) Gamma.  The objective is
locally, not globally, convex (h can be indefinite where ybar < y / 2), so the
Newton steps are damped by backtracking on Phi and the Hessian at the result
is checked positive definite by the tests.

Dense matrices: for small problems only (A is [N_i, N_j], the Hessian
[N_k N_j, N_k N_j]).
"""

from __future__ import annotations

import numpy as np

from . import model, projector
from . import penalty as pen


def ray_hessian(prob, x):
    """h [N_k, N_k, N_i]: the per-ray Hessian of the data term in the material
    line integrals at x."""
    if prob.blur is not None:
        raise ValueError("the Newton reference is written for problems without a blur")
    l = model.line_integrals(prob, x)
    t = model.transmission(prob, l)                                   # [E, V, B]
    r = model.mean_counts(prob, t) - prob.y                          # [C, V, B]
    J = -np.einsum("ce,ek,evb->ckvb", prob.S, prob.Q, t)              # [C, K, V, B]
    d2 = np.einsum("ce,ek,el,evb->cklvb", prob.S, prob.Q, prob.Q, t)  # [C, K, K, V, B]
    h = (np.einsum("cvb,ckvb,clvb->klvb", prob.w, J, J)
         + np.einsum("cvb,cvb,cklvb->klvb", prob.w, r, d2))
    K = prob.n_mat
    return h.reshape(K, K, -1)


def hessian(prob, x, A=None):
    """The dense Hessian of Phi at x, [N_k N_j, N_k N_j] (quadratic penalty)."""
    if prob.penalty["kind"] != "quadratic":
        raise ValueError("the Newton reference needs the quadratic penalty (twice differentiable)")
    A = projector.dense_matrix(prob.geom) if A is None else A
    K = prob.n_mat
    nj = A.shape[1]
    h = ray_hessian(prob, x)
    H = np.zeros((K * nj, K * nj))
    for k in range(K):
        for kk in range(k, K):
            blk = A.T @ (h[k, kk][:, None] * A)
            H[k * nj:(k + 1) * nj, kk * nj:(kk + 1) * nj] = blk
            H[kk * nj:(kk + 1) * nj, k * nj:(k + 1) * nj] = blk.T
    shape = prob.image_shape
    for col in range(K * nj):
        e = np.zeros(K * nj)
        e[col] = 1.0
        H[:, col] += pen.hessian_apply(prob, e.reshape(shape)).ravel()
    return H


def minimise(prob, x0=None, max_iter=100, gtol=1e-10):
    """Newton from x0 (default 0), damped in the Levenberg-Marquardt way:
    the step solves (H + mu I) s = g with mu = 0 while H is positive definite
    and the step lowers Phi, else mu grows tenfold (from 1e-12 of H's largest
    diagonal entry) until it does; mu shrinks again after a success.  Stops
    when the gradient norm falls below gtol times its value at x0, when no
    damping lowers Phi any more, or after max_iter steps.  Returns (x_hat,
    H at x_hat, final gradient norm, steps taken)."""
    A = projector.dense_matrix(prob.geom)
    x = np.zeros(prob.image_shape) if x0 is None else np.array(x0, dtype=np.float64)
    g = model.gradient(prob, x)
    g0 = np.linalg.norm(g)
    phi = model.objective(prob, x)
    H = hessian(prob, x, A)
    scale = float(np.abs(np.diag(H)).max())
    mu = 0.0
    it = 0
    while it < max_iter and np.linalg.norm(g) > gtol * g0:
        while True:
            try:
                L = np.linalg.cholesky(H + mu * np.eye(H.shape[0]))
                step = np.linalg.solve(L.T, np.linalg.solve(L, g.ravel())).reshape(x.shape)
                xn = x - step
                phin = model.objective(prob, xn)
                if phin <= phi:
                    break
            except np.linalg.LinAlgError:
                pass
            mu = max(10.0 * mu, 1e-12 * scale)
            if mu > 1e3 * scale:
                return x, H, float(np.linalg.norm(g)), it
        x, phi = xn, phin
        mu = mu / 10.0 if mu > 1e-12 * scale else 0.0
        g = model.gradient(prob, x)
        H = hessian(prob, x, A)
        it += 1
    return x, H, float(np.linalg.norm(g)), it
