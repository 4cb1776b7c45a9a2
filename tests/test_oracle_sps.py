"""Pins of the oracle's plain and preconditioned SPS iterations (CPU only):
monotone decrease, brute-force Newton on an 8x8 problem, the shared
minimiser of every preconditioned variant, and the ideal preconditioner."""

import numpy as np
import pytest

import oracle
from oracle import model, precond, projector as P, sps, penalty as pen
from workloads import configs as C
from workloads import phantoms as ph


def _monotone(phi, rel=1e-12):
    return bool(np.all(np.diff(phi) <= rel * abs(phi[0])))


def test_plain_sps_monotone_c1():
    wl = C.make_c1()
    prob = oracle.OracleProblem.from_workload(wl)
    x, phi = sps.sps_plain(prob, 50)
    assert _monotone(phi)
    assert phi[-1] < 0.01 * phi[0]


def test_plain_sps_monotone_huber_with_clamp():
    wl = C.make_small_fan(n=32, views=40, bins=64, penalty="huber")
    prob = oracle.OracleProblem.from_workload(wl)
    x, phi = sps.sps_plain(prob, 30, clamp=True)
    assert _monotone(phi) and np.all(x >= 0)


def test_plain_sps_monotone_mbmd():
    wl = C.make_small_mbmd(n=16, views=20, bins=32, n_mat=3, n_energy_step=10)
    prob = oracle.OracleProblem.from_workload(wl)
    x, phi = sps.sps_plain(prob, 20)
    assert _monotone(phi)


def _newton_problem(beta=30.0):
    """8x8 parallel-beam single-energy problem with mild attenuation."""
    rng = np.random.default_rng(11)
    g = C.geometry("parallel", 8, 8, 1.0, 1.0, 12, np.pi, 12, 1.0)
    ell = [(0.0, 0.0, 3.6, 3.0, 0.4, 0.05), (1.0, -0.5, 1.2, 1.0, 0.0, 0.04)]
    xt = ph.pixelise(ell, 8, 8, 1.0, 1.0)
    ybar = 1e4 * np.exp(-ph.line_integrals(ell, g))
    y = rng.poisson(ybar).astype(float)[None]
    w = 1.0 / np.maximum(y, 1.0)
    prob = oracle.OracleProblem(g, np.ones((1, 1)), np.array([[1e4]]), y, w,
                                dict(kind="quadratic", beta=np.array([[beta]]), delta=0.0))
    return prob, xt


def _newton(prob, iters=40):
    """Brute-force Newton on the exact objective with the dense matrix A."""
    A = P.dense_matrix(prob.geom)
    I0 = prob.S[0, 0]
    y, w = prob.y[0].ravel(), prob.w[0].ravel()
    N = A.shape[1]
    G = np.zeros((N, N))
    for j in range(N):
        e = np.zeros((1, 8, 8))
        e.flat[j] = 1.0
        G[:, j] = pen.hessian_apply(prob, e).ravel()
    x = np.zeros(N)
    for _ in range(iters):
        t = np.exp(-A @ x)
        r = w * (I0 * t - y)
        g = A.T @ (-I0 * t * r) + G @ x
        h2 = w * I0 * I0 * t * t + I0 * t * r
        H = A.T @ (h2[:, None] * A) + G
        x = x - np.linalg.solve(H, g)
    return x.reshape(1, 8, 8), H, np.linalg.norm(g)


def test_newton_reference_and_gradient():
    prob, _ = _newton_problem()
    xhat, H, gnorm = _newton(prob)
    assert gnorm < 1e-8
    assert np.linalg.eigvalsh(H).min() > 0.0          # a strict local minimum
    np.testing.assert_allclose(model.gradient(prob, xhat), 0.0, atol=1e-7)


@pytest.mark.parametrize("kind", [None, "blockdiag", "fourier", "haar", "daub4"])
def test_every_variant_converges_to_the_newton_minimiser(kind):
    """Any invertible M leaves the minimiser unchanged; all iterations are
    monotone and approach the Newton x_hat (beta = 3000: condition ~50, so
    plain SPS gets there too)."""
    prob, _ = _newton_problem(3000.0)
    xhat, _, _ = _newton(prob)
    if kind is None:
        x, phi = sps.sps_plain(prob, 1500)
    else:
        tab = precond.build(prob, kind)
        x, phi, _ = sps.sps_precond(prob, tab, 1500)
    assert _monotone(phi)
    assert np.linalg.norm(x - xhat) / np.linalg.norm(xhat) < 1e-6


def test_preconditioning_speeds_up_convergence():
    """At condition ~4e3 the preconditioned forms reach x_hat, plain SPS does not."""
    prob, _ = _newton_problem(30.0)
    xhat, _, _ = _newton(prob)
    rel = lambda x: np.linalg.norm(x - xhat) / np.linalg.norm(xhat)
    xp, _ = sps.sps_plain(prob, 1500, trace=False)
    assert rel(xp) > 1e-2
    for kind in ("blockdiag", "fourier", "haar", "daub4"):
        x, _, _ = sps.sps_precond(prob, precond.build(prob, kind), 1500, trace=False)
        assert rel(x) < 1e-5, kind


def test_ideal_preconditioner_whitens_the_hessian():
    """eq:preconditionerEigenBasis: M = U^T Lambda^-1/2 U gives M^T H M = I."""
    prob, _ = _newton_problem()
    _, H, _ = _newton(prob)
    lam, V = np.linalg.eigh(H)            # H = V diag(lam) V^T, i.e. U_H = V^T
    M = V @ np.diag(lam ** -0.5) @ V.T
    np.testing.assert_allclose(M.T @ H @ M, np.eye(H.shape[0]), atol=1e-10)
    np.testing.assert_allclose(M, M.T, atol=1e-12)


def test_identity_geometry_truth_is_a_fixed_point():
    """Projection-domain decomposition, noise-free: the true line integrals
    are stationary, and the per-ray step keeps them."""
    wl = C.make_c3(noise=False, n_views=4, n_bins=6)
    prob = oracle.OracleProblem.from_workload(wl)
    tab = precond.build(prob, "blockdiag")
    x, _ = sps.precond_step(prob, wl.x_true, tab)
    np.testing.assert_allclose(x, wl.x_true, rtol=1e-9, atol=1e-9)


def test_identity_geometry_blockdiag_monotone_and_per_ray():
    wl = C.make_c3(noise=True, n_views=5, n_bins=8)
    prob = oracle.OracleProblem.from_workload(wl)
    tab = precond.build(prob, "blockdiag")
    x, phi, alphas = sps.sps_precond(prob, tab, 30)
    assert _monotone(phi)
    assert np.ndim(alphas[0]) == 2          # one step size per ray


def test_unmodified_fourier_monotone():
    wl = C.make_small_fan(n=32, views=40, bins=64, penalty="quadratic")
    prob = oracle.OracleProblem.from_workload(wl)
    tab = precond.build(prob, "fourier", modified=False)
    x, phi, _ = sps.sps_precond(prob, tab, 20)
    assert _monotone(phi)


def test_mbmd_preconditioned_variants_monotone():
    wl = C.make_small_mbmd(n=16, views=20, bins=32, n_mat=3, n_energy_step=10)
    prob = oracle.OracleProblem.from_workload(wl)
    for kind in ("blockdiag", "fourier", "haar"):
        x, phi, _ = sps.sps_precond(prob, precond.build(prob, kind), 15)
        assert _monotone(phi), kind
