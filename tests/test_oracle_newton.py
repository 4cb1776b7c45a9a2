"""Pins of the oracle's Newton minimiser (CPU only): its Hessian against
central differences of the gradient (itself pinned by differences of the
objective), the minimiser's stationarity and positive definiteness, agreement
with the brute-force single-energy Newton, and the SPS iterations reaching it."""

import numpy as np
import pytest

import oracle
from oracle import model, newton, precond, sps
from workloads import configs as C


def _mbmd(n_mat, n=8):
    wl = C.make_small_mbmd(n=n, views=12, bins=16, n_mat=n_mat, n_energy_step=10)
    return oracle.OracleProblem.from_workload(wl), wl


@pytest.mark.parametrize("n_mat", [1, 2, 3])
def test_hessian_matches_differences_of_the_gradient(n_mat):
    """Exact for the data term's second derivatives including the residual
    (non Gauss-Newton) term, and the penalty's beta (x) Gamma."""
    if n_mat == 1:
        wl = C.make_small_fan(n=8, views=12, bins=16, penalty="quadratic")
        prob = oracle.OracleProblem.from_workload(wl)
    else:
        prob, wl = _mbmd(n_mat)
    rng = np.random.default_rng(7 + n_mat)
    x = np.abs(wl.x_true) * rng.uniform(0.5, 1.5, size=wl.x_true.shape)
    H = newton.hessian(prob, x)
    h = 1e-6 * max(1.0, float(np.abs(x).max()))
    N = x.size
    Hfd = np.empty((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = h
        e = e.reshape(x.shape)
        Hfd[:, j] = ((model.gradient(prob, x + e) - model.gradient(prob, x - e)) / (2 * h)).ravel()
    np.testing.assert_allclose(H, Hfd, rtol=1e-5, atol=1e-6 * np.abs(H).max())
    np.testing.assert_allclose(H, H.T, rtol=1e-12, atol=1e-12 * np.abs(H).max())


def test_single_energy_matches_the_brute_force_newton():
    from test_oracle_sps import _newton, _newton_problem
    prob, _ = _newton_problem()
    want, _, _ = _newton(prob)
    got, H, gnorm, _ = newton.minimise(prob)
    np.testing.assert_allclose(got, want, rtol=1e-7, atol=1e-9)
    assert np.linalg.eigvalsh(H).min() > 0.0


@pytest.mark.parametrize("n_mat", [2, 3])
def test_mbmd_minimiser_is_a_strict_local_minimum(n_mat):
    """Newton's x_hat of a small MBMD problem: the gradient vanishes, the
    Hessian is positive definite, no random nearby point is lower, and it is
    lower than what the preconditioned SPS iterations reach in 300 steps."""
    prob, wl = _mbmd(n_mat)
    x0, _, _ = sps.sps_precond(prob, precond.build(prob, "blockdiag"), 200, trace=False)
    xhat, H, gnorm, steps = newton.minimise(prob, x0)
    g0 = np.linalg.norm(model.gradient(prob, np.zeros(prob.image_shape)))
    assert gnorm <= 1e-9 * g0
    assert np.linalg.eigvalsh(H).min() > 0.0
    phi = model.objective(prob, xhat)
    rng = np.random.default_rng(n_mat)
    for _ in range(8):
        d = rng.normal(size=xhat.shape) * 1e-3 * np.abs(xhat).max()
        assert model.objective(prob, xhat + d) > phi
    x, tr, _ = sps.sps_precond(prob, precond.build(prob, "fourier"), 300, trace=True)
    assert phi <= tr[-1]
