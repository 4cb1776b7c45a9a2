"""Pins of the oracle's Daubechies-4 wavelet transform and of the wavelet
preconditioner built on it (CPU only)."""

import numpy as np
import pytest

import oracle
from oracle import daub, precond
from workloads import configs as C


def test_filter_is_the_four_tap_daubechies_filter():
    """The four equations that define it (sum sqrt 2, unit norm, orthogonal to
    its shift by two, two vanishing moments of the high-pass filter), which
    fix h up to reversal, and its orientation (largest taps first)."""
    h, g = daub.H, daub.G
    k = np.arange(4)
    np.testing.assert_allclose(h.sum(), np.sqrt(2.0), rtol=1e-15)
    np.testing.assert_allclose(np.dot(h, h), 1.0, rtol=1e-15)
    np.testing.assert_allclose(h[0] * h[2] + h[1] * h[3], 0.0, atol=1e-16)
    np.testing.assert_allclose(g.sum(), 0.0, atol=1e-15)
    np.testing.assert_allclose(np.dot(k, g), 0.0, atol=1e-15)
    assert h[1] > h[0] > 0 and h[3] < 0
    np.testing.assert_allclose(g, [(-1) ** i * h[3 - i] for i in range(4)], rtol=1e-15)


@pytest.mark.parametrize("m", [2, 4, 8, 16, 64])
def test_analysis_matrix_is_orthogonal(m):
    W = daub.analysis_matrix(m)
    np.testing.assert_allclose(W @ W.T, np.eye(m), atol=1e-14)


def test_orthonormal_and_round_trip():
    n = 8
    U = np.stack([daub.forward(e.reshape(n, n)).ravel() for e in np.eye(n * n)], 1)
    np.testing.assert_allclose(U @ U.T, np.eye(n * n), atol=1e-13)
    x = np.random.default_rng(1).normal(size=(3, 32, 32))
    np.testing.assert_allclose(daub.inverse(daub.forward(x)), x, atol=1e-13)
    np.testing.assert_allclose(np.linalg.norm(daub.forward(x)), np.linalg.norm(x), rtol=1e-13)


def test_constant_image_and_test_function():
    n = 16
    c = daub.forward(np.full((n, n), 3.0))
    assert abs(c[0, 0] - 3.0 * n) < 1e-12
    c[0, 0] = 0.0
    assert np.abs(c).max() < 1e-12
    dx = daub.inverse(np.ones((n, n)))
    np.testing.assert_allclose(daub.forward(dx), 1.0, atol=1e-12)       # U Delta x = 1


def test_two_vanishing_moments_on_a_ramp():
    """An image linear in x and constant in y: every first-level detail
    vanishes except the last row-detail column, where the periodisation
    wraps (Haar, with one vanishing moment, leaves them all nonzero)."""
    n = 32
    img = np.tile(np.arange(n, dtype=float), (n, 1))
    c = daub.forward(img)
    assert np.abs(c[n // 2:, :]).max() < 1e-10                   # column details
    assert np.abs(c[:n // 2, n // 2:n - 1]).max() < 1e-10        # row details but the wrapped one
    assert np.abs(c[:n // 2, n - 1]).min() > 1.0


def _toy(n):
    wl = C.make_small_fan(n=n, views=12, bins=2 * n, penalty="quadratic")
    return oracle.OracleProblem.from_workload(wl)


def _dense(op, shape):
    N = int(np.prod(shape))
    return np.stack([op(e.reshape(shape)).ravel() for e in np.eye(N)], 1)


def test_exact_for_a_daubechies_diagonal_hessian():
    """H = U^T Lambda U: the test function U^T 1 reads Lambda exactly and M
    whitens H."""
    n = 8
    prob = _toy(n)
    lam = np.random.default_rng(2).uniform(0.5, 4.0, size=(n, n))
    hop = lambda v: daub.inverse(lam * daub.forward(v[0]))[None]
    t = precond.build(prob, "daub4", modified=False, hop=hop, eps=1e-12)
    np.testing.assert_allclose(t["P"][..., 0, 0], lam ** -0.5, rtol=1e-12)
    M = _dense(lambda v: precond.apply_M(t, v), (1, n, n))
    H = _dense(hop, (1, n, n))
    np.testing.assert_allclose(M.T @ H @ M, np.eye(n * n), atol=1e-12)
