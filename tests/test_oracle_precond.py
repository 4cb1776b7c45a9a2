"""Pins of the oracle's preconditioner builds (CPU only): exact cases where the
approximate eigenbasis is the true one, the Haar transform, the block
inverse square roots, and the Fisher weights from the data and from a
reference image."""

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import haar, precond, sps, model
from workloads import configs as C
from workloads import spectra as SP


def test_haar_2x2_closed_form():
    a, b, c, d = 1.0, 2.0, 5.0, 11.0
    out = haar.forward(np.array([[a, b], [c, d]]))
    want = np.array([[a + b + c + d, a - b + c - d], [a + b - c - d, a - b - c + d]]) / 2.0
    np.testing.assert_allclose(out, want, rtol=1e-15)


def test_haar_orthonormal_and_round_trip():
    n = 8
    U = np.stack([haar.forward(e.reshape(n, n)).ravel() for e in np.eye(n * n)], 1)
    np.testing.assert_allclose(U.T @ U, np.eye(n * n), atol=1e-14)
    x = np.random.default_rng(1).normal(size=(3, 32, 32))
    np.testing.assert_allclose(haar.inverse(haar.forward(x)), x, atol=1e-13)
    np.testing.assert_allclose(np.linalg.norm(haar.forward(x)), np.linalg.norm(x), rtol=1e-14)


def test_haar_constant_image_and_test_function():
    n = 16
    c = haar.forward(np.full((n, n), 3.0))
    assert np.isclose(c[0, 0], 3.0 * n) and np.allclose(c.ravel()[1:], 0.0)
    dx = haar.inverse(np.ones((n, n)))
    np.testing.assert_allclose(haar.forward(dx), 1.0, atol=1e-13)     # U Delta x = 1


def _toy(n=8, K=1):
    g = C.geometry("parallel", n, n, 1.0, 1.0, 4, np.pi, n, 1.0)
    Q = np.ones((1, K))
    S = np.ones((1, 1))
    y = np.ones((1, 4, n))
    return oracle.OracleProblem(g, Q, S, y, y.copy(), dict(kind="quadratic", beta=np.zeros((K, K))))


def _dense(op, shape):
    N = int(np.prod(shape))
    return np.stack([op(e.reshape(shape)).ravel() for e in np.eye(N)], 1)


def test_fourier_exact_for_circulant_hessian():
    """eq:fourierEigenbasis: for a shift-invariant H the impulse response gives
    its eigenvalues exactly, and M^T H M = I."""
    n = 8
    prob = _toy(n)

    def hop(v):
        x = v[0]
        lap = 4 * x - np.roll(x, 1, 0) - np.roll(x, -1, 0) - np.roll(x, 1, 1) - np.roll(x, -1, 1)
        return (2.0 * x + 3.0 * lap + 0.25 * (np.roll(x, 2, 1) + np.roll(x, -2, 1)))[None]

    t = precond.build(prob, "fourier", modified=False, hop=hop, eps=1e-12)
    assert t["n_floored"] == 0
    M = _dense(lambda v: precond.apply_M(t, v), (1, n, n))
    H = _dense(hop, (1, n, n))
    np.testing.assert_allclose(M.T @ H @ M, np.eye(n * n), atol=1e-12)
    # the DC eigenvalue is the sum of the impulse response
    r = hop(np.eye(n * n)[(n // 2) * n + n // 2].reshape(1, n, n))
    lam = precond.fourier_blocks(prob, None, t["M0"], hop=hop)
    assert np.isclose(lam[0, 0, 0, 0].real, r.sum())


def test_cross_material_fourier_exact_for_block_circulant_hessian():
    """Per-frequency N_k x N_k blocks (eq:localImpulseResponse) are exact for
    a Hessian beta (x) C with C circulant and beta a material coupling."""
    n, K = 8, 2
    prob = _toy(n, K)
    beta = np.array([[2.0, 0.7], [0.7, 1.0]])

    def hop(v):
        out = []
        for x in v:
            lap = 4 * x - np.roll(x, 1, 0) - np.roll(x, -1, 0) - np.roll(x, 1, 1) - np.roll(x, -1, 1)
            out.append(x + lap)
        return np.einsum("kl,lyx->kyx", beta, np.stack(out))

    t = precond.build(prob, "fourier", modified=False, hop=hop, eps=1e-12)
    M = _dense(lambda v: precond.apply_M(t, v), (K, n, n))
    H = _dense(hop, (K, n, n))
    np.testing.assert_allclose(M.T @ H @ M, np.eye(K * n * n), atol=1e-11)


def test_haar_exact_for_haar_diagonal_hessian():
    """H = U^T Lambda U: the test function U^T 1 reads Lambda exactly."""
    n = 8
    prob = _toy(n)
    lam = np.random.default_rng(2).uniform(0.5, 4.0, size=(n, n))
    hop = lambda v: haar.inverse(lam * haar.forward(v[0]))[None]
    t = precond.build(prob, "haar", modified=False, hop=hop, eps=1e-12)
    np.testing.assert_allclose(t["P"][..., 0, 0], lam ** -0.5, rtol=1e-12)
    M = _dense(lambda v: precond.apply_M(t, v), (1, n, n))
    H = _dense(hop, (1, n, n))
    np.testing.assert_allclose(M.T @ H @ M, np.eye(n * n), atol=1e-12)


def test_blockdiag_exact_for_identity_geometry():
    """A = I, R = 0: H is block diagonal per ray, so M0^T H M0 = I."""
    wl = C.make_c3(noise=True, n_views=3, n_bins=5)
    prob = oracle.OracleProblem.from_workload(wl)
    W = precond.fisher_weights(prob)
    t = precond.build(prob, "blockdiag", W=W)
    hop = lambda v: precond.hessian_apply(prob, W, v)
    M = _dense(lambda v: precond.apply_M(t, v), prob.image_shape)
    H = _dense(hop, prob.image_shape)
    np.testing.assert_allclose(M.T @ H @ M, np.eye(M.shape[0]), atol=1e-9)


def test_m0_single_material_is_diagonal_formula():
    """eq:diagonalPreconditioner: M0 = D{[F + R] 1}^-1/2 for one material."""
    wl = C.make_small_fan(n=16, views=12, bins=32, penalty="quadratic")
    prob = oracle.OracleProblem.from_workload(wl)
    W = precond.fisher_weights(prob)
    M0 = precond.build_m0(prob, W)
    H1 = precond.hessian_apply(prob, W, np.ones(prob.image_shape))[0]
    np.testing.assert_allclose(M0[..., 0, 0], H1 ** -0.5, rtol=1e-12)


def test_block_inverse_square_root_matches_scipy():
    rng = np.random.default_rng(3)
    A = rng.normal(size=(50, 3, 3))
    B = A @ np.swapaxes(A, 1, 2) + 0.1 * np.eye(3)
    out, nf = precond.block_inv_sqrt(B, floor_rel=1e-12)
    assert nf == 0
    for b, o in zip(B, out):
        np.testing.assert_allclose(o, scipy.linalg.fractional_matrix_power(b, -0.5).real, rtol=1e-10)
        np.testing.assert_allclose(o @ b @ o, np.eye(3), atol=1e-10)
    # an all-zero block maps to zero; a floored block has bounded inverse
    z, _ = precond.block_inv_sqrt(np.zeros((1, 3, 3)), floor_rel=1e-6)
    assert np.all(z == 0.0)
    s, nf = precond.block_inv_sqrt(np.diag([1.0, 1e-9, 0.5])[None], floor_rel=1e-6)
    assert nf == 1 and np.isclose(s[0, 1, 1], 1e3)


def test_single_energy_fisher_weight_is_the_count():
    """D = y / I0 gives W = I0^2 (y/I0)^2 w = y for y >= 1."""
    wl = C.make_small_fan(n=16, views=12, bins=32)
    prob = oracle.OracleProblem.from_workload(wl)
    W = precond.fisher_weights(prob)
    m = wl.y[0] >= 1
    np.testing.assert_allclose(W[0, 0][m], wl.y[0][m], rtol=1e-12)


def test_water_only_estimate_recovers_water_path():
    """Noise-free polyenergetic data of water alone: Gauss-Newton recovers l_w."""
    E = np.arange(20.0, 141.0)
    Q = np.stack([SP.attenuation("water", E), SP.attenuation("iodine", E)], 1)
    S = SP.kvp_switching_sensitivity(E)
    lw = np.linspace(0.0, 120.0, 13).reshape(1, 13)
    ybar = np.einsum("ce,evb->cvb", S, np.exp(-Q[:, 0][:, None, None] * lw[None]))
    g = C.identity_geometry(1, 13)
    prob = oracle.OracleProblem(g, Q, S, ybar, 1.0 / np.maximum(ybar, 1.0),
                                dict(kind="quadratic", beta=np.zeros((2, 2))))
    est = precond.water_only_estimate(prob)
    np.testing.assert_allclose(est, lw, rtol=1e-8, atol=1e-8)


def test_floors_are_reported_and_positive():
    wl = C.make_small_fan(n=32, views=40, bins=64, penalty="quadratic")
    prob = oracle.OracleProblem.from_workload(wl)
    for kind in ("fourier", "haar"):
        t = precond.build(prob, kind)
        assert t["n_floored"] > 0
        eig = np.linalg.eigvalsh(t["P"])
        assert np.all(eig > 0)


def test_reference_weights_equal_data_weights_on_consistent_data():
    """Single energy: with counts y = I0 exp(-A x_ref) exactly, the data-based
    D = y / I0 and the transmission at x_ref are the same, so are the weights."""
    wl = C.make_small_fan(n=16, views=12, bins=32)
    prob = oracle.OracleProblem.from_workload(wl)
    x_ref = np.abs(wl.x_true) + 0.01
    y = prob.S[0, 0] * np.exp(-oracle.projector.project(prob.geom, x_ref))
    prob_c = oracle.OracleProblem(prob.geom, prob.Q, prob.S, y, prob.w, prob.penalty)
    np.testing.assert_allclose(precond.fisher_weights(prob_c, x_ref), precond.fisher_weights(prob_c), rtol=1e-12)


def test_reference_weights_are_the_gram_of_the_jacobian():
    """Three materials, four channels: the weights at x_ref are sum_c w_c J_ck J_cl
    with J the Jacobian of ybar_c with respect to the material line integrals
    l_k, here by central differences of the forward model."""
    wl = C.make_small_mbmd(n=16, views=10, bins=24, n_mat=3, n_energy_step=10)
    prob = oracle.OracleProblem.from_workload(wl)
    x_ref = np.abs(wl.x_true) * 0.5
    W = precond.fisher_weights(prob, x_ref)
    l0 = model.line_integrals(prob, x_ref)
    h = 1e-5
    J = np.empty((prob.n_chan, prob.n_mat) + prob.sino_shape)
    for k in range(prob.n_mat):
        dl = np.zeros_like(l0)
        dl[k] = h
        up = model.mean_counts(prob, model.transmission(prob, l0 + dl))
        dn = model.mean_counts(prob, model.transmission(prob, l0 - dl))
        J[:, k] = (up - dn) / (2 * h)
    W_fd = np.einsum("cvb,ckvb,clvb->klvb", prob.w, J, J)
    np.testing.assert_allclose(W, W_fd, rtol=1e-6, atol=1e-9 * np.abs(W_fd).max())



@pytest.mark.parametrize("kind", ["haar", "daub4"])
@pytest.mark.parametrize("K", [2, 3])
def test_cross_material_wavelet_exact_for_coefficient_block_hessian(kind, K):
    """Cross-material wavelet preconditioner: for a Hessian that is block
    diagonal in the wavelet domain, H = (I (x) U^T) D{B_w} (I (x) U), with a
    different symmetric positive definite N_k x N_k material coupling B_w for
    every coefficient w, the excitation U^T 1 (x) e_k reads column k of every
    B_w at once (U U^T 1 = 1), so the per-coefficient blocks K_w equal B_w and
    M = U^T K^-1/2 U whitens H exactly.  Exciting all materials together
    (U^T 1 in every material), the test function U 1 in place of U^T 1, or
    the inverse transform of the response in place of U, each fails it."""
    n = 8
    wv = precond.WAVELETS[kind]
    prob = _toy(n, K)
    rng = np.random.default_rng(40 + K)
    A = rng.normal(size=(n, n, K, K))
    Bw = A @ np.swapaxes(A, -1, -2) + 0.5 * np.eye(K)             # SPD per coefficient

    def hop(v):
        c = np.stack([wv.forward(vk) for vk in v])                 # [K, n, n] coefficients
        c = np.einsum("yxkl,lyx->kyx", Bw, c)
        return np.stack([wv.inverse(ck) for ck in c])

    t = precond.build(prob, kind, modified=False, hop=hop, eps=1e-12)
    assert t["n_floored"] == 0
    Kb = precond.wavelet_blocks(prob, None, t["M0"], hop=hop, wavelet=wv)
    np.testing.assert_allclose(Kb, Bw, rtol=1e-12, atol=1e-12)
    want = np.stack([scipy.linalg.fractional_matrix_power(b, -0.5).real for b in Bw.reshape(-1, K, K)])
    np.testing.assert_allclose(t["P"].reshape(-1, K, K), want, rtol=1e-9, atol=1e-12)
    M = _dense(lambda v: precond.apply_M(t, v), (K, n, n))
    H = _dense(hop, (K, n, n))
    np.testing.assert_allclose(M.T @ H @ M, np.eye(K * n * n), atol=1e-10)
