"""Pins of the oracle's forward model, objective, gradient, penalty and SPS
surrogate quantities (CPU only)."""

import numpy as np
import pytest

import oracle
from oracle import model, penalty as pen, projector as P, sps
from workloads import configs as C


def _tiny_mbmd(n_mat=3, noise=True):
    wl = C.make_small_mbmd(n=16, views=12, bins=32, n_mat=n_mat, noise=noise, n_energy_step=10)
    return oracle.OracleProblem.from_workload(wl), wl


def _tiny_mono(kind="quadratic"):
    wl = C.make_small_fan(n=16, views=12, bins=32, penalty=kind)
    return oracle.OracleProblem.from_workload(wl), wl


def _fd_gradient(f, x, idx, h):
    out = []
    for j in idx:
        e = np.zeros_like(x)
        e.flat[j] = h
        out.append((f(x + e) - f(x - e)) / (2 * h))
    return np.array(out)


@pytest.mark.parametrize("maker", [lambda: _tiny_mono("quadratic"), lambda: _tiny_mono("huber"),
                                   lambda: _tiny_mbmd(3), lambda: _tiny_mbmd(2)])
def test_gradient_matches_central_differences(maker):
    prob, wl = maker()
    rng = np.random.default_rng(7)
    x = wl.x_true * rng.uniform(0.8, 1.2, size=wl.x_true.shape)
    if prob.penalty["kind"] == "huber":
        # keep every neighbour difference away from the Huber kink at +-delta
        x = wl.x_true + 0.01 * rng.normal(size=wl.x_true.shape)
    g = model.gradient(prob, x)
    idx = rng.choice(x.size, 12, replace=False)
    scale = np.abs(x).max()
    fd = _fd_gradient(lambda z: model.objective(prob, z), x, idx, 1e-6 * scale)
    np.testing.assert_allclose(g.flat[idx], fd, rtol=2e-6, atol=2e-6 * np.abs(g).max())


def test_noise_free_identity_geometry_has_zero_objective_at_truth():
    """With A = I, beta = 0 and noise-free data, Phi(l_true) = 0 and grad = 0."""
    wl = C.make_c3(noise=False, n_views=6, n_bins=10)
    prob = oracle.OracleProblem.from_workload(wl)
    assert model.objective(prob, wl.x_true) < 1e-20 * np.sum(wl.y ** 2)
    g = model.gradient(prob, wl.x_true)
    assert np.abs(g).max() < 1e-9


def test_single_energy_reduces_to_beer_lambert():
    """N_k = N_E = N_c = 1: ybar = I0 exp(-A mu)."""
    prob, wl = _tiny_mono()
    x = wl.x_true
    np.testing.assert_allclose(model.forward(prob, x)[0],
                               wl.S[0, 0] * np.exp(-P.project(wl.geom, x[0])), rtol=1e-14)


def test_surrogate_gradient_equals_true_gradient():
    """The SPS gradient AA^T(-eta t^2 - rho t) (readings of rho and of the
    printed gradient) equals dL/dx at x^(n)."""
    for prob, wl in (_tiny_mono(), _tiny_mbmd(3)):
        x = wl.x_true * 0.7
        l = model.line_integrals(prob, x)
        t, ybar, rho, hdot, c = sps.ray_terms(prob, l)
        np.testing.assert_allclose(hdot, model.hdot(prob, t), rtol=1e-10,
                                   atol=1e-12 * np.abs(hdot).max())
        u = np.einsum("ek,evb->kvb", prob.Q, hdot)
        np.testing.assert_allclose(P.backproject(wl.geom, u), model.data_gradient(prob, x),
                                   rtol=1e-10, atol=1e-12 * np.abs(u).max())


def test_decoupled_surrogate_majorises_likelihood_in_t():
    """L(t) <= sum_iE (eta/2 t^2 + rho t) + const, equality at t^(n)
    (needs S^T W S >= 0 entrywise, true for counts)."""
    prob, wl = _tiny_mbmd(3)
    rng = np.random.default_rng(3)
    l0 = model.line_integrals(prob, wl.x_true * 0.9)
    t0, _, rho, _, _ = sps.ray_terms(prob, l0)
    eta = sps.eta(prob)

    def L(t):
        r = prob.y - model.mean_counts(prob, t)
        return 0.5 * np.sum(prob.w * r * r)

    def Ls(t):
        return np.sum(0.5 * eta * t * t + rho * t)

    const = L(t0) - Ls(t0)
    for _ in range(50):
        t = np.exp(-model.energy_line_integrals(prob, l0 * rng.uniform(0.0, 2.0, size=l0.shape)))
        assert Ls(t) + const >= L(t) - 1e-9 * abs(L(t))


def test_max_curvature_parabola_majorises_on_nonnegative_l():
    """c = max(2 eta + rho, 0) gives a parabola above h(l) = eta/2 e^-2l + rho e^-l
    on l >= 0, touching at l^(n)."""
    rng = np.random.default_rng(4)
    eta = rng.uniform(0.1, 10.0, 200)
    rho = rng.uniform(-15.0, 5.0, 200)
    ln = rng.uniform(0.0, 4.0, 200)
    c = np.maximum(2 * eta + rho, 0.0)
    h = lambda l: 0.5 * eta * np.exp(-2 * l) + rho * np.exp(-l)
    dh = -eta * np.exp(-2 * ln) - rho * np.exp(-ln)
    for l in np.linspace(0.0, 8.0, 801):
        q = h(ln) + dh * (l - ln) + 0.5 * c * (l - ln) ** 2
        assert np.all(q >= h(l) - 1e-12 * (1 + np.abs(h(l))))
    # the bound is tight: at l = 0 the curvature of h equals c where c > 0
    np.testing.assert_allclose((2 * eta + rho)[c > 0], c[c > 0])


def test_single_energy_curvature_is_constant():
    """One energy: eta = I0^2 w, rho = -I0 w y, c = max(2 I0^2 w - I0 w y, 0)
    whatever x is."""
    prob, wl = _tiny_mono()
    I0 = wl.S[0, 0]
    for s in (0.0, 0.5, 1.3):
        _, _, rho, _, c = sps.ray_terms(prob, model.line_integrals(prob, s * wl.x_true))
        np.testing.assert_allclose(rho[0], -I0 * wl.w[0] * wl.y[0], rtol=1e-12)
        np.testing.assert_allclose(c[0], np.maximum(2 * I0 * I0 * wl.w[0] - I0 * wl.w[0] * wl.y[0], 0),
                                   rtol=1e-12)


def _dense_gamma(ny, nx):
    """Graph Laplacian by brute force over 4-neighbour pairs."""
    N = ny * nx
    G = np.zeros((N, N))
    for iy in range(ny):
        for ix in range(nx):
            j = iy * nx + ix
            for dy, dx in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                y2, x2 = iy + dy, ix + dx
                if 0 <= y2 < ny and 0 <= x2 < nx:
                    G[j, j] += 1
                    G[j, y2 * nx + x2] -= 1
    return G


def test_quadratic_penalty_matches_dense_definition():
    rng = np.random.default_rng(5)
    ny, nx, K = 5, 7, 2
    Bm = rng.normal(size=(K, K))
    beta = Bm @ Bm.T
    prob, _ = _tiny_mbmd(2)
    prob.penalty = dict(kind="quadratic", beta=beta, delta=0.0)
    x = rng.normal(size=(K, ny, nx))
    G = _dense_gamma(ny, nx)
    R = np.kron(beta, G)
    xv = x.reshape(-1)
    assert np.isclose(pen.value(prob, x), 0.5 * xv @ R @ xv, rtol=1e-12)
    np.testing.assert_allclose(pen.gradient(prob, x).reshape(-1), R @ xv, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(pen.sps_curvature(prob, x).reshape(-1), np.abs(R).sum(1), rtol=1e-12)
    p = rng.normal(size=x.shape)
    assert np.isclose(pen.curvature_quadform(prob, x, p), p.reshape(-1) @ R @ p.reshape(-1), rtol=1e-12)
    # Gamma 1 = 0 and |Gamma| 1 = 2 |N_j|
    assert np.allclose(G.sum(1), 0.0)
    np.testing.assert_allclose(np.abs(G).sum(1), 2 * pen.neighbour_count(ny, nx).reshape(-1))
    # the double sum of quadReg_summation counts every pair twice
    s316 = 0.0
    for k in range(K):
        for kp in range(K):
            for j in range(ny * nx):
                for jp in np.nonzero(G[j] < 0)[0]:
                    s316 += 0.5 * beta[k, kp] * (xv[k * ny * nx + j] - xv[k * ny * nx + jp]) * \
                        (xv[kp * ny * nx + j] - xv[kp * ny * nx + jp])
    assert np.isclose(s316, 2 * pen.value(prob, x), rtol=1e-12)


def test_huber_reduces_to_quadratic_for_large_delta():
    prob, wl = _tiny_mono("huber")
    x = wl.x_true + 0.01 * np.random.default_rng(6).normal(size=wl.x_true.shape)
    q = oracle.OracleProblem(wl.geom, wl.Q, wl.S, wl.y, wl.w,
                             dict(kind="quadratic", beta=prob.penalty["beta"], delta=0.0))
    prob.penalty["delta"] = 1e6
    p = np.random.default_rng(7).normal(size=x.shape)
    assert np.isclose(pen.value(prob, x), pen.value(q, x), rtol=1e-12)
    np.testing.assert_allclose(pen.gradient(prob, x), pen.gradient(q, x), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(pen.sps_curvature(prob, x), pen.sps_curvature(q, x), rtol=1e-12)
    assert np.isclose(pen.curvature_quadform(prob, x, p), pen.curvature_quadform(q, x, p), rtol=1e-12)


def test_huber_separable_surrogate_majorises():
    """R(x) <= R(x^n) + dR^T (x - x^n) + 1/2 sum d_R (x - x^n)^2 for Huber."""
    prob, wl = _tiny_mono("huber")
    rng = np.random.default_rng(8)
    xn = wl.x_true + 0.002 * rng.normal(size=wl.x_true.shape)
    g = pen.gradient(prob, xn)
    d = pen.sps_curvature(prob, xn)
    for _ in range(30):
        x = xn + 0.004 * rng.normal(size=xn.shape)
        s = pen.value(prob, xn) + np.sum(g * (x - xn)) + 0.5 * np.sum(d * (x - xn) ** 2)
        assert s >= pen.value(prob, x) - 1e-12 * abs(pen.value(prob, x))


def test_forward_vjp_matches_finite_differences():
    """Backward of the polyenergetic forward model: d<gbar, ybar(x)>/dx."""
    prob, wl = _tiny_mbmd(3)
    rng = np.random.default_rng(9)
    x = wl.x_true * 0.8
    gbar = rng.normal(size=wl.y.shape)
    g = model.forward_vjp(prob, x, gbar)
    idx = rng.choice(x.size, 10, replace=False)
    fd = _fd_gradient(lambda z: np.sum(gbar * model.forward(prob, z)), x, idx, 1e-6)
    np.testing.assert_allclose(g.flat[idx], fd, rtol=1e-6, atol=1e-7 * np.abs(g).max())
