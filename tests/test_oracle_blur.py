"""Pins of the oracle's projection-domain blur: BB = B S in the mean model,
its gradient, the decoupled SPS surrogate, the Fisher operator the
preconditioners are built from, and convergence to a brute-force Newton
minimiser (CPU only)."""

import numpy as np
import pytest

import oracle
from oracle import model, penalty as pen, precond, projector as P, sps
from workloads import configs as C
from workloads import phantoms as ph

TAPS3 = np.array([0.2, 0.6, 0.2])


def _with_blur(prob, taps):
    taps = np.atleast_2d(taps)
    if taps.shape[0] == 1:
        taps = np.repeat(taps, prob.n_chan, axis=0)
    return oracle.OracleProblem(prob.geom, prob.Q, prob.S, prob.y, prob.w, prob.penalty, blur=taps)


def _mono(kind="quadratic"):
    wl = C.make_small_fan(n=16, views=12, bins=32, penalty=kind)
    return oracle.OracleProblem.from_workload(wl), wl


def _mbmd(n_mat=3):
    wl = C.make_small_mbmd(n=16, views=12, bins=32, n_mat=n_mat, n_energy_step=10)
    return oracle.OracleProblem.from_workload(wl), wl


def _channel_taps(n_chan):
    """Different, asymmetric kernels per channel (h = 2)."""
    rng = np.random.default_rng(5)
    t = rng.uniform(0.05, 1.0, size=(n_chan, 5))
    return t / t.sum(axis=1, keepdims=True)


def test_blur_is_zero_padded_correlation_along_the_bins():
    """B z is the correlation of each view's row with the taps and B^T y the
    convolution, both with zeros beyond the detector (numpy's 'same' modes)."""
    prob, _ = _mbmd()
    taps = _channel_taps(prob.n_chan)
    pb = _with_blur(prob, taps)
    rng = np.random.default_rng(1)
    z = rng.normal(size=(prob.n_chan,) + prob.sino_shape)
    Bz, Btz = model.blur(pb, z), model.blur(pb, z, transpose=True)
    for c in range(prob.n_chan):
        for v in range(prob.sino_shape[0]):
            np.testing.assert_allclose(Bz[c, v], np.correlate(z[c, v], taps[c], mode="same"), rtol=1e-13,
                                       atol=1e-14)
            np.testing.assert_allclose(Btz[c, v], np.convolve(z[c, v], taps[c], mode="same"), rtol=1e-13,
                                       atol=1e-14)


def test_delta_taps_give_the_unblurred_problem():
    for prob, wl in (_mono(), _mbmd()):
        pb = _with_blur(prob, [0.0, 1.0, 0.0])
        x = wl.x_true * 0.8
        np.testing.assert_allclose(model.objective(pb, x), model.objective(prob, x), rtol=1e-14)
        np.testing.assert_allclose(model.gradient(pb, x), model.gradient(prob, x), rtol=1e-13, atol=1e-13)
        l = model.line_integrals(prob, x)
        for a, b in zip(sps.ray_terms(pb, l), sps.ray_terms(prob, l)):
            np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-13 * np.abs(b).max())


def _fd_gradient(f, x, idx, h):
    out = []
    for j in idx:
        e = np.zeros_like(x)
        e.flat[j] = h
        out.append((f(x + e) - f(x - e)) / (2 * h))
    return np.array(out)


@pytest.mark.parametrize("maker", [_mono, _mbmd])
def test_blurred_gradient_matches_central_differences(maker):
    prob, wl = maker()
    pb = _with_blur(prob, _channel_taps(prob.n_chan))
    rng = np.random.default_rng(7)
    x = wl.x_true * rng.uniform(0.8, 1.2, size=wl.x_true.shape)
    g = model.gradient(pb, x)
    idx = rng.choice(x.size, 12, replace=False)
    fd = _fd_gradient(lambda z: model.objective(pb, z), x, idx, 1e-6 * np.abs(x).max())
    np.testing.assert_allclose(g.flat[idx], fd, rtol=2e-6, atol=2e-6 * np.abs(g).max())


def test_blurred_forward_vjp_matches_finite_differences():
    prob, wl = _mbmd()
    pb = _with_blur(prob, _channel_taps(prob.n_chan))
    rng = np.random.default_rng(8)
    x = wl.x_true * 0.9
    gbar = rng.normal(size=prob.y.shape)
    vj = model.forward_vjp(pb, x, gbar)
    idx = rng.choice(x.size, 10, replace=False)
    f = lambda z: float(np.sum(gbar * model.forward(pb, z)))
    fd = _fd_gradient(f, x, idx, 1e-6 * np.abs(x).max())
    np.testing.assert_allclose(vj.flat[idx], fd, rtol=2e-6, atol=2e-6 * np.abs(vj).max())


def test_blurred_surrogate_gradient_equals_true_gradient():
    """-eta t^2 - rho t with the blurred eta and rho is dL/dl_E at t^(n)."""
    prob, wl = _mbmd()
    pb = _with_blur(prob, _channel_taps(prob.n_chan))
    l = model.line_integrals(pb, wl.x_true * 0.7)
    t, _, _, hd, _ = sps.ray_terms(pb, l)
    np.testing.assert_allclose(hd, model.hdot(pb, t), rtol=1e-10, atol=1e-12 * np.abs(hd).max())


def test_blurred_decoupled_surrogate_majorises_likelihood_in_t():
    """L(t) <= sum_iE (eta/2 t^2 + rho t) + const, equal at t^(n); with the blur
    eta = S^T B^T W B S 1 also covers the coupling between neighbouring bins."""
    prob, wl = _mbmd()
    pb = _with_blur(prob, _channel_taps(prob.n_chan))
    rng = np.random.default_rng(3)
    l0 = model.line_integrals(pb, wl.x_true * 0.9)
    t0, _, rho, _, _ = sps.ray_terms(pb, l0)
    eta = sps.eta(pb)

    def L(t):
        r = pb.y - model.mean_counts(pb, t)
        return 0.5 * np.sum(pb.w * r * r)

    def Ls(t):
        return np.sum(0.5 * eta * t * t + rho * t)

    const = L(t0) - Ls(t0)
    for _ in range(50):
        t = np.exp(-model.energy_line_integrals(pb, l0 * rng.uniform(0.0, 2.0, size=l0.shape)))
        assert Ls(t) + const >= L(t) - 1e-9 * abs(L(t))


def test_blurred_eta_is_the_row_sum_of_the_likelihood_hessian_in_t():
    """eta = BB^T W BB 1: L is quadratic in t with Hessian M = BB^T W BB, so
    eta_i = (M 1)_i = dL/dt_i at t = 1 minus dL/dt_i at t = 0, here by
    central differences of the blurred likelihood (exact for a quadratic up
    to rounding) at sampled (energy, view, bin)."""
    prob, wl = _mbmd()
    pb = _with_blur(prob, _channel_taps(prob.n_chan))
    eta = sps.eta(pb)

    def L(t):
        r = pb.y - model.mean_counts(pb, t)
        return 0.5 * np.sum(pb.w * r * r)

    rng = np.random.default_rng(10)
    shape = eta.shape
    h = 0.5
    for _ in range(12):
        idx = tuple(int(rng.integers(n)) for n in shape)
        if rng.random() < 0.3:
            idx = idx[:2] + (int(rng.choice([0, 1, shape[2] - 1])),)    # detector edges
        d = []
        for base in (1.0, 0.0):
            t = np.full(shape, base)
            tp, tm = t.copy(), t.copy()
            tp[idx] += h
            tm[idx] -= h
            d.append((L(tp) - L(tm)) / (2 * h))
        np.testing.assert_allclose(d[0] - d[1], eta[idx], rtol=1e-8)


def test_one_energy_curvature_depends_on_x_under_blur():
    """Without a blur the one-energy curvature is constant; with one, rho picks
    up the neighbours' transmissions and c changes with x."""
    prob, wl = _mono()
    pb = _with_blur(prob, TAPS3)
    c = [sps.ray_terms(pb, model.line_integrals(pb, s * wl.x_true))[4] for s in (0.2, 1.0)]
    assert np.abs(c[0] - c[1]).max() > 1e-3 * np.abs(c[1]).max()


def test_blurred_fisher_is_the_gram_of_the_jacobian():
    """At a reference image, A^T (J^T B^T W B J) A v equals (d ybar/dx)^T W
    (d ybar/dx) v, the Jacobian-vector product by central differences of the
    blurred forward model and the transpose by its (pinned) VJP."""
    prob, wl = _mbmd()
    pb = _with_blur(prob, _channel_taps(prob.n_chan))
    x_ref = np.abs(wl.x_true) * 0.5
    Wj = precond.fisher_weights(pb, x_ref)
    assert Wj.shape == (pb.n_chan, pb.n_mat) + pb.sino_shape
    rng = np.random.default_rng(9)
    v = rng.normal(size=x_ref.shape) * np.abs(x_ref).max()
    Fv = P.backproject(pb.geom, precond.fisher_sino_apply(pb, Wj, P.project(pb.geom, v)))
    h = 1e-6
    jv = (model.forward(pb, x_ref + h * v) - model.forward(pb, x_ref - h * v)) / (2 * h)
    Fv_fd = model.forward_vjp(pb, x_ref, pb.w * jv)
    np.testing.assert_allclose(Fv, Fv_fd, rtol=1e-6, atol=1e-7 * np.abs(Fv_fd).max())


def _dense_blur(taps, nb):
    """Brute force: entry (b, b') = taps[b' - b + h] inside the band."""
    h = (len(taps) - 1) // 2
    Bm = np.zeros((nb, nb))
    for b in range(nb):
        for bp in range(nb):
            if abs(bp - b) <= h:
                Bm[b, bp] = taps[bp - b + h]
    return Bm


def _newton_blur_problem(beta):
    rng = np.random.default_rng(12)
    g = C.geometry("parallel", 8, 8, 1.0, 1.0, 12, np.pi, 12, 1.0)
    ell = [(0.0, 0.0, 3.6, 3.0, 0.4, 0.05), (1.0, -0.5, 1.2, 1.0, 0.0, 0.04)]
    xt = ph.pixelise(ell, 8, 8, 1.0, 1.0)
    Bm = _dense_blur(TAPS3, 12)
    ybar = (1e4 * np.exp(-ph.line_integrals(ell, g))) @ Bm.T
    y = rng.poisson(ybar).astype(float)[None]
    w = 1.0 / np.maximum(y, 1.0)
    prob = oracle.OracleProblem(g, np.ones((1, 1)), np.array([[1e4]]), y, w,
                                dict(kind="quadratic", beta=np.array([[beta]]), delta=0.0), blur=TAPS3[None])
    return prob, Bm


def _newton_blur(prob, Bm, iters=40):
    """Newton on the exact blurred objective with dense A and the dense
    block-diagonal blur BB = I_V (x) B."""
    A = P.dense_matrix(prob.geom)
    V = prob.sino_shape[0]
    BB = np.kron(np.eye(V), Bm)
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
        r = w * (BB @ (I0 * t) - y)
        s = BB.T @ r
        g = A.T @ (-I0 * t * s) + G @ x
        Jl = -(BB * (I0 * t)[None, :])                      # d ybar / d l
        H = A.T @ (Jl.T @ (w[:, None] * Jl) + np.diag(I0 * t * s)) @ A + G
        x = x - np.linalg.solve(H, g)
    return x.reshape(1, 8, 8), H, np.linalg.norm(g)


def test_blurred_newton_reference():
    prob, Bm = _newton_blur_problem(3000.0)
    xhat, H, gnorm = _newton_blur(prob, Bm)
    assert gnorm < 1e-8
    assert np.linalg.eigvalsh(H).min() > 0.0
    np.testing.assert_allclose(model.gradient(prob, xhat), 0.0, atol=1e-7)


def _monotone(phi):
    return bool(np.all(np.diff(phi) <= 1e-9 * np.abs(phi[:-1])))


@pytest.mark.parametrize("kind", [None, "blockdiag", "fourier", "haar"])
def test_blurred_variants_converge_to_the_newton_minimiser(kind):
    prob, Bm = _newton_blur_problem(3000.0)
    xhat, _, _ = _newton_blur(prob, Bm)
    if kind is None:
        x, phi = sps.sps_plain(prob, 1500)
    else:
        x, phi, _ = sps.sps_precond(prob, precond.build(prob, kind), 1500)
    assert _monotone(phi)
    assert np.linalg.norm(x - xhat) / np.linalg.norm(xhat) < 1e-6
