"""GPU parity of the projection-domain blur (mbmd_problem_set_blur) against
the FP64 oracle: forward model and VJP, gradient / curvature / objective,
plain and preconditioned SPS iterates, and the preconditioner applies built
from the blurred Fisher information."""

import numpy as np
import pytest

import oracle
from gpu_util import announce, dev, host, l2rel, maxrel
from oracle import model, penalty as pen, precond as opre, sps as osps
from workloads import configs as C

import paper_2010_01371_amd as mb

pytestmark = pytest.mark.gpu

# Same bars as the unblurred parity tests (the blur adds a few FP32 taps per
# residual and no cancellation of its own).
TOL_GRAD = 2e-3
TOL_CURV = 1e-5
TOL_OBJ = 1e-5
TOL_ITER = 1e-4
TOL_APPLY = 1e-4


def _fan():
    return C.make_small_fan(n=64, views=90, bins=128, penalty="huber")


def _mbmd():
    return C.make_small_mbmd(n=32, views=60, bins=64, n_mat=3)


CASES = {"fan64": _fan, "mbmd32": _mbmd}


def _taps(n_chan, case):
    """fan64: one symmetric 3-tap kernel; mbmd32: a different asymmetric
    5-tap kernel per channel."""
    if case == "fan64":
        return np.array([[0.25, 0.5, 0.25]])
    t = np.random.default_rng(31).uniform(0.05, 1.0, size=(n_chan, 5))
    return t / t.sum(axis=1, keepdims=True)


def _problems(case):
    wl = CASES[case]()
    taps = _taps(wl.S.shape[0], case)
    full = np.repeat(taps, wl.S.shape[0], axis=0) if taps.shape[0] == 1 else taps
    op = oracle.OracleProblem(wl.geom, wl.Q, wl.S, wl.y, wl.w, wl.penalty,
                              blur=full.astype(np.float32).astype(np.float64))
    P = mb.Problem.from_workload(wl)
    P.set_blur(taps)
    return wl, op, P


@pytest.mark.parametrize("case", sorted(CASES))
def test_blurred_forward_and_vjp(case):
    wl, op, P = _problems(case)
    x = wl.x_true * 0.9
    gbar = np.random.default_rng(20).normal(size=wl.y.shape)
    announce("blur forward/vjp", case)
    ybar, l = P.forward(dev(x))
    assert maxrel(host(ybar), model.forward(op, x)) <= 1e-5
    got = host(P.forward_vjp(l, dev(gbar)))
    want = model.forward_vjp(op, x, gbar)
    assert l2rel(got, want) <= 1e-5, l2rel(got, want)


@pytest.mark.parametrize("case", sorted(CASES))
def test_blurred_gradient_curvature_objective(case):
    wl, op, P = _problems(case)
    x = wl.x_true * np.random.default_rng(10).uniform(0.7, 1.1, size=wl.x_true.shape)
    announce("blur gradient", case)
    g, d, phi = P.gradient(dev(x), curvature=True, objective=True)
    g, d = host(g), host(d)
    gL, dL = osps.surrogate_terms(op, x)
    assert l2rel(g, model.gradient(op, x)) <= TOL_GRAD, l2rel(g, model.gradient(op, x))
    d_want = dL + pen.sps_curvature(op, x)
    assert maxrel(d, d_want) <= TOL_CURV, maxrel(d, d_want)
    phi_want = model.objective(op, x)
    assert abs(phi - phi_want) <= TOL_OBJ * abs(phi_want), (phi, phi_want)


def _rmse(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2)) / np.sqrt(np.mean(b ** 2)))


@pytest.mark.parametrize("kind", ["none", "blockdiag", "fourier", "haar"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_blurred_sps_iterates(case, kind):
    """Iterates after 30 iterations (Haar: 10) and the objective trace over
    the first 5, the schedule of the unblurred MBMD test.  The preconditioned
    MBMD iterations are sensitive to their tables: in the FP64 oracle a
    relative 1e-6 perturbation of the Fourier tables moves the blurred
    iterate by 7e-4 after 10 iterations and 4.6e-4 after 30 (unblurred 4.4e-4
    and 2.8e-4), and cross-material Haar is chaotic after 10."""
    wl, op, P = _problems(case)
    n = 10 if kind == "haar" else 30
    announce("blur sps", case, kind, n)
    if kind != "none":
        P.precond_build(kind)
    x = P.zeros_image()
    tg = P.sps_step(x, kind, n, trace=True)
    if kind == "none":
        xo, to = osps.sps_plain(op, n)
    else:
        xo, to, _ = osps.sps_precond(op, opre.build(op, kind), n)
    assert np.all(np.isfinite(tg))
    assert _rmse(host(x), xo) <= TOL_ITER, _rmse(host(x), xo)
    np.testing.assert_allclose(tg[:5], to[:5], rtol=1e-4)


@pytest.mark.parametrize("kind", ["blockdiag", "fourier", "haar", "daub4"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_blurred_precond_apply(case, kind):
    wl, op, P = _problems(case)
    g = np.random.default_rng(12).normal(size=wl.x_true.shape)
    announce("blur precond_apply", case, kind)
    P.precond_build(kind)
    got = host(P.precond_apply(kind, dev(g)))
    tab = opre.build(op, kind)
    want = opre.apply_M(tab, opre.apply_Mt(tab, g))
    assert l2rel(got, want) <= TOL_APPLY, l2rel(got, want)


def test_removing_the_blur_restores_the_unblurred_iterates():
    """set_blur(None) after a blurred run gives the bits of a problem that
    never had a blur (the blur voids the builds; rebuild them)."""
    wl = _fan()
    announce("blur removed", "fan64")
    ref = mb.Problem.from_workload(wl)
    ref.precond_build("fourier")
    x_ref = ref.zeros_image()
    ref.sps_step(x_ref, "fourier", 5)
    P = mb.Problem.from_workload(wl)
    P.precond_build("fourier")
    P.set_blur([[0.25, 0.5, 0.25]])
    with pytest.raises(RuntimeError):
        P.precond_apply("fourier", ref.zeros_image())
    x = P.zeros_image()
    P.precond_build("fourier")
    P.sps_step(x, "fourier", 3)
    P.set_blur(None)
    P.precond_build("fourier")
    x = P.zeros_image()
    P.sps_step(x, "fourier", 5)
    np.testing.assert_array_equal(host(x), host(x_ref))


def test_blur_argument_errors():
    wl = _fan()
    P = mb.Problem.from_workload(wl)
    announce("blur errors")
    with pytest.raises(RuntimeError):
        P.set_blur([[0.2, -0.1, 0.9]])                 # negative tap
    with pytest.raises(RuntimeError):
        P.set_blur(np.ones((1, 11)) / 11)              # half width 5 > 4
    with pytest.raises(RuntimeError):
        P.set_blur([[0.2, np.nan, 0.8]])
    Pi = mb.Problem.from_workload(C.make_c3(n_views=8, n_bins=12))
    with pytest.raises(RuntimeError):
        Pi.set_blur([[0.25, 0.5, 0.25]])               # identity geometry
    Pi.set_blur(None)                                  # removing none is fine
