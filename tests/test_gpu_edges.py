"""Edge cases of the iteration on the GPU: no iterations, a start at the exact
minimiser, no penalty, and the largest image the partial-sum buffers admit
(2048 x 2048: 256 threads x 16384 blocks)."""

import os

import numpy as np
import pytest
import torch

import oracle
from gpu_util import announce, dev, host, l2rel, maxrel
from oracle import model, precond as opre, sps as osps
from workloads import configs as C

import paper_2010_01371_amd as mb

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("kind", ["none", "fourier", "blockdiag"])
def test_zero_iterations_leave_x_and_report_its_objective(kind):
    """n_iter = 0: x is untouched (bit for bit) and the trace holds one value,
    the objective at x."""
    wl = C.make_small_fan(n=32, views=48, bins=64)
    op = oracle.OracleProblem.from_workload(wl)
    x0 = wl.x_true * np.random.default_rng(3).uniform(0.8, 1.1, size=wl.x_true.shape)
    announce("zero iterations", kind)
    P = mb.Problem.from_workload(wl)
    if kind != "none":
        P.precond_build(kind)
    x = dev(x0)
    before = host(x)
    tr = P.sps_step(x, kind, 0, trace=True)
    assert len(tr) == 1
    np.testing.assert_array_equal(host(x), before)
    phi = model.objective(op, before)
    assert abs(tr[0] - phi) <= 1e-5 * abs(phi), (tr[0], phi)
    P.close()


@pytest.mark.parametrize("kind", ["none", "fourier", "haar", "blockdiag"])
def test_start_at_the_minimiser(kind):
    """From the oracle's Newton minimiser of the 64x64 parallel problem the
    gradient nearly vanishes (g^T p ~ 0): the step sizes stay finite, no
    failure flag is raised, the objective does not rise beyond FP32
    evaluation noise, and the iterate stays at the minimiser to the FP32
    floor of the converged runs (relative RMSE ~1e-4)."""
    wl = C.make_c1()
    ref = np.load(os.path.join(GOLDEN, "newton_xhat_c1.npz"))
    xhat = ref["xhat"]
    announce("start at the minimiser", kind)
    P = mb.Problem.from_workload(wl)
    if kind != "none":
        P.precond_build(kind)
    x = dev(xhat)
    tr = P.sps_step(x, kind, 20, trace=True)
    P.check()                                   # raises on a failure flag
    assert np.all(np.isfinite(tr))
    phi_hat = float(ref["objective"])
    assert np.all(tr <= phi_hat * (1 + 1e-5)), (tr.max(), phi_hat)
    assert l2rel(host(x), xhat) <= 2e-4, l2rel(host(x), xhat)
    P.close()


@pytest.mark.parametrize("kind", ["none", "fourier", "blockdiag"])
def test_zero_penalty_matches_oracle(kind):
    """beta = 0: no penalty terms in the gradient, the curvature or the step
    size (the launches take no penalty arguments)."""
    wl = C.make_small_fan(n=64, views=90, bins=128, penalty="quadratic")
    pen = dict(kind="quadratic", beta=np.zeros((1, 1)), delta=0.0)
    wl0 = C.Workload(wl.name + "_nopen", wl.geom, wl.Q, wl.S, wl.y, wl.w, pen, wl.x_true, 20, [kind])
    op = oracle.OracleProblem.from_workload(wl0)
    n = 20
    announce("zero penalty", kind, n)
    P = mb.Problem.from_workload(wl0)
    if kind != "none":
        P.precond_build(kind)
    x = P.zeros_image()
    tr = P.sps_step(x, kind, n, trace=True)
    if kind == "none":
        xo, phio = osps.sps_plain(op, n, trace=True)
    else:
        xo, phio, _ = osps.sps_precond(op, opre.build(op, kind), n, trace=True)
    assert l2rel(host(x), xo) <= 1e-4, l2rel(host(x), xo)
    np.testing.assert_allclose(tr[-1], phio[-1], rtol=1e-4)
    P.close()


def _max_geometry():
    """2048 x 2048 pixels of 0.25 mm (the partial-sum limit), parallel beam,
    180 views over 180 degrees, 2900 bins of 0.25 mm covering the diagonal."""
    return C.geometry("parallel", 2048, 2048, 0.25, 0.25, 180, np.pi, 2900, 0.25)


def test_projector_adjoint_at_the_largest_image():
    """<A x, y> = <x, A^T y> for positive random x and y at 2048 x 2048
    (about 1.5e9 nonzeros): both sides in FP64 from the FP32 results."""
    g = _max_geometry()
    rng = np.random.default_rng(2048)
    x = rng.uniform(0.0, 1.0, size=(1, 2048, 2048))
    y = rng.uniform(0.0, 1.0, size=(1, g["n_views"], g["n_bins"]))
    announce("adjoint at 2048^2")
    Ax = host(mb.project(g, dev(x)))
    Aty = host(mb.backproject(g, dev(y)))
    lhs = float(np.sum(Ax * y))
    rhs = float(np.sum(x * Aty))
    mb.cache_clear()
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs), (lhs, rhs)


def _disk_problem():
    """Two materials in concentric disks on the largest image, with counts
    from the disks' exact chord lengths (the same at every parallel view)."""
    g = _max_geometry()
    Q = np.array([[0.030, 0.60], [0.024, 0.35], [0.020, 0.22], [0.018, 0.15]])   # per mm, 4 energies
    S = np.array([[4e4, 3e4, 1e4, 2e3], [1e3, 1e4, 3e4, 4e4]])                   # 2 channels
    u = (np.arange(g["n_bins"]) - (g["n_bins"] - 1) / 2) * g["du"]
    chord = lambda r: 2 * np.sqrt(np.maximum(r * r - u * u, 0.0))
    l = np.stack([0.9 * chord(220.0), 0.05 * chord(60.0)])                       # [K][bins]
    ybar = S @ np.exp(-(Q @ l))                                                  # [C][bins]
    y = np.random.default_rng(5).poisson(np.broadcast_to(ybar[:, None, :], (2, g["n_views"], g["n_bins"])))
    y = np.maximum(y, 1.0).astype(np.float64)
    pen = dict(kind="quadratic", beta=np.diag([1e-2, 1.0]), delta=0.0)
    return g, Q, S, y, pen


@pytest.mark.parametrize("kind", ["none", "blockdiag"])
def test_iterations_at_the_largest_image(kind):
    """Two materials x two channels at 2048 x 2048: every partial-sum region
    at or near its capacity (16384 pixel blocks; the direction's dot product
    over both materials needs two elements per thread).  Three traced
    iterations: finite, decreasing objective, no failure flag."""
    g, Q, S, y, pen = _disk_problem()
    announce("iterations at 2048^2", kind)
    P = mb.Problem(g, Q, S, y, None, pen)
    if kind != "none":
        P.precond_build(kind)
    x = P.zeros_image()
    tr = P.sps_step(x, kind, 3, trace=True)
    P.check()
    assert np.all(np.isfinite(tr)), tr
    assert np.all(np.diff(tr) < 0), tr
    assert np.all(np.isfinite(host(x)))
    P.close()
    mb.cache_clear()


@pytest.mark.parametrize("n", [1024, 2048])
def test_fourier_apply_at_large_images(n):
    """The 2D FFT at 1024 (compiled length) and 2048 (general length, 256
    threads per transform: the largest one block holds), against the oracle."""
    # The counts depend on the views, the bins and the phantom's ellipses, not on
    # the pixel grid: the 64x64 workload's data on the same 128 mm field of view
    # at n x n pixels (no pixelised phantom needed).
    small = C.make_small_fan(n=64, views=24, bins=96)
    geom = dict(small.geom, nx=n, ny=n, dx=128.0 / n, dy=128.0 / n)
    wl = C.Workload("fan%d_from64" % n, geom, small.Q, small.S, small.y, small.w, small.penalty,
                    np.zeros((1, n, n)), 1, ["fourier"])
    op = oracle.OracleProblem.from_workload(wl)
    g = np.random.default_rng(n).normal(size=(1, n, n))
    announce("precond_apply", "fan%d" % n, "fourier")
    P = mb.Problem.from_workload(wl)
    P.precond_build("fourier")
    got = host(P.precond_apply("fourier", dev(g)))
    tab = opre.build(op, "fourier")
    want = opre.apply_M(tab, opre.apply_Mt(tab, g))
    assert l2rel(got, want) <= 1e-4, l2rel(got, want)         # as at the smaller sizes
    P.close()
