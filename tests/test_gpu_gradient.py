"""GPU parity of the per-ray spectral pass, penalty and fused gradient /
SPS-curvature / objective (mbmd_gradient) against the FP64 oracle."""

import numpy as np
import pytest

import oracle
from gpu_util import announce, dev, host, l2rel, maxrel
from oracle import model, penalty as pen, sps
from workloads import configs as C

import paper_2010_01371_amd as mb

pytestmark = pytest.mark.gpu

# The data gradient is A^T of t * S^T w (ybar - y): the residual ybar - y is a
# difference of FP32 numbers of size ybar, so its absolute error is ~ 1e-6
# ybar while its size is ~ sqrt(y) (noise).  Normwise the gradient therefore
# carries a relative error ~ 1e-6 sqrt(max y) ~ 2e-4 at 5e4 counts; 2e-3
# leaves an order of magnitude.  Curvatures and objectives have no
# cancellation: 1e-5.
TOL_GRAD = 2e-3
TOL_CURV = 1e-5
TOL_OBJ = 1e-5

CASES = {
    "c1": lambda: C.make_c1(),
    "fan64_huber": lambda: C.make_small_fan(n=64, views=90, bins=128, penalty="huber"),
    "fan64_quad": lambda: C.make_small_fan(n=64, views=90, bins=128, penalty="quadratic"),
    "mbmd32_3mat": lambda: C.make_small_mbmd(n=32, views=60, bins=64, n_mat=3),
    "mbmd32_2mat": lambda: C.make_small_mbmd(n=32, views=60, bins=64, n_mat=2),
    "identity_c3": lambda: C.make_c3(n_views=24, n_bins=40),
}


def _x_for(wl):
    rng = np.random.default_rng(10)
    return wl.x_true * rng.uniform(0.7, 1.1, size=wl.x_true.shape)


@pytest.mark.parametrize("case", sorted(CASES))
def test_gradient_curvature_objective(case):
    wl = CASES[case]()
    op = oracle.OracleProblem.from_workload(wl)
    x = _x_for(wl)
    announce("gradient", case)
    P = mb.Problem.from_workload(wl)
    g, d, phi = P.gradient(dev(x), curvature=True, objective=True)
    g, d = host(g), host(d)
    g_want = model.gradient(op, x)
    gL, dL = sps.surrogate_terms(op, x)
    d_want = dL + pen.sps_curvature(op, x)
    phi_want = model.objective(op, x)
    assert l2rel(g, g_want) <= TOL_GRAD, l2rel(g, g_want)
    assert maxrel(d, d_want) <= TOL_CURV, maxrel(d, d_want)
    assert abs(phi - phi_want) <= TOL_OBJ * abs(phi_want), (phi, phi_want)


def test_gradient_at_zero_matches():
    """x = 0: every transmission is 1 (the largest counts); no cancellation
    beyond the residual."""
    wl = C.make_small_fan(n=64, views=90, bins=128)
    op = oracle.OracleProblem.from_workload(wl)
    x = np.zeros(wl.x_true.shape)
    announce("gradient at 0")
    P = mb.Problem.from_workload(wl)
    g, _, phi = P.gradient(dev(x), objective=True)
    assert l2rel(host(g), model.gradient(op, x)) <= 1e-5
    assert abs(phi - model.objective(op, x)) <= TOL_OBJ * model.objective(op, x)
