"""GPU parity of the polyenergetic forward model and its hand-written
backward (mbmd_forward / mbmd_forward_vjp, torch.autograd.Function)."""

import numpy as np
import pytest
import torch

import oracle
from gpu_util import announce, dev, host, l2rel, maxrel
from oracle import model
from workloads import configs as C

import paper_2010_01371_amd as mb

pytestmark = pytest.mark.gpu

CASES = {
    "mbmd32_3mat": lambda: C.make_small_mbmd(n=32, views=60, bins=64, n_mat=3),
    "fan64": lambda: C.make_small_fan(n=64, views=90, bins=128),
    "c3_identity": lambda: C.make_c3(n_views=24, n_bins=40),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_forward_and_backward_match_oracle(case):
    wl = CASES[case]()
    op = oracle.OracleProblem.from_workload(wl)
    x = wl.x_true * 0.9
    gbar = np.random.default_rng(20).normal(size=wl.y.shape)
    announce("autograd", case)
    P = mb.Problem.from_workload(wl)
    xt = dev(x).requires_grad_(True)
    ybar = mb.poly_forward(xt, P)
    (ybar * dev(gbar)).sum().backward()
    assert maxrel(host(ybar), model.forward(op, x)) <= 1e-5
    want = model.forward_vjp(op, x, gbar)
    assert l2rel(host(xt.grad), want) <= 1e-5, l2rel(host(xt.grad), want)


def test_autograd_gradient_of_wls_loss_matches_objective_gradient():
    """d/dx of 1/2 sum w (y - ybar)^2 through the autograd function equals the
    oracle's data gradient."""
    wl = C.make_small_mbmd(n=32, views=60, bins=64, n_mat=2)
    op = oracle.OracleProblem.from_workload(wl)
    x = wl.x_true * 1.05
    announce("autograd wls")
    P = mb.Problem.from_workload(wl)
    xt = dev(x).requires_grad_(True)
    y, w = dev(wl.y), dev(wl.w)
    ybar = mb.poly_forward(xt, P)
    loss = 0.5 * (w.double() * (y.double() - ybar.double()) ** 2).sum()
    loss.backward()
    assert l2rel(host(xt.grad), model.data_gradient(op, x)) <= 2e-3


def test_no_ray_energy_tensor_is_saved():
    wl = C.make_small_mbmd(n=32, views=60, bins=64, n_mat=3)
    P = mb.Problem.from_workload(wl)
    xt = dev(wl.x_true).requires_grad_(True)
    ybar = mb.poly_forward(xt, P)
    saved = ybar.grad_fn.saved_tensors
    assert len(saved) == 1 and tuple(saved[0].shape) == (3,) + P.sino_shape
