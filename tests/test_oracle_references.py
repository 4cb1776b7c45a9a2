"""CPU checks of the stored references and of the sensitivity that fixes how
long iterates can be compared step by step (oracle only, no GPU values).

* tests/golden/newton_xhat_*.npz (written by make_newton_references.py with
  the oracle alone) are minimisers of the oracle's objective: the gradient
  vanishes there relative to its size at zero, and no random nearby point is
  lower.
* The cross-material wavelet iterations of the 32x32 three-material problem
  are sensitive in exact arithmetic: a relative 1e-7 perturbation of the FP64
  iterate after every iteration grows beyond 1e-3 within 50 iterations,
  whereas the Fourier and block-diagonal iterations keep it below 1e-5.  So no
  implementation in other arithmetic can follow the wavelet iterations step
  by step much beyond 10 iterations, and they are compared with the oracle
  at their common limit instead.
"""

import os

import numpy as np
import pytest

import oracle
from oracle import model, precond, projector, sps
from workloads import configs as C

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _workload(name):
    if name == "c1":
        return C.make_c1()
    return C.make_small_mbmd(n=32, views=60, bins=64, n_mat=3, seed_slice=int(name[len("mbmd32_s"):]))


@pytest.mark.parametrize("name", ["c1", "mbmd32_s50", "mbmd32_s51", "mbmd32_s52"])
def test_stored_newton_references_are_minimisers(name):
    ref = np.load(os.path.join(GOLDEN, "newton_xhat_%s.npz" % name))
    prob = oracle.OracleProblem.from_workload(_workload(name))
    xhat = ref["xhat"]
    assert xhat.shape == prob.image_shape
    g = model.gradient(prob, xhat)
    g0 = model.gradient(prob, np.zeros_like(xhat))
    assert np.linalg.norm(g) <= 1e-9 * np.linalg.norm(g0)
    phi = model.objective(prob, xhat)
    np.testing.assert_allclose(phi, float(ref["objective"]), rtol=1e-12)
    assert float(ref["eig_min"]) > 0.0
    rng = np.random.default_rng(1)
    for _ in range(4):
        d = rng.normal(size=xhat.shape) * 1e-3 * np.abs(xhat).max()
        assert model.objective(prob, xhat + d) > phi


def _growth(prob, tab, n, eps=1e-7, seed=0):
    rng = np.random.default_rng(seed)
    x = np.zeros(prob.image_shape)
    xp = x.copy()
    worst = 0.0
    for _ in range(n):
        x, _ = sps.precond_step(prob, x, tab)
        xp, _ = sps.precond_step(prob, xp, tab)
        xp = xp * (1.0 + eps * rng.standard_normal(xp.shape))
        worst = max(worst, float(np.linalg.norm(xp - x) / np.linalg.norm(x)))
    return worst


def test_wavelet_iterations_are_sensitive_and_fourier_is_not():
    threads = projector.threads()
    projector.set_threads(1)
    try:
        prob = oracle.OracleProblem.from_workload(_workload("mbmd32_s50"))
        grow = {k: _growth(prob, precond.build(prob, k), 50) for k in ("fourier", "blockdiag", "haar", "daub4")}
    finally:
        projector.set_threads(threads)
    assert grow["fourier"] < 1e-5 and grow["blockdiag"] < 1e-5, grow
    assert grow["haar"] > 1e-3 and grow["daub4"] > 1e-3, grow
