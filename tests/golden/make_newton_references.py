"""Writes the Newton minimisers x_hat stored beside this script, with the FP64
oracle only (oracle.newton: damped Newton with the exact dense Hessian, from
a start given by the oracle's own block-diagonal SPS iterations).

x_hat = argmin Phi (eq:mapEstimator) is the point every SPS variant of
"Preconditioned Optimization" converges to (any invertible M leaves it
unchanged); the GPU tests compare converged iterates with it, and the
time-to-RMSE measurement uses it as the reference.

Usage: python tests/golden/make_newton_references.py [name ...]
Each output newton_xhat_<name>.npz holds x_hat [N_k, ny, nx] (float64), the
final gradient norm, the gradient norm at x = 0, the smallest and largest
Hessian eigenvalues at x_hat, the objective there and the Newton steps.
"""

from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import model, newton, precond, projector, sps  # noqa: E402
from workloads import configs as C  # noqa: E402


def workload(name):
    """The workloads with stored minimisers (names as in the file names)."""
    if name == "c1":
        return C.make_c1()
    if name.startswith("mbmd32_s"):
        return C.make_small_mbmd(n=32, views=60, bins=64, n_mat=3, seed_slice=int(name[len("mbmd32_s"):]))
    raise ValueError(name)


NAMES = ["c1", "mbmd32_s50", "mbmd32_s51", "mbmd32_s52"]


def make(name, start_iters=300):
    wl = workload(name)
    prob = oracle.OracleProblem.from_workload(wl)
    t0 = time.time()
    x0, _, _ = sps.sps_precond(prob, precond.build(prob, "blockdiag"), start_iters, trace=False)
    xhat, H, gnorm, steps = newton.minimise(prob, x0, max_iter=200, gtol=1e-13)
    g0 = float(np.linalg.norm(model.gradient(prob, np.zeros(prob.image_shape))))
    ev = np.linalg.eigvalsh(H)
    out = os.path.join(HERE, "newton_xhat_%s.npz" % name)
    np.savez_compressed(out, xhat=xhat, gnorm=gnorm, gnorm0=g0, eig_min=ev[0], eig_max=ev[-1],
                        objective=model.objective(prob, xhat), steps=steps)
    print("%s: %d Newton steps, |g|/|g0| = %.2e, Hessian eigenvalues [%.3e, %.3e], %.1f s"
          % (name, steps, gnorm / g0, ev[0], ev[-1], time.time() - t0), flush=True)


if __name__ == "__main__":
    projector.set_threads(min(projector.threads(), 8))
    for n in sys.argv[1:] or NAMES:
        make(n)
