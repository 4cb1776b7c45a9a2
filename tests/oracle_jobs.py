"""FP64 oracle runs for the full-size parity tests, executed in worker
processes (spawned: no GPU, no torch) so that they overlap the GPU work.

Each job receives the problem as arrays (the workload is generated once, in
the test process) and returns the oracle's iterate after n iterations, with
the objective trace or only its last value.
"""

from __future__ import annotations

import numpy as np

import oracle
from oracle import model, precond, projector, sps


def run_sps(geom, Q, S, y, w, penalty, kind, n_iter, trace=False, threads=1):
    """(x after n_iter iterations, objective trace [n_iter + 1] or [Phi(x)])."""
    projector.set_threads(threads)
    prob = oracle.OracleProblem(geom, Q, S, y, w, penalty)
    if kind == "none":
        x, phi = sps.sps_plain(prob, n_iter, trace=trace)
    else:
        x, phi, _ = sps.sps_precond(prob, precond.build(prob, kind), n_iter, trace=trace)
    if not trace:
        phi = np.array([model.objective(prob, x)])
    return x, np.asarray(phi)
