"""FP64 CPU oracle for preconditioned SPS / model-based material decomposition.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import, call or link anything in
this package.  The GPU library never routes through it, and the two share no
code: the oracle has its own projector (``dd_oracle.c``), its own FFT usage
(NumPy), its own Haar transform and its own eigen-solves (NumPy LAPACK).

Every function follows the paper (Tivnan, Wang & Stayman, "A Preconditioned
Algorithm for Model-Based Iterative CT Reconstruction and Material
Decomposition from Spectral CT Data", arXiv 2010.01371) step by step, in
float64, without blocking, fusion or reordering beyond what the equations
state.  Where the paper is silent or garbled, the readings listed in the
module docstrings are used.

Pinned by ``tests/test_oracle_*.py`` against closed forms, invariants,
library routines and brute force.  Functions that no such test pins say
"parity unpinned" in their docstring.
"""

from .problem import OracleProblem  # noqa: F401
from . import projector, model, penalty, precond, sps, haar  # noqa: F401
