"""Seeded synthetic inputs for the preconditioned-SPS / MBMD workloads.

This package is the only code shared by the FP64 oracle tests and the GPU
path.  It holds no arithmetic of the estimation method itself (no projector,
no surrogate, no preconditioner): it draws phantoms, evaluates their exact
(continuous-domain) line integrals, builds synthetic attenuation curves and
source spectra, and simulates noisy measurements of a scanner.  Every random
number is drawn here from NumPy's PCG64 with a stated seed.
"""

from .configs import (  # noqa: F401
    Workload,
    make_c1,
    make_c2,
    make_c3,
    make_c4,
    make_c5,
    make_small_fan,
    make_small_mbmd,
    seed_for,
)
