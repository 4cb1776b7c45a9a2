"""MI355X-native preconditioned SPS for PWLS CT reconstruction and model-based
material decomposition (Tivnan, Wang & Stayman, arXiv 2010.01371).

The compute path is ``libmbmd.so`` (HIP kernels for gfx950, C-ABI in
include/mbmd.h); this package only marshals arguments to it.
"""

from .api import (Batch, KernelProfile, Problem, backproject, cache_clear, project, projector_nnz,  # noqa: F401
                  workspace_bytes, PRECONDS)
from .autograd import PolyForward, poly_forward  # noqa: F401
