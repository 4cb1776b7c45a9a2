"""ctypes loader of ``libmbmd.so`` (the HIP library built by ``build.py``).

Loading fails loudly: there is no CPU fallback anywhere in this package.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmbmd.so")

c_int, c_double, c_void_p, c_size_t = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
P = ctypes.POINTER


class Geometry(ctypes.Structure):
    _fields_ = [("kind", c_int), ("nx", c_int), ("ny", c_int), ("dx", c_double), ("dy", c_double),
                ("n_views", c_int), ("theta0", c_double), ("dtheta", c_double), ("n_bins", c_int),
                ("du", c_double), ("u_offset", c_double), ("dso", c_double), ("dsd", c_double)]


class Spectral(ctypes.Structure):
    _fields_ = [("n_mat", c_int), ("n_energy", c_int), ("n_chan", c_int),
                ("Q_host", P(c_double)), ("S_host", P(c_double))]


class Penalty(ctypes.Structure):
    _fields_ = [("kind", c_int), ("beta_host", P(c_double)), ("delta", c_double)]


_SIGNATURES = {
    "mbmd_version": (c_int, []),
    "mbmd_last_error": (ctypes.c_char_p, []),
    "mbmd_status_string": (ctypes.c_char_p, [c_int]),
    "mbmd_project": (c_int, [P(Geometry), c_void_p, c_void_p, c_int, c_void_p]),
    "mbmd_backproject": (c_int, [P(Geometry), c_void_p, c_void_p, c_int, c_void_p]),
    "mbmd_project_noalloc": (c_int, [P(Geometry), c_void_p, c_void_p, c_int, c_void_p]),
    "mbmd_workspace_bytes": (c_int, [P(Geometry), P(Spectral), c_int, P(c_size_t)]),
    "mbmd_problem_create": (c_int, [P(Geometry), P(Spectral), P(Penalty), c_void_p, c_void_p, c_void_p,
                                    c_size_t, c_int, c_void_p, P(c_void_p)]),
    "mbmd_problem_destroy": (None, [c_void_p]),
    "mbmd_problem_check": (c_int, [c_void_p, P(c_int), c_void_p]),
    "mbmd_cache_clear": (c_int, []),
    "mbmd_precond_build": (c_int, [c_void_p, c_int, c_void_p]),
    "mbmd_precond_build_ex": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p]),
    "mbmd_problem_set_blur": (c_int, [c_void_p, c_void_p, c_int, c_void_p]),
    "mbmd_precond_apply": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    "mbmd_gradient": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, P(c_double), c_void_p]),
    "mbmd_sps_step": (c_int, [c_void_p, c_void_p, c_int, c_int, P(c_double), c_void_p]),
    "mbmd_forward": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "mbmd_forward_vjp": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "mbmd_batch_workspace_bytes": (c_int, [P(c_void_p), c_int, P(c_size_t)]),
    "mbmd_batch_create": (c_int, [P(c_void_p), c_int, c_void_p, c_size_t, c_int, P(c_void_p)]),
    "mbmd_batch_destroy": (None, [c_void_p]),
    "mbmd_batch_sps_step": (c_int, [c_void_p, P(c_void_p), c_int, c_int, c_int, c_void_p]),
    "mbmd_projector_nnz": (c_int, [P(Geometry), P(ctypes.c_longlong), c_void_p]),
    "mbmd_profile_enable": (c_int, [c_int]),
    "mbmd_profile_reset": (c_int, []),
    "mbmd_profile_select": (c_int, [ctypes.c_char_p]),
    "mbmd_profile_query": (c_int, [ctypes.c_char_p, P(ctypes.c_longlong), P(c_double)]),
    "mbmd_profile_kernels": (c_int, [ctypes.c_char_p, c_size_t]),
}

_lib = None


class MbmdError(RuntimeError):
    def __init__(self, status, where):
        lib = load()
        msg = lib.mbmd_last_error().decode(errors="replace")
        super().__init__("%s failed: %s (%d): %s" % (where, lib.mbmd_status_string(status).decode(), status, msg))
        self.status = status


def load():
    """Load the shared library; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmbmd.so is not built: run paper_2010_01371_amd/build.py "
                              "(or __graft_entry__.build()) first")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status, where):
    if status != 0:
        raise MbmdError(status, where)
