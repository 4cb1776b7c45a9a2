"""ctypes front of the FP64 distance-driven projector in ``dd_oracle.c``.

The C file is compiled by :func:`build` (called from ``__graft_entry__.build``
and lazily on first use) with gcc into ``oracle/_dd_oracle.so``.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dd_oracle.c")
_LIB = os.path.join(_HERE, "_dd_oracle.so")
_lib = None

KIND = {"parallel": 0, "fan": 1, "identity": 2}


class _Geom(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("n_views", ctypes.c_int), ("n_bins", ctypes.c_int),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("theta0", ctypes.c_double), ("dtheta", ctypes.c_double),
                ("du", ctypes.c_double), ("u_offset", ctypes.c_double),
                ("dso", ctypes.c_double), ("dsd", ctypes.c_double)]


def build(force=True):
    """Compile the oracle projector with gcc (FP64, OpenMP)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        lib.oracle_ray_weights.argtypes = [P(_Geom), ctypes.c_int, ctypes.c_int,
                                           P(ctypes.c_int), P(ctypes.c_double), ctypes.c_int]
        lib.oracle_ray_weights.restype = ctypes.c_int
        lib.oracle_project.argtypes = [P(_Geom), P(ctypes.c_double), P(ctypes.c_double), ctypes.c_int]
        lib.oracle_project.restype = ctypes.c_int
        lib.oracle_backproject.argtypes = [P(_Geom), P(ctypes.c_double), P(ctypes.c_double), ctypes.c_int]
        lib.oracle_backproject.restype = ctypes.c_int
        lib.oracle_sweeps_rows.argtypes = [P(_Geom), ctypes.c_int]
        lib.oracle_sweeps_rows.restype = ctypes.c_int
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _geom(g):
    return _Geom(KIND[g["kind"]], g["nx"], g["ny"], g["n_views"], g["n_bins"], g["dx"], g["dy"],
                 g["theta0"], g["dtheta"], g["du"], g["u_offset"], g["dso"], g["dsd"])


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def threads():
    return _load().oracle_threads()


def set_threads(n):
    _load().oracle_set_threads(int(n))


def sweeps_rows(g, v):
    return bool(_load().oracle_sweeps_rows(ctypes.byref(_geom(g)), int(v)))


def ray_weights(g, v, b):
    """(flat pixel indices, weights) of row (v, b) of A."""
    cap = (g["nx"] + 2) * (g["ny"] + 2)
    idx = np.zeros(cap, dtype=np.int32)
    wt = np.zeros(cap)
    n = _load().oracle_ray_weights(ctypes.byref(_geom(g)), int(v), int(b),
                                   idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dptr(wt), cap)
    if n < 0:
        raise ValueError("ray (%d, %d) is degenerate for this geometry" % (v, b))
    return idx[:n].copy(), wt[:n].copy()


def project(g, x):
    """A x for x of shape [n_mat, ny, nx] (or [ny, nx]); returns [n_mat, V, B]."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    squeeze = x.ndim == 2
    if squeeze:
        x = x[None]
    out = np.zeros((x.shape[0], g["n_views"], g["n_bins"]))
    if g["kind"] == "identity":
        out[:] = x.reshape(out.shape)
    elif _load().oracle_project(ctypes.byref(_geom(g)), _dptr(x), _dptr(out), x.shape[0]) != 0:
        raise ValueError("degenerate ray in projection")
    return out[0] if squeeze else out


def backproject(g, s):
    """A^T s for s of shape [n_mat, V, B] (or [V, B]); returns [n_mat, ny, nx]."""
    s = np.ascontiguousarray(s, dtype=np.float64)
    squeeze = s.ndim == 2
    if squeeze:
        s = s[None]
    out = np.zeros((s.shape[0], g["ny"], g["nx"]))
    if g["kind"] == "identity":
        out[:] = s.reshape(out.shape)
    elif _load().oracle_backproject(ctypes.byref(_geom(g)), _dptr(s), _dptr(out), s.shape[0]) != 0:
        raise ValueError("degenerate ray in backprojection")
    return out[0] if squeeze else out


def dense_matrix(g):
    """The full system matrix A [V*B, ny*nx] (small geometries only)."""
    nj = g["nx"] * g["ny"]
    A = np.zeros((g["n_views"] * g["n_bins"], nj))
    for v in range(g["n_views"]):
        for b in range(g["n_bins"]):
            idx, wt = ray_weights(g, v, b)
            np.add.at(A[v * g["n_bins"] + b], idx, wt)
    return A
