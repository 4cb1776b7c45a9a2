"""Python front of the C-ABI in include/mbmd.h (argument marshalling only).

Torch supplies device memory and the stream; every step of the method runs in
the HIP kernels of libmbmd.so.  Geometries are dicts with the fields of
``mbmd_geometry`` (``kind`` as 'parallel' | 'fan' | 'identity').
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check

KINDS = {"parallel": 0, "fan": 1, "identity": 2}
PRECONDS = {"none": 0, "fourier": 1, "haar": 2, "blockdiag": 3, "daub4": 4}
PRECOND_UNMODIFIED = 1          # mbmd_precond_flags
PENALTIES = {"quadratic": 0, "huber": 1}
WORKSPACE_BLUR = 1              # mbmd_workspace_flags
# mbmd_numeric_flags
FLAG_NONFINITE, FLAG_NO_CURVATURE, FLAG_ASCENT, FLAG_INCREASE = 1, 2, 4, 8


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _dev_f32(t, shape=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != torch.float32:
        raise TypeError("%s must be float32" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return t


def geometry_struct(g):
    k = g["kind"]
    return _lib.Geometry(KINDS[k] if isinstance(k, str) else int(k), int(g["nx"]), int(g["ny"]),
                         float(g.get("dx", 1.0)), float(g.get("dy", 1.0)), int(g["n_views"]),
                         float(g.get("theta0", 0.0)), float(g.get("dtheta", 0.0)), int(g["n_bins"]),
                         float(g.get("du", 1.0)), float(g.get("u_offset", 0.0)), float(g.get("dso", 0.0)),
                         float(g.get("dsd", 0.0)))


def project(geom, x):
    """A x for x [n_mat, ny, nx] (float32, on the GPU) -> [n_mat, V, B]."""
    lib = _lib.load()
    x = x if x.dim() == 3 else x.unsqueeze(0)
    _dev_f32(x, (x.shape[0], geom["ny"], geom["nx"]), "x")
    out = torch.empty((x.shape[0], geom["n_views"], geom["n_bins"]), device=x.device, dtype=torch.float32)
    g = geometry_struct(geom)
    check(lib.mbmd_project(ctypes.byref(g), _ptr(x), _ptr(out), x.shape[0], _stream()), "mbmd_project")
    return out


def backproject(geom, sino):
    """A^T s for s [n_ch, V, B] -> [n_ch, ny, nx]."""
    lib = _lib.load()
    sino = sino if sino.dim() == 3 else sino.unsqueeze(0)
    _dev_f32(sino, (sino.shape[0], geom["n_views"], geom["n_bins"]), "sino")
    out = torch.empty((sino.shape[0], geom["ny"], geom["nx"]), device=sino.device, dtype=torch.float32)
    g = geometry_struct(geom)
    check(lib.mbmd_backproject(ctypes.byref(g), _ptr(sino), _ptr(out), sino.shape[0], _stream()),
          "mbmd_backproject")
    return out


def cache_clear():
    """mbmd_cache_clear: free the standalone projector calls' cached tables."""
    check(_lib.load().mbmd_cache_clear(), "mbmd_cache_clear")


def _spectral_struct(Q, S):
    return _lib.Spectral(Q.shape[1], Q.shape[0], S.shape[0], Q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         S.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))


def workspace_bytes(geom, Q, S, flags=0):
    """mbmd_workspace_bytes: device bytes of a problem's state."""
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    g = geometry_struct(geom)
    sp = _spectral_struct(Q, S)
    n = ctypes.c_size_t(0)
    check(_lib.load().mbmd_workspace_bytes(ctypes.byref(g), ctypes.byref(sp), int(flags), ctypes.byref(n)),
          "mbmd_workspace_bytes")
    return int(n.value)


def projector_nnz(geom):
    """Nonzeros of A for a geometry (counted on the GPU from the projector tables)."""
    lib = _lib.load()
    g = geometry_struct(geom)
    n = ctypes.c_longlong(0)
    check(lib.mbmd_projector_nnz(ctypes.byref(g), ctypes.byref(n), _stream()), "mbmd_projector_nnz")
    return int(n.value)


class Problem:
    """A PWLS / MBMD estimation problem living on the GPU.

    workspace: "torch" (default) passes a torch uint8 tensor of
    mbmd_workspace_bytes as the problem's device memory, so torch owns it;
    None lets the library allocate it; or a CUDA uint8 tensor to use.
    blur_room: size the workspace for a projection-domain blur (set_blur);
    by default only a torch-made workspace is (a library block grows on demand).
    """

    def __init__(self, geom, Q, S, y, w=None, penalty=None, device="cuda", workspace="torch", blur_room=None):
        lib = _lib.load()
        self.geom = dict(geom)
        Q = np.ascontiguousarray(Q, dtype=np.float64)
        S = np.ascontiguousarray(S, dtype=np.float64)
        self.n_energy, self.n_mat = Q.shape
        self.n_chan = S.shape[0]
        self.image_shape = (self.n_mat, geom["ny"], geom["nx"])
        self.sino_shape = (geom["n_views"], geom["n_bins"])
        penalty = penalty or dict(kind="quadratic", beta=np.zeros((self.n_mat, self.n_mat)), delta=0.0)
        beta = np.ascontiguousarray(penalty.get("beta", np.zeros((self.n_mat, self.n_mat))), dtype=np.float64)
        if not torch.is_tensor(y):
            y = torch.as_tensor(np.asarray(y, dtype=np.float32), device=device)
        y = _dev_f32(y.contiguous(), (self.n_chan,) + self.sino_shape, "y")
        if w is not None:
            if not torch.is_tensor(w):
                w = torch.as_tensor(np.asarray(w, dtype=np.float32), device=device)
            w = _dev_f32(w.contiguous(), (self.n_chan,) + self.sino_shape, "w")
        self.device = y.device
        g = geometry_struct(geom)
        sp = _spectral_struct(Q, S)
        pen = _lib.Penalty(PENALTIES[penalty.get("kind", "quadratic")],
                           beta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(penalty.get("delta", 0.0)))
        made_by_torch = isinstance(workspace, str) and workspace == "torch"
        if blur_room is None:
            blur_room = made_by_torch
        flags = WORKSPACE_BLUR if blur_room else 0
        if made_by_torch:
            workspace = torch.empty(workspace_bytes(geom, Q, S, flags), dtype=torch.uint8, device=self.device)
        if workspace is not None and (not torch.is_tensor(workspace) or not workspace.is_cuda
                                      or workspace.dtype != torch.uint8 or not workspace.is_contiguous()):
            raise TypeError("workspace must be a contiguous CUDA uint8 tensor, 'torch' or None")
        self._ws = workspace
        h = ctypes.c_void_p()
        check(lib.mbmd_problem_create(ctypes.byref(g), ctypes.byref(sp), ctypes.byref(pen), _ptr(y),
                                      _ptr(w) if w is not None else None,
                                      _ptr(workspace) if workspace is not None else None,
                                      workspace.numel() if workspace is not None else 0, flags, _stream(),
                                      ctypes.byref(h)),
              "mbmd_problem_create")
        self._h = h
        self._lib = lib

    @classmethod
    def from_workload(cls, wl, device="cuda", **kw):
        """A problem from a workload's arrays; keyword arguments named like the
        constructor's data arguments (Q, S, y, w, penalty) replace the workload's."""
        data = dict(geom=wl.geom, Q=wl.Q, S=wl.S, y=wl.y, w=wl.w, penalty=wl.penalty)
        for k in list(kw):
            if k in data:
                data[k] = kw.pop(k)
        return cls(device=device, **data, **kw)

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "_batches", 0):
            raise RuntimeError("this problem belongs to %d open batch(es): close them first" % self._batches)
        if getattr(self, "_h", None):
            self._lib.mbmd_problem_destroy(self._h)
            self._h = None
        self._ws = None                  # the workspace outlives the problem

    def check(self):
        """mbmd_problem_check: the numeric flags raised since the last read
        (cleared); raises MbmdError (MBMD_ERR_NUMERIC) on a failure flag."""
        f = ctypes.c_int(0)
        check(self._lib.mbmd_problem_check(self._h, ctypes.byref(f), _stream()), "mbmd_problem_check")
        return int(f.value)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def zeros_image(self):
        return torch.zeros(self.image_shape, device=self.device, dtype=torch.float32)

    def set_blur(self, taps=None):
        """mbmd_problem_set_blur: taps [n_chan, 2 h + 1] (one row is used for
        every channel), or None to remove the blur."""
        if taps is None:
            check(self._lib.mbmd_problem_set_blur(self._h, None, 0, _stream()), "mbmd_problem_set_blur")
            return
        t = np.atleast_2d(np.asarray(taps, dtype=np.float32))
        if t.shape[0] == 1 and self.n_chan > 1:
            t = np.repeat(t, self.n_chan, axis=0)
        if t.ndim != 2 or t.shape[0] != self.n_chan or t.shape[1] % 2 != 1:
            raise ValueError("blur taps must be [n_chan, 2h+1], got %s" % (t.shape,))
        t = np.ascontiguousarray(t)
        check(self._lib.mbmd_problem_set_blur(self._h, t.ctypes.data_as(ctypes.c_void_p), (t.shape[1] - 1) // 2,
                                              _stream()), "mbmd_problem_set_blur")

    def precond_build(self, kind, modified=True, x_ref=None):
        """mbmd_precond_build, or mbmd_precond_build_ex with M0 = I
        (modified=False) and / or the Fisher weights at the image x_ref."""
        if modified and x_ref is None:
            check(self._lib.mbmd_precond_build(self._h, PRECONDS[kind], _stream()), "mbmd_precond_build")
            return
        if x_ref is not None:
            _dev_f32(x_ref, self.image_shape, "x_ref")
        flags = 0 if modified else PRECOND_UNMODIFIED
        check(self._lib.mbmd_precond_build_ex(self._h, PRECONDS[kind], flags,
                                              _ptr(x_ref) if x_ref is not None else None, _stream()),
              "mbmd_precond_build_ex")

    def precond_apply(self, kind, g):
        _dev_f32(g, self.image_shape, "g")
        out = torch.empty_like(g)
        check(self._lib.mbmd_precond_apply(self._h, PRECONDS[kind], _ptr(g), _ptr(out), _stream()),
              "mbmd_precond_apply")
        return out

    def gradient(self, x, curvature=False, objective=False):
        _dev_f32(x, self.image_shape, "x")
        g = torch.empty_like(x)
        d = torch.empty_like(x) if curvature else None
        phi = ctypes.c_double(0.0)
        check(self._lib.mbmd_gradient(self._h, _ptr(x), _ptr(g), _ptr(d) if d is not None else None,
                                      ctypes.byref(phi) if objective else None, _stream()), "mbmd_gradient")
        return g, d, (phi.value if objective else None)

    def sps_step(self, x, precond="none", n_iter=1, trace=False):
        """Run n_iter iterations in place on x; returns the objective trace (n_iter+1) or None."""
        _dev_f32(x, self.image_shape, "x")
        tr = np.zeros(n_iter + 1) if trace else None
        ptr = tr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if trace else None
        check(self._lib.mbmd_sps_step(self._h, _ptr(x), PRECONDS[precond], int(n_iter), ptr, _stream()),
              "mbmd_sps_step")
        return tr

    def forward(self, x, keep_l=True):
        _dev_f32(x, self.image_shape, "x")
        ybar = torch.empty((self.n_chan,) + self.sino_shape, device=x.device, dtype=torch.float32)
        l = torch.empty((self.n_mat,) + self.sino_shape, device=x.device, dtype=torch.float32) if keep_l else None
        check(self._lib.mbmd_forward(self._h, _ptr(x), _ptr(ybar), _ptr(l) if keep_l else None, _stream()),
              "mbmd_forward")
        return ybar, l

    def forward_vjp(self, l, gbar):
        _dev_f32(l, (self.n_mat,) + self.sino_shape, "l")
        _dev_f32(gbar, (self.n_chan,) + self.sino_shape, "gbar")
        dx = torch.empty(self.image_shape, device=l.device, dtype=torch.float32)
        check(self._lib.mbmd_forward_vjp(self._h, _ptr(l), _ptr(gbar), _ptr(dx), _stream()), "mbmd_forward_vjp")
        return dx


class Batch:
    """Several problems iterated together (optionally as one hipGraph per iteration).

    shared=True lets problems with equal launch parameters share every kernel
    launch of the plain, Fourier and block-diagonal iterations (one workgroup
    grid over all members); shared=False gives each problem launches of its
    own.  workspace="torch" puts the batch's table of per-member offsets in a
    torch allocation held by this object; None lets the library allocate it."""

    BATCH_SEPARATE_LAUNCHES = 1

    def __init__(self, problems, shared=True, workspace="torch"):
        self.problems = list(problems)
        lib = _lib.load()
        n = len(self.problems)
        arr = (ctypes.c_void_p * n)(*[p._h for p in self.problems])
        self._ws = None
        ws_ptr, ws_bytes = None, 0
        if workspace == "torch":
            nb = ctypes.c_size_t()
            check(lib.mbmd_batch_workspace_bytes(arr, n, ctypes.byref(nb)), "mbmd_batch_workspace_bytes")
            ws_bytes = nb.value
            dev = torch.device("cuda", torch.cuda.current_device())
            self._ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
            ws_ptr = (self._ws.data_ptr() + 255) // 256 * 256
        elif workspace is not None:
            raise ValueError("workspace must be 'torch' or None")
        flags = 0 if shared else self.BATCH_SEPARATE_LAUNCHES
        h = ctypes.c_void_p()
        check(lib.mbmd_batch_create(arr, n, ws_ptr, ws_bytes, flags, ctypes.byref(h)), "mbmd_batch_create")
        self._h = h
        self._lib = lib
        for p in self.problems:              # the C batch borrows them: no close while it is open
            p._batches = getattr(p, "_batches", 0) + 1

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mbmd_batch_destroy(self._h)
            self._h = None
            for p in self.problems:
                p._batches -= 1

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sps_step(self, xs, precond="fourier", n_iter=1, use_graph=True):
        for p, x in zip(self.problems, xs):
            _dev_f32(x, p.image_shape, "x")
        arr = (ctypes.c_void_p * len(xs))(*[x.data_ptr() for x in xs])
        check(self._lib.mbmd_batch_sps_step(self._h, arr, PRECONDS[precond], int(n_iter), int(bool(use_graph)),
                                            _stream()), "mbmd_batch_sps_step")


class KernelProfile:
    """Per-kernel HIP-event timing of the library's launches (see mbmd_profile_*)."""

    def __init__(self, only=None):
        self._lib = _lib.load()
        self._only = ",".join(only) if only else ""

    def __enter__(self):
        check(self._lib.mbmd_profile_reset(), "mbmd_profile_reset")
        check(self._lib.mbmd_profile_select(self._only.encode()), "mbmd_profile_select")
        check(self._lib.mbmd_profile_enable(1), "mbmd_profile_enable")
        return self

    def __exit__(self, *exc):
        self._lib.mbmd_profile_enable(0)
        self._lib.mbmd_profile_select(b"")
        return False

    def kernels(self):
        buf = ctypes.create_string_buffer(1 << 16)
        check(self._lib.mbmd_profile_kernels(buf, len(buf)), "mbmd_profile_kernels")
        return [k for k in buf.value.decode().split(",") if k]

    def query(self, name):
        n = ctypes.c_longlong(0)
        ms = ctypes.c_double(0.0)
        check(self._lib.mbmd_profile_query(name.encode(), ctypes.byref(n), ctypes.byref(ms)), "mbmd_profile_query")
        return int(n.value), float(ms.value)

    def table(self):
        return {k: self.query(k) for k in self.kernels()}
