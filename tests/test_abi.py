"""The C-ABI library loads and exports every symbol include/mbmd.h declares
(CPU only: no compute calls)."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mbmd.h")
LIB = os.path.join(ROOT, "paper_2010_01371_amd", "libmbmd.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mbmd_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary_calls():
    names = declared()
    for want in ("mbmd_project", "mbmd_backproject", "mbmd_gradient", "mbmd_sps_step",
                 "mbmd_precond_build", "mbmd_forward", "mbmd_forward_vjp", "mbmd_batch_sps_step"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmbmd.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(mbmd_[a-z_0-9]+)", out))
    assert set(declared()) <= exported


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmbmd.so not built (run __graft_entry__.build())")
def test_python_binding_signatures_cover_the_header():
    from paper_2010_01371_amd import _lib
    assert set(declared()) == set(_lib._SIGNATURES)
    lib = _lib.load()
    assert lib.mbmd_version() == 1
    assert lib.mbmd_status_string(-5) == b"non-finite objective or step"


def test_binding_has_no_cpu_fallback():
    """The package imports nothing from the oracle and has no compute path in Python."""
    pkg = os.path.join(ROOT, "paper_2010_01371_amd")
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            text = open(os.path.join(pkg, f)).read()
            assert "oracle" not in text.replace("the oracle", ""), f
            assert "workloads" not in text, f


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmbmd.so not built (run __graft_entry__.build())")
def test_workspace_bytes_without_a_gpu():
    """mbmd_workspace_bytes is host arithmetic: it sizes a problem's device block
    (geometry tables, state, scratch), grows with the blur's room, and rejects
    unknown flags and bad sizes, all without touching a device."""
    import numpy as np
    from paper_2010_01371_amd import api, _lib
    from workloads import configs as C
    wl = C.make_small_fan(n=32, views=48, bins=64)
    n0 = api.workspace_bytes(wl.geom, wl.Q, wl.S)
    n1 = api.workspace_bytes(wl.geom, wl.Q, wl.S, flags=api.WORKSPACE_BLUR)
    V, B = wl.geom["n_views"], wl.geom["n_bins"]
    assert n1 - n0 >= 4 * 4 * V * B                      # (3 + n_mat) n_chan rays floats
    assert n0 > 8 * 6 * 16384                              # the FP64 partial sums alone
    g2 = dict(wl.geom, nx=64, ny=64)
    assert api.workspace_bytes(g2, wl.Q, wl.S) > n0
    with pytest.raises(_lib.MbmdError):
        api.workspace_bytes(wl.geom, wl.Q, wl.S, flags=4)
    with pytest.raises(_lib.MbmdError):
        api.workspace_bytes(dict(wl.geom, nx=0), wl.Q, wl.S)
    Q5 = np.ones((3, 5))
    with pytest.raises(_lib.MbmdError):
        api.workspace_bytes(wl.geom, Q5, np.ones((1, 3)))    # five materials


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmbmd.so not built (run __graft_entry__.build())")
def test_largest_image_is_sized_and_one_more_column_is_refused():
    """The partial-sum buffers hold one sum per 256 pixels or rays in 16384
    slots: 2048 x 2048 pixels is the largest image a problem accepts (its
    workspace is sized on the host), and one more column is MBMD_ERR_SHAPE."""
    import numpy as np
    from paper_2010_01371_amd import api, _lib
    from workloads import configs as C
    g = C.geometry("parallel", 2048, 2048, 0.25, 0.25, 180, np.pi, 2900, 0.25)
    Q, S = np.ones((4, 2)), np.ones((2, 4))
    assert api.workspace_bytes(g, Q, S) > 2 * 2 * 2048 * 2048 * 4
    with pytest.raises(_lib.MbmdError) as e:
        api.workspace_bytes(dict(g, nx=2049), Q, S)
    assert e.value.status == -2
    with pytest.raises(_lib.MbmdError):
        api.workspace_bytes(dict(g, n_views=1447, n_bins=2900), Q, S)   # more than 2^22 rays
