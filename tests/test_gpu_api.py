"""The boundary's device-memory and failure conventions on the GPU: a problem
carved from a caller-owned (torch) workspace allocates nothing and iterates
bit for bit like one in library memory; workspace size, alignment and blur-room
errors; numeric failures (non-finite data, no positive curvature along the
direction) surface as MBMD_ERR_NUMERIC at the synchronizing calls; an iterate
saved to the host resumes bit for bit in a fresh problem; the standalone
projector calls on two streams at once."""

import ctypes

import numpy as np
import pytest
import torch

from gpu_util import announce, dev, host
from workloads import configs as C

import paper_2010_01371_amd as mb
from paper_2010_01371_amd import _lib, api

pytestmark = pytest.mark.gpu

MBMD_ERR_ARG, MBMD_ERR_NUMERIC, MBMD_ERR_UNSUPPORTED = -1, -5, -6


def _fan():
    return C.make_small_fan(n=64, views=90, bins=128, penalty="huber")


def _status(excinfo):
    return excinfo.value.status


def test_caller_workspace_allocates_nothing_and_matches_library_memory():
    wl = C.make_small_fan(n=128, views=120, bins=200, penalty="huber")
    announce("workspace: library vs caller memory")
    P_lib = mb.Problem.from_workload(wl, workspace=None)
    for kind in ("fourier", "haar"):                  # first launches load every kernel used below
        P_lib.precond_build(kind)
    x_lib = P_lib.zeros_image()
    P_lib.sps_step(x_lib, "fourier", 20)
    P_lib.sps_step(P_lib.zeros_image(), "haar", 2)
    P_lib.sps_step(P_lib.zeros_image(), "none", 2)
    nbytes = mb.workspace_bytes(wl.geom, wl.Q, wl.S)
    # every torch tensor the second problem uses exists before the measurement
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    y, w, x_ws = dev(wl.y), dev(wl.w), P_lib.zeros_image()
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    P_ws = mb.Problem(wl.geom, wl.Q, wl.S, y, w, wl.penalty, workspace=ws)
    P_ws.precond_build("fourier")
    P_ws.sps_step(x_ws, "fourier", 20)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free0 - free1 < nbytes // 4, (free0 - free1, nbytes)
    np.testing.assert_array_equal(host(x_ws), host(x_lib))
    P_ws.close()
    # without a workspace the library allocates a block of that size itself
    torch.cuda.synchronize()
    free2, _ = torch.cuda.mem_get_info()
    P_new = mb.Problem(wl.geom, wl.Q, wl.S, y, w, wl.penalty, workspace=None)
    torch.cuda.synchronize()
    free3, _ = torch.cuda.mem_get_info()
    assert free2 - free3 >= nbytes - (64 << 10), (free2 - free3, nbytes)
    P_new.close()
    P_lib.close()


def test_workspace_size_alignment_and_blur_room():
    wl = _fan()
    nbytes = mb.workspace_bytes(wl.geom, wl.Q, wl.S)
    nblur = mb.workspace_bytes(wl.geom, wl.Q, wl.S, flags=api.WORKSPACE_BLUR)
    assert nblur > nbytes
    announce("workspace errors")
    with pytest.raises(_lib.MbmdError) as e:
        mb.Problem.from_workload(wl, workspace=torch.empty(nbytes - 256, dtype=torch.uint8, device="cuda"))
    assert _status(e) == MBMD_ERR_ARG
    big = torch.empty(nbytes + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(_lib.MbmdError) as e:
        mb.Problem.from_workload(wl, workspace=big[16:])             # not 256-byte aligned
    assert _status(e) == MBMD_ERR_ARG
    P = mb.Problem.from_workload(wl, workspace=torch.empty(nbytes, dtype=torch.uint8, device="cuda"),
                                 blur_room=False)
    with pytest.raises(_lib.MbmdError) as e:
        P.set_blur([[0.25, 0.5, 0.25]])
    assert _status(e) == MBMD_ERR_UNSUPPORTED
    P.close()
    # with room for the blur, a caller workspace gives the library-memory results
    out = []
    for ws in ("torch", None):
        Q = mb.Problem.from_workload(wl, workspace=ws)            # torch: with blur room (the default)
        Q.set_blur([[0.25, 0.5, 0.25]])
        Q.precond_build("fourier")
        x = Q.zeros_image()
        Q.sps_step(x, "fourier", 10)
        out.append(host(x))
        Q.close()
    np.testing.assert_array_equal(out[0], out[1])


@pytest.mark.parametrize("kind", ["none", "fourier"])
def test_non_finite_data_is_a_numeric_failure(kind):
    """A NaN count makes the objective and the step non-finite: an untraced run
    only enqueues (MBMD_OK), the next synchronizing call reports
    MBMD_ERR_NUMERIC and clears the flag; a traced run reports it itself."""
    wl = _fan()
    y = wl.y.copy()
    y[0, 3, 40] = np.nan
    announce("numeric failure", kind)
    P = mb.Problem(wl.geom, wl.Q, wl.S, y, wl.w, wl.penalty)
    if kind != "none":
        P.precond_build(kind)
    x = P.zeros_image()
    P.sps_step(x, kind, 3)                                 # no error yet
    with pytest.raises(_lib.MbmdError) as e:
        P.check()
    assert _status(e) == MBMD_ERR_NUMERIC
    assert P.check() == 0                                  # read and cleared
    with pytest.raises(_lib.MbmdError) as e:
        P.sps_step(P.zeros_image(), kind, 2, trace=True)
    assert _status(e) == MBMD_ERR_NUMERIC
    with pytest.raises(_lib.MbmdError) as e:
        P.gradient(P.zeros_image(), objective=True)
    assert _status(e) == MBMD_ERR_NUMERIC
    P.close()


def test_negative_curvature_is_a_numeric_failure():
    """A strongly negative quadratic penalty (beta = -1e12: not positive
    semi-definite, which the interface requires but only the symmetry of beta
    is checked) makes the 1D majoriser's curvature sum c q^2 + p^T R'' p
    negative: the step is skipped (x stays at its start, as the oracle's
    alpha = 0) and MBMD_FLAG_NO_CURVATURE surfaces as MBMD_ERR_NUMERIC.  The
    block-diagonal direction does not depend on beta (the penalty's rows sum
    to zero), so the sign of that curvature is certain; the Fourier table of
    such a beta comes from floored negative spectra instead."""
    kind = "blockdiag"
    wl = C.make_small_fan(n=32, views=48, bins=64, penalty="quadratic")
    pen = dict(kind="quadratic", beta=np.array([[-1e12]]), delta=0.0)
    announce("negative curvature", kind)
    P = mb.Problem(wl.geom, wl.Q, wl.S, wl.y, wl.w, pen)
    P.precond_build(kind)
    x = P.zeros_image()
    P.sps_step(x, kind, 2)
    with pytest.raises(_lib.MbmdError) as e:
        P.check()
    assert _status(e) == MBMD_ERR_NUMERIC
    assert "no positive curvature" in str(e.value)
    assert not np.any(host(x))
    P.close()


def test_resume_from_a_saved_iterate():
    """The iteration's whole state between calls is x (each call recomputes the
    line integrals from it; the tables are built deterministically from the
    data): an iterate saved to the host after 12 iterations and resumed in a
    fresh problem ends bit for bit where the uninterrupted two calls end."""
    wl = _fan()
    announce("checkpoint and resume")
    P = mb.Problem.from_workload(wl)
    P.precond_build("fourier")
    x = P.zeros_image()
    P.sps_step(x, "fourier", 12)
    saved = x.detach().cpu().numpy().copy()                 # the checkpoint (FP32, exact)
    P.sps_step(x, "fourier", 13)
    straight = host(x)
    P.close()
    Q = mb.Problem.from_workload(wl)
    Q.precond_build("fourier")
    y = torch.as_tensor(saved, device="cuda")
    Q.sps_step(y, "fourier", 13)
    np.testing.assert_array_equal(host(y), straight)
    Q.close()


def test_healthy_run_raises_no_failure_flag():
    wl = _fan()
    announce("numeric flags, healthy run")
    P = mb.Problem.from_workload(wl)
    P.precond_build("fourier")
    x = P.zeros_image()
    P.sps_step(x, "fourier", 30)
    assert P.check() & (api.FLAG_NONFINITE | api.FLAG_NO_CURVATURE | api.FLAG_ASCENT) == 0
    P.close()


def test_projector_calls_on_two_streams_at_once():
    """Each stream has its own cached scratch: interleaved projections and back
    projections of different inputs on two streams give the single-stream
    results bit for bit."""
    wl = _fan()
    g = wl.geom
    rng = np.random.default_rng(5)
    xs = [dev(rng.uniform(0.0, 0.03, size=(1, g["ny"], g["nx"]))) for _ in range(2)]
    ss = [dev(rng.uniform(0.0, 2.0, size=(1, g["n_views"], g["n_bins"]))) for _ in range(2)]
    announce("projector on two streams")
    want = [(host(mb.project(g, xs[i])), host(mb.backproject(g, ss[i]))) for i in range(2)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    got = [[], []]
    for rep in range(8):
        for i in range(2):
            with torch.cuda.stream(streams[i]):
                got[i].append((mb.project(g, xs[i]), mb.backproject(g, ss[i])))
    torch.cuda.synchronize()
    for i in range(2):
        for a, b in got[i]:
            np.testing.assert_array_equal(host(a), want[i][0])
            np.testing.assert_array_equal(host(b), want[i][1])
    mb.cache_clear()
