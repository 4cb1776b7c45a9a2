"""Batched iterations over uneven slices (mbmd_batch_sps_step), eager and as a
replayed hipGraph, with slices of one size sharing launches and with one
launch per slice, against the per-problem iteration (bit for bit)."""

import ctypes

import numpy as np
import pytest
import torch

from gpu_util import announce, host
from workloads import configs as C

import paper_2010_01371_amd as mb
from paper_2010_01371_amd import _lib

pytestmark = pytest.mark.gpu

ERR_ARG = -1                    # MBMD_ERR_ARG
SIZES = [(32, 1.0, 36, 64), (64, 0.75, 72, 128), (128, 0.5, 90, 200)]


def _slices(per_size=2):
    """Two slices of each size: three classes of two problems each."""
    return C.make_c5(per_size=per_size, sizes=SIZES)


def _reference(wls, kind, calls, blur=None, edit=None):
    """Each slice iterated alone, with the same calls as the batch (every call
    starts by recomputing the line integrals from x)."""
    refs = []
    for i, w in enumerate(wls):
        p = mb.Problem.from_workload(w, **(edit(i) if edit else {}))
        if blur is not None:
            p.set_blur(blur)
        if kind != "none":
            p.precond_build(kind)
        x = p.zeros_image()
        for n in calls:
            p.sps_step(x, kind, n)
        refs.append(host(x))
        p.close()
    return refs


@pytest.mark.parametrize("kind", ["fourier", "none", "blockdiag", "haar", "daub4"])
def test_batch_matches_single_problem_iterations(kind):
    _batch_vs_single(kind)


@pytest.mark.parametrize("kind", ["fourier", "none", "daub4"])
def test_batch_of_blurred_problems(kind):
    """Slices with a projection-domain blur: its three ray passes, inside the
    captured graph, shared by the slices of one size like every other launch."""
    _batch_vs_single(kind, blur=[[0.2, 0.6, 0.2]])


def test_blur_buffers_outside_the_block_and_different_taps():
    """Slices of one size whose blur buffers were grown outside their blocks
    (library blocks sized without blur room) cannot be reached by one offset
    per slice, so they keep launches of their own; slices with different taps
    form different classes.  Every slice matches itself run alone."""
    wls = _slices(per_size=4)[:4]                      # four 32^2 slices
    taps = [[[0.2, 0.6, 0.2]], [[0.2, 0.6, 0.2]], [[0.1, 0.8, 0.1]], [[0.1, 0.8, 0.1]]]
    kw = [dict(workspace=None, blur_room=False), dict(workspace=None, blur_room=False), {}, {}]
    calls = (6, 7)
    announce("batch blur: grown buffers, two tap sets")
    refs = []
    for w, t, k in zip(wls, taps, kw):
        p = mb.Problem.from_workload(w, **k)
        p.set_blur(t)
        p.precond_build("fourier")
        x = p.zeros_image()
        for n in calls:
            p.sps_step(x, "fourier", n)
        refs.append(host(x))
        p.close()
    probs = [mb.Problem.from_workload(w, **k) for w, k in zip(wls, kw)]
    for p, t in zip(probs, taps):
        p.set_blur(t)
        p.precond_build("fourier")
    for use_graph in (False, True):
        xs = [p.zeros_image() for p in probs]
        batch = mb.Batch(probs)
        for n in calls:
            batch.sps_step(xs, "fourier", n, use_graph=use_graph)
        got = [host(x) for x in xs]
        batch.close()
        for i, (a, r) in enumerate(zip(got, refs)):
            np.testing.assert_array_equal(a, r, err_msg="slice %d graph=%s" % (i, use_graph))
    for p in probs:
        p.close()


def _batch_vs_single(kind, blur=None):
    wls = _slices()
    n = 30
    calls = (n // 2, n - n // 2)
    announce("batch", kind, "blur" if blur else "", len(wls), "slices")
    refs = _reference(wls, kind, calls, blur)
    probs = [mb.Problem.from_workload(w) for w in wls]
    for p in probs:
        if blur is not None:
            p.set_blur(blur)
        if kind != "none":
            p.precond_build(kind)
    for shared in (True, False):
        for use_graph in (False, True):
            announce("batch", kind, "shared" if shared else "separate", "graph" if use_graph else "eager")
            xs = [p.zeros_image() for p in probs]
            batch = mb.Batch(probs, shared=shared)
            # two calls, with eager work and synchronisation in between
            batch.sps_step(xs, kind, calls[0], use_graph=use_graph)
            torch.cuda.synchronize()
            _ = (xs[0] * 2).sum().item()
            batch.sps_step(xs, kind, calls[1], use_graph=use_graph)
            got = [host(x) for x in xs]
            batch.close()
            for i, (a, r) in enumerate(zip(got, refs)):
                np.testing.assert_array_equal(a, r, err_msg="slice %d, shared=%s, graph=%s" % (i, shared, use_graph))
    for p in probs:
        p.close()


@pytest.mark.parametrize("kind", ["fourier", "none", "blockdiag", "haar", "daub4"])
def test_shared_launches_read_each_members_own_data(kind):
    """Members of one class (same geometry and sizes) with different penalty
    weights and spectra: the shared launches must read every member's own
    block, not the first member's."""
    wls = _slices(per_size=3)[:3]                      # three 32^2 slices: one class
    scale = [1.0, 0.8, 1.3]

    def edit(i):
        w = wls[i]
        return dict(S=w.S * scale[i], penalty=dict(w.penalty, beta=w.penalty["beta"] * (1 + i)))

    calls = (7, 9)
    announce("batch one class, different data", kind)
    refs = _reference(wls, kind, calls, edit=edit)
    probs = [mb.Problem.from_workload(w, **edit(i)) for i, w in enumerate(wls)]
    for p in probs:
        if kind != "none":
            p.precond_build(kind)
    for use_graph in (False, True):
        xs = [p.zeros_image() for p in probs]
        batch = mb.Batch(probs)
        for n in calls:
            batch.sps_step(xs, kind, n, use_graph=use_graph)
        got = [host(x) for x in xs]
        batch.close()
        for i, (a, r) in enumerate(zip(got, refs)):
            np.testing.assert_array_equal(a, r, err_msg="member %d graph=%s" % (i, use_graph))
        assert not np.array_equal(got[0], got[1])
    for p in probs:
        p.close()


def test_batch_with_mixed_classes_and_lone_problems():
    """A class of two, a blurred problem of the same size (a class of its own)
    and a lone problem of another size, with images that are views of one
    tensor."""
    wls = _slices(per_size=3)
    pick = [wls[0], wls[1], wls[2], wls[3]]             # three 32^2, one 64^2
    blur = [[0.2, 0.6, 0.2]]
    calls = (11,)
    announce("batch mixed classes")
    refs = []
    for i, w in enumerate(pick):
        refs += _reference([w], "fourier", calls, blur if i == 2 else None)
    probs = [mb.Problem.from_workload(w) for w in pick]
    probs[2].set_blur(blur)
    for p in probs:
        p.precond_build("fourier")
    sizes = [int(np.prod(p.image_shape)) for p in probs]
    flat = torch.zeros(sum(sizes) + 16, dtype=torch.float32, device="cuda")
    xs, off = [], 16                                    # deliberately not at the start of the tensor
    for p, m in zip(probs, sizes):
        xs.append(flat[off:off + m].view(p.image_shape))
        off += m
    for use_graph in (True, False):
        flat.zero_()
        batch = mb.Batch(probs, workspace=None)        # library-allocated offsets table
        batch.sps_step(xs, "fourier", calls[0], use_graph=use_graph)
        got = [host(x) for x in xs]
        batch.close()
        for i, (a, r) in enumerate(zip(got, refs)):
            np.testing.assert_array_equal(a, r, err_msg="problem %d graph=%s" % (i, use_graph))
    for p in probs:
        p.close()


def test_batch_workspace_and_flag_errors():
    wls = _slices(per_size=1)[:2]
    probs = [mb.Problem.from_workload(w) for w in wls]
    lib = _lib.load()
    arr = (ctypes.c_void_p * 2)(*[p._h for p in probs])
    nb = ctypes.c_size_t()
    assert lib.mbmd_batch_workspace_bytes(arr, 2, ctypes.byref(nb)) == 0
    assert nb.value >= 32 and nb.value % 256 == 0
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    st = lib.mbmd_batch_create(arr, 2, ctypes.c_void_p(ws.data_ptr()), 16, 0, ctypes.byref(h))
    assert st == ERR_ARG and not h.value
    st = lib.mbmd_batch_create(arr, 2, ctypes.c_void_p(ws.data_ptr() + 4), nb.value, 0, ctypes.byref(h))
    assert st == ERR_ARG and not h.value
    st = lib.mbmd_batch_create(arr, 2, None, 0, 2, ctypes.byref(h))
    assert st == ERR_ARG and not h.value
    dup = (ctypes.c_void_p * 2)(probs[0]._h, probs[0]._h)
    st = lib.mbmd_batch_create(dup, 2, None, 0, 0, ctypes.byref(h))
    assert st == ERR_ARG and not h.value
    batch = mb.Batch(probs)
    with pytest.raises(RuntimeError):
        probs[0].close()                                   # borrowed by an open batch
    batch.close()
    for p in probs:
        p.close()


def test_batch_graph_recaptured_after_a_blur_is_set():
    """A blur set between two graph calls changes the launch sequence (the
    blurred problems leave their class): the batch captures its iteration
    again (the per-problem runs are the check)."""
    wls = _slices()
    announce("batch", "fourier", "blur set between graph calls")
    taps = [[0.2, 0.6, 0.2]]
    refs = []
    for w in wls:
        p = mb.Problem.from_workload(w)
        p.precond_build("fourier")
        x = p.zeros_image()
        p.sps_step(x, "fourier", 10)
        p.set_blur(taps)
        p.precond_build("fourier")
        p.sps_step(x, "fourier", 10)
        refs.append(host(x))
        p.close()
    probs = [mb.Problem.from_workload(w) for w in wls]
    for p in probs:
        p.precond_build("fourier")
    xs = [p.zeros_image() for p in probs]
    batch = mb.Batch(probs)
    batch.sps_step(xs, "fourier", 10, use_graph=True)
    for p in probs:
        p.set_blur(taps)
        p.precond_build("fourier")
    batch.sps_step(xs, "fourier", 10, use_graph=True)
    got = [host(x) for x in xs]
    batch.close()
    for a, r in zip(got, refs):
        np.testing.assert_array_equal(a, r)
    for p in probs:
        p.close()
