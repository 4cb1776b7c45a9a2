"""Batched iterations over uneven slices (mbmd_batch_sps_step), eager and as a
replayed hipGraph, against the per-problem iteration."""

import numpy as np
import pytest
import torch

from gpu_util import announce, host
from workloads import configs as C

import paper_2010_01371_amd as mb

pytestmark = pytest.mark.gpu

SIZES = [(32, 1.0, 36, 64), (64, 0.75, 72, 128), (128, 0.5, 90, 200)]


def _slices():
    return C.make_c5(per_size=1, sizes=SIZES)


@pytest.mark.parametrize("kind", ["fourier", "none", "blockdiag", "daub4"])
def test_batch_matches_single_problem_iterations(kind):
    _batch_vs_single(kind)


@pytest.mark.parametrize("kind", ["fourier", "daub4"])
def test_batch_of_blurred_problems(kind):
    """Slices with a projection-domain blur (its three ray passes inside the
    captured graph)."""
    _batch_vs_single(kind, blur=[[0.2, 0.6, 0.2]])


def _batch_vs_single(kind, blur=None):
    wls = _slices()
    announce("batch", kind, "blur" if blur else "")
    probs = [mb.Problem.from_workload(w) for w in wls]
    ref_probs = [mb.Problem.from_workload(w) for w in wls]
    for p in probs + ref_probs:
        if blur is not None:
            p.set_blur(blur)
        if kind != "none":
            p.precond_build(kind)
    n = 30
    refs = []
    for p in ref_probs:
        # the same two calls as the batch below: each call starts by recomputing
        # the line integrals from x, so the runs match step for step
        x = p.zeros_image()
        p.sps_step(x, kind, n // 2)
        p.sps_step(x, kind, n - n // 2)
        refs.append(host(x))
    results = {}
    for use_graph in (False, True):
        xs = [p.zeros_image() for p in probs]
        batch = mb.Batch(probs)
        # two calls, with eager work and synchronisation in between
        batch.sps_step(xs, kind, n // 2, use_graph=use_graph)
        torch.cuda.synchronize()
        _ = (xs[0] * 2).sum().item()
        batch.sps_step(xs, kind, n - n // 2, use_graph=use_graph)
        results[use_graph] = [host(x) for x in xs]
        batch.close()
    for a, b, r in zip(results[False], results[True], refs):
        np.testing.assert_array_equal(a, b)          # graph replay == eager launches
        np.testing.assert_array_equal(a, r)          # batch == per-problem iterations


def test_batch_graph_recaptured_after_a_blur_is_set():
    """A blur set between two graph calls changes the launch sequence: the
    batch captures its iteration again (the per-problem runs are the check)."""
    wls = _slices()
    announce("batch", "fourier", "blur set between graph calls")
    taps = [[0.2, 0.6, 0.2]]
    probs = [mb.Problem.from_workload(w) for w in wls]
    ref_probs = [mb.Problem.from_workload(w) for w in wls]
    refs = []
    for p in ref_probs:
        p.precond_build("fourier")
        x = p.zeros_image()
        p.sps_step(x, "fourier", 10)
        p.set_blur(taps)
        p.precond_build("fourier")
        p.sps_step(x, "fourier", 10)
        refs.append(host(x))
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
