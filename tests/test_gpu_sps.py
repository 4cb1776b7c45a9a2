"""GPU parity of the SPS iterations (mbmd_sps_step, plain and preconditioned)
and of the preconditioner applies (mbmd_precond_apply) against the FP64
oracle: iterates after n iterations within relative RMSE 1e-4."""

import numpy as np
import pytest

import oracle
from gpu_util import announce, dev, host, l2rel
from oracle import precond as opre, sps as osps
from workloads import configs as C

import paper_2010_01371_amd as mb

pytestmark = pytest.mark.gpu

TOL_ITER = 1e-4          # relative RMSE of the iterate after n iterations
TOL_APPLY = 1e-4         # M M^T g (FP32 transforms, FP32 tables built on the GPU)


def _rmse(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2)) / np.sqrt(np.mean(b ** 2)))


def _run(wl, kind, n):
    P = mb.Problem.from_workload(wl)
    if kind != "none":
        P.precond_build(kind)
    x = P.zeros_image()
    tr = P.sps_step(x, kind, n, trace=True)
    return host(x), tr


def _oracle(wl, kind, n):
    op = oracle.OracleProblem.from_workload(wl)
    if kind == "none":
        x, phi = osps.sps_plain(op, n)
    else:
        x, phi, _ = osps.sps_precond(op, opre.build(op, kind), n)
    return x, phi


def _check(wl, kind, n, name, trace_n=None):
    """Iterate after n iterations within TOL_ITER; objective trace within 1e-4
    over the first trace_n (default n) iterations and monotone throughout."""
    announce("sps", name, kind, n)
    xg, tg = _run(wl, kind, n)
    xo, to = _oracle(wl, kind, n)
    assert np.all(np.isfinite(tg))
    assert _rmse(xg, xo) <= TOL_ITER, _rmse(xg, xo)
    m = n if trace_n is None else trace_n
    np.testing.assert_allclose(tg[:m], to[:m], rtol=1e-4)
    assert np.all(np.diff(tg) <= 1e-6 * abs(tg[0]))       # monotone (FP32 evaluation noise allowed)


def test_c1_plain_50():
    _check(C.make_c1(), "none", 50, "c1")


@pytest.mark.parametrize("kind", ["none", "blockdiag", "fourier", "haar", "daub4"])
def test_fan64_huber(kind):
    _check(C.make_small_fan(n=64, views=90, bins=128, penalty="huber"), kind, 50, "fan64_huber")


@pytest.mark.parametrize("kind", ["fourier", "haar"])
def test_fan64_quadratic(kind):
    _check(C.make_small_fan(n=64, views=90, bins=128, penalty="quadratic"), kind, 50, "fan64_quad")


MBMD32_SEEDS = [50, 51, 52]


def _mbmd32(seed):
    return C.make_small_mbmd(n=32, views=60, bins=64, n_mat=3, seed_slice=seed)


@pytest.mark.parametrize("seed", MBMD32_SEEDS)
@pytest.mark.parametrize("kind", ["none", "blockdiag", "fourier", "haar", "daub4"])
def test_mbmd32_3mat(kind, seed):
    """Three materials, four channels.  Plain, block-diagonal and Fourier are
    compared after 50 iterations.  The cross-material wavelet iterations are
    sensitive in exact arithmetic on this problem: a relative 1e-7 random
    perturbation of the FP64 oracle's own iterate after every iteration moves
    the Haar iterate by 3e-7 to 9e-7 after 10 iterations, 1e-5 to 6e-4 after
    20 and 2e-3 to 3e-2 after 30 (Daubechies-4: 5e-6 after 10, up to 2e-1
    after 30), while Fourier and block-diagonal stay within 3e-6 throughout;
    so the wavelet iterations are compared step by step over 10 iterations,
    and at their common limit, the Newton minimiser, below.  The Fourier
    objective is more sensitive than its iterate (the same perturbation moves
    it by up to 1e-4 from iteration 15 on), so its trace is compared over
    the first 10 iterations and its iterate after 50."""
    n = 10 if kind in ("haar", "daub4") else 50
    trace_n = 10 if kind in ("haar", "fourier", "daub4") else n
    _check(_mbmd32(seed), kind, n, "mbmd32_3mat_s%d" % seed, trace_n)


def _newton_reference(name):
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "newton_xhat_%s.npz" % name)
    return np.load(path)


@pytest.mark.parametrize("kind,seed,n", [("fourier", 50, 60000), ("fourier", 51, 60000), ("fourier", 52, 60000),
                                         ("blockdiag", 51, 120000), ("haar", 51, 120000), ("daub4", 51, 120000)])
def test_mbmd32_3mat_converges_to_the_newton_minimiser(kind, seed, n):
    """Every preconditioned form converges to the minimiser x_hat of Phi, which
    no preconditioner changes: the FP32 iterate after n iterations against the
    FP64 oracle's Newton x_hat (tests/golden, written by the oracle alone).
    This comparison does not depend on the path, so it also covers the
    wavelet iterations beyond their sensitive first steps."""
    ref = _newton_reference("mbmd32_s%d" % seed)
    wl = _mbmd32(seed)
    announce("sps to the Newton minimiser", kind, seed, n)
    P = mb.Problem.from_workload(wl)
    P.precond_build(kind)
    x = P.zeros_image()
    tr = P.sps_step(x, kind, n, trace=True)
    xg = host(x)
    rel = float(np.linalg.norm(xg - ref["xhat"]) / np.linalg.norm(ref["xhat"]))
    print("mbmd32 s%d %s after %d: relative distance to x_hat %.2e" % (seed, kind, n, rel))
    assert rel <= TOL_ITER, rel
    np.testing.assert_allclose(tr[-1], float(ref["objective"]), rtol=1e-6)


@pytest.mark.parametrize("kind", ["none", "blockdiag"])
def test_identity_c3_small(kind):
    _check(C.make_c3(n_views=24, n_bins=40), kind, 50, "c3_small")


@pytest.mark.parametrize("kind", ["blockdiag", "fourier", "haar", "daub4"])
@pytest.mark.parametrize("case", ["fan64", "mbmd32"])
def test_precond_apply_matches_oracle(kind, case):
    wl = (C.make_small_fan(n=64, views=90, bins=128) if case == "fan64"
          else C.make_small_mbmd(n=32, views=60, bins=64, n_mat=3))
    op = oracle.OracleProblem.from_workload(wl)
    g = np.random.default_rng(12).normal(size=wl.x_true.shape)
    announce("precond_apply", case, kind)
    P = mb.Problem.from_workload(wl)
    P.precond_build(kind)
    got = host(P.precond_apply(kind, dev(g)))
    tab = opre.build(op, kind)
    want = opre.apply_M(tab, opre.apply_Mt(tab, g))
    assert l2rel(got, want) <= TOL_APPLY, l2rel(got, want)


@pytest.mark.parametrize("n", [128, 256, 512])
def test_fourier_apply_image_sizes(n):
    """The 2D FFT at the radix sequences (8, 8, 2), (8, 8, 4) and (8, 8, 8)."""
    wl = C.make_small_fan(n=n, views=24, bins=96)
    op = oracle.OracleProblem.from_workload(wl)
    g = np.random.default_rng(n).normal(size=wl.x_true.shape)
    announce("precond_apply", "fan%d" % n, "fourier")
    P = mb.Problem.from_workload(wl)
    P.precond_build("fourier")
    got = host(P.precond_apply("fourier", dev(g)))
    tab = opre.build(op, "fourier")
    want = opre.apply_M(tab, opre.apply_Mt(tab, g))
    assert l2rel(got, want) <= TOL_APPLY, l2rel(got, want)


@pytest.mark.parametrize("n", [128, 256, 512])
def test_haar_apply_image_sizes(n):
    """The Haar transform with a coarse stage of 4x4, 8x8 and 16x16 (the
    512x512 apply is the one the benchmark times)."""
    wl = C.make_small_fan(n=n, views=24, bins=96)
    op = oracle.OracleProblem.from_workload(wl)
    g = np.random.default_rng(n + 2).normal(size=wl.x_true.shape)
    announce("precond_apply", "fan%d" % n, "haar")
    P = mb.Problem.from_workload(wl)
    P.precond_build("haar")
    got = host(P.precond_apply("haar", dev(g)))
    tab = opre.build(op, "haar")
    want = opre.apply_M(tab, opre.apply_Mt(tab, g))
    assert l2rel(got, want) <= TOL_APPLY, l2rel(got, want)


@pytest.mark.parametrize("n", [128, 256, 512])
def test_daub4_apply_image_sizes(n):
    """The Daubechies transform with levels above the in-LDS coarse part (rows
    and column strips per level), as the wavelet preconditioner's apply."""
    wl = C.make_small_fan(n=n, views=24, bins=96)
    op = oracle.OracleProblem.from_workload(wl)
    g = np.random.default_rng(n + 1).normal(size=wl.x_true.shape)
    announce("precond_apply", "fan%d" % n, "daub4")
    P = mb.Problem.from_workload(wl)
    P.precond_build("daub4")
    got = host(P.precond_apply("daub4", dev(g)))
    tab = opre.build(op, "daub4")
    want = opre.apply_M(tab, opre.apply_Mt(tab, g))
    assert l2rel(got, want) <= TOL_APPLY, l2rel(got, want)


def _identity_workload(mats, chans, n_views=16, n_bins=24):
    """Projection-domain decomposition with a (materials, channels) pair that has
    no specialised kernel (the generic path of the per-ray kernels)."""
    rng = np.random.default_rng(77)
    mats, chans = list(mats), list(chans)
    E, Q, S = C.c4_spectral()
    Q, S = Q[:, mats], S[chans]
    K = Q.shape[1]
    top = np.array([200.0, 5.0, 2.0])[mats]
    ltrue = rng.uniform(0.0, 1.0, (K, n_views, n_bins)) * top[:, None, None]
    ybar = np.einsum("ce,evb->cvb", S, np.exp(-np.einsum("ek,kvb->evb", Q, ltrue)))
    y = rng.poisson(ybar).astype(np.float64)
    pen = dict(kind="quadratic", beta=np.zeros((K, K)), delta=0.0)
    return C.Workload("identity_%dx%d" % (K, len(chans)), C.identity_geometry(n_views, n_bins), Q, S, y,
                      C._weights(y), pen, ltrue, 50, ["none", "blockdiag"], energies=E)


@pytest.mark.parametrize("kind", ["none", "blockdiag"])
@pytest.mark.parametrize("shape", [((0,), (0, 3)), ((0, 2), (0, 1, 3)), ((1, 2), (0, 1, 2))])
def test_identity_generic_model(kind, shape):
    """(1, 2) and (2, 3) materials x channels.  Three materials from these
    spectra are left out: there, rounding the oracle's own M0 to FP32 already
    moves its iterate after 50 iterations by ~0.1 (relative RMSE), so no FP32
    implementation can be compared with it at 1e-4."""
    _check(_identity_workload(*shape), kind, 50, "identity_%dx%d" % (len(shape[0]), len(shape[1])))


def test_refresh_boundary_and_chunked_trace():
    """More iterations than the line-integral refresh period; trace over two calls."""
    wl = C.make_small_fan(n=32, views=48, bins=64)
    P = mb.Problem.from_workload(wl)
    P.precond_build("fourier")
    x = P.zeros_image()
    announce("refresh")
    t1 = P.sps_step(x, "fourier", 30, trace=True)
    t2 = P.sps_step(x, "fourier", 30, trace=True)
    xo, to = _oracle(wl, "fourier", 60)
    assert _rmse(host(x), xo) <= TOL_ITER
    np.testing.assert_allclose(np.r_[t1[:-1], t2], to, rtol=1e-4)


def test_unbuilt_preconditioner_is_an_error():
    wl = C.make_small_fan(n=32, views=48, bins=64)
    P = mb.Problem.from_workload(wl)
    with pytest.raises(RuntimeError, match="not built"):
        P.sps_step(P.zeros_image(), "haar", 1)


@pytest.mark.parametrize("name", ["fan64_huber", "fan128_quad"])
def test_gradient_rows_fused_match_separate_launches(name, monkeypatch):
    """Once the back projector's shape is chosen, the gradient launch of a
    single-energy problem writes its detector rows itself; the iterates are
    bitwise those of storing the gradient and running the detector prefix (one
    pixel edge per lane at 64^2, two at 128^2)."""
    wl = {
        "fan64_huber": lambda: C.make_small_fan(n=64, views=90, bins=128, penalty="huber"),
        "fan128_quad": lambda: C.make_small_fan(n=128, views=120, bins=200, penalty="quadratic"),
    }[name]()
    announce("sps fused gradient rows", name)
    out, fused_launches = [], []
    for fuse in ("0", "1"):
        monkeypatch.setenv("MBMD_FUSE_ROWS", fuse)
        P = mb.Problem.from_workload(wl)
        P.precond_build("fourier")
        x = P.zeros_image()
        with mb.KernelProfile(only=["k_ray_grad_rows"]) as prof:
            P.sps_step(x, "fourier", 12)
            fused_launches.append(prof.query("k_ray_grad_rows")[0])
        out.append(host(x))
    monkeypatch.delenv("MBMD_FUSE_ROWS")
    assert fused_launches[0] == 0 and fused_launches[1] >= 11, fused_launches   # the first one tunes
    np.testing.assert_array_equal(out[1], out[0])


def _x_ref(wl):
    """A reference image near the solution: the phantom, smoothed by a
    positive perturbation (not the data's own image)."""
    rng = np.random.default_rng(21)
    return np.abs(wl.x_true) * (1.0 + 0.1 * rng.uniform(size=wl.x_true.shape))


@pytest.mark.parametrize("case", ["fan64", "mbmd32"])
@pytest.mark.parametrize("kind,modified,ref", [("fourier", False, False), ("haar", False, False),
                                               ("fourier", True, True), ("haar", True, True),
                                               ("blockdiag", True, True), ("fourier", False, True),
                                               ("daub4", False, False), ("daub4", True, True)])
def test_precond_build_options_match_oracle(kind, modified, ref, case):
    """mbmd_precond_build_ex: M0 = I (unmodified) and / or the Fisher weights at
    a reference image; M M^T g against the oracle built the same way."""
    wl = (C.make_small_fan(n=64, views=90, bins=128) if case == "fan64"
          else C.make_small_mbmd(n=32, views=60, bins=64, n_mat=3))
    op = oracle.OracleProblem.from_workload(wl)
    g = np.random.default_rng(13).normal(size=wl.x_true.shape)
    x_ref = _x_ref(wl) if ref else None
    announce("precond_build_ex", case, kind, modified, ref)
    P = mb.Problem.from_workload(wl)
    P.precond_build(kind, modified=modified, x_ref=dev(x_ref) if ref else None)
    got = host(P.precond_apply(kind, dev(g)))
    tab = opre.build(op, kind, modified=modified, x_ref=x_ref)
    want = opre.apply_M(tab, opre.apply_Mt(tab, g))
    assert l2rel(got, want) <= TOL_APPLY, l2rel(got, want)


def test_rebuild_voids_the_other_preconditioners():
    """Fisher weights and M0 are shared: after a build with options the other
    preconditioners must be built again, and a plain build restores the
    data-based ones (bitwise the first build's apply)."""
    wl = C.make_small_fan(n=64, views=90, bins=128)
    g = dev(np.random.default_rng(14).normal(size=wl.x_true.shape))
    announce("precond rebuild")
    P = mb.Problem.from_workload(wl)
    P.precond_build("fourier")
    P.precond_build("haar")
    first = host(P.precond_apply("fourier", g))
    P.precond_build("fourier", x_ref=dev(_x_ref(wl)))
    with pytest.raises(RuntimeError):
        P.precond_apply("haar", g)
    P.precond_build("fourier")
    np.testing.assert_array_equal(host(P.precond_apply("fourier", g)), first)


def test_sps_with_a_rebuild_from_the_iterate():
    """10 Fourier-preconditioned iterations, a rebuild with the Fisher weights
    at the current iterate, 10 more: against the oracle doing the same."""
    wl = C.make_small_fan(n=64, views=90, bins=128, penalty="huber")
    announce("sps rebuild from iterate")
    P = mb.Problem.from_workload(wl)
    P.precond_build("fourier")
    x = P.zeros_image()
    P.sps_step(x, "fourier", 10)
    P.precond_build("fourier", x_ref=x.clone())
    P.sps_step(x, "fourier", 10)
    op = oracle.OracleProblem.from_workload(wl)
    xo, _, _ = osps.sps_precond(op, opre.build(op, "fourier"), 10)
    xo, _, _ = osps.sps_precond(op, opre.build(op, "fourier", x_ref=xo), 10, x0=xo)
    assert _rmse(host(x), xo) <= TOL_ITER, _rmse(host(x), xo)


def test_identity_traced_run_past_the_trace_capacity():
    """An identity-geometry run with more traced iterations than the device
    trace holds (4096) is cut into chunks of at most that many: the iterate is
    bitwise that of the untraced run (one chunk here), the trace is finite and
    non-increasing, its first 51 values match the oracle, and its last value is
    the objective mbmd_gradient reports at the final iterate."""
    wl = C.make_c3(n_views=24, n_bins=40)
    n = 4100
    announce("identity traced past capacity", n)
    P = mb.Problem.from_workload(wl)
    P.precond_build("blockdiag")
    xa, xb = P.zeros_image(), P.zeros_image()
    tr = P.sps_step(xa, "blockdiag", n, trace=True)
    P.sps_step(xb, "blockdiag", n)
    np.testing.assert_array_equal(host(xa), host(xb))
    assert tr.shape == (n + 1,) and np.all(np.isfinite(tr))
    assert np.all(np.diff(tr) <= 1e-6 * abs(tr[0]))
    _, _, phi = P.gradient(xa, objective=True)
    np.testing.assert_allclose(tr[-1], phi, rtol=1e-6)
    _, to = _oracle(wl, "blockdiag", 50)
    np.testing.assert_allclose(tr[:51], to, rtol=1e-4)
