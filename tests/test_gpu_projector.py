"""GPU parity of the distance-driven projector pair (mbmd_project /
mbmd_backproject) against the FP64 oracle."""

import numpy as np
import pytest
import torch

from gpu_util import announce, dev, host, l2rel, maxrel
from oracle import projector as OP
from workloads import configs as C

import paper_2010_01371_amd as mb

pytestmark = pytest.mark.gpu

# Projection tolerance: max |A x_gpu - A x_oracle| / max |A x_oracle| <= 1e-5.
TOL_PROJ = 1e-5

GEOMS = {
    "c1_parallel": C.make_c1().geom,
    "fan64": C.geometry("fan", 64, 64, 2.0, 2.0, 90, 2 * np.pi, 128, 1.6, dso=300.0, dsd=550.0),
    # ragged: non-square, bins not a multiple of the block, 45-degree views present
    "fan_ragged": C.geometry("fan", 70, 50, 1.3, 1.7, 36, 2 * np.pi, 301, 0.9, dso=250.0, dsd=480.0,
                             u_offset=0.37),
    "parallel_offset": C.geometry("parallel", 40, 40, 1.0, 1.0, 8, np.pi, 67, 0.85, theta0=0.1, u_offset=-0.4),
    "fan_c4": C.geometry("fan", 256, 256, 0.75, 0.75, 360, 2 * np.pi, 512, 1.0, dso=600.0, dsd=1100.0),
    # ragged with both sides above one back projection wavefront segment (127
    # pixels), so that one or two channels take two pixel edges per lane
    "fan_ragged_wide": C.geometry("fan", 150, 131, 0.9, 1.1, 37, 2 * np.pi, 301, 1.1, dso=400.0,
                                  dsd=700.0, u_offset=-0.23),
    # every view in one sweep frame (rows only / columns only), the swept lines
    # long enough for two pixel edges per lane while the other side is short
    "parallel_rows_only": C.geometry("parallel", 140, 40, 1.0, 1.0, 6, 0.6, 170, 0.9, theta0=-0.3),
    "parallel_cols_only": C.geometry("parallel", 40, 150, 1.0, 1.0, 6, 0.6, 170, 0.9,
                                     theta0=np.pi / 2 - 0.3),
}


def _image(g, nmat, seed):
    rng = np.random.default_rng(seed)
    ny, nx = g["ny"], g["nx"]
    yy, xx = np.mgrid[0:ny, 0:nx]
    smooth = np.exp(-(((xx - nx / 2) / (0.3 * nx)) ** 2 + ((yy - ny / 2) / (0.35 * ny)) ** 2))
    return np.stack([smooth * (1 + m) + 0.3 * rng.uniform(size=(ny, nx)) for m in range(nmat)])


@pytest.mark.parametrize("name", sorted(GEOMS))
@pytest.mark.parametrize("nmat", [1, 3])
def test_project_matches_oracle(name, nmat):
    g = GEOMS[name]
    x = _image(g, nmat, 1)
    announce("project", name, nmat)
    got = host(mb.project(g, dev(x)))
    want = OP.project(g, x)
    assert maxrel(got, want) <= TOL_PROJ, maxrel(got, want)


@pytest.mark.parametrize("name", sorted(GEOMS))
@pytest.mark.parametrize("nch", [1, 2, 3, 6])
def test_backproject_matches_oracle(name, nch):
    g = GEOMS[name]
    rng = np.random.default_rng(2)
    s = rng.uniform(0.0, 1.0, size=(nch, g["n_views"], g["n_bins"]))
    announce("backproject", name, nch)
    got = host(mb.backproject(g, dev(s)))
    want = OP.backproject(g, s)
    assert maxrel(got, want) <= TOL_PROJ, maxrel(got, want)


@pytest.mark.parametrize("name", ["fan_ragged", "parallel_offset", "fan_ragged_wide"])
@pytest.mark.parametrize("nch", [4, 5, 7, 10])
def test_backproject_mixed_row_layouts(name, nch):
    """Channel counts whose detector rows mix packed triples with rows of their
    own (4 = 3 + 1, 5 = 3 + 2, 7 = 6 + 1, 10 = 9 + 1, the largest count):
    every channel within the bound, each against its own largest pixel."""
    g = GEOMS[name]
    rng = np.random.default_rng(20 + nch)
    s = rng.uniform(-0.2, 1.0, size=(nch, g["n_views"], g["n_bins"])) * rng.uniform(0.1, 10.0, size=(nch, 1, 1))
    announce("backproject mixed layouts", name, nch)
    got = host(mb.backproject(g, dev(s)))
    want = OP.backproject(g, s)
    for c in range(nch):
        assert maxrel(got[c], want[c]) <= TOL_PROJ, (c, maxrel(got[c], want[c]))


# Degenerate shapes: one view, one or two bins, a one-pixel-wide image, a
# 3 x 2 image, one fan-beam view.
DEGENERATE = {
    "one_view": C.geometry("parallel", 24, 20, 1.0, 1.0, 1, np.pi, 31, 1.0, theta0=0.3),
    "two_bins": C.geometry("parallel", 16, 16, 1.0, 1.0, 5, np.pi, 2, 9.0, theta0=0.1),
    "one_bin": C.geometry("parallel", 8, 8, 1.0, 1.0, 3, np.pi, 1, 12.0, theta0=0.2),
    "one_column": C.geometry("parallel", 1, 33, 1.0, 1.0, 7, np.pi, 41, 1.0, theta0=0.05),
    "three_by_two": C.geometry("parallel", 3, 2, 1.0, 1.0, 4, np.pi, 5, 1.0, theta0=0.4),
    "fan_one_view": C.geometry("fan", 20, 24, 1.0, 1.0, 1, 2 * np.pi, 45, 1.2, theta0=0.7, dso=100.0,
                               dsd=180.0),
}


@pytest.mark.parametrize("name", sorted(DEGENERATE))
def test_projection_pair_at_degenerate_shapes(name):
    """Forward (one and three materials) and back projection (one channel,
    a packed triple, a triple and a row of its own) against the oracle at
    degenerate shapes, where every sweep line is a tail or a frame has no
    views."""
    g = DEGENERATE[name]
    rng = np.random.default_rng(30)
    x = rng.uniform(size=(3, g["ny"], g["nx"]))
    s = rng.uniform(size=(4, g["n_views"], g["n_bins"]))
    announce("degenerate projection pair", name)
    for nmat in (1, 3):
        got = host(mb.project(g, dev(x[:nmat])))
        want = OP.project(g, x[:nmat])
        assert maxrel(got, want) <= TOL_PROJ, (nmat, maxrel(got, want))
    for nch in (1, 3, 4):
        got = host(mb.backproject(g, dev(s[:nch])))
        want = OP.backproject(g, s[:nch])
        for c in range(nch):
            assert maxrel(got[c], want[c]) <= TOL_PROJ, (nch, c, maxrel(got[c], want[c]))


def test_backproject_signed_data():
    """Mixed-sign sinograms (residual-like) keep the same normwise bound."""
    g = GEOMS["fan64"]
    s = np.random.default_rng(3).normal(size=(1, g["n_views"], g["n_bins"]))
    announce("backproject signed")
    got = host(mb.backproject(g, dev(s)))
    want = OP.backproject(g, s)
    assert l2rel(got, want) <= TOL_PROJ


@pytest.mark.parametrize("name", ["fan_ragged", "fan_c4"])
def test_packed_rows_keep_each_channel_apart(name):
    """From three channels on, the detector rows hold two channels per entry,
    each row with its own power-of-two scale: a channel keeps the normwise bound
    of its own output whatever the magnitudes of the others (here 1, 1e-6 and
    1e6, two of them with mixed signs), an all-zero channel gives exact zeros,
    and changing one channel's data leaves the others' outputs bitwise
    unchanged.  (Zero-mean data would cancel in the image to where FP32 sums,
    packed or not, reach 1.2e-5 of the largest pixel at 256^2.)"""
    g = GEOMS[name]
    rng = np.random.default_rng(12)
    shape = (g["n_views"], g["n_bins"])
    s = np.stack([rng.uniform(-0.3, 1.0, size=shape), 1e-6 * rng.uniform(size=shape),
                  1e6 * rng.uniform(-0.3, 1.0, size=shape), np.zeros(shape)])
    announce("packed rows per channel", name)
    got = host(mb.backproject(g, dev(s)))
    want = OP.backproject(g, s)
    for c in range(3):
        assert maxrel(got[c], want[c]) <= TOL_PROJ, (c, maxrel(got[c], want[c]))
    assert not np.any(got[3])
    s2 = s.copy()
    s2[1] = rng.uniform(size=shape)
    got2 = host(mb.backproject(g, dev(s2)))
    for c in (0, 2, 3):
        np.testing.assert_array_equal(got2[c], got[c])
    assert maxrel(got2[1], OP.backproject(g, s2[1:2])[0]) <= TOL_PROJ


def test_packed_rows_carry_a_nonfinite_value():
    """A NaN in one channel's data (a packed row's scale becomes NaN) makes that
    channel's output NaN where the view reaches and leaves the other channels
    bitwise as without it."""
    g = GEOMS["fan_ragged"]
    s = np.random.default_rng(13).uniform(size=(3, g["n_views"], g["n_bins"]))
    announce("packed rows nonfinite")
    clean = host(mb.backproject(g, dev(s)))
    s[1, 5, 150] = np.nan
    bad = host(mb.backproject(g, dev(s)))
    assert np.isnan(bad[1]).any()
    np.testing.assert_array_equal(bad[0], clean[0])
    np.testing.assert_array_equal(bad[2], clean[2])


@pytest.mark.parametrize("name", ["fan64", "fan_ragged", "c1_parallel"])
def test_adjoint_identity_fp32(name):
    """<A x, y> = <x, A^T y> for the GPU pair; FP32 sums of ~1e5 terms:
    relative mismatch bounded by 1e-5."""
    g = GEOMS[name]
    rng = np.random.default_rng(4)
    x = rng.uniform(size=(1, g["ny"], g["nx"]))
    y = rng.uniform(size=(1, g["n_views"], g["n_bins"]))
    announce("adjoint", name)
    Ax = host(mb.project(g, dev(x)))
    Aty = host(mb.backproject(g, dev(y)))
    a, b = np.sum(Ax * y), np.sum(x * Aty)
    assert abs(a - b) / abs(a) <= 1e-5


def test_backproject_is_deterministic():
    g = GEOMS["fan_c4"]
    s = dev(np.random.default_rng(5).normal(size=(2, g["n_views"], g["n_bins"])))
    announce("determinism")
    a = mb.backproject(g, s)
    b = mb.backproject(g, s)
    c = mb.backproject(g, s)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(b, c)


def test_projection_pair_is_deterministic_at_full_size():
    """The forward adds two half-line sums per bin with atomics and the back
    projector packs the line tails; both must still give bitwise-identical
    results on repeated calls (two additions onto zero commute)."""
    wl = C.make_c2(noise=False)
    g = wl.geom
    x = dev(wl.x_true)
    s = dev(np.random.default_rng(7).normal(size=(1, g["n_views"], g["n_bins"])))
    announce("determinism full size")
    p = [mb.project(g, x) for _ in range(3)]
    b = [mb.backproject(g, s) for _ in range(3)]
    torch.cuda.synchronize()
    assert torch.equal(p[0], p[1]) and torch.equal(p[1], p[2])
    assert torch.equal(b[0], b[1]) and torch.equal(b[1], b[2])


def test_identity_geometry_is_a_copy():
    g = C.identity_geometry(5, 7)
    x = np.random.default_rng(6).normal(size=(2, 5, 7))
    announce("identity projector")
    np.testing.assert_array_equal(host(mb.project(g, dev(x))), x.astype(np.float32))
    np.testing.assert_array_equal(host(mb.backproject(g, dev(x))), x.astype(np.float32))


def test_c2_full_size_projection_pair():
    """512^2 fan beam, 720 views x 888 bins (the benchmarked geometry): the whole
    forward and back projection against the oracle."""
    wl = C.make_c2(noise=True)
    g = wl.geom
    x = wl.x_true
    announce("c2 project")
    got = host(mb.project(g, dev(x)))
    want = OP.project(g, x)
    assert maxrel(got, want) <= TOL_PROJ, maxrel(got, want)
    s = np.log(5e4 / np.maximum(wl.y, 1.0))
    announce("c2 backproject")
    gotb = host(mb.backproject(g, dev(s)))
    wantb = OP.backproject(g, s)
    assert maxrel(gotb, wantb) <= TOL_PROJ, maxrel(gotb, wantb)


def test_errors_are_reported_not_raised_in_c():
    g = dict(GEOMS["fan64"])
    g["dso"] = 10.0            # source inside the image circle
    with pytest.raises(RuntimeError, match="source"):
        mb.project(g, dev(np.zeros((1, 64, 64))))


@pytest.mark.parametrize("name", ["fan64", "fan_ragged", "c1_parallel", "parallel_offset"])
def test_nonzero_count_matches_oracle(name):
    """nnz(A) counted on the device equals the oracle's count of positive
    weights, up to pixels a footprint touches at zero width: where bin edges
    coincide with pixel edges (parallel views at 0 and 90 degrees with
    du = dx) FP64 rounding leaves ~1e-16 overlaps that FP32 does not see
    (0.12% of the pairs for the 64^2 parallel case)."""
    g = GEOMS[name]
    announce("nnz", name)
    got = mb.projector_nnz(g)
    want = sum(OP.ray_weights(g, v, b)[0].size for v in range(g["n_views"]) for b in range(g["n_bins"]))
    assert abs(got - want) <= 5e-3 * want, (got, want)


def _back_shapes(g, nch):
    """Number of back projection tile shapes the autotuner chooses from: two
    pixel edges per lane (five shapes) for one or two channels when both image
    sides reach 127 pixels, else one edge per lane (four shapes)."""
    return 5 if nch <= 2 and min(g["nx"], g["ny"]) >= 127 else 4


@pytest.mark.parametrize("name", ["fan_ragged", "fan_ragged_wide"])
@pytest.mark.parametrize("nch", [1, 2, 3, 6])
def test_back_projector_tile_shapes_agree(name, nch, monkeypatch):
    """The tile shapes the autotuner chooses from (lines per wavefront, views
    in flight, views split over two wavefronts or not) sum every pixel as the
    same two halves of views in the same order, so their outputs are bitwise
    equal -- the result does not depend on which one the timing picked; and
    they match the oracle."""
    g = GEOMS[name]
    s = np.random.default_rng(7).uniform(size=(nch, g["n_views"], g["n_bins"]))
    sd = dev(s)
    outs = []
    for v in range(_back_shapes(g, nch)):
        monkeypatch.setenv("MBMD_BACK_VARIANT", str(v))
        mb.cache_clear()                      # the hook is read when the tables are built
        announce("back tile shape", name, nch, v)
        outs.append(host(mb.backproject(g, sd)))
    monkeypatch.delenv("MBMD_BACK_VARIANT")
    mb.cache_clear()
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])
    assert maxrel(outs[0], OP.backproject(g, s)) <= TOL_PROJ


def test_tuned_shape_is_timed_once_per_geometry():
    """The back projector times its candidate tile shapes on the first back
    projection of a geometry and channel count in the process; tables built
    again for that geometry (here after mbmd_cache_clear) take the recorded
    choice without timing, and give the same bits."""
    g = C.geometry("fan", 150, 140, 0.9, 0.9, 84, 2 * np.pi, 190, 1.0, dso=400.0, dsd=700.0)
    s = dev(np.random.default_rng(11).uniform(size=(1, g["n_views"], g["n_bins"])))
    announce("back projector tuning once per geometry")
    mb.cache_clear()
    with mb.KernelProfile(only=["k_dd_back"]) as prof:
        first = host(mb.backproject(g, s))
        torch.cuda.synchronize()
        n_first, _ = prof.query("k_dd_back")
    mb.cache_clear()
    with mb.KernelProfile(only=["k_dd_back"]) as prof:
        second = host(mb.backproject(g, s))
        torch.cuda.synchronize()
        n_second, _ = prof.query("k_dd_back")
    mb.cache_clear()
    assert n_first > 40, n_first                 # two warm-up passes and six timed rounds of every shape
    assert n_second == 1, n_second
    np.testing.assert_array_equal(first, second)
