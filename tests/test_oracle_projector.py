"""Pins of the FP64 oracle's distance-driven projector (CPU only).

The paper leaves the projector undefined; these tests fix the distance-driven
model against closed forms, brute force and the adjoint identity.
"""

import numpy as np
import pytest

from oracle import projector as P
from workloads import configs as C
from workloads import phantoms as ph


def _par(n=32, views=24, bins=48, du=1.0, span=np.pi, theta0=0.0, u_off=0.0):
    return C.geometry("parallel", n, n, 1.0, 1.0, views, span, bins, du, theta0=theta0, u_offset=u_off)


def _fan(n=32, views=36, bins=64, pix=1.0, du=1.0):
    return C.geometry("fan", n, n, pix, pix, views, 2 * np.pi, bins, du, dso=100.0, dsd=180.0)


@pytest.mark.parametrize("geom", [_par(), _par(n=16, views=7, bins=21, du=0.7, u_off=0.3), _fan(),
                                  _fan(n=24, views=13, bins=50, pix=0.8, du=1.3),
                                  C.geometry("fan", 20, 12, 1.0, 1.5, 11, 2 * np.pi, 40, 1.1,
                                             dso=60.0, dsd=110.0)])
def test_adjoint_identity(geom):
    """<A x, y> = <x, A^T y> to 1e-12 relative in FP64."""
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, geom["ny"], geom["nx"]))
    y = rng.normal(size=(2, geom["n_views"], geom["n_bins"]))
    a = np.sum(P.project(geom, x) * y)
    b = np.sum(x * P.backproject(geom, y))
    assert abs(a - b) <= 1e-12 * np.sqrt(np.sum(P.project(geom, x) ** 2) * np.sum(y ** 2))


def test_theta0_column_sums():
    """Parallel beam at theta = 0 with du = dx and B = nx: A x = dy * column sums."""
    g = C.geometry("parallel", 16, 12, 1.0, 0.5, 1, np.pi, 16, 1.0)
    x = np.random.default_rng(2).uniform(size=(12, 16))
    np.testing.assert_allclose(P.project(g, x)[0], 0.5 * x.sum(axis=0), rtol=1e-14, atol=1e-14)


def test_theta90_row_sums():
    """At theta = 90 deg the sweep runs over columns and the rays integrate rows."""
    g = C.geometry("parallel", 16, 16, 1.0, 1.0, 1, np.pi, 16, 1.0, theta0=np.pi / 2)
    x = np.random.default_rng(3).uniform(size=(16, 16))
    assert not P.sweeps_rows(g, 0)
    # the ray direction is d = (-1, 0); bin u sits at y = u, so bin b sees row b
    np.testing.assert_allclose(P.project(g, x)[0], x.sum(axis=1), rtol=1e-13, atol=1e-13)


def _chord_through_box(p, r, half_x, half_y):
    """Exact chord of the line p + s r (|r| = 1) through the box |x|<=hx, |y|<=hy."""
    lo, hi = -np.inf, np.inf
    for a, h in ((0, half_x), (1, half_y)):
        if abs(r[a]) < 1e-15:
            if abs(p[a]) > h:
                return 0.0
            continue
        s1, s2 = (-h - p[a]) / r[a], (h - p[a]) / r[a]
        lo, hi = max(lo, min(s1, s2)), min(hi, max(s1, s2))
    return max(0.0, hi - lo)


@pytest.mark.parametrize("geom", [_par(n=24, views=17, bins=60), _fan(n=24, views=19, bins=70)])
def test_ones_projection_is_chord_through_image(geom):
    """(A 1) equals the exact chord length of the bin-centre ray through the
    image square for rays that cross both faces normal to the sweep axis,
    averaged over the footprint (the DD row weights sum to dy/|cos phi_b|)."""
    n = geom["nx"]
    ones = np.ones((n, n))
    A1 = P.project(geom, ones)
    p, r = ph.ray_bundle(geom)
    checked = 0
    for v in range(geom["n_views"]):
        rows = P.sweeps_rows(geom, v)
        ax = 1 if rows else 0
        for b in range(geom["n_bins"]):
            # both boundary rays must enter and leave through the sweep-normal faces
            idx, wt = P.ray_weights(geom, v, b)
            if wt.size == 0:
                continue
            half = n / 2.0
            # chord through the slab between the two faces normal to the sweep axis
            slab = n / abs(r[v, b, ax])
            chord = _chord_through_box(p[v, b], r[v, b], half, half)
            if abs(chord - slab) > 1e-9:
                continue
            # the bin footprint must stay inside the image on every line
            lines = np.unique(idx // n if rows else idx % n)
            if lines.size != n:
                continue
            along = idx % n if rows else idx // n
            if along.min() == 0 or along.max() == n - 1:
                continue
            np.testing.assert_allclose(A1[v, b], slab, rtol=1e-12)
            checked += 1
    assert checked > 100


def _brute_weights(geom, v, b, samples=4000):
    """Brute-force DD weights: sample the footprint on each sweep line densely
    and histogram the samples into pixels."""
    th = geom["theta0"] + v * geom["dtheta"]
    c, s = np.cos(th), np.sin(th)
    e, d = np.array([c, s]), np.array([-s, c])
    uc = (b - (geom["n_bins"] - 1) / 2.0) * geom["du"] + geom["u_offset"]

    def ray(u):
        if geom["kind"] == "parallel":
            return u * e, d
        src = -geom["dso"] * d
        return src, (geom["dsd"] - geom["dso"]) * d + u * e - src

    rows = abs(c) >= abs(s)
    ia, it = (1, 0) if rows else (0, 1)
    nl = geom["ny"] if rows else geom["nx"]
    na = geom["nx"] if rows else geom["ny"]
    dl = geom["dy"] if rows else geom["dx"]
    da = geom["dx"] if rows else geom["dy"]
    _, rc = ray(uc)
    path = dl * np.linalg.norm(rc) / abs(rc[ia])
    W = np.zeros(geom["nx"] * geom["ny"])
    for q in range(nl):
        a = (q - (nl - 1) / 2.0) * dl
        ts = []
        for u in (uc - geom["du"] / 2, uc + geom["du"] / 2):
            p0, r0 = ray(u)
            ts.append(p0[it] + (a - p0[ia]) * r0[it] / r0[ia])
        lo, hi = min(ts), max(ts)
        t = lo + (np.arange(samples) + 0.5) / samples * (hi - lo)
        k = np.floor(t / da + na / 2.0).astype(int)
        ok = (k >= 0) & (k < na)
        cnt = np.bincount(k[ok], minlength=na)
        for kk in np.nonzero(cnt)[0]:
            j = q * geom["nx"] + kk if rows else kk * geom["nx"] + q
            W[j] += cnt[kk] / samples * path
    return W


@pytest.mark.parametrize("geom", [_par(n=12, views=9, bins=20, du=0.9, u_off=0.2),
                                  _fan(n=12, views=11, bins=24, pix=1.1, du=0.8)])
def test_weights_match_brute_force_footprint(geom):
    for v in range(geom["n_views"]):
        for b in range(0, geom["n_bins"], 3):
            idx, wt = P.ray_weights(geom, v, b)
            dense = np.zeros(geom["nx"] * geom["ny"])
            np.add.at(dense, idx, wt)
            brute = _brute_weights(geom, v, b)
            # sampling error: one sample (1/4000 of the footprint) per pixel edge
            assert np.max(np.abs(dense - brute)) <= 2.5e-4 * max(1.0, brute.max()) * 2


def _disk_error(pix, r=20.0):
    n = int(round(64.0 / pix))
    g = C.geometry("parallel", n, n, pix, pix, 6, np.pi, 120, 0.5)
    disk = [(0.0, 0.0, r, r, 0.0, 1.0)]
    img = ph.pixelise(disk, n, n, pix, pix, oversample=8)
    proj = P.project(g, img)
    u = (np.arange(g["n_bins"]) - (g["n_bins"] - 1) / 2.0) * g["du"]
    exact = 2.0 * np.sqrt(np.maximum(r * r - u * u, 0.0))
    inside = np.abs(u) < 0.9 * r
    return np.max(np.abs(proj[:, inside] - exact[None, inside]) / exact[None, inside])


def test_uniform_disk_converges_to_closed_form():
    """Projection of a pixelised uniform disk -> mu * 2 sqrt(r^2 - s^2), O(h)."""
    e1, e2, e3 = _disk_error(1.0), _disk_error(0.5), _disk_error(0.25)
    assert e1 < 0.05 and e2 < e1 and e3 < e2
    assert e1 / e3 > 2.5          # roughly halves per halving of the pixel


def _ellipse_l1_error(pix):
    n = int(round(64.0 / pix))
    g = C.geometry("fan", n, n, pix, pix, 24, 2 * np.pi, 200, 0.6, dso=100.0, dsd=180.0)
    ell = [(0.0, 0.0, 25.0, 18.0, 0.3, 0.02), (5.0, -3.0, 6.0, 4.0, 1.1, 0.01)]
    img = ph.pixelise(ell, n, n, pix, pix)
    proj = P.project(g, img)
    exact = ph.line_integrals(ell, g)
    return np.sum(np.abs(proj - exact)) / np.sum(exact)


def test_fan_ellipse_phantom_converges_to_analytic():
    """Fan-beam DD projections of a pixelised ellipse phantom approach its
    exact line integrals as the pixels shrink (l1 error at least halves)."""
    e1, e2, e3 = _ellipse_l1_error(1.0), _ellipse_l1_error(0.5), _ellipse_l1_error(0.25)
    assert e2 < 5e-3
    assert e1 / e2 > 2.0 and e2 / e3 > 2.0


def test_opposite_parallel_views_mirror():
    """Parallel views theta and theta + pi see the same rays in reverse bin order."""
    g = C.geometry("parallel", 20, 20, 1.0, 1.0, 2, np.pi + 0.3, 40, 0.8, theta0=0.3)
    g["dtheta"] = np.pi
    x = np.random.default_rng(5).uniform(size=(20, 20))
    s = P.project(g, x)
    np.testing.assert_allclose(s[1], s[0][::-1], rtol=1e-12, atol=1e-12)


def test_dense_matrix_consistent():
    g = _fan(n=8, views=5, bins=12)
    A = P.dense_matrix(g)
    x = np.random.default_rng(6).normal(size=(8, 8))
    np.testing.assert_allclose(A @ x.ravel(), P.project(g, x).ravel(), rtol=1e-13, atol=1e-13)
    assert np.all(A >= 0.0)
