"""Random-ellipse phantoms, their pixelisation and their exact line integrals.

An ellipse is (cx, cy, a, b, phi, value) in mm; ``value`` is ADDED to the
image inside it.  Inner ellipses are drawn disjoint and inside a body
ellipse, and their additive value is (wanted value - body value), so the
painted image takes exactly the wanted value inside each insert and the line
integral of the image is the plain sum of per-ellipse chord lengths times
values.  That keeps the measured data exact (no inverse crime: the data come
from continuous ellipses sampled at detector-bin centres, the estimator uses
a pixel basis and detector-bin footprints).
"""

from __future__ import annotations

import numpy as np


def _circle_inside_ellipse(c, r, e, margin=1.0):
    """True when the disk of centre c, radius r+margin lies inside ellipse e."""
    cx, cy, a, b, phi, _ = e
    t = np.linspace(0.0, 2.0 * np.pi, 96, endpoint=False)
    px = c[0] + (r + margin) * np.cos(t) - cx
    py = c[1] + (r + margin) * np.sin(t) - cy
    cs, sn = np.cos(phi), np.sin(phi)
    xr = cs * px + sn * py
    yr = -sn * px + cs * py
    return bool(np.all((xr / a) ** 2 + (yr / b) ** 2 < 1.0))


def random_inserts(rng, body, n, axis_range, value_sampler, others=(), max_tries=4000):
    """Draw ``n`` disjoint inserts inside ``body`` and away from ``others``.

    Each insert is an ellipse whose bounding circle (radius = larger semi-axis)
    is inside the body and disjoint from every other bounding circle.
    Returns a list of (cx, cy, a, b, phi, painted_value) with painted (not
    additive) values.
    """
    placed = list(others)
    out = []
    lo, hi = axis_range
    tries = 0
    while len(out) < n and tries < max_tries:
        tries += 1
        shrink = 1.0 if tries < max_tries // 2 else 0.5
        a = rng.uniform(lo, lo + (hi - lo) * shrink)
        b = rng.uniform(lo, lo + (hi - lo) * shrink)
        r = max(a, b)
        R = max(body[2], body[3])
        cx, cy = rng.uniform(-R, R, size=2)
        if not _circle_inside_ellipse((cx, cy), r, body):
            continue
        if any(np.hypot(cx - p[0], cy - p[1]) < r + p[2] + 1.0 for p in placed):
            continue
        phi = rng.uniform(0.0, np.pi)
        placed.append((cx, cy, r))
        out.append((cx, cy, a, b, phi, value_sampler()))
    if len(out) < n:
        raise RuntimeError("could not place %d disjoint inserts" % n)
    return out, placed


def additive_list(body_value, body, inserts):
    """Convert painted inserts inside a body into additive ellipses."""
    ell = [tuple(body[:5]) + (body_value,)]
    for (cx, cy, a, b, phi, v) in inserts:
        ell.append((cx, cy, a, b, phi, v - body_value))
    return ell


def pixelise(ellipses, nx, ny, dx, dy, oversample=8):
    """Area-weighted pixel values: mean of an ``oversample``^2 sub-grid.

    Pixel (ix, iy) has centre ((ix-(nx-1)/2) dx, (iy-(ny-1)/2) dy); the
    result has shape [ny, nx] (x fastest), float64.
    """
    img = np.zeros((ny, nx))
    sub = (np.arange(oversample) + 0.5) / oversample - 0.5
    xc = (np.arange(nx) - (nx - 1) / 2.0) * dx
    yc = (np.arange(ny) - (ny - 1) / 2.0) * dy
    xs = (xc[:, None] + sub[None, :] * dx).ravel()
    ys = (yc[:, None] + sub[None, :] * dy).ravel()
    # process in row bands to bound memory
    band = max(oversample, ((1 << 22) // xs.size) // oversample * oversample)
    for r0 in range(0, ys.size, band):
        yy = ys[r0:r0 + band][:, None]
        xx = xs[None, :]
        acc = np.zeros((yy.shape[0], xs.size))
        for (cx, cy, a, b, phi, v) in ellipses:
            cs, sn = np.cos(phi), np.sin(phi)
            px, py = xx - cx, yy - cy
            xr = cs * px + sn * py
            yr = -sn * px + cs * py
            acc += v * (((xr / a) ** 2 + (yr / b) ** 2) <= 1.0)
        rows = acc.reshape(-1, oversample, nx, oversample)
        img_rows = rows.mean(axis=(1, 3))
        i0 = r0 // oversample
        img[i0:i0 + img_rows.shape[0]] = img_rows
    return img


def ray_bundle(geom):
    """Bin-centre rays of a parallel or flat-fan geometry.

    Returns (p, r): points [V, B, 2] on each ray and unit directions [V, B, 2].
    Conventions: view angle theta_v = theta0 + v*dtheta, detector axis
    e = (cos, sin), central-ray direction d = (-sin, cos), bin centre
    u_b = (b-(B-1)/2) du + u_offset.  Parallel rays pass through u_b e with
    direction d; fan rays leave the source -dso*d towards the detector point
    (dsd-dso) d + u_b e.
    """
    V, B = geom["n_views"], geom["n_bins"]
    th = geom["theta0"] + np.arange(V) * geom["dtheta"]
    e = np.stack([np.cos(th), np.sin(th)], -1)[:, None, :]
    d = np.stack([-np.sin(th), np.cos(th)], -1)[:, None, :]
    u = ((np.arange(B) - (B - 1) / 2.0) * geom["du"] + geom["u_offset"])[None, :, None]
    if geom["kind"] == "parallel":
        p = u * e + 0.0 * d
        r = np.broadcast_to(d, p.shape).copy()
    elif geom["kind"] == "fan":
        src = -geom["dso"] * d
        det = (geom["dsd"] - geom["dso"]) * d + u * e
        p = np.broadcast_to(src, det.shape).copy()
        r = det - src
        r = r / np.linalg.norm(r, axis=-1, keepdims=True)
    else:
        raise ValueError("rays exist only for parallel and fan geometries")
    return p, r


def line_integrals(ellipses, geom):
    """Exact line integrals of a sum of ellipses along bin-centre rays [V, B]."""
    p, r = ray_bundle(geom)
    out = np.zeros(p.shape[:2])
    for (cx, cy, a, b, phi, v) in ellipses:
        cs, sn = np.cos(phi), np.sin(phi)
        px, py = p[..., 0] - cx, p[..., 1] - cy
        qx = (cs * px + sn * py) / a
        qy = (-sn * px + cs * py) / b
        dx_ = (cs * r[..., 0] + sn * r[..., 1]) / a
        dy_ = (-sn * r[..., 0] + cs * r[..., 1]) / b
        A = dx_ * dx_ + dy_ * dy_
        Bq = 2.0 * (qx * dx_ + qy * dy_)
        C = qx * qx + qy * qy - 1.0
        disc = Bq * Bq - 4.0 * A * C
        chord = np.where(disc > 0.0, np.sqrt(np.maximum(disc, 0.0)) / A, 0.0)
        out += v * chord
    return out
