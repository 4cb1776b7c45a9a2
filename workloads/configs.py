"""The five synthetic workloads (and small variants used by tests).

Seeds: ``seed_for(config, slice)`` = 20201003 + 100*config + slice, NumPy
PCG64.  The phantom is drawn first, then the noise, from one Generator.

Geometry dicts carry the fields every consumer needs:
  kind ('parallel' | 'fan' | 'identity'), nx, ny, dx, dy [mm],
  n_views, theta0, dtheta [rad], n_bins, du, u_offset [mm], dso, dsd [mm].
For 'identity' the unknown is a [V, B] sinogram of line integrals, so
(ny, nx) = (n_views, n_bins).
"""

from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from . import phantoms as ph
from . import spectra as sp

BASE_SEED = 20201003


def seed_for(config: int, slice_index: int = 0) -> int:
    return BASE_SEED + 100 * config + slice_index


def geometry(kind, nx, ny, dx, dy, n_views, span, n_bins, du, dso=0.0, dsd=0.0,
             theta0=0.0, u_offset=0.0):
    return dict(kind=kind, nx=int(nx), ny=int(ny), dx=float(dx), dy=float(dy),
                n_views=int(n_views), theta0=float(theta0),
                dtheta=float(span) / int(n_views), n_bins=int(n_bins), du=float(du),
                u_offset=float(u_offset), dso=float(dso), dsd=float(dsd))


def identity_geometry(n_views, n_bins):
    return dict(kind="identity", nx=int(n_bins), ny=int(n_views), dx=1.0, dy=1.0,
                n_views=int(n_views), theta0=0.0, dtheta=0.0, n_bins=int(n_bins),
                du=1.0, u_offset=0.0, dso=0.0, dsd=0.0)


@dataclasses.dataclass
class Workload:
    name: str
    geom: dict
    Q: np.ndarray            # [n_energy, n_mat] attenuation per unit of x
    S: np.ndarray            # [n_chan, n_energy] sensitivity, gain and I0 folded in
    y: np.ndarray            # [n_chan, V, B] measured counts (float64)
    w: np.ndarray            # [n_chan, V, B] inverse variances 1/max(y, 1)
    penalty: dict            # {'kind': 'quadratic'|'huber', 'beta': [n_mat, n_mat], 'delta'}
    x_true: np.ndarray       # [n_mat, ny, nx] pixelised phantom (or true line integrals)
    n_iter: int
    preconds: List[str]
    energies: Optional[np.ndarray] = None
    materials: Optional[List[str]] = None

    @property
    def n_mat(self):
        return self.Q.shape[1]

    @property
    def n_chan(self):
        return self.S.shape[0]

    @property
    def n_energy(self):
        return self.Q.shape[0]


def _weights(y):
    return 1.0 / np.maximum(y, 1.0)


def _mono(geom, ell, i0, rng, noise=True):
    p = ph.line_integrals(ell, geom)
    ybar = i0 * np.exp(-p)
    y = rng.poisson(ybar).astype(np.float64) if noise else ybar
    return y[None], np.array([[1.0]]), np.array([[i0]])


def _spectral(geom, ell_per_mat, Q, S, rng, noise=True):
    ls = np.stack([ph.line_integrals(e, geom) for e in ell_per_mat])      # [K, V, B]
    lE = np.einsum("ek,kvb->evb", Q, ls)
    ybar = np.einsum("ce,evb->cvb", S, np.exp(-lE))
    y = rng.poisson(ybar).astype(np.float64) if noise else ybar
    return y


def _single_energy_phantom(rng, fov_r, body_axes, n_inner, inner_axes, inner_mu,
                           body_mu, n_bone=0, bone_axes=(4.0, 15.0), bone_mu=0.05):
    ba = rng.uniform(*body_axes[0]), rng.uniform(*body_axes[1])
    body = (rng.uniform(-0.05, 0.05) * fov_r, rng.uniform(-0.05, 0.05) * fov_r,
            ba[0], ba[1], rng.uniform(0.0, np.pi), body_mu)
    inserts, placed = ph.random_inserts(rng, body, n_inner, inner_axes,
                                        lambda: rng.uniform(*inner_mu))
    if n_bone:
        bones, _ = ph.random_inserts(rng, body, n_bone, bone_axes, lambda: bone_mu,
                                     others=placed)
        inserts = inserts + bones
    return ph.additive_list(body_mu, body, inserts)


def make_c1(noise=True):
    """64x64 parallel-beam PWLS: 1 mm pixels, 90 views over 180 deg, 96 bins."""
    rng = np.random.default_rng(seed_for(1))
    g = geometry("parallel", 64, 64, 1.0, 1.0, 90, np.pi, 96, 1.0)
    k = int(rng.integers(5, 11))               # 5..10 ellipses in total
    body_mu = rng.uniform(0.01, 0.03)
    ell = _single_energy_phantom(rng, 32.0, ((22.0, 28.0), (18.0, 26.0)), k - 1,
                                 (3.0, 9.0), (0.01, 0.03), body_mu)
    x = ph.pixelise(ell, g["nx"], g["ny"], g["dx"], g["dy"])
    y, Q, S = _mono(g, ell, 1e4, rng, noise)
    pen = dict(kind="quadratic", beta=np.array([[1e2]]), delta=0.0)
    return Workload("c1_parallel64", g, Q, S, y, _weights(y), pen, x[None], 50, ["none"])


def make_c2(noise=True):
    """512x512 fan beam, Huber penalty: 0.5 mm pixels, 720 views, 888 bins."""
    rng = np.random.default_rng(seed_for(2))
    g = geometry("fan", 512, 512, 0.5, 0.5, 720, 2 * np.pi, 888, 1.0, dso=600.0, dsd=1100.0)
    n_inner = int(rng.integers(5, 11))
    n_bone = int(rng.integers(2, 5))
    ell = _single_energy_phantom(rng, 128.0, ((105.0, 115.0), (85.0, 95.0)), n_inner,
                                 (8.0, 30.0), (0.015, 0.03), 0.02, n_bone=n_bone)
    x = ph.pixelise(ell, g["nx"], g["ny"], g["dx"], g["dy"])
    y, Q, S = _mono(g, ell, 5e4, rng, noise)
    pen = dict(kind="huber", beta=np.array([[1e3]]), delta=1e-3)
    return Workload("c2_fan512_huber", g, Q, S, y, _weights(y), pen, x[None], 100,
                    ["none", "fourier", "haar"])


def make_small_fan(n=64, views=90, bins=128, penalty="huber", noise=True, seed_slice=50):
    """A small fan-beam single-energy problem for fast parity tests."""
    rng = np.random.default_rng(seed_for(2, seed_slice))
    pix = 128.0 / n
    g = geometry("fan", n, n, pix, pix, views, 2 * np.pi, bins, 1.0 * 128.0 / bins * 1.6,
                 dso=300.0, dsd=550.0)
    ell = _single_energy_phantom(rng, 64.0, ((50.0, 56.0), (40.0, 46.0)), 5,
                                 (4.0, 12.0), (0.015, 0.03), 0.02, n_bone=2,
                                 bone_axes=(3.0, 6.0))
    x = ph.pixelise(ell, g["nx"], g["ny"], g["dx"], g["dy"])
    y, Q, S = _mono(g, ell, 5e4, rng, noise)
    if penalty == "huber":
        pen = dict(kind="huber", beta=np.array([[1e3]]), delta=1e-3)
    else:
        pen = dict(kind="quadratic", beta=np.array([[1e2]]), delta=0.0)
    return Workload("small_fan%d" % n, g, Q, S, y, _weights(y), pen, x[None], 50,
                    ["none", "fourier", "haar"])


def c3_spectral(n_energy_max=140.0):
    E = np.arange(20.0, n_energy_max + 0.5, 1.0)
    Q = np.stack([sp.attenuation("water", E), sp.attenuation("iodine", E)], 1)
    S = sp.kvp_switching_sensitivity(E, (80.0, 140.0), 5e4)
    return E, Q, S


def make_c3(noise=True, n_views=720, n_bins=888):
    """Projection-domain 2-material x 2-kVp decomposition on 720x888 rays."""
    rng = np.random.default_rng(seed_for(3))
    E, Q, S = c3_spectral()
    g = identity_geometry(n_views, n_bins)
    lw = rng.uniform(0.0, 300.0, (n_views, n_bins))
    li = rng.uniform(0.0, 5.0, (n_views, n_bins))
    ltrue = np.stack([lw, li])
    ybar = np.einsum("ce,evb->cvb", S, np.exp(-np.einsum("ek,kvb->evb", Q, ltrue)))
    y = rng.poisson(ybar).astype(np.float64) if noise else ybar
    pen = dict(kind="quadratic", beta=np.zeros((2, 2)), delta=0.0)
    return Workload("c3_projdomain_2x2", g, Q, S, y, _weights(y), pen, ltrue, 50,
                    ["none", "blockdiag"], energies=E, materials=["water", "iodine"])


def c4_spectral():
    E = np.arange(20.0, 120.5, 1.0)
    Q = np.stack([sp.attenuation("water", E), sp.attenuation("calcium", E),
                  sp.attenuation("iodine", E)], 1)
    S = sp.threshold_pcd_sensitivity(E, 120.0, (25.0, 45.0, 65.0, 85.0), 2e4)
    return E, Q, S


def _mbmd_phantom(rng, fov_r, body_axes, n_ca, n_io, n_soft, insert_axes, materials):
    ba = rng.uniform(*body_axes[0]), rng.uniform(*body_axes[1])
    body = (rng.uniform(-0.05, 0.05) * fov_r, rng.uniform(-0.05, 0.05) * fov_r,
            ba[0], ba[1], rng.uniform(0.0, np.pi), 1.0)
    soft, placed = ph.random_inserts(rng, body, n_soft, (insert_axes[0] * 2, insert_axes[1] * 2),
                                     lambda: rng.uniform(0.9, 1.1))
    water = ph.additive_list(1.0, body, soft)
    per_mat = {"water": water}
    if "calcium" in materials:
        ca, placed = ph.random_inserts(rng, body, n_ca, insert_axes,
                                       lambda: rng.uniform(0.1, 0.3), others=placed)
        per_mat["calcium"] = [c[:5] + (c[5],) for c in ca]
    io, placed = ph.random_inserts(rng, body, n_io, insert_axes,
                                   lambda: rng.uniform(0.005, 0.02), others=placed)
    per_mat["iodine"] = [c[:5] + (c[5],) for c in io]
    return [per_mat[m] for m in materials]


def make_c4(noise=True):
    """One-step MBMD: water/Ca/I, 4 PCD channels, 256^2 fan beam, 360x512."""
    rng = np.random.default_rng(seed_for(4))
    E, Q, S = c4_spectral()
    g = geometry("fan", 256, 256, 0.75, 0.75, 360, 2 * np.pi, 512, 1.0, dso=600.0, dsd=1100.0)
    mats = ["water", "calcium", "iodine"]
    ells = _mbmd_phantom(rng, 96.0, ((70.0, 80.0), (55.0, 65.0)), int(rng.integers(2, 5)),
                         int(rng.integers(2, 5)), 3, (4.0, 12.0), mats)
    x = np.stack([ph.pixelise(e, g["nx"], g["ny"], g["dx"], g["dy"]) for e in ells])
    y = _spectral(g, ells, Q, S, rng, noise)
    pen = dict(kind="quadratic", beta=np.diag([1e1, 1e2, 1e4]), delta=0.0)
    return Workload("c4_mbmd_3mat_4ch", g, Q, S, y, _weights(y), pen, x, 50,
                    ["none", "blockdiag", "fourier"], energies=E, materials=mats)


def make_small_mbmd(n=32, views=60, bins=64, n_mat=3, noise=True, n_energy_step=5, seed_slice=50):
    """A small one-step MBMD problem (coarser energy grid) for fast tests;
    seed_slice picks another phantom and noise draw."""
    rng = np.random.default_rng(seed_for(4, seed_slice))
    if n_mat == 3:
        E, Q, S = c4_spectral()
        mats = ["water", "calcium", "iodine"]
        beta = np.diag([1e1, 1e2, 1e4])
    else:
        E, Q, S = c3_spectral()
        mats = ["water", "iodine"]
        beta = np.diag([1e1, 1e4])
    sel = slice(0, None, n_energy_step)
    E, Q = E[sel], Q[sel]
    S = S[:, sel] * n_energy_step
    pix = 96.0 / n
    g = geometry("fan", n, n, pix, pix, views, 2 * np.pi, bins, 160.0 / bins,
                 dso=300.0, dsd=550.0)
    ells = _mbmd_phantom(rng, 48.0, ((34.0, 38.0), (28.0, 32.0)), 2, 2, 1, (3.0, 6.0), mats)
    x = np.stack([ph.pixelise(e, g["nx"], g["ny"], g["dx"], g["dy"]) for e in ells])
    y = _spectral(g, ells, Q, S, rng, noise)
    pen = dict(kind="quadratic", beta=beta, delta=0.0)
    return Workload("small_mbmd%d_%dmat" % (n, n_mat), g, Q, S, y, _weights(y), pen, x, 30,
                    ["none", "blockdiag", "fourier"], energies=E, materials=mats)


C5_SIZES = [  # (n, pixel mm, views, bins)
    (128, 1.0, 180, 256),
    (256, 0.75, 360, 512),
    (512, 0.5, 720, 888),
]


def make_c5(noise=True, per_size=8, sizes=None):
    """24 slices of uneven size, water/iodine with the two kVp spectra."""
    E, Q, S = c3_spectral()
    out = []
    sizes = C5_SIZES if sizes is None else sizes
    for si, (n, pix, views, bins) in enumerate(sizes):
        for j in range(per_size):
            idx = si * per_size + j
            rng = np.random.default_rng(seed_for(5, idx))
            g = geometry("fan", n, n, pix, pix, views, 2 * np.pi, bins, 1.0,
                         dso=600.0, dsd=1100.0)
            fov_r = n * pix / 2.0
            ells = _mbmd_phantom(rng, fov_r, ((0.78 * fov_r, 0.86 * fov_r), (0.62 * fov_r, 0.7 * fov_r)),
                                 0, int(rng.integers(2, 4)), 2, (0.03 * fov_r, 0.09 * fov_r),
                                 ["water", "iodine"])
            x = np.stack([ph.pixelise(e, n, n, pix, pix) for e in ells])
            y = _spectral(g, ells, Q, S, rng, noise)
            pen = dict(kind="quadratic", beta=np.diag([1e1, 1e4]), delta=0.0)
            out.append(Workload("c5_slice%02d_%d" % (idx, n), g, Q, S, y, _weights(y), pen, x, 50,
                                ["fourier"], energies=E, materials=["water", "iodine"]))
    return out
