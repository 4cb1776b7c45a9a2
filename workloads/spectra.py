"""Synthetic attenuation curves, source spectra and channel sensitivities.

None of these are measured data.  Each basis material gets a two-term curve
mu(E) = a E^-3 + b f_KN(E): a photoelectric-like power law plus the shape of
the Klein-Nishina total cross-section.  The constants were chosen so that the
curves have plausible magnitudes over 20-140 keV; they are not fits to any
table.  Water and aluminium are in 1/mm, calcium and iodine in mm^2/mg (so a
density image in mg/mm^3 or a line integral in mg/mm^2 multiplies them).
"""

from __future__ import annotations

import numpy as np

ELECTRON_REST_KEV = 510.975

# (a [keV^3 * unit], b [unit]) for mu(E) = a E^-3 + b f_KN(E)
MATERIALS = {
    "water": (470.0, 0.01686),
    "aluminium": (6799.0, 0.04024),
    "calcium": (1.067e4, 0.004012),
    "iodine": (2.184e4, 0.1315),
}
# K-edges (keV) and the factor on the photoelectric term above them.  The
# calcium edge (4 keV) lies below every grid energy used here, so its curve
# is the above-edge one throughout.
K_EDGE = {"iodine": (33.2, 6.0), "calcium": (4.0, 1.0)}


def klein_nishina_shape(E):
    """Klein-Nishina total cross-section shape (dimensionless), E in keV."""
    k = np.asarray(E, dtype=np.float64) / ELECTRON_REST_KEV
    l2 = np.log1p(2.0 * k)
    return ((1.0 + k) / k ** 2 * (2.0 * (1.0 + k) / (1.0 + 2.0 * k) - l2 / k)
            + l2 / (2.0 * k) - (1.0 + 3.0 * k) / (1.0 + 2.0 * k) ** 2)


def attenuation(material, E):
    """mu(E) of a basis material on the energy grid E (keV)."""
    a, b = MATERIALS[material]
    E = np.asarray(E, dtype=np.float64)
    pe = a / E ** 3
    if material in K_EDGE:
        edge, factor = K_EDGE[material]
        pe = np.where(E >= edge, factor * pe, pe)
    return pe + b * klein_nishina_shape(E)


def kramers(kvp, E, al_mm=2.0):
    """Kramers bremsstrahlung (kVp-E)/E, filtered by al_mm of aluminium."""
    E = np.asarray(E, dtype=np.float64)
    phi = np.where(E < kvp, (kvp - E) / E, 0.0)
    return phi * np.exp(-al_mm * attenuation("aluminium", E))


def kvp_switching_sensitivity(E, kvps=(80.0, 140.0), i0=5e4):
    """One channel per tube voltage; photon counting (no energy weight).

    Row c is I0 times the normalised filtered spectrum of kVp c, so each
    channel sums to I0 over the energy grid.
    """
    S = np.stack([kramers(k, E) for k in kvps])
    return i0 * S / S.sum(axis=1, keepdims=True)


def threshold_pcd_sensitivity(E, kvp=120.0, edges=(25.0, 45.0, 65.0, 85.0), i0=2e4):
    """Ideal photon-counting detector with energy windows [edges[c], edges[c+1]).

    The last window is closed at kVp.  The whole filtered spectrum sums to I0
    over the grid; energies below the first threshold are not counted.
    """
    phi = kramers(kvp, E)
    phi = i0 * phi / phi.sum()
    E = np.asarray(E, dtype=np.float64)
    hi_edges = list(edges[1:]) + [kvp + 1e-9]
    rows = [np.where((E >= lo) & (E < hi), phi, 0.0) for lo, hi in zip(edges, hi_edges)]
    return np.stack(rows)
