"""The estimation problem the oracle solves (generalized model of the Methods).

Mean model (eq:meanModel): ybar(x) = BB exp(-AA x), with
  AA = Q (x) A  (material spectra times the projector; one-step MBMD),
  BB = B S      (channel sensitivity S with gain and I0 folded in, then the
                 projection-domain blur B of the standard-CT, projection-domain
                 and MBMD models; B = I unless a blur is given).
The blur, when given, acts per channel along the detector bins of each view:
taps [N_c, 2h+1], (B_c z)_b = sum_{|d|<=h} taps[c, d+h] z_{b+d}, with bins
beyond the detector dropped; the taps are non-negative, so that BB^T W BB has
no negative entry and the decoupled surrogate of the SPS section majorises.
Standard CT is N_k = N_E = N_c = 1 with S = I0, Q = 1; projection-domain
decomposition is the identity geometry (A = I).

Shapes: x [N_k, ny, nx]; line integrals l [N_k, V, B]; per-energy arrays
[N_E, V, B]; data y, w [N_c, V, B]; Q [N_E, N_k]; S [N_c, N_E].
Covariance: Sigma_y = diag(1 / w), w = 1 / max(y, 1) (data-based Poisson
variance, fixed; the paper only says the covariance is known).
"""

from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class OracleProblem:
    geom: dict
    Q: np.ndarray
    S: np.ndarray
    y: np.ndarray
    w: np.ndarray
    penalty: dict
    blur: np.ndarray = None

    def __post_init__(self):
        self.Q = np.asarray(self.Q, dtype=np.float64)
        self.S = np.asarray(self.S, dtype=np.float64)
        self.y = np.asarray(self.y, dtype=np.float64)
        self.w = np.asarray(self.w, dtype=np.float64)
        beta = np.asarray(self.penalty.get("beta", np.zeros((self.n_mat, self.n_mat))), dtype=np.float64)
        self.penalty = dict(kind=self.penalty.get("kind", "quadratic"), beta=beta,
                            delta=float(self.penalty.get("delta", 0.0)))
        if self.penalty["kind"] == "huber" and self.n_mat != 1:
            raise ValueError("the Huber penalty is defined for one material only")
        if self.blur is not None:
            self.blur = np.atleast_2d(np.asarray(self.blur, dtype=np.float64))
            if (self.blur.shape[0] != self.n_chan or self.blur.shape[1] % 2 != 1
                    or np.any(self.blur < 0.0) or not np.all(np.isfinite(self.blur))):
                raise ValueError("blur taps must be finite, non-negative, [n_chan, 2h+1]")
        if self.geom["kind"] == "identity":
            assert self.geom["nx"] == self.geom["n_bins"] and self.geom["ny"] == self.geom["n_views"]

    @classmethod
    def from_workload(cls, wl):
        return cls(wl.geom, wl.Q, wl.S, wl.y, wl.w, wl.penalty)

    @property
    def n_mat(self):
        return self.Q.shape[1]

    @property
    def n_energy(self):
        return self.Q.shape[0]

    @property
    def n_chan(self):
        return self.S.shape[0]

    @property
    def image_shape(self):
        return (self.n_mat, self.geom["ny"], self.geom["nx"])

    @property
    def sino_shape(self):
        return (self.geom["n_views"], self.geom["n_bins"])
