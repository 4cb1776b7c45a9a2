"""Orthonormal full-depth 2D Haar transform (FP64), the U_DWT of the wavelet
preconditioners (Methods, "Wavelet Precondtioner" and "Cross-Material
Wavelet Precondtioner").

Standard (Mallat) layout on a square power-of-two image: at each level the
current low-pass block [0:m, 0:m] is transformed along rows, pair (2i, 2i+1)
-> low (a+b)/sqrt2 at i and high (a-b)/sqrt2 at m/2+i, then along columns the
same way; the next level works on [0:m/2, 0:m/2], down to 1x1.
"""

from __future__ import annotations

import numpy as np

R2 = np.sqrt(0.5)


def _check(img):
    n = img.shape[-1]
    if img.shape[-2] != n or n & (n - 1):
        raise ValueError("Haar transform needs a square power-of-two image")
    return n


def forward(img):
    """U_DWT img for img [..., n, n]."""
    n = _check(img)
    a = np.array(img, dtype=np.float64, copy=True)
    m = n
    while m > 1:
        h = m // 2
        blk = a[..., :m, :m]
        lo = (blk[..., :, 0::2] + blk[..., :, 1::2]) * R2
        hi = (blk[..., :, 0::2] - blk[..., :, 1::2]) * R2
        rows = np.concatenate([lo, hi], axis=-1)
        lo = (rows[..., 0::2, :] + rows[..., 1::2, :]) * R2
        hi = (rows[..., 0::2, :] - rows[..., 1::2, :]) * R2
        a[..., :m, :m] = np.concatenate([lo, hi], axis=-2)
        m = h
    return a


def inverse(coef):
    """U_DWT^T coef (the inverse, U being orthogonal)."""
    n = _check(coef)
    a = np.array(coef, dtype=np.float64, copy=True)
    m = 2
    while m <= n:
        h = m // 2
        blk = a[..., :m, :m].copy()
        lo, hi = blk[..., :h, :], blk[..., h:, :]
        rows = np.empty_like(blk)
        rows[..., 0::2, :] = (lo + hi) * R2
        rows[..., 1::2, :] = (lo - hi) * R2
        lo, hi = rows[..., :, :h], rows[..., :, h:]
        out = np.empty_like(blk)
        out[..., :, 0::2] = (lo + hi) * R2
        out[..., :, 1::2] = (lo - hi) * R2
        a[..., :m, :m] = out
        m *= 2
    return a
