"""Orthonormal full-depth 2D Daubechies-4 wavelet transform (FP64), the other
unitary U_DWT the wavelet preconditioner section names beside Haar.

The four-tap filter with two vanishing moments (Daubechies, "Ten Lectures on
Wavelets"): h = (1 + r3, 3 + r3, 3 - r3, 1 - r3) / (4 r2), r3 = sqrt 3,
r2 = sqrt 2; the high-pass filter g_k = (-1)^k h_{3-k}.  On a signal of
length m (even), periodised:
    lo_i = sum_k h_k x_{(2i+k) mod m},  hi_i = sum_k g_k x_{(2i+k) mod m},
stored lo at i and hi at m/2 + i, for i < m/2.  This is an orthogonal m x m
matrix for every even m >= 2 (at m = 2 the wrapped taps add up to the Haar
pair).  Layout as the Haar transform: at each level the current block
[0:m, 0:m] goes along rows, then along columns, down to 1 x 1.
"""

from __future__ import annotations

import numpy as np

_R3 = np.sqrt(3.0)
H = np.array([1.0 + _R3, 3.0 + _R3, 3.0 - _R3, 1.0 - _R3]) / (4.0 * np.sqrt(2.0))
G = np.array([H[3], -H[2], H[1], -H[0]])


def analysis_matrix(m):
    """The periodised one-level analysis matrix W [m, m]: rows 0..m/2-1 low-pass,
    rows m/2..m-1 high-pass."""
    W = np.zeros((m, m))
    for i in range(m // 2):
        for k in range(4):
            W[i, (2 * i + k) % m] += H[k]
            W[m // 2 + i, (2 * i + k) % m] += G[k]
    return W


def _check(img):
    n = img.shape[-1]
    if img.shape[-2] != n or n & (n - 1):
        raise ValueError("the Daubechies transform needs a square power-of-two image")
    return n


def forward(img):
    """U_DWT img for img [..., n, n]."""
    n = _check(img)
    a = np.array(img, dtype=np.float64, copy=True)
    m = n
    while m > 1:
        W = analysis_matrix(m)
        blk = a[..., :m, :m]
        blk = blk @ W.T                  # along rows: each row x -> W x
        blk = W @ blk                    # along columns
        a[..., :m, :m] = blk
        m //= 2
    return a


def inverse(coef):
    """U_DWT^T coef (the inverse, U being orthogonal): undo the levels from the
    coarsest, columns then rows."""
    n = _check(coef)
    a = np.array(coef, dtype=np.float64, copy=True)
    m = 2
    while m <= n:
        W = analysis_matrix(m)
        blk = a[..., :m, :m]
        blk = W.T @ blk
        blk = blk @ W
        a[..., :m, :m] = blk
        m *= 2
    return a
