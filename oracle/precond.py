"""Preconditioner builds and applies (FP64).

Methods, "Preconditioned Optimization" and the per-application sections:
  * Hessian / Fisher information with a data-based D (the Hessian formulas of
    the standard-CT, projection-domain and one-step MBMD sections).  D is not
    computed from x_hat: for one energy and one channel D = y / I0 ("from the
    gain-corrected measured data"); with several energies D_iE =
    exp(-mu_w(E) l_w,i) from a water-only per-ray estimate l_w (the
    projection-domain section's suggestion, used for one-step MBMD too).  The
    first basis material plays water.  The estimate takes 10 Gauss-Newton
    steps from 0 on sum_c w (y - sum_E S exp(-mu_w l))^2, clamped at l >= 0.
    Per ray J[c,k] = -sum_E S_cE D_iE Q_Ek and W_i = J^T diag(w_i) J, so
    H v = A^T [W_i (A v)_i] + (beta (x) Gamma) v.  With a projection-domain
    blur B the data term couples neighbouring bins: H v = A^T [J^T B^T W B J
    (A v)] + (beta (x) Gamma) v, with J the per-ray Jacobian of the unblurred
    means (the Hessian formulas with BB = B S).  The data-based D then ignores
    the blur (the estimate is per ray, from the blurred counts).  The blur
    also makes the off-diagonal material blocks of F non-symmetric across
    pixels, so the material columns below give non-symmetric Htilde_j; their
    symmetric part is used (block_inv_sqrt symmetrises).
  * M0 (eq:diagonalPreconditioner; eq:materialColumns and the MBMD
    cross-material preconditioner): the N_k x N_k block of pixel j is read
    from the material columns (F + R) 1_k (row sums, i.e. the zero-frequency
    response, as the paper computes it), and M0_j = Htilde_j^(-1/2).
    Eigenvalues are floored at 1e-6 lambda_max of the block; an all-zero
    block (a pixel no ray sees) gives M0_j = 0.
  * Fourier (eq:fourierEigenbasis, modified Fourier, eq:localImpulseResponse):
    impulse at j = (ny/2, nx/2) in material k; column k of the per-frequency
    blocks L_f is DFT(M0^T H M0 delta_jk) / DFT(delta_j), which is the DFT of
    the response circularly shifted so that j sits at the origin.  The real
    part is kept (the even part of the response), each block is symmetrised,
    eigenvalues are floored at eps_F max_f lambda_max(L_f) (eps_F = 1e-2; the
    paper gives no floor, and its approximate eigenvalues can be <= 0).
  * Haar, and Daubechies-4 as the other unitary wavelet the section names
    (same build and apply with its transform; floor eps_H).
  * Haar (wavelet and cross-material wavelet sections): test function
    Delta x = U^T 1 in material k, so U Delta x = 1 and column k of the
    per-coefficient blocks K_w is U M0^T H M0 (Delta x (x) e_k); symmetrised
    and floored like L with eps_H = 1e-2.
  * Composition: the paper writes M = M0^T U^T Lambda^-1/2 U M0, which does
    not whiten M0^T H M0 = U^T Lambda U (it gives M^T H M ~ M0^2).  The
    reading used is M = M0 U^H Lambda^-1/2 U, M^T = U^H Lambda^-1/2 U M0,
    which does: M^T H M = U^H Lambda^-1/2 (U M0 H M0 U^H) Lambda^-1/2 U.
  * Block-diagonal (projection-domain cross-material preconditioner and the
    MBMD M0): M = M0.
"""

from __future__ import annotations

import numpy as np

from . import daub, haar, model, projector
from . import penalty as pen

WAVELETS = {"haar": haar, "daub4": daub}
M0_FLOOR = 1e-6
EPS_FOURIER = 1e-2
EPS_HAAR = 1e-2
GN_STEPS = 10


def water_only_estimate(prob, n_steps=GN_STEPS):
    """Per-ray water-equivalent path length l_w [V, B] (Gauss-Newton, >= 0)."""
    mu = prob.Q[:, 0]
    S, y, w = prob.S, prob.y, prob.w
    lw = np.zeros(prob.sino_shape)
    for _ in range(n_steps):
        e = np.exp(-mu[:, None, None] * lw[None])                     # [E, V, B]
        r = np.einsum("ce,evb->cvb", S, e) - y                          # ybar - y
        J = -np.einsum("ce,evb->cvb", S, mu[:, None, None] * e)        # d ybar / d l
        num = np.sum(w * J * r, axis=0)
        den = np.sum(w * J * J, axis=0)
        step = np.where(den > 0.0, num / np.where(den > 0.0, den, 1.0), 0.0)
        lw = np.maximum(lw - step, 0.0)
    return lw


def transmission_estimate(prob, x_ref=None):
    """D per (energy, ray) [N_E, V, B] approximating exp(-AA x_hat).

    With a reference image x_ref [N_k, ny, nx], the transmission there,
    exp(-AA x_ref) (the Fisher information at an iterate, for a rebuild during
    the iterations); else from the data: y / I0 for one energy and channel, the
    water-only estimate otherwise.
    """
    if x_ref is not None:
        return model.transmission(prob, model.line_integrals(prob, np.asarray(x_ref, dtype=np.float64)))
    if prob.n_energy == 1 and prob.n_chan == 1:
        return (prob.y[0] / prob.S[0, 0])[None]
    lw = water_only_estimate(prob)
    return np.exp(-prob.Q[:, 0][:, None, None] * lw[None])


def fisher_weights(prob, x_ref=None):
    """W_i = J_i^T diag(w_i) J_i  ->  [N_k, N_k, V, B], J = -S D{D_i} Q with D
    from transmission_estimate(prob, x_ref).  With a blur the data term does
    not split by ray, and J itself [N_c, N_k, V, B] is returned (see
    fisher_sino_apply)."""
    D = transmission_estimate(prob, x_ref)
    J = -np.einsum("ce,evb,ek->ckvb", prob.S, D, prob.Q)
    if prob.blur is not None:
        return J
    return np.einsum("cvb,ckvb,clvb->klvb", prob.w, J, J)


def fisher_sino_apply(prob, W, q):
    """The data part of the Fisher information on line integrals q [N_k, V, B]:
    W_i q_i per ray, or with a blur J^T B^T W B J q (W holding J)."""
    if prob.blur is None:
        return np.einsum("klvb,lvb->kvb", W, q)
    z = model.blur(prob, np.einsum("ckvb,kvb->cvb", W, q))
    return np.einsum("ckvb,cvb->kvb", W, model.blur(prob, prob.w * z, transpose=True))


def hessian_apply(prob, W, v):
    """H v = A^T [F_data (A v)] + (beta (x) Gamma) v for v [N_k, ny, nx]."""
    Av = projector.project(prob.geom, v)
    return projector.backproject(prob.geom, fisher_sino_apply(prob, W, Av)) + pen.hessian_apply(prob, v)


def block_inv_sqrt(blocks, floor_rel=None, floor_abs=None):
    """Symmetric inverse square root of [..., K, K] blocks with eigenvalue floors.

    floor_rel: per block, eigenvalues below floor_rel * lambda_max(block) are
    raised to it; a block with lambda_max <= 0 maps to 0.  floor_abs: a
    global lower bound on every eigenvalue.  Returns (inv_sqrt, n_floored).
    """
    B = 0.5 * (blocks + np.swapaxes(blocks, -1, -2))
    lam, V = np.linalg.eigh(B)
    lmax = lam[..., -1:]
    floor = np.zeros_like(lam)
    if floor_rel is not None:
        floor = np.maximum(floor, floor_rel * lmax)
    if floor_abs is not None:
        floor = np.maximum(floor, floor_abs)
    n_floored = int(np.sum(lam < floor))
    lam = np.maximum(lam, floor)
    good = (lmax[..., 0] > 0.0) if floor_abs is None else np.ones(lam.shape[:-1], bool)
    inv = np.where(lam > 0.0, 1.0 / np.sqrt(np.where(lam > 0.0, lam, 1.0)), 0.0)
    out = np.einsum("...ik,...k,...jk->...ij", V, inv, V)
    out[~good] = 0.0
    return out, n_floored


def _hop(prob, W, hop):
    if hop is not None:
        return hop
    return lambda v: hessian_apply(prob, W, v)


def m0_blocks(prob, W, hop=None):
    """Htilde_j [ny, nx, K, K] from the material columns (F + R) 1_k."""
    K = prob.n_mat
    ny, nx = prob.geom["ny"], prob.geom["nx"]
    H = _hop(prob, W, hop)
    Ht = np.zeros((ny, nx, K, K))
    for k in range(K):
        ones_k = np.zeros((K, ny, nx))
        ones_k[k] = 1.0
        col = H(ones_k)                                      # [K, ny, nx]: column k
        Ht[:, :, :, k] = np.moveaxis(col, 0, -1)
    return Ht


def build_m0(prob, W, hop=None):
    Ht = m0_blocks(prob, W, hop)
    M0, _ = block_inv_sqrt(Ht, floor_rel=M0_FLOOR)
    return M0


def apply_blocks(blocks, v):
    """Per-pixel (or per-coefficient) block times vector: [ny,nx,K,K] x [K,ny,nx]."""
    return np.einsum("yxkl,lyx->kyx", blocks, v)


def fourier_blocks(prob, W, M0, hop=None):
    """Per-frequency blocks L_f [ny, nx, K, K] (complex, before any floor)."""
    H = _hop(prob, W, hop)
    K = prob.n_mat
    ny, nx = prob.geom["ny"], prob.geom["nx"]
    jc = (ny // 2, nx // 2)
    L = np.zeros((ny, nx, K, K), dtype=np.complex128)
    for k in range(K):
        delta = np.zeros((K, ny, nx))
        delta[k, jc[0], jc[1]] = 1.0
        r = apply_blocks(M0, H(apply_blocks(M0, delta)))
        for kp in range(K):
            L[:, :, kp, k] = np.fft.fft2(np.roll(r[kp], (-jc[0], -jc[1]), axis=(0, 1)))
    return L


def wavelet_blocks(prob, W, M0, hop=None, wavelet=haar):
    """Per-coefficient blocks K_w [ny, nx, K, K] (before any floor) of the
    wavelet transform ``wavelet`` (the haar or daub module)."""
    H = _hop(prob, W, hop)
    K = prob.n_mat
    ny, nx = prob.geom["ny"], prob.geom["nx"]
    dx = wavelet.inverse(np.ones((ny, nx)))
    Kb = np.zeros((ny, nx, K, K))
    for k in range(K):
        e = np.zeros((K, ny, nx))
        e[k] = dx
        r = apply_blocks(M0, H(apply_blocks(M0, e)))
        for kp in range(K):
            Kb[:, :, kp, k] = wavelet.forward(r[kp])
    return Kb


def haar_blocks(prob, W, M0, hop=None):
    return wavelet_blocks(prob, W, M0, hop, haar)


def _global_floor(blocks, eps):
    B = 0.5 * (blocks + np.swapaxes(blocks, -1, -2))
    lmax = np.linalg.eigvalsh(B)[..., -1].max()
    return block_inv_sqrt(B, floor_abs=eps * lmax)


def build(prob, kind, eps=None, modified=True, W=None, hop=None, x_ref=None):
    """Build the tables of preconditioner ``kind`` in {'blockdiag','fourier','haar','daub4'}
    ('daub4': the wavelet preconditioner with the Daubechies-4 transform).

    ``modified=False`` gives the unmodified preconditioners (M0 = I), e.g. the
    Fourier preconditioner of eq:fourierEigenbasis.  ``x_ref`` takes the Fisher
    weights at that image instead of from the data.  ``hop`` replaces the
    Hessian operator v -> H v (tests use it to feed known operators).
    """
    K = prob.n_mat
    ny, nx = prob.geom["ny"], prob.geom["nx"]
    if hop is None:
        W = fisher_weights(prob, x_ref) if W is None else W
    if not modified:
        M0 = np.broadcast_to(np.eye(K), (ny, nx, K, K)).copy()
    else:
        M0 = build_m0(prob, W, hop)
    t = dict(kind=kind, M0=M0, P=None, n_floored=0)
    if kind == "blockdiag":
        return t
    if kind == "fourier":
        L = fourier_blocks(prob, W, M0, hop).real
        t["P"], t["n_floored"] = _global_floor(L, EPS_FOURIER if eps is None else eps)
        return t
    if kind in ("haar", "daub4"):
        Kb = wavelet_blocks(prob, W, M0, hop, WAVELETS[kind])
        t["P"], t["n_floored"] = _global_floor(Kb, EPS_HAAR if eps is None else eps)
        return t
    raise ValueError("unknown preconditioner %r" % kind)


def _apply_P(t, v):
    if t["P"] is None:
        return v
    if t["kind"] == "fourier":
        Vf = np.stack([np.fft.fft2(vk) for vk in v])
        Wf = np.einsum("yxkl,lyx->kyx", t["P"], Vf)
        return np.stack([np.fft.ifft2(wk).real for wk in Wf])
    wv = WAVELETS[t["kind"]]
    c = np.stack([wv.forward(vk) for vk in v])
    c = apply_blocks(t["P"], c)
    return np.stack([wv.inverse(ck) for ck in c])


def apply_M(t, v):
    """x = M x' with M = M0 P."""
    return apply_blocks(t["M0"], _apply_P(t, v))


def apply_Mt(t, g):
    """M^T g = P M0 g (M0 blocks and P are symmetric)."""
    return _apply_P(t, apply_blocks(t["M0"], g))
