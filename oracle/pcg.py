"""Preconditioned conjugate gradients, plainly (oracle; tests and CPU baseline only).

Alg. 2 of the paper is unpreconditioned CG on G mu = b with x0 given and the stopping rule
||r|| <= eps ||r0||; the paper notes that preconditioning can be added (Section 3.2, remarks after
Alg. 2).  This is that algorithm with a left preconditioner Minv inserted in the standard way
(z = Minv r, rho = <r, z>, p = z + beta p), which reduces to Alg. 2 when Minv = I.

Readings of Alg. 2 used here: the operator is Q + B^T C B and the right-hand side B^T C y (as in
eq. (Axb)); the first search direction is the initial (preconditioned) residual; the stopping test
uses the Euclidean norm of the unpreconditioned residual.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import operator as op


def block_jacobi(prob, G=None, kind: str = "block"):
    """Preconditioner blocks taken from the assembled matrix G.

    'block'  : per pixel p, the k x k block G[(i, p), (j, p)] (prior diagonal + mixing), inverted.
    'jacobi' : 1 / diag(G).
    'none'   : identity.
    Returns a function r[k, n_pix] -> z[k, n_pix] and, for 'block', the [n_pix, k, k] inverses.
    """
    k, n_pix = prob.k, prob.n_pix
    if kind == "none":
        return (lambda r: np.array(r, dtype=np.float64, copy=True)), None
    if G is None:
        G = op.posterior_precision(prob)
    G = sp.csr_matrix(G)
    if kind == "jacobi":
        d = G.diagonal().reshape(k, n_pix)
        return (lambda r: np.asarray(r) / d), None
    if kind != "block":
        raise ValueError(kind)
    blocks = np.zeros((n_pix, k, k))
    pix = np.arange(n_pix)
    for i in range(k):
        for j in range(k):
            blocks[:, i, j] = np.asarray(G[i * n_pix + pix, j * n_pix + pix]).ravel()
    inv = np.linalg.inv(blocks)

    def apply_inv(r):
        rr = np.asarray(r, dtype=np.float64).reshape(k, n_pix).T[..., None]   # [n_pix, k, 1]
        return (inv @ rr)[..., 0].T.copy()

    return apply_inv, inv


def fourier_preconditioner(prob, scaled: bool = False):
    """Minv = (Q + I (x) Mbar)^-1 applied mode by mode in the basis that diagonalises the grid
    Laplacian: the 2-D DFT on periodic grids, the 2-D cosine transform (DCT-II) on face grids.

    Each prior block Q_j = tau_j (kappa_j^2 I - Lap)^2 is a polynomial in the Laplacian, so the
    mode whose -Lap eigenvalue is lam gets tau_j (kappa_j^2 + lam)^2.  Periodic grid: the Fourier
    modes, lam = 4 - 2 cos(2 pi u / nx) - 2 cos(2 pi v / ny).  Face grid (links only inside the
    grid): -Lap is the Kronecker sum of two path-graph Laplacians, whose eigenvectors are the
    cosines cos(pi u (i + 1/2) / n), lam = 2 - 2 cos(pi u / nx) + 2 - 2 cos(pi v / ny).  The data
    term's per-pixel blocks M_p = sum_f W[f, p] a_f a_f^T are replaced by their mean over pixels,
    Mbar = sum_f mean_p(W[f, :]) a_f a_f^T, so one k x k block remains per mode (a fixed SPD
    operator; the paper allows any preconditioner, Section 3.2, remarks after Alg. 2).  When W
    does not depend on the pixel this is G^-1 exactly.
    scaled: True (or "diag") gives the diagonally matched variant z = S^-1 (Q + I (x) Mbar)^-1
    S^-1 r, S = diag(s) with s^2 = diag(G) / diag(Q + I (x) Mbar) per pixel and component, so that
    the operator it inverts, S (Q + I (x) Mbar) S, has the diagonal of G (still fixed and SPD;
    s = 1 when W does not depend on the pixel).  "block" gives the block-matched variant
    z = T^T (Q + I (x) Mbar)^-1 T r with T block diagonal over the pixels, T_p = L0_p Lp^-1 from
    the Cholesky factors of G's k x k block at pixel p (Lp Lp^T) and of the same block of
    Q + I (x) Mbar (L0_p L0_p^T): the operator it inverts, T^-1 (Q + I (x) Mbar) T^-T, has G's
    pixel blocks.
    Returns a function r[k, n_pix] -> z[k, n_pix]."""
    from scipy import fft as sfft
    from .solve import fourier_symbols
    k, ny, nx = prob.k, prob.ny, prob.nx
    face = op.boundary_of(prob) == "face"
    wbar = prob.W.mean(axis=1)                          # [f]
    mbar = (prob.A.T * wbar) @ prob.A                   # sum_f wbar_f a_f a_f^T, [k, k]
    if face:
        lam = ((2.0 - 2.0 * np.cos(np.pi * np.arange(nx) / nx))[None, :]
               + (2.0 - 2.0 * np.cos(np.pi * np.arange(ny) / ny))[:, None])
    else:
        lam = fourier_symbols(prob)                     # [ny, nx]
    blk = np.broadcast_to(mbar, (ny, nx, k, k)).copy()
    for j in range(k):
        blk[:, :, j, j] += prob.tau[j] * (prob.kappa[j] ** 2 + lam) ** 2
    inv = np.linalg.inv(blk)                            # [ny, nx, k, k]

    def apply_inv(r):
        rr = np.asarray(r, dtype=np.float64).reshape(k, ny, nx)
        if face:
            rh = sfft.dctn(rr, type=2, norm="ortho", axes=(1, 2))
            zh = np.einsum("yxij,jyx->iyx", inv, rh)
            return sfft.idctn(zh, type=2, norm="ortho", axes=(1, 2)).reshape(k, ny * nx)
        rh = np.fft.fft2(rr, axes=(1, 2))
        zh = np.einsum("yxij,jyx->iyx", inv, rh)
        return np.fft.ifft2(zh, axes=(1, 2)).real.reshape(k, ny * nx)

    if not scaled:
        return apply_inv
    if scaled == "block":
        T = block_scale(prob)                           # [n_pix, k, k], lower triangular

        def apply_block(r):
            u = np.einsum("pij,jp->ip", T, np.asarray(r, dtype=np.float64).reshape(k, ny * nx))
            return np.einsum("pji,jp->ip", T, apply_inv(u))

        return apply_block
    s = diagonal_scale(prob)

    def apply_scaled(r):
        return apply_inv(np.asarray(r, dtype=np.float64).reshape(k, ny * nx) / s) / s

    return apply_scaled


def block_scale(prob):
    """T[n_pix, k, k] = L0_p Lp^-1 per pixel: Lp, L0_p the Cholesky factors of the k x k pixel
    blocks of G and of Q + I (x) Mbar, both read from the assembled operators (entry (i, j) of
    pixel p's block sits on the diagonal at offset (j - i) n_pix)."""
    G = op.posterior_precision(prob)
    Q = G - op.likelihood_term(prob)
    k, n = prob.k, prob.n_pix
    wbar = prob.W.mean(axis=1)
    mbar = (prob.A.T * wbar) @ prob.A
    Bp = np.empty((n, k, k))
    B0 = np.empty((n, k, k))
    for i in range(k):
        for j in range(i, k):
            g = G.diagonal((j - i) * n)[i * n:(i + 1) * n]
            q = Q.diagonal((j - i) * n)[i * n:(i + 1) * n]
            Bp[:, i, j] = Bp[:, j, i] = g
            B0[:, i, j] = B0[:, j, i] = q + mbar[i, j]
    return np.linalg.cholesky(B0) @ np.linalg.inv(np.linalg.cholesky(Bp))


def diagonal_scale(prob):
    """s[k, n_pix] with s^2 = diag(G) / diag(Q + I (x) Mbar), both diagonals read from the
    assembled operators (Q = G minus the data term)."""
    G = op.posterior_precision(prob)
    Q = G - op.likelihood_term(prob)
    wbar = prob.W.mean(axis=1)
    mbar = (prob.A.T * wbar) @ prob.A
    dG = G.diagonal().reshape(prob.k, prob.n_pix)
    dM0 = Q.diagonal().reshape(prob.k, prob.n_pix) + np.diag(mbar)[:, None]
    return np.sqrt(dG / dM0)


def pcg(prob, b=None, x0=None, tol=1e-12, max_iter=10000, precond="block", G=None,
        record=False):
    """Solve G x = b.  Returns dict(x, iters, relres_rec, relres_true, history[, iterates])."""
    if G is None:
        G = op.posterior_precision(prob)
    if b is None:
        b = op.rhs(prob)
    k, n_pix = prob.k, prob.n_pix
    if precond == "fourier":
        Minv = fourier_preconditioner(prob)
    elif precond == "fourier_diag":
        Minv = fourier_preconditioner(prob, scaled=True)
    elif precond == "fourier_block":
        Minv = fourier_preconditioner(prob, scaled="block")
    else:
        Minv, _ = block_jacobi(prob, G, precond)
    bv = np.asarray(b, dtype=np.float64).reshape(k, n_pix)
    x = np.zeros((k, n_pix)) if x0 is None else np.array(x0, dtype=np.float64).reshape(k, n_pix)

    def Gv(v):
        return (G @ v.ravel()).reshape(k, n_pix)

    r = bv - Gv(x)
    z = Minv(r)
    p = z.copy()
    rho = float(np.vdot(r, z))
    r0 = float(np.linalg.norm(r))
    hist = [r0]
    iterates = [x.copy()] if record else None
    it = 0
    rn = r0
    while rn > tol * r0 and it < max_iter:
        q = Gv(p)
        pq = float(np.vdot(p, q))
        if not pq > 0:
            break
        alpha = rho / pq
        x = x + alpha * p
        r = r - alpha * q
        z = Minv(r)
        rho_new = float(np.vdot(r, z))
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
        it += 1
        rn = float(np.linalg.norm(r))
        hist.append(rn)
        if record:
            iterates.append(x.copy())
    bn = float(np.linalg.norm(bv))
    true = float(np.linalg.norm(bv - Gv(x)) / bn) if bn > 0 else 0.0
    out = dict(x=x, iters=it, relres_rec=rn / r0 if r0 > 0 else 0.0, relres_true=true,
               history=np.array(hist))
    if record:
        out["iterates"] = iterates
    return out
