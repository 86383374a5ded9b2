"""Block preconditioned conjugate gradients (O'Leary's block CG, cited with the block Lanczos
method of Section 3.3) for G X = B with s right-hand sides at once.  Oracle: test infrastructure
only (the tests call it; the library never does).

With R = B - G X, Z = M^-1 R and the s x s matrices of the block recurrence:

    P = Z (first step),  Q = G P,  (P^T Q) alpha = R^T Z,  X += P alpha,  R -= Q alpha,
    Z = M^-1 R,  (R_old^T Z_old) beta = R^T Z,  P = Z + P beta.

Iterate j minimises the G-norm of the error of every column over X0 + the block Krylov space
K_j(M^-1 G, M^-1 R0) spanned by all columns (tests/test_oracle_block_pcg.py checks exactly that
by brute force).  No deflation: the runs here stop before any column converges.
"""
from __future__ import annotations

import numpy as np

from . import operator as op
from .pcg import block_jacobi


def block_pcg(prob, B, X0=None, max_iter: int = 10, precond: str = "none", G=None):
    """max_iter steps of block PCG for the right-hand sides B ([s, k, n_pix] or [s, k * n_pix]).
    Returns the list of iterates X_0 .. X_max_iter, each [s, k * n_pix]."""
    if G is None:
        G = op.posterior_precision(prob)
    k, n_pix = prob.k, prob.n_pix
    Bm = np.asarray(B, dtype=np.float64).reshape(-1, k * n_pix).T            # columns
    X = np.zeros_like(Bm) if X0 is None else \
        np.asarray(X0, dtype=np.float64).reshape(-1, k * n_pix).T.copy()
    if precond == "none":
        def Minv(V):
            return V
    else:
        Mb, _ = block_jacobi(prob, G, precond)

        def Minv(V):
            return np.stack([Mb(V[:, c].reshape(k, n_pix)).ravel() for c in range(V.shape[1])],
                            axis=1)
    R = Bm - G @ X
    Z = Minv(R)
    P = Z.copy()
    rz = R.T @ Z
    iterates = [X.T.copy()]
    for _ in range(max_iter):
        Q = G @ P
        alpha = np.linalg.solve(P.T @ Q, rz)
        X = X + P @ alpha
        R = R - Q @ alpha
        Z = Minv(R)
        rz_new = R.T @ Z
        beta = np.linalg.solve(rz, rz_new)
        P = Z + P @ beta
        rz = rz_new
        iterates.append(X.T.copy())
    return iterates
