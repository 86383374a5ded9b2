"""Exact solves of the posterior-mean system (oracle; tests only).

solve_dense   the definition: assemble G and b, factor G = R^T R (LAPACK dpotrf), solve.
              G is symmetric positive definite even though Q is only semi-definite (Section 3).
solve_fft     homoscedastic periodic problems (W[f, p] = w_f): the 2-D DFT diagonalises every
              shift-invariant prior block, leaving one k x k system per Fourier mode.  Exact to
              rounding at any grid size.
solve_kohler  the sparse-dense Sylvester method of Alg. 3 (Section 3.3.1) for the case the paper
              treats: one common prior factor (all kappa_j equal) and separable noise
              W[f, p] = t_f n_p.  The system then reads N^-1 Q0 M + M Lhat = F with
              Lhat = A^T T A P^-1, P = diag(tau), F = Y^T T A P^-1 (eq. (Axb-Sylv)).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import operator as op


def solve_dense(prob, b=None, return_factor: bool = False):
    """x* = G^-1 b by dense Cholesky.  b defaults to B^T C Y.  Returns [k, n_pix]."""
    G = op.posterior_precision(prob, dense=True)
    if b is None:
        b = op.rhs(prob)
    fac = sla.cho_factor(G, lower=False, check_finite=True)
    x = sla.cho_solve(fac, np.asarray(b, dtype=np.float64).reshape(-1))
    x = x.reshape(prob.k, prob.n_pix)
    return (x, fac) if return_factor else x


def fourier_symbols(prob):
    """Eigenvalues of -Lap for every 2-D Fourier mode, shape [ny, nx]:
    lam(u, v) = 4 - 2 cos(2 pi u / nx) - 2 cos(2 pi v / ny)."""
    u = np.arange(prob.nx)
    v = np.arange(prob.ny)
    return (4.0 - 2.0 * np.cos(2.0 * np.pi * u / prob.nx)[None, :]
            - 2.0 * np.cos(2.0 * np.pi * v / prob.ny)[:, None])


def _homoscedastic_weights(prob) -> np.ndarray:
    if op.boundary_of(prob) != "periodic":
        raise ValueError("the Fourier solve needs a periodic grid")
    w = prob.W[:, :1]
    if not np.all(prob.W == w):
        raise ValueError("solve_fft needs W[f, p] independent of p")
    return w[:, 0]


def operator_spectrum(prob) -> np.ndarray:
    """Per-mode k x k blocks of G in the Fourier basis: diag_j tau_j (kappa_j^2 + lam)^2 + M,
    M = sum_f w_f a_f a_f^T.  Shape [ny, nx, k, k]."""
    w = _homoscedastic_weights(prob)
    lam = fourier_symbols(prob)
    M = (prob.A.T * w) @ prob.A
    blk = np.broadcast_to(M, (prob.ny, prob.nx, prob.k, prob.k)).copy()
    for j in range(prob.k):
        blk[:, :, j, j] += prob.tau[j] * (prob.kappa[j] ** 2 + lam) ** 2
    return blk


def solve_fft(prob, b=None) -> np.ndarray:
    """Exact solve for homoscedastic noise via the 2-D DFT; b defaults to B^T C Y."""
    if b is None:
        b = op.rhs(prob)
    bh = np.fft.fft2(np.asarray(b).reshape(prob.k, prob.ny, prob.nx), axes=(1, 2))
    blk = operator_spectrum(prob)
    rhs = np.moveaxis(bh, 0, -1)[..., None]            # [ny, nx, k, 1]
    xh = np.linalg.solve(blk.astype(np.complex128), rhs)[..., 0]
    x = np.fft.ifft2(np.moveaxis(xh, -1, 0), axes=(1, 2)).real
    return x.reshape(prob.k, prob.n_pix)


def condition_number_fft(prob) -> float:
    """cond_2(G) from the exact spectrum (homoscedastic problems only)."""
    ev = np.linalg.eigvalsh(operator_spectrum(prob))
    return float(ev.max() / ev.min())


def solve_kohler(prob, t: np.ndarray, nvec: np.ndarray) -> np.ndarray:
    """Alg. 3 for N^-1 Q0 M + M Lhat = F (separable noise W = t (x) n, common kappa).

    Steps in the paper's order: real Schur form Lhat = U R U^T; Fhat = F U; for each column i,
    subtract the already-solved columns times R_{l i} and solve the shifted sparse system
    (N^-1 Q0 + R_ii I) xhat_i = fhat_i (here multiplied through by N so that the matrix
    Q0 + R_ii N is symmetric, and factored with SuperLU as in the paper); finally M = Xhat U^T.
    Returns the solution as [k, n_pix].
    """
    kap = prob.kappa
    if not np.allclose(kap, kap[0], rtol=0, atol=0):
        raise ValueError("solve_kohler needs a common kappa")
    t = np.asarray(t, dtype=np.float64)
    nvec = np.asarray(nvec, dtype=np.float64)
    if not np.allclose(prob.W, np.outer(t, nvec), rtol=1e-14, atol=0):
        raise ValueError("solve_kohler needs W = t (x) n")
    Q0 = op.prior_block(prob.ny, prob.nx, kap[0], 1.0,        # tau factored out into P
                        op.boundary_of(prob))
    P = np.diag(prob.tau)
    Pinv = np.diag(1.0 / prob.tau)
    T = np.diag(t)
    Lhat = prob.A.T @ T @ prob.A @ Pinv                         # k x k
    Ymat = prob.Y.T                                             # N x f (columns = maps)
    F = Ymat @ T @ prob.A @ Pinv                                # N x k
    R, U = sla.schur(Lhat, output="real")
    Fh = F @ U
    N = sp.diags(nvec)
    Xh = np.zeros_like(Fh)
    for i in range(prob.k):
        fi = Fh[:, i] - Xh[:, :i] @ R[:i, i]
        if i + 1 < prob.k and abs(R[i + 1, i]) > 0:
            raise ValueError("Lhat has complex eigenvalues; Lemma 2 says it cannot")
        lu = spla.splu((Q0 + R[i, i] * N).tocsc())
        Xh[:, i] = lu.solve(N @ fi)
    M = Xh @ U.T
    del P
    return M.T.copy()
